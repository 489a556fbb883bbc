// Two Jacobi sweeps in one pass over HBM (temporal blocking in z).
//
// u2 = J(J(u0)).  A workgroup of BY 64-lane wavefronts, each thread owning
// RY consecutive rows (register blocking in y), covers a block of
// 64 x (BY*RY) columns: lane l, row r of wavefront w is column
// (x0 - 1 + l, y0 - 1 + w*RY + r).  The inner 62 x (BY*RY - 2) columns are
// the tile's outputs; the outer ring is recomputed redundantly by the
// neighbouring tiles.  Marching through z, at
// step k the block
//   1. computes the intermediate iterate u1 at plane k on all its columns
//      (from u0 planes k-1, k, k+1 held in registers and u0's x/y
//      neighbours read through the cache), with u1 = u0 on the Dirichlet
//      halo, and stores it in an LDS plane buffer;
//   2. after one barrier, computes u2 at plane k-1 on the inner columns from
//      u1's x/y neighbours in LDS and u1 at planes k-2 and k in registers.
// u1 never reaches HBM: per pair of sweeps the pass streams u0 and f once and
// writes u2 once.  The LDS plane buffers rotate over three slots so one
// barrier per plane suffices (a slot is rewritten two steps after it was
// last read, and every thread has passed the barrier in between).
//
// Each point of u1 and u2 is computed with exactly the arithmetic of a
// single sweep (same neighbour order, no contraction), so the result equals
// two separate sweeps bit for bit.  The fused residual, when requested, is
// that of u0 (the input), accumulated by the inner columns only.
#pragma once

#include "sweep.h"

namespace j3d {
namespace sweep_detail {

constexpr int kSweep2Cols = WAVE - 2;  // output columns per tile in x

// Rows per thread of the two-sweep pass (variant bits 2 and 16, as in the
// one-sweep pass).
template <int BY, int VAR>
struct Smem2 {
  static constexpr int TR = BY * rows_per_thread(VAR);  // rows of the block
  double pl[3][TR][WAVE];
  double red[BY];
};

template <int BY, int VAR, unsigned FL>
__device__ __forceinline__ void sweep2_tile(const GridArgs& g, int t, double* __restrict__ partials,
                                            Smem2<BY, VAR>& sm) {
  constexpr int RY = rows_per_thread(VAR);
  constexpr int TR = BY * RY;   // block rows
  constexpr int W = kSweep2Cols;
  constexpr int H = TR - 2;     // output rows per tile
  constexpr bool NT = (VAR & 4) != 0;
  static_assert(TR >= 3, "a block needs at least one inner row");
  const int lane = threadIdx.x;
  const int wy = threadIdx.y;
  const int tx = t % g.tiles_x;
  const int t2 = t / g.tiles_x;
  const int ty = t2 % g.tiles_y;
  const int tz = t2 / g.tiles_y;
  const int xi = tx * W + lane;  // column x (0 .. beyond nx+1 on the last tile)
  const int k0 = 1 + tz * g.planes;
  const int k1 = min(k0 + g.planes, g.nz + 1);
  const bool lane_in = lane >= 1 && lane <= W;
  const bool x_in = xi >= 1 && xi <= g.nx;
  // Every address is clamped into the array, halo included.
  const int xc = min(xi, g.nx + 1);
  const int xm = max(xc - 1, 0), xp = min(xc + 1, g.nx + 1);
  const double* __restrict__ u0 = static_cast<const double*>(g.u);
  const double* __restrict__ f = static_cast<const double*>(g.f);
  double* __restrict__ out = static_cast<double*>(g.o);
  const double h2 = g.h2;
  const int ztop = g.nz + 1;

  int br[RY], cu[RY], cf[RY], co[RY];
  bool inner[RY], col_in[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    br[r] = wy * RY + r;                  // block row
    const int yj = ty * H + br[r];        // column y
    const int yc = min(yj, g.ny + 1);
    cu[r] = xc + g.su_y * yc;
    cf[r] = xc + g.sf_y * yc;
    co[r] = xc + g.so_y * yc;
    inner[r] = lane_in && br[r] >= 1 && br[r] <= H;
    col_in[r] = x_in && yj >= 1 && yj <= g.ny;
  }
  // y-neighbour rows outside this thread's rows: one below the first, one
  // above the last (clamped).
  const int ylo = max(min(ty * H + br[0], g.ny + 1) - 1, 0);
  const int yhi = min(ty * H + br[RY - 1] + 1, g.ny + 1);
  const int cym = xc + g.su_y * ylo, cyp = xc + g.su_y * yhi;

  double acc = 0.0;
  double u0m[RY], u0c[RY], u1m2[RY], fprev[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    u0m[r] = u0[cu[r] + g.su_z * max(k0 - 2, 0)];
    u0c[r] = u0[cu[r] + g.su_z * (k0 - 1)];
    u1m2[r] = 0.0;
    fprev[r] = 0.0;
  }
  double u1m1[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) u1m1[r] = 0.0;

  for (int k = k0 - 1; k <= k1; ++k) {
    // Stage 1: u1 at plane k on every column of the block.
    const int kp = min(k + 1, ztop);
    const int kf = min(max(k, 1), g.nz);
    const int zk = g.su_z * k;
    double u0p[RY], fk[RY], nxm[RY], nxp[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      u0p[r] = u0[cu[r] + g.su_z * kp];
      fk[r] = f[cf[r] + g.sf_z * kf];
      nxm[r] = u0[cu[r] - xc + xm + zk];
      nxp[r] = u0[cu[r] - xc + xp + zk];
    }
    const double nylo = u0[cym + zk], nyhi = u0[cyp + zk];
    double u1[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const double nym = r == 0 ? nylo : u0c[r - 1];
      const double nyp = r == RY - 1 ? nyhi : u0c[r + 1];
      const bool pt_in = col_in[r] && k >= 1 && k <= g.nz;
      double s = nxm[r] + nxp[r];
      s = s + nym;
      s = s + nyp;
      s = s + u0m[r];
      s = s + u0p[r];
      u1[r] = pt_in ? (s + h2 * fk[r]) / 6.0 : u0c[r];
      if (FL & F_RES) {
        const double res = fk[r] - (6.0 * u0c[r] - s) / h2;
        acc += (inner[r] && pt_in && k >= k0 && k < k1) ? res * res : 0.0;
      }
      sm.pl[k % 3][br[r]][lane] = u1[r];
    }
    __syncthreads();
    // Stage 2: u2 at plane k-1 on the inner columns.
    if (k - 1 >= k0) {
      const double(*p1)[WAVE] = sm.pl[(k + 2) % 3];  // slot of plane k-1
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        if (inner[r]) {
          double s1 = p1[br[r]][lane - 1] + p1[br[r]][lane + 1];
          s1 = s1 + p1[br[r] - 1][lane];
          s1 = s1 + p1[br[r] + 1][lane];
          s1 = s1 + u1m2[r];
          s1 = s1 + u1[r];
          const double u2 = (s1 + h2 * fprev[r]) / 6.0;
          if (col_in[r]) put<double, NT>(out + co[r] + g.so_z * (k - 1), u2);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      u0m[r] = u0c[r];
      u0c[r] = u0p[r];
      u1m2[r] = u1m1[r];
      u1m1[r] = u1[r];
      fprev[r] = fk[r];
    }
  }

  if (FL & F_RES) {
    const double v = wave_sum(acc);
    if (lane == 0) sm.red[wy] = v;
    __syncthreads();
    if (wy == 0 && lane == 0) {
      double tot = 0.0;
#pragma unroll
      for (int q = 0; q < BY; ++q) tot += sm.red[q];
      partials[g.tile0 + t] = tot;
    }
  }
  __syncthreads();
}

template <int BY, int VAR, unsigned FL>
__global__ void __launch_bounds__(WAVE * BY)
    k_sweep2_one(GridArgs g, double* __restrict__ partials, const int* __restrict__ done) {
  if (done != nullptr && *done != 0) return;
  __shared__ Smem2<BY, VAR> sm;
  const int ntiles = g.tiles_x * g.tiles_y * g.tiles_z;
  if (g.order == 0) {
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < ntiles; t += gridDim.x)
      sweep2_tile<BY, VAR, FL>(g, t, partials, sm);
  } else {
    const int nv = virtual_tiles(ntiles, g.order, g.chunk);
    for (int vb = blockIdx.x; vb < nv; vb += gridDim.x) {
      const int t = g.order == 2 ? xcd_chunked(vb, g.chunk) : vb;
      if (t < ntiles) sweep2_tile<BY, VAR, FL>(g, t, partials, sm);
    }
  }
}

hipError_t dispatch_sweep2(unsigned flags, const Launch& L);

}  // namespace sweep_detail
}  // namespace j3d
