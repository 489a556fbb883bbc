// Two Jacobi sweeps in one pass over HBM (temporal blocking in z), in FP64
// or FP32.
//
// u2 = J(J(u0)).  A workgroup of BY 64-lane wavefronts, each thread owning
// RY consecutive rows (register blocking in y), covers a block of 64 x
// (BY*RY) columns: thread (l, w), row r is column (x0 - 2 + l, y0 - 1 +
// w*RY + r).  Marching through z, at step k the block
//   1. computes the intermediate iterate u1 at plane k on lanes 1..62 of
//      every row (u1 = u0 on the Dirichlet halo), from u0 planes k-1, k, k+1
//      held in registers;
//   2. computes u2 at plane k-1 on lanes 2..61 of the inner rows from u1
//      planes k-2, k-1, k held in registers.
// The x-neighbours in both stages come from the adjacent lanes of the same
// wavefront by DPP wave shifts (no memory access: the lanes at the block's
// x edges only feed columns that are not output), and the y-neighbours from
// the thread's own rows, except at a wavefront's first and last row: those
// come from the neighbouring wavefront through LDS (u0 rows in stage 1, u1
// rows in stage 2), and only the block's outer wavefronts load the u0 rows
// beyond the block through the cache.  The edge rows rotate over plane slots
// so one barrier per plane suffices.  u1 never reaches HBM: per pair of sweeps the pass streams u0
// and f once and writes u2 once.  The outputs of a block are its inner 60 x
// (BY*RY - 2) columns; the ring around them is recomputed by the
// neighbouring blocks.
//
// Each point of u1 and u2 is computed with exactly the arithmetic of a
// single sweep (same neighbour order, no contraction), so the result equals
// two separate sweeps bit for bit.  The fused residual, when requested, is
// that of u0 (the input), accumulated by the output columns only.
#pragma once

#include "sweep.h"

namespace j3d {
namespace sweep_detail {

// Output columns per tile in x (one wavefront along x).
constexpr int sweep2_cols(int wx) { return wx == 1 ? WAVE - 4 : 0; }

template <typename T, int BY, int WX, int VAR>
struct Smem2 {
  T edge[3][BY][2][WAVE];   // plane slot, wavefront, first/last row of u1
  T u0edge[2][BY][2][WAVE]; // plane parity, wavefront, first/last row of u0
  double red[BY];
};

// Flags: F_WRITE (store u2 to g.o), F_RES (FP64: residual of u0), F_FIRST
// (u0 is identically zero and not read; the first two sweeps of a correction
// cycle), F_LAST (add (double) u2 to g.u64 instead of storing it; the last
// two sweeps of a correction cycle).
template <typename T, int BY, int WX, int VAR, unsigned FL>
__device__ __forceinline__ void sweep2_tile(const GridArgs& g, int t, double* __restrict__ partials,
                                            Smem2<T, BY, WX, VAR>& sm) {
  static_assert(WX == 1, "the two-sweep pass uses one wavefront along x");
  constexpr int RY = rows_per_thread(VAR);
  constexpr int TR = BY * RY;   // block rows
  constexpr int W = sweep2_cols(1);
  constexpr int H = TR - 2;     // output rows per tile
  constexpr bool NT = (VAR & 4) != 0;
  constexpr bool ZERO = (FL & F_FIRST) != 0;
  static_assert(TR >= 3, "a block needs at least one inner row");
  static_assert(!(FL & F_RES) || sizeof(T) == 8, "the fused residual is an FP64 pass");
  const int lane = threadIdx.x;
  const int wy = threadIdx.y;
  const int tx = t % g.tiles_x;
  const int t2 = t / g.tiles_x;
  const int ty = t2 % g.tiles_y;
  const int tz = t2 / g.tiles_y;
  const int xi = tx * W - 1 + lane;  // column x (-1 .. beyond nx+1 at the x ends)
  const int k0 = 1 + tz * g.planes;
  const int k1 = min(k0 + g.planes, g.nz + 1);
  const bool lane_out = lane >= 2 && lane <= W + 1;
  const bool x_in = xi >= 1 && xi <= g.nx;
  // Every address is clamped into the array, halo included.
  const int xc = min(max(xi, 0), g.nx + 1);
  const T* __restrict__ u0 = static_cast<const T*>(g.u);
  const T* __restrict__ f = static_cast<const T*>(g.f);
  T* __restrict__ out = static_cast<T*>(g.o);
  double* __restrict__ u64 = g.u64;
  const T h2 = h2_of<T>(g);
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
    co[r] = (FL & F_LAST) ? xc + g.s64_y * yc : xc + g.so_y * yc;
    inner[r] = lane_out && br[r] >= 1 && br[r] <= H;
    col_in[r] = x_in && yj >= 1 && yj <= g.ny;
  }
  // y-neighbour rows outside this thread's rows: one below the first, one
  // above the last (clamped).
  const int ylo = max(min(ty * H + br[0], g.ny + 1) - 1, 0);
  const int yhi = min(ty * H + br[RY - 1] + 1, g.ny + 1);
  const int cym = xc + g.su_y * ylo, cyp = xc + g.su_y * yhi;

  double acc = 0.0;
  T u0m[RY], u0c[RY], u1m1[RY], u1m2[RY], fprev[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    u0m[r] = ZERO ? T(0) : u0[cu[r] + g.su_z * max(k0 - 2, 0)];
    u0c[r] = ZERO ? T(0) : u0[cu[r] + g.su_z * (k0 - 1)];
    u1m1[r] = T(0);
    u1m2[r] = T(0);
    fprev[r] = T(0);
  }
  // The u0 rows just below and above a wavefront's rows are the neighbouring
  // wavefronts' edge rows: they pass through LDS (two plane slots), and only
  // the block's outer wavefronts load the rows beyond the block.
  if (!ZERO) {
    sm.u0edge[(k0 - 1) & 1][wy][0][lane] = u0c[0];
    sm.u0edge[(k0 - 1) & 1][wy][1][lane] = u0c[RY - 1];
    __syncthreads();
  }

  for (int k = k0 - 1; k <= k1; ++k) {
    // Stage 1: u1 at plane k on every row of the block.
    const int kp = min(k + 1, ztop);
    const int kf = min(max(k, 1), g.nz);
    const int zk = g.su_z * k;
    T u0p[RY], fk[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      fk[r] = f[cf[r] + g.sf_z * kf];
      u0p[r] = ZERO ? T(0) : u0[cu[r] + g.su_z * kp];
    }
    T nylo = T(0), nyhi = T(0);
    if (!ZERO) {
      nylo = wy > 0 ? sm.u0edge[k & 1][wy - 1][1][lane] : u0[cym + zk];
      nyhi = wy < BY - 1 ? sm.u0edge[k & 1][wy + 1][0][lane] : u0[cyp + zk];
      // plane k+1 for the next step (read after this step's barrier)
      sm.u0edge[(k + 1) & 1][wy][0][lane] = u0p[0];
      sm.u0edge[(k + 1) & 1][wy][1][lane] = u0p[RY - 1];
    }
    T u1[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const T nym = r == 0 ? nylo : u0c[r - 1];
      const T nyp = r == RY - 1 ? nyhi : u0c[r + 1];
      const bool pt_in = col_in[r] && k >= 1 && k <= g.nz;
      T s = ZERO ? T(0) : from_left(u0c[r]) + from_right(u0c[r]);
      s = s + nym;
      s = s + nyp;
      s = s + u0m[r];
      s = s + u0p[r];
      u1[r] = pt_in ? div6(s + h2 * fk[r]) : u0c[r];
      if (FL & F_RES) {
        const double res = static_cast<double>(fk[r]) -
                           (6.0 * static_cast<double>(u0c[r]) - static_cast<double>(s)) / g.h2;
        acc += (inner[r] && pt_in && k >= k0 && k < k1) ? res * res : 0.0;
      }
    }
    sm.edge[k % 3][wy][0][lane] = u1[0];
    sm.edge[k % 3][wy][1][lane] = u1[RY - 1];
    __syncthreads();
    // Stage 2: u2 at plane k-1 on the output columns.
    if (k - 1 >= k0) {
      const int sl = (k + 2) % 3;  // slot of plane k-1
      const T above = wy > 0 ? sm.edge[sl][wy - 1][1][lane] : T(0);
      const T below = wy < BY - 1 ? sm.edge[sl][wy + 1][0][lane] : T(0);
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const T xm = from_left(u1m1[r]);
        const T xp = from_right(u1m1[r]);
        if (inner[r]) {
          const T ym = r == 0 ? above : u1m1[r - 1];
          const T yp = r == RY - 1 ? below : u1m1[r + 1];
          T s1 = xm + xp;
          s1 = s1 + ym;
          s1 = s1 + yp;
          s1 = s1 + u1m2[r];
          s1 = s1 + u1[r];
          const T u2 = div6(s1 + h2 * fprev[r]);
          if (col_in[r]) {
            if (FL & F_LAST) {
              double* q = u64 + co[r] + g.s64_z * (k - 1);
              q[0] = q[0] + static_cast<double>(u2);
            } else {
              put<T, NT>(out + co[r] + g.so_z * (k - 1), u2);
            }
          }
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
    const double tot = block_sum<BY * WX>(acc, sm.red);
    if (wy == 0 && lane == 0) partials[g.tile0 + t] = tot;
  }
  __syncthreads();
}

template <typename T, int BY, int WX, int VAR, unsigned FL>
__global__ void __launch_bounds__(WAVE * WX * BY)
    k_sweep2_one(GridArgs g, double* __restrict__ partials, const int* __restrict__ done) {
  if (done != nullptr && *done != 0) return;
  __shared__ Smem2<T, BY, WX, VAR> sm;
  const int ntiles = g.tiles_x * g.tiles_y * g.tiles_z;
  if (g.order == 0) {
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < ntiles; t += gridDim.x)
      sweep2_tile<T, BY, WX, VAR, FL>(g, t, partials, sm);
  } else {
    const int nv = virtual_tiles(ntiles, g.order, g.chunk);
    for (int vb = blockIdx.x; vb < nv; vb += gridDim.x) {
      const int t = g.order == 2 ? xcd_chunked(vb, g.chunk) : vb;
      if (t < ntiles) sweep2_tile<T, BY, WX, VAR, FL>(g, t, partials, sm);
    }
  }
}

// The two-sweep pass over a table of grids (as k_pass_batch).
template <typename T, int BY, int WX, int VAR, unsigned FL>
__global__ void __launch_bounds__(WAVE * WX * BY)
    k_sweep2_batch(const GridArgs* __restrict__ table, int ngrids, int ntiles,
                   double* __restrict__ partials, const int* __restrict__ done, int order, int chunk) {
  __shared__ Smem2<T, BY, WX, VAR> sm;
  const int nv = order == 0 ? ntiles : virtual_tiles(ntiles, order, chunk);
  const int first = order == 0 ? xcd_remap(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  for (int vb = first; vb < nv; vb += gridDim.x) {
    const int t = order == 2 ? xcd_chunked(vb, chunk) : vb;
    if (t >= ntiles) continue;
    int lo = 0, hi = ngrids - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (table[mid].tile0 <= t) lo = mid; else hi = mid - 1;
    }
    if (done != nullptr && done[table[lo].id] != 0) continue;
    const GridArgs g = table[lo];
    sweep2_tile<T, BY, WX, VAR, FL>(g, t - g.tile0, partials, sm);
  }
}

// Instantiated two-sweep shapes: one wavefront along x, blocks of 4 to 32
// rows.  FP32 passes (the correction sweeps of the mixed solve) keep the
// nontemporal-store variants only.
constexpr bool shape2_instantiated(int esize, int by, int wx, int var) {
  const int tr = by * rows_per_thread(var);
  if (wx != 1 || tr < 4 || tr > 32 || by > 16) return false;
  const bool nt_var = var == 4 || var == 6 || var == 20;
  if (esize == 4) return nt_var;
  return nt_var || var == 0 || var == 2 || var == 16;
}

// ---------------------------------------------------------------------
// Host-side launch templates of the two-sweep pass
// ---------------------------------------------------------------------

template <typename T, int BY, int WX, int VAR, unsigned FL>
hipError_t go2(const Launch& L) {
  if constexpr (!shape2_instantiated(sizeof(T), BY, WX, VAR)) {
    return hipErrorInvalidValue;
  } else {
    constexpr int THREADS = WAVE * WX * BY;
    if (L.batch) {
      const int chunk = kBatchChunk;
      int grid = virtual_tiles(L.ntiles, L.c->order, chunk);
      if (L.c->persistent) {
        static int cap = 0;
        if (cap == 0) cap = resident_blocks(k_sweep2_batch<T, BY, WX, VAR, FL>, THREADS);
        grid = min(grid, cap);
      }
      if (grid <= 0 || L.ngrids <= 0) return hipSuccess;
      hipLaunchKernelGGL((k_sweep2_batch<T, BY, WX, VAR, FL>), dim3(grid), dim3(WAVE * WX, BY), 0, L.st,
                         L.table, L.ngrids, L.ntiles, L.partials, L.done, L.c->order, chunk);
    } else {
      const GridArgs& g = *L.one;
      int grid = virtual_tiles(g.tiles_x * g.tiles_y * g.tiles_z, g.order, g.chunk);
      if (L.c->persistent) {
        static int cap = 0;
        if (cap == 0) cap = resident_blocks(k_sweep2_one<T, BY, WX, VAR, FL>, THREADS);
        grid = min(grid, cap);
      }
      if (grid <= 0) return hipSuccess;
      hipLaunchKernelGGL((k_sweep2_one<T, BY, WX, VAR, FL>), dim3(grid), dim3(WAVE * WX, BY), 0, L.st, g,
                         L.partials, L.done);
    }
    return hipGetLastError();
  }
}

template <typename T, int BY, int WX, unsigned FL>
hipError_t by_variant2(const Launch& L) {
  switch (L.c->variant) {
    case 0: return go2<T, BY, WX, 0, FL>(L);
    case 4: return go2<T, BY, WX, 4, FL>(L);
    case 2: return go2<T, BY, WX, 2, FL>(L);
    case 6: return go2<T, BY, WX, 6, FL>(L);
    case 16: return go2<T, BY, WX, 16, FL>(L);
    case 20: return go2<T, BY, WX, 20, FL>(L);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int BY, unsigned FL>
hipError_t by_cols2(const Launch& L) {
  switch (L.c->cols) {
    case 1: return by_variant2<T, BY, 1, FL>(L);
    case 2: return by_variant2<T, BY, 2, FL>(L);
    case 4: return by_variant2<T, BY, 4, FL>(L);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, unsigned FL>
hipError_t by_rows2(const Launch& L) {
  switch (L.c->rows) {
    case 1: return by_cols2<T, 1, FL>(L);
    case 2: return by_cols2<T, 2, FL>(L);
    case 4: return by_cols2<T, 4, FL>(L);
    case 8: return by_cols2<T, 8, FL>(L);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch_sweep2_f64(unsigned flags, const Launch& L);
hipError_t dispatch_sweep2_f32(unsigned flags, const Launch& L);

}  // namespace sweep_detail
}  // namespace j3d
