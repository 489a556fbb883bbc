// Three Jacobi sweeps in one pass over HBM (temporal blocking in z), in FP64
// or FP32.
//
// u3 = J(J(J(u0))).  A workgroup of BY 64-lane wavefronts, each thread owning
// RY consecutive rows, covers a block of 64 x (BY*RY) columns: thread (l, w),
// row r is column (x0 - 3 + l, y0 - 2 + w*RY + r), x0 = 1 + 58 tx.  Marching
// through z, at step k the block
//   1. computes u1 at plane k on lanes 1..62 of every row (u1 = u0 on the
//      Dirichlet halo), from u0 planes k-1, k, k+1 in registers;
//   2. computes u2 at plane k-1 on lanes 2..61 of rows 1 .. BY*RY-2;
//   3. computes u3 at plane k-2 on lanes 3..60 of rows 2 .. BY*RY-3, the
//      outputs (58 x (BY*RY - 4) columns per block; the ring around them is
//      recomputed by the neighbouring blocks).
// x-neighbours come from the adjacent lanes by DPP wave shifts, y-neighbours
// from the thread's own rows, and at a wavefront's first and last row from
// the neighbouring wavefront through LDS: u0 rows (two plane slots), u1 rows
// (three) and u2 rows (two); only the block's outer wavefronts load the u0
// rows beyond the block.  One barrier per plane.  u1 and u2 never reach HBM:
// per three sweeps the pass streams u0 and f once and writes u3 once.
//
// Each point of u1, u2 and u3 is computed with exactly the arithmetic of a
// single sweep (same neighbour order, no contraction), so the result equals
// three separate sweeps bit for bit.  The fused residual, when requested, is
// that of u0 (F_RES, in stage 1), u1 (F_RES1, stage 2) or u2 (F_RES2,
// stage 3): each stage's neighbour sum is exactly the one the residual of
// its input needs.  Only the output columns accumulate it, plane by plane
// in increasing z whichever the stage.
#pragma once

#include "sweep.h"

namespace j3d {
namespace sweep_detail {

// Output columns per tile in x.
constexpr int kSweep3Cols = WAVE - 6;

// Edge rows exchanged between the wavefronts of a block, in three slots per
// array: the slot of a plane is the phase (position in the z loop unrolled
// by three) of the step that writes it, so every slot index is a
// compile-time constant of the unrolled code.
template <typename T, int BY>
struct Smem3 {
  T e0[3][BY][2][WAVE];  // u0: slot, wavefront, first/last row
  T e1[3][BY][2][WAVE];  // u1
  T e2[3][BY][2][WAVE];  // u2
  double red[BY];
};

// The value of lane l-1 (shl: l+1) of the wavefront; lane 0 (63) gets 0.
// One DPP move per 32-bit half, with no copy of the destination first: the
// three-sweep tile never uses the shifted value at its edge lanes.
__device__ __forceinline__ double shift_in_left(double v) {
  const dpp_i2 a = __builtin_bit_cast(dpp_i2, v);
  dpp_i2 r;
  r.x = __builtin_amdgcn_mov_dpp(a.x, 0x138, 0xF, 0xF, true);
  r.y = __builtin_amdgcn_mov_dpp(a.y, 0x138, 0xF, 0xF, true);
  return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double shift_in_right(double v) {
  const dpp_i2 a = __builtin_bit_cast(dpp_i2, v);
  dpp_i2 r;
  r.x = __builtin_amdgcn_mov_dpp(a.x, 0x130, 0xF, 0xF, true);
  r.y = __builtin_amdgcn_mov_dpp(a.y, 0x130, 0xF, 0xF, true);
  return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ float shift_in_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}
__device__ __forceinline__ float shift_in_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}

// Flags as for the two-sweep pass: F_WRITE (store u3 to g.o), F_RES (FP64:
// residual of u0; F_RES1, F_RES2: of u1, u2), F_FIRST (u0 is identically
// zero and not read), F_LAST (add (double) u3 to g.u64 instead of storing
// it).
//
// The loads of plane step k+1 (u0 at plane k+2, f at k+1, and the outer
// wavefronts' u0 rows beyond the block at k+1) are issued at the start of
// step k, before its arithmetic, so a whole step of work covers their
// latency; one extra plane of registers per streamed array holds them.
template <typename T, int BY, int VAR, unsigned FL>
__device__ __forceinline__ void sweep3_tile(const GridArgs& g, int t, double* __restrict__ partials,
                                            Smem3<T, BY>& sm) {
  constexpr int RY = rows_per_thread(VAR);
  constexpr int TR = BY * RY;  // block rows
  constexpr int W = kSweep3Cols;
  constexpr int H = TR - 4;    // output rows per tile
  constexpr bool NT = (VAR & 4) != 0;
  constexpr bool ZERO = (FL & F_FIRST) != 0;
  constexpr uint32_t ES = sizeof(T);
  static_assert(TR >= 5, "a block needs at least one output row");
  constexpr unsigned RES_ANY = FL & (F_RES | F_RES1 | F_RES2);
  static_assert(RES_ANY == 0 || sizeof(T) == 8, "the fused residual is an FP64 pass");
  static_assert(RES_ANY == 0 || RES_ANY == F_RES || RES_ANY == F_RES1 || RES_ANY == F_RES2,
                "one fused residual per pass");
  const int lane = threadIdx.x;
  const int wy = __builtin_amdgcn_readfirstlane(threadIdx.y);  // uniform in the wavefront
  const int tx = t % g.tiles_x;
  const int t2 = t / g.tiles_x;
  const int ty = t2 % g.tiles_y;
  const int tz = t2 / g.tiles_y;
  const int xi = tx * W - 2 + lane;  // column x (-2 .. beyond nx+1 at the x ends)
  const int k0 = 1 + tz * g.planes;
  const int k1 = min(k0 + g.planes, g.nz + 1);
  const bool lane_out = lane >= 3 && lane <= W + 2;
  const bool x_in = xi >= 1 && xi <= g.nx;
  const int xc = min(max(xi, 0), g.nx + 1);
  const char* u0b = static_cast<const char*>(g.u);
  const char* fb = static_cast<const char*>(g.f);
  char* ob = static_cast<char*>(g.o);
  char* u64b = reinterpret_cast<char*>(g.u64);
  const T h2 = h2_of<T>(g);
  const int ztop = g.nz + 1;

  // A wavefront whose rows all lie past the boundary row y = ny + 1 (in a
  // grid's last block row when H does not divide ny) feeds no output: the
  // wavefront below it ends on the boundary row or beyond, and those rows
  // keep their values whatever their neighbours, so what this wavefront
  // would leave in the shared edge rows is never selected.  It only takes
  // its part in the block's barriers (the set-up one, one per plane step,
  // the residual's and the last) and adds zero to the residual.  Wavefront
  // 0 is never such a wavefront (its first row is ty*H - 1 <= ny - 2).
  if (ty * H - 1 + wy * RY >= g.ny + 2) {
    __syncthreads();
    for (int k = k0 - 2; k <= k1 + 1; ++k) __syncthreads();
    if (RES_ANY != 0) (void)block_sum<BY>(0.0, sm.red);
    __syncthreads();
    return;
  }

  // byte offsets within a plane of the thread's rows
  uint32_t ou[RY], of[RY], oo[RY];
  bool inner2[RY], inner3[RY], col_in[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int br = wy * RY + r;       // block row
    const int yj = ty * H + br - 1;   // column y (block row 2 is the first output row)
    const int yc = min(max(yj, 0), g.ny + 1);
    ou[r] = (uint32_t)(xc + g.su_y * yc) * ES;
    of[r] = (uint32_t)(xc + g.sf_y * yc) * ES;
    oo[r] = (FL & F_LAST) ? (uint32_t)(xc + g.s64_y * yc) * 8u : (uint32_t)(xc + g.so_y * yc) * ES;
    inner2[r] = br >= 1 && br <= TR - 2;
    inner3[r] = lane_out && br >= 2 && br <= TR - 3;
    col_in[r] = x_in && yj >= 1 && yj <= g.ny;
  }
  // u0 rows just below and above this wavefront's rows (clamped); only the
  // block's first and last wavefronts load them, the others take them from
  // the neighbouring wavefront through LDS
  const int ylo = max(min(max(ty * H - 1 + wy * RY, 0), g.ny + 1) - 1, 0);
  const int yhi = min(max(ty * H - 1 + wy * RY + RY, 0), g.ny + 1);
  const uint32_t oylo = (uint32_t)(xc + g.su_y * ylo) * ES, oyhi = (uint32_t)(xc + g.su_y * yhi) * ES;
  const bool wlo = wy == 0, whi = wy == BY - 1;
  const int wdn = wlo ? 0 : wy - 1, wup = whi ? BY - 1 : wy + 1;  // neighbouring wavefronts

  // plane kk >= 0 of u, f, the output
  const uint64_t zu = (uint64_t)g.su_z * ES, zf = (uint64_t)g.sf_z * ES;
  const uint64_t zo = (FL & F_LAST) ? (uint64_t)g.s64_z * 8 : (uint64_t)g.so_z * ES;
  auto u_plane = [&](int kk) { return plane_rsrc(u0b + (uint64_t)(uint32_t)kk * zu); };
  auto f_plane = [&](int kk) { return plane_rsrc(fb + (uint64_t)(uint32_t)kk * zf); };

  double acc = 0.0;
  // Three buffers per plane array, whose roles rotate with k (below,
  // current, above for u0; k-2, k-1, k for u1 and f; k-3, k-2, k-1 for u2):
  // the z loop is unrolled by three, so the rotation is a renaming, not
  // register moves.  pu, pf, pylo, pyhi: the next step's loads in flight.
  T u0A[RY], u0B[RY], u0C[RY], u1A[RY], u1B[RY], u1C[RY], u2A[RY], u2B[RY], u2C[RY];
  T fA[RY], fB[RY], fC[RY], pu[RY], pf[RY];
  T pylo = T(0), pyhi = T(0);
  // u3 of the plane the previous step computed, stored at the start of the
  // next step together with that step's loads (so that a wait for loads
  // never waits for stores issued just before it); with F_LAST, pq holds
  // the FP64 values it is added to, loaded one step ahead like the
  // streamed planes
  T st[RY];
  double pq[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    st[r] = T(0);
    pq[r] = 0.0;
  }
  auto out_plane = [&](int kk) {
    return plane_rsrc(((FL & F_LAST) ? u64b : ob) + (uint64_t)(uint32_t)kk * zo);
  };
  // store u3 of plane kk (held in st)
  auto flush = [&](int kk) {
    const auto ro = out_plane(kk);
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (inner3[r] && col_in[r]) {
        if (FL & F_LAST)
          bstore<double, false>(pq[r] + static_cast<double>(st[r]), ro, oo[r]);
        else
          bstore<T, NT>(st[r], ro, oo[r]);
      }
    }
  };
  // the loads step k consumes: u0 at plane k+1, f at k, the outer rows at k
  auto issue = [&](int k) {
    const auto rp = u_plane(min(max(k + 1, 0), ztop));
    const auto rf = f_plane(min(max(k, 1), g.nz));
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      pu[r] = ZERO ? T(0) : bload<T>(rp, ou[r]);
      pf[r] = bload<T>(rf, of[r]);
    }
    if (!ZERO) {
      const auto rc = u_plane(min(max(k, 0), ztop));
      if (wlo) pylo = bload<T>(rc, oylo);
      if (whi) pyhi = bload<T>(rc, oyhi);
    }
  };
  {
    const auto ra = u_plane(max(k0 - 3, 0));
    const auto rb = u_plane(max(k0 - 2, 0));
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      u0A[r] = ZERO ? T(0) : bload<T>(ra, ou[r]);
      u0B[r] = ZERO ? T(0) : bload<T>(rb, ou[r]);
      u1A[r] = u1B[r] = u2A[r] = u2B[r] = fA[r] = fB[r] = T(0);
    }
  }
  issue(k0 - 2);
  if (!ZERO) {
    // plane k0-2 is read by the first step (phase 0)
    sm.e0[0][wy][0][lane] = u0B[0];
    sm.e0[0][wy][1][lane] = u0B[RY - 1];
  }
  __syncthreads();

  // One plane step: u0m/u0c/u0p are u0 at planes k-1, k, k+1, fm2/fm1/fk
  // are f at k-2, k-1, k, u1m2/u1m1/u1 u1 at k-2, k-1, k (u1 computed here)
  // and u2m2/u2m1/u2 u2 at k-3, k-2, k-1 (u2 computed here).
  // ph: the step's phase p in the unrolled loop (std::integral_constant).
  // Slots: e0 of plane k is p (written by step k-1 as its p+1), e1 of plane k
  // p, of k-1 p+2; e2 of plane k-1 (formed here) p, of k-2 p+2 (mod 3).
  auto step = [&](auto ph, int k, T(&u0m)[RY], T(&u0c)[RY], T(&u0p)[RY], T(&fm2)[RY], T(&fm1)[RY], T(&fk)[RY],
                  T(&u1m2)[RY], T(&u1m1)[RY], T(&u1)[RY], T(&u2m2)[RY], T(&u2m1)[RY], T(&u2)[RY]) {
    constexpr int P = decltype(ph)::value, P1 = (P + 1) % 3, P2 = (P + 2) % 3;
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      u0p[r] = pu[r];
      fk[r] = pf[r];
    }
    const T elo = pylo, ehi = pyhi;
    if (k <= k1) issue(k + 1);
    if (k - 3 >= k0) flush(k - 3);
    if ((FL & F_LAST) && k - 2 >= k0) {
      const auto rq = out_plane(k - 2);
#pragma unroll
      for (int r = 0; r < RY; ++r)
        if (inner3[r] && col_in[r]) pq[r] = bload<double>(rq, oo[r]);
    }
    T nylo = T(0), nyhi = T(0);
    if (!ZERO) {
      nylo = wlo ? elo : sm.e0[P][wdn][1][lane];
      nyhi = whi ? ehi : sm.e0[P][wup][0][lane];
      // plane k+1 for the next step (read after this step's barrier)
      sm.e0[P1][wy][0][lane] = u0p[0];
      sm.e0[P1][wy][1][lane] = u0p[RY - 1];
    }
    const bool kin1 = k >= 1 && k <= g.nz;
    const bool kout1 = k >= k0 && k < k1;
    // stage 1: u1 at plane k on every row of the block (the quotients by 6
    // in their fused form, then the rare exact divisions, see div6)
    T x1[RY];
    uint64_t small1 = 0;  // lanes whose quotient needs the division
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const T nym = r == 0 ? nylo : u0c[r - 1];
      const T nyp = r == RY - 1 ? nyhi : u0c[r + 1];
      const bool pt_in = col_in[r] && kin1;
      T s = ZERO ? T(0) : shift_in_left(u0c[r]) + shift_in_right(u0c[r]);
      s = s + nym;
      s = s + nyp;
      s = s + u0m[r];
      s = s + u0p[r];
      x1[r] = s + h2 * fk[r];
      u1[r] = pt_in ? div6_fused(x1[r]) : u0c[r];
      small1 |= __builtin_amdgcn_ballot_w64(pt_in && div6_small(x1[r]));
      if (FL & F_RES) {
        if (inner3[r] && pt_in && kout1) {
          const double res = static_cast<double>(fk[r]) -
                             (6.0 * static_cast<double>(u0c[r]) - static_cast<double>(s)) / g.h2;
          acc += res * res;
        }
      }
    }
    if (small1 != 0) {
#pragma unroll
      for (int r = 0; r < RY; ++r)
        if (col_in[r] && kin1 && div6_small(x1[r])) u1[r] = x1[r] / T(6);
    }
    sm.e1[P][wy][0][lane] = u1[0];
    sm.e1[P][wy][1][lane] = u1[RY - 1];
    __syncthreads();
    // stage 2: u2 at plane k-1 (from u1 at k-2, k-1, k)
    {
      const T below = wlo ? T(0) : sm.e1[P2][wdn][1][lane];
      const T above = whi ? T(0) : sm.e1[P2][wup][0][lane];
      const bool kin2 = k - 1 >= 1 && k - 1 <= g.nz;
      const bool kout2 = k - 1 >= k0 && k - 1 < k1;
      T x2[RY];
      uint64_t small2 = 0;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const T xm = shift_in_left(u1m1[r]), xp = shift_in_right(u1m1[r]);
        const T ym = r == 0 ? below : u1m1[r - 1];
        const T yp = r == RY - 1 ? above : u1m1[r + 1];
        T s = xm + xp;
        s = s + ym;
        s = s + yp;
        s = s + u1m2[r];
        s = s + u1[r];
        const bool pt_in = col_in[r] && kin2;
        x2[r] = s + h2 * fm1[r];
        u2[r] = (pt_in && inner2[r]) ? div6_fused(x2[r]) : u1m1[r];
        small2 |= __builtin_amdgcn_ballot_w64(pt_in && inner2[r] && div6_small(x2[r]));
        if (FL & F_RES1) {
          if (inner3[r] && pt_in && kout2) {
            const double res = static_cast<double>(fm1[r]) -
                               (6.0 * static_cast<double>(u1m1[r]) - static_cast<double>(s)) / g.h2;
            acc += res * res;
          }
        }
      }
      if (small2 != 0) {
#pragma unroll
        for (int r = 0; r < RY; ++r)
          if (col_in[r] && kin2 && inner2[r] && div6_small(x2[r])) u2[r] = x2[r] / T(6);
      }
    }
    // stage 3: u3 at plane k-2 (from u2 at k-3, k-2, k-1); the u2 edge rows
    // of plane k-2 were written in the previous step
    if (k - 2 >= k0) {
      const T below = wlo ? T(0) : sm.e2[P2][wdn][1][lane];
      const T above = whi ? T(0) : sm.e2[P2][wup][0][lane];
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const T xm = shift_in_left(u2m1[r]), xp = shift_in_right(u2m1[r]);
        if (inner3[r]) {
          const T ym = r == 0 ? below : u2m1[r - 1];
          const T yp = r == RY - 1 ? above : u2m1[r + 1];
          T s = xm + xp;
          s = s + ym;
          s = s + yp;
          s = s + u2m2[r];
          s = s + u2[r];
          st[r] = div6(s + h2 * fm2[r]);
          if (FL & F_RES2) {
            if (col_in[r]) {
              const double res = static_cast<double>(fm2[r]) -
                                 (6.0 * static_cast<double>(u2m1[r]) - static_cast<double>(s)) / g.h2;
              acc += res * res;
            }
          }
        }
      }
    }
    sm.e2[P][wy][0][lane] = u2[0];
    sm.e2[P][wy][1][lane] = u2[RY - 1];
  };
  // k runs from k0 - 2 to k1 + 1; the bounds are the same for the whole
  // workgroup, so every wavefront takes the same steps and barriers.
  for (int k = k0 - 2; k <= k1 + 1; k += 3) {
    step(std::integral_constant<int, 0>(), k, u0A, u0B, u0C, fA, fB, fC, u1A, u1B, u1C, u2A, u2B, u2C);
    if (k + 1 > k1 + 1) break;
    step(std::integral_constant<int, 1>(), k + 1, u0B, u0C, u0A, fB, fC, fA, u1B, u1C, u1A, u2B, u2C, u2A);
    if (k + 2 > k1 + 1) break;
    step(std::integral_constant<int, 2>(), k + 2, u0C, u0A, u0B, fC, fA, fB, u1C, u1A, u1B, u2C, u2A, u2B);
  }
  flush(k1 - 1);  // the last step computed u3 of plane k1 - 1

  if (RES_ANY != 0) {
    const double tot = block_sum<BY>(acc, sm.red);
    if (wy == 0 && lane == 0) partials[g.tile0 + t] = tot;
  }
  __syncthreads();
}

template <typename T, int BY, int VAR, unsigned FL>
__global__ void __launch_bounds__(WAVE * BY)
    k_sweep3_one(GridArgs g, double* __restrict__ partials, const int* __restrict__ done) {
  if (done != nullptr && *done != 0) return;
  __shared__ Smem3<T, BY> sm;
  const int ntiles = g.tiles_x * g.tiles_y * g.tiles_z;
  if (g.order == 0) {
    for (int t = xcd_remap(blockIdx.x, gridDim.x); t < ntiles; t += gridDim.x)
      sweep3_tile<T, BY, VAR, FL>(g, t, partials, sm);
  } else {
    const int nv = virtual_tiles(ntiles, g.order, g.chunk);
    for (int vb = blockIdx.x; vb < nv; vb += gridDim.x) {
      const int t = g.order == 2 ? xcd_chunked(vb, g.chunk) : vb;
      if (t < ntiles) sweep3_tile<T, BY, VAR, FL>(g, t, partials, sm);
    }
  }
}

// The three-sweep pass over a table of grids: grid g owns tiles
// [table[g].tile0, table[g].tile0 + tiles(g)) of one flat list (found by
// binary search over tile0), as the two-sweep batched pass.
template <typename T, int BY, int VAR, unsigned FL>
__global__ void __launch_bounds__(WAVE * BY)
    k_sweep3_batch(const GridArgs* __restrict__ table, int ngrids, int ntiles, double* __restrict__ partials,
                   const int* __restrict__ done, int order, int chunk, const TileSlot* __restrict__ slots) {
  __shared__ Smem3<T, BY> sm;
  if (slots != nullptr) {
    // one workgroup per slot: the tile and its grid come with the slot
    const TileSlot s = slots[blockIdx.x];
    if (s.tile < 0 || (done != nullptr && done[table[s.grid].id] != 0)) return;
    const GridArgs g = table[s.grid];
    sweep3_tile<T, BY, VAR, FL>(g, s.tile - g.tile0, partials, sm);
    return;
  }
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
    sweep3_tile<T, BY, VAR, FL>(g, t - g.tile0, partials, sm);
  }
}

// Instantiated three-sweep shapes: one wavefront along x, 2, 4, 8 or 16
// wavefronts of 2 or 4 rows per thread (blocks of 8 to 32 rows),
// nontemporal stores.
constexpr bool shape3_instantiated(int by, int var) {
  const int tr = by * rows_per_thread(var);
  const bool by_ok = by == 2 || by == 4 || by == 8 || by == 16;
  return (var == 6 || var == 20) && tr >= 8 && tr <= 32 && by_ok;
}

template <typename T, int BY, int VAR, unsigned FL>
hipError_t go3(const GridArgs& g, double* partials, const int* done, hipStream_t st) {
  if constexpr (!shape3_instantiated(BY, VAR)) {
    return hipErrorInvalidValue;
  } else {
    const int grid = virtual_tiles(g.tiles_x * g.tiles_y * g.tiles_z, g.order, g.chunk);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_sweep3_one<T, BY, VAR, FL>), dim3(grid), dim3(WAVE, BY), 0, st, g, partials, done);
    return hipGetLastError();
  }
}

// Batched launch: one workgroup per tile of the flat list (order 0 remaps
// blocks to XCDs, order 2 chunks the list per XCD in runs of kBatchChunk).
template <typename T, int BY, int VAR, unsigned FL>
hipError_t go3_batch(const TileCfg& c, const GridArgs* table, int ngrids, int ntiles, const TileSlot* slots,
                     int nslots, double* partials, const int* done, hipStream_t st) {
  if constexpr (!shape3_instantiated(BY, VAR)) {
    return hipErrorInvalidValue;
  } else {
    const int chunk = kBatchChunk;
    const int grid = slots != nullptr ? nslots : virtual_tiles(ntiles, c.order, chunk);
    if (grid <= 0 || ngrids <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_sweep3_batch<T, BY, VAR, FL>), dim3(grid), dim3(WAVE, BY), 0, st, table, ngrids,
                       ntiles, partials, done, c.order, chunk, slots);
    return hipGetLastError();
  }
}

template <typename T, unsigned FL>
hipError_t by_shape3_batch(const TileCfg& c, const GridArgs* table, int ngrids, int ntiles, const TileSlot* slots,
                           int nslots, double* partials, const int* done, hipStream_t st) {
  switch (c.rows * 100 + c.variant) {
    case 206: return go3_batch<T, 2, 6, FL>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case 220: return go3_batch<T, 2, 20, FL>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case 406: return go3_batch<T, 4, 6, FL>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case 420: return go3_batch<T, 4, 20, FL>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case 806: return go3_batch<T, 8, 6, FL>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case 820: return go3_batch<T, 8, 20, FL>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    case 1606: return go3_batch<T, 16, 6, FL>(c, table, ngrids, ntiles, slots, nslots, partials, done, st);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, unsigned FL>
hipError_t by_shape3(const TileCfg& c, const GridArgs& g, double* partials, const int* done, hipStream_t st) {
  switch (c.rows * 100 + c.variant) {
    case 206: return go3<T, 2, 6, FL>(g, partials, done, st);
    case 220: return go3<T, 2, 20, FL>(g, partials, done, st);
    case 406: return go3<T, 4, 6, FL>(g, partials, done, st);
    case 420: return go3<T, 4, 20, FL>(g, partials, done, st);
    case 806: return go3<T, 8, 6, FL>(g, partials, done, st);
    case 820: return go3<T, 8, 20, FL>(g, partials, done, st);
    case 1606: return go3<T, 16, 6, FL>(g, partials, done, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch_sweep3_f64(unsigned flags, const TileCfg& c, const GridArgs& g, double* partials,
                               const int* done, hipStream_t st);
hipError_t dispatch_sweep3_f32(unsigned flags, const TileCfg& c, const GridArgs& g, double* partials,
                               const int* done, hipStream_t st);
hipError_t dispatch_sweep3_batch_f64(unsigned flags, const TileCfg& c, const GridArgs* table, int ngrids,
                                     int ntiles, const TileSlot* slots, int nslots, double* partials,
                                     const int* done, hipStream_t st);
hipError_t dispatch_sweep3_batch_f32(unsigned flags, const TileCfg& c, const GridArgs* table, int ngrids,
                                     int ntiles, const TileSlot* slots, int nslots, double* partials,
                                     const int* done, hipStream_t st);

}  // namespace sweep_detail
}  // namespace j3d
