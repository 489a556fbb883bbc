// The z-marching tile kernel shared by every sweep-shaped pass of libj3d
// (FP64 sweep, fused residual, defect residual, FP32 correction sweeps,
// norms), its single-grid and batched entry points, and the launch
// templates.  Included by kernels_f64.hip and kernels_f32.hip, which
// instantiate it for their element type.
//
// Memory layout: Fortran column-major arrays with a one-cell halo; x is the
// unit-stride axis.  A workgroup owns a tile of 64*WX x-points (WX 64-lane
// wavefronts side by side) by BY*RY y-rows by `planes` z-planes and marches through
// z, keeping the previous, current and next value of its column in
// registers, so every plane of u and f is fetched from HBM once per tile.
// The sweep streams about 24 bytes per FP64 point update and does 8 flops,
// far below the ridge of the FP64 VALU: it is HBM-bound and there is no dense
// contraction, hence no MFMA.
//
// VAR selects how the tile is fed (bits may be combined):
//   1  the current plane is staged in LDS with its x/y halo ring
//      (double-buffered, one barrier per plane); otherwise x-neighbours come
//      from the adjacent lanes of the wavefront by DPP wave shifts (the two
//      halo columns from one gather load per plane) and the y-neighbours at
//      the block's edge rows through the vector caches;
//   2, 16  each thread owns 2^(bit2 + 2*bit16) consecutive rows (1, 2, 4 or
//      8): register blocking in y, which multiplies the independent HBM
//      loads each wavefront has in flight per plane;
//   4  outputs are written with nontemporal stores (streamed past L2).
//
// Arithmetic order is fixed and the library is built with contraction off:
//   S  = ((((u[i-1] + u[i+1]) + u[j-1]) + u[j+1]) + u[k-1]) + u[k+1]
//   u' = (S + h2 * f) / 6                  (the IEEE quotient, see div6)
//   r  = f - (6 * u - S) / h2              (FP64)
// A tile's sum of r^2 is reduced by a fixed butterfly within the wavefront
// and in wave order across wavefronts into one fixed slot per tile.
#pragma once

#include "j3d_internal.h"

namespace j3d {
namespace sweep_detail {

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2); dispatch index b runs on XCD b % 8.  Three orders map dispatch
// indices to tiles:
//   0  each XCD receives one contiguous block of all tiles (halo rows stay in
//      one L2, but the XCDs stream from 8 distant regions);
//   1  as launched (all XCDs stream one region together; neighbouring tiles
//      land on different XCDs);
//   2  the tiles are cut into groups of 8*chunk (about one z-slab of one
//      grid); within a group XCD x takes the contiguous chunk x, so all XCDs
//      stream the same slab while each keeps its own neighbours in its L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, idx = b >> 3;
  return x * q + min(x, r) + idx;
}

__device__ __forceinline__ int xcd_chunked(int vb, int chunk) {
  const int x = vb & 7, idx = vb >> 3;
  return (idx / chunk) * 8 * chunk + x * chunk + (idx % chunk);
}

// Number of dispatch indices that cover ntiles tiles under an order.
__host__ __device__ __forceinline__ int virtual_tiles(int ntiles, int order, int chunk) {
  return order == 2 ? (ntiles + 8 * chunk - 1) / (8 * chunk) * (8 * chunk) : ntiles;
}

template <typename T>
__device__ __forceinline__ T h2_of(const GridArgs& g);
template <>
__device__ __forceinline__ double h2_of<double>(const GridArgs& g) { return g.h2; }
template <>
__device__ __forceinline__ float h2_of<float>(const GridArgs& g) { return g.h2f; }

template <typename T, bool NT>
__device__ __forceinline__ void put(T* p, T v) {
  if (NT)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

typedef int dpp_i2 __attribute__((ext_vector_type(2)));

// The value of lane l-1 (from_left) or l+1 (from_right) of the wavefront;
// lane 0 (resp. 63) gets its own value.  DPP wave_shr:1 / wave_shl:1; every
// lane of the wavefront must execute the call.
__device__ __forceinline__ float from_left(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, v),
                                                               __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, false));
}
__device__ __forceinline__ float from_right(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, v),
                                                               __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, false));
}
__device__ __forceinline__ double from_left(double v) {
  const dpp_i2 a = __builtin_bit_cast(dpp_i2, v);
  dpp_i2 r;
  r.x = __builtin_amdgcn_update_dpp(a.x, a.x, 0x138, 0xF, 0xF, false);
  r.y = __builtin_amdgcn_update_dpp(a.y, a.y, 0x138, 0xF, 0xF, false);
  return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ double from_right(double v) {
  const dpp_i2 a = __builtin_bit_cast(dpp_i2, v);
  dpp_i2 r;
  r.x = __builtin_amdgcn_update_dpp(a.x, a.x, 0x130, 0xF, 0xF, false);
  r.y = __builtin_amdgcn_update_dpp(a.y, a.y, 0x130, 0xF, 0xF, false);
  return __builtin_bit_cast(double, r);
}

// The value lane `src` (a constant) of the wavefront holds, in every lane.
__device__ __forceinline__ float lane_value(float v, int src) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), src));
}
__device__ __forceinline__ double lane_value(double v, int src) {
  const dpp_i2 a = __builtin_bit_cast(dpp_i2, v);
  dpp_i2 r;
  r.x = __builtin_amdgcn_readlane(a.x, src);
  r.y = __builtin_amdgcn_readlane(a.y, src);
  return __builtin_bit_cast(double, r);
}

// x / 6 rounded to nearest, without a division instruction, by the method
// of Brisebarre, Muller and Raina for a divisor known in advance (IEEE
// Trans. Computers 53(8), 2004): with zh = RN(1/6) and zl = RN(1/6 - zh),
// q = RN(x * zh + RN(x * zl)) in one fused multiply-add.  It equals the IEEE
// quotient x / 6 for every x whose quotient is normal: x = m 2^e with an
// integer m makes x / 6 = (m / 3) 2^(e-1) a multiple of a third of its own
// ulp, so it lies at least ulp / 6 from every rounding boundary, while the
// fused value differs from x / 6 by less than 2^-20 ulp.  Below that range
// (|x| < 2^-1000 in FP64, 2^-100 in FP32, where the quotient may be
// subnormal and a tie possible) the lane divides.  Infinities, NaNs and
// signed zeros come out as the division gives them.  The library is
// otherwise built without contraction; this fma is explicit.
__device__ __forceinline__ double div6(double x) {
  const double q = __builtin_fma(x, 0x1.5555555555555p-3, x * 0x1.5555555555555p-57);
  if (__builtin_fabs(x) < 0x1p-1000) return x / 6.0;
  return q;
}
__device__ __forceinline__ float div6(float x) {
  const float q = __builtin_fmaf(x, 0x1.555556p-3f, x * -0x1.555556p-28f);
  if (__builtin_fabsf(x) < 0x1p-100f) return x / 6.0f;
  return q;
}

// div6 in two parts, for code that tests a whole row block at once: the
// fused quotient, and whether x lies below the range where it is exact
// (then the quotient must come from the division instead).
__device__ __forceinline__ double div6_fused(double x) {
  return __builtin_fma(x, 0x1.5555555555555p-3, x * 0x1.5555555555555p-57);
}
__device__ __forceinline__ float div6_fused(float x) {
  return __builtin_fmaf(x, 0x1.555556p-3f, x * -0x1.555556p-28f);
}
__device__ __forceinline__ bool div6_small(double x) { return __builtin_fabs(x) < 0x1p-1000; }
__device__ __forceinline__ bool div6_small(float x) { return __builtin_fabsf(x) < 0x1p-100f; }

// Buffer resource for a wave-uniform base address: every load and store of
// a plane then takes the plane's address in scalar registers and a per-lane
// 32-bit byte offset that is fixed for the whole tile, so the z march needs
// no per-lane address arithmetic.  The descriptor's range is the largest it
// allows (4 GiB past the base; a plane of the three-sweep pass is smaller,
// which the host checks); the kernel keeps every access inside the array
// itself, as with plain pointers.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, -1, 0x00020000);
}

typedef unsigned buf_u2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <>
__device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
template <>
__device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

// Store; NT streams it past the caches (cache policy "nt").
template <typename T, bool NT>
__device__ __forceinline__ void bstore(T v, __amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(T) == 8)
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(buf_u2, v), r, off, 0, NT ? 2 : 0);
  else
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, NT ? 2 : 0);
}

// Rows per thread encoded in the variant bits 2 and 16.
constexpr int rows_per_thread(int var) { return 1 << (((var >> 1) & 1) + 2 * ((var >> 4) & 1)); }

// Shared memory of a workgroup: the double-buffered plane with its x/y halo
// ring (LDS variants only; one element otherwise) and one partial sum per
// wavefront.
template <typename T, int BY, int WX, int VAR>
struct Smem {
  static constexpr bool LDS = (VAR & 1) != 0;
  static constexpr int TR = BY * rows_per_thread(VAR);
  T pl[LDS ? 2 : 1][LDS ? TR + 2 : 1][LDS ? WAVE * WX + 2 : 1];
  double red[BY * WX];
};

// Sum of one double per wavefront of the workgroup: a fixed butterfly within
// each wavefront, then the wavefront sums in wavefront order.  The result is
// valid in thread (0, 0).
template <int NW>
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.y * (blockDim.x / WAVE) + threadIdx.x / WAVE;
  if ((threadIdx.x & (WAVE - 1)) == 0) red[w] = v;
  __syncthreads();
  double tot = 0.0;
  if (threadIdx.x == 0 && threadIdx.y == 0) {
#pragma unroll
    for (int q = 0; q < NW; ++q) tot += red[q];
  }
  return tot;
}

// Offset that puts a buffer access out of range: the buffer-addressed path
// runs only on grids whose planes are all shorter than 2^31 bytes
// (GridArgs::wide_planes == 0), and the hardware drops stores whose offset
// lies past the resource's range, so a store given this offset writes
// nothing.
constexpr uint32_t kDropOffset = 0x80000000u;

// Buffer resource for plane kk of an array with base b and plane stride z
// bytes, covering rec bytes (the plane's interior and halo).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc_n(const void* b, uint64_t z, int kk, uint32_t rec) {
  return __builtin_amdgcn_make_buffer_rsrc(
      const_cast<char*>(static_cast<const char*>(b)) + (uint64_t)(uint32_t)kk * z, 0, (int)rec, 0x00020000);
}

// One tile of the cache-fed variants (x-neighbours from the adjacent lanes,
// the wavefront's two halo columns from one gather, y-neighbours from
// registers inside the row block and two edge loads outside it).
//
// Loads run one plane ahead: step k takes the loads issued one step
// earlier (its one wait), issues the loads of plane k+1, stores the results
// of step k-1 and computes plane k, so the loads it waits for had a whole
// step of arithmetic to arrive, and the stores it issues are waited for
// only at the start of the next step.  Every lane issues every memory
// operation of every step: loads come from in-bounds addresses (lanes and
// rows past the interior are clamped onto the halo; the last step reloads
// its own plane), stores of masked lanes (and the empty store of the first
// step) are given an out-of-range offset and dropped by the hardware.  The
// loop therefore has no branches around memory operations, which lets the
// compiler count exactly which loads a wait needs.  Addresses are a scalar
// per-plane buffer resource plus a per-lane byte offset fixed for the tile.
// The arithmetic and its order are those of the LDS variant (same bits).
template <typename T, int BY, int WX, int VAR, unsigned FL>
__device__ __forceinline__ void sweep_tile_cf(const GridArgs& g, int t, double* __restrict__ partials,
                                              Smem<T, BY, WX, VAR>& sm) {
  constexpr bool STENCIL = !(FL & (F_FIRST | F_NORM));
  constexpr int RY = rows_per_thread(VAR);
  constexpr int TX = WAVE * WX;
  constexpr bool NT = (VAR & 4) != 0;
  constexpr bool OUT = (FL & (F_WRITE | F_LAST | F_R32)) != 0;
  constexpr uint32_t ES = sizeof(T);
  const int lane = threadIdx.x;
  const int wy = __builtin_amdgcn_readfirstlane(threadIdx.y);
  const int tx = t % g.tiles_x;
  const int t2 = t / g.tiles_x;
  const int ty = t2 % g.tiles_y;
  const int tz = t2 / g.tiles_y;
  const int i = 1 + tx * TX + lane;
  const int jb = 1 + ty * (BY * RY) + wy * RY;  // first row of this thread
  const int k0 = 1 + tz * g.planes;
  const int k1 = min(k0 + g.planes, g.nz + 1);
  const bool ix = i <= g.nx;
  const int ic = min(i, g.nx + 1);  // lanes past the interior read the halo column

  // byte offsets within a plane: rows jb .. jb+RY-1 clamped onto the halo
  // row ny+1 (so the register of row r+1 is the y-neighbour of row r on
  // every interior row), stores of rows and lanes outside the interior
  // dropped
  uint32_t ou[RY], of[RY], oo[RY], orr[RY], oq[RY];
  bool act[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    const int y = min(jb + r, g.ny + 1);
    act[r] = ix && (jb + r <= g.ny);
    ou[r] = (uint32_t)(ic + g.su_y * y) * ES;
    of[r] = (uint32_t)(ic + g.sf_y * y) * ES;
    oo[r] = act[r] ? (uint32_t)(ic + g.so_y * y) * ES : kDropOffset;
    orr[r] = act[r] ? (uint32_t)(ic + g.sr_y * y) * 4u : kDropOffset;
    oq[r] = (uint32_t)(ic + g.s64_y * y) * 8u;
  }
  // the halo gather: lane q < RY reads the column left of the wavefront in
  // row q, lane 32 + q the column right of it; the other lanes read a
  // clamped row of the same columns, whose values go unused
  const int lw = lane & (WAVE - 1);
  const int xw = 1 + tx * TX + (lane - lw);
  const int gq = lw < 32 ? lw : lw - 32;
  const int gx = lw < 32 ? xw - 1 : min(xw + WAVE, g.nx + 1);
  const uint32_t oh = (uint32_t)(gx + g.su_y * min(jb + min(gq, RY - 1), g.ny + 1)) * ES;
  const uint32_t ob = (uint32_t)(ic + g.su_y * (min(jb, g.ny) - 1)) * ES;
  const uint32_t oa = (uint32_t)(ic + g.su_y * min(jb + RY, g.ny + 1)) * ES;

  // planes: a resource per array and plane, each covering the plane's
  // interior and halo
  const uint32_t nxy = (uint32_t)(g.nx + 1);
  const uint32_t ru = (nxy + (uint32_t)g.su_y * (uint32_t)(g.ny + 1) + 1u) * ES;
  const uint32_t rf = (nxy + (uint32_t)g.sf_y * (uint32_t)(g.ny + 1) + 1u) * ES;
  const uint32_t ro = (nxy + (uint32_t)g.so_y * (uint32_t)(g.ny + 1) + 1u) * ES;
  const uint32_t rr = (nxy + (uint32_t)g.sr_y * (uint32_t)(g.ny + 1) + 1u) * 4u;
  const uint32_t rq = (nxy + (uint32_t)g.s64_y * (uint32_t)(g.ny + 1) + 1u) * 8u;
  const uint64_t zu = (uint64_t)g.su_z * ES, zf = (uint64_t)g.sf_z * ES, zo = (uint64_t)g.so_z * ES;
  const uint64_t zr = (uint64_t)g.sr_z * 4, zq = (uint64_t)g.s64_z * 8;
  const T h2 = h2_of<T>(g);

  double acc = 0.0;
  T um[RY], uc[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    um[r] = uc[r] = T(0);
    if (STENCIL) {
      um[r] = bload<T>(plane_rsrc_n(g.u, zu, k0 - 1, ru), ou[r]);
      uc[r] = bload<T>(plane_rsrc_n(g.u, zu, k0, ru), ou[r]);
    }
  }

  // the loads a step consumes: f at its plane, u one plane above, the halo
  // gather and the rows below and above the block at its plane, and (F_LAST)
  // the FP64 values the update is added to
  struct Loads {
    T f[RY], u[RY], halo, below, above;
    double q[RY];
  };
  auto issue = [&](Loads& L, int kk) {
    const auto pf = plane_rsrc_n(g.f, zf, kk, rf);
#pragma unroll
    for (int r = 0; r < RY; ++r) L.f[r] = bload<T>(pf, of[r]);
    if (STENCIL) {
      const auto pu1 = plane_rsrc_n(g.u, zu, kk + 1, ru);
      const auto pu0 = plane_rsrc_n(g.u, zu, kk, ru);
#pragma unroll
      for (int r = 0; r < RY; ++r) L.u[r] = bload<T>(pu1, ou[r]);
      L.halo = bload<T>(pu0, oh);
      L.below = bload<T>(pu0, ob);
      L.above = bload<T>(pu0, oa);
    }
    if (FL & F_LAST) {
      const auto pq = plane_rsrc_n(g.u64, zq, kk, rq);
#pragma unroll
      for (int r = 0; r < RY; ++r) L.q[r] = bload<double>(pq, oq[r]);
    }
  };
  // results of the previous step, stored at the start of the next one
  T sv[RY];
  float sr[RY];
  double sq[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    sv[r] = T(0);
    sr[r] = 0.0f;
    sq[r] = 0.0;
  }
  auto flush = [&](int kk, bool any) {
    if (FL & F_WRITE) {
      const auto p = plane_rsrc_n(g.o, zo, kk, ro);
#pragma unroll
      for (int r = 0; r < RY; ++r) bstore<T, NT>(sv[r], p, any ? oo[r] : kDropOffset);
    }
    if (FL & F_R32) {
      const auto p = plane_rsrc_n(g.r32, zr, kk, rr);
#pragma unroll
      for (int r = 0; r < RY; ++r) bstore<float, NT>(sr[r], p, any ? orr[r] : kDropOffset);
    }
    if (FL & F_LAST) {
      const auto p = plane_rsrc_n(g.u64, zq, kk, rq);
#pragma unroll
      for (int r = 0; r < RY; ++r) bstore<double, false>(sq[r], p, any && act[r] ? oq[r] : kDropOffset);
    }
  };
  // plane k from the loads in L
  auto compute = [&](const Loads& L) {
    T s[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      s[r] = T(0);
      if (STENCIL) {
        T xm = from_left(uc[r]), xp = from_right(uc[r]);
        const T hl = lane_value(L.halo, r), hr = lane_value(L.halo, 32 + r);
        if (lw == 0) xm = hl;
        if (lw == WAVE - 1) xp = hr;
        const T ym = r == 0 ? L.below : uc[r - 1];
        const T yp = r + 1 < RY ? uc[r + 1] : L.above;
        T v = xm + xp;
        v = v + ym;
        v = v + yp;
        v = v + um[r];
        v = v + L.u[r];
        s[r] = v;
      }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      if (FL & F_NORM) {
        const double v = static_cast<double>(L.f[r]) * static_cast<double>(L.f[r]);
        acc += act[r] ? v : 0.0;
      }
      if (STENCIL && (FL & (F_RES | F_R32))) {
        const double res = static_cast<double>(L.f[r]) -
                           (6.0 * static_cast<double>(uc[r]) - static_cast<double>(s[r])) / g.h2;
        if (FL & F_RES) acc += act[r] ? res * res : 0.0;
        sr[r] = static_cast<float>(res);
      }
    }
    if (FL & (F_WRITE | F_LAST)) {
      // the quotients by 6 in their fused form, then the rare exact
      // divisions (see div6)
      T x[RY];
      uint64_t small = 0;
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        x[r] = s[r] + h2 * L.f[r];
        sv[r] = div6_fused(x[r]);
        small |= __builtin_amdgcn_ballot_w64(div6_small(x[r]));
      }
      if (small != 0) {
#pragma unroll
        for (int r = 0; r < RY; ++r) sv[r] = div6(x[r]);
      }
      if (FL & F_LAST) {
#pragma unroll
        for (int r = 0; r < RY; ++r) sq[r] = L.q[r] + static_cast<double>(sv[r]);
      }
    }
    if (STENCIL) {
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        um[r] = uc[r];
        uc[r] = L.u[r];
      }
    }
  };

  // N: the loads in flight; C: the ones the step consumes (taking them is
  // the step's one wait)
  Loads N, C;
  issue(N, k0);
  for (int k = k0; k < k1; ++k) {
    C = N;
    issue(N, min(k + 1, k1 - 1));
    if (OUT) flush(k - 1, k > k0);
    compute(C);
  }
  if (OUT) flush(k1 - 1, true);

  if (FL & (F_RES | F_NORM)) {
    const double tot = block_sum<BY * WX>(acc, sm.red);
    if (wy == 0 && lane == 0) partials[g.tile0 + t] = tot;
  }
  // The next tile of a persistent workgroup reuses the shared buffers.
  __syncthreads();
}

// One tile: local tile index t of grid g.  Writes the tile's partial sum
// (F_RES / F_NORM) to partials[g.tile0 + t].  The cache-fed variants run
// sweep_tile_cf unless a plane of the grid spans 2^31 bytes or more; this
// pointer-addressed body serves the LDS variants and those grids.
//
// Each thread owns RY consecutive rows of its column (register blocking in
// y as well as z): per plane it issues the 2*RY HBM loads of its rows at
// once, the y-neighbours inside its block come from registers and, in the
// cache-fed variants, the x-neighbours from the adjacent lanes.  Every lane
// loads from in-bounds addresses (lanes and rows past the interior are
// clamped onto the halo column/row), so loads need no per-lane branches;
// only stores and sums are masked.
template <typename T, int BY, int WX, int VAR, unsigned FL>
__device__ __forceinline__ void sweep_tile(const GridArgs& g, int t, double* __restrict__ partials,
                                           Smem<T, BY, WX, VAR>& sm) {
  constexpr bool STENCIL = !(FL & (F_FIRST | F_NORM));
  constexpr bool USE_LDS = (VAR & 1) && STENCIL;
  constexpr int RY = rows_per_thread(VAR);
  constexpr int TR = BY * RY;      // rows per tile
  constexpr int TX = WAVE * WX;    // columns per tile
  constexpr bool NT = (VAR & 4) != 0;
  if constexpr ((VAR & 1) == 0) {
    if (g.wide_planes == 0) {
      sweep_tile_cf<T, BY, WX, VAR, FL>(g, t, partials, sm);
      return;
    }
  }
  const int lane = threadIdx.x;    // column within the tile
  const int wy = threadIdx.y;
  const int tx = t % g.tiles_x;
  const int t2 = t / g.tiles_x;
  const int ty = t2 % g.tiles_y;
  const int tz = t2 / g.tiles_y;
  const int i = 1 + tx * TX + lane;
  const int jb = 1 + ty * TR + wy * RY;  // first row of this thread
  const int k0 = 1 + tz * g.planes;
  const int k1 = min(k0 + g.planes, g.nz + 1);
  const bool ix = i <= g.nx;
  const int ic = min(i, g.nx + 1);  // lanes past the interior read the halo column
  const int jc = min(jb, g.ny);

  // Row r of the block is row jb + r, clamped onto the halo row ny+1; dj[r]
  // is its offset in rows from row jc (uniform across the wavefront).  With
  // the clamp, the register holding row r+1 is the correct y-neighbour of
  // row r for every interior row.
  int dj[RY];
  bool act[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    dj[r] = min(jb + r, g.ny + 1) - jc;
    act[r] = ix && (jb + r <= g.ny);
  }
  // Cache-fed stencil: x-neighbours come from the adjacent lanes (DPP), the
  // two halo columns of the wavefront's rows from one gather per plane: lane
  // q < RY loads the column left of the wavefront in row q, lane 32 + q the
  // column right of it.
  const int lw = lane & (WAVE - 1);
  const int xw = 1 + tx * TX + (lane - lw);  // first column of this wavefront
  const int gq = lw < 32 ? lw : lw - 32;
  const bool gat = gq < RY;
  const int goff = (lw < 32 ? xw - 1 : min(xw + WAVE, g.nx + 1)) - ic +
                   (min(jb + min(gq, RY - 1), g.ny + 1) - jc) * g.su_y;
  const int yhi_off = (min(jb + RY, g.ny + 1) - jc) * g.su_y;

  const T* __restrict__ pu = static_cast<const T*>(g.u) + (ic + g.su_y * jc + g.su_z * k0);
  const T* __restrict__ pf = static_cast<const T*>(g.f) + (ic + g.sf_y * jc + g.sf_z * k0);
  T* __restrict__ po = static_cast<T*>(g.o) + (ic + g.so_y * jc + g.so_z * k0);
  float* __restrict__ pr = g.r32 + (ic + g.sr_y * jc + g.sr_z * k0);
  double* __restrict__ p64 = g.u64 + (ic + g.s64_y * jc + g.s64_z * k0);
  const T h2 = h2_of<T>(g);

  double acc = 0.0;
  T um[RY], uc[RY];
#pragma unroll
  for (int r = 0; r < RY; ++r) {
    um[r] = T(0);
    uc[r] = T(0);
    if (STENCIL) {
      um[r] = pu[dj[r] * g.su_y - g.su_z];
      uc[r] = pu[dj[r] * g.su_y];
    }
  }

  for (int k = k0; k < k1; ++k) {
    T fc[RY], up[RY], xm[RY], xp[RY], ym[RY], yp[RY];
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      const T* u_r = pu + dj[r] * g.su_y;
      fc[r] = pf[dj[r] * g.sf_y];
      up[r] = STENCIL ? u_r[g.su_z] : T(0);
      xm[r] = xp[r] = ym[r] = yp[r] = T(0);
    }
    if (STENCIL && !USE_LDS) {
      const T halo = gat ? pu[goff] : T(0);
      const T below = pu[-g.su_y];
      const T above = pu[yhi_off];
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        xm[r] = from_left(uc[r]);
        xp[r] = from_right(uc[r]);
        const T hl = lane_value(halo, r), hr = lane_value(halo, 32 + r);
        if (lw == 0) xm[r] = hl;
        if (lw == WAVE - 1) xp[r] = hr;
        // y-neighbours: registers inside the block, loads at its edges.
        ym[r] = r == 0 ? below : uc[r - 1];
        yp[r] = r + 1 < RY ? uc[r + 1] : above;
      }
    }
    if (USE_LDS) {
      auto& pl = sm.pl[(k - k0) & 1];
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        if (act[r]) {
          const T* u_r = pu + dj[r] * g.su_y;
          const int row = wy * RY + r + 1;
          pl[row][lane + 1] = uc[r];
          if (lane == 0) pl[row][0] = u_r[-1];
          if (lane == TX - 1 || i == g.nx) pl[row][lane + 2] = u_r[1];
          if (row == 1) pl[0][lane + 1] = u_r[-g.su_y];
          if (row == TR || jb + r == g.ny) pl[row + 1][lane + 1] = u_r[g.su_y];
        }
      }
      __syncthreads();
#pragma unroll
      for (int r = 0; r < RY; ++r) {
        const int row = wy * RY + r + 1;
        xm[r] = pl[row][lane];
        xp[r] = pl[row][lane + 2];
        ym[r] = pl[row - 1][lane + 1];
        yp[r] = pl[row + 1][lane + 1];
      }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      T s = T(0);
      if (STENCIL) {
        s = xm[r] + xp[r];
        s = s + ym[r];
        s = s + yp[r];
        s = s + um[r];
        s = s + up[r];
      }
      if (FL & F_NORM) {
        const double v = static_cast<double>(fc[r]) * static_cast<double>(fc[r]);
        acc += act[r] ? v : 0.0;
      } else {
        if (STENCIL && (FL & (F_RES | F_R32))) {
          const double res = static_cast<double>(fc[r]) -
                             (6.0 * static_cast<double>(uc[r]) - static_cast<double>(s)) / g.h2;
          if (FL & F_RES) acc += act[r] ? res * res : 0.0;
          if ((FL & F_R32) && act[r]) put<float, NT>(pr + dj[r] * g.sr_y, static_cast<float>(res));
        }
        if (FL & (F_WRITE | F_LAST)) {
          const T v = div6(s + h2 * fc[r]);
          if ((FL & F_WRITE) && act[r]) put<T, NT>(po + dj[r] * g.so_y, v);
          if ((FL & F_LAST) && act[r]) {
            double* q = p64 + dj[r] * g.s64_y;
            q[0] = q[0] + static_cast<double>(v);
          }
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RY; ++r) {
      um[r] = uc[r];
      uc[r] = up[r];
    }
    pu += g.su_z;
    pf += g.sf_z;
    po += g.so_z;
    pr += g.sr_z;
    p64 += g.s64_z;
  }

  if (FL & (F_RES | F_NORM)) {
    const double tot = block_sum<BY * WX>(acc, sm.red);
    if (wy == 0 && lane == 0) partials[g.tile0 + t] = tot;
  }
  // The next tile of a persistent workgroup reuses the shared buffers.
  __syncthreads();
}

// The previous pass's check (PreReduce), reduced by one workgroup of any
// size that divides 1024 into the same bits as the 1024-thread reduction
// kernels: thread t stands in for threads t, t + T, t + 2T, ... of those,
// each with its own sum in slot order, and the wavefront butterflies and
// the sums of the 16 wavefronts follow in the same order.
__device__ __forceinline__ void pre_reduce(const PreReduce& pr) {
  constexpr int VT = 1024;  // threads of the reduction kernels
  __shared__ double ws[VT / WAVE];
  const int T = blockDim.x * blockDim.y;
  const int t = threadIdx.y * blockDim.x + threadIdx.x;
  for (int q = t; q < VT; q += T) {
    double a = 0.0;
    for (int m = q; m < pr.n; m += VT) a += pr.partials[m];
    a = wave_sum(a);
    if ((q & (WAVE - 1)) == 0) ws[q / WAVE] = a;
  }
  __syncthreads();
  if (t == 0) {
    double tot = ws[0];
#pragma unroll
    for (int w = 1; w < VT / WAVE; ++w) tot += ws[w];
    const long long q = *pr.qnext;
    const double r = sqrt(tot);
    pr.hist[q] = r;
    const bool bad = !isfinite(r);
    if (bad || r <= pr.rtol * (*pr.normf)) {
      *pr.done = 1;
      *pr.conv_at = q;
      if (bad) *pr.nonfinite = 1;
    }
    *pr.qnext = q + 1;
  }
}

// One pass over one grid; with pr.partials set, the last workgroup reduces
// the previous pass's check instead of taking tiles.
template <typename T, int BY, int WX, int VAR, unsigned FL>
__global__ void __launch_bounds__(WAVE * WX * BY)
    k_pass_one(GridArgs g, double* __restrict__ partials, const int* __restrict__ done, PreReduce pr) {
  if (done != nullptr && *done != 0) return;
  const int nb = (int)gridDim.x - (pr.partials != nullptr ? 1 : 0);  // workgroups taking tiles
  if ((int)blockIdx.x == nb) {
    pre_reduce(pr);
    return;
  }
  __shared__ Smem<T, BY, WX, VAR> sm;
  const int ntiles = g.tiles_x * g.tiles_y * g.tiles_z;
  if (g.order == 0) {
    for (int t = xcd_remap(blockIdx.x, nb); t < ntiles; t += nb)
      sweep_tile<T, BY, WX, VAR, FL>(g, t, partials, sm);
  } else {
    const int nv = virtual_tiles(ntiles, g.order, g.chunk);
    for (int vb = blockIdx.x; vb < nv; vb += nb) {
      const int t = g.order == 2 ? xcd_chunked(vb, g.chunk) : vb;
      if (t < ntiles) sweep_tile<T, BY, WX, VAR, FL>(g, t, partials, sm);
    }
  }
}

template <typename T, int BY, int WX, int VAR, unsigned FL>
__global__ void __launch_bounds__(WAVE * WX * BY)
    k_pass_batch(const GridArgs* __restrict__ table, int ngrids, int ntiles,
                 double* __restrict__ partials, const int* __restrict__ done, int order, int chunk) {
  __shared__ Smem<T, BY, WX, VAR> sm;
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
    sweep_tile<T, BY, WX, VAR, FL>(g, t - g.tile0, partials, sm);
  }
}

// ---------------------------------------------------------------------
// Host-side launch templates
// ---------------------------------------------------------------------

int device_cus();

template <typename K>
int resident_blocks(K kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb <= 0)
    nb = 1;
  return nb * device_cus();
}

// Chunk length of order 2 for batched launches (tiles per XCD per group).
constexpr int kBatchChunk = 32;

struct Launch {
  bool batch;
  const TileCfg* c;
  const GridArgs* one;
  const GridArgs* table;
  int ngrids, ntiles;
  double* partials;
  const int* done;
  hipStream_t st;
  PreReduce pr{};  // one-sweep passes over one grid only
};

template <typename T, int BY, int WX, int VAR, unsigned FL>
hipError_t go(const Launch& L) {
  constexpr int THREADS = WAVE * WX * BY;
  int grid;
  if (L.batch) {
    const int chunk = kBatchChunk;
    grid = virtual_tiles(L.ntiles, L.c->order, chunk);
    if (L.c->persistent) {
      static int cap = 0;
      if (cap == 0) cap = resident_blocks(k_pass_batch<T, BY, WX, VAR, FL>, THREADS);
      grid = min(grid, cap);
    }
    if (grid <= 0 || L.ngrids <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_pass_batch<T, BY, WX, VAR, FL>), dim3(grid), dim3(WAVE * WX, BY), 0, L.st,
                       L.table, L.ngrids, L.ntiles, L.partials, L.done, L.c->order, chunk);
  } else {
    const GridArgs& g = *L.one;
    grid = virtual_tiles(g.tiles_x * g.tiles_y * g.tiles_z, g.order, g.chunk);
    if (L.c->persistent) {
      static int cap = 0;
      if (cap == 0) cap = resident_blocks(k_pass_one<T, BY, WX, VAR, FL>, THREADS);
      grid = min(grid, cap);
    }
    if (grid <= 0) return hipSuccess;
    if (L.pr.partials != nullptr) ++grid;  // the workgroup that reduces the previous check
    hipLaunchKernelGGL((k_pass_one<T, BY, WX, VAR, FL>), dim3(grid), dim3(WAVE * WX, BY), 0, L.st, g,
                       L.partials, L.done, L.pr);
  }
  return hipGetLastError();
}

// Instantiated shapes: one wavefront along x with every variant; two or four
// wavefronts along x (at most 1024 threads) with the cache-fed variants that
// use nontemporal stores and 1, 2 or 4 rows per thread.
constexpr bool shape_instantiated(int by, int wx, int var) {
  if (wx == 1) return true;
  return by * wx <= 16 && (var == 4 || var == 6 || var == 20);
}

template <typename T, int BY, int WX, unsigned FL>
hipError_t by_variant(const Launch& L) {
#define J3D_VAR_CASE(V)                                                      \
  case V:                                                                    \
    if constexpr (shape_instantiated(BY, WX, V)) return go<T, BY, WX, V, FL>(L); \
    else return hipErrorInvalidValue;
  switch (L.c->variant) {
    J3D_VAR_CASE(0) J3D_VAR_CASE(1) J3D_VAR_CASE(2) J3D_VAR_CASE(3)
    J3D_VAR_CASE(4) J3D_VAR_CASE(5) J3D_VAR_CASE(6) J3D_VAR_CASE(7)
    J3D_VAR_CASE(16) J3D_VAR_CASE(17) J3D_VAR_CASE(18) J3D_VAR_CASE(19)
    J3D_VAR_CASE(20) J3D_VAR_CASE(21) J3D_VAR_CASE(22) J3D_VAR_CASE(23)
    default: return hipErrorInvalidValue;
  }
#undef J3D_VAR_CASE
}

template <typename T, int BY, unsigned FL>
hipError_t by_cols(const Launch& L) {
  switch (L.c->cols) {
    case 1: return by_variant<T, BY, 1, FL>(L);
    case 2: return by_variant<T, BY, 2, FL>(L);
    case 4: return by_variant<T, BY, 4, FL>(L);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, unsigned FL>
hipError_t by_shape(const Launch& L) {
  switch (L.c->rows) {
    case 1: return by_cols<T, 1, FL>(L);
    case 2: return by_cols<T, 2, FL>(L);
    case 4: return by_cols<T, 4, FL>(L);
    case 8: return by_cols<T, 8, FL>(L);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch_f64(unsigned flags, const Launch& L);
hipError_t dispatch_f32(unsigned flags, const Launch& L);

}  // namespace sweep_detail
}  // namespace j3d
