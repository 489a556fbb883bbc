// gfx950 kernels of libj3d: the 7-point Jacobi sweep and everything shaped
// like it (fused residual, defect residual, FP32 correction sweeps, norms),
// the deterministic reductions, and input fills.
//
// Memory layout: Fortran column-major arrays with a one-cell halo; x is the
// unit-stride axis.  A workgroup owns a tile of 64 x-points (one 64-lane
// wavefront per row) by BY y-rows by `planes` z-planes and marches through
// z, keeping the previous, current and next value of its column in
// registers, so every plane of u and f is fetched from HBM once per tile.
// x and y neighbours come from the cache (variant 0) or from the current
// plane staged in LDS (variant 1).  The sweep streams about 24 bytes per
// FP64 point update and does 8 flops, far below the ridge of the FP64 VALU:
// it is HBM-bound and there is no dense contraction, hence no MFMA.
//
// Arithmetic order is fixed and the library is built with contraction off:
//   S  = ((((u[i-1] + u[i+1]) + u[j-1]) + u[j+1]) + u[k-1]) + u[k+1]
//   u' = (S + h2 * f) / 6                  (true IEEE division)
//   r  = f - (6 * u - S) / h2              (FP64)
// Residual sums of squares are reduced within a wavefront by a fixed
// butterfly, across wavefronts in wave order, to one partial per tile in a
// fixed slot, and the partials of a grid are summed by a second kernel in a
// fixed pattern: the norm depends only on the grid and the tile shape.
#include <math.h>

#include "j3d_internal.h"

namespace j3d {
namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Map dispatch order to logical tile order so that each XCD receives
// one contiguous block of tiles: neighbouring tiles then share halo rows in
// the same L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, r = n & 7, x = b & 7, idx = b >> 3;
  return x * q + min(x, r) + idx;
}

template <typename T>
__device__ __forceinline__ T h2_of(const GridArgs& g);
template <>
__device__ __forceinline__ double h2_of<double>(const GridArgs& g) { return g.h2; }
template <>
__device__ __forceinline__ float h2_of<float>(const GridArgs& g) { return g.h2f; }

template <typename T, int BY>
struct Smem {
  T pl[2][BY + 2][WAVE + 2];  // double-buffered plane with x/y halo ring
  double red[BY];
};

// One tile: local tile index t of grid g.  Returns nothing; writes the
// tile's partial sum (F_RES / F_NORM) to partials[g.tile0 + t].
template <typename T, int BY, int VAR, unsigned FL>
__device__ __forceinline__ void sweep_tile(const GridArgs& g, int t, double* __restrict__ partials,
                                           Smem<T, BY>& sm) {
  constexpr bool STENCIL = !(FL & (F_FIRST | F_NORM));
  constexpr bool USE_LDS = (VAR == 1) && STENCIL;
  const int lane = threadIdx.x;
  const int wy = threadIdx.y;
  const int tx = t % g.tiles_x;
  const int t2 = t / g.tiles_x;
  const int ty = t2 % g.tiles_y;
  const int tz = t2 / g.tiles_y;
  const int i = 1 + tx * WAVE + lane;
  const int j = 1 + ty * BY + wy;
  const int k0 = 1 + tz * g.planes;
  const int k1 = min(k0 + g.planes, g.nz + 1);
  const bool act = (i <= g.nx) && (j <= g.ny);
  // Inactive lanes keep in-bounds addresses; they never load or store.
  const int ic = min(i, g.nx), jc = min(j, g.ny);

  const T* __restrict__ pu = static_cast<const T*>(g.u) + (ic + g.su_y * jc + g.su_z * k0);
  const T* __restrict__ pf = static_cast<const T*>(g.f) + (ic + g.sf_y * jc + g.sf_z * k0);
  T* __restrict__ po = static_cast<T*>(g.o) + (ic + g.so_y * jc + g.so_z * k0);
  float* __restrict__ pr = g.r32 + (ic + g.sr_y * jc + g.sr_z * k0);
  double* __restrict__ p64 = g.u64 + (ic + g.s64_y * jc + g.s64_z * k0);
  const T h2 = h2_of<T>(g);

  double acc = 0.0;
  T um = T(0), uc = T(0);
  if (STENCIL && act) {
    um = pu[-g.su_z];
    uc = pu[0];
  }

  for (int k = k0; k < k1; ++k) {
    T s = T(0);
    T fc = T(0);
    T up = T(0);
    if (USE_LDS) {
      if (act) {
        up = pu[g.su_z];
        fc = pf[0];
      }
      T(*pl)[WAVE + 2] = sm.pl[(k - k0) & 1];
      if (act) {
        pl[wy + 1][lane + 1] = uc;
        if (lane == 0) pl[wy + 1][0] = pu[-1];
        if (lane == WAVE - 1 || i == g.nx) pl[wy + 1][lane + 2] = pu[1];
        if (wy == 0) pl[0][lane + 1] = pu[-g.su_y];
        if (wy == BY - 1 || j == g.ny) pl[wy + 2][lane + 1] = pu[g.su_y];
      }
      __syncthreads();
      if (act) {
        s = pl[wy + 1][lane] + pl[wy + 1][lane + 2];
        s = s + pl[wy][lane + 1];
        s = s + pl[wy + 2][lane + 1];
        s = s + um;
        s = s + up;
      }
    } else if (act) {
      fc = pf[0];
      if (STENCIL) {
        up = pu[g.su_z];
        s = pu[-1] + pu[1];
        s = s + pu[-g.su_y];
        s = s + pu[g.su_y];
        s = s + um;
        s = s + up;
      }
    }
    if (act) {
      if (FL & F_NORM) {
        acc += static_cast<double>(fc) * static_cast<double>(fc);
      } else {
        if (STENCIL && (FL & (F_RES | F_R32))) {
          const double r = static_cast<double>(fc) -
                           (6.0 * static_cast<double>(uc) - static_cast<double>(s)) / g.h2;
          if (FL & F_RES) acc += r * r;
          if (FL & F_R32) pr[0] = static_cast<float>(r);
        }
        if (FL & (F_WRITE | F_LAST)) {
          const T v = (s + h2 * fc) / T(6);
          if (FL & F_WRITE) po[0] = v;
          if (FL & F_LAST) p64[0] = p64[0] + static_cast<double>(v);
        }
      }
      um = uc;
      uc = up;
    }
    pu += g.su_z;
    pf += g.sf_z;
    po += g.so_z;
    pr += g.sr_z;
    p64 += g.s64_z;
  }

  if (FL & (F_RES | F_NORM)) {
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
  // The next tile of a persistent workgroup reuses the shared buffers.
  __syncthreads();
}

template <typename T, int BY, int VAR, unsigned FL>
__global__ void __launch_bounds__(WAVE * BY)
    k_pass_one(GridArgs g, double* __restrict__ partials, const int* __restrict__ done) {
  if (done != nullptr && *done != 0) return;
  __shared__ Smem<T, BY> sm;
  const int ntiles = g.tiles_x * g.tiles_y * g.tiles_z;
  for (int t = xcd_remap(blockIdx.x, gridDim.x); t < ntiles; t += gridDim.x)
    sweep_tile<T, BY, VAR, FL>(g, t, partials, sm);
}

template <typename T, int BY, int VAR, unsigned FL>
__global__ void __launch_bounds__(WAVE * BY)
    k_pass_batch(const GridArgs* __restrict__ table, int ngrids, int ntiles,
                 double* __restrict__ partials, const int* __restrict__ done) {
  __shared__ Smem<T, BY> sm;
  for (int t = xcd_remap(blockIdx.x, gridDim.x); t < ntiles; t += gridDim.x) {
    int lo = 0, hi = ngrids - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (table[mid].tile0 <= t) lo = mid; else hi = mid - 1;
    }
    if (done != nullptr && done[table[lo].id] != 0) continue;
    const GridArgs g = table[lo];
    sweep_tile<T, BY, VAR, FL>(g, t - g.tile0, partials, sm);
  }
}

// ---------------------------------------------------------------------
// Deterministic reduction of per-tile partials
// ---------------------------------------------------------------------

constexpr int RED_THREADS = 256;

__device__ __forceinline__ double reduce_slots(const double* __restrict__ p, int n, double* s) {
  double a = 0.0;
  for (int q = threadIdx.x; q < n; q += RED_THREADS) a += p[q];
  a = wave_sum(a);
  if ((threadIdx.x & (WAVE - 1)) == 0) s[threadIdx.x / WAVE] = a;
  __syncthreads();
  return ((s[0] + s[1]) + s[2]) + s[3];
}

__global__ void __launch_bounds__(RED_THREADS)
    k_reduce_one(const double* __restrict__ partials, int part0, int n, double* out,
                 const double* test_normf, double rtol, long long s, int* done,
                 long long* conv_at, int* nonfinite) {
  if (done != nullptr && *done != 0) return;
  __shared__ double sred[RED_THREADS / WAVE];
  const double tot = reduce_slots(partials + part0, n, sred);
  if (threadIdx.x == 0) {
    const double r = sqrt(tot);
    *out = r;
    if (test_normf != nullptr) {
      const bool bad = !isfinite(r);
      if (bad || r <= rtol * (*test_normf)) {
        *done = 1;
        *conv_at = s;
        if (bad) *nonfinite = 1;
      }
    }
  }
}

__global__ void __launch_bounds__(RED_THREADS)
    k_reduce_batch(const double* __restrict__ partials, const GridArgs* __restrict__ table,
                   double* out, int ostride, int q, const double* normf, const double* rtol,
                   long long s, int* done, long long* conv_at, int* nonfinite) {
  const GridArgs& a = table[blockIdx.x];
  const int g = a.id;
  if (done != nullptr && done[g] != 0) return;
  __shared__ double sred[RED_THREADS / WAVE];
  const int n = a.tiles_x * a.tiles_y * a.tiles_z;
  const double tot = reduce_slots(partials + a.tile0, n, sred);
  if (threadIdx.x == 0) {
    const double r = sqrt(tot);
    if (out != nullptr) out[(long long)g * ostride + q] = r;
    if (normf != nullptr) {
      const bool bad = !isfinite(r);
      if (bad || r <= rtol[g] * normf[g]) {
        done[g] = 1;
        conv_at[g] = s;
        if (bad) nonfinite[g] = 1;
      }
    }
  }
}

// ---------------------------------------------------------------------
// Fills and utilities
// ---------------------------------------------------------------------

// SplitMix64 (Steele, Lea, Flood 2014): output number n+1 of the generator
// whose state starts at `key`.
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long key,
                                                         unsigned long long n) {
  unsigned long long z = key + (n + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ void __launch_bounds__(256)
    k_fill_uniform(double* a, int ex, int ey, int ez, long long sy, long long sz,
                   unsigned long long key, double lo, double hi, double halo) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  if (i >= ex) return;
  double v = halo;
  if (i > 0 && j > 0 && k > 0 && i < ex - 1 && j < ey - 1 && k < ez - 1) {
    const unsigned long long nx = ex - 2, ny = ey - 2;
    const unsigned long long lin = (unsigned long long)(i - 1) +
                                   nx * ((unsigned long long)(j - 1) + ny * (unsigned long long)(k - 1));
    const unsigned long long bits = splitmix64(key, lin);
    const double u = static_cast<double>(bits >> 11) * 0x1.0p-53;
    v = lo + (hi - lo) * u;
  }
  a[i + sy * j + sz * k] = v;
}

template <typename T>
__global__ void __launch_bounds__(256)
    k_fill_const(T* a, int ex, long long sy, long long sz, T v) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < ex) a[i + sy * blockIdx.y + sz * blockIdx.z] = v;
}

__global__ void __launch_bounds__(256) k_copy(const double2* __restrict__ src,
                                              double2* __restrict__ dst, long long n2) {
  for (long long q = (long long)blockIdx.x * 256 + threadIdx.x; q < n2;
       q += (long long)gridDim.x * 256)
    dst[q] = src[q];
}

__global__ void k_copy_tail(const double* __restrict__ src, double* __restrict__ dst, long long n) {
  if (threadIdx.x == 0 && (n & 1)) dst[n - 1] = src[n - 1];
}

__global__ void __launch_bounds__(256)
    k_copy_interior(const double* __restrict__ src, double* __restrict__ dst, int nx, long long ssy,
                    long long ssz, long long dsy, long long dsz) {
  const int i = 1 + blockIdx.x * 256 + threadIdx.x;
  const int j = 1 + blockIdx.y;
  const int k = 1 + blockIdx.z;
  if (i <= nx) dst[i + dsy * j + dsz * k] = src[i + ssy * j + ssz * k];
}

__global__ void k_set_int(int* p, int n, int v) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) p[q] = v;
}

// ---------------------------------------------------------------------
// Host-side dispatch
// ---------------------------------------------------------------------

int device_cus() {
  static int cus[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
      n = 256;
    cus[dev] = n;
  }
  return cus[dev];
}

template <typename K>
int resident_blocks(K kernel, int threads) {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, 0) != hipSuccess || nb <= 0)
    nb = 1;
  return nb * device_cus();
}

template <typename T, int BY, int VAR, unsigned FL>
hipError_t launch_one_t(const TileCfg& c, const GridArgs& g, double* partials, const int* done,
                        hipStream_t st) {
  const int ntiles = g.tiles_x * g.tiles_y * g.tiles_z;
  int grid = ntiles;
  if (c.persistent) {
    static int cap = 0;
    if (cap == 0) cap = resident_blocks(k_pass_one<T, BY, VAR, FL>, WAVE * BY);
    grid = min(ntiles, cap);
  }
  if (grid <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_pass_one<T, BY, VAR, FL>), dim3(grid), dim3(WAVE, BY), 0, st, g, partials,
                     done);
  return hipGetLastError();
}

template <typename T, int BY, int VAR, unsigned FL>
hipError_t launch_batch_t(const TileCfg& c, const GridArgs* table, int ngrids, int ntiles,
                          double* partials, const int* done, hipStream_t st) {
  int grid = ntiles;
  if (c.persistent) {
    static int cap = 0;
    if (cap == 0) cap = resident_blocks(k_pass_batch<T, BY, VAR, FL>, WAVE * BY);
    grid = min(ntiles, cap);
  }
  if (grid <= 0 || ngrids <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_pass_batch<T, BY, VAR, FL>), dim3(grid), dim3(WAVE, BY), 0, st, table,
                     ngrids, ntiles, partials, done);
  return hipGetLastError();
}

struct Launch {
  bool batch;
  const TileCfg* c;
  const GridArgs* one;
  const GridArgs* table;
  int ngrids, ntiles;
  double* partials;
  const int* done;
  hipStream_t st;
};

template <typename T, int BY, int VAR, unsigned FL>
hipError_t go(const Launch& L) {
  return L.batch ? launch_batch_t<T, BY, VAR, FL>(*L.c, L.table, L.ngrids, L.ntiles, L.partials,
                                                  L.done, L.st)
                 : launch_one_t<T, BY, VAR, FL>(*L.c, *L.one, L.partials, L.done, L.st);
}

template <typename T, unsigned FL>
hipError_t by_shape(const Launch& L) {
  const int v = L.c->variant;
  switch (L.c->rows) {
    case 1: return v ? go<T, 1, 1, FL>(L) : go<T, 1, 0, FL>(L);
    case 2: return v ? go<T, 2, 1, FL>(L) : go<T, 2, 0, FL>(L);
    case 4: return v ? go<T, 4, 1, FL>(L) : go<T, 4, 0, FL>(L);
    case 8: return v ? go<T, 8, 1, FL>(L) : go<T, 8, 0, FL>(L);
    default: return hipErrorInvalidValue;
  }
}

hipError_t dispatch(int dtype, unsigned flags, const Launch& L) {
  if (dtype == J3D_F64) {
    switch (flags) {
      case F_WRITE: return by_shape<double, F_WRITE>(L);
      case F_WRITE | F_RES: return by_shape<double, F_WRITE | F_RES>(L);
      case F_RES: return by_shape<double, F_RES>(L);
      case F_RES | F_R32: return by_shape<double, F_RES | F_R32>(L);
      case F_NORM: return by_shape<double, F_NORM>(L);
      default: return hipErrorInvalidValue;
    }
  }
  if (dtype == J3D_F32) {
    switch (flags) {
      case F_WRITE: return by_shape<float, F_WRITE>(L);
      case F_WRITE | F_FIRST: return by_shape<float, F_WRITE | F_FIRST>(L);
      case F_LAST: return by_shape<float, F_LAST>(L);
      case F_LAST | F_FIRST: return by_shape<float, F_LAST | F_FIRST>(L);
      default: return hipErrorInvalidValue;
    }
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool tile_cfg_supported(const TileCfg& c) {
  const bool rows_ok = c.rows == 1 || c.rows == 2 || c.rows == 4 || c.rows == 8;
  return rows_ok && (c.variant == 0 || c.variant == 1) && c.planes >= 1 && c.planes <= 4096 &&
         (c.persistent == 0 || c.persistent == 1);
}

void tile_counts(int nx, int ny, int nz, const TileCfg& c, int* tx, int* ty, int* tz) {
  *tx = (nx + WAVE - 1) / WAVE;
  *ty = (ny + c.rows - 1) / c.rows;
  *tz = (nz + c.planes - 1) / c.planes;
}

int persistent_grid(const TileCfg& c) {
  // Upper bound used for sizing only; launches query the exact occupancy.
  return device_cus() * (32 / c.rows);
}

hipError_t launch_pass_one(int dtype, unsigned flags, const TileCfg& c, const GridArgs& g,
                           double* partials, const int* done, hipStream_t st) {
  Launch L{false, &c, &g, nullptr, 1, 0, partials, done, st};
  return dispatch(dtype, flags, L);
}

hipError_t launch_pass_batch(int dtype, unsigned flags, const TileCfg& c, const GridArgs* table,
                             int ngrids, int ntiles, double* partials, const int* done,
                             hipStream_t st) {
  Launch L{true, &c, nullptr, table, ngrids, ntiles, partials, done, st};
  return dispatch(dtype, flags, L);
}

hipError_t launch_reduce_one(const double* partials, int part0, int n, double* out,
                             const double* test_normf, double rtol, long long s, int* done,
                             long long* conv_at, int* nonfinite, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_one, dim3(1), dim3(RED_THREADS), 0, st, partials, part0, n, out,
                     test_normf, rtol, s, done, conv_at, nonfinite);
  return hipGetLastError();
}

hipError_t launch_reduce_batch(const double* partials, const GridArgs* table, int ngrids,
                               double* out, int ostride, int q, const double* normf,
                               const double* rtol, long long s, int* done, long long* conv_at,
                               int* nonfinite, hipStream_t st) {
  if (ngrids <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_batch, dim3(ngrids), dim3(RED_THREADS), 0, st, partials, table, out,
                     ostride, q, normf, rtol, s, done, conv_at, nonfinite);
  return hipGetLastError();
}

hipError_t launch_fill_uniform(double* a, int ex, int ey, int ez, long long sy, long long sz,
                               unsigned long long key, double lo, double hi, double halo,
                               hipStream_t st) {
  dim3 grid((ex + 255) / 256, ey, ez);
  hipLaunchKernelGGL(k_fill_uniform, grid, dim3(256), 0, st, a, ex, ey, ez, sy, sz, key, lo, hi,
                     halo);
  return hipGetLastError();
}

hipError_t launch_fill_const(void* a, int dtype, int ex, int ey, int ez, long long sy,
                             long long sz, double v, hipStream_t st) {
  dim3 grid((ex + 255) / 256, ey, ez);
  if (dtype == J3D_F64)
    hipLaunchKernelGGL(k_fill_const<double>, grid, dim3(256), 0, st, static_cast<double*>(a), ex,
                       sy, sz, v);
  else
    hipLaunchKernelGGL(k_fill_const<float>, grid, dim3(256), 0, st, static_cast<float*>(a), ex, sy,
                       sz, static_cast<float>(v));
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, long long n, hipStream_t st) {
  const long long n2 = n / 2;
  const int grid = static_cast<int>(min(n2 / 256 + 1, (long long)device_cus() * 16));
  hipLaunchKernelGGL(k_copy, dim3(grid), dim3(256), 0, st, reinterpret_cast<const double2*>(src),
                     reinterpret_cast<double2*>(dst), n2);
  hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_copy_interior(const double* src, double* dst, int nx, int ny, int nz,
                                long long ssy, long long ssz, long long dsy, long long dsz,
                                hipStream_t st) {
  dim3 grid((nx + 255) / 256, ny, nz);
  hipLaunchKernelGGL(k_copy_interior, grid, dim3(256), 0, st, src, dst, nx, ssy, ssz, dsy, dsz);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int n, int v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_set_int, dim3((n + 255) / 256), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}

}  // namespace j3d
