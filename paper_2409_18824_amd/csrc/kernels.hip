// gfx950 kernels of libj3d other than the sweep-shaped passes (which live
// in sweep.h and are instantiated per element type in kernels_f64.hip and
// kernels_f32.hip): the deterministic reduction of per-tile partial sums,
// input fills, the copy used as a bandwidth probe, and the launch entry
// points declared in j3d_internal.h.
//
// A grid's partials (one per tile, in fixed slots) are summed in a fixed
// pattern: thread q adds slots q, q+256, ... in order, then a fixed
// butterfly within each wavefront and the four wavefront sums in order.  The
// norm therefore depends only on the grid and the tile shape, never on the
// batch it was computed in.
#include <math.h>

#include "sweep2.h"
#include "sweep3.h"

namespace j3d {
namespace {

using sweep_detail::WAVE;
using sweep_detail::wave_sum;

// ---------------------------------------------------------------------
// Deterministic reduction of per-tile partials
// ---------------------------------------------------------------------

constexpr int RED_THREADS = 1024;
constexpr int RED_WAVES = RED_THREADS / WAVE;
constexpr int RED_UNROLL = 16;
constexpr int SUM_THREADS = 256;
constexpr int SUM_UNROLL = 8;

// Thread q adds slots q, q + 1024, q + 2048, ... in that order (loads are
// issued 16 at a time so they overlap, the additions stay in order), then the
// wavefront butterfly and the 16 wavefront sums in wave order.
__device__ __forceinline__ double reduce_slots(const double* __restrict__ p, int n, double* s) {
  double a = 0.0;
  int m = threadIdx.x;
  for (; m + (RED_UNROLL - 1) * RED_THREADS < n; m += RED_UNROLL * RED_THREADS) {
    double v[RED_UNROLL];
#pragma unroll
    for (int u = 0; u < RED_UNROLL; ++u) v[u] = p[m + u * RED_THREADS];
#pragma unroll
    for (int u = 0; u < RED_UNROLL; ++u) a += v[u];
  }
  for (; m < n; m += RED_THREADS) a += p[m];
  a = wave_sum(a);
  if ((threadIdx.x & (WAVE - 1)) == 0) s[threadIdx.x / WAVE] = a;
  __syncthreads();
  double t = s[0];
#pragma unroll
  for (int w = 1; w < RED_WAVES; ++w) t += s[w];
  return t;
}

__global__ void __launch_bounds__(RED_THREADS)
    k_reduce_one(const double* __restrict__ partials, int part0, int n, double* out,
                 const double* test_normf, double rtol, long long s, int* done,
                 long long* conv_at, int* nonfinite) {
  if (done != nullptr && *done != 0) return;
  __shared__ double sred[RED_WAVES];
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

// As k_reduce_one for the solve drivers' checks, with the check index kept
// on the device: check *qnext goes to hist[*qnext], then *qnext advances.
// Every check of a replayed graph chunk is therefore the same kernel with the
// same arguments.
__global__ void __launch_bounds__(RED_THREADS)
    k_reduce_count(const double* __restrict__ partials, int n, double* hist, const double* normf,
                   double rtol, int* done, long long* conv_at, int* nonfinite, long long* qnext) {
  if (*done != 0) return;
  __shared__ double sred[RED_WAVES];
  const double tot = reduce_slots(partials, n, sred);
  if (threadIdx.x == 0) {
    const long long q = *qnext;
    const double r = sqrt(tot);
    hist[q] = r;
    const bool bad = !isfinite(r);
    if (bad || r <= rtol * (*normf)) {
      *done = 1;
      *conv_at = q;
      if (bad) *nonfinite = 1;
    }
    *qnext = q + 1;
  }
}

__global__ void __launch_bounds__(RED_THREADS)
    k_reduce_batch(const double* __restrict__ partials, const GridArgs* __restrict__ table,
                   double* out, int ostride, int q, const double* normf, const double* rtol,
                   long long s, int* done, long long* conv_at, int* nonfinite) {
  const GridArgs& a = table[blockIdx.x];
  const int g = a.id;
  if (done != nullptr && done[g] != 0) return;
  __shared__ double sred[RED_WAVES];
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

__global__ void __launch_bounds__(RED_THREADS)
    k_reduce_plain(const double* __restrict__ partials, int n, double* out) {
  __shared__ double sred[RED_WAVES];
  const double tot = reduce_slots(partials, n, sred);
  if (threadIdx.x == 0) *out = tot;
}

// ---------------------------------------------------------------------
// sum / dot_product over FP64 vectors
// ---------------------------------------------------------------------

// Block b adds the addends of [b*chunk, min(n, (b+1)*chunk)): thread t takes
// elements t, t+256, t+512, ... in that order (eight loads issued at once,
// additions in order), then the wavefront butterfly and the four wavefront
// sums in order; the block's sum goes to partials[b].  The partition depends
// on n only, so the result is reproducible bit for bit.
template <bool DOT>
__global__ void __launch_bounds__(SUM_THREADS)
    k_sum_partials(const double* __restrict__ x, const double* __restrict__ y, long long n,
                   long long chunk, double* __restrict__ partials) {
  __shared__ double red[SUM_THREADS / WAVE];
  const long long lo = (long long)blockIdx.x * chunk;
  const long long hi = min(n, lo + chunk);
  double a = 0.0;
  long long i = lo + threadIdx.x;
  for (; i + (SUM_UNROLL - 1) * SUM_THREADS < hi; i += SUM_UNROLL * SUM_THREADS) {
    double v[SUM_UNROLL];
#pragma unroll
    for (int u = 0; u < SUM_UNROLL; ++u) {
      v[u] = x[i + u * SUM_THREADS];
      if (DOT) v[u] = v[u] * y[i + u * SUM_THREADS];
    }
#pragma unroll
    for (int u = 0; u < SUM_UNROLL; ++u) a += v[u];
  }
  for (; i < hi; i += SUM_THREADS) a += DOT ? x[i] * y[i] : x[i];
  a = wave_sum(a);
  if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = a;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
#pragma unroll
    for (int w = 1; w < SUM_THREADS / WAVE; ++w) t += red[w];
    partials[blockIdx.x] = t;
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

// Copy probes of other shapes: U 16-byte elements per thread (consecutive
// blocks of 256 elements, so every load instruction stays coalesced), with
// or without nontemporal loads and stores.
typedef double copy_vd2 __attribute__((ext_vector_type(2)));

template <int U, bool NT>
__global__ void __launch_bounds__(256) k_copy_u(const copy_vd2* __restrict__ src, copy_vd2* __restrict__ dst,
                                                long long n2) {
  const long long base = (long long)blockIdx.x * 256 * U + threadIdx.x;
  copy_vd2 v[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long q = base + 256LL * u;
    if (q < n2) v[u] = NT ? __builtin_nontemporal_load(src + q) : src[q];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long q = base + 256LL * u;
    if (q < n2) {
      if (NT)
        __builtin_nontemporal_store(v[u], dst + q);
      else
        dst[q] = v[u];
    }
  }
}

__global__ void k_copy_tail(const double* __restrict__ src, double* __restrict__ dst, long long n) {
  if (threadIdx.x == 0 && (n & 1)) dst[n - 1] = src[n - 1];
}

// Two streams read, one written (dst = a + b), the traffic mix of the sweep
// passes: U 16-byte elements per thread, plain or nontemporal stores.
template <int U, bool NT>
__global__ void __launch_bounds__(256) k_triad_u(const copy_vd2* __restrict__ a, const copy_vd2* __restrict__ b,
                                                 copy_vd2* __restrict__ dst, long long n2) {
  const long long base = (long long)blockIdx.x * 256 * U + threadIdx.x;
  copy_vd2 v[U], w[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long q = base + 256LL * u;
    if (q < n2) {
      v[u] = a[q];
      w[u] = b[q];
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const long long q = base + 256LL * u;
    if (q < n2) {
      const copy_vd2 s = v[u] + w[u];
      if (NT)
        __builtin_nontemporal_store(s, dst + q);
      else
        dst[q] = s;
    }
  }
}

__global__ void k_triad_tail(const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ dst,
                             long long n) {
  if (threadIdx.x == 0 && (n & 1)) dst[n - 1] = a[n - 1] + b[n - 1];
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

}  // namespace

namespace sweep_detail {
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
}  // namespace sweep_detail

using sweep_detail::device_cus;

bool tile_cfg_supported(const TileCfg& c) {
  const bool rows_ok = c.rows == 1 || c.rows == 2 || c.rows == 4 || c.rows == 8;
  const bool cols_ok = c.cols == 1 || c.cols == 2 || c.cols == 4;
  const bool var_ok = c.variant >= 0 && c.variant <= 23 && (c.variant & 8) == 0;
  return rows_ok && cols_ok && var_ok && sweep_detail::shape_instantiated(c.rows, c.cols, c.variant) &&
         c.order >= 0 && c.order <= 2 && c.planes >= 1 && c.planes <= 4096 &&
         (c.persistent == 0 || c.persistent == 1);
}

void tile_counts(int nx, int ny, int nz, const TileCfg& c, int* tx, int* ty, int* tz) {
  const int tr = c.rows * sweep_detail::rows_per_thread(c.variant);
  const int tc = WAVE * c.cols;
  *tx = (nx + tc - 1) / tc;
  *ty = (ny + tr - 1) / tr;
  *tz = (nz + c.planes - 1) / c.planes;
}

bool tile2_cfg_supported(int dtype, const TileCfg& c) {
  const bool rows_ok = c.rows == 1 || c.rows == 2 || c.rows == 4 || c.rows == 8;
  const bool cols_ok = c.cols == 1 || c.cols == 2 || c.cols == 4;
  if (!rows_ok || !cols_ok || c.variant < 0 || c.variant > 23) return false;
  if (dtype != J3D_F64 && dtype != J3D_F32) return false;
  const int es = dtype == J3D_F64 ? 8 : 4;
  return sweep_detail::shape2_instantiated(es, c.rows, c.cols, c.variant) && c.order >= 0 && c.order <= 2 &&
         c.planes >= 1 && c.planes <= 4096 && (c.persistent == 0 || c.persistent == 1);
}

void tile2_counts(int nx, int ny, int nz, const TileCfg& c, int* tx, int* ty, int* tz) {
  // Unsupported shapes (zero or negative extents) count one tile per axis; they
  // are rejected before any launch.
  const int w = max(1, sweep_detail::sweep2_cols(c.cols));
  const int h = max(1, c.rows * sweep_detail::rows_per_thread(c.variant) - 2);
  *tx = (nx + w - 1) / w;
  *ty = (ny + h - 1) / h;
  *tz = (nz + c.planes - 1) / c.planes;
}

static hipError_t dispatch2(int dtype, unsigned flags, const sweep_detail::Launch& L) {
  if (!tile2_cfg_supported(dtype, *L.c)) return hipErrorInvalidValue;
  if (dtype == J3D_F64) return sweep_detail::dispatch_sweep2_f64(flags, L);
  return sweep_detail::dispatch_sweep2_f32(flags, L);
}

bool tile3_cfg_supported(int dtype, const TileCfg& c) {
  if (dtype != J3D_F64 && dtype != J3D_F32) return false;
  return sweep_detail::shape3_instantiated(c.rows, c.variant) && c.cols == 1 && c.persistent == 0 &&
         c.order >= 0 && c.order <= 2 && c.planes >= 1 && c.planes <= 4096;
}

void tile3_counts(int nx, int ny, int nz, const TileCfg& c, int* tx, int* ty, int* tz) {
  const int w = sweep_detail::kSweep3Cols;
  const int h = max(1, c.rows * sweep_detail::rows_per_thread(c.variant) - 4);
  *tx = (nx + w - 1) / w;
  *ty = (ny + h - 1) / h;
  *tz = (nz + max(1, c.planes) - 1) / max(1, c.planes);
}

hipError_t launch_sweep3_one(int dtype, unsigned flags, const TileCfg& c, const GridArgs& g,
                             double* partials, const int* done, hipStream_t st) {
  if (!tile3_cfg_supported(dtype, c)) return hipErrorInvalidValue;
  if (dtype == J3D_F64) return sweep_detail::dispatch_sweep3_f64(flags, c, g, partials, done, st);
  return sweep_detail::dispatch_sweep3_f32(flags, c, g, partials, done, st);
}

hipError_t launch_sweep3_batch(int dtype, unsigned flags, const TileCfg& c, const GridArgs* table, int ngrids,
                               int ntiles, double* partials, const int* done, hipStream_t st,
                               const TileSlot* slots, int nslots) {
  TileCfg k = c;
  if (k.order == kOrderSlots) {
    if (slots == nullptr) return hipErrorInvalidValue;
    k.order = 0;  // the slot list replaces the order
  }
  if (!tile3_cfg_supported(dtype, k) || (slots != nullptr && nslots < 0)) return hipErrorInvalidValue;
  if (dtype == J3D_F64)
    return sweep_detail::dispatch_sweep3_batch_f64(flags, k, table, ngrids, ntiles, slots, nslots, partials, done,
                                                   st);
  return sweep_detail::dispatch_sweep3_batch_f32(flags, k, table, ngrids, ntiles, slots, nslots, partials, done, st);
}

hipError_t launch_sweep2_one(int dtype, unsigned flags, const TileCfg& c, const GridArgs& g,
                             double* partials, const int* done, hipStream_t st) {
  sweep_detail::Launch L{false, &c, &g, nullptr, 1, 0, partials, done, st};
  return dispatch2(dtype, flags, L);
}

hipError_t launch_sweep2_batch(int dtype, unsigned flags, const TileCfg& c, const GridArgs* table,
                               int ngrids, int ntiles, double* partials, const int* done,
                               hipStream_t st) {
  sweep_detail::Launch L{true, &c, nullptr, table, ngrids, ntiles, partials, done, st};
  return dispatch2(dtype, flags, L);
}

int persistent_grid(const TileCfg& c) {
  // Upper bound used for sizing only; launches query the exact occupancy.
  return device_cus() * (32 / c.rows);
}

static hipError_t dispatch(int dtype, unsigned flags, const sweep_detail::Launch& L) {
  if (!tile_cfg_supported(*L.c)) return hipErrorInvalidValue;
  if (dtype == J3D_F64) return sweep_detail::dispatch_f64(flags, L);
  if (dtype == J3D_F32) return sweep_detail::dispatch_f32(flags, L);
  return hipErrorInvalidValue;
}

hipError_t launch_pass_one(int dtype, unsigned flags, const TileCfg& c, const GridArgs& g,
                           double* partials, const int* done, hipStream_t st) {
  sweep_detail::Launch L{false, &c, &g, nullptr, 1, 0, partials, done, st};
  return dispatch(dtype, flags, L);
}

hipError_t launch_pass_one_pre(int dtype, unsigned flags, const TileCfg& c, const GridArgs& g,
                               double* partials, const int* done, const PreReduce& pr, hipStream_t st) {
  sweep_detail::Launch L{false, &c, &g, nullptr, 1, 0, partials, done, st};
  L.pr = pr;
  return dispatch(dtype, flags, L);
}

hipError_t launch_pass_batch(int dtype, unsigned flags, const TileCfg& c, const GridArgs* table,
                             int ngrids, int ntiles, double* partials, const int* done,
                             hipStream_t st) {
  sweep_detail::Launch L{true, &c, nullptr, table, ngrids, ntiles, partials, done, st};
  return dispatch(dtype, flags, L);
}

hipError_t launch_reduce_one(const double* partials, int part0, int n, double* out,
                             const double* test_normf, double rtol, long long s, int* done,
                             long long* conv_at, int* nonfinite, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_one, dim3(1), dim3(RED_THREADS), 0, st, partials, part0, n, out,
                     test_normf, rtol, s, done, conv_at, nonfinite);
  return hipGetLastError();
}

hipError_t launch_reduce_count(const double* partials, int n, double* hist, const double* normf,
                               double rtol, int* done, long long* conv_at, int* nonfinite,
                               long long* qnext, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_count, dim3(1), dim3(RED_THREADS), 0, st, partials, n, hist, normf, rtol,
                     done, conv_at, nonfinite, qnext);
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

long long sum_chunk(long long n) {
  const long long step = (long long)SUM_THREADS * SUM_UNROLL;
  const long long per = (n + (long long)kSumMaxBlocks * step - 1) / ((long long)kSumMaxBlocks * step);
  return step * (per < 1 ? 1 : per);
}

int sum_blocks(long long n) { return n <= 0 ? 0 : (int)((n + sum_chunk(n) - 1) / sum_chunk(n)); }

hipError_t launch_sum(const double* x, const double* y, long long n, double* partials, double* out,
                      hipStream_t st) {
  const int nb = sum_blocks(n);
  if (nb > 0) {
    if (y != nullptr)
      hipLaunchKernelGGL(k_sum_partials<true>, dim3(nb), dim3(SUM_THREADS), 0, st, x, y, n, sum_chunk(n),
                         partials);
    else
      hipLaunchKernelGGL(k_sum_partials<false>, dim3(nb), dim3(SUM_THREADS), 0, st, x, y, n, sum_chunk(n),
                         partials);
  }
  hipLaunchKernelGGL(k_reduce_plain, dim3(1), dim3(RED_THREADS), 0, st, partials, nb, out);
  return hipGetLastError();
}

hipError_t launch_copy_variant(int v, const double* src, double* dst, long long n, hipStream_t st) {
  if (v == 0) return launch_copy(src, dst, n, st);
  const long long n2 = n / 2;
  const int u = (v == 1 || v == 2) ? 1 : 4;
  const bool nt = v == 2 || v == 4;
  const long long blocks = (n2 + 256LL * u - 1) / (256LL * u);
  if (blocks > (1LL << 30)) return hipErrorInvalidValue;
  const auto* s2 = reinterpret_cast<const copy_vd2*>(src);
  auto* d2 = reinterpret_cast<copy_vd2*>(dst);
  if (u == 1 && !nt) hipLaunchKernelGGL((k_copy_u<1, false>), dim3(blocks), dim3(256), 0, st, s2, d2, n2);
  if (u == 1 && nt) hipLaunchKernelGGL((k_copy_u<1, true>), dim3(blocks), dim3(256), 0, st, s2, d2, n2);
  if (u == 4 && !nt) hipLaunchKernelGGL((k_copy_u<4, false>), dim3(blocks), dim3(256), 0, st, s2, d2, n2);
  if (u == 4 && nt) hipLaunchKernelGGL((k_copy_u<4, true>), dim3(blocks), dim3(256), 0, st, s2, d2, n2);
  hipLaunchKernelGGL(k_copy_tail, dim3(1), dim3(64), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_triad_variant(int v, const double* a, const double* b, double* dst, long long n,
                                hipStream_t st) {
  const long long n2 = n / 2;
  const int u = v == 2 ? 4 : 1;
  const bool nt = v != 1;
  const long long blocks = (n2 + 256LL * u - 1) / (256LL * u);
  if (blocks > (1LL << 30)) return hipErrorInvalidValue;
  const auto* a2 = reinterpret_cast<const copy_vd2*>(a);
  const auto* b2 = reinterpret_cast<const copy_vd2*>(b);
  auto* d2 = reinterpret_cast<copy_vd2*>(dst);
  if (blocks > 0) {
    if (u == 1 && nt) hipLaunchKernelGGL((k_triad_u<1, true>), dim3(blocks), dim3(256), 0, st, a2, b2, d2, n2);
    if (u == 1 && !nt) hipLaunchKernelGGL((k_triad_u<1, false>), dim3(blocks), dim3(256), 0, st, a2, b2, d2, n2);
    if (u == 4) hipLaunchKernelGGL((k_triad_u<4, true>), dim3(blocks), dim3(256), 0, st, a2, b2, d2, n2);
  }
  hipLaunchKernelGGL(k_triad_tail, dim3(1), dim3(64), 0, st, a, b, dst, n);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, long long n, hipStream_t st) {
  // One 16-byte element per thread and one short-lived wavefront per 1 KiB:
  // on MI355X this streams faster than persistent grid-stride copies.
  const long long n2 = n / 2;
  const int grid = static_cast<int>(min(n2 / 256 + 1, (long long)(1 << 30)));
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
