// C-ABI entry points of libj3d: single sweeps, residual norms, fills,
// bandwidth probe and housekeeping.  Solves, batches and serving live in
// solve.cpp, batch.cpp and serve.cpp.
#include <cmath>
#include <cstring>
#include <vector>

#include "runtime.h"

namespace j3d {
const char* last_error_text();
int release_all_scratch();
bool tune_cache_lookup_single(int dtype, int nx, int ny, int nz, TileCfg* out);

namespace {
// The supported tile shapes, enumerated once: every (rows, planes, variant,
// persistent, order, cols) that tile_cfg_supported accepts.
const std::vector<TileCfg>& tune_table() {
  static const std::vector<TileCfg> table = [] {
    std::vector<TileCfg> v;
    for (int rows : {1, 2, 4, 8})
      for (int planes : {1, 2, 4, 8, 16, 32, 64, 128})
        for (int var : {0, 1, 2, 3, 4, 5, 6, 7, 16, 17, 18, 19, 20, 21, 22, 23})
          for (int pers : {0, 1})
            for (int order : {0, 1, 2})
              for (int cols : {1, 2, 4}) {
                TileCfg c{rows, planes, var, pers, order, cols};
                if (tile_cfg_supported(c)) v.push_back(c);
              }
    return v;
  }();
  return table;
}
}  // namespace

TileCfg default_cfg(int dtype, int nx, int ny, int nz) {
  TileCfg c;
  if (tune_cache_lookup_single(dtype, nx, ny, nz, &c)) return c;
  // FP64 grids of at most 64^3 points: four wavefronts of two rows per
  // thread, two planes per tile, XCD-blocked (7.45 us per sweep at 64^3 with
  // a residual after every sweep, against 7.8 with four rows per thread and
  // one plane, 16.0 with the large-grid shape).  Otherwise one wavefront of
  // four rows per thread, 16 planes per tile (the loads run one plane
  // ahead, so deep tiles cost no latency), per-slab XCD chunks: 572 us per
  // FP64 pass at 512^3 against 643 with 2 planes, 70.7 us at 256^3.
  const bool small = dtype == J3D_F64 && (long long)nx * ny * nz <= 64LL * 64 * 64;
  c.rows = small ? 4 : 1;
  c.planes = small ? 2 : 16;
  c.variant = small ? 6 : 20;  // two or four rows per thread, nontemporal stores
  c.persistent = 0;
  c.order = small ? 0 : 2;
  c.cols = 1;
  return c;
}

TileCfg default_cfg3(int dtype, int nx, int ny, int nz) {
  TileCfg c;
  const int kind = dtype == J3D_F32 ? J3D_KIND_F32X3 : J3D_KIND_F64X3;
  if (tune_cache_lookup_single(kind, nx, ny, nz, &c) && tile3_cfg_supported(dtype, c)) return c;
  // measured on cubes from 96^3 to 512^3 (nontemporal stores throughout):
  // up to about 200^3 points 4 wavefronts of 2 rows per thread and 16
  // planes (more, thinner tiles), XCD-blocked; up to about 300^3, 4
  // wavefronts of 4 rows per thread, per-slab XCD chunks; beyond, 8
  // wavefronts of 2 rows per thread (about 95 registers per thread against
  // 160 with 4 rows, so twice the wavefronts per CU), 32 planes in
  // per-slab XCD chunks.  Above 400^3 (measured at 512^3): FP64 16
  // wavefronts of 2 rows (32-row blocks, one workgroup per CU) and 144
  // planes in launch order, 712 us per pass against 731 with 8 wavefronts
  // and 96 planes (the block's waste on ragged y edges is small since
  // wavefronts wholly past the grid skip their work; 144 planes make four
  // z-slabs, the last one short); FP32 8 wavefronts of 2 rows, 48 planes,
  // per-slab XCD chunks, 419 us against 439 with 4 wavefronts of 4 rows and
  // 24 planes.  Other sizes above 400^3 are best tuned (j3d_autotune_single).
  const long long pts = (long long)nx * ny * nz;
  const bool small = pts <= 200LL * 200 * 200;
  const bool large = pts > 300LL * 300 * 300;
  const bool huge = pts > 400LL * 400 * 400;
  c.rows = large ? 8 : 4;
  c.planes = large ? 32 : 16;
  c.variant = (small || large) ? 6 : 20;
  c.persistent = 0;
  c.order = small ? 0 : 2;
  c.cols = 1;
  if (huge) {
    if (dtype == J3D_F32) {
      c.rows = 8;
      c.planes = 48;
      c.order = 2;
    } else {
      c.rows = 16;
      c.planes = 144;
      c.order = 1;
    }
  }
  return c;
}

TileCfg default_cfg2(int dtype, int nx, int ny, int nz) {
  TileCfg c;
  if (tune_cache_lookup_single(dtype == J3D_F32 ? J3D_KIND_F32X2 : J3D_KIND_F64X2, nx, ny, nz, &c) &&
      tile2_cfg_supported(dtype == J3D_F32 ? J3D_F32 : J3D_F64, c))
    return c;
  // measured at 512^3: FP64 16 rows per block, 16 planes, launch order;
  // FP32 32 rows per block, 8 planes, XCD-blocked order (4 rows per thread,
  // nontemporal stores in both)
  c.rows = dtype == J3D_F32 ? 8 : 4;
  c.planes = dtype == J3D_F32 ? 8 : 16;
  c.variant = 20;
  c.persistent = 0;
  c.order = dtype == J3D_F32 ? 0 : 1;
  c.cols = 1;
  return c;
}

// Sum-of-squares pass over (u, f) followed by the deterministic reduce into
// `out` (device).  flags is F_RES (residual of u) or F_NORM (norm of f).
static int norm_pass(unsigned flags, const Field& u, const Field& f, const Field* o, double h,
                     const TileCfg& c, double* out, hipStream_t st, Scratch* s) {
  const Field* up = (flags & F_NORM) ? nullptr : &u;
  GridArgs g = make_args(up, o, &f, nullptr, nullptr, h, c, 0);
  const int nt = g.tiles_x * g.tiles_y * g.tiles_z;
  J3D_TRY(ensure_partials(s, nt));
  J3D_HIP(launch_pass_one(J3D_F64, flags, c, g, s->partials, nullptr, st));
  J3D_HIP(launch_reduce_one(s->partials, 0, nt, out, nullptr, 0.0, 0, nullptr, nullptr, nullptr, st));
  return J3D_OK;
}

int check_sweep3_call(const j3d_array* u_in, const j3d_array* u_out, const j3d_array* f, double h,
                      uint32_t flags, const double* resid_out, Sweep3Call* k) {
  Field& a = k->a;
  Field& b = k->b;
  Field& c = k->c;
  J3D_TRY(check_field(u_in, -1, &a, "u_in"));
  J3D_TRY(check_field(u_out, a.dtype, &b, "u_out"));
  J3D_TRY(check_field(f, a.dtype, &c, "f"));
  J3D_TRY(check_same_interior(a, b, "u_in", "u_out"));
  J3D_TRY(check_same_interior(a, c, "u_in", "f"));
  J3D_TRY(check_h(h));
  if ((flags & ~(J3D_HOST_RESULT | J3D_RESID_AFTER_1 | J3D_RESID_AFTER_2)) != 0)
    return fail(J3D_EINVAL, "unknown flags 0x%x", flags);
  const unsigned after = flags & (J3D_RESID_AFTER_1 | J3D_RESID_AFTER_2);
  if (after == (J3D_RESID_AFTER_1 | J3D_RESID_AFTER_2))
    return fail(J3D_EINVAL, "J3D_RESID_AFTER_1 and J3D_RESID_AFTER_2 are exclusive");
  if (after != 0 && resid_out == nullptr) return fail(J3D_EINVAL, "J3D_RESID_AFTER_*: resid_out is null");
  if (fields_overlap(a, b)) return fail(J3D_EALIAS, "u_in and u_out overlap");
  if (fields_overlap(b, c)) return fail(J3D_EALIAS, "u_out and f overlap");
  if (resid_out != nullptr && a.dtype != J3D_F64)
    return fail(J3D_EDTYPE, "a fused residual needs FP64 arrays");
  if (!plane_fits_u32(a) || !plane_fits_u32(b) || !plane_fits_u32(c))
    return fail(J3D_EINVAL, "a z-plane spans 4 GiB or more: the three-sweep pass needs smaller planes");
  k->res_flag = after == J3D_RESID_AFTER_1 ? F_RES1 : after == J3D_RESID_AFTER_2 ? F_RES2 : F_RES;
  k->cfg = default_cfg3(a.dtype, a.nx(), a.ny(), a.nz());
  k->g = make_args3(&a, &b, &c, nullptr, h, k->cfg, 0);
  return J3D_OK;
}

}  // namespace j3d

using namespace j3d;

extern "C" {

int j3d_abi_version(void) { return J3D_ABI_VERSION; }

const char* j3d_last_error(void) { return last_error_text(); }

int j3d_element_offset(const j3d_array* a, int64_t i, int64_t j, int64_t k, int64_t* offset) {
  J3D_TRY(check_field(a, -1, nullptr, "array"));
  if (offset == nullptr) return fail(J3D_EINVAL, "offset: null pointer");
  const int64_t idx[3] = {i, j, k};
  int64_t off = 0;
  for (int d = 0; d < 3; ++d) {
    if (idx[d] < a->lbound[d] || idx[d] > a->ubound[d])
      return fail(J3D_EINVAL, "index %lld outside bounds %lld:%lld on axis %d", (long long)idx[d],
                  (long long)a->lbound[d], (long long)a->ubound[d], d);
    off += (idx[d] - a->lbound[d]) * a->stride[d];
  }
  *offset = off;
  return J3D_OK;
}

int j3d_check_array(const j3d_array* a, int32_t dtype) { return check_field(a, dtype, nullptr, "array"); }

int j3d_tune_query_single(int32_t kind, int32_t nx, int32_t ny, int32_t nz, j3d_tune* out) {
  if (out == nullptr) return fail(J3D_EINVAL, "tune: null pointer");
  if (nx < 1 || ny < 1 || nz < 1) return fail(J3D_EINVAL, "extents must be >= 1");
  TileCfg c;
  if (kind == J3D_F64 || kind == J3D_F32)
    c = default_cfg(kind, nx, ny, nz);
  else if (kind == J3D_KIND_F64X2 || kind == J3D_KIND_F32X2)
    c = default_cfg2(kind == J3D_KIND_F32X2 ? J3D_F32 : J3D_F64, nx, ny, nz);
  else if (kind == J3D_KIND_F64X3 || kind == J3D_KIND_F32X3)
    c = default_cfg3(kind == J3D_KIND_F32X3 ? J3D_F32 : J3D_F64, nx, ny, nz);
  else
    return fail(J3D_EDTYPE, "kind must be J3D_F64, J3D_F32 or a J3D_KIND_* pass kind");
  out->rows = c.rows;
  out->planes = c.planes;
  out->variant = c.variant;
  out->persistent = c.persistent;
  out->order = c.order;
  out->cols = c.cols;
  return J3D_OK;
}

int j3d_tune_count(void) { return (int)tune_table().size(); }

int j3d_tune_get(int32_t index, j3d_tune* out) {
  if (out == nullptr || index < 0 || index >= (int)tune_table().size())
    return fail(J3D_EINVAL, "tune index out of range");
  const TileCfg& c = tune_table()[(size_t)index];
  out->rows = c.rows;
  out->planes = c.planes;
  out->variant = c.variant;
  out->persistent = c.persistent;
  out->order = c.order;
  out->cols = c.cols;
  return J3D_OK;
}

int jacobi3d_sweep(const j3d_array* u_in, j3d_array* u_out, const j3d_array* f, double h,
                   uint32_t flags, double* resid_out, void* stream) {
  Field a, b, c;
  J3D_TRY(check_field(u_in, -1, &a, "u_in"));
  J3D_TRY(check_field(u_out, a.dtype, &b, "u_out"));
  J3D_TRY(check_field(f, a.dtype, &c, "f"));
  J3D_TRY(check_same_interior(a, b, "u_in", "u_out"));
  J3D_TRY(check_same_interior(a, c, "u_in", "f"));
  J3D_TRY(check_h(h));
  if ((flags & ~J3D_HOST_RESULT) != 0) return fail(J3D_EINVAL, "unknown flags 0x%x", flags);
  if (fields_overlap(a, b)) return fail(J3D_EALIAS, "u_in and u_out overlap");
  if (fields_overlap(b, c)) return fail(J3D_EALIAS, "u_out and f overlap");
  if (resid_out != nullptr && a.dtype != J3D_F64)
    return fail(J3D_EDTYPE, "a fused residual needs FP64 arrays");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const TileCfg cfg = default_cfg(a.dtype, a.nx(), a.ny(), a.nz());
  GridArgs g = make_args(&a, &b, &c, nullptr, nullptr, h, cfg, 0);
  if (resid_out == nullptr) {
    J3D_HIP(launch_pass_one(a.dtype, F_WRITE, cfg, g, nullptr, nullptr, st));
    return J3D_OK;
  }
  Scratch* s = nullptr;
  J3D_TRY(get_scratch(st, &s));
  const int nt = g.tiles_x * g.tiles_y * g.tiles_z;
  J3D_TRY(ensure_partials(s, nt));
  J3D_HIP(launch_pass_one(J3D_F64, F_WRITE | F_RES, cfg, g, s->partials, nullptr, st));
  const bool host = (flags & J3D_HOST_RESULT) != 0;
  double* dst = host ? &s->ctl->value : resid_out;
  J3D_HIP(launch_reduce_one(s->partials, 0, nt, dst, nullptr, 0.0, 0, nullptr, nullptr, nullptr, st));
  if (host) {
    J3D_HIP(hipMemcpyAsync(&s->ctl_host->value, &s->ctl->value, sizeof(double),
                           hipMemcpyDeviceToHost, st));
    J3D_HIP(hipStreamSynchronize(st));
    *resid_out = s->ctl_host->value;
  }
  return J3D_OK;
}

int jacobi3d_sweep2(const j3d_array* u_in, j3d_array* u_out, const j3d_array* f, double h,
                    uint32_t flags, double* resid_out, void* stream) {
  Field a, b, c;
  J3D_TRY(check_field(u_in, -1, &a, "u_in"));
  J3D_TRY(check_field(u_out, a.dtype, &b, "u_out"));
  J3D_TRY(check_field(f, a.dtype, &c, "f"));
  J3D_TRY(check_same_interior(a, b, "u_in", "u_out"));
  J3D_TRY(check_same_interior(a, c, "u_in", "f"));
  J3D_TRY(check_h(h));
  if ((flags & ~J3D_HOST_RESULT) != 0) return fail(J3D_EINVAL, "unknown flags 0x%x", flags);
  if (fields_overlap(a, b)) return fail(J3D_EALIAS, "u_in and u_out overlap");
  if (fields_overlap(b, c)) return fail(J3D_EALIAS, "u_out and f overlap");
  if (resid_out != nullptr && a.dtype != J3D_F64)
    return fail(J3D_EDTYPE, "a fused residual needs FP64 arrays");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const TileCfg cfg = default_cfg2(a.dtype, a.nx(), a.ny(), a.nz());
  GridArgs g = make_args2(&a, &b, &c, nullptr, h, cfg, 0);
  if (resid_out == nullptr) {
    J3D_HIP(launch_sweep2_one(a.dtype, F_WRITE, cfg, g, nullptr, nullptr, st));
    return J3D_OK;
  }
  Scratch* s = nullptr;
  J3D_TRY(get_scratch(st, &s));
  const int nt = g.tiles_x * g.tiles_y * g.tiles_z;
  J3D_TRY(ensure_partials(s, nt));
  J3D_HIP(launch_sweep2_one(J3D_F64, F_WRITE | F_RES, cfg, g, s->partials, nullptr, st));
  const bool host = (flags & J3D_HOST_RESULT) != 0;
  double* dst = host ? &s->ctl->value : resid_out;
  J3D_HIP(launch_reduce_one(s->partials, 0, nt, dst, nullptr, 0.0, 0, nullptr, nullptr, nullptr, st));
  if (host) {
    J3D_HIP(hipMemcpyAsync(&s->ctl_host->value, &s->ctl->value, sizeof(double),
                           hipMemcpyDeviceToHost, st));
    J3D_HIP(hipStreamSynchronize(st));
    *resid_out = s->ctl_host->value;
  }
  return J3D_OK;
}

int jacobi3d_sweep3(const j3d_array* u_in, j3d_array* u_out, const j3d_array* f, double h,
                    uint32_t flags, double* resid_out, void* stream) {
  Sweep3Call k;
  J3D_TRY(check_sweep3_call(u_in, u_out, f, h, flags, resid_out, &k));
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (resid_out == nullptr) {
    J3D_HIP(launch_sweep3_one(k.a.dtype, F_WRITE, k.cfg, k.g, nullptr, nullptr, st));
    return J3D_OK;
  }
  Scratch* s = nullptr;
  J3D_TRY(get_scratch(st, &s));
  const int nt = k.g.tiles_x * k.g.tiles_y * k.g.tiles_z;
  J3D_TRY(ensure_partials(s, nt));
  J3D_HIP(launch_sweep3_one(J3D_F64, F_WRITE | k.res_flag, k.cfg, k.g, s->partials, nullptr, st));
  const bool host = (flags & J3D_HOST_RESULT) != 0;
  double* dst = host ? &s->ctl->value : resid_out;
  J3D_HIP(launch_reduce_one(s->partials, 0, nt, dst, nullptr, 0.0, 0, nullptr, nullptr, nullptr, st));
  if (host) {
    J3D_HIP(hipMemcpyAsync(&s->ctl_host->value, &s->ctl->value, sizeof(double),
                           hipMemcpyDeviceToHost, st));
    J3D_HIP(hipStreamSynchronize(st));
    *resid_out = s->ctl_host->value;
  }
  return J3D_OK;
}

int residual_l2(const j3d_array* u, const j3d_array* f, double h, uint32_t flags, double* out,
                void* stream) {
  Field a, c;
  J3D_TRY(check_field(u, J3D_F64, &a, "u"));
  J3D_TRY(check_field(f, J3D_F64, &c, "f"));
  J3D_TRY(check_same_interior(a, c, "u", "f"));
  J3D_TRY(check_h(h));
  if ((flags & ~J3D_HOST_RESULT) != 0) return fail(J3D_EINVAL, "unknown flags 0x%x", flags);
  if (out == nullptr) return fail(J3D_EINVAL, "out: null pointer");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Scratch* s = nullptr;
  J3D_TRY(get_scratch(st, &s));
  const TileCfg cfg = default_cfg(J3D_F64, a.nx(), a.ny(), a.nz());
  const bool host = (flags & J3D_HOST_RESULT) != 0;
  J3D_TRY(norm_pass(F_RES, a, c, nullptr, h, cfg, host ? &s->ctl->value : out, st, s));
  if (host) {
    J3D_HIP(hipMemcpyAsync(&s->ctl_host->value, &s->ctl->value, sizeof(double),
                           hipMemcpyDeviceToHost, st));
    J3D_HIP(hipStreamSynchronize(st));
    *out = s->ctl_host->value;
  }
  return J3D_OK;
}

int j3d_fill_uniform(j3d_array* a, uint64_t seed, uint32_t stream_id, double lo, double hi,
                     double halo, void* stream) {
  Field x;
  J3D_TRY(check_field_wide(a, J3D_F64, &x, "a"));
  if (x.ey > 65535 || x.ez > 65535) return fail(J3D_EINVAL, "fill: y/z extents above 65535");
  const unsigned long long key = seed ^ (static_cast<unsigned long long>(stream_id) << 40);
  J3D_HIP(launch_fill_uniform(reinterpret_cast<double*>(x.base), x.ex, x.ey, x.ez, x.sy, x.sz, key,
                              lo, hi, halo, static_cast<hipStream_t>(stream)));
  return J3D_OK;
}

int j3d_fill_const(j3d_array* a, double value, void* stream) {
  Field x;
  J3D_TRY(check_field_wide(a, -1, &x, "a"));
  if (x.ey > 65535 || x.ez > 65535) return fail(J3D_EINVAL, "fill: y/z extents above 65535");
  J3D_HIP(launch_fill_const(x.base, x.dtype, x.ex, x.ey, x.ez, x.sy, x.sz, value,
                            static_cast<hipStream_t>(stream)));
  return J3D_OK;
}

int j3d_bandwidth_probe(const double* src, double* dst, int64_t n, int32_t reps, double* gbps,
                        void* stream) {
  if (src == nullptr || dst == nullptr || gbps == nullptr || n < 2 || reps < 1)
    return fail(J3D_EINVAL, "bandwidth probe: bad arguments");
  if ((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return fail(J3D_EINVAL, "bandwidth probe: buffers must be 16-byte aligned");
  if ((src < dst && src + n > dst) || (dst < src && dst + n > src) || src == dst)
    return fail(J3D_EALIAS, "bandwidth probe: buffers overlap");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  J3D_HIP(hipEventCreate(&e0));
  J3D_HIP(hipEventCreate(&e1));
  double best = 0.0;
  for (int v = 0; v < kCopyVariants; ++v) {
    J3D_HIP(launch_copy_variant(v, src, dst, n, st));  // warm-up
    for (int r = 0; r < reps; ++r) {
      J3D_HIP(hipEventRecord(e0, st));
      J3D_HIP(launch_copy_variant(v, src, dst, n, st));
      J3D_HIP(hipEventRecord(e1, st));
      J3D_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      J3D_HIP(hipEventElapsedTime(&ms, e0, e1));
      const double rate = 2.0 * 8.0 * (double)n / (ms * 1e-3) / 1e9;
      if (rate > best) best = rate;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *gbps = best;
  return J3D_OK;
}

int j3d_bandwidth_probe_triad(const double* a, const double* b, double* dst, int64_t n, int32_t reps,
                              double* gbps, void* stream) {
  if (a == nullptr || b == nullptr || dst == nullptr || gbps == nullptr || n < 2 || reps < 1)
    return fail(J3D_EINVAL, "triad probe: bad arguments");
  if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(dst)) % 16 != 0)
    return fail(J3D_EINVAL, "triad probe: buffers must be 16-byte aligned");
  auto overlap = [n](const double* x, const double* y) { return x < y + n && y < x + n; };
  if (overlap(a, dst) || overlap(b, dst)) return fail(J3D_EALIAS, "triad probe: dst overlaps a source");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  J3D_HIP(hipEventCreate(&e0));
  J3D_HIP(hipEventCreate(&e1));
  double best = 0.0;
  for (int v = 0; v < kTriadVariants; ++v) {
    J3D_HIP(launch_triad_variant(v, a, b, dst, n, st));  // warm-up
    for (int r = 0; r < reps; ++r) {
      J3D_HIP(hipEventRecord(e0, st));
      J3D_HIP(launch_triad_variant(v, a, b, dst, n, st));
      J3D_HIP(hipEventRecord(e1, st));
      J3D_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      J3D_HIP(hipEventElapsedTime(&ms, e0, e1));
      const double rate = 3.0 * 8.0 * (double)n / (ms * 1e-3) / 1e9;
      if (rate > best) best = rate;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *gbps = best;
  return J3D_OK;
}

// sum and dot_product share one path: y == nullptr selects the sum.
static int reduce_vec(const double* x, const double* y, int64_t n, uint32_t flags, double* out, void* stream,
                      const char* what) {
  if (out == nullptr) return fail(J3D_EINVAL, "%s: out is a null pointer", what);
  if (n < 0) return fail(J3D_EINVAL, "%s: n must be >= 0", what);
  if ((flags & ~J3D_HOST_RESULT) != 0) return fail(J3D_EINVAL, "%s: unknown flags 0x%x", what, flags);
  if (n > 0 && x == nullptr) return fail(J3D_EINVAL, "%s: x is a null pointer", what);
  if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y) | reinterpret_cast<uintptr_t>(out)) % 8 != 0)
    return fail(J3D_EINVAL, "%s: pointers must be 8-byte aligned", what);
  const bool host = (flags & J3D_HOST_RESULT) != 0;
  if (!host && n > 0) {
    const bool in_x = out >= x && out < x + n;
    const bool in_y = y != nullptr && out >= y && out < y + n;
    if (in_x || in_y) return fail(J3D_EALIAS, "%s: out overlaps an input", what);
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  Scratch* s = nullptr;
  J3D_TRY(get_scratch(st, &s));
  J3D_TRY(ensure_partials(s, (size_t)sum_blocks(n)));
  double* dst = host ? &s->ctl->value : out;
  J3D_HIP(launch_sum(x, y, n, s->partials, dst, st));
  if (host) {
    J3D_HIP(hipMemcpyAsync(&s->ctl_host->value, &s->ctl->value, sizeof(double), hipMemcpyDeviceToHost, st));
    J3D_HIP(hipStreamSynchronize(st));
    *out = s->ctl_host->value;
  }
  return J3D_OK;
}

int j3d_sum(const double* x, int64_t n, uint32_t flags, double* out, void* stream) {
  return reduce_vec(x, nullptr, n, flags, out, stream, "j3d_sum");
}

int j3d_dot(const double* x, const double* y, int64_t n, uint32_t flags, double* out, void* stream) {
  if (n > 0 && y == nullptr) return fail(J3D_EINVAL, "j3d_dot: y is a null pointer");
  return reduce_vec(x, y, n, flags, out, stream, "j3d_dot");
}

int j3d_release_cache(void) {
  release_batch_cache();
  return release_all_scratch();
}

}  // extern "C"
