// Host runtime of libj3d: error reporting, descriptor validation, scratch.
#include "runtime.h"

#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <map>
#include <mutex>
#include <utility>

namespace j3d {

namespace {
thread_local std::string t_err;
std::mutex g_scratch_mu;
std::map<std::pair<int, hipStream_t>, Scratch*> g_scratch;
}  // namespace

const char* last_error_text() { return t_err.c_str(); }

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  t_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(J3D_EHIP, "%s: %s (%d)", what, hipGetErrorString(e), (int)e);
}

double now_seconds() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

namespace {

int check_field_impl(const j3d_array* a, int dtype, Field* out, const char* name, bool wide) {
  if (a == nullptr) return fail(J3D_EINVAL, "%s: null descriptor", name);
  if (a->base == nullptr) return fail(J3D_EINVAL, "%s: null base address", name);
  if (a->reserved != 0) return fail(J3D_EINVAL, "%s: reserved field must be 0", name);
  if (a->dtype != J3D_F64 && a->dtype != J3D_F32)
    return fail(J3D_EDTYPE, "%s: unknown dtype %d", name, a->dtype);
  if (dtype >= 0 && a->dtype != dtype)
    return fail(J3D_EDTYPE, "%s: dtype %s where %s is required", name,
                a->dtype == J3D_F64 ? "F64" : "F32", dtype == J3D_F64 ? "F64" : "F32");
  long long ext[3];
  for (int d = 0; d < 3; ++d) {
    ext[d] = a->ubound[d] - a->lbound[d] + 1;
    if (a->ubound[d] < a->lbound[d] || ext[d] < 3)
      return fail(J3D_EINVAL, "%s: axis %d bounds %lld:%lld leave no interior", name, d,
                  (long long)a->lbound[d], (long long)a->ubound[d]);
    if (ext[d] > (1LL << 30)) return fail(J3D_EINVAL, "%s: axis %d too long", name, d);
  }
  if (a->stride[0] != 1) return fail(J3D_EINVAL, "%s: stride[0] must be 1 (x is unit stride)", name);
  if (a->stride[1] < ext[0])
    return fail(J3D_EINVAL, "%s: stride[1]=%lld < extent[0]=%lld", name, (long long)a->stride[1], ext[0]);
  if (a->stride[2] < a->stride[1] * ext[1])
    return fail(J3D_EINVAL, "%s: stride[2]=%lld < stride[1]*extent[1]=%lld", name,
                (long long)a->stride[2], (long long)(a->stride[1] * ext[1]));
  const long long plane_off = (ext[1] - 1) * a->stride[1] + (ext[0] - 1);
  if (wide) {
    if (plane_off >= (1LL << 31) - 1)
      return fail(J3D_EINVAL, "%s: largest offset within a plane %lld exceeds 2^31", name, plane_off);
    if (a->stride[2] > ((1LL << 46) - 1) / ext[2])
      return fail(J3D_EINVAL, "%s: array spans more than 2^46 elements", name);
  } else {
    const long long maxoff = (ext[2] - 1) * a->stride[2] + plane_off;
    if (maxoff >= (1LL << 31) - 1)
      return fail(J3D_EINVAL, "%s: largest element offset %lld exceeds 2^31", name, maxoff);
  }
  const int esize = a->dtype == J3D_F64 ? 8 : 4;
  if (reinterpret_cast<uintptr_t>(a->base) % esize != 0)
    return fail(J3D_EINVAL, "%s: base is not aligned to its element size", name);
  if (out) {
    out->base = static_cast<char*>(a->base);
    out->dtype = a->dtype;
    out->esize = esize;
    out->ex = (int)ext[0];
    out->ey = (int)ext[1];
    out->ez = (int)ext[2];
    out->sy = a->stride[1];
    out->sz = a->stride[2];
  }
  return J3D_OK;
}

}  // namespace

int check_field(const j3d_array* a, int dtype, Field* out, const char* name) {
  return check_field_impl(a, dtype, out, name, false);
}

int check_field_wide(const j3d_array* a, int dtype, Field* out, const char* name) {
  return check_field_impl(a, dtype, out, name, true);
}

int check_field2d(const j3d_array* a, int dtype, Field* out, const char* name) {
  if (a == nullptr) return fail(J3D_EINVAL, "%s: null descriptor", name);
  if (a->lbound[2] != a->ubound[2])
    return fail(J3D_EINVAL, "%s: a rank-2 array has lbound[2] == ubound[2]", name);
  j3d_array b = *a;  // validate axes 0 and 1 with a stand-in third axis of extent 3
  b.ubound[2] = b.lbound[2] + 2;
  b.stride[2] = b.stride[1] * (b.ubound[1] - b.lbound[1] + 1);
  J3D_TRY(check_field(&b, dtype, out, name));
  if (out) {
    out->ez = 1;
    out->sz = 0;
  }
  return J3D_OK;
}

bool fields_overlap(const Field& a, const Field& b) {
  const char* a0 = a.base;
  const char* a1 = a.base + a.span_bytes();
  const char* b0 = b.base;
  const char* b1 = b.base + b.span_bytes();
  return a0 < b1 && b0 < a1;
}

int check_same_interior(const Field& a, const Field& b, const char* an, const char* bn) {
  if (a.ex != b.ex || a.ey != b.ey || a.ez != b.ez)
    return fail(J3D_EINVAL, "%s interior %dx%dx%d differs from %s interior %dx%dx%d", an, a.nx(),
                a.ny(), a.nz(), bn, b.nx(), b.ny(), b.nz());
  return J3D_OK;
}

bool plane_fits_u32(const Field& a) {
  const long long span = ((long long)(a.ey - 1) * a.sy + a.ex) * (long long)a.esize;
  return span < (1LL << 32);
}

int check_h(double h) {
  if (!(h > 0.0) || !std::isfinite(h)) return fail(J3D_EINVAL, "h must be positive and finite");
  return J3D_OK;
}

GridArgs make_args(const Field* u, const Field* o, const Field* f, const Field* u64,
                   const Field* r32, double h, const TileCfg& c, int tile0) {
  GridArgs g{};
  const Field* any = u ? u : (f ? f : o);
  g.u = u ? u->base : nullptr;
  g.o = o ? o->base : nullptr;
  g.f = f ? f->base : nullptr;
  g.u64 = u64 ? reinterpret_cast<double*>(u64->base) : nullptr;
  g.r32 = r32 ? reinterpret_cast<float*>(r32->base) : nullptr;
  g.nx = any->nx();
  g.ny = any->ny();
  g.nz = any->nz();
  g.su_y = u ? (int)u->sy : 0;
  g.su_z = u ? (int)u->sz : 0;
  g.so_y = o ? (int)o->sy : 0;
  g.so_z = o ? (int)o->sz : 0;
  g.sf_y = f ? (int)f->sy : 0;
  g.sf_z = f ? (int)f->sz : 0;
  g.s64_y = u64 ? (int)u64->sy : 0;
  g.s64_z = u64 ? (int)u64->sz : 0;
  g.sr_y = r32 ? (int)r32->sy : 0;
  g.sr_z = r32 ? (int)r32->sz : 0;
  tile_counts(g.nx, g.ny, g.nz, c, &g.tiles_x, &g.tiles_y, &g.tiles_z);
  g.tile0 = tile0;
  g.planes = c.planes;
  g.h2 = h * h;
  g.h2f = static_cast<float>(h * h);
  g.order = c.order;
  g.chunk = (g.tiles_x * g.tiles_y + 7) / 8;
  // the buffer-addressed one-sweep path needs every plane (interior and
  // halo) under 2^31 bytes
  const Field* fs[5] = {u, o, f, u64, r32};
  for (const Field* a : fs)
    if (a && ((long long)(g.ny + 1) * a->sy + (g.nx + 2)) * a->esize >= (1LL << 31)) g.wide_planes = 1;
  return g;
}

GridArgs make_args2(const Field* u, const Field* o, const Field* f, const Field* u64, double h,
                    const TileCfg& c, int tile0) {
  GridArgs g = make_args(u, o, f, u64, nullptr, h, c, tile0);
  tile2_counts(g.nx, g.ny, g.nz, c, &g.tiles_x, &g.tiles_y, &g.tiles_z);
  g.chunk = (g.tiles_x * g.tiles_y + 7) / 8;
  return g;
}

GridArgs make_args3(const Field* u, const Field* o, const Field* f, const Field* u64, double h,
                    const TileCfg& c, int tile0) {
  GridArgs g = make_args(u, o, f, u64, nullptr, h, c, tile0);
  tile3_counts(g.nx, g.ny, g.nz, c, &g.tiles_x, &g.tiles_y, &g.tiles_z);
  g.chunk = (g.tiles_x * g.tiles_y + 7) / 8;
  return g;
}

int dev_alloc(void** p, size_t bytes, const char* what) {
  *p = nullptr;
  hipError_t e = hipMalloc(p, bytes < 256 ? 256 : bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(J3D_ENOMEM, "%s: hipMalloc(%zu) failed: %s", what, bytes, hipGetErrorString(e));
  }
  return J3D_OK;
}

int get_scratch(hipStream_t st, Scratch** out) {
  int dev = 0;
  J3D_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto key = std::make_pair(dev, st);
  auto it = g_scratch.find(key);
  if (it != g_scratch.end()) {
    *out = it->second;
    return J3D_OK;
  }
  Scratch* s = new Scratch();
  s->device = dev;
  s->stream = st;
  void* p = nullptr;
  int rc = dev_alloc(&p, sizeof(Control), "control block");
  if (rc != J3D_OK) {
    delete s;
    return rc;
  }
  s->ctl = static_cast<Control*>(p);
  hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&s->ctl_host), sizeof(Control), hipHostMallocDefault);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev[0], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev[1], hipEventDisableTiming);
  if (e != hipSuccess) {
    (void)hipFree(s->ctl);
    delete s;
    return hip_fail(e, "scratch set-up");
  }
  g_scratch[key] = s;
  *out = s;
  return J3D_OK;
}

int ensure_partials(Scratch* s, size_t n) {
  if (n <= s->partials_cap) return J3D_OK;
  if (s->partials) J3D_HIP(hipFree(s->partials));
  s->partials = nullptr;
  s->partials_cap = 0;
  size_t cap = n + n / 4 + 1024;
  void* p = nullptr;
  J3D_TRY(dev_alloc(&p, cap * sizeof(double), "tile partials"));
  s->partials = static_cast<double*>(p);
  s->partials_cap = cap;
  return J3D_OK;
}

int ensure_hist(Scratch* s, size_t n) {
  if (n <= s->hist_cap) return J3D_OK;
  if (s->hist) J3D_HIP(hipFree(s->hist));
  s->hist = nullptr;
  s->hist_cap = 0;
  size_t cap = n + 64;
  void* p = nullptr;
  J3D_TRY(dev_alloc(&p, cap * sizeof(double), "residual history"));
  s->hist = static_cast<double*>(p);
  s->hist_cap = cap;
  return J3D_OK;
}

int ensure_work(Scratch* s, size_t bytes) {
  if (bytes <= s->work_bytes) return J3D_OK;
  if (s->work) J3D_HIP(hipFree(s->work));
  s->work = nullptr;
  s->work_bytes = 0;
  J3D_TRY(dev_alloc(&s->work, bytes, "solver work arrays"));
  s->work_bytes = bytes;
  return J3D_OK;
}

void free_solve_graph(SolveGraph* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
}

int release_all_scratch() {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (auto& kv : g_scratch) {
    Scratch* s = kv.second;
    (void)hipSetDevice(s->device);
    (void)hipStreamSynchronize(s->stream);
    if (s->partials) (void)hipFree(s->partials);
    if (s->hist) (void)hipFree(s->hist);
    if (s->work) (void)hipFree(s->work);
    if (s->ctl) (void)hipFree(s->ctl);
    if (s->ctl_host) (void)hipHostFree(s->ctl_host);
    for (auto& ev : s->ev)
      if (ev) (void)hipEventDestroy(ev);
    for (SolveGraph& g : s->graphs) free_solve_graph(&g);
    if (s->capture) (void)hipStreamDestroy(s->capture);
    delete s;
  }
  g_scratch.clear();
  (void)hipSetDevice(cur);
  return J3D_OK;
}

}  // namespace j3d
