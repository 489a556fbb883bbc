// pw_advection / tracer_advection: the multi-field stencils standing in for
// the paper's pw-advection and tra-adv benchmarks (Sec. "Flang performance
// comparison": field counts and grid sizes only).
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "advect.h"
#include "runtime.h"

using namespace j3d;

namespace {

// Tile shapes measured fastest on the paper's grids, nontemporal stores
// throughout: for the momentum advection (2048 x 1024 x 1024) 4 rows per
// thread, 64 z-planes per wavefront, loads one plane ahead (19.5 ms per call
// against 20.2 with 8 rows, 128 planes and no prefetch); for the tracer
// (1024 x 512 x 512) 8 rows, 64 planes.
// J3D_ADVECT_TILE="ry,planes,nt[,pf]" overrides both (shape sweeps).
AdvectCfg advect_cfg(bool tracer) {
  AdvectCfg c = tracer ? AdvectCfg{8, 64, 1, 0} : AdvectCfg{4, 64, 1, 1};
  if (const char* e = std::getenv("J3D_ADVECT_TILE")) {
    AdvectCfg t{0, 0, 0, 0};
    const int n = std::sscanf(e, "%d,%d,%d,%d", &t.ry, &t.planes, &t.nt, &t.pf);
    if (n >= 3 && advect_cfg_supported(t)) c = t;
  }
  return c;
}

// Every plane (interior and halo) of the field under 2^31 bytes.
bool plane_below_2gib(const Field& a) {
  return ((long long)(a.ey - 1) * a.sy + a.ex) * (long long)a.esize < (1LL << 31);
}

// Two-step tracer pass: 6 rows per thread, 64 planes, nontemporal stores
// (fastest at 1024 x 512 x 512).  J3D_TRACER2_TILE="ry,planes,nt" overrides
// it; J3D_TRACER_STEPS_PER_PASS=1 runs every step as its own pass.
AdvectCfg tracer2_cfg() {
  AdvectCfg c{6, 64, 1};
  if (const char* e = std::getenv("J3D_TRACER2_TILE")) {
    AdvectCfg t{0, 0, 0};
    if (std::sscanf(e, "%d,%d,%d", &t.ry, &t.planes, &t.nt) == 3 && tracer2_cfg_supported(t)) c = t;
  }
  return c;
}

bool tracer_two_steps_per_pass() {
  const char* e = std::getenv("J3D_TRACER_STEPS_PER_PASS");
  return !(e != nullptr && std::atoi(e) == 1);
}

int check_spacing(double d, const char* name) {
  if (!(std::isfinite(d) && d > 0.0)) return fail(J3D_EINVAL, "%s must be finite and > 0", name);
  return J3D_OK;
}

int check_same_layout(const Field& a, const Field& b, const char* an, const char* bn) {
  J3D_TRY(check_same_interior(a, b, an, bn));
  if (a.sy != b.sy || a.sz != b.sz)
    return fail(J3D_EINVAL, "%s strides (%lld, %lld) differ from %s strides (%lld, %lld)", an, a.sy, a.sz, bn,
                b.sy, b.sz);
  return J3D_OK;
}

}  // namespace

extern "C" int pw_advection(const j3d_array* u, const j3d_array* v, const j3d_array* w, j3d_array* su,
                            j3d_array* sv, j3d_array* sw, double dx, double dy, double dz,
                            void* stream) {
  const j3d_array* d[6] = {u, v, w, su, sv, sw};
  const char* names[6] = {"u", "v", "w", "su", "sv", "sw"};
  Field f[6];
  for (int q = 0; q < 6; ++q) J3D_TRY(check_field_wide(d[q], J3D_F64, &f[q], names[q]));
  for (int q = 1; q < 3; ++q) J3D_TRY(check_same_layout(f[0], f[q], names[0], names[q]));
  J3D_TRY(check_same_interior(f[0], f[3], names[0], names[3]));
  for (int q = 4; q < 6; ++q) J3D_TRY(check_same_layout(f[3], f[q], names[3], names[q]));
  J3D_TRY(check_spacing(dx, "dx"));
  J3D_TRY(check_spacing(dy, "dy"));
  J3D_TRY(check_spacing(dz, "dz"));
  for (int o = 3; o < 6; ++o)
    for (int q = 0; q < o; ++q)
      if (fields_overlap(f[o], f[q]))
        return fail(J3D_EALIAS, "%s overlaps %s", names[o], names[q]);
  AdvArgs a{};
  for (int q = 0; q < 3; ++q) {
    a.in[q] = reinterpret_cast<const double*>(f[q].base);
    a.out[q] = reinterpret_cast<double*>(f[3 + q].base);
  }
  a.nx = f[0].nx();
  a.ny = f[0].ny();
  a.nz = f[0].nz();
  a.siy = (int)f[0].sy;
  a.siz = f[0].sz;
  a.soy = (int)f[3].sy;
  a.soz = f[3].sz;
  a.cx = 0.25 / dx;
  a.cy = 0.25 / dy;
  a.cz = 0.25 / dz;
  a.buffer_ok = 1;
  for (int q = 0; q < 6; ++q)
    if (!plane_below_2gib(f[q])) a.buffer_ok = 0;
  J3D_HIP(launch_pw_advect(a, advect_cfg(false), static_cast<hipStream_t>(stream)));
  return J3D_OK;
}

extern "C" int tracer_advection(j3d_array* t_a, j3d_array* t_b, const j3d_array* u,
                                const j3d_array* v, const j3d_array* w, const j3d_array* r, int64_t niter,
                                void* stream) {
  const j3d_array* d[6] = {t_a, t_b, u, v, w, r};
  const char* names[6] = {"t_a", "t_b", "u", "v", "w", "r"};
  Field f[6];
  for (int q = 0; q < 6; ++q) J3D_TRY(check_field_wide(d[q], J3D_F64, &f[q], names[q]));
  for (int q = 1; q < 6; ++q) J3D_TRY(check_same_layout(f[0], f[q], names[0], names[q]));
  if (niter < 0) return fail(J3D_EINVAL, "niter must be >= 0");
  for (int o = 0; o < 2; ++o)
    for (int q = 0; q < 6; ++q)
      if (q != o && fields_overlap(f[o], f[q])) return fail(J3D_EALIAS, "%s overlaps %s", names[o], names[q]);
  AdvArgs a{};
  for (int q = 0; q < 4; ++q) a.in[q] = reinterpret_cast<const double*>(f[2 + q].base);
  a.nx = f[0].nx();
  a.ny = f[0].ny();
  a.nz = f[0].nz();
  a.siy = a.soy = (int)f[0].sy;
  a.siz = a.soz = f[0].sz;
  const AdvectCfg c1 = advect_cfg(true);
  const AdvectCfg c2 = tracer2_cfg();
  hipStream_t st = static_cast<hipStream_t>(stream);
  double* ta = reinterpret_cast<double*>(f[0].base);
  double* tb = reinterpret_cast<double*>(f[1].base);
  // n2 launches of two steps, then n1 of one; every launch swaps the arrays,
  // so the number of launches keeps the parity of niter (one two-step launch
  // is split in two when it would not) and the result is in t_a exactly when
  // niter is even.
  int64_t n2 = tracer_two_steps_per_pass() ? niter / 2 : 0;
  int64_t n1 = niter - 2 * n2;
  if (((n2 + n1) & 1) != (niter & 1)) {
    n2 -= 1;
    n1 += 2;
  }
  bool from_a = true;
  for (int64_t q = 0; q < n2 + n1; ++q) {
    a.t = from_a ? ta : tb;
    a.out[0] = from_a ? tb : ta;
    if (q < n2)
      J3D_HIP(launch_tracer2_advect(a, c2, st));
    else
      J3D_HIP(launch_tracer_advect(a, c1, st));
    from_a = !from_a;
  }
  return J3D_OK;
}
