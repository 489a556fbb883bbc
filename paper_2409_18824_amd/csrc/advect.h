// Launch interface of the multi-field stencil kernels (momentum advection,
// tracer advection) of libj3d.
#pragma once

#include <hip/hip_runtime.h>

namespace j3d {

// Multi-field stencils (momentum advection, tracer advection).  Every
// pointer addresses the array corner (Fortran lbound); interior point
// (i,j,k) of an input is at i + siy*j + siz*k, of an output at
// i + soy*j + soz*k.
struct AdvArgs {
  const double* in[4];  // momentum: u, v, w; tracer: u, v, w, r
  const double* t;      // tracer: the input iterate (shares the input strides)
  double* out[3];       // momentum: su, sv, sw; tracer: out[0] = next iterate
  int nx, ny, nz;
  int siy;
  long long siz;
  int soy;
  long long soz;
  double cx, cy, cz;    // momentum: 0.25 / spacing
  int tiles_x, tiles_y, yblocks, planes;  // set by the launchers
  int buffer_ok;        // every plane of every field spans less than 2^31 bytes
};

// Tile shape of the advection kernels: rows per thread (2, 4 or 8), z-planes
// per wavefront, nontemporal stores (0 or 1), and for the momentum advection
// whether its loads run one plane ahead (pf = 1: 2 or 4 rows per thread;
// taken only where AdvArgs::buffer_ok, else the kernel without it runs).
struct AdvectCfg {
  int ry;
  int planes;
  int nt;
  int pf = 0;
};
bool advect_cfg_supported(const AdvectCfg& c);
hipError_t launch_pw_advect(const AdvArgs& a, const AdvectCfg& c, hipStream_t st);
hipError_t launch_tracer_advect(const AdvArgs& a, const AdvectCfg& c, hipStream_t st);
// Two tracer steps per launch (t = in iterate, out[0] = iterate two steps
// later); rows per thread 2, 4 or 6.
bool tracer2_cfg_supported(const AdvectCfg& c);
hipError_t launch_tracer2_advect(const AdvArgs& a, const AdvectCfg& c, hipStream_t st);

}  // namespace j3d
