// jacobi2d_sweeps: the paper's 2D Laplace jacobi benchmark (Sec. "Flang
// performance comparison") as a library call.
//
// nsweeps sweeps run as launches of 8 sweeps (plus 4, 2, 1 for the rest),
// ping-ponging between the two arrays.  The number of launches is kept at the
// parity of nsweeps (one launch is split in two when needed), so the result
// lands in u_a exactly when nsweeps is even, as if the arrays alternated every
// sweep.  Long runs replay a captured graph of 64 launches.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "runtime.h"

using namespace j3d;

namespace {

// Sweeps per launch for nsweeps sweeps, with the launch count's parity equal
// to nsweeps'.
std::vector<int> schedule(long long nsweeps) {
  std::vector<int> v((size_t)(nsweeps / 8), 8);
  for (int t : {4, 2, 1})
    if (nsweeps % 8 & t) v.push_back(t);
  if (v.size() % 2 != (size_t)(nsweeps % 2)) {
    // split the last launch of more than one sweep into two halves
    for (size_t i = v.size(); i-- > 0;)
      if (v[i] > 1) {
        const int half = v[i] / 2;
        v[i] = half;
        v.insert(v.begin() + (long)i, half);
        break;
      }
  }
  return v;
}

constexpr long long kGraphLaunches = 64;  // even: the arrays return to their roles

}  // namespace

extern "C" int jacobi2d_sweeps(j3d_array* u_a, j3d_array* u_b, int64_t nsweeps, double h,
                               uint32_t flags, double* resid_out, void* stream) {
  Field a, b;
  J3D_TRY(check_field2d(u_a, J3D_F64, &a, "u_a"));
  J3D_TRY(check_field2d(u_b, J3D_F64, &b, "u_b"));
  if (a.ex != b.ex || a.ey != b.ey)
    return fail(J3D_EINVAL, "u_a interior %dx%d differs from u_b interior %dx%d", a.nx(), a.ny(), b.nx(), b.ny());
  if (nsweeps < 0) return fail(J3D_EINVAL, "nsweeps must be >= 0");
  if ((flags & ~J3D_HOST_RESULT) != 0) return fail(J3D_EINVAL, "unknown flags 0x%x", flags);
  if (resid_out != nullptr) J3D_TRY(check_h(h));
  if (fields_overlap(a, b)) return fail(J3D_EALIAS, "u_a and u_b overlap");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int nx = a.ex - 2, ny = a.ey - 2;
  const int sa = (int)a.sy, sb = (int)b.sy;
  double* pa = reinterpret_cast<double*>(a.base);
  double* pb = reinterpret_cast<double*>(b.base);

  const std::vector<int> plan = schedule(nsweeps);
  size_t i = 0;
  bool in_a = true;  // the current iterate is in u_a
  // Whole graphs of kGraphLaunches launches of 8 sweeps (the plan starts
  // with its 8-sweep launches) when there are two or more of them.
  long long eights = 0;
  while (eights < (long long)plan.size() && plan[(size_t)eights] == 8) ++eights;
  if (eights / kGraphLaunches >= 2) {
    Scratch* s = nullptr;
    J3D_TRY(get_scratch(st, &s));
    std::string key = "jacobi2d";
    const long long meta[6] = {(long long)(uintptr_t)pa, (long long)(uintptr_t)pb, nx, ny, sa, sb};
    key.append(reinterpret_cast<const char*>(meta), sizeof meta);
    hipGraphExec_t exec = nullptr;
    J3D_TRY(solve_graph(s, key, [&](hipStream_t q) -> int {
      for (long long l = 0; l < kGraphLaunches; ++l) {
        const bool from_a = (l % 2) == 0;
        J3D_HIP(launch_jacobi2d(8, from_a ? pa : pb, from_a ? pb : pa, nx, ny, from_a ? sa : sb,
                                from_a ? sb : sa, nullptr, q));
      }
      return J3D_OK;
    }, &exec));
    for (long long g = 0; g < eights / kGraphLaunches; ++g) J3D_HIP(hipGraphLaunch(exec, st));
    i = (size_t)(eights / kGraphLaunches * kGraphLaunches);
  }
  for (; i < plan.size(); ++i) {
    J3D_HIP(launch_jacobi2d(plan[i], in_a ? pa : pb, in_a ? pb : pa, nx, ny, in_a ? sa : sb, in_a ? sb : sa,
                            nullptr, st));
    in_a = !in_a;
  }
  // after the graphs the iterate is in u_a again, so in_a only tracks the rest
  if (resid_out == nullptr) return J3D_OK;
  const bool res_in_a = (nsweeps % 2) == 0;
  Scratch* s = nullptr;
  J3D_TRY(get_scratch(st, &s));
  const int nb = laplace2d_res_blocks(ny);
  J3D_TRY(ensure_partials(s, (size_t)nb));
  J3D_HIP(launch_laplace2d_res(res_in_a ? pa : pb, nx, ny, res_in_a ? sa : sb, h, s->partials, st));
  const bool host = (flags & J3D_HOST_RESULT) != 0;
  double* dst = host ? &s->ctl->value : resid_out;
  J3D_HIP(launch_reduce_one(s->partials, 0, nb, dst, nullptr, 0.0, 0, nullptr, nullptr, nullptr, st));
  if (host) {
    J3D_HIP(hipMemcpyAsync(&s->ctl_host->value, &s->ctl->value, sizeof(double), hipMemcpyDeviceToHost, st));
    J3D_HIP(hipStreamSynchronize(st));
    *resid_out = s->ctl_host->value;
  }
  return J3D_OK;
}
