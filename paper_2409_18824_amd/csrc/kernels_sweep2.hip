// Instantiations of the FP64 two-sweep (temporally blocked) pass: plain
// sweeps, optionally with the fused residual of the input iterate.
#include "sweep2.h"

namespace j3d {
namespace sweep_detail {

hipError_t dispatch_sweep2_f64(unsigned flags, const Launch& L) {
  switch (flags) {
    case F_WRITE: return by_rows2<double, F_WRITE>(L);
    case F_WRITE | F_RES: return by_rows2<double, F_WRITE | F_RES>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sweep_detail
}  // namespace j3d
