// FP64 instantiations of the sweep-shaped passes: sweep, sweep with fused
// residual, residual only, defect step (residual + FP32 copy), norm of f.
#include "sweep.h"

namespace j3d {
namespace sweep_detail {

hipError_t dispatch_f64(unsigned flags, const Launch& L) {
  switch (flags) {
    case F_WRITE: return by_shape<double, F_WRITE>(L);
    case F_WRITE | F_RES: return by_shape<double, F_WRITE | F_RES>(L);
    case F_RES: return by_shape<double, F_RES>(L);
    case F_RES | F_R32: return by_shape<double, F_RES | F_R32>(L);
    case F_NORM: return by_shape<double, F_NORM>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sweep_detail
}  // namespace j3d
