// FP32 instantiations of the correction sweeps of the mixed-precision solve:
// plain sweep, first sweep from a zero iterate, last sweep folded into the
// FP64 update, and the one-sweep cycle (first and last at once).
#include "sweep.h"

namespace j3d {
namespace sweep_detail {

hipError_t dispatch_f32(unsigned flags, const Launch& L) {
  switch (flags) {
    case F_WRITE: return by_shape<float, F_WRITE>(L);
    case F_WRITE | F_FIRST: return by_shape<float, F_WRITE | F_FIRST>(L);
    case F_LAST: return by_shape<float, F_LAST>(L);
    case F_LAST | F_FIRST: return by_shape<float, F_LAST | F_FIRST>(L);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace sweep_detail
}  // namespace j3d
