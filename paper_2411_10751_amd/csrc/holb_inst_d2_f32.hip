// Instantiation unit: every kernel of lattice D2Q37 for FP32 storage.
#include "holb_kernels.h"

namespace holb {

hipError_t dispatch_d2_f32(HOLB_DISPATCH_ARGS) { return dispatch_set<D2Q37, false>(c, op, a, b, d, o1, o2, o3, dout); }

}  // namespace holb
