// Instantiation unit: every kernel of lattice D2Q37 for FP16 and BF16 storage.
#include "holb_kernels.h"

namespace holb {

hipError_t dispatch_d2_16(HOLB_DISPATCH_ARGS) { return dispatch_set<D2Q37, true>(c, op, a, b, d, o1, o2, o3, dout); }

}  // namespace holb
