// Instantiation unit: every kernel of lattice D3Q39 for FP16 and BF16 storage.
#include "holb_kernels.h"

namespace holb {

hipError_t dispatch_d3_16(HOLB_DISPATCH_ARGS) { return dispatch_set<D3Q39, true>(c, op, a, b, d, o1, o2, o3, dout); }

}  // namespace holb
