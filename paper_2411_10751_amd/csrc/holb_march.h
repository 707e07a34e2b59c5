// Plane-marching fused kernels (variants >= 1).  Placeholder until written:
// no marching variant exists yet, so every configuration runs the generic path.
#pragma once

#include "holb_internal.h"

namespace holb {

inline int march_num_variants(const LaunchCtx&) { return 0; }
inline bool march_variant_supported(const LaunchCtx&, int) { return false; }

template <class L, int ST, int FAM>
hipError_t march_step(const LaunchCtx&)
{
    return hipErrorNotSupported;
}

}  // namespace holb
