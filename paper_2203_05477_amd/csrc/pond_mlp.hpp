// pond_mlp.hpp -- learned seed of the face-frame iteration (placeholder until the MLP
// kernels are in): the device-side network and its launch.
#pragma once
#include <hip/hip_runtime.h>

#include "pond_kernels.hpp"

namespace pond {

struct MlpDevice {
    bool ready = false;
};

inline void mlp_free(MlpDevice &) {}

template <int D, typename R>
hipError_t mlp_seed_launch(const MlpDevice &, const Params &, const State<R> &, hipStream_t)
{
    return hipErrorNotSupported;
}

} // namespace pond
