// Cross-lane reads for wave64 kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace ssn {

// lane l's v, for a wave-uniform l (v_readlane into scalar registers)
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
    return __hiloint2double(hi, lo);
}

}  // namespace ssn
