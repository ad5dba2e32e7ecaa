// Device arithmetic shared by the pair-sum kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace mfs {

// 1/sqrt(r2) in FP64.  The hardware estimate y = v_rsq_f64(r2) has a relative
// error of about 2^-24 (measured over 2^20 arguments in [1e-8, 1e8]).  With
// e = 1 - r2 y^2, the exact value is y (1 - e)^(-1/2) = y (1 + e/2 + 3e^2/8 +
// O(e^3)), so one step y + y e (1/2 + 3e/8) leaves a truncation error near
// (5/16) e^3, about 2^-70: below FP64 rounding.  The same arguments give at
// most 0.99 ulp against a long-double reference, as two Newton steps do, in
// five FP64 operations instead of eight.
__device__ __forceinline__ double rsqrt_f64(double r2) {
    const double y = __builtin_amdgcn_rsq(r2);
    const double e = __builtin_fma(-r2 * y, y, 1.0);
    const double c = __builtin_fma(0.375, e, 0.5);
    return __builtin_fma(y * e, c, y);
}

}  // namespace mfs
