// Device helpers of the FP32C state (hi, q) of one atom, shared by the
// sub-step kernels and by the kernels that read or write the state.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace l2t {

// ---- the FP32C state of one atom --------------------------------------------------
// T = hi + q * s(hi) exactly in FP64, with hi = fl32(T) (what neighbours read),
// s(hi) = 2^(max(f, -125) - 39) for f the frexp exponent of hi (hi = m 2^f,
// 1/2 <= m < 1; for a normal hi in [2^e, 2^(e+1)), f = e + 1 and s = 2^(e-38)),
// and q a 16-bit integer.  Rounding to nearest leaves |T - hi| <= ulp(hi)/2 =
// 2^(e-24) (2^-150 below the normal range), so |q| <= 2^14: q carries 15 bits
// below hi's last one, 39 significant bits in all, and a split rounds T by at
// most s (s/2 but for the halfway case below), 2^-38 of T.  Decoding and encoding are exact scalings by powers of
// two (v_frexp_exp, v_ldexp).
__device__ __forceinline__ int state_shift(float hi) {
    return max(__builtin_amdgcn_frexp_expf(hi), -125) - 39;
}
__device__ __forceinline__ double state_value(float hi, int16_t q) {
    return (double)hi + __builtin_ldexp((double)q, state_shift(hi));
}
// q of T given hi = fl32(T).  |q| = 2^14 puts hi + q s halfway between hi and
// its FP32 neighbour; it is kept only when hi is the even one of the two, so
// that fl32(hi + q s) = hi for every stored pair and a value read back and
// written again is the same pair (with an odd hi, q rounds to 2^14 - 1 instead,
// still within s of T).  A T that is not finite (flagged by the caller) gives
// a clamped q.
__device__ __forceinline__ int16_t state_lo(double T, float hi) {
    const double r = rint(__builtin_ldexp(T - (double)hi, -state_shift(hi)));
    const double lim = 16384.0 - (double)(__float_as_uint(hi) & 1u);
    return (int16_t)(int)fmin(fmax(r, -lim), lim);
}

}  // namespace l2t
