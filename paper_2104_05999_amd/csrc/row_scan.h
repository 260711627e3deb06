// Sums over the 16 lanes of a row, in lane order, with DPP row operations
// (no LDS round trip): the result is the sequential sum a one-thread loop over
// the row's terms would give, bit for bit.  Every lane of the row must be
// active.
#pragma once

#include <cstdint>

// x from another lane of the row (DPP control CTRL); lanes without a source
// lane receive an unspecified value.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
    const int lo = __builtin_amdgcn_mov_dpp(static_cast<int>(b & 0xffffffffu), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp(static_cast<int>(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) |
                                                       static_cast<uint32_t>(lo)));
}

// ((c + t_0) + t_1) + ... + t_15 over the lanes k = 0..15 of the row (lane k
// = g), skipping the lanes whose take is false; c is lane 0's.  Lane k adds
// its term to lane k - 1's partial (row shift right by one), so the partials
// form in order; the total is returned in lane 0 (row mirror of lane 15).  A
// skipped lane adds -0.0, which leaves every value, zeros of either sign
// included, as it is.
__device__ __forceinline__ double row_seq_sum(double c, double t, bool take, int g) {
    const double tt = take ? t : -0.0;
    double x = c + tt;
#pragma unroll
    for (int k = 1; k < 16; ++k) {
        const double y = dpp_f64<0x111>(x);  // row_shr:1
        x = g == k ? y + tt : x;
    }
    return dpp_f64<0x140>(x);  // row_mirror
}
