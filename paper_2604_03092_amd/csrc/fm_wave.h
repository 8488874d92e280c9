// fm_wave.h -- wave64 cross-lane helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fm {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// Row rotate (16-lane rows) by N through DPP: lane j of a row receives lane
// (j - N) mod 16 of the same row.  All lanes must be active.
template <int N> __device__ __forceinline__ float row_ror(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x120 + N, 0xF, 0xF, false));
}

// Sum of x over the 16 lanes of each row, broadcast to every lane of the row.
__device__ __forceinline__ float row_sum(float x) {
    x += row_ror<8>(x);
    x += row_ror<4>(x);
    x += row_ror<2>(x);
    x += row_ror<1>(x);
    return x;
}

// Transposing reduction of 16 values over the wave.  Every lane holds
// v[0..15]; on return, the lane with (lane & 15) < 4 holds the wave sum of
// component 4 * (lane >> 4) + (lane & 15); other lanes hold junk.
// Steps: v_permlane32_swap pairs component c with c+8 across wave halves,
// v_permlane16_swap pairs c with c+4 across rows, then a DPP row sum of the
// remaining four components.  Must run with all 64 lanes active.
__device__ __forceinline__ float wave_reduce16(float v[16]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 8]),
                                                  false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v[i]), __float_as_uint(v[i + 4]),
                                                  false, false);
        v[i] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    const float r0 = row_sum(v[0]), r1 = row_sum(v[1]), r2 = row_sum(v[2]), r3 = row_sum(v[3]);
    const int j = lane_id();
    const float lo = (j & 1) ? r1 : r0;
    const float hi = (j & 1) ? r3 : r2;
    return (j & 2) ? hi : lo;
}

// Component index held by this lane after wave_reduce16 (or -1).
__device__ __forceinline__ int wave_reduce16_component() {
    const int l = lane_id();
    return ((l & 15) < 4) ? (4 * (l >> 4) + (l & 15)) : -1;
}

// Plain wave sum broadcast to all lanes (all lanes active).
__device__ __forceinline__ float wave_sum(float x) {
    x = row_sum(x);
    auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    x = __uint_as_float(r[0]) + __uint_as_float(r[1]);   // rows {0,1} and {2,3}
    auto s = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(s[0]) + __uint_as_float(s[1]);
}

}  // namespace fm
