// fm_wave.h -- wave64 cross-lane helpers for gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fm {

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __builtin_amdgcn_ballot_w64(p); }

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

// DPP move within 16-lane rows (all lanes active).  CTRL: 0x120 + N rotates
// right by N, 0x141 mirrors each 8-lane half (lane j <- lane j ^ 7),
// 0xB1 / 0x4E swap lanes j ^ 1 / j ^ 2 inside each quad.
template <int CTRL> __device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// In-place half swaps: lanes 32..63 of a with lanes 0..31 of b (swap32),
// and the odd 16-lane rows of a with the even rows of b (swap16).  Written as
// inline asm with both operands read-write: through the builtins the
// compiler copied the second operand before every swap in the adjoint's
// loop (12 moves per reduction).  The leading s_nop 1 gives the two wait
// states a permlane swap needs after a VALU write of its operands; the
// results may be read right away.
__device__ __forceinline__ void swap32(float &a, float &b) {
    asm volatile("s_nop 1\n\tv_permlane32_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}
__device__ __forceinline__ void swap16(float &a, float &b) {
    asm volatile("s_nop 1\n\tv_permlane16_swap_b32 %0, %1" : "+v"(a), "+v"(b));
}

// Transposing reduction of 16 values over the wave.  Every lane holds
// v[0..15]; on return, every lane holds the wave sum of component
// 4 * (lane >> 4) + ((lane >> 2) & 3) (the four lanes of a quad agree).
// Each step halves the values a lane carries and doubles the lanes a value
// spans: v_permlane32_swap pairs component c with c+8 across wave halves,
// v_permlane16_swap pairs c with c+4 across rows, then inside each row a
// rotation by 8 pairs c with c+2, a half mirror pairs c with c+1, and two
// quad swaps finish the sums.  v is overwritten.  Must run with all 64
// lanes active.
__device__ __forceinline__ float wave_reduce16(float v[16]) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        swap32(v[i], v[i + 8]);
        v[i] = v[i] + v[i + 8];
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        swap16(v[i], v[i + 4]);
        v[i] = v[i] + v[i + 4];
    }
    // row r now holds components 4r + 0..3 in v[0..3], each partial over its 16 lanes
    const int j = lane_id();
    const bool b3 = (j & 8) != 0, b2 = (j & 4) != 0;
    const float t0 = b3 ? v[2] : v[0], u0 = b3 ? v[0] : v[2];
    const float t1 = b3 ? v[3] : v[1], u1 = b3 ? v[1] : v[3];
    const float a0 = t0 + dpp<0x128>(u0);  // component 2 b3,     over lanes j, j ^ 8
    const float a1 = t1 + dpp<0x128>(u1);  // component 2 b3 + 1
    const float keep = b2 ? a1 : a0, give = b2 ? a0 : a1;
    float x = keep + dpp<0x141>(give);     // component 2 b3 + b2, over 4 lanes
    x += dpp<0xB1>(x);
    x += dpp<0x4E>(x);
    return x;
}

// Component index held by this lane after wave_reduce16, for one lane per
// quad (the others get -1).
__device__ __forceinline__ int wave_reduce16_component() {
    const int l = lane_id();
    return ((l & 3) == 0) ? (4 * (l >> 4) + ((l >> 2) & 3)) : -1;
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
