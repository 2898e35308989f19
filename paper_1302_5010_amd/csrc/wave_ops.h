// Wave-wide reductions without the LDS crossbar.  A 64-lane wave is combined in
// five steps: DPP moves inside each row of 16 lanes (lane ^ 1 and lane ^ 2 as quad
// permutes, then the row's half mirror and mirror, which pair the two quads of each
// 8 and the two 8s of each 16), one ds_swizzle across the two rows of each 32-lane
// half (lane ^ 16), and readlane of lanes 0 and 32.  Every partner pairing is an
// involution, so both lanes of a pair combine the same two values and every lane ends
// with the same result.  All 64 lanes must be active (the readlane sources included).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmpl {

// GFX9 DPP controls: quad_perm(1,0,3,2), quad_perm(2,3,0,1), row_half_mirror, row_mirror.
constexpr int DPP_XOR1 = 0xB1;
constexpr int DPP_XOR2 = 0x4E;
constexpr int DPP_HALF_MIRROR = 0x141;
constexpr int DPP_MIRROR = 0x140;
// ds_swizzle bit mode over 32 lanes: source = ((lane & 0x1F) | 0) ^ 0x10.
constexpr int SWZ_XOR16 = 0x401F;

template <int CTRL>
__device__ inline int dpp_move(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}

// The value of the partner lane under DPP control CTRL (or the xor-16 swizzle when CTRL < 0).
template <int CTRL>
__device__ inline int lane_move(int v)
{
    if constexpr (CTRL < 0)
        return __builtin_amdgcn_ds_swizzle(v, SWZ_XOR16);
    else
        return dpp_move<CTRL>(v);
}

template <int CTRL>
__device__ inline float lane_move(float v)
{
    return __int_as_float(lane_move<CTRL>(__float_as_int(v)));
}

template <int CTRL>
__device__ inline double lane_move(double v)
{
    const int64_t b = __double_as_longlong(v);
    const int lo = lane_move<CTRL>((int)(uint32_t)b), hi = lane_move<CTRL>((int)(b >> 32));
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

__device__ inline float read_lane(float v, int lane)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

__device__ inline double read_lane(double v, int lane)
{
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)b, lane), hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double((int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo));
}

// Combine steps inside each 32-lane half; OP(a, b) must be commutative.
template <typename T, typename OP>
__device__ inline T half_reduce(T v, OP op)
{
    v = op(v, lane_move<DPP_XOR1>(v));
    v = op(v, lane_move<DPP_XOR2>(v));
    v = op(v, lane_move<DPP_HALF_MIRROR>(v));
    v = op(v, lane_move<DPP_MIRROR>(v));
    v = op(v, lane_move<-1>(v));
    return v;
}

__device__ inline double wave_sum(double v)
{
    v = half_reduce(v, [](double a, double b) { return a + b; });
    return read_lane(v, 0) + read_lane(v, 32);
}

__device__ inline int wave_sum(int v)
{
    v = half_reduce(v, [](int a, int b) { return a + b; });
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 32);
}

__device__ inline double wave_max(double v)
{
    v = half_reduce(v, [](double a, double b) { return fmax(a, b); });
    return fmax(read_lane(v, 0), read_lane(v, 32));
}

__device__ inline float wave_max(float v)
{
    v = half_reduce(v, [](float a, float b) { return fmaxf(a, b); });
    return fmaxf(read_lane(v, 0), read_lane(v, 32));
}

// Eight sums over the wave at once: a[e] summed over all 64 lanes for e = 0..7.  Each exchange halves
// the values a lane carries (lane ^ 1 and lane ^ 2 by DPP, lane ^ 4 by a permute), then the lanes that
// carry the same index are summed (lane ^ 8, ^ 16, ^ 32): 10 exchanges instead of 8 full reductions.
// Lane l returns the sum for e = 4 (l & 1) + 2 ((l >> 1) & 1) + ((l >> 2) & 1) (wave_sum8_index).
__device__ inline int wave_sum8_index(int lane) { return 4 * (lane & 1) + 2 * ((lane >> 1) & 1) + ((lane >> 2) & 1); }

__device__ inline double wave_sum8(const double (&a)[8])
{
    const int lane = threadIdx.x & 63;
    const bool b0 = lane & 1, b1 = (lane >> 1) & 1, b2 = (lane >> 2) & 1;
    double s4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double recv = lane_move<DPP_XOR1>(b0 ? a[i] : a[i + 4]);
        s4[i] = (b0 ? a[i + 4] : a[i]) + recv;
    }
    double s2[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double recv = lane_move<DPP_XOR2>(b1 ? s4[i] : s4[i + 2]);
        s2[i] = (b1 ? s4[i + 2] : s4[i]) + recv;
    }
    double s1 = (b2 ? s2[1] : s2[0]) + __shfl_xor(b2 ? s2[0] : s2[1], 4);
    s1 += __shfl_xor(s1, 8);
    s1 += lane_move<-1>(s1);
    s1 += __shfl_xor(s1, 32);
    return s1;
}

// Sum over groups of P consecutive lanes (P = 1, 2 or 4; the group's lanes active together).
__device__ inline double group_sum(double v, int P)
{
    if (P >= 2) v += lane_move<DPP_XOR1>(v);
    if (P >= 4) v += lane_move<DPP_XOR2>(v);
    return v;
}

// Sum over each row of 16 lanes (every lane of the row gets it; the row's lanes active together).
__device__ inline double row16_sum(double v)
{
    v += lane_move<DPP_XOR1>(v);
    v += lane_move<DPP_XOR2>(v);
    v += lane_move<DPP_HALF_MIRROR>(v);
    v += lane_move<DPP_MIRROR>(v);
    return v;
}

}  // namespace bmpl
