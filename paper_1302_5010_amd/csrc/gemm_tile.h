// Shared MFMA main loop for the contractions C[r][c] = sum_k X[r][k] W[c][k]
// with both operands K-contiguous (rows of X and of W are k-vectors).
//
// Tiling (gfx950, wave64): a workgroup computes a BM x BN tile of C; each wave
// a WM x WN sub-tile as (WM/32) x (WN/32) blocks of 32x32 MFMA accumulators.
// K is consumed 128 bytes at a time (32 float32, 64 bfloat16 or 128 e4m3 values) through
// two LDS buffers, one barrier per stage; the next K-slice is prefetched into
// registers while the current one feeds the matrix cores.  Within each 16-byte
// chunk of k, lane half h supplies the chunk's half h (float32: k = 8b + 4h + t
// at step t of four v_mfma_f32_32x32x2f32; bfloat16: 8 consecutive k of one
// v_mfma_f32_32x32x16_bf16; e4m3: 32 consecutive bytes of k for one
// v_mfma_scale_f32_32x32x64_f8f6f4), so every LDS fragment read is one or two 16-byte ds_reads; both
// operands use the same lane-to-k assignment, so the summation order over k is immaterial to the
// contraction.
//
// The caller owns the row mapping: it passes, per staging load, the element
// offset of the row start (plus this thread's 16-byte column) in X and in W.
// Every load is unconditional, so rows past the end must point at readable
// memory (a zero row or a clamped row whose results are discarded).
//
// Accumulator layout of a 32x32 block (both instructions): lane l, register r
// holds row 8(r/4) + 4(l/32) + r%4 and column l%32 of the block, the row
// coming from X and the column from W.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bmpl {

typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

constexpr int TILE_ROW_BYTES = 128;                 // k bytes per LDS stage and row
constexpr int TILE_LDS_ROW = TILE_ROW_BYTES + 16;   // 16-byte aligned, staggers banks

template <int BM, int BN, int WM, int WN>
struct TileShape {
    static constexpr int WAVES = (BM / WM) * (BN / WN);
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int TI = WM / 32;                 // MFMA blocks per wave along X rows
    static constexpr int TJ = WN / 32;                 // along W rows
    static constexpr int LX = BM * 8 / THREADS;        // 16-byte loads per thread, X tile
    static constexpr int LW = BN * 8 / THREADS;        // W tile
    static constexpr int RSTEP = THREADS / 8;          // row step between a thread's loads
    static constexpr int WAVES_M = BM / WM;
    static_assert(LX * THREADS == BM * 8 && LW * THREADS == BN * 8, "tile/thread mismatch");
};

template <int BM, int BN>
struct TileLds {
    char x[2][BM * TILE_LDS_ROW];
    char w[2][BN * TILE_LDS_ROW];
};

// A staged slice held in registers until its LDS store.  Without this the compiler turns the load and
// the later store of the same 16 bytes into one global-to-LDS copy at the store, i.e. at the end of the
// stage, and the loads' whole latency is exposed once per stage; the empty asm needs the value in
// registers, so the load stays where it was issued, a stage ahead.
__device__ __forceinline__ void staged(float4& v)
{
    asm volatile("" : "+v"(v.x), "+v"(v.y), "+v"(v.z), "+v"(v.w));
}

// Thread-to-load mapping: 16-byte column c4 = tid % 8 of the k slice, rows r0 + RSTEP q.
__device__ __forceinline__ int tile_c4(int tid) { return tid & 7; }
__device__ __forceinline__ int tile_r0(int tid) { return tid >> 3; }

// The matrix work of one LDS stage (both operands' fragments read from the stage's buffers).
template <class E, int BM, int BN, int WM, int WN>
__device__ __forceinline__ void mfma_tile_stage(const char* cX, const char* cW, int ws, int wa, int l32, int h,
                                                floatx16 (&acc)[TileShape<BM, BN, WM, WN>::TI][TileShape<BM, BN, WM, WN>::TJ])
{
    using S = TileShape<BM, BN, WM, WN>;
    if constexpr (sizeof(E) == 1) {
        // e4m3: two v_mfma_scale_f32_32x32x64_f8f6f4 per stage (unit scales); lane half h supplies
        // the 32 bytes [64 t + 32 h, +32) of k to both operands
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            intx8 fx[S::TI], fw[S::TJ];
#pragma unroll
            for (int i = 0; i < S::TI; ++i) {
                const char* pp = &cX[(ws + 32 * i + l32) * TILE_LDS_ROW + 64 * t + 32 * h];
                const float4 lo = *reinterpret_cast<const float4*>(pp);
                const float4 hi = *reinterpret_cast<const float4*>(pp + 16);
                fx[i] = intx8{__float_as_int(lo.x), __float_as_int(lo.y), __float_as_int(lo.z), __float_as_int(lo.w),
                              __float_as_int(hi.x), __float_as_int(hi.y), __float_as_int(hi.z), __float_as_int(hi.w)};
            }
#pragma unroll
            for (int j = 0; j < S::TJ; ++j) {
                const char* pp = &cW[(wa + 32 * j + l32) * TILE_LDS_ROW + 64 * t + 32 * h];
                const float4 lo = *reinterpret_cast<const float4*>(pp);
                const float4 hi = *reinterpret_cast<const float4*>(pp + 16);
                fw[j] = intx8{__float_as_int(lo.x), __float_as_int(lo.y), __float_as_int(lo.z), __float_as_int(lo.w),
                              __float_as_int(hi.x), __float_as_int(hi.y), __float_as_int(hi.z), __float_as_int(hi.w)};
            }
#pragma unroll
            for (int i = 0; i < S::TI; ++i)
#pragma unroll
                for (int j = 0; j < S::TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fx[i], fw[j], acc[i][j], 0, 0, 0, 127,
                                                                               0, 127);
        }
    } else {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {       // 4 x 16-byte chunks per lane half per stage
            float4 fx[S::TI], fw[S::TJ];
#pragma unroll
            for (int i = 0; i < S::TI; ++i)
                fx[i] = *reinterpret_cast<const float4*>(&cX[(ws + 32 * i + l32) * TILE_LDS_ROW + kb * 32 + 16 * h]);
#pragma unroll
            for (int j = 0; j < S::TJ; ++j)
                fw[j] = *reinterpret_cast<const float4*>(&cW[(wa + 32 * j + l32) * TILE_LDS_ROW + kb * 32 + 16 * h]);
            if constexpr (sizeof(E) == 2) {
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, fx[i]), __builtin_bit_cast(bf16x8, fw[j]), acc[i][j], 0, 0, 0);
            } else {
                // k step outermost so consecutive MFMAs write different accumulators
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fx[i].x, fw[j].x, acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fx[i].y, fw[j].y, acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fx[i].z, fw[j].z, acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fx[i].w, fw[j].w, acc[i][j], 0, 0, 0);
            }
        }
    }
}

// Run the K loop of one tile.  ws / wa: the wave's row offsets within the tile (X / W rows).
// DEPTH = 1: the next slice is loaded into registers at the top of a stage and stored to LDS at its end.
// DEPTH = 2: two register sets alternate, so a slice's loads are issued two stages before the stage
// that reads it (twice the latency a stage of matrix work hides; short 16- and 8-bit stages need it).
template <class E, int BM, int BN, int WM, int WN, int DEPTH = 1>
__device__ __forceinline__ void mfma_tile_loop(const E* __restrict__ X, const int64_t (&oX)[TileShape<BM, BN, WM, WN>::LX],
                                               const E* __restrict__ W, const int64_t (&oW)[TileShape<BM, BN, WM, WN>::LW],
                                               int kpad, TileLds<BM, BN>& lds, int ws, int wa,
                                               floatx16 (&acc)[TileShape<BM, BN, WM, WN>::TI][TileShape<BM, BN, WM, WN>::TJ])
{
    using S = TileShape<BM, BN, WM, WN>;
    static_assert(DEPTH == 1 || DEPTH == 2, "register prefetch depth");
    constexpr int BK = TILE_ROW_BYTES / (int)sizeof(E);   // k per stage
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int c4 = tile_c4(tid);
    const int r0 = tile_r0(tid);
    const int l32 = lane & 31;
    const int h = lane >> 5;

#pragma unroll
    for (int i = 0; i < S::TI; ++i)
#pragma unroll
        for (int j = 0; j < S::TJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    float4 gX[DEPTH][S::LX], gW[DEPTH][S::LW];
    // slices past the last re-read the last one (never used)
    const int klast = kpad - BK;
#define TILE_LOAD_SLICE(d, k0)                                                                              \
    do {                                                                                                    \
        const int kk_ = (k0) < klast ? (k0) : klast;                                                        \
        _Pragma("unroll") for (int q = 0; q < S::LX; ++q)                                                  \
            gX[d][q] = *reinterpret_cast<const float4*>(X + oX[q] + kk_);                                   \
        _Pragma("unroll") for (int q = 0; q < S::LW; ++q)                                                  \
            gW[d][q] = *reinterpret_cast<const float4*>(W + oW[q] + kk_);                                   \
    } while (0)
#define TILE_STORE_SLICE(d, buf)                                                                            \
    do {                                                                                                    \
        _Pragma("unroll") for (int q = 0; q < S::LX; ++q) {                                                \
            staged(gX[d][q]);                                                                               \
            *reinterpret_cast<float4*>(&lds.x[buf][(r0 + S::RSTEP * q) * TILE_LDS_ROW + 16 * c4]) = gX[d][q]; \
        }                                                                                                   \
        _Pragma("unroll") for (int q = 0; q < S::LW; ++q) {                                                \
            staged(gW[d][q]);                                                                               \
            *reinterpret_cast<float4*>(&lds.w[buf][(r0 + S::RSTEP * q) * TILE_LDS_ROW + 16 * c4]) = gW[d][q]; \
        }                                                                                                   \
    } while (0)

    TILE_LOAD_SLICE(0, 0);
    TILE_STORE_SLICE(0, 0);
    if constexpr (DEPTH == 2) TILE_LOAD_SLICE(1, BK);   // slice 1, held through stage 0
    __syncthreads();
    int cur = 0;
    if constexpr (DEPTH == 1) {
        for (int k0 = 0; k0 < kpad; k0 += BK) {
            TILE_LOAD_SLICE(0, k0 + BK);
            asm volatile("" ::: "memory");       // issue the prefetch before the matrix work
            mfma_tile_stage<E, BM, BN, WM, WN>(lds.x[cur], lds.w[cur], ws, wa, l32, h, acc);
            asm volatile("" ::: "memory");       // and consume it only after
            TILE_STORE_SLICE(0, cur ^ 1);
            __syncthreads();
            cur ^= 1;
        }
    } else {
        // stage s holds slice s + 1 in one register set and loads slice s + 2 into the other
        for (int k0 = 0; k0 < kpad; k0 += 2 * BK) {
            TILE_LOAD_SLICE(0, k0 + 2 * BK);
            asm volatile("" ::: "memory");
            mfma_tile_stage<E, BM, BN, WM, WN>(lds.x[cur], lds.w[cur], ws, wa, l32, h, acc);
            asm volatile("" ::: "memory");
            TILE_STORE_SLICE(1, cur ^ 1);
            __syncthreads();
            cur ^= 1;
            if (k0 + BK >= kpad) break;           // an odd number of stages
            TILE_LOAD_SLICE(1, k0 + 3 * BK);
            asm volatile("" ::: "memory");
            mfma_tile_stage<E, BM, BN, WM, WN>(lds.x[cur], lds.w[cur], ws, wa, l32, h, acc);
            asm volatile("" ::: "memory");
            TILE_STORE_SLICE(0, cur ^ 1);
            __syncthreads();
            cur ^= 1;
        }
    }
#undef TILE_LOAD_SLICE
#undef TILE_STORE_SLICE
}

// ---------------------------------------------------------------------------------------------------
// The same contraction with the operand tiles copied from global memory straight into LDS
// (global_load_lds_dwordx4: each lane's 16 bytes land at the wave's LDS base + 16 lane), so the slices
// take no registers and no LDS store instructions, and a stage waits for its copies only at its end.
//
// LDS rows are 128 bytes with no padding.  Chunk c (16 bytes of k) of tile row r sits at slot
// c ^ dma_swz(r), dma_swz(r) = (r & 7) ^ ((r >> 3) & 1): the 32 rows of one chunk that a fragment read
// touches then fall on distinct banks within every 8 consecutive lanes (128 bytes) and every 16 (256
// bytes).  One copy instruction fills 8 consecutive rows (1 KB): lane l writes slot l & 7 of row
// 8 g + (l >> 3), so it loads chunk (l & 7) ^ (l >> 3) ^ (g & 1) of that row.  Two LDS buffers: the copy
// of slice s + 1 is issued at the top of stage s into the buffer stage s - 1 read, and every wave waits
// for its own copies and then the barrier before stage s + 1 reads them.
// ---------------------------------------------------------------------------------------------------
__device__ __forceinline__ int dma_swz(int r) { return (r & 7) ^ ((r >> 3) & 1); }

template <int BM, int BN>
struct DmaLds {
    char x[2][BM * TILE_ROW_BYTES];
    char w[2][BN * TILE_ROW_BYTES];
};

template <int BM, int BN, int WM, int WN>
struct DmaShape {
    using S = TileShape<BM, BN, WM, WN>;
    static constexpr int GX = BM / 8 / S::WAVES;   // 1 KB copies per wave and stage, X tile
    static constexpr int GW = BN / 8 / S::WAVES;   // W tile
    static_assert(GX * 8 * S::WAVES == BM && GW * 8 * S::WAVES == BN, "copy groups per wave");
};

// Tile row and chunk of this lane in copy group g (8 rows).
__device__ __forceinline__ int dma_row(int g, int lane) { return 8 * g + (lane >> 3); }
__device__ __forceinline__ int dma_chunk(int g, int lane) { return (lane & 7) ^ (lane >> 3) ^ (g & 1); }

// The matrix work of one stage from swizzled buffers (same fragments, same order as mfma_tile_stage).
template <class E, int BM, int BN, int WM, int WN>
__device__ __forceinline__ void mfma_tile_stage_swz(const char* cX, const char* cW, int ws, int wa, int l32, int h,
                                                    floatx16 (&acc)[TileShape<BM, BN, WM, WN>::TI][TileShape<BM, BN, WM, WN>::TJ])
{
    using S = TileShape<BM, BN, WM, WN>;
    const int sw = dma_swz(l32);                    // ws + 32 i and wa + 32 j are multiples of 16
    auto at = [&](const char* base, int row, int chunk) {
        return *reinterpret_cast<const float4*>(base + row * TILE_ROW_BYTES + ((chunk ^ sw) << 4));
    };
    if constexpr (sizeof(E) == 1) {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            intx8 fx[S::TI], fw[S::TJ];
#pragma unroll
            for (int i = 0; i < S::TI; ++i) {
                const float4 lo = at(cX, ws + 32 * i + l32, 4 * t + 2 * h), hi = at(cX, ws + 32 * i + l32, 4 * t + 2 * h + 1);
                fx[i] = intx8{__float_as_int(lo.x), __float_as_int(lo.y), __float_as_int(lo.z), __float_as_int(lo.w),
                              __float_as_int(hi.x), __float_as_int(hi.y), __float_as_int(hi.z), __float_as_int(hi.w)};
            }
#pragma unroll
            for (int j = 0; j < S::TJ; ++j) {
                const float4 lo = at(cW, wa + 32 * j + l32, 4 * t + 2 * h), hi = at(cW, wa + 32 * j + l32, 4 * t + 2 * h + 1);
                fw[j] = intx8{__float_as_int(lo.x), __float_as_int(lo.y), __float_as_int(lo.z), __float_as_int(lo.w),
                              __float_as_int(hi.x), __float_as_int(hi.y), __float_as_int(hi.z), __float_as_int(hi.w)};
            }
#pragma unroll
            for (int i = 0; i < S::TI; ++i)
#pragma unroll
                for (int j = 0; j < S::TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fx[i], fw[j], acc[i][j], 0, 0, 0, 127,
                                                                               0, 127);
        }
    } else {
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) {
            float4 fx[S::TI], fw[S::TJ];
#pragma unroll
            for (int i = 0; i < S::TI; ++i) fx[i] = at(cX, ws + 32 * i + l32, 2 * kb + h);
#pragma unroll
            for (int j = 0; j < S::TJ; ++j) fw[j] = at(cW, wa + 32 * j + l32, 2 * kb + h);
            if constexpr (sizeof(E) == 2) {
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, fx[i]), __builtin_bit_cast(bf16x8, fw[j]), acc[i][j], 0, 0, 0);
            } else {
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fx[i].x, fw[j].x, acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fx[i].y, fw[j].y, acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fx[i].z, fw[j].z, acc[i][j], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < S::TI; ++i)
#pragma unroll
                    for (int j = 0; j < S::TJ; ++j)
                        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(fx[i].w, fw[j].w, acc[i][j], 0, 0, 0);
            }
        }
    }
}

typedef __attribute__((address_space(1))) const void global_cvoid;
typedef __attribute__((address_space(3))) void lds_void;

// Wait for this wave's outstanding vector-memory operations (its LDS copies) only.
__device__ __forceinline__ void wait_vm0() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// K loop with direct-to-LDS copies.  oX / oW: per copy group of this wave, the element offset of this
// lane's row and chunk (dma_row, dma_chunk) in X / W; rows past the end must be readable (zero rows).
template <class E, int BM, int BN, int WM, int WN>
__device__ __forceinline__ void mfma_tile_loop_dma(const E* __restrict__ X, const int64_t (&oX)[DmaShape<BM, BN, WM, WN>::GX],
                                                   const E* __restrict__ W, const int64_t (&oW)[DmaShape<BM, BN, WM, WN>::GW],
                                                   int kpad, DmaLds<BM, BN>& lds, int ws, int wa,
                                                   floatx16 (&acc)[TileShape<BM, BN, WM, WN>::TI][TileShape<BM, BN, WM, WN>::TJ])
{
    using S = TileShape<BM, BN, WM, WN>;
    using D = DmaShape<BM, BN, WM, WN>;
    constexpr int BK = TILE_ROW_BYTES / (int)sizeof(E);
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    const int l32 = lane & 31;
    const int h = lane >> 5;
    const int nst = kpad / BK;
#pragma unroll
    for (int i = 0; i < S::TI; ++i)
#pragma unroll
        for (int j = 0; j < S::TJ; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    auto issue = [&](int st, int buf) {
        const int k0 = st * BK;
#pragma unroll
        for (int i = 0; i < D::GX; ++i)
            __builtin_amdgcn_global_load_lds((global_cvoid*)(X + oX[i] + k0),
                                             (lds_void*)(lds.x[buf] + (wave + S::WAVES * i) * 1024), 16, 0, 0);
#pragma unroll
        for (int i = 0; i < D::GW; ++i)
            __builtin_amdgcn_global_load_lds((global_cvoid*)(W + oW[i] + k0),
                                             (lds_void*)(lds.w[buf] + (wave + S::WAVES * i) * 1024), 16, 0, 0);
    };
    issue(0, 0);
    wait_vm0();
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        const int cur = st & 1;
        if (st + 1 < nst) issue(st + 1, cur ^ 1);
        mfma_tile_stage_swz<E, BM, BN, WM, WN>(lds.x[cur], lds.w[cur], ws, wa, l32, h, acc);
        wait_vm0();
        __syncthreads();
    }
}

// XCD-aware tile order: workgroups are dealt round-robin to the 8 XCDs, so give each XCD a
// contiguous run of tile indices (neighbouring tiles share operand rows in that XCD's L2).
__device__ __forceinline__ int xcd_tile_index(int wid, int nwg)
{
    const int per = nwg / 8, rem = nwg % 8, xcd = wid % 8, loc = wid / 8;
    return (xcd < rem) ? xcd * (per + 1) + loc : rem * (per + 1) + (xcd - rem) * per + loc;
}

// Grouped tile order: consecutive tile indices walk GM tiles along the first dimension (signals / rows
// of X), then the next tile along the second (atoms / rows of W).  The workgroups an XCD runs at the
// same time then cover a GM x (concurrent / GM) block of tiles, so both operands' tiles are shared in
// that XCD's L2, instead of every workgroup streaming its own X tile when the X operand is large.
template <int GM>
__device__ __forceinline__ void grouped_tile(int tile, int tiles_m, int tiles_n, int& tm, int& tn)
{
    const int group = tile / (GM * tiles_n);
    const int first = group * GM;
    const int gm = tiles_m - first < GM ? tiles_m - first : GM;
    const int in = tile - group * GM * tiles_n;
    tm = first + in % gm;
    tn = in / gm;
}

}  // namespace bmpl
