// Shared pieces of the complex GEMM kernels (FP32 and BF16 hi+lo split):
// the accumulator layout of the 32 x 32 MFMA blocks and the epilogues.
#pragma once
#include "common.hpp"

namespace tlr {

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Output layout of a 32x32 MFMA accumulator (f32 result of the 32x32x2 f32 and
// 32x32x16 bf16 instructions): lane l holds column l % 32, register r holds
// row (r % 4) + 8 (r / 4) + 4 (l / 32).
__device__ __forceinline__ int acc_row(int r, int lane) {
    return (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct EpiArgs {
    float2 *C;         // output (GM_LINE: a)
    float2 *C2;        // GM_LINE: b
    int64_t ldc;
    const float2 *E;   // GM_RESID: U (true shape Me x Ne); GM_LINE: r
    int64_t lde;
    int32_t Me, Ne;
    double *partials;  // this problem's partial sums
    int32_t Mrows;     // rows of C (a 256-row tile may overhang it by 128; WROWS = 4 only)
    int32_t slot_step; // WROWS = 4: partial slot of the second 128-row half = first + slot_step
};

// Epilogue of a workgroup tile of WROWS x 64 rows and 128 complex columns held as 2 WROWS waves
// (wave w: rows 64 (w / 2), columns 64 (w % 2)) of 2 x 4 accumulator blocks. GM_STORE: C = acc.
// GM_RESID: C = acc - E, partial sum |C|^2. GM_LINE: blocks bn = 0,1 are a and bn = 2,3 are b at the
// same columns; partial sums Re<r,a>, |a|^2, Re<r,b>, Re<a,b>, |b|^2. Partial sums of 16 products are
// formed in FP32 registers and folded into FP64; each 128-row half's four waves are reduced in a
// fixed order into one partial slot (WROWS = 2: slot pid; WROWS = 4: slots pid and pid + slot_step,
// the second only when that half lies inside C).
template <int MODE, int WROWS = 2>
__device__ __forceinline__ void gemm_epilogue(floatx16 (&acc)[2][4], const EpiArgs &ea, int m0, int n0, int pid) {
    constexpr int NWAVE = 2 * WROWS;
    __shared__ double red[NWAVE][5];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int j32 = lane & 31;
    // WROWS = 4: the waves of a 128-row half past the end of C write nothing
    if (WROWS == 4 && m0 + wm * 64 >= ea.Mrows) {
        if (MODE != GM_STORE) {
            if (lane == 0)
#pragma unroll
                for (int s = 0; s < 5; ++s) red[wave][s] = 0.0;
            __syncthreads();
        }
        return;
    }
    // ---- epilogues ----
    float *C = reinterpret_cast<float *>(ea.C);
    const int64_t ldc2 = 2 * (int64_t)ea.ldc;
    if (MODE == GM_STORE) {
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
            for (int bn = 0; bn < 4; ++bn) {
                const int64_t fcol = 2 * (int64_t)(n0 + wn * 64 + bn * 16) + j32;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm * 64 + bm * 32 + acc_row(r, lane);
                    C[row * ldc2 + fcol] = acc[bm][bn][r];
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        return;
    }

    const float *E = reinterpret_cast<const float *>(ea.E);
    const int64_t lde2 = 2 * (int64_t)ea.lde;
    double sums[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (MODE == GM_RESID) {
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
            for (int bn = 0; bn < 4; ++bn) {
                const int col = n0 + wn * 64 + bn * 16 + (j32 >> 1);
                const int64_t fcol = 2 * (int64_t)(n0 + wn * 64 + bn * 16) + j32;
                float blk = 0.f;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm * 64 + bm * 32 + acc_row(r, lane);
                    const bool in = row < ea.Me && col < ea.Ne;   // U has the true (unpadded) shape
                    const float v = acc[bm][bn][r] - (in ? E[row * lde2 + fcol] : 0.f);
                    C[row * ldc2 + fcol] = v;
                    blk = fmaf(v, v, blk);
                }
                sums[0] += (double)blk;
                // one accumulator block at a time: keeps the epilogue's loads from being
                // hoisted together (register pressure)
                __builtin_amdgcn_sched_barrier(0);
            }
    } else {  // GM_LINE
        float *C2 = reinterpret_cast<float *>(ea.C2);
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
            for (int bn = 0; bn < 2; ++bn) {
                const int64_t fcol = 2 * (int64_t)(n0 + wn * 32 + bn * 16) + j32;
                // 16 products per sum in FP32 registers, then folded into the FP64 sums
                float blk[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm * 64 + bm * 32 + acc_row(r, lane);
                    const float av = acc[bm][bn][r];
                    const float bv = acc[bm][bn + 2][r];
                    const float rv = E[row * lde2 + fcol];
                    C[row * ldc2 + fcol] = av;
                    C2[row * ldc2 + fcol] = bv;
                    blk[0] = fmaf(rv, av, blk[0]);
                    blk[1] = fmaf(av, av, blk[1]);
                    blk[2] = fmaf(rv, bv, blk[2]);
                    blk[3] = fmaf(av, bv, blk[3]);
                    blk[4] = fmaf(bv, bv, blk[4]);
                }
#pragma unroll
                for (int q = 0; q < 5; ++q) sums[q] += (double)blk[q];
                __builtin_amdgcn_sched_barrier(0);
            }
    }
    constexpr int NS = (MODE == GM_RESID) ? 1 : 5;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double v = wave_sum(sums[s]);
        if (lane == 0) red[wave][s] = v;
    }
    __syncthreads();
    if (WROWS == 2) {
        if (t < NS) {
            const double v = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
            ea.partials[(int64_t)pid * NS + t] = v;
        }
    } else if (t < 2 * NS) {
        const int h = t / NS, q = t % NS;
        if (m0 + 128 * h < ea.Mrows) {
            const double v = ((red[4 * h][q] + red[4 * h + 1][q]) + red[4 * h + 2][q]) + red[4 * h + 3][q];
            ea.partials[(int64_t)(pid + h * ea.slot_step) * NS + q] = v;
        }
    }
}

}  // namespace tlr
