// Complex64 GEMM on CDNA4 FP32 matrix cores.
//
// The dense products of the method (ADMM solver section: r = D X - U in the
// objective of eq. X2LQR_lst, W = D^H r in the gradient equations DXLR, and
// the line-search products D X1, D X2) are complex. A complex product
// C = A B is evaluated as ONE real GEMM of size M x 2N x 2K: A (interleaved
// re/im, row-major) is read as a real M x 2K matrix, and every complex b of B
// becomes the real 2x2 block [[Re b, Im b], [-Im b, Re b]], so the real
// output rows come out interleaved (re, im) - the complex64 layout - with
// exactly the 8MNK flops of the four-real-product form and no separate
// subtraction pass.
//
// Tiling: 256 threads = 4 waves (2 x 2); workgroup tile 128 rows x 128
// complex columns, 16 complex k per stage, double-buffered LDS (A stored
// k-major with an odd pitch so the MFMA operand reads are conflict free).
// Each wave owns 2 x 4 v_mfma_f32_32x32x2_f32 blocks (64 rows x 64 complex
// columns). One MFMA consumes one complex k: its A operand is (Re, Im) of
// A[m][k] and its B operand one realified row pair of B.
//
// Epilogues: GM_STORE (C = AB), GM_RESID (C = AB - U plus FP64 partial sums
// of |C|^2) and GM_LINE (a = D X1, b = D X2 for the same columns in one
// workgroup, plus FP64 partial sums of Re<r,a>, |a|^2, Re<r,b>, Re<a,b>,
// |b|^2 for the exact line search).
#include "common.hpp"

namespace tlr {

typedef float floatx16 __attribute__((ext_vector_type(16)));

namespace {

constexpr int BM = GEMM_BM, BN = GEMM_BN, BK = GEMM_BK;
constexpr int A_PITCH = BM + 1;             // floats per real-k row (k-major A tile)
constexpr int A_STAGE = 2 * BK * A_PITCH;   // floats per A stage
constexpr int B_PITCH = 2 * BN;             // floats per k row of the B tile
constexpr int B_STAGE = BK * B_PITCH;
constexpr int NSUM_MAX = 5;

// Output layout of the 32x32 MFMA accumulator: lane l holds column l % 32,
// register r holds row (r % 4) + 8 (r / 4) + 4 (l / 32).
__device__ __forceinline__ int acc_row(int r, int lane) {
    return (r & 3) + 8 * (r >> 2) + 4 * (lane >> 5);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <int MODE>
__global__ __launch_bounds__(256, 2) void cgemm_f32_kernel(GemmArgs g) {
    __shared__ float As[2][A_STAGE];
    __shared__ float Bs[2][B_STAGE];
    __shared__ double red[4][NSUM_MAX];

    const int z = blockIdx.y;
    const float2 *A = g.A + z * g.sA;
    const float2 *B = g.B + z * g.sB;
    const float2 *B2 = (MODE == GM_LINE) ? g.B2 + z * g.sB : nullptr;

    // workgroup -> tile: contiguous tile ranges per XCD, grouped by 8 tile rows
    const int nb = gridDim.x;
    int pid = blockIdx.x;
    if ((nb & 7) == 0) pid = (pid & 7) * (nb >> 3) + (pid >> 3);
    const int group_rows = 8;
    const int per_group = group_rows * g.tiles_n;
    const int grp = pid / per_group;
    const int first_m = grp * group_rows;
    const int gsz = min(g.tiles_m - first_m, group_rows);
    const int tm = first_m + (pid % per_group) % gsz;
    const int tn = (pid % per_group) / gsz;

    const int m0 = tm * BM;
    const int n0 = (MODE == GM_LINE) ? tn * (BN / 2) : tn * BN;

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int M = g.M, N = g.N, K = g.K;

    // ---- global -> register loaders ----
    float4 ra[4], rb[4];
    const int a_row = t >> 3, a_fq = t & 7;     // A: 8 lanes per row, 4 floats each
    const int b_row = t >> 6, b_cq = t & 63;    // B: 64 lanes per k row, 2 complex each

    auto load_a = [&](int k0) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int row = m0 + a_row + 32 * p;
            const int kc = k0 + 2 * a_fq;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (row < M && kc < K) {
                v = *reinterpret_cast<const float4 *>(A + (int64_t)row * g.lda + kc);
                if (kc + 1 >= K) { v.z = 0.f; v.w = 0.f; }
            }
            ra[p] = v;
        }
    };
    auto load_b = [&](int k0) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int kr = k0 + b_row + 4 * p;
            const int c = 2 * b_cq;  // complex column inside the LDS tile
            const float2 *src = B;
            int col;
            if (MODE == GM_LINE) {
                const int grp2 = c >> 5;
                src = (grp2 & 1) ? B2 : B;
                col = n0 + (grp2 >> 1) * 32 + (c & 31);
            } else {
                col = n0 + c;
            }
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (kr < K && col < N) {
                v = *reinterpret_cast<const float4 *>(src + (int64_t)kr * g.ldb + col);
                if (col + 1 >= N) { v.z = 0.f; v.w = 0.f; }
            }
            rb[p] = v;
        }
    };
    auto store_lds = [&](int buf) {
        float *as = As[buf];
        float *bs = Bs[buf];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int row = a_row + 32 * p;
            as[(4 * a_fq + 0) * A_PITCH + row] = ra[p].x;
            as[(4 * a_fq + 1) * A_PITCH + row] = ra[p].y;
            as[(4 * a_fq + 2) * A_PITCH + row] = ra[p].z;
            as[(4 * a_fq + 3) * A_PITCH + row] = ra[p].w;
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            *reinterpret_cast<float4 *>(bs + (b_row + 4 * p) * B_PITCH + 4 * b_cq) = rb[p];
        }
    };

    floatx16 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int j32 = lane & 31;
    const int half = lane >> 5;
    const int bswz = j32 ^ half;                         // (re,im) swap for the second k row
    const uint32_t bsign = (half && !(j32 & 1)) ? 0x80000000u : 0u;   // -Im b

    const int nk = (K + BK - 1) / BK;
    load_a(0);
    load_b(0);
    store_lds(0);
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) {
            load_a((kt + 1) * BK);
            load_b((kt + 1) * BK);
        }
        const float *as = As[buf];
        const float *bs = Bs[buf];
#pragma unroll 4
        for (int kc = 0; kc < BK; ++kc) {
            const float *arow = as + (2 * kc + half) * A_PITCH + wm * 64 + j32;
            const float a0 = arow[0];
            const float a1 = arow[32];
            const float *brow = bs + kc * B_PITCH + 2 * (wn * 64) + bswz;
#pragma unroll
            for (int bn = 0; bn < 4; ++bn) {
                const float braw = brow[32 * bn];
                const float bv = __uint_as_float(__float_as_uint(braw) ^ bsign);
                acc[0][bn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a0, bv, acc[0][bn], 0, 0, 0);
                acc[1][bn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, bv, acc[1][bn], 0, 0, 0);
            }
        }
        if (kt + 1 < nk) store_lds(buf ^ 1);
        __syncthreads();
    }

    // ---- epilogues ----
    float *C = reinterpret_cast<float *>(g.C + z * g.sC);
    const int64_t ldc2 = 2 * g.ldc;
    if (MODE == GM_STORE) {
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
            for (int bn = 0; bn < 4; ++bn) {
                const int col = n0 + wn * 64 + bn * 16 + (j32 >> 1);
                const int64_t fcol = 2 * (int64_t)(n0 + wn * 64 + bn * 16) + j32;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm * 64 + bm * 32 + acc_row(r, lane);
                    if (row < M && col < N) C[row * ldc2 + fcol] = acc[bm][bn][r];
                }
            }
        return;
    }

    const float *E = reinterpret_cast<const float *>(g.E + z * g.sE);
    const int64_t lde2 = 2 * g.lde;
    double sums[NSUM_MAX] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (MODE == GM_RESID) {
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
            for (int bn = 0; bn < 4; ++bn) {
                const int col = n0 + wn * 64 + bn * 16 + (j32 >> 1);
                const int64_t fcol = 2 * (int64_t)(n0 + wn * 64 + bn * 16) + j32;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm * 64 + bm * 32 + acc_row(r, lane);
                    if (row < M && col < N) {
                        const float v = acc[bm][bn][r] - E[row * lde2 + fcol];
                        C[row * ldc2 + fcol] = v;
                        sums[0] += (double)v * (double)v;
                    }
                }
            }
    } else {  // GM_LINE
        float *C2 = reinterpret_cast<float *>(g.C2 + z * g.sC);
#pragma unroll
        for (int bm = 0; bm < 2; ++bm)
#pragma unroll
            for (int bn = 0; bn < 2; ++bn) {
                const int col = n0 + wn * 32 + bn * 16 + (j32 >> 1);
                const int64_t fcol = 2 * (int64_t)(n0 + wn * 32 + bn * 16) + j32;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm * 64 + bm * 32 + acc_row(r, lane);
                    if (row < M && col < N) {
                        const float av = acc[bm][bn][r];
                        const float bv = acc[bm][bn + 2][r];
                        const float rv = E[row * lde2 + fcol];
                        C[row * ldc2 + fcol] = av;
                        C2[row * ldc2 + fcol] = bv;
                        const double ad = av, bd = bv, rd = rv;
                        sums[0] += rd * ad;
                        sums[1] += ad * ad;
                        sums[2] += rd * bd;
                        sums[3] += ad * bd;
                        sums[4] += bd * bd;
                    }
                }
            }
    }
    constexpr int NS = (MODE == GM_RESID) ? 1 : 5;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double v = wave_sum(sums[s]);
        if (lane == 0) red[wave][s] = v;
    }
    __syncthreads();
    if (t < NS) {
        const double v = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
        g.partials[z * g.sP + (int64_t)pid * NS + t] = v;
    }
}

}  // namespace

int gemm_partials_per_problem(int mode, int M, int N) {
    const int tm = (M + BM - 1) / BM;
    const int tn = (mode == GM_LINE) ? (N + BN / 2 - 1) / (BN / 2) : (N + BN - 1) / BN;
    const int ns = (mode == GM_RESID) ? 1 : (mode == GM_LINE ? 5 : 0);
    return tm * tn * ns;
}

hipError_t launch_cgemm(int mode, const GemmArgs &a0, int batch, hipStream_t s) {
    GemmArgs a = a0;
    a.tiles_m = (a.M + BM - 1) / BM;
    a.tiles_n = (mode == GM_LINE) ? (a.N + BN / 2 - 1) / (BN / 2) : (a.N + BN - 1) / BN;
    if (a.M <= 0 || a.N <= 0 || batch <= 0) return hipSuccess;
    dim3 grid(a.tiles_m * a.tiles_n, batch);
    switch (mode) {
        case GM_STORE: hipLaunchKernelGGL(cgemm_f32_kernel<GM_STORE>, grid, dim3(256), 0, s, a); break;
        case GM_RESID: hipLaunchKernelGGL(cgemm_f32_kernel<GM_RESID>, grid, dim3(256), 0, s, a); break;
        case GM_LINE:  hipLaunchKernelGGL(cgemm_f32_kernel<GM_LINE>, grid, dim3(256), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tlr
