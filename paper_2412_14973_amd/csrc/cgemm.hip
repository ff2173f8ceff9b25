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
#include "gemm_common.hpp"

namespace tlr {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = GEMM_BM, BN = GEMM_BN, BK = GEMM_BK;
constexpr int A_PITCH = BM + 1;             // floats per real-k row (k-major A tile)
constexpr int A_STAGE = 2 * BK * A_PITCH;   // floats per A stage
constexpr int B_PITCH = 2 * BN;             // floats per k row of the B tile
constexpr int B_STAGE = BK * B_PITCH;

template <int MODE>
__global__ __launch_bounds__(256, 2) void cgemm_f32_kernel(GemmArgs g) {
    __shared__ float As[2][A_STAGE];
    __shared__ float Bs[2][B_STAGE];

    const int z = blockIdx.y;
    const float2 *A = g.A + z * g.sA;
    const float2 *B = g.B + z * g.sB;

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
    const int K = g.K;

    // ---- global -> register loaders ----
    float4 ra[4], rb[4];
    const int a_row = t >> 3, a_fq = t & 7;     // A: 8 lanes per row, 4 floats each
    const int b_row = t >> 6, b_cq = t & 63;    // B: 64 lanes per k row, 2 complex each

    // The host pads every operand to whole tiles (M, N multiples of 128, K of 16)
    // with zeros, so the loads carry no bounds checks. They are buffer loads: a
    // uniform resource (base, byte size) plus a per-lane 32-bit offset that stays
    // fixed across stages (the stage advance is the uniform soffset), so all eight
    // 16-byte loads of a stage are in flight together while the previous stage
    // runs on the matrix cores, and any access outside an operand reads zero.
    const __amdgpu_buffer_rsrc_t rsA =
        __builtin_amdgcn_make_buffer_rsrc((void *)A, (short)0, (int)g.bytesA, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsB =
        __builtin_amdgcn_make_buffer_rsrc((void *)B, (short)0, (int)g.bytesB, 0x00020000);
    uint32_t offA[4], offB[4];
#pragma unroll
    for (int p = 0; p < 4; ++p)
        offA[p] = (uint32_t)(((int64_t)(m0 + a_row + 32 * p) * g.lda + 2 * a_fq) * 8);
    {
        const int c = 2 * b_cq;  // complex column inside the LDS tile
        int64_t base = n0 + c;
        if (MODE == GM_LINE) {
            const int grp2 = c >> 5;
            base = n0 + (grp2 >> 1) * 32 + (c & 31) + ((grp2 & 1) ? g.b2_off : 0);
        }
#pragma unroll
        for (int p = 0; p < 4; ++p) offB[p] = (uint32_t)((base + (int64_t)(b_row + 4 * p) * g.ldb) * 8);
    }
    auto ld16 = [](__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
        return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
    };
    auto load_a = [&](int k0) {
        const uint32_t so = (uint32_t)k0 * 8u;
#pragma unroll
        for (int p = 0; p < 4; ++p) ra[p] = ld16(rsA, offA[p], so);
    };
    auto load_b = [&](int k0) {
        const uint32_t so = (uint32_t)((int64_t)k0 * g.ldb * 8);
#pragma unroll
        for (int p = 0; p < 4; ++p) rb[p] = ld16(rsB, offB[p], so);
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
        const float *as = As[buf] + half * A_PITCH + wm * 64 + j32;
        const float *bs = Bs[buf] + 2 * (wn * 64) + bswz;
        // operand fragments double-buffered in registers: the reads of step kc+1
        // are issued before the eight MFMAs of step kc
        float a_cur[2], b_cur[4], a_nxt[2], b_nxt[4];
        auto frag = [&](int kc, float *af, float *bf) {
            af[0] = as[2 * kc * A_PITCH];
            af[1] = as[2 * kc * A_PITCH + 32];
#pragma unroll
            for (int bn = 0; bn < 4; ++bn)
                bf[bn] = __uint_as_float(__float_as_uint(bs[kc * B_PITCH + 32 * bn]) ^ bsign);
        };
        frag(0, a_cur, b_cur);
#pragma unroll
        for (int kc = 0; kc < BK; ++kc) {
            if (kc + 1 < BK) frag(kc + 1, a_nxt, b_nxt);
#pragma unroll
            for (int bn = 0; bn < 4; ++bn) {
                acc[0][bn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_cur[0], b_cur[bn], acc[0][bn], 0, 0, 0);
                acc[1][bn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a_cur[1], b_cur[bn], acc[1][bn], 0, 0, 0);
            }
            if (kc + 1 < BK) {
                a_cur[0] = a_nxt[0];
                a_cur[1] = a_nxt[1];
#pragma unroll
                for (int bn = 0; bn < 4; ++bn) b_cur[bn] = b_nxt[bn];
            }
        }
        if (kt + 1 < nk) store_lds(buf ^ 1);
        __syncthreads();
    }

    EpiArgs ea;
    ea.C = g.C + z * g.sC;
    ea.C2 = (MODE == GM_LINE) ? g.C2 + z * g.sC : nullptr;
    ea.ldc = g.ldc;
    ea.E = (MODE == GM_STORE) ? nullptr : g.E + z * g.sE;
    ea.lde = g.lde;
    ea.Me = g.Me;
    ea.Ne = g.Ne;
    ea.partials = g.partials ? g.partials + z * g.sP : nullptr;
    gemm_epilogue<MODE>(acc, ea, m0, n0, pid);
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
    if (a.M % BM || a.N % BN || a.K % BK || a.K <= 0) return hipErrorInvalidValue;   // padded operands only
    // byte extents of the buffer resources (32-bit): A is M x lda, B is K x ldb (GM_LINE: B2 follows B)
    const int64_t bytesA = (int64_t)a.M * a.lda * 8;
    int64_t bytesB = (int64_t)a.K * a.ldb * 8;
    a.b2_off = 0;
    if (mode == GM_LINE) {
        a.b2_off = a.B2 - a.B;
        if (a.b2_off < 0) return hipErrorInvalidValue;
        bytesB += a.b2_off * 8;
    }
    if (bytesA >= (int64_t)1 << 32 || bytesB >= (int64_t)1 << 32) return hipErrorInvalidValue;
    a.bytesA = (uint32_t)bytesA;
    a.bytesB = (uint32_t)bytesB;
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
