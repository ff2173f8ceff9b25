// Tile kernels: assembly of X = C(Zbar, Lbar, Rbar) and the per-tile gradient
// contractions.
//
// Assembly (Tile Low-rank MDD section): X_ij = L_ij R_ij for i > j and
// X_ji = X_ij^T; X_ii = Q_ii Q_ii^T or (Z_ii + Z_ii^T)/2. The directional
// form used by the exact line search expands C(theta + a p) = C(theta) +
// a X1 + a^2 X2, tile by tile: X1 = P_L R + L P_R, X2 = P_L P_R (and the
// Q Q^T / dense analogues). Each workgroup builds one 64 x 64 block on the
// FP32 matrix cores from factors staged in LDS 16 rank entries at a time;
// every product is staged through LDS once and written from there twice
// (directly and transposed, both with whole rows per wave), so X = X^T holds
// bit for bit; Q Q^T tiles are built on and below the block diagonal only
// and mirrored.
//
// Gradient (ADMM solver section, eqs. DXLR): with W = D^H r and W' = W + W^T,
// grad L = W' R^H, grad R = L^H W', grad Q = W' conj(Q), grad Z = W'/2.
// W' is never formed: each block of W'_ij is built in LDS from a block of
// W_ij plus the transposed block of W_ji, both read coalesced.
#include "gemm_common.hpp"

namespace tlr {
namespace {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {  // a * conj(b)
    return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }

// Output: complex64 (OUTB = false) or split BF16 planes (OUTB = true, see launch_assemble).
template <bool OUTB>
__device__ __forceinline__ void put(float2 *X, int64_t o, int64_t low, float2 v) {
    if (OUTB) {
        uint32_t h, l;
        split_c(v, h, l);
        uint32_t *w = reinterpret_cast<uint32_t *>(X);
        w[o] = h;
        w[o + low] = l;
    } else {
        X[o] = v;
    }
}

constexpr int AB = ASM_B;            // block edge (rows and columns)
constexpr int AKC = ASM_KC;          // rank entries staged per step
constexpr int AAP = AB + 1;          // row-factor planes [AKC][AAP] floats (k-major: rows fastest)
constexpr int ABP = AB + 1;          // column-factor stage [AKC][ABP] complex
constexpr int ST_P = AB + 1;         // transpose stage [AB][ST_P] complex
constexpr int A_PL = AKC * AAP;      // floats per row-factor plane
constexpr int B_ST = AKC * ABP;      // complex per column-factor stage

// Each workgroup builds one 64 x 64 block of a tile on the FP32 matrix cores. A factor product
// F G (F: 64 x k rows of L, P_L or Q; G: k x 64 columns of R, P_R or Q^T) is a complex GEMM with
// K = k, evaluated in realified form: one v_mfma_f32_32x32x2_f32 per complex k takes (Re, Im) of
// F[m][k] as its two A entries and the real 2 x 2 block [[Re g, Im g], [-Im g, Re g]] of G[k][n] as
// B, so the real output columns come out as interleaved (re, im) pairs. Wave w owns complex columns
// 16 w .. 16 w + 15 of the block and both 32-row halves: X (or X1 and X2) in two (four) accumulators.
// The row factors sit in LDS as separate real and imaginary planes, k-major, so a lane's A entry
// is one conflict-free float read; the column factors stay interleaved complex. 33 KB of LDS and
// at most 128 VGPRs (launch bound: 4 waves per SIMD) keep four workgroups on a CU, so the write
// phases of some overlap the loads and products of others.
template <bool DIR, bool OUTB>
__global__ __launch_bounds__(256, 4) void assemble_kernel(const TileDesc *__restrict__ tiles,
                                                       const AsmItem *__restrict__ items,
                                                       const ProbOff *__restrict__ probs,
                                                       const float2 *__restrict__ theta_base,
                                                       const float2 *__restrict__ p_base,
                                                       float2 *__restrict__ X_base,
                                                       float2 *__restrict__ X2_base,
                                                       int64_t x2w, int64_t low) {
    constexpr int NF = DIR ? 2 : 1;   // factor sets: (L, R) and, for the directional form, (P_L, P_R)
    constexpr int SA_F = NF * 2 * A_PL;                 // floats
    constexpr int SB_F = NF * 2 * B_ST;                 // floats
    constexpr int ST_F = 2 * AB * ST_P;
    constexpr int SM_F = (SA_F + SB_F > ST_F) ? SA_F + SB_F : ST_F;
    __shared__ float smem[SM_F];
    float *sA = smem;                                  // [NF][re, im][AKC][AAP]
    float2 *sB = reinterpret_cast<float2 *>(smem + SA_F);   // [NF][AKC][ABP]
    float2 *sT = reinterpret_cast<float2 *>(smem);     // transpose stage, reused after the k loop

    const AsmItem it = items[blockIdx.x];
    const TileDesc td = tiles[it.tile];
    const ProbOff po = probs[it.prob];
    const float2 *theta = theta_base + po.theta;
    const float2 *pv = DIR ? p_base + po.theta : nullptr;
    // complex64: X at element po.x; split planes: X hi plane at word 2 po.x, X2 at + x2w words
    float2 *X = OUTB ? reinterpret_cast<float2 *>(reinterpret_cast<uint32_t *>(X_base) + 2 * po.x) : X_base + po.x;
    float2 *X2 = !DIR ? nullptr
                      : (OUTB ? reinterpret_cast<float2 *>(reinterpret_cast<uint32_t *>(X_base) + 2 * po.x + x2w)
                              : X2_base + po.x);
    const int64_t ldx = po.ldx;

    const int t = threadIdx.x;
    const int r0 = it.r0, c0 = it.c0;
    const int nrow = min(AB, td.di - r0);
    const int ncol = min(AB, td.dj - c0);

    if (td.kind == TILE_DENSE) {
        // X = (Z + Z^T)/2 ; X1 = (P + P^T)/2 ; X2 = 0 (element-wise, no products)
        const float2 *Z = DIR ? pv + td.offA : theta + td.offA;
        const int d = td.di;
        for (int e = t; e < AB * AB; e += 256) {   // transposed block Z[c0+cc][r0+rr]
            const int cc = e >> 6, rr = e & 63;
            float2 v = make_float2(0.f, 0.f);
            if (cc < ncol && rr < nrow) v = Z[(int64_t)(c0 + cc) * d + r0 + rr];
            sT[cc * ST_P + rr] = v;
        }
        __syncthreads();
        for (int e = t; e < AB * AB; e += 256) {
            const int rr = e >> 6, cc = e & 63;
            if (rr < nrow && cc < ncol) {
                const float2 zd = Z[(int64_t)(r0 + rr) * d + c0 + cc];
                const float2 zt = sT[cc * ST_P + rr];
                const int64_t o = (td.row0 + r0 + rr) * ldx + td.col0 + c0 + cc;
                put<OUTB>(X, o, low, make_float2(0.5f * (zd.x + zt.x), 0.5f * (zd.y + zt.y)));
                if (DIR) put<OUTB>(X2, o, low, make_float2(0.f, 0.f));
            }
        }
        return;
    }

    const int lane = t & 63, wave = t >> 6;
    const int j32 = lane & 31, half = lane >> 5;
    const int cb = 16 * wave;                                   // first complex column of the wave
    const int bidx = 2 * cb + (j32 ^ half);                     // float of the realified B entry
    const uint32_t bsign = (half && !(j32 & 1)) ? 0x80000000u : 0u;   // -Im g in the second k row

    floatx16 acc[2][2];   // [X | X1, X2][row half]
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[f][i][r] = 0.f;

    const bool qq = (td.kind == TILE_QQ);
    const int k = td.k;
    const float2 *Lf = theta + td.offA;                 // L (di x k) or Q (d x k)
    const float2 *Rf = qq ? Lf : theta + td.offB;       // R (k x dj) or Q again
    const float2 *PLf = DIR ? pv + td.offA : nullptr;
    const float2 *PRf = DIR ? (qq ? PLf : pv + td.offB) : nullptr;
    for (int kc0 = 0; kc0 < k; kc0 += AKC) {
        const int kn = min(AKC, k - kc0);
        for (int e = t; e < AB * AKC; e += 256) {    // row factors: rows r0.., k contiguous in theta
            const int rr = e / AKC, kk = e % AKC;
            const bool ok = rr < nrow && kk < kn;
            const int64_t o = (int64_t)(r0 + rr) * k + kc0 + kk;
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                const float2 v = ok ? (f ? PLf : Lf)[o] : make_float2(0.f, 0.f);
                float *pl = sA + f * 2 * A_PL + kk * AAP + rr;
                pl[0] = v.x;
                pl[A_PL] = v.y;
            }
        }
        for (int e = t; e < AKC * AB; e += 256) {    // column factors G[kk][cc] = R[kc0+kk][c0+cc] or Q[c0+cc][kc0+kk]
            int kk, cc;
            int64_t o;
            if (qq) { cc = e / AKC; kk = e % AKC; o = (int64_t)(c0 + cc) * k + kc0 + kk; }
            else { kk = e >> 6; cc = e & 63; o = (int64_t)(kc0 + kk) * td.dj + c0 + cc; }
            const bool ok = cc < ncol && kk < kn;
#pragma unroll
            for (int f = 0; f < NF; ++f)
                sB[f * B_ST + kk * ABP + cc] = ok ? (f ? PRf : Rf)[o] : make_float2(0.f, 0.f);
        }
        __syncthreads();
        const float *bf = reinterpret_cast<const float *>(sB);
#pragma unroll 2
        for (int kk = 0; kk < kn; ++kk) {
            float a[NF][2], b[NF];
#pragma unroll
            for (int f = 0; f < NF; ++f) {
#pragma unroll
                for (int i = 0; i < 2; ++i) a[f][i] = sA[f * 2 * A_PL + half * A_PL + kk * AAP + 32 * i + j32];
                b[f] = __uint_as_float(__float_as_uint(bf[2 * (f * B_ST + kk * ABP) + bidx]) ^ bsign);
            }
            if (!DIR) {
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    acc[0][i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][i], b[0], acc[0][i], 0, 0, 0);
            } else {
                // X1 += P_L R + L P_R ; X2 += P_L P_R (the two X1 products of a row half three apart)
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    acc[0][i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[NF - 1][i], b[0], acc[0][i], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    acc[1][i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[NF - 1][i], b[NF - 1], acc[1][i], 0, 0, 0);
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    acc[0][i] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0][i], b[NF - 1], acc[0][i], 0, 0, 0);
            }
        }
        __syncthreads();
    }

    // Lane (j32, half) holds component j32 & 1 of complex column cb + j32 / 2 for rows
    // acc_row(r, lane) (+ 32 for the second half). Each product is staged through LDS once and
    // written from there twice, both times with whole rows per wave: X_ij directly and X_ji = X_ij^T.
    // Q Q^T tiles are built on and below the block diagonal only and mirrored, so the tile is
    // symmetric bit for bit: direct write where row >= column, transposed write where row > column.
    const int ccol = cb + (j32 >> 1);
    const int comp = j32 & 1;
    float *sTf = smem;   // [row][ST_P] complex
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                sTf[2 * ((32 * i + acc_row(r, lane)) * ST_P + ccol) + comp] = acc[f][i][r];
        __syncthreads();
        float2 *dst = f ? X2 : X;
        for (int e = t; e < AB * AB; e += 256) {
            const int rr = e >> 6, cc = e & 63;
            if (rr < nrow && cc < ncol && (!qq || r0 + rr >= c0 + cc))
                put<OUTB>(dst, (td.row0 + r0 + rr) * ldx + td.col0 + c0 + cc, low, sT[rr * ST_P + cc]);
        }
        for (int e = t; e < AB * AB; e += 256) {
            const int cc = e >> 6, rr = e & 63;
            if (cc < ncol && rr < nrow && (!qq || r0 + rr > c0 + cc))
                put<OUTB>(dst, (td.col0 + c0 + cc) * ldx + td.row0 + r0 + rr, low, sT[rr * ST_P + cc]);
        }
    }
}

constexpr int GW_P = GR_ROWS + 1;      // W' planes [GR_CH][GW_P] floats (contraction index major)
constexpr int GF_P = GR_KK + 1;        // factor stage [GR_CH][GF_P] complex
constexpr int GW_PL = GR_CH * GW_P;    // floats per W' plane
constexpr int GO_P = GR_ROWS + 1;      // output stage of G_R [GR_KK][GO_P] complex

// One gradient item: a 64 x kn block (kn <= 64 rank entries from b0) of G = W' conj(F), where
//   G_L: rows of the tile, F[c][kk] = R[kk][c]    (G_L = W' R^H, contraction over tile columns)
//   G_Q: rows of the tile, F[c][kk] = Q[c][kk]    (G_Q = (W + W^T) conj(Q))
//   G_R: cols of the tile, F[r][kk] = L[r][kk]    (G_R^T = W'^T conj(L), contraction over tile rows)
// with W' = W_ij + W_ji^T built in LDS chunk by chunk (both parts' loads issued together, each read
// along its own rows). Chunks are only 4 contraction steps wide: that keeps a workgroup at 72 VGPRs
// and 17 KB of LDS, and the seven workgroups per CU that this allows hide the W loads far better
// than fewer, wider ones (32-wide chunks: 3 workgroups per CU, 1.3x the time). The contraction runs on the FP32 matrix cores in realified form (one
// v_mfma_f32_32x32x2_f32 per complex contraction step: (Re, Im) of W'[m][c] as the two A entries,
// the real 2 x 2 block of conj(F[c][n]) as B). Wave w owns rank entries 16 w .. 16 w + 15 and both
// 32-row halves; waves past the item's rank only stage data. W' sits in LDS as re / im planes with
// the contraction index major (one conflict-free float per A entry); G_R is transposed through LDS
// so its rows are written whole.
__device__ __forceinline__ void grad_block(const GradItem &it, const TileDesc &td, const float2 *__restrict__ W,
                                           int64_t ldw, const float2 *__restrict__ theta, float2 *__restrict__ g,
                                           float *smem) {
    float *sW = smem;                                              // [re, im][GR_CH][GW_P]
    float2 *sF = reinterpret_cast<float2 *>(smem + 2 * GW_PL);     // [GR_CH][GF_P]
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int j32 = lane & 31, half = lane >> 5;
    const int k = td.k;
    const int a0 = it.a0, b0 = it.b0;
    const int kn = min(GR_KK, k - b0);
    const bool colside = it.kind == G_R;
    const int nout = min(GR_ROWS, (colside ? td.dj : td.di) - a0);   // out-rows in this item
    const int ncon = colside ? td.di : td.dj;                        // contraction length
    const float2 *F = it.kind == G_L ? theta + td.offB : theta + td.offA;
    const bool active = 16 * wave < kn;
    const int fidx = 2 * 16 * wave + (j32 ^ half);                   // float of the realified B entry
    const uint32_t fsign = (!half && (j32 & 1)) ? 0x80000000u : 0u;  // conj: -Im f in the first k row

    floatx16 acc[2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;

    for (int c0 = 0; c0 < ncon; c0 += GR_CH) {
        const int cn = min(GR_CH, ncon - c0);
        // W' = W_ij part + W_ji part: both parts' loads are issued before either is stored
        //   part 0: W'[m][c] = W_ij[a0+m][c0+c] (G_L, G_Q) or W_ij[c0+c][a0+m] (G_R)
        //   part 1: + W_ji[c0+c][a0+m] (G_L, G_Q) or + W_ji[a0+m][c0+c] (G_R)
        float2 v0[GR_ROWS * GR_CH / 256], v1[GR_ROWS * GR_CH / 256];
#pragma unroll
        for (int u = 0; u < GR_ROWS * GR_CH / 256; ++u) {
            const int e = t + 256 * u;
            int m, c;
            int64_t o;
            if (!colside) { m = e / GR_CH; c = e % GR_CH; o = (td.row0 + a0 + m) * ldw + td.col0 + c0 + c; }
            else { c = e / GR_ROWS; m = e % GR_ROWS; o = (td.row0 + c0 + c) * ldw + td.col0 + a0 + m; }
            v0[u] = (m < nout && c < cn) ? W[o] : make_float2(0.f, 0.f);
            if (!colside) { c = e / GR_ROWS; m = e % GR_ROWS; o = (td.col0 + c0 + c) * ldw + td.row0 + a0 + m; }
            else { m = e / GR_CH; c = e % GR_CH; o = (td.col0 + a0 + m) * ldw + td.row0 + c0 + c; }
            v1[u] = (m < nout && c < cn) ? W[o] : make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int u = 0; u < GR_ROWS * GR_CH / 256; ++u) {
            const int e = t + 256 * u;
            int m, c;
            if (!colside) { m = e / GR_CH; c = e % GR_CH; } else { c = e / GR_ROWS; m = e % GR_ROWS; }
            sW[c * GW_P + m] = v0[u].x;
            sW[GW_PL + c * GW_P + m] = v0[u].y;
        }
        for (int e = t; e < GR_CH * GR_KK; e += 256) {
            int c, kk;
            int64_t o;
            if (it.kind == G_L) { kk = e / GR_CH; c = e % GR_CH; o = (int64_t)(b0 + kk) * td.dj + c0 + c; }
            else { c = e / GR_KK; kk = e % GR_KK; o = (int64_t)(c0 + c) * k + b0 + kk; }
            sF[c * GF_P + kk] = (c < cn && kk < kn) ? F[o] : make_float2(0.f, 0.f);
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < GR_ROWS * GR_CH / 256; ++u) {
            const int e = t + 256 * u;
            int m, c;
            if (!colside) { c = e / GR_ROWS; m = e % GR_ROWS; } else { m = e / GR_CH; c = e % GR_CH; }
            sW[c * GW_P + m] += v1[u].x;
            sW[GW_PL + c * GW_P + m] += v1[u].y;
        }
        __syncthreads();
        if (active) {
            const float *fw = reinterpret_cast<const float *>(sF);
#pragma unroll 4
            for (int c = 0; c < cn; ++c) {
                const float b = __uint_as_float(__float_as_uint(fw[2 * c * GF_P + fidx]) ^ fsign);
#pragma unroll
                for (int i = 0; i < 2; ++i)
                    acc[i] = __builtin_amdgcn_mfma_f32_32x32x2f32(sW[half * GW_PL + c * GW_P + 32 * i + j32], b,
                                                                   acc[i], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // lane (j32, half) holds component j32 & 1 of rank entry 16 wave + j32 / 2 for out-rows
    // 32 i + acc_row(r, lane)
    const int kk = 16 * wave + (j32 >> 1), comp = j32 & 1;
    if (!colside) {
        // grad L / grad Q at the factor's own offset, rows of k entries
        if (active)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int m = 32 * i + acc_row(r, lane);
                    if (m < nout && kk < kn)
                        reinterpret_cast<float *>(g)[2 * (td.offA + (int64_t)(a0 + m) * k + b0 + kk) + comp] = acc[i][r];
                }
        return;
    }
    // grad R = L^H W' has the entries of G_R^T: stage [kk][m] (32 rank entries at a time: the
    // waves that own them) and write rows of R's gradient
    float *sO = smem;   // [GR_KK / 2][GO_P] complex
    const float2 *sO2 = reinterpret_cast<const float2 *>(sO);
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
        if (active && (wave >> 1) == hh)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int r = 0; r < 16; ++r)
                    sO[2 * ((kk - 32 * hh) * GO_P + 32 * i + acc_row(r, lane)) + comp] = acc[i][r];
        __syncthreads();
        for (int e = t; e < (GR_KK / 2) * GR_ROWS; e += 256) {
            const int q = e >> 6, m = e & 63;
            const int qq = 32 * hh + q;
            if (qq < kn && m < nout) g[td.offB + (int64_t)(b0 + qq) * td.dj + a0 + m] = sO2[q * GO_P + m];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void grad_kernel(const TileDesc *__restrict__ tiles,
                                                   const GradItem *__restrict__ items,
                                                   const ProbOff *__restrict__ probs,
                                                   const float2 *__restrict__ W_base,
                                                   const float2 *__restrict__ theta_base,
                                                   float2 *__restrict__ g_base) {
    constexpr int SM_G = 2 * GW_PL + 2 * GR_CH * GF_P;
    constexpr int SM_O = 2 * (GR_KK / 2) * GO_P;
    constexpr int SM_Z = 2 * GZ_BC * (GZ_BR + 1);
    constexpr int SM_F = SM_G > SM_O ? (SM_G > SM_Z ? SM_G : SM_Z) : (SM_O > SM_Z ? SM_O : SM_Z);
    __shared__ float smem[SM_F];
    const GradItem it = items[blockIdx.x];
    const TileDesc td = tiles[it.tile];
    const ProbOff po = probs[it.prob];
    const float2 *W = W_base + po.x;
    const int64_t ldw = po.ldx;
    const float2 *theta = theta_base + po.theta;
    float2 *g = g_base + po.theta;
    const int t = threadIdx.x;

    if (it.kind == G_Z) {
        // grad Z = (W_ii + W_ii^T)/2 on the block rows a0.., cols b0..
        float2 *sW = reinterpret_cast<float2 *>(smem);
        const int d = td.di;
        const int a0 = it.a0, b0 = it.b0;
        const int nrow = min(GZ_BR, d - a0), ncol = min(GZ_BC, d - b0);
        for (int e = t; e < GZ_BC * GZ_BR; e += 256) {
            const int cc = e >> 5, rr = e & 31;
            float2 v = make_float2(0.f, 0.f);
            if (cc < ncol && rr < nrow) v = W[(td.row0 + b0 + cc) * ldw + td.col0 + a0 + rr];
            sW[cc * (GZ_BR + 1) + rr] = v;
        }
        __syncthreads();
        for (int e = t; e < GZ_BR * GZ_BC; e += 256) {
            const int rr = e >> 6, cc = e & 63;
            if (rr < nrow && cc < ncol) {
                const float2 wd = W[(td.row0 + a0 + rr) * ldw + td.col0 + b0 + cc];
                const float2 wt = sW[cc * (GZ_BR + 1) + rr];
                g[td.offA + (int64_t)(a0 + rr) * d + b0 + cc] =
                    make_float2(0.5f * (wd.x + wt.x), 0.5f * (wd.y + wt.y));
            }
        }
        return;
    }
    grad_block(it, td, W, ldw, theta, g, smem);
}

}  // namespace

hipError_t launch_assemble(bool dir, const TileDesc *tiles, const AsmItem *items, int nitems,
                           const ProbOff *probs, const float2 *theta, const float2 *p,
                           float2 *X, float2 *X2, hipStream_t s, bool out_bf16, int64_t x2_words,
                           int64_t lo_words) {
    if (nitems <= 0) return hipSuccess;
    const dim3 g(nitems), b(256);
    if (dir && out_bf16)
        hipLaunchKernelGGL((assemble_kernel<true, true>), g, b, 0, s, tiles, items, probs, theta, p, X, X2, x2_words, lo_words);
    else if (dir)
        hipLaunchKernelGGL((assemble_kernel<true, false>), g, b, 0, s, tiles, items, probs, theta, p, X, X2, x2_words, lo_words);
    else if (out_bf16)
        hipLaunchKernelGGL((assemble_kernel<false, true>), g, b, 0, s, tiles, items, probs, theta, p, X, X2, x2_words, lo_words);
    else
        hipLaunchKernelGGL((assemble_kernel<false, false>), g, b, 0, s, tiles, items, probs, theta, p, X, X2, x2_words, lo_words);
    return hipGetLastError();
}

hipError_t launch_grad(const TileDesc *tiles, const GradItem *items, int nitems,
                       const ProbOff *probs, const float2 *W, const float2 *theta, float2 *g,
                       hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(grad_kernel, dim3(nitems), dim3(256), 0, s, tiles, items, probs, W, theta, g);
    return hipGetLastError();
}

}  // namespace tlr
