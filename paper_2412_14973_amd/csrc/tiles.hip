// Tile kernels: assembly of X = C(Zbar, Lbar, Rbar) and the per-tile gradient
// contractions.
//
// Assembly (Tile Low-rank MDD section): X_ij = L_ij R_ij for i > j and
// X_ji = X_ij^T; X_ii = Q_ii Q_ii^T or (Z_ii + Z_ii^T)/2. The directional
// form used by the exact line search expands C(theta + a p) = C(theta) +
// a X1 + a^2 X2, tile by tile: X1 = P_L R + L P_R, X2 = P_L P_R (and the
// Q Q^T / dense analogues). Each workgroup builds one 32 x 64 block from
// factors staged in LDS 32 rank entries at a time; sub-diagonal blocks are
// written twice (directly and transposed through LDS, both coalesced), so
// X = X^T holds bit for bit. Q Q^T entries are computed with the operands
// ordered by (max(a,b), min(a,b)) so the (a,b) and (b,a) entries follow the
// same rounding path.
//
// Gradient (ADMM solver section, eqs. DXLR): with W = D^H r and W' = W + W^T,
// grad L = W' R^H, grad R = L^H W', grad Q = W' conj(Q), grad Z = W'/2.
// W' is never formed: each block of W'_ij is built in LDS from a block of
// W_ij plus the transposed block of W_ji, both read coalesced.
#include "common.hpp"

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
constexpr int SL_P = ASM_KC + 1;     // row-factor stage [AB][SL_P]
constexpr int SR_P = AB + 1;         // column-factor stage [ASM_KC][SR_P]
constexpr int ST_P = AB + 1;         // transpose stage [AB][ST_P]
constexpr int STAGE_F2 = AB * SL_P + ASM_KC * SR_P;

// Each workgroup builds one 64 x 64 block of a tile; thread (ty, tx) = (t / 16, t % 16) owns
// rows ty + 16 i and columns tx + 16 j (i, j < 4): a 4 x 4 register block, so every complex
// value read from LDS feeds 4 (12 in the directional form) complex multiply-adds.
template <bool DIR, bool OUTB>
__global__ __launch_bounds__(256) void assemble_kernel(const TileDesc *__restrict__ tiles,
                                                       const AsmItem *__restrict__ items,
                                                       const ProbOff *__restrict__ probs,
                                                       const float2 *__restrict__ theta_base,
                                                       const float2 *__restrict__ p_base,
                                                       float2 *__restrict__ X_base,
                                                       float2 *__restrict__ X2_base,
                                                       int64_t x2w, int64_t low) {
    constexpr int NSTAGE = DIR ? 2 : 1;
    constexpr int SM_F2 = (NSTAGE * STAGE_F2 > AB * ST_P) ? NSTAGE * STAGE_F2 : AB * ST_P;
    __shared__ float2 smem[SM_F2];
    float2 *sL = smem;                               // [NSTAGE][AB][SL_P]
    float2 *sR = smem + NSTAGE * AB * SL_P;          // [NSTAGE][ASM_KC][SR_P]
    float2 *sT = smem;                               // transpose stage, reused after the k loop

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
    const int tx = t & 15, ty = t >> 4;
    const int r0 = it.r0, c0 = it.c0;
    const int nrow = min(AB, td.di - r0);
    const int ncol = min(AB, td.dj - c0);

    float2 acc[4][4], acc2[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) { acc[i][j] = make_float2(0.f, 0.f); acc2[i][j] = acc[i][j]; }

    if (td.kind == TILE_DENSE) {
        // X = (Z + Z^T)/2 ; X1 = (P + P^T)/2 ; X2 = 0
        const float2 *Z = DIR ? pv + td.offA : theta + td.offA;
        const int d = td.di;
        for (int e = t; e < AB * AB; e += 256) {   // transposed block Z[c0+cc][r0+rr]
            const int cc = e >> 6, rr = e & 63;
            float2 v = make_float2(0.f, 0.f);
            if (cc < ncol && rr < nrow) v = Z[(int64_t)(c0 + cc) * d + r0 + rr];
            sT[cc * ST_P + rr] = v;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int rr = ty + 16 * i, cc = tx + 16 * j;
                if (rr < nrow && cc < ncol) {
                    const float2 zd = Z[(int64_t)(r0 + rr) * d + c0 + cc];
                    const float2 zt = sT[cc * ST_P + rr];
                    acc[i][j] = make_float2(0.5f * (zd.x + zt.x), 0.5f * (zd.y + zt.y));
                }
            }
        __syncthreads();
    } else {
        const bool qq = (td.kind == TILE_QQ);
        const int k = td.k;
        const float2 *Lf = theta + td.offA;                 // L (di x k) or Q (d x k)
        const float2 *Rf = qq ? Lf : theta + td.offB;       // R (k x dj) or Q again
        const float2 *PLf = DIR ? pv + td.offA : nullptr;
        const float2 *PRf = DIR ? (qq ? PLf : pv + td.offB) : nullptr;
        for (int kc0 = 0; kc0 < k; kc0 += ASM_KC) {
            const int kn = min(ASM_KC, k - kc0);
            for (int e = t; e < AB * ASM_KC; e += 256) {    // row factor rows r0.. : [rr][kk]
                const int rr = e >> 5, kk = e & 31;
                const bool ok = rr < nrow && kk < kn;
                const int64_t o = (int64_t)(r0 + rr) * k + kc0 + kk;
                sL[rr * SL_P + kk] = ok ? Lf[o] : make_float2(0.f, 0.f);
                if (DIR) sL[AB * SL_P + rr * SL_P + kk] = ok ? PLf[o] : make_float2(0.f, 0.f);
            }
            for (int e = t; e < ASM_KC * AB; e += 256) {    // column factor R[kc0+kk][c0+cc] or Q[c0+cc][kc0+kk]
                int kk, cc;
                int64_t o;
                if (qq) { cc = e >> 5; kk = e & 31; o = (int64_t)(c0 + cc) * k + kc0 + kk; }
                else { kk = e >> 6; cc = e & 63; o = (int64_t)(kc0 + kk) * td.dj + c0 + cc; }
                const bool ok = cc < ncol && kk < kn;
                sR[kk * SR_P + cc] = ok ? Rf[o] : make_float2(0.f, 0.f);
                if (DIR) sR[ASM_KC * SR_P + kk * SR_P + cc] = ok ? PRf[o] : make_float2(0.f, 0.f);
            }
            __syncthreads();
#pragma unroll 2
            for (int kk = 0; kk < kn; ++kk) {
                float2 lv[4], rv[4], plv[4], prv[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    lv[i] = sL[(ty + 16 * i) * SL_P + kk];
                    rv[i] = sR[kk * SR_P + tx + 16 * i];
                    if (DIR) {
                        plv[i] = sL[AB * SL_P + (ty + 16 * i) * SL_P + kk];
                        prv[i] = sR[ASM_KC * SR_P + kk * SR_P + tx + 16 * i];
                    }
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        if (!DIR) {
                            acc[i][j] = cadd(acc[i][j], cmul(lv[i], rv[j]));
                        } else {
                            acc[i][j] = cadd(acc[i][j], cadd(cmul(plv[i], rv[j]), cmul(lv[i], prv[j])));
                            acc2[i][j] = cadd(acc2[i][j], cmul(plv[i], prv[j]));
                        }
                    }
            }
            __syncthreads();
        }
    }

    // Q Q^T tiles are built on and below the block diagonal only and mirrored, so the tile is
    // symmetric bit for bit: direct write where row >= column, transposed write where row > column
    const bool qq = td.kind == TILE_QQ;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int rr = ty + 16 * i, cc = tx + 16 * j;
            if (rr < nrow && cc < ncol && (!qq || r0 + rr >= c0 + cc)) {
                const int64_t o = (td.row0 + r0 + rr) * ldx + td.col0 + c0 + cc;
                put<OUTB>(X, o, low, acc[i][j]);
                if (DIR) put<OUTB>(X2, o, low, acc2[i][j]);
            }
        }
    if (td.kind == TILE_DENSE) return;
    // transposed block X_ji = X_ij^T, staged through LDS for coalesced rows
    for (int pass = 0; pass < (DIR ? 2 : 1); ++pass) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                sT[(tx + 16 * j) * ST_P + ty + 16 * i] = (pass == 0) ? acc[i][j] : acc2[i][j];
        __syncthreads();
        float2 *dst = (pass == 0) ? X : X2;
        for (int e = t; e < AB * AB; e += 256) {
            const int cc = e >> 6, rr = e & 63;
            if (cc < ncol && rr < nrow && (!qq || r0 + rr > c0 + cc))
                put<OUTB>(dst, (td.col0 + c0 + cc) * ldx + td.row0 + r0 + rr, low, sT[cc * ST_P + rr]);
        }
    }
}

constexpr int GW_P = GR_CH + 1;        // sW [GR_ROWS][GW_P]: W' with the contraction index fastest
constexpr int GF_P = GR_KK + 1;        // sF [GR_CH][GF_P]: conjugated factor, rank index fastest

// One gradient item: a 64 x (16 KQ) block of G = W' conj(F) where
//   G_L: rows of the tile, F[c][kk] = R[kk][c]    (G_L = W' R^H, contraction over tile columns)
//   G_Q: rows of the tile, F[c][kk] = Q[c][kk]    (G_Q = (W + W^T) conj(Q))
//   G_R: cols of the tile, F[r][kk] = L[r][kk]    (G_R^T = W'^T conj(L), contraction over tile rows)
// with W' = W_ij + W_ji^T built in LDS chunk by chunk. Thread (ty, tx) owns out-rows ty + 16 i
// (i < 4) and rank entries tx + 16 j (j < KQ).
template <int KQ>
__device__ __forceinline__ void grad_block(const GradItem &it, const TileDesc &td, const float2 *__restrict__ W,
                                           int64_t ldw, const float2 *__restrict__ theta, float2 *__restrict__ g,
                                           float2 *sW, float2 *sF) {
    const int t = threadIdx.x;
    const int tx = t & 15, ty = t >> 4;
    const int k = td.k;
    const int a0 = it.a0, b0 = it.b0;
    const int kn = min(16 * KQ, k - b0);
    const bool colside = it.kind == G_R;
    const int nout = min(GR_ROWS, (colside ? td.dj : td.di) - a0);   // out-rows in this item
    const int ncon = colside ? td.di : td.dj;                        // contraction length
    const float2 *F = it.kind == G_L ? theta + td.offB : theta + td.offA;

    float2 acc[4][KQ];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < KQ; ++j) acc[i][j] = make_float2(0.f, 0.f);

    for (int c0 = 0; c0 < ncon; c0 += GR_CH) {
        const int cn = min(GR_CH, ncon - c0);
        if (!colside) {
            // sW[rr][cc] = W_ij[a0+rr][c0+cc] + W_ji[c0+cc][a0+rr]
            for (int e = t; e < GR_ROWS * GR_CH; e += 256) {
                const int rr = e >> 5, cc = e & 31;
                float2 v = make_float2(0.f, 0.f);
                if (rr < nout && cc < cn) v = W[(td.row0 + a0 + rr) * ldw + td.col0 + c0 + cc];
                sW[rr * GW_P + cc] = v;
            }
        } else {
            // sW[cc][rr] = W_ij[c0+rr][a0+cc] + W_ji[a0+cc][c0+rr]   (out-row cc is a tile column)
            for (int e = t; e < GR_CH * GR_ROWS; e += 256) {
                const int rr = e >> 6, cc = e & 63;
                float2 v = make_float2(0.f, 0.f);
                if (cc < nout && rr < cn) v = W[(td.row0 + c0 + rr) * ldw + td.col0 + a0 + cc];
                sW[cc * GW_P + rr] = v;
            }
        }
        for (int e = t; e < GR_CH * 16 * KQ; e += 256) {
            const int cc = e / (16 * KQ), kk = e % (16 * KQ);
            float2 v = make_float2(0.f, 0.f);
            if (cc < cn && kk < kn) {
                const int64_t o = it.kind == G_L ? (int64_t)(b0 + kk) * td.dj + c0 + cc
                                                 : (int64_t)(c0 + cc) * k + b0 + kk;
                v = F[o];
            }
            sF[cc * GF_P + kk] = v;
        }
        __syncthreads();
        if (!colside) {
            for (int e = t; e < GR_CH * GR_ROWS; e += 256) {
                const int cc = e >> 6, rr = e & 63;
                if (rr < nout && cc < cn) {
                    const float2 wt = W[(td.col0 + c0 + cc) * ldw + td.row0 + a0 + rr];
                    sW[rr * GW_P + cc] = cadd(sW[rr * GW_P + cc], wt);
                }
            }
        } else {
            for (int e = t; e < GR_ROWS * GR_CH; e += 256) {
                const int cc = e >> 5, rr = e & 31;
                if (cc < nout && rr < cn) {
                    const float2 wt = W[(td.col0 + a0 + cc) * ldw + td.row0 + c0 + rr];
                    sW[cc * GW_P + rr] = cadd(sW[cc * GW_P + rr], wt);
                }
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int cc = 0; cc < cn; ++cc) {
            float2 w[4], f[KQ];
#pragma unroll
            for (int i = 0; i < 4; ++i) w[i] = sW[(ty + 16 * i) * GW_P + cc];
#pragma unroll
            for (int j = 0; j < KQ; ++j) f[j] = sF[cc * GF_P + tx + 16 * j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < KQ; ++j) acc[i][j] = cadd(acc[i][j], cmulc(w[i], f[j]));
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < KQ; ++j) {
            const int rr = ty + 16 * i, kk = tx + 16 * j;
            if (rr < nout && kk < kn) {
                // grad L / grad Q at the factor's own offset; grad R = L^H W' has the entries of acc
                if (!colside) g[td.offA + (int64_t)(a0 + rr) * k + b0 + kk] = acc[i][j];
                else g[td.offB + (int64_t)(b0 + kk) * td.dj + a0 + rr] = acc[i][j];
            }
        }
}

__global__ __launch_bounds__(256) void grad_kernel(const TileDesc *__restrict__ tiles,
                                                   const GradItem *__restrict__ items,
                                                   const ProbOff *__restrict__ probs,
                                                   const float2 *__restrict__ W_base,
                                                   const float2 *__restrict__ theta_base,
                                                   float2 *__restrict__ g_base) {
    __shared__ float2 sW[GR_ROWS * GW_P];
    __shared__ float2 sF[GR_CH * GF_P];
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
    switch (it.kq) {
    case 1: grad_block<1>(it, td, W, ldw, theta, g, sW, sF); break;
    case 2: grad_block<2>(it, td, W, ldw, theta, g, sW, sF); break;
    case 3: grad_block<3>(it, td, W, ldw, theta, g, sW, sF); break;
    default: grad_block<4>(it, td, W, ldw, theta, g, sW, sF); break;
    }
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
