// Complex64 GEMM on FP32 matrix cores in the three-real-product ("3M") form.
//
// C = A B with A = Ar + i Ai, B = Br + i Bi is formed from three real products
//   T1 = Ar Br,  T2 = Ai Bi,  T3 = (Ar + Ai)(Br + Bi),
//   Re C = T1 - T2,  Im C = T3 - T1 - T2,
// i.e. 6MNK real flops instead of the 8MNK of the four-product (realified) form,
// at the price of one extra rounding level in Im C (the sums Ar + Ai, Br + Bi
// and the final differences). Operands are the same interleaved complex64
// matrices as for the four-product kernel: every loaded tile is split into
// its real and imaginary planes while it is stored to LDS, and each lane forms
// the sums Ar + Ai, Br + Bi of its operand fragments after reading them.
//
// Tiling: 256 threads = 4 waves (2 x 2), two workgroups per CU (the barrier and
// epilogue of one overlap the products of the other); workgroup tile 128 rows x
// 128 complex columns, 16 complex k per stage, double-buffered LDS (two A planes
// k-major with an odd pitch, two B planes row-major: conflict-free operand reads;
// 2 x 32.1 KiB). Each wave owns 64 rows x 64 columns: accumulators T1, T2, T3 for
// 2 x 2 blocks of 32 x 32 (192 of its 256 VGPRs), so each operand fragment read
// from LDS feeds two MFMAs. One v_mfma_f32_32x32x2_f32 consumes two complex k of
// one plane pair.
//   GM_STORE / GM_RESID: wave columns wn*64 .. +63;
//   GM_LINE: the B tile holds X1 and X2 at the same 64 columns; a wave's column
//     block 0 is 32 columns of X1 and block 1 the same 32 columns of X2, so a, b
//     and r meet in one thread.
// Epilogues as the four-product kernel: C; C = AB - U with FP64 partial sums of
// |C|^2; a, b with the five line-search sums. K must be a multiple of 16.
// The GM_STORE products of the tile forms may have N a multiple of 64: a last 64-column tile runs as
// its own instantiation (HALF), in which each wave takes 32 rows of all 64 columns (one row block,
// two column blocks) and the B tile's other 64 columns are not loaded.
#include <algorithm>
#include <type_traits>

#include "gemm_common.hpp"

namespace tlr {

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = GEMM_BM, BN = GEMM_BN;
constexpr int BK = GEMM_BK;           // complex k per stage
constexpr int AP = BM + 1;            // A plane pitch (floats per complex-k row, k-major)
constexpr int A_PLANE = BK * AP;
constexpr int BP = BN;                // B plane pitch (floats per k row)
constexpr int B_PLANE = BK * BP;
constexpr int STAGE = 2 * A_PLANE + 2 * B_PLANE;   // floats: re and im planes of A and B

// ROLE (GemmRole): 0 = the solver's dense products, 1 = the stages of the tile-form line search and
// gradient (the same code; separate instantiations so that profiles tell them apart), 2 = a tile-form
// gradient stage whose A is given transposed (a K x M source with row pitch lda, read along M like a
// B tile) and whose B enters conjugated
// HALF (GM_STORE tile stages): the launch covers one column tile of 64 columns at g.n_half
template <int MODE, int ROLE, bool HALF = false>
__global__ __launch_bounds__(256, 2) void cgemm3m_kernel(GemmArgs g) {
    __shared__ float sm[2][STAGE];

    // batch entry: z1 * s + z2 * s2 (two-level batch) or z * s; GM_STORE tile stages may split z2
    // further into operand sets (z4, strides s4) and contraction parts (z3, strides s3)
    const int zz = blockIdx.y;
    const int z = g.nz2 > 1 ? zz / g.nz2 : zz;
    int z2 = g.nz2 > 1 ? zz % g.nz2 : 0;
    int z3 = 0, z4 = 0;
    if (MODE == GM_STORE && ROLE != 0) {
        if (g.nz4 > 1) {
            z4 = z2 % g.nz4;
            z2 = z2 / g.nz4;
        }
        if (g.nz3 > 1) {
            z3 = z2 % g.nz3;
            z2 = z2 / g.nz3;
        }
    }
    const float2 *A = g.A + z * g.sA + z2 * g.sA2 + z3 * g.sA3 + z4 * g.sA4;
    const float2 *B = g.B + z * g.sB + z2 * g.sB2 + z3 * g.sB3 + z4 * g.sB4;

    // workgroup -> tile: contiguous tile ranges per XCD, grouped by 4 tile rows. With 1024-row operands
    // (8 row tiles) an XCD's 16 tiles of a problem are then 4 rows x 4 columns: it reads half of A and a
    // quarter of B instead of all of A (8 x 2), and the products fetch 15-30 % fewer bytes from beyond L2
    const int nb = gridDim.x;
    int pid = blockIdx.x;
    if ((nb & 7) == 0) pid = (pid & 7) * (nb >> 3) + (pid >> 3);
    const int group_rows = 4;
    const int per_group = group_rows * g.tiles_n;
    const int grp = pid / per_group;
    const int first_m = grp * group_rows;
    const int gsz = min(g.tiles_m - first_m, group_rows);
    const int tm = first_m + (pid % per_group) % gsz;
    const int tn = (pid % per_group) / gsz;
    const int m0 = tm * BM;
    // a 64-column tile: its four waves each take 32 rows of all 64 columns, and the other 64
    // columns are not loaded
    static_assert(!HALF || (MODE == GM_STORE && ROLE != 0), "64-column tiles: tile-stage GM_STORE only");
    constexpr bool halfn = HALF;
    const int n0 = HALF ? g.n_half : (MODE == GM_LINE) ? tn * (BN / 2) : tn * BN;

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int j32 = lane & 31, half = lane >> 5;

    // ---- global -> register loaders (operands padded to whole tiles: no bounds checks) ----
    // A: row t/2, complex k 8 (t%2) .. +7 (four float4); B: k row t/16, complex columns
    // 4 (t%16) .. +3 and 64 + 4 (t%16) .. +3 (two float4 each)
    constexpr int AQ = BK / 8;                     // threads per A row (8 complex k each)
    constexpr int BR = 256 / 16;                   // B rows per pass (16 threads per row)
    static_assert(BK % 8 == 0 && BK <= 16, "A loader");
    const int a_row = t / AQ, a_q = t % AQ;
    const int b_row = t >> 4, b_q = t & 15;
    const __amdgpu_buffer_rsrc_t rsA =
        __builtin_amdgcn_make_buffer_rsrc((void *)A, (short)0, (int)g.bytesA, 0x00020000);
    const __amdgpu_buffer_rsrc_t rsB =
        __builtin_amdgcn_make_buffer_rsrc((void *)B, (short)0, (int)g.bytesB, 0x00020000);
    constexpr bool TA = ROLE == 2;                 // A source K x M: k row t/16, m 4 (t%16) .. +3, 64 + ..
    const uint32_t offA = TA ? (uint32_t)(((int64_t)b_row * g.lda + m0 + 4 * b_q) * 8)
                             : (uint32_t)(((int64_t)(m0 + a_row) * g.lda + 8 * a_q) * 8);
    uint32_t offB[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int c = 64 * h + 4 * b_q;   // complex column inside the LDS tile
        int64_t base = n0 + c;
        if (MODE == GM_LINE) base = h ? n0 + (c - 64) + g.b2_off : n0 + c;   // X1 | X2
        offB[h] = (uint32_t)((base + (int64_t)b_row * g.ldb) * 8);
    }
    auto ld16 = [](__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
        const u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, (int)voff, (int)soff, 0);
        return make_float4(__uint_as_float(v.x), __uint_as_float(v.y), __uint_as_float(v.z), __uint_as_float(v.w));
    };
    constexpr int NBQ = BK / BR;                   // B row passes per stage
    float4 ra[4], rb[NBQ][4];
    // b2: this stage also needs the B2 half of the tile (GM_LINE past K2 reads B only)
    auto load = [&](int k0, bool b2) {
        if (TA) {
            const uint32_t sa = (uint32_t)((int64_t)k0 * g.lda * 8);
#pragma unroll
            for (int q = 0; q < 4; ++q) ra[q] = ld16(rsA, offA + 512 * (q >> 1) + 16 * (q & 1), sa);
        } else {
            const uint32_t sa = (uint32_t)k0 * 8u;
#pragma unroll
            for (int q = 0; q < 4; ++q) ra[q] = ld16(rsA, offA + 16 * q, sa);
        }
#pragma unroll
        for (int pb = 0; pb < NBQ; ++pb) {
            const uint32_t sb = (uint32_t)((int64_t)(k0 + BR * pb) * g.ldb * 8);
#pragma unroll
            for (int q = 0; q < 2; ++q) rb[pb][q] = ld16(rsB, offB[0] + 16 * q, sb);
            if (b2) {
#pragma unroll
                for (int q = 2; q < 4; ++q) rb[pb][q] = ld16(rsB, offB[1] + 16 * (q & 1), sb);
            }
        }
    };
    // split into re and im planes (the sums re + im are formed after the operand reads)
    auto store_lds = [&](int buf, bool b2) {
        float *ar = sm[buf], *ai = ar + A_PLANE;
        float *br = ai + A_PLANE, *bi = br + B_PLANE;
        if (TA) {   // k row b_row, m = 64 (q / 2) + 4 b_q + 2 (q % 2) + {0, 1}
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int o = b_row * AP + 64 * (q >> 1) + 4 * b_q + 2 * (q & 1);
                ar[o] = ra[q].x;
                ai[o] = ra[q].y;
                ar[o + 1] = ra[q].z;
                ai[o + 1] = ra[q].w;
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int o = (8 * a_q + 2 * q) * AP + a_row;
                ar[o] = ra[q].x;
                ai[o] = ra[q].y;
                ar[o + AP] = ra[q].z;
                ai[o + AP] = ra[q].w;
            }
        }
#pragma unroll
        for (int pb = 0; pb < NBQ; ++pb)
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                if (h == 1 && !b2) continue;
                const float4 *rr = rb[pb];
                const int ob = (b_row + BR * pb) * BP + 64 * h + 4 * b_q;
                *reinterpret_cast<float4 *>(br + ob) = make_float4(rr[2 * h].x, rr[2 * h].z, rr[2 * h + 1].x, rr[2 * h + 1].z);
                float4 vi = make_float4(rr[2 * h].y, rr[2 * h].w, rr[2 * h + 1].y, rr[2 * h + 1].w);
                if (ROLE == 2) vi = make_float4(-vi.x, -vi.y, -vi.z, -vi.w);   // conj(B)
                *reinterpret_cast<float4 *>(bi + ob) = vi;
            }
    };

    // wave tile (2 x 2 waves): rows wm*64 + 32 i (i < 2); STORE/RESID columns wn*64 + 32 j (j < 2),
    // LINE columns wn*32 of X1 (j = 0, LDS column wn*32) and X2 (j = 1, LDS column 64 + wn*32)
    const int wm = wave >> 1, wn = wave & 1;
    int aoff[2], boff[2];
    aoff[0] = wm * 64 + j32;
    aoff[1] = wm * 64 + 32 + j32;
    if (MODE == GM_LINE) {
        boff[0] = wn * 32 + j32;
        boff[1] = 64 + wn * 32 + j32;
    } else {
        boff[0] = wn * 64 + j32;
        boff[1] = wn * 64 + 32 + j32;
    }
    if (halfn) {   // rows wm*64 + wn*32 (one row block), columns 0 .. 63 (two column blocks)
        aoff[0] = aoff[1] = wm * 64 + wn * 32 + j32;
        boff[0] = j32;
        boff[1] = 32 + j32;
    }
    floatx16 acc[3][2][2];   // [T1, T2, T3][row block][column block]
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[p][i][j][r] = 0.f;

    // GM_LINE stages of the tile-form line search: b = A B2 only over the first K2 k (B2 is zero
    // beyond), so later stages skip the B2 loads and the column-block-1 products
    constexpr bool SPLIT_K2 = MODE == GM_LINE && ROLE == 1;
    const int nk = g.K / BK;
    const int nk2 = (SPLIT_K2 && g.K2 > 0) ? g.K2 / BK : nk;
    load(0, 0 < nk2 && !halfn);
    store_lds(0, 0 < nk2 && !halfn);
    __syncthreads();
    auto stage = [&](int kt, auto full_tag) {
        constexpr bool FULL = decltype(full_tag)::value;
        constexpr int NJ = FULL ? 2 : 1;   // column blocks with products in this stage
        const int buf = kt & 1;
        if (kt + 1 < nk) load((kt + 1) * BK, kt + 1 < nk2 && !halfn);
        const float *ar = sm[buf], *ai = ar + A_PLANE;
        const float *br = ai + A_PLANE, *bi = br + B_PLANE;
        // operand fragments [A|B][re, im, re + im][block], double-buffered in registers: the
        // reads of step kc + 2 are issued between the twelve MFMAs of step kc
        float cur[2][3][2], nxt[2][3][2];
        auto frag = [&](int kc, float (&f)[2][3][2]) {
            const int ka = (kc + half) * AP, kb = (kc + half) * BP;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                f[0][0][i] = ar[ka + aoff[i]];
                f[0][1][i] = ai[ka + aoff[i]];
                f[1][0][i] = br[kb + boff[i]];
                f[1][1][i] = bi[kb + boff[i]];
            }
        };
        auto sums = [&](float (&f)[2][3][2]) {
#pragma unroll
            for (int o = 0; o < 2; ++o)
#pragma unroll
                for (int i = 0; i < 2; ++i) f[o][2][i] = f[o][0][i] + f[o][1][i];
        };
        frag(0, cur);
        sums(cur);
#pragma unroll
        for (int kc = 0; kc < BK; kc += 2) {
            if (kc + 2 < BK) frag(kc + 2, nxt);
#pragma unroll
            for (int p = 0; p < 3; ++p)
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    if (i == 1 && halfn) continue;
#pragma unroll
                    for (int j = 0; j < NJ; ++j)
                        acc[p][i][j] = __builtin_amdgcn_mfma_f32_32x32x2f32(cur[0][p][i], cur[1][p][j], acc[p][i][j], 0, 0, 0);
                }
            if (kc + 2 < BK) {
                sums(nxt);
#pragma unroll
                for (int o = 0; o < 2; ++o)
#pragma unroll
                    for (int p = 0; p < 3; ++p)
#pragma unroll
                        for (int i = 0; i < 2; ++i) cur[o][p][i] = nxt[o][p][i];
            }
        }
        if (kt + 1 < nk) store_lds(buf ^ 1, kt + 1 < nk2 && !halfn);
        __syncthreads();
    };
    int kt = 0;
    for (; kt < nk2; ++kt) stage(kt, std::true_type{});
    if constexpr (SPLIT_K2)
        for (; kt < nk; ++kt) stage(kt, std::false_type{});

    // ---- epilogue: C = (T1 - T2) + i (T3 - T1 - T2) ----
    __shared__ double red[4][5];
    float2 *C = g.C + z * g.sC + z2 * g.sC2 + z3 * g.sC3 + z4 * g.sC4;
    const int64_t ldc = g.ldc;
    auto cval = [&](int i, int j, int r) {
        const float t1 = acc[0][i][j][r], t2 = acc[1][i][j][r], t3 = acc[2][i][j][r];
        return make_float2(t1 - t2, t3 - t1 - t2);
    };
    if (MODE == GM_STORE) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                if (i == 1 && halfn) continue;
                const int col = n0 + (halfn ? 0 : wn * 64) + 32 * j + j32;
                int64_t ccol = col;
                if (ROLE != 0 && g.scat_kp > 0) {
                    if (col >= g.scat_lim) continue;
                    ccol += (int64_t)((col % g.scat_w) / g.scat_kp) * g.scat_js;
                }
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm * 64 + (halfn ? wn * 32 : 32 * i) + acc_row(r, lane);
                    C[(int64_t)row * ldc + ccol] = cval(i, j, r);
                }
            }
        return;
    }
    const float2 *E = g.E + z * g.sE + z2 * g.sE2;
    const int64_t lde = g.lde;
    double sums[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (MODE == GM_RESID) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int col = n0 + wn * 64 + 32 * j + j32;
                float blk = 0.f;
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    const int row = m0 + wm * 64 + 32 * i + acc_row(r, lane);
                    const bool in = row < g.Me && col < g.Ne;   // U has the true (unpadded) shape
                    const float2 e = in ? E[(int64_t)row * lde + col] : make_float2(0.f, 0.f);
                    const float2 c = cval(i, j, r);
                    const float2 v = make_float2(c.x - e.x, c.y - e.y);
                    C[(int64_t)row * ldc + col] = v;
                    blk = fmaf(v.x, v.x, fmaf(v.y, v.y, blk));
                }
                sums[0] += (double)blk;
                __builtin_amdgcn_sched_barrier(0);
            }
    } else {   // GM_LINE: column block 0 = a = D X1, block 1 = b = D X2 at the same (row, column)
        float2 *C2 = g.C2 + z * g.sC + z2 * g.sC2;
        const int col = n0 + wn * 32 + j32;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            float blk[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = m0 + wm * 64 + 32 * i + acc_row(r, lane);
                const float2 av = cval(i, 0, r), bv = cval(i, 1, r);
                const float2 rv = E[(int64_t)row * lde + col];
                C[(int64_t)row * ldc + col] = av;
                C2[(int64_t)row * ldc + col] = bv;
                blk[0] = fmaf(rv.x, av.x, fmaf(rv.y, av.y, blk[0]));
                blk[1] = fmaf(av.x, av.x, fmaf(av.y, av.y, blk[1]));
                blk[2] = fmaf(rv.x, bv.x, fmaf(rv.y, bv.y, blk[2]));
                blk[3] = fmaf(av.x, bv.x, fmaf(av.y, bv.y, blk[3]));
                blk[4] = fmaf(bv.x, bv.x, fmaf(bv.y, bv.y, blk[4]));
            }
#pragma unroll
            for (int q = 0; q < 5; ++q) sums[q] += (double)blk[q];
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
        const double v = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
        g.partials[z * g.sP + z2 * g.sP2 + (int64_t)pid * NS + t] = v;
    }
}

}  // namespace

hipError_t launch_cgemm3m(int mode, const GemmArgs &a0, int batch, hipStream_t s, int role) {
    const bool tile_stage = role != GR_DENSE;
    if (role < GR_DENSE || role > GR_TILE_TA_CB || (role == GR_TILE_TA_CB && mode != GM_STORE))
        return hipErrorInvalidValue;
    GemmArgs a = a0;
    a.tiles_m = a.M / BM;
    // GM_STORE tile stages take N a multiple of 64: the whole 128-column tiles in one launch, a last
    // column tile of 64 in a second one; all else whole tiles
    const bool half_ok = mode == GM_STORE && tile_stage;
    a.tiles_n = (mode == GM_LINE) ? a.N / (BN / 2) : a.N / BN;
    if (a.M <= 0 || a.N <= 0 || batch <= 0) return hipSuccess;
    if (a.M % BM || a.N % (half_ok ? BN / 2 : BN) || a.K % BK || a.K <= 0) return hipErrorInvalidValue;
    const bool half_tile = half_ok && a.N % BN != 0;
    a.n_half = half_tile ? a.tiles_n * BN : 0;
    if (a.K2 < 0 || a.K2 > a.K || a.K2 % BK || (a.K2 && !(mode == GM_LINE && tile_stage)))
        return hipErrorInvalidValue;
    if (a.nz3 > 1 || a.nz4 > 1) {
        const int64_t inner = (int64_t)std::max(1, a.nz3) * std::max(1, a.nz4);
        if (!(mode == GM_STORE && tile_stage && a.nz2 > 1 && a.nz2 % inner == 0)) return hipErrorInvalidValue;
    }
    if (a.scat_kp < 0 || (a.scat_kp && (!(mode == GM_STORE && tile_stage) || a.scat_w < a.scat_kp ||
                                        a.scat_lim <= 0 || a.scat_lim > a.N)))
        return hipErrorInvalidValue;
    // byte extents of the buffer resources (32-bit): A is M x lda (transposed source: K x lda), B is
    // K x ldb (GM_LINE: B2 follows B)
    const int64_t bytesA = (int64_t)(role == GR_TILE_TA_CB ? a.K : a.M) * a.lda * 8;
    if (role == GR_TILE_TA_CB && a.lda < a.M) return hipErrorInvalidValue;
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
    if (half_tile) {
        GemmArgs h = a;
        h.tiles_n = 1;
        const dim3 hgrid(a.tiles_m, batch);
        if (role == GR_TILE_TA_CB) hipLaunchKernelGGL((cgemm3m_kernel<GM_STORE, 2, true>), hgrid, dim3(256), 0, s, h);
        else hipLaunchKernelGGL((cgemm3m_kernel<GM_STORE, 1, true>), hgrid, dim3(256), 0, s, h);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess || a.tiles_n == 0) return e;
    }
    switch (mode) {
        case GM_STORE:
            if (role == GR_TILE_TA_CB) hipLaunchKernelGGL((cgemm3m_kernel<GM_STORE, 2>), grid, dim3(256), 0, s, a);
            else if (tile_stage) hipLaunchKernelGGL((cgemm3m_kernel<GM_STORE, 1>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((cgemm3m_kernel<GM_STORE, 0>), grid, dim3(256), 0, s, a);
            break;
        case GM_RESID:
            if (tile_stage) hipLaunchKernelGGL((cgemm3m_kernel<GM_RESID, 1>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((cgemm3m_kernel<GM_RESID, 0>), grid, dim3(256), 0, s, a);
            break;
        case GM_LINE:
            if (tile_stage) hipLaunchKernelGGL((cgemm3m_kernel<GM_LINE, 1>), grid, dim3(256), 0, s, a);
            else hipLaunchKernelGGL((cgemm3m_kernel<GM_LINE, 0>), grid, dim3(256), 0, s, a);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tlr
