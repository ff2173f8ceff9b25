// Internal declarations shared by the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>

namespace tlr {

// records `msg` as the calling thread's last error (tlrmdd_last_error) and returns `status`
int set_error(int status, const std::string &msg);

// ---- tile tables (Tile Low-rank MDD section: diagonal Q Q^T / P Z, sub-diagonal L R) ----
enum TileKind : int32_t { TILE_LR = 0, TILE_QQ = 1, TILE_DENSE = 2 };

struct TileDesc {
    int32_t kind;   // TileKind
    int32_t di;     // rows of the tile (tile i)
    int32_t dj;     // cols of the tile (tile j); == di on the diagonal
    int32_t k;      // rank (LR: k_ij, QQ: k_ii, DENSE: d_i)
    int64_t row0;   // first row of the tile in X
    int64_t col0;   // first col of the tile in X
    int64_t offA;   // theta offset of L_ij / Q_ii / Z_ii
    int64_t offB;   // theta offset of R_ij (LR only)
};

// Per-problem offsets (a batch of frequencies shares one launch per phase).
struct ProbOff {
    int64_t theta;  // offset (complex elements) of this problem's theta / p / g vectors
    int64_t x;      // offset of its X / X1 / X2 / W matrices
    int64_t ldx;    // leading dimension (complex) of those matrices
    int64_t pad;
};

// Assembly work item: one 64 x 64 block of a tile (rows r0.., cols c0.. inside the tile).
struct AsmItem {
    int32_t tile;   // index into the tile table
    int32_t r0;
    int32_t c0;
    int32_t prob;   // index into the ProbOff table
};
constexpr int ASM_B = 64;    // assembly block edge (rows and columns of a tile block)
constexpr int ASM_KC = 16;   // rank entries staged per step

// Gradient work item.
enum GradKind : int32_t { G_L = 0, G_Q = 1, G_R = 2, G_Z = 3 };
struct GradItem {
    int32_t tile;
    int32_t kind;   // GradKind
    int32_t a0;     // G_L/G_Q: first row; G_R: first col; G_Z: first row
    int32_t b0;     // G_L/G_Q/G_R: first rank index; G_Z: first col
    int32_t prob;
    int32_t kq;     // G_L/G_Q/G_R: rank entries in the item, in units of 16 (1..4)
};
constexpr int GR_ROWS = 64;   // rows (G_L/G_Q) or cols (G_R) per item
constexpr int GR_KK = 64;     // rank entries per item (at most)
constexpr int GR_CH = 4;      // contraction chunk (small: many workgroups per CU hide the W loads)
constexpr int GZ_BR = 32, GZ_BC = 64;

// ---- complex GEMM on MFMA ----
enum GemmMode : int32_t { GM_STORE = 0, GM_RESID = 1, GM_LINE = 2 };

struct GemmArgs {
    const float2 *A;  int64_t lda;   // M x K complex, row-major
    const float2 *B;  int64_t ldb;   // K x N complex, row-major
    const float2 *B2;                // GM_LINE: second B (same ldb)
    float2 *C;        int64_t ldc;   // M x N output
    float2 *C2;                      // GM_LINE: second output (same ldc)
    const float2 *E;  int64_t lde;   // GM_RESID: U (C = AB - U); GM_LINE: residual r
    double *partials;                // per-workgroup FP64 sums (GM_RESID: 1, GM_LINE: 5)
    int32_t M, N, K;                 // padded sizes: M, N multiples of 128, K of 16 (zero padding)
    int32_t Me, Ne;                  // GM_RESID: true shape of E (reads outside are zero)
    int64_t b2_off;                  // GM_LINE: B2 - B in complex elements (set by the launcher)
    uint32_t bytesA, bytesB;         // buffer extents (set by the launcher)
    int32_t tiles_m, tiles_n;
    // uniform batch (grid.y): element strides between problems
    int64_t sA, sB, sC, sE;
    int64_t sP;                      // partial stride (doubles) between problems
    // two-level batch (three-product kernel): grid.y = nz * nz2, entry z = z1 * nz2 + z2 is at
    // z1 * s + z2 * s2 for every operand (nz2 <= 1: one level, the s2 are unused)
    int32_t nz2;
    int32_t K2;                      // GM_LINE: b = A B2 sums over k < K2 only (0: all K; a multiple of 16)
    int64_t sA2, sB2, sC2, sE2, sP2;
    // further levels (GM_STORE tile stages): the second-level index first splits into (z2 / nz4,
    // z4 = z2 mod nz4) when nz4 > 1 (strides s4: operand sets of one launch, s4 may be the distance
    // between two buffers), then into (z2 / nz3, z3 = z2 mod nz3) when nz3 > 1 (strides s3); nz2
    // counts all of them (grid.y = nz * nz2)
    int32_t nz3, nz4;
    int64_t sA3, sB3, sC3, sA4, sB4, sC4;
    // GM_STORE tile stages: output column n < scat_lim is stored at column
    // n + ((n mod scat_w) / scat_kp) * scat_js, columns from scat_lim on are dropped (scat_kp = 0:
    // plain), which regroups blocks of scat_kp columns across batch entries
    int32_t scat_kp, scat_w, scat_lim;
    int64_t scat_js;
    int32_t n_half;                  // GM_STORE tile stages: first column of a last 64-column tile (set by the launcher)
};
// roles of the three-product kernel: the solver's dense products; the tile-form stages; the same
// with A given transposed (K x M source, row pitch lda) and B conjugated
enum GemmRole : int32_t { GR_DENSE = 0, GR_TILE = 1, GR_TILE_TA_CB = 2 };
constexpr int GEMM_BM = 128;
constexpr int GEMM_BN = 128;   // complex columns per workgroup (64 of a + 64 of b in GM_LINE)
constexpr int GEMM_BK = 16;    // complex k per stage
constexpr int GEMM_PAD = 128;  // internal matrices are padded to multiples of this

// BF16 hi+lo split: hi = bf16(x) (round to nearest even), lo = bf16(x - hi)
__device__ __forceinline__ uint32_t bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;   // NaN stays NaN
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ void split_c(float2 v, uint32_t &hi, uint32_t &lo) {
    const uint32_t hr = bf16_rne(v.x), hi_ = bf16_rne(v.y);
    const uint32_t lr = bf16_rne(v.x - __uint_as_float(hr << 16));
    const uint32_t li = bf16_rne(v.y - __uint_as_float(hi_ << 16));
    hi = hr | (hi_ << 16);
    lo = lr | (li << 16);
}

// BF16 hi+lo split operands: planes of interleaved complex BF16 (one uint32 per complex).
struct GemmArgsB {
    const uint16_t *Ahi, *Alo;  int64_t lda;   // M x K complex (row-major planes)
    const uint16_t *Bhi, *Blo;  int64_t ldb;   // B TRANSPOSED: N x K complex planes
    int64_t b2_rows;                           // GM_LINE: B2's rows start this many rows after B's
    float2 *C;        int64_t ldc;
    float2 *C2;
    const float2 *E;  int64_t lde;
    double *partials;
    int32_t M, N, K, Me, Ne;
    int32_t tiles_m, tiles_n;
    int64_t sA, sB, sC, sE, sP;                // batch strides (complex elements / doubles)
    uint32_t bytesA, bytesB;                   // set by the launcher
};
hipError_t launch_cgemm_bf16(int mode, const GemmArgsB &a, int batch, hipStream_t s);

// ---- vector / scalar kernels ----
constexpr int RED_THREADS = 256;
constexpr int MAX_LBFGS_M = 32;

struct SolveScalars {
    double f;
    double fdata;                // 1/2 ||r||^2 of the tracked residual (no penalty)
    double sy, yy, gamma;
    double gp;
    double coef[4];
    double step;
    double pnorm2, tp;           // lambda terms: ||p||^2, Re<theta,p>
    double thnorm2;              // ||theta||^2 after update (lambda term of f)
    double rho[MAX_LBFGS_M + 1];
    double alpha[MAX_LBFGS_M];
    int32_t head, count, restart, frozen;
};

// host launchers (stream ordered)
hipError_t launch_cgemm(int mode, const GemmArgs &a, int batch, hipStream_t s);
// the same products in the three-real-product form (FP32 MFMA, interleaved complex64 operands)
hipError_t launch_cgemm3m(int mode, const GemmArgs &a, int batch, hipStream_t s, int role = GR_DENSE);
int gemm_partials_per_problem(int mode, int M, int N);

// out_bf16 == false: X / X2 are complex64 matrices (ProbOff.x offsets, ld ProbOff.ldx).
// out_bf16 == true: the same region holds split planes of uint32 words; a problem's
// X hi plane starts at word 2 * ProbOff.x, X2 hi at + x2_words, each lo plane at + lo_words.
hipError_t launch_assemble(bool dir, const TileDesc *tiles, const AsmItem *items, int nitems,
                           const ProbOff *probs, const float2 *theta, const float2 *p,
                           float2 *X, float2 *X2, hipStream_t s, bool out_bf16 = false,
                           int64_t x2_words = 0, int64_t lo_words = 0);
hipError_t launch_grad(const TileDesc *tiles, const GradItem *items, int nitems,
                       const ProbOff *probs, const float2 *W, const float2 *theta, float2 *g,
                       hipStream_t s);

hipError_t launch_stage_d(const float2 *D, int64_t ns, int64_t nr, float2 *Ds, int64_t ldk,
                          float2 *DHs, int64_t lds, hipStream_t s);
// split staging: Dhi/Dlo (lds x ldk planes) and DHhi/DHlo (ldk x lds planes, conjugate transpose)
hipError_t launch_stage_d_split(const float2 *D, int64_t ns, int64_t nr, uint32_t *Dh, uint32_t *Dl, int64_t ldk,
                                uint32_t *DHh, uint32_t *DHl, int64_t lds, hipStream_t s);
// rT = r^T split into planes: r is rows x cols (ld ldr), rT planes are cols x rows (ld ldt)
hipError_t launch_split_transpose(const float2 *r, int64_t ldr, int64_t rows, int64_t cols, uint32_t *th,
                                  uint32_t *tl, int64_t ldt, int batch, int64_t s_r, int64_t s_t, hipStream_t s);
// zero the padding of nplanes ld x ld uint32 planes (true size n x n), per problem of a batch
hipError_t launch_zero_pad(uint32_t *base, int64_t ld, int64_t n, int nplanes, int64_t plane_stride, int batch,
                           int64_t batch_stride, hipStream_t s);
hipError_t launch_copy2d(const float2 *src, int64_t lds, float2 *dst, int64_t ldd,
                         int64_t rows, int64_t cols, hipStream_t s);
// bad: device int32 or NULL, set to 1 when a perm entry lies outside [0, cols) (its column is zeroed)
hipError_t launch_permute_cols(const float2 *in, const int64_t *perm, float2 *out,
                               int64_t rows, int64_t cols, int32_t *bad, hipStream_t s);
// zero `bytes` (a multiple of 4, 4-byte aligned) at p with a kernel (no memset node in captured graphs)
hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s);

}  // namespace tlr
