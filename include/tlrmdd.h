/*
 * tlrmdd.h - C ABI of the MI355X (gfx950) tile low-rank multidimensional
 * deconvolution (TLR-MDD) library.
 *
 * Method: Chen, Ravasi, Keyes, "Reciprocity-aware adaptive tile low-rank
 * factorization for large-scale 3D multidimensional deconvolution"
 * (arXiv 2412.14973). For one frequency the library evaluates
 *     f(theta) = 1/2 || D C(theta) - U ||_F^2            (ADMM solver, eq. X2LQR_lst)
 * and its gradient with respect to every tile factor (ADMM solver, eqs. DXLR),
 * where X = C(theta) is the complex-symmetric Green's function assembled from
 * tiles (Tile Low-rank MDD section):
 *     X_ii = Q_ii Q_ii^T  (low-rank diagonal)  or  X_ii = (Z_ii + Z_ii^T)/2  (dense),
 *     X_ij = L_ij R_ij  (i > j),   X_ji = X_ij^T.
 * Columns of D and U are expected in Hilbert order (Receivers re-ordering
 * section, eq. axb_sd); hilbert_order() and tlrmdd_permute_columns() produce it.
 *
 * Conventions shared by every entry point
 *  - Complex data is complex64 interleaved (re, im float pairs), row-major and
 *    contiguous: D and U are ns x nr, X is nr x nr, theta is a flat vector.
 *  - "device" pointers are HIP device memory; "host" pointers are host memory.
 *    The caller owns every buffer; the library never frees caller memory and
 *    keeps no pointer to it after the call returns (work is stream ordered).
 *  - Device calls enqueue work on `stream` and return without synchronising;
 *    scalar results are written to device FP64 memory (synchronise the stream
 *    before reading them on the host).
 *  - No C++ exception crosses the ABI. Every int-returning call returns one of
 *    the TLRMDD_* status codes; tlrmdd_last_error() gives a thread-local
 *    message for the most recent failure on the calling thread.
 *  - Gradient convention: grad = df/dRe(theta) + i df/dIm(theta)
 *    (= 2 df/d conj(theta)); with W = D^H (D X - U) this is the convention in
 *    which the paper writes grad L = W' R^H, grad R = L^H W', grad Q = W' conj(Q),
 *    grad Z = W'/2 with W' = W + W^T.
 *
 * theta packing (stacks Zbar, Lbar, Rbar of the Tile Low-rank MDD section):
 *   all diagonal blocks in tile order (Q_ii: d_i x k_ii, or Z_ii: d_i x d_i),
 *   then every L_t (d_i x k_t), then every R_t (k_t x d_j), each row-major,
 *   with sub-diagonal tiles (i > j) numbered t = i(i-1)/2 + j (0-based).
 */
#ifndef TLRMDD_H
#define TLRMDD_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define TLRMDD_OK               0
#define TLRMDD_INVALID_ARGUMENT 1  /* bad pointer, size, layout or option        */
#define TLRMDD_WORKSPACE        2  /* workspace too small / allocation failed    */
#define TLRMDD_HIP_ERROR        3  /* a HIP runtime call failed                  */
#define TLRMDD_NONFINITE        4  /* non-finite value met (solve)               */
#define TLRMDD_UNSUPPORTED      5  /* e.g. unknown precision                     */
#define TLRMDD_NOT_CONVERGED    6  /* per-tile Jacobi SVD still rotating after its
                                      sweep limit (outputs not written)          */

/* ---- precisions of the bulk complex products ------------------------------ */
#define TLRMDD_FP32      0  /* FP32 MFMA, complex as a real 2x2 block (4 real products) */
#define TLRMDD_BF16X3    1  /* BF16 hi+lo split (hi*hi + hi*lo + lo*hi), FP32 accumulate */
#define TLRMDD_FP32_3M   2  /* FP32 MFMA, three real products per complex product (3M form):
                               Re = ArBr - AiBi, Im = (Ar+Ai)(Br+Bi) - ArBr - AiBi; 3/4 of the flops */

/* ---- optimisers ------------------------------------------------------------ */
#define TLRMDD_LBFGS 0
#define TLRMDD_GD    1

/* Tile layout of one frequency (Tile Low-rank MDD section).
 * tile_size: host, ntiles entries d_i >= 1 with sum d_i == nr (a ragged last
 *            tile is allowed; the paper notes equal sizes are not required).
 * rank_off:  host, ntiles(ntiles-1)/2 entries, k_t for tile (i, j), i > j,
 *            t = i(i-1)/2 + j, 1 <= k_t <= min(d_i, d_j).
 * rank_diag: host, ntiles entries: k_ii in [1, d_i] -> Q_ii Q_ii^T, or -1 ->
 *            dense symmetrised Z_ii.
 * ns:        number of sources (rows of D and U). */
typedef struct {
    int64_t nr;
    int64_t ns;
    int32_t ntiles;
    const int32_t *tile_size;
    const int32_t *rank_off;
    const int32_t *rank_diag;
} tlrmdd_layout;

/* Options of tlrmdd_solve (ADMM solver section: the X-update uses limited-
 * memory BFGS; here with an exact line search on the quartic f(theta+a p)). */
typedef struct {
    int32_t iters;          /* fixed iteration count T >= 0                        */
    int32_t optimizer;      /* TLRMDD_LBFGS or TLRMDD_GD                           */
    int32_t lbfgs_m;        /* L-BFGS memory, 1..32 (default 5)                     */
    int32_t precision;      /* TLRMDD_FP32, TLRMDD_BF16X3 or TLRMDD_FP32_3M           */
    double  lambda;         /* Frobenius regulariser lambda ||theta||^2 (0 = none)  */
    int32_t resid_refresh;  /* recompute r = D C(theta) - U every this many iters (0 = never); the
                               tracked r accumulates FP32 rounding, 20 keeps long solves oracle-close */
    int32_t streams;        /* batched calls: 0 or 1 = all problems in one launch per phase on
                               `stream` (with one library-owned side stream on which the tile-form
                               gradient runs beside the adjoint product of the other problems, and
                               every other tile-form line-search range beside the rest);
                               2..8 = problem i in sub-batch i % streams, each sub-batch on its own
                               stream (the first on `stream`, the others on streams the library
                               creates at default priority for each (device, caller stream) pair
                               and keeps until the process ends, forked from and joined to
                               `stream` with events owned by the call), so the matrix-core
                               products of one sub-batch overlap the HBM-bound passes of another.
                               Results are bit-identical for every value; single-problem calls
                               ignore it. */
    int32_t line_products;  /* TLRMDD_LINE_DENSE (0): the line search's [a | b] = D [X1 | X2] from
                               the assembled X1, X2; TLRMDD_LINE_TILE (1): in tile form wherever that
                               needs fewer flops (precisions TLRMDD_FP32_3M and TLRMDD_BF16X3; see
                               tlrmdd_line_form for the bounds); batched calls still run
                               every phase as one launch per sub-batch, except the line-search
                               products: one launch for the dense-form problems and the tile-form
                               stages once per (tile size, padded rank) class;
                               TLRMDD_LINE_TILE_GRAD (2): as 1, and the gradient in tile form too
                               where its three products (3 Wg / nr of the adjoint product D^H r,
                               Wg = nt kpad rounded up to 64) cost at most 0.6 of the adjoint
                               (0.3 in BF16X3 mode):
                               W_ij B_ij^H = D_:,i^H (r_:,j B_ij^H), A_ij^H W_ij = (D_:,i A_ij)^H r_:,j
                               with X_ij = A_ij B_ij (gradient equations); the adjoint product then
                               runs on the other problems only */
    int32_t reserved;       /* 0 */
} tlrmdd_opts;

#define TLRMDD_LINE_DENSE 0
#define TLRMDD_LINE_TILE  1
#define TLRMDD_LINE_TILE_GRAD 2

/* Opaque plan: validated layout plus device-side tile tables. The calls take a
 * plan instead of the layout itself so that the tile tables of a frequency are
 * built and uploaded once (at plan creation) and not on every call. */
typedef struct tlrmdd_plan_s *tlrmdd_plan;

/* Message for a status code (static storage). */
const char *tlrmdd_status_string(int status);
/* Thread-local detail for the last failing call on this thread ("" if none). */
const char *tlrmdd_last_error(void);

/* Number of complex unknowns in theta for `layout`; < 0 if the layout is
 * invalid (same checks as tlrmdd_plan_create). Host only. */
int64_t tlrmdd_theta_size(const tlrmdd_layout *layout);

/* Validate `layout` and build a plan on the current HIP device: host tables
 * plus a small device allocation holding the tile tables (freed by
 * tlrmdd_plan_destroy). Status 1 on any of: null pointer, nr/ns/ntiles <= 0,
 * sum d_i != nr, off-diagonal rank outside [1, min(d_i, d_j)], diagonal rank
 * neither -1 nor in [1, d_i]. */
int tlrmdd_plan_create(const tlrmdd_layout *layout, tlrmdd_plan *plan_out);
int tlrmdd_plan_destroy(tlrmdd_plan plan);

/* Workspace (device bytes) needed by an operation on this plan.
 * op: 0 = forward, 1 = grad, 2 = solve (opts required for solve, may be NULL
 * otherwise). The workspace need not be zeroed and is reused by the library
 * as scratch; it may be shared between calls that do not overlap in time. */
#define TLRMDD_OP_FORWARD 0
#define TLRMDD_OP_GRAD    1
#define TLRMDD_OP_SOLVE   2
int tlrmdd_workspace_bytes(tlrmdd_plan plan, int op, const tlrmdd_opts *opts, size_t *bytes);

/* Objective (eq. X2LQR_lst): f = 1/2 || D C(theta) - U ||_F^2.
 * D, U:    device, ns x nr complex64 (Hilbert column order).
 * theta:   device, tlrmdd_theta_size complex64.
 * f_dev:   device, one double (accumulated in FP64 from FP32 residuals).
 * r_out:   device or NULL; receives r = D X - U (ns x nr complex64).
 * X_out:   device or NULL; receives X = C(theta) (nr x nr complex64, exactly
 *          symmetric bit for bit).
 * precision: TLRMDD_FP32, TLRMDD_BF16X3 or TLRMDD_FP32_3M. */
int tlrmdd_forward(tlrmdd_plan plan, const void *D, const void *U, const void *theta,
                   double *f_dev, void *r_out, void *X_out, int precision,
                   void *workspace, size_t ws_bytes, hipStream_t stream);

/* Objective and gradient (eqs. DXLR): W = D^H r, W' = W + W^T,
 * grad L_ij = W'_ij R_ij^H, grad R_ij = L_ij^H W'_ij, grad Q_ii = W'_ii conj(Q_ii),
 * grad Z_ii = W'_ii / 2. The assembled X is recomputed here, never read from
 * a previous call. grad_out: device, packed like theta. f_dev may be NULL. */
int tlrmdd_grad(tlrmdd_plan plan, const void *D, const void *U, const void *theta,
                double *f_dev, void *grad_out, int precision,
                void *workspace, size_t ws_bytes, hipStream_t stream);

/* tlrmdd_grad without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the scratch lives in a fixed device array of the
 * library, TLRMDD_NOALLOC_SCRATCH_MIB MiB per GPU, held from the first call on
 * a GPU until the process ends. The call allocates nothing (no hipMalloc, no
 * hipFree, no host-pinned memory); the caller passes inputs and outputs as for
 * tlrmdd_grad and still creates the plan beforehand. Returns TLRMDD_WORKSPACE
 * when tlrmdd_workspace_bytes(plan, TLRMDD_OP_GRAD) exceeds the array (e.g.
 * nr = ns = 1024 needs about 40 MiB and fits). Every call on one GPU shares that
 * GPU's array: calls that overlap in time on one GPU (different streams, or
 * threads) race and give wrong results; calls ordered on one stream are safe. */
#define TLRMDD_NOALLOC_SCRATCH_MIB 64
int tlrmdd_grad_noalloc(tlrmdd_plan plan, const void *D, const void *U, const void *theta,
                        double *f_dev, void *grad_out, int precision, hipStream_t stream);

/* Fixed-count solve of min f(theta) (+ lambda ||theta||^2) from theta_inout
 * (overwritten with theta_T). Each iteration: gradient from the tracked
 * residual, L-BFGS two-loop direction (real inner product Re<a,b>, pairs
 * kept only when Re<s,y> > 0, steepest-descent restart when Re<g,p> >= 0),
 * exact line search along the quartic phi(a) = f(theta + a p) using
 * a = D C1(theta;p), b = D C2(p) (one product D [X1 | X2]), then
 * theta += a* p and r += a* a + a*^2 b. All scalars stay on the device in
 * FP64; the host only enqueues work.
 * f_hist_dev: device, iters+1 doubles: f_hist[t] = tracked objective after t
 * iterations. Returns TLRMDD_OK once everything is enqueued; a non-finite
 * step length freezes theta for the remaining iterations (f_hist repeats). */
int tlrmdd_solve(tlrmdd_plan plan, const void *D, const void *U, void *theta_inout,
                 const tlrmdd_opts *opts, double *f_hist_dev,
                 void *workspace, size_t ws_bytes, hipStream_t stream);

/* Form of the exact line search's (and gradient's) products for this plan
 * under opts (tlrmdd_solve and the batched / ADMM calls): *tile_form = 1
 * when opts->line_products is TLRMDD_LINE_TILE or TLRMDD_LINE_TILE_GRAD, the
 * precision is TLRMDD_FP32_3M or TLRMDD_BF16X3 (the tile-form products run on
 * the three-product FP32 kernel in both; the dense ones keep the precision's
 * kernels) and the layout qualifies - all tiles of one
 * size d (a multiple of 128), nr a multiple of 128, Q Q^T diagonal tiles -
 * with 2.5 kpad / d <= 0.6, where kpad is the largest rank rounded up so
 * that a stage-1 row of 2 nt blocks of kpad columns is a whole number of
 * 128-column tiles (2.5 kpad / d: the tile form's share of the dense
 * products' flops; the paper's Discussion section names the TLR product as
 * the way to cut the cost of the dense products); 2 when the gradient is in tile form
 * as well (TLRMDD_LINE_TILE_GRAD and 3 Wg / nr <= 0.6). In TLRMDD_BF16X3 mode
 * both bounds are 0.3: the BF16 dense products they replace run about twice
 * as fast. In a batched call a
 * problem whose gradient would be in tile form keeps the dense gradient when
 * a problem of another form follows it in the call's order (the library
 * orders problems by form itself). *kpad (may be NULL) gets the padded rank,
 * 0 for the dense form. */
int tlrmdd_line_form(tlrmdd_plan plan, const tlrmdd_opts *opts, int *tile_form, int *kpad);

/* Batched solve of independent frequencies (the paper solves each frequency
 * independently, Theory section, eq. standard_solver). Arrays have `count`
 * entries; every problem uses the same opts. Work of all problems (of each
 * sub-batch when opts->streams > 1) is fused into shared launches per phase.
 * workspace: sized by tlrmdd_workspace_bytes_batched with the same opts. */
int tlrmdd_workspace_bytes_batched(int count, const tlrmdd_plan *plans,
                                   const tlrmdd_opts *opts, size_t *bytes);
int tlrmdd_solve_batched(int count, const tlrmdd_plan *plans, const void *const *D,
                         const void *const *U, void *const *theta_inout,
                         const tlrmdd_opts *opts, double *const *f_hist_dev,
                         void *workspace, size_t ws_bytes, hipStream_t stream);

/* ADMM with lambda continuation (ADMM solver section: X-update, Z-update
 * eq. proxofFro2, dual update; hyper-parameter selection: lambda stages
 * 10 -> 1 -> 0.1). The problem is min f(theta) + lambda ||theta||^2 on the
 * factors, split as theta = z with the scaled dual u (u <- u + theta - z; the
 * paper prints the unscaled dual step, the scaled form keeps its X-update
 * consistent). Starting from z = theta_in, u = 0, for every stage and every
 * outer step:
 *   X-update: inner.iters iterations of the solver above on
 *             f(theta) + rho/2 ||theta - z + u||^2 from the current theta
 *             (fresh L-BFGS memory, tracked residual carried over);
 *   Z-update: z = (theta + u) / (1 + 2 lambda / rho);
 *   dual:     u = u + theta - z.
 * theta_inout receives the X-variable. f_hist_dev: device, 1 + nstages *
 * outer doubles per problem: the data misfit 1/2||D C(theta) - U||^2 of the
 * tracked residual at the start and after every X-update. inner.lambda and
 * inner.resid_refresh are ignored / used as in tlrmdd_solve; inner.streams
 * splits batched calls into sub-batches on their own streams as in
 * tlrmdd_solve_batched (same results). */
typedef struct {
    tlrmdd_opts inner;       /* X-update: iters per update, optimizer, lbfgs_m, precision */
    int32_t nstages;         /* number of lambda stages, >= 1                               */
    int32_t outer;           /* ADMM steps per stage, >= 0                                  */
    const double *lambdas;   /* host, nstages values >= 0                                   */
    double rho;              /* ADMM penalty, > 0                                           */
} tlrmdd_admm_opts;

int tlrmdd_workspace_bytes_admm(int count, const tlrmdd_plan *plans, const tlrmdd_admm_opts *opts,
                                size_t *bytes);
int tlrmdd_admm(tlrmdd_plan plan, const void *D, const void *U, void *theta_inout,
                const tlrmdd_admm_opts *opts, double *f_hist_dev,
                void *workspace, size_t ws_bytes, hipStream_t stream);
int tlrmdd_admm_batched(int count, const tlrmdd_plan *plans, const void *const *D,
                        const void *const *U, void *const *theta_inout,
                        const tlrmdd_admm_opts *opts, double *const *f_hist_dev,
                        void *workspace, size_t ws_bytes, hipStream_t stream);

/* Tile low-rank product (Discussion section: the TLR matrix-matrix product as the way to cut
 * the dense products' cost): f = 1/2 ||D C(theta) - U||^2 without forming X. With every tile
 * X_ij = A_ij B_ij (i > j: L_ij R_ij; i < j: R_ji^T L_ji^T; Q Q^T; dense: I and (Z+Z^T)/2),
 * P_i = D_:,i [A_i0 | A_i1 | ...] per tile row, then r_:,j = sum_i P_ij B_ij - U_:,j per tile
 * column: 16 ns sum_ij d_i k_ij flops instead of 8 ns nr^2 (about 2k/d of the dense product).
 * FP32 MFMA. D, U: device ns x nr complex64; theta: device theta_size complex64; f_dev:
 * device double; r_out: device ns x nr complex64 or NULL. Stream ordered (the packing tables
 * go through a library-owned pinned buffer). Workspace: tlrmdd_workspace_bytes_tlr. */
int tlrmdd_workspace_bytes_tlr(tlrmdd_plan plan, size_t *bytes);
int tlrmdd_forward_tlr(tlrmdd_plan plan, const void *D, const void *U, const void *theta,
                       double *f_dev, void *r_out, void *workspace, size_t ws_bytes,
                       hipStream_t stream);

/* ---- rank / tile-size estimate and warm start --------------------------
 * (Hyper-parameter selection and initialization; the examples' rank study.)
 * X is a reference solution: device, nr x nr complex64, symmetric, in the
 * receiver order of the solve (Hilbert). Tiles of size d cover nr with a
 * ragged last tile. Every tile X_ij, i >= j, is decomposed in FP64 on the GPU
 * by one-sided Jacobi (round-robin pairs, sweeps until no pair is rotated,
 * at most 30). Tile sizes up to 1024.
 *
 * tlrmdd_tile_ranks: v0 = largest singular value over all tiles; the rank of a
 * tile is the number of its singular values >= eps * v0 (0 possible; all of
 * them = numerically full rank). k_off_out: host, N(N-1)/2 entries in t order
 * (t = i(i-1)/2 + j); k_diag_out: host, N entries; v0_out: host (nullable).
 * Synchronises `stream` (host outputs). Workspace: tlrmdd_workspace_bytes_ranks.
 *
 * tlrmdd_choose_layout: for every candidate tile size the estimated layout
 * (ranks at least 1; a diagonal tile dense, rank_diag = -1, when its rank is
 * at least half its size, else Q Q^T) and its entry count (complex unknowns:
 * sum k_t (d_i + d_j) + sum of d_i^2 or d_i k_ii) into entries_out[c] (host,
 * nullable); the candidate with the fewest entries (first on ties) is written
 * to d_out, rank_off_out (capacity off_capacity) and rank_diag_out (capacity
 * diag_capacity); status 1 when a chosen layout does not fit. Workspace: the
 * largest candidate's tlrmdd_workspace_bytes_ranks. Synchronises `stream`.
 *
 * tlrmdd_warm_start: theta_out (device, theta_size complex64 of the plan's
 * layout) from X: L = U_k S_k^(1/2), R = S_k^(1/2) V_k^H of every off-diagonal
 * tile (truncated SVD, k = the layout's rank), Q = U_k D^(1/2) S_k^(1/2) of
 * every Q Q^T tile (Takagi factorisation from the SVD of the symmetric tile,
 * d_c = u_c^H conj(v_c); eq. qqinit), Z_ii = X_ii for dense tiles.
 * Synchronises `stream` (the sweep count is decided on the host).
 * Workspace: tlrmdd_workspace_bytes_warm. */
int tlrmdd_workspace_bytes_ranks(int64_t nr, int32_t d, size_t *bytes);
int tlrmdd_tile_ranks(const void *X, int64_t nr, int32_t d, double eps, int32_t *k_off_out,
                      int32_t *k_diag_out, double *v0_out, void *workspace, size_t ws_bytes,
                      hipStream_t stream);
int tlrmdd_choose_layout(const void *X, int64_t nr, const int32_t *candidates, int32_t ncand,
                         double eps, int32_t *d_out, int64_t *entries_out,
                         int32_t *rank_off_out, int64_t off_capacity,
                         int32_t *rank_diag_out, int64_t diag_capacity,
                         void *workspace, size_t ws_bytes, hipStream_t stream);
int tlrmdd_workspace_bytes_warm(tlrmdd_plan plan, size_t *bytes);
int tlrmdd_warm_start(tlrmdd_plan plan, const void *X, void *theta_out, void *workspace,
                      size_t ws_bytes, hipStream_t stream);

/* Adjoint (cross-correlation) solution X_adj = D^H U (MDD Solver Evaluation section: the
 * adjoint solution that needs no inversion). D, U: device ns x nr complex64; X_out: device
 * nr x nr complex64. Uses the plan's sizes only (its tiles are ignored). Workspace: as for
 * TLRMDD_OP_GRAD. */
int tlrmdd_adjoint(tlrmdd_plan plan, const void *D, const void *U, void *X_out, int precision,
                   void *workspace, size_t ws_bytes, hipStream_t stream);

/* Hilbert ordering of receivers (Receivers re-ordering section, eq. hilbert).
 * ix, iy: host, n non-negative 0-based grid coordinates (x = station along a
 * line, y = line). perm_out: host, n entries: perm_out[k] is the natural
 * index (input position) of the k-th receiver along the Hilbert curve on the
 * smallest 2^m x 2^m grid enclosing all points (start (0,0), end (2^m-1,0));
 * equal cells keep input order. Status 1 on NULL pointers with n > 0,
 * n < 0 or negative coordinates. Host only, no GPU needed. */
int hilbert_order(const int32_t *ix, const int32_t *iy, int64_t n, int64_t *perm_out);

/* Column gather Dhat = D S (eq. axb_sd): out[s, k] = in[s, perm[k]].
 * in, out: device, rows x cols complex64 (must not overlap);
 * perm: device int64, cols entries, each expected in [0, cols). The device
 * entries are checked in the kernel: an entry outside [0, cols) writes a zero
 * column k and sets *bad_dev to 1 (bad_dev: device int32 or NULL; the library
 * only ever writes 1 into it, so the caller clears it before the call). The
 * call is stream ordered: read *bad_dev after synchronising the stream. */
int tlrmdd_permute_columns(const void *in, const int64_t *perm, void *out,
                           int64_t rows, int64_t cols, int32_t *bad_dev, hipStream_t stream);

/* ---- kernel timing (instrumentation) -------------------------------------
 * Between tlrmdd_timing_begin() and tlrmdd_timing_end(), every launch of the
 * kernel kinds below made by this library (any thread, any stream) is
 * bracketed by two HIP events recorded on its own stream, and its algorithmic
 * work is counted on the true (unpadded) sizes and ranks. timing_end waits for
 * the last event and writes one tlrmdd_kernel_stats per kind into
 * stats[TLRMDD_K_NKINDS] (host array, may be NULL). Calls that run while
 * timing is active are serialised with the recorder by a mutex. */
#define TLRMDD_K_GEMM_RESID    0  /* r = D X - U with FP64 |r|^2 partials (dense)            */
#define TLRMDD_K_GEMM_ADJOINT  1  /* W = D^H r                                              */
#define TLRMDD_K_GEMM_LINE     2  /* [a | b] = D [X1 | X2] + line-search sums               */
#define TLRMDD_K_ASSEMBLE      3  /* X = C(theta)                                           */
#define TLRMDD_K_ASSEMBLE_DIR  4  /* X1, X2 of the line search                              */
#define TLRMDD_K_GRAD          5  /* per-tile gradient contractions                         */
#define TLRMDD_K_LINE_PACK     6  /* tile forms: factor packing, gradient summation, P update */
#define TLRMDD_K_LINE_TILE     7  /* tile-form line search: both product stages             */
#define TLRMDD_K_GRAD_TILE     8  /* tile-form gradient: its three products                 */
#define TLRMDD_K_RESID_TILE    9  /* tile-form residual product r_:,j = sum_i P_ij B_ij - U  */
#define TLRMDD_K_STAGE        10  /* staging of D (padded copy, D^H, split planes) and of U   */
#define TLRMDD_K_PERMUTE      11  /* column gather D S (tlrmdd_permute_columns)               */
#define TLRMDD_K_GRAM         12  /* L-BFGS Gram pass                                        */
#define TLRMDD_K_COMBINE      13  /* L-BFGS direction p = sum_b c_b v_b                       */
#define TLRMDD_K_THETA_UPDATE 14  /* theta += a* p (and the newest s pair)                  */
#define TLRMDD_K_RESID_UPDATE 15  /* r += a* a + a*^2 b                                     */
#define TLRMDD_K_NKINDS       16

#define TLRMDD_DT_NONE  (-1)      /* no matrix-core flops counted (memory-bound kind)        */
#define TLRMDD_DT_FP32  0
#define TLRMDD_DT_BF16  1
#define TLRMDD_DT_MIXED 2         /* launches of one kind ran in different instruction types */

typedef struct {
    double  ms;          /* summed launch durations (HIP events on the launch stream)          */
    int64_t launches;
    double  cflops;      /* complex products counted 8 m n k (true sizes and ranks)             */
    double  flops;       /* real flops of the product form that ran, on the same sizes:
                            four-product FP32 8 m n k, three-product FP32 6 m n k,
                            BF16 hi+lo split 24 m n k (BF16 instructions)                     */
    double  bytes;       /* algorithmic HBM bytes: each operand read once, each output written
                            once (L-BFGS passes: the held pairs of a run without restarts)    */
    int32_t flop_dtype;  /* TLRMDD_DT_* of `flops`                                            */
    int32_t reserved;
} tlrmdd_kernel_stats;

int tlrmdd_timing_begin(void);
int tlrmdd_timing_end(tlrmdd_kernel_stats *stats);

/* tlrmdd_timing_begin restricted to some kinds: only launches of the kinds whose
 * bit (1u << TLRMDD_K_*) is set in `kinds` are bracketed and counted; the others
 * run as without timing and their stats read zero. Each bracketed launch adds two
 * event records to its stream (a few microseconds of device time each), so timing
 * one kind perturbs a run far less than timing all of them. Returns
 * TLRMDD_INVALID_ARGUMENT for an empty set or a bit at or above TLRMDD_K_NKINDS.
 * tlrmdd_timing_begin() equals this call with every kind's bit set. */
int tlrmdd_timing_begin_kinds(uint32_t kinds);

/* ---- HIP graphs of library calls ------------------------------------------
 * A fixed-count solve of one frequency (Theory section, eq. standard_solver: every
 * frequency is its own problem) is a fixed sequence of launches; at small sizes its
 * time is the launch latency. The calls made on `stream` between tlrmdd_graph_begin
 * and tlrmdd_graph_end are recorded into a HIP graph instead of being run, and
 * tlrmdd_graph_launch replays the whole sequence as one submission.
 *   - `stream` must be a created stream, not the null stream. Capture is per thread
 *     (relaxed mode); one capture may be open per thread.
 *   - Every pointer a recorded call received (data, theta, f-history, workspace) is
 *     baked into the graph: the caller keeps those buffers alive and unmoved until
 *     tlrmdd_graph_destroy, and changes their contents between launches as needed
 *     (a solve updates theta in place, so a fresh solve per launch means restoring
 *     theta first). Host tables that a recorded call would upload (batched tables,
 *     tile-form tables) are copied into pinned host memory owned by the graph.
 *   - Calls whose results are host values (tlrmdd_tile_ranks, tlrmdd_choose_layout,
 *     tlrmdd_warm_start) synchronise and cannot be recorded: they fail, and so does
 *     the capture (tlrmdd_graph_end returns TLRMDD_HIP_ERROR and no graph).
 *   - Kernel timing (tlrmdd_timing_*) does not see recorded calls.
 * tlrmdd_graph_end always closes the capture opened on `stream`, also when a
 * recorded call failed. Statuses: TLRMDD_INVALID_ARGUMENT for a null stream, a second
 * begin on one thread, or an end without a begin on that stream; TLRMDD_HIP_ERROR
 * when HIP refuses the capture or the instantiation. */
typedef struct tlrmdd_graph_s *tlrmdd_graph;
int tlrmdd_graph_begin(hipStream_t stream);
int tlrmdd_graph_end(hipStream_t stream, tlrmdd_graph *graph_out);
int tlrmdd_graph_launch(tlrmdd_graph graph, hipStream_t stream);
int tlrmdd_graph_destroy(tlrmdd_graph graph);

#ifdef __cplusplus
}
#endif
#endif /* TLRMDD_H */
