// Batched per-tile FP64 SVD (one-sided Jacobi) for the rank estimate and the warm start (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace tlr {

// One tile of X at (row0, col0), decomposed as A = X_ij (trans = 0) or A = X_ij^T (trans = 1, used
// when X_ij has fewer rows than columns, so that A is never wide); A is m x n. W and V are complex128
// column-major per tile.
struct SvdTile {
    int32_t m, n;    // rows / columns of A
    int32_t trans;
    int32_t pad;
    int64_t row0, col0;
    int64_t offW;    // W: m x n
    int64_t offV;    // V: n x n (warm start of a factored tile), -1 without V
    int64_t offS;    // sigma / order: n entries
    int32_t npad;    // n rounded up to even (round-robin players)
    int32_t pair0;   // first block of this tile in a round launch (prefix sum of npad / 2)
};

enum WarmKind : int32_t { WARM_LR = 0, WARM_QQ = 1, WARM_DENSE = 2 };
struct WarmItem {
    int32_t tile;    // SvdTile index
    int32_t kind;    // WarmKind
    int32_t k;       // rank kept
    int32_t pad;
    int64_t offA;    // theta offset of L / Q / Z
    int64_t offB;    // theta offset of R (LR)
};

constexpr int SVD_MAX_N = 1024;     // tile columns handled by the per-tile sort
constexpr int SVD_MAX_SWEEPS = 30;  // sweeps enqueued; converged sweeps return at once
constexpr double SVD_TOL = 1e-13;   // rotate a pair while |w_p^H w_q| > tol ||w_p|| ||w_q||

hipError_t launch_svd_gather(const SvdTile *tiles, int ntiles, const float2 *X, int64_t ldx, double2 *W, double2 *V,
                             hipStream_t s);
hipError_t launch_svd_round(const SvdTile *tiles, const int32_t *pair_tile, int npairs, int round, double2 *W,
                            double2 *V, const int32_t *flags, int32_t *busy, double tol, hipStream_t s);
hipError_t launch_svd_sweep_end(int32_t *flags, int32_t *busy, hipStream_t s);
hipError_t launch_svd_sigma(const SvdTile *tiles, int ntiles, const double2 *W, double *sig, hipStream_t s);
hipError_t launch_svd_rank(const SvdTile *tiles, int ntiles, const double *sig, int64_t nsig, double eps,
                           int32_t *kout, double *v0out, hipStream_t s);
hipError_t launch_svd_order(const SvdTile *tiles, int ntiles, const double *sig, int32_t *order, hipStream_t s);
hipError_t launch_svd_factors(const SvdTile *tiles, const WarmItem *items, int nitems, const double2 *W,
                              const double2 *V, const double *sig, const int32_t *order, const float2 *X,
                              int64_t ldx, float2 *theta, hipStream_t s);

}  // namespace tlr
