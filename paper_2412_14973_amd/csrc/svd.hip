// Per-tile SVD in FP64 for the rank / tile-size estimate and the warm start
// (Hyper-parameter selection and initialization; the examples' rank study).
//
// Every tile X_ij (i >= j) of a reference solution is copied to FP64 and
// decomposed by one-sided (Hestenes) Jacobi: column pairs of W = X_ij are
// rotated until all columns are mutually orthogonal, accumulating the same
// rotations in V, so that X_ij V = W with the columns of W equal to
// sigma_c u_c. A launch performs one round of the round-robin ordering for all
// tiles at once (each pair of a round is disjoint from the others, one wave per
// pair); a sweep is n' - 1 rounds (n' = columns rounded up to even). After each
// sweep a flag records whether any pair was still rotated above the tolerance;
// once none is, the remaining launches return at once.
#include <hip/hip_runtime.h>

#include "svd.hpp"

extern "C" __device__ double __ockl_wfred_add_f64(double);

namespace tlr {
namespace {

__device__ __forceinline__ double wsum(double v) { return __ockl_wfred_add_f64(v); }

// X (complex64, row-major, ld ldx) -> W (complex128, column-major m x n per tile); V = I when wanted
__global__ __launch_bounds__(256) void svd_gather_kernel(const SvdTile *__restrict__ tiles,
                                                         const float2 *__restrict__ X, int64_t ldx,
                                                         double2 *__restrict__ W, double2 *__restrict__ V) {
    const SvdTile t = tiles[blockIdx.x];
    for (int c = blockIdx.y; c < t.n; c += gridDim.y) {
        for (int r = threadIdx.x; r < t.m; r += blockDim.x) {   // A[r][c] = X_ij[r][c] or X_ij[c][r]
            const float2 x = t.trans ? X[(int64_t)(t.row0 + c) * ldx + t.col0 + r]
                                     : X[(int64_t)(t.row0 + r) * ldx + t.col0 + c];
            W[t.offW + (int64_t)c * t.m + r] = make_double2(x.x, x.y);
        }
        if (V && t.offV >= 0)
            for (int r = threadIdx.x; r < t.n; r += blockDim.x)
                V[t.offV + (int64_t)c * t.n + r] = make_double2(r == c ? 1.0 : 0.0, 0.0);
    }
}

// pair k of round r in the circle ordering of n' (even) columns: every pair once per n' - 1 rounds
__device__ __forceinline__ void round_pair(int np, int r, int k, int &p, int &q) {
    const int L = np - 1;
    if (k == 0) {
        p = r % L;
        q = L;
    } else {
        p = (r + k) % L;
        q = (r - k + L) % L;
    }
    if (p > q) { const int s = p; p = q; q = s; }
}

// One round for all tiles: block b handles pair (b - pair0[tile]) of tile pair_tile[b].
__global__ __launch_bounds__(64) void svd_round_kernel(const SvdTile *__restrict__ tiles,
                                                       const int32_t *__restrict__ pair_tile, int round,
                                                       double2 *__restrict__ W, double2 *__restrict__ V,
                                                       const int32_t *__restrict__ flags, int32_t *__restrict__ busy,
                                                       double tol) {
    if (flags[0]) return;   // converged in an earlier sweep
    const int tid = pair_tile[blockIdx.x];
    const SvdTile t = tiles[tid];
    int p, q;
    round_pair(t.npad, round % (t.npad - 1), blockIdx.x - t.pair0, p, q);
    if (q >= t.n) return;   // the padding column
    double2 *wp = W + t.offW + (int64_t)p * t.m;
    double2 *wq = W + t.offW + (int64_t)q * t.m;
    double a = 0.0, b = 0.0, gr = 0.0, gi = 0.0;
    for (int r = threadIdx.x; r < t.m; r += 64) {
        const double2 x = wp[r], y = wq[r];
        a = fma(x.x, x.x, fma(x.y, x.y, a));
        b = fma(y.x, y.x, fma(y.y, y.y, b));
        gr = fma(x.x, y.x, fma(x.y, y.y, gr));   // gamma = conj(x) . y
        gi = fma(x.x, y.y, fma(-x.y, y.x, gi));
    }
    a = wsum(a);
    b = wsum(b);
    gr = wsum(gr);
    gi = wsum(gi);
    const double g = sqrt(gr * gr + gi * gi);
    if (!(g > tol * sqrt(a * b))) return;   // orthogonal enough (or a zero column)
    if (threadIdx.x == 0) busy[0] = 1;
    // with e = gamma/|gamma|: w_p' = c w_p - s conj(e) w_q,  w_q' = s w_p + c conj(e) w_q
    // (the real rotation that makes (w_p, conj(e) w_q) orthogonal; conj(e) w_q is a unit-modulus
    // rescaling of a column, which V records as well)
    const double zeta = (b - a) / (2.0 * g);
    const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + tt * tt), s = c * tt;
    const double er = gr / g, ei = -gi / g;   // conj(e)
    for (int r = threadIdx.x; r < t.m; r += 64) {
        const double2 x = wp[r], y = wq[r];
        const double yr = er * y.x - ei * y.y, yi = er * y.y + ei * y.x;   // conj(e) y
        wp[r] = make_double2(c * x.x - s * yr, c * x.y - s * yi);
        wq[r] = make_double2(s * x.x + c * yr, s * x.y + c * yi);
    }
    if (V && t.offV >= 0) {
        double2 *vp = V + t.offV + (int64_t)p * t.n;
        double2 *vq = V + t.offV + (int64_t)q * t.n;
        for (int r = threadIdx.x; r < t.n; r += 64) {
            const double2 x = vp[r], y = vq[r];
            const double yr = er * y.x - ei * y.y, yi = er * y.y + ei * y.x;
            vp[r] = make_double2(c * x.x - s * yr, c * x.y - s * yi);
            vq[r] = make_double2(s * x.x + c * yr, s * x.y + c * yi);
        }
    }
}

// end of a sweep: converged when no pair was rotated; clear the marker for the next sweep
__global__ void svd_sweep_end_kernel(int32_t *flags, int32_t *busy) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (!flags[0] && busy[0] == 0) flags[0] = 1;
        busy[0] = 0;
    }
}

// sigma of every column (one wave per column); sig index = tile's sigma offset + column
__global__ __launch_bounds__(256) void svd_sigma_kernel(const SvdTile *__restrict__ tiles,
                                                        const double2 *__restrict__ W, double *__restrict__ sig) {
    const SvdTile t = tiles[blockIdx.x];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int c = wv; c < t.n; c += 4) {
        const double2 *w = W + t.offW + (int64_t)c * t.m;
        double a = 0.0;
        for (int r = lane; r < t.m; r += 64) a = fma(w[r].x, w[r].x, fma(w[r].y, w[r].y, a));
        a = wsum(a);
        if (lane == 0) sig[t.offS + c] = sqrt(a);
    }
}

// v0 = max sigma over all tiles; k of every tile = #{sigma >= eps v0}  (one block, fixed order)
__global__ __launch_bounds__(256) void svd_rank_kernel(const SvdTile *__restrict__ tiles, int ntiles,
                                                       const double *__restrict__ sig, int64_t nsig, double eps,
                                                       int32_t *__restrict__ kout, double *__restrict__ v0out) {
    __shared__ double red[256];
    double m = 0.0;
    for (int64_t e = threadIdx.x; e < nsig; e += 256) m = fmax(m, sig[e]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    const double v0 = red[0];
    for (int ti = threadIdx.x; ti < ntiles; ti += 256) {
        const SvdTile t = tiles[ti];
        int k = 0;
        for (int c = 0; c < t.n; ++c) k += (sig[t.offS + c] >= eps * v0) ? 1 : 0;
        kout[ti] = k;
    }
    if (threadIdx.x == 0) v0out[0] = v0;
}

// per tile: column indices sorted by sigma, descending (ties: lower column first); n <= 1024
__global__ __launch_bounds__(256) void svd_order_kernel(const SvdTile *__restrict__ tiles,
                                                        const double *__restrict__ sig, int32_t *__restrict__ order) {
    __shared__ double key[1024];
    __shared__ int32_t idx[1024];
    const SvdTile t = tiles[blockIdx.x];
    int n2 = 1;
    while (n2 < t.n) n2 <<= 1;
    for (int e = threadIdx.x; e < n2; e += 256) {
        key[e] = e < t.n ? sig[t.offS + e] : -1.0;
        idx[e] = e;
    }
    __syncthreads();
    // bitonic sort, "before" = larger sigma, then lower index
    for (int sz = 2; sz <= n2; sz <<= 1) {
        for (int st = sz >> 1; st > 0; st >>= 1) {
            for (int e = threadIdx.x; e < n2; e += 256) {
                const int o = e ^ st;
                if (o > e) {
                    const bool asc = (e & sz) == 0;   // this run in "before" order
                    const bool e_first = key[e] > key[o] || (key[e] == key[o] && idx[e] < idx[o]);
                    if (e_first != asc) {
                        const double kk = key[e]; key[e] = key[o]; key[o] = kk;
                        const int32_t ii = idx[e]; idx[e] = idx[o]; idx[o] = ii;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int e = threadIdx.x; e < t.n; e += 256) order[t.offS + e] = idx[e];
}

// Warm-start factors of one tile (one block per tile): off-diagonal L = U_k S_k^(1/2) = W_c / sqrt(s_c),
// R = S_k^(1/2) V_k^H; diagonal Q Q^T: Q = U_k D^(1/2) S_k^(1/2) with d_c = u_c^H conj(v_c) made unit
// (Takagi from the SVD of a complex symmetric tile); dense diagonal: Z = X_ii.
__global__ __launch_bounds__(256) void svd_factors_kernel(const SvdTile *__restrict__ tiles,
                                                          const WarmItem *__restrict__ items,
                                                          const double2 *__restrict__ W,
                                                          const double2 *__restrict__ V,
                                                          const double *__restrict__ sig,
                                                          const int32_t *__restrict__ order,
                                                          const float2 *__restrict__ X, int64_t ldx,
                                                          float2 *__restrict__ theta) {
    const WarmItem it = items[blockIdx.x];
    const SvdTile t = tiles[it.tile];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (it.kind == WARM_DENSE) {
        for (int e = threadIdx.x; e < t.m * t.n; e += 256) {
            const int r = e / t.n, c = e % t.n;
            theta[it.offA + e] = X[(int64_t)(t.row0 + r) * ldx + t.col0 + c];
        }
        return;
    }
    for (int l = wv; l < it.k; l += 4) {
        const int c = order[t.offS + l];
        const double s = sig[t.offS + c];
        const double2 *w = W + t.offW + (int64_t)c * t.m;
        const double2 *v = V + t.offV + (int64_t)c * t.n;
        if (it.kind == WARM_LR && !t.trans) {   // X_ij = U S V^H
            const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;   // u sqrt(s) = w / sqrt(s)
            for (int r = lane; r < t.m; r += 64)
                theta[it.offA + (int64_t)r * it.k + l] = make_float2((float)(w[r].x * inv), (float)(w[r].y * inv));
            const double rs = sqrt(s);
            for (int r = lane; r < t.n; r += 64)   // R[l][col] = sqrt(s) conj(V[col][c])
                theta[it.offB + (int64_t)l * t.n + r] = make_float2((float)(rs * v[r].x), (float)(-rs * v[r].y));
        } else if (it.kind == WARM_LR) {   // X_ij^T = U' S V'^H, so X_ij = conj(V') S U'^T
            const double rs = sqrt(s);
            for (int r = lane; r < t.n; r += 64)   // L[r][l] = conj(V'[r][c]) sqrt(s); L has t.n = d_i rows
                theta[it.offA + (int64_t)r * it.k + l] = make_float2((float)(rs * v[r].x), (float)(-rs * v[r].y));
            const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
            for (int r = lane; r < t.m; r += 64)   // R[l][col] = sqrt(s) U'[col][c] = W[col][c] / sqrt(s)
                theta[it.offB + (int64_t)l * t.m + r] = make_float2((float)(w[r].x * inv), (float)(w[r].y * inv));
        } else {   // WARM_QQ: d = u^H conj(v) = sum conj(w/s) conj(v)
            double dr = 0.0, di = 0.0;
            for (int r = lane; r < t.m; r += 64) {
                // conj(w) * conj(v) = conj(w v)
                dr += w[r].x * v[r].x - w[r].y * v[r].y;
                di -= w[r].x * v[r].y + w[r].y * v[r].x;
            }
            dr = wsum(dr);
            di = wsum(di);
            const double mod = sqrt(dr * dr + di * di);
            double hr = 1.0, hi = 0.0;   // sqrt(d / |d|): half the angle
            if (mod > 0.0) {
                const double ang = 0.5 * atan2(di, dr);
                hr = cos(ang);
                hi = sin(ang);
            }
            const double f = s > 0.0 ? 1.0 / sqrt(s) : 0.0;   // u sqrt(s) = w / sqrt(s)
            for (int r = lane; r < t.m; r += 64) {
                const double xr = w[r].x * f, xi = w[r].y * f;
                theta[it.offA + (int64_t)r * it.k + l] =
                    make_float2((float)(xr * hr - xi * hi), (float)(xr * hi + xi * hr));
            }
        }
    }
}

}  // namespace

hipError_t launch_svd_gather(const SvdTile *tiles, int ntiles, const float2 *X, int64_t ldx, double2 *W, double2 *V,
                             hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(svd_gather_kernel, dim3((unsigned)ntiles, 64), dim3(256), 0, s, tiles, X, ldx, W, V);
    return hipGetLastError();
}

hipError_t launch_svd_round(const SvdTile *tiles, const int32_t *pair_tile, int npairs, int round, double2 *W,
                            double2 *V, const int32_t *flags, int32_t *busy, double tol, hipStream_t s) {
    if (npairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(svd_round_kernel, dim3((unsigned)npairs), dim3(64), 0, s, tiles, pair_tile, round, W, V, flags,
                       busy, tol);
    return hipGetLastError();
}

hipError_t launch_svd_sweep_end(int32_t *flags, int32_t *busy, hipStream_t s) {
    hipLaunchKernelGGL(svd_sweep_end_kernel, dim3(1), dim3(64), 0, s, flags, busy);
    return hipGetLastError();
}

hipError_t launch_svd_sigma(const SvdTile *tiles, int ntiles, const double2 *W, double *sig, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(svd_sigma_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, tiles, W, sig);
    return hipGetLastError();
}

hipError_t launch_svd_rank(const SvdTile *tiles, int ntiles, const double *sig, int64_t nsig, double eps,
                           int32_t *kout, double *v0out, hipStream_t s) {
    hipLaunchKernelGGL(svd_rank_kernel, dim3(1), dim3(256), 0, s, tiles, ntiles, sig, nsig, eps, kout, v0out);
    return hipGetLastError();
}

hipError_t launch_svd_order(const SvdTile *tiles, int ntiles, const double *sig, int32_t *order, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(svd_order_kernel, dim3((unsigned)ntiles), dim3(256), 0, s, tiles, sig, order);
    return hipGetLastError();
}

hipError_t launch_svd_factors(const SvdTile *tiles, const WarmItem *items, int nitems, const double2 *W,
                              const double2 *V, const double *sig, const int32_t *order, const float2 *X,
                              int64_t ldx, float2 *theta, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(svd_factors_kernel, dim3((unsigned)nitems), dim3(256), 0, s, tiles, items, W, V, sig, order,
                       X, ldx, theta);
    return hipGetLastError();
}

}  // namespace tlr
