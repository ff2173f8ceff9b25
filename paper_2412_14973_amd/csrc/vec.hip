// Memory-bound kernels: staging of D, column permutation (eq. axb_sd), and the
// optimiser's vector / scalar work (L-BFGS two-loop recursion, exact line
// search, updates). All reductions are FP64, deterministic (fixed-order
// per-segment partials, then one fixed-order tree per problem), with no
// atomics. Scalars never leave the device.
#include "common.hpp"
#include "vec.hpp"

namespace tlr {
namespace {

// ---------------------------------------------------------------------------
// staging: Ds = D (padded rows), DHs = conj(D)^T  (32 x 32 tiles through LDS)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void stage_d_kernel(const float2 *__restrict__ D, int64_t ns, int64_t nr,
                                                      float2 *__restrict__ Ds, int64_t ldk,
                                                      float2 *__restrict__ DHs, int64_t lds) {
    // grid covers the padded lds x ldk block; padding is written as zeros
    __shared__ float2 tile[32][33];
    const int64_t s0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t s = s0 + r, c = c0 + tx;
        float2 v = make_float2(0.f, 0.f);
        if (s < ns && c < nr) v = D[s * nr + c];
        if (Ds && s < lds && c < ldk) Ds[s * ldk + c] = v;
        tile[r][tx] = v;
    }
    if (!DHs) return;
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t c = c0 + r, s = s0 + tx;
        if (s < lds && c < ldk) {
            const float2 v = tile[tx][r];
            DHs[c * lds + s] = make_float2(v.x, -v.y);
        }
    }
}

__global__ __launch_bounds__(256) void stage_d_split_kernel(const float2 *__restrict__ D, int64_t ns, int64_t nr,
                                                            uint32_t *__restrict__ Dh, uint32_t *__restrict__ Dl,
                                                            int64_t ldk, uint32_t *__restrict__ DHh,
                                                            uint32_t *__restrict__ DHl, int64_t lds) {
    __shared__ float2 tile[32][33];
    const int64_t s0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int64_t s = s0 + r, c = c0 + tx;
        float2 v = make_float2(0.f, 0.f);
        if (s < ns && c < nr) v = D[s * nr + c];
        if (s < lds && c < ldk) {
            uint32_t h, l;
            split_c(v, h, l);
            Dh[s * ldk + c] = h;
            Dl[s * ldk + c] = l;
        }
        tile[r][tx] = v;
    }
    if (!DHh) return;
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t c = c0 + r, s = s0 + tx;
        if (s < lds && c < ldk) {
            const float2 v = tile[tx][r];
            uint32_t h, l;
            split_c(make_float2(v.x, -v.y), h, l);
            DHh[c * lds + s] = h;
            DHl[c * lds + s] = l;
        }
    }
}

__global__ __launch_bounds__(256) void split_transpose_kernel(const float2 *__restrict__ r, int64_t ldr, int64_t rows,
                                                              int64_t cols, uint32_t *__restrict__ th,
                                                              uint32_t *__restrict__ tl, int64_t ldt, int64_t s_r,
                                                              int64_t s_t) {
    __shared__ float2 tile[32][33];
    const int z = blockIdx.z;
    r += z * s_r;
    th += z * s_t;
    tl += z * s_t;
    const int64_t r0 = (int64_t)blockIdx.y * 32, c0 = (int64_t)blockIdx.x * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int q = ty; q < 32; q += 8) {
        const int64_t i = r0 + q, j = c0 + tx;
        tile[q][tx] = (i < rows && j < cols) ? r[i * ldr + j] : make_float2(0.f, 0.f);
    }
    __syncthreads();
    for (int q = ty; q < 32; q += 8) {
        const int64_t j = c0 + q, i = r0 + tx;
        if (i < rows && j < cols) {
            uint32_t h, l;
            split_c(tile[tx][q], h, l);
            th[j * ldt + i] = h;
            tl[j * ldt + i] = l;
        }
    }
}

// zero the padding (rows >= n, and columns >= n of rows < n) of ld x ld word planes
__global__ void zero_pad_kernel(uint32_t *__restrict__ base, int64_t ld, int64_t n, int64_t plane_stride,
                                int64_t batch_stride) {
    const int64_t row = blockIdx.x;
    uint32_t *p = base + (int64_t)blockIdx.z * batch_stride + (int64_t)blockIdx.y * plane_stride + row * ld;
    const int64_t c0 = row < n ? n : 0;
    for (int64_t c = c0 + threadIdx.x; c < ld; c += blockDim.x) p[c] = 0u;
}

__global__ void copy2d_kernel(const float2 *__restrict__ src, int64_t lds, float2 *__restrict__ dst,
                              int64_t ldd, int64_t rows, int64_t cols) {
    const int64_t r = blockIdx.y;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += (int64_t)gridDim.x * blockDim.x)
        if (r < rows) dst[r * ldd + c] = src[r * lds + c];
}

__global__ void permute_kernel(const float2 *__restrict__ in, const int64_t *__restrict__ perm,
                               float2 *__restrict__ out, int64_t rows, int64_t cols) {
    const int64_t r = blockIdx.y;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += (int64_t)gridDim.x * blockDim.x)
        out[r * cols + c] = in[r * cols + perm[c]];
}

// ---------------------------------------------------------------------------
// segment helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) r = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
    return r;  // valid on thread 0
}

__device__ __forceinline__ int ring_slot(const SolveScalars &sc, int i, int m1) {
    int s = sc.head - 1 - i;
    s %= m1;
    if (s < 0) s += m1;
    return s;
}

// y = g_new - g_prev (into Y[head]); partials: Re<s, y>, Re<y, y>
__global__ __launch_bounds__(256) void pair_kernel(const VecSeg *__restrict__ segs, const float *__restrict__ gnew,
                                                   const float *__restrict__ gprev, float *__restrict__ Yb,
                                                   const float *__restrict__ Sb, int64_t stride2,
                                                   const SolveScalars *__restrict__ sc, double *__restrict__ part) {
    __shared__ double red[4];
    const VecSeg sg = segs[blockIdx.x];
    const int slot = sc[sg.prob].head;
    float *Y = Yb + slot * stride2;
    const float *S = Sb + slot * stride2;
    double a = 0.0, b = 0.0;
    for (int e = threadIdx.x; e < sg.n; e += 256) {
        const int64_t o = sg.off + e;
        const float y = gnew[o] - gprev[o];
        Y[o] = y;
        a += (double)S[o] * y;
        b += (double)y * y;
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) { part[2 * sg.part] = a; part[2 * sg.part + 1] = b; }
}

// first loop of the two-loop recursion, step i (newest pair first):
//   q = (i == 0 ? g : q - alpha_{i-1} y_{i-1});  partial Re<s_i, q>
__global__ __launch_bounds__(256) void twoloop1_kernel(const VecSeg *__restrict__ segs, int i, int m1,
                                                       float *__restrict__ q, const float *__restrict__ g,
                                                       const float *__restrict__ Sb, const float *__restrict__ Yb,
                                                       int64_t stride2, const SolveScalars *__restrict__ sc,
                                                       double *__restrict__ part) {
    __shared__ double red[4];
    const VecSeg sg = segs[blockIdx.x];
    const SolveScalars &s = sc[sg.prob];
    const int count = s.count;
    const bool upd = (i > 0) && (i - 1 < count);
    const bool dot = i < count;
    const float al = upd ? (float)s.alpha[i - 1] : 0.f;
    const float *Y = upd ? Yb + ring_slot(s, i - 1, m1) * stride2 : nullptr;
    const float *S = dot ? Sb + ring_slot(s, i, m1) * stride2 : nullptr;
    double acc = 0.0;
    for (int e = threadIdx.x; e < sg.n; e += 256) {
        const int64_t o = sg.off + e;
        float v = (i == 0) ? g[o] : q[o];
        if (upd) v -= al * Y[o];
        q[o] = v;
        if (dot) acc += (double)S[o] * v;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[sg.part] = acc;
}

// second loop of the two-loop recursion (oldest pair first):
//   start: z = gamma q (else z from the previous step), then z += cb s_iu when iu is a valid pair;
//   last:  p = -z with partial Re<g, p>;   otherwise store z with partial Re<y_inext, z>
__global__ __launch_bounds__(256) void twoloop2_kernel(const VecSeg *__restrict__ segs, int start, int last, int iu,
                                                       int inext, int m1, const float *__restrict__ q,
                                                       float *__restrict__ zv, float *__restrict__ p,
                                                       const float *__restrict__ g, const float *__restrict__ Sb,
                                                       const float *__restrict__ Yb, int64_t stride2,
                                                       const SolveScalars *__restrict__ sc,
                                                       double *__restrict__ part) {
    __shared__ double red[4];
    const VecSeg sg = segs[blockIdx.x];
    const SolveScalars &s = sc[sg.prob];
    const int count = s.count;
    const bool upd = (iu >= 0) && (iu < count);
    const bool dot = !last && (inext >= 0) && (inext < count);
    const float cb = upd ? (float)s.beta_coef : 0.f;
    const float gam = (float)s.gamma;
    const float *S = upd ? Sb + ring_slot(s, iu, m1) * stride2 : nullptr;
    const float *Y = dot ? Yb + ring_slot(s, inext, m1) * stride2 : nullptr;
    double acc = 0.0;
    for (int e = threadIdx.x; e < sg.n; e += 256) {
        const int64_t o = sg.off + e;
        float v = start ? gam * q[o] : zv[o];
        if (upd) v += cb * S[o];
        if (last) {
            const float pv = -v;
            p[o] = pv;
            acc += (double)g[o] * pv;
        } else {
            zv[o] = v;
            if (dot) acc += (double)Y[o] * v;
        }
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[sg.part] = acc;
}

// p = -g where the problem restarts (or always when force != 0); partial Re<g,p> not needed
__global__ __launch_bounds__(256) void restart_kernel(const VecSeg *__restrict__ segs, int force,
                                                      float *__restrict__ p, const float *__restrict__ g,
                                                      const SolveScalars *__restrict__ sc) {
    const VecSeg sg = segs[blockIdx.x];
    if (!force && !sc[sg.prob].restart) return;
    for (int e = threadIdx.x; e < sg.n; e += 256) {
        const int64_t o = sg.off + e;
        p[o] = -g[o];
    }
}

// g += 2 lambda theta
__global__ __launch_bounds__(256) void reg_grad_kernel(const VecSeg *__restrict__ segs, float *__restrict__ g,
                                                       const float *__restrict__ th, float lam2) {
    const VecSeg sg = segs[blockIdx.x];
    for (int e = threadIdx.x; e < sg.n; e += 256) {
        const int64_t o = sg.off + e;
        g[o] += lam2 * th[o];
    }
}

// partials Re<x0,y0>, Re<x1,y1>
__global__ __launch_bounds__(256) void dot2_kernel(const VecSeg *__restrict__ segs, const float *__restrict__ x0,
                                                   const float *__restrict__ y0, const float *__restrict__ x1,
                                                   const float *__restrict__ y1, double *__restrict__ part) {
    __shared__ double red[4];
    const VecSeg sg = segs[blockIdx.x];
    double a = 0.0, b = 0.0;
    for (int e = threadIdx.x; e < sg.n; e += 256) {
        const int64_t o = sg.off + e;
        a += (double)x0[o] * y0[o];
        b += (double)x1[o] * y1[o];
    }
    a = block_sum(a, red);
    b = block_sum(b, red);
    if (threadIdx.x == 0) { part[2 * sg.part] = a; part[2 * sg.part + 1] = b; }
}

// theta += step p ; S[head] = step p ; partial ||theta||^2
__global__ __launch_bounds__(256) void theta_update_kernel(const VecSeg *__restrict__ segs, float *__restrict__ th,
                                                           const float *__restrict__ p, float *__restrict__ Sb,
                                                           int64_t stride2, const SolveScalars *__restrict__ sc,
                                                           double *__restrict__ part) {
    __shared__ double red[4];
    const VecSeg sg = segs[blockIdx.x];
    const SolveScalars &s = sc[sg.prob];
    const float a = (float)s.step;
    const bool frozen = s.frozen != 0;   // a non-finite step froze this problem: theta stays as is
    float *S = (Sb && !frozen) ? Sb + s.head * stride2 : nullptr;
    double acc = 0.0;
    for (int e = threadIdx.x; e < sg.n; e += 256) {
        const int64_t o = sg.off + e;
        float v = th[o];
        if (!frozen) {
            const float sp = a * p[o];
            v += sp;
            th[o] = v;
            if (S) S[o] = sp;
        }
        acc += (double)v * v;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[sg.part] = acc;
}

// r += step a + step^2 b ; partial ||r||^2
__global__ __launch_bounds__(256) void resid_update_kernel(const VecSeg *__restrict__ segs, float *__restrict__ r,
                                                           const float *__restrict__ a, const float *__restrict__ b,
                                                           const SolveScalars *__restrict__ sc,
                                                           double *__restrict__ part) {
    __shared__ double red[4];
    const VecSeg sg = segs[blockIdx.x];
    const SolveScalars &s = sc[sg.prob];
    const float al = (float)s.step;
    const float al2 = (float)(s.step * s.step);
    const bool frozen = s.frozen != 0;
    double acc = 0.0;
    for (int e = threadIdx.x; e < sg.n; e += 256) {
        const int64_t o = sg.off + e;
        float v = r[o];
        if (!frozen) {
            v += al * a[o] + al2 * b[o];
            r[o] = v;
        }
        acc += (double)v * v;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[sg.part] = acc;
}

// ---------------------------------------------------------------------------
// exact step: positive minimiser of phi with phi'(a) = c0 + c1 a + c2 a^2 + c3 a^3
// ---------------------------------------------------------------------------
__device__ double phi_inc(const double *c, double a) {
    return a * (c[0] + a * (c[1] / 2 + a * (c[2] / 3 + a * c[3] / 4)));
}

__device__ double polish(const double *c, double x) {
    for (int it = 0; it < 6; ++it) {
        const double f = ((c[3] * x + c[2]) * x + c[1]) * x + c[0];
        const double fp = (3 * c[3] * x + 2 * c[2]) * x + c[1];
        if (fp == 0.0 || !isfinite(fp)) break;
        const double nx = x - f / fp;
        if (!isfinite(nx)) break;
        x = nx;
    }
    return x;
}

__device__ double exact_step_dev(const double *c) {
    double roots[3];
    int nroot = 0;
    const double scale = fabs(c[0]) + fabs(c[1]) + fabs(c[2]) + fabs(c[3]);
    if (!(scale > 0.0) || !isfinite(scale)) return 0.0;
    if (c[3] == 0.0 && c[2] == 0.0) {
        if (c[1] != 0.0) roots[nroot++] = -c[0] / c[1];
    } else if (c[3] == 0.0) {
        const double disc = c[1] * c[1] - 4 * c[2] * c[0];
        if (disc >= 0.0) {
            const double sq = sqrt(disc);
            const double qv = -0.5 * (c[1] + (c[1] >= 0 ? sq : -sq));
            if (qv != 0.0) roots[nroot++] = c[0] / qv;
            roots[nroot++] = qv / c[2];
        }
    } else {
        // depressed cubic t^3 + P t + Q = 0 with a = t - A/3
        const double A = c[2] / c[3], B = c[1] / c[3], C = c[0] / c[3];
        const double P = B - A * A / 3.0;
        const double Q = 2.0 * A * A * A / 27.0 - A * B / 3.0 + C;
        const double disc = 0.25 * Q * Q + P * P * P / 27.0;
        if (disc > 0.0) {
            const double sq = sqrt(disc);
            const double u = cbrt(-0.5 * Q + (Q <= 0 ? sq : -sq));
            const double v = (u != 0.0) ? -P / (3.0 * u) : 0.0;
            roots[nroot++] = u + v - A / 3.0;
        } else if (P == 0.0) {
            roots[nroot++] = -A / 3.0;
        } else {
            const double rr = 2.0 * sqrt(-P / 3.0);
            double arg = (3.0 * Q / (2.0 * P)) * sqrt(-3.0 / P);
            arg = fmin(1.0, fmax(-1.0, arg));
            const double ph = acos(arg) / 3.0;
            const double tp = 2.0943951023931954923;  // 2 pi / 3
            for (int k = 0; k < 3; ++k) roots[nroot++] = rr * cos(ph - k * tp) - A / 3.0;
        }
    }
    double best = 0.0, bestv = 0.0;
    bool have = false;
    for (int k = 0; k < nroot; ++k) {
        const double x = polish(c, roots[k]);
        if (!(x > 0.0) || !isfinite(x)) continue;
        const double v = phi_inc(c, x);
        if (!have || v < bestv || (v == bestv && x < best)) { best = x; bestv = v; have = true; }
    }
    return have ? best : 0.0;
}

// ---------------------------------------------------------------------------
// per-problem finalisation (one block per problem)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void finalize_kernel(FinArgs fa) {
    __shared__ double red[4];
    __shared__ double tot[8];
    const int prob = blockIdx.x;
    const int count = fa.counts ? fa.counts[prob] : fa.ucount;
    const double *base = fa.partials + (int64_t)prob * fa.pstride * fa.nsum;
    for (int k = 0; k < fa.nsum; ++k) {
        double v = 0.0;
        for (int i = threadIdx.x; i < count; i += 256) v += base[(int64_t)i * fa.nsum + k];
        v = block_sum(v, red);
        if (threadIdx.x == 0) tot[k] = v;
    }
    if (threadIdx.x != 0) return;
    SolveScalars &s = fa.sc[prob];
    const int m1 = fa.m1;
    switch (fa.op) {
        case FIN_INIT:
            s.head = 0; s.count = 0; s.restart = 0; s.frozen = 0; s.gamma = 1.0; s.step = 0.0;
            s.f = 0.0; s.thnorm2 = 0.0; s.tp = 0.0; s.pnorm2 = 0.0;
            break;
        case FIN_F: {  // tot[0] = ||r||^2
            const double f = 0.5 * tot[0] + fa.lam * s.thnorm2;
            s.f = f;
            if (fa.fhist) fa.fhist[prob][fa.t] = f;
            else if (fa.fhist0) fa.fhist0[fa.t] = f;
            break;
        }
        case FIN_F_OUT: {  // plain objective into fout[prob]
            if (fa.fout) fa.fout[prob] = 0.5 * tot[0];
            break;
        }
        case FIN_THNORM:
            s.thnorm2 = tot[0];
            break;
        case FIN_PAIR: {  // tot = (Re<s,y>, Re<y,y>)
            const double sy = tot[0], yy = tot[1];
            s.sy = sy; s.yy = yy;
            if (sy > 0.0 && yy > 0.0 && isfinite(sy) && isfinite(yy) && !s.frozen) {
                s.rho[s.head] = 1.0 / sy;
                s.gamma = sy / yy;
                s.head = (s.head + 1) % m1;
                s.count = min(s.count + 1, m1 - 1);
            }
            break;
        }
        case FIN_ALPHA: {  // alpha_i = rho_i Re<s_i, q>
            const int i = fa.i;
            if (i < s.count) s.alpha[i] = s.rho[ring_slot(s, i, m1)] * tot[0];
            break;
        }
        case FIN_BETA: {  // coefficient alpha_i - rho_i Re<y_i, z>
            const int i = fa.i;
            if (i >= 0 && i < s.count) s.beta_coef = s.alpha[i] - s.rho[ring_slot(s, i, m1)] * tot[0];
            break;
        }
        case FIN_GP: {  // Re<g, p>: restart when not a descent direction
            s.gp = tot[0];
            s.restart = (tot[0] >= 0.0 || !isfinite(tot[0])) ? 1 : 0;
            if (s.restart) { s.count = 0; s.gamma = 1.0; }
            break;
        }
        case FIN_LAMTERMS:  // (Re<theta,p>, ||p||^2)
            s.tp = tot[0];
            s.pnorm2 = tot[1];
            break;
        case FIN_LINE: {  // tot = (Re<r,a>, |a|^2, Re<r,b>, Re<a,b>, |b|^2)
            double c[4];
            c[0] = tot[0] + 2.0 * fa.lam * s.tp;
            c[1] = tot[1] + 2.0 * tot[2] + 2.0 * fa.lam * s.pnorm2;
            c[2] = 3.0 * tot[3];
            c[3] = 2.0 * tot[4];
            for (int k = 0; k < 4; ++k) s.coef[k] = c[k];
            double a = exact_step_dev(c);
            bool bad = !isfinite(a);
            for (int k = 0; k < 4; ++k) bad = bad || !isfinite(c[k]);
            if (bad) s.frozen = 1;
            if (s.frozen) a = 0.0;
            s.step = a;
            break;
        }
        default: break;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_stage_d(const float2 *D, int64_t ns, int64_t nr, float2 *Ds, int64_t ldk,
                          float2 *DHs, int64_t lds, hipStream_t s) {
    dim3 grid((unsigned)((ldk + 31) / 32), (unsigned)((lds + 31) / 32));
    hipLaunchKernelGGL(stage_d_kernel, grid, dim3(256), 0, s, D, ns, nr, Ds, ldk, DHs, lds);
    return hipGetLastError();
}

hipError_t launch_stage_d_split(const float2 *D, int64_t ns, int64_t nr, uint32_t *Dh, uint32_t *Dl, int64_t ldk,
                                uint32_t *DHh, uint32_t *DHl, int64_t lds, hipStream_t s) {
    dim3 grid((unsigned)((ldk + 31) / 32), (unsigned)((lds + 31) / 32));
    hipLaunchKernelGGL(stage_d_split_kernel, grid, dim3(256), 0, s, D, ns, nr, Dh, Dl, ldk, DHh, DHl, lds);
    return hipGetLastError();
}

hipError_t launch_split_transpose(const float2 *r, int64_t ldr, int64_t rows, int64_t cols, uint32_t *th,
                                  uint32_t *tl, int64_t ldt, int batch, int64_t s_r, int64_t s_t, hipStream_t s) {
    if (rows <= 0 || cols <= 0 || batch <= 0) return hipSuccess;
    dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32), (unsigned)batch);
    hipLaunchKernelGGL(split_transpose_kernel, grid, dim3(256), 0, s, r, ldr, rows, cols, th, tl, ldt, s_r, s_t);
    return hipGetLastError();
}

hipError_t launch_zero_pad(uint32_t *base, int64_t ld, int64_t n, int nplanes, int64_t plane_stride, int batch,
                           int64_t batch_stride, hipStream_t s) {
    if (ld <= n || nplanes <= 0 || batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_pad_kernel, dim3((unsigned)ld, (unsigned)nplanes, (unsigned)batch), dim3(128), 0, s, base, ld,
                       n, plane_stride, batch_stride);
    return hipGetLastError();
}

hipError_t launch_copy2d(const float2 *src, int64_t lds, float2 *dst, int64_t ldd, int64_t rows,
                         int64_t cols, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::min<int64_t>((cols + 255) / 256, 64);
    hipLaunchKernelGGL(copy2d_kernel, dim3(gx, (unsigned)rows), dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
    return hipGetLastError();
}

hipError_t launch_permute_cols(const float2 *in, const int64_t *perm, float2 *out, int64_t rows,
                               int64_t cols, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::min<int64_t>((cols + 255) / 256, 64);
    hipLaunchKernelGGL(permute_kernel, dim3(gx, (unsigned)rows), dim3(256), 0, s, in, perm, out, rows, cols);
    return hipGetLastError();
}

#define SEGS_LAUNCH(kern, nseg, s, ...)                                              \
    do {                                                                             \
        if ((nseg) <= 0) return hipSuccess;                                          \
        hipLaunchKernelGGL(kern, dim3((unsigned)(nseg)), dim3(256), 0, s, __VA_ARGS__); \
        return hipGetLastError();                                                    \
    } while (0)

hipError_t launch_pair(const VecSeg *segs, int nseg, const float *gnew, const float *gprev, float *Yb,
                       const float *Sb, int64_t stride2, const SolveScalars *sc, double *part, hipStream_t s) {
    SEGS_LAUNCH(pair_kernel, nseg, s, segs, gnew, gprev, Yb, Sb, stride2, sc, part);
}
hipError_t launch_twoloop1(const VecSeg *segs, int nseg, int i, int m1, float *q, const float *g,
                           const float *Sb, const float *Yb, int64_t stride2, const SolveScalars *sc,
                           double *part, hipStream_t s) {
    SEGS_LAUNCH(twoloop1_kernel, nseg, s, segs, i, m1, q, g, Sb, Yb, stride2, sc, part);
}
hipError_t launch_twoloop2(const VecSeg *segs, int nseg, int start, int last, int iu, int inext, int m1,
                           const float *q, float *z, float *p, const float *g, const float *Sb,
                           const float *Yb, int64_t stride2, const SolveScalars *sc, double *part,
                           hipStream_t s) {
    SEGS_LAUNCH(twoloop2_kernel, nseg, s, segs, start, last, iu, inext, m1, q, z, p, g, Sb, Yb, stride2, sc, part);
}
hipError_t launch_restart(const VecSeg *segs, int nseg, int force, float *p, const float *g,
                          const SolveScalars *sc, hipStream_t s) {
    SEGS_LAUNCH(restart_kernel, nseg, s, segs, force, p, g, sc);
}
hipError_t launch_reg_grad(const VecSeg *segs, int nseg, float *g, const float *th, float lam2, hipStream_t s) {
    SEGS_LAUNCH(reg_grad_kernel, nseg, s, segs, g, th, lam2);
}
hipError_t launch_dot2(const VecSeg *segs, int nseg, const float *x0, const float *y0, const float *x1,
                       const float *y1, double *part, hipStream_t s) {
    SEGS_LAUNCH(dot2_kernel, nseg, s, segs, x0, y0, x1, y1, part);
}
hipError_t launch_theta_update(const VecSeg *segs, int nseg, float *th, const float *p, float *Sb,
                               int64_t stride2, const SolveScalars *sc, double *part, hipStream_t s) {
    SEGS_LAUNCH(theta_update_kernel, nseg, s, segs, th, p, Sb, stride2, sc, part);
}
hipError_t launch_resid_update(const VecSeg *segs, int nseg, float *r, const float *a, const float *b,
                               const SolveScalars *sc, double *part, hipStream_t s) {
    SEGS_LAUNCH(resid_update_kernel, nseg, s, segs, r, a, b, sc, part);
}
hipError_t launch_finalize(const FinArgs &fa, int nprob, hipStream_t s) {
    if (nprob <= 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)nprob), dim3(256), 0, s, fa);
    return hipGetLastError();
}

}  // namespace tlr
