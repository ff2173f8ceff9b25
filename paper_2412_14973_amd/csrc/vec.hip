// Memory-bound kernels: staging of D, column permutation (eq. axb_sd), and the
// optimiser's vector / scalar work (L-BFGS two-loop recursion, exact line
// search, updates). All reductions are FP64, deterministic (fixed-order
// per-segment partials, then one fixed-order tree per problem), with no
// atomics. Scalars never leave the device.
#include "common.hpp"
#include "exact_step.hpp"
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
    for (int64_t r = blockIdx.y; r < rows; r += gridDim.y)
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += (int64_t)gridDim.x * blockDim.x)
            dst[r * ldd + c] = src[r * lds + c];
}

// out[r, c] = in[r, perm[c]]; a perm entry outside [0, cols) gives a zero column and sets *bad
__global__ void permute_kernel(const float2 *__restrict__ in, const int64_t *__restrict__ perm,
                               float2 *__restrict__ out, int64_t rows, int64_t cols, int32_t *__restrict__ bad) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < cols; c += (int64_t)gridDim.x * blockDim.x) {
        const int64_t q = perm[c];
        const bool ok = q >= 0 && q < cols;
        if (!ok && bad && blockIdx.y == 0) *bad = 1;
        for (int64_t r = blockIdx.y; r < rows; r += gridDim.y)
            out[r * cols + c] = ok ? in[r * cols + q] : make_float2(0.f, 0.f);
    }
}

// zero `words` 32-bit words at p (16-byte stores over the aligned body)
__global__ void fill_zero_kernel(uint32_t *__restrict__ p, int64_t words) {
    const int64_t mis = (int64_t)((16 - ((uintptr_t)p & 15)) & 15) / 4;   // words before a 16-byte boundary
    const int64_t lead = mis < words ? mis : words;
    const int64_t nvec = (words - lead) / 4;
    uint4 *v = reinterpret_cast<uint4 *>(p + lead);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t i = t; i < nvec; i += stride) v[i] = make_uint4(0u, 0u, 0u, 0u);
    if (t < lead) p[t] = 0u;
    const int64_t tail = lead + 4 * nvec;
    if (t < words - tail) p[tail + t] = 0u;
}

// ---------------------------------------------------------------------------
// segment helpers
// ---------------------------------------------------------------------------
}  // namespace
// wave-wide FP64 sum of the ROCm device library (DPP row shifts and lane reads, fixed order, no LDS)
extern "C" __device__ double __ockl_wfred_add_f64(double);
namespace {

__device__ __forceinline__ double wave_sum64(double v) { return __ockl_wfred_add_f64(v); }

__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum64(v);
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

// A thread's share of a segment: float4 chunks t, t + 256, t + 512, t + 768 (VEC_CH = 4096 floats).
// Segment offsets are multiples of 4 floats and lengths are even (complex entries); a problem's
// theta span is padded to an even number of complex entries, so the float4 that holds a segment's
// ragged end lies inside the span. Loads and stores are buffer instructions over the segment
// rounded up to whole float4s: chunks past the end read 0 and are not written (no branches, all
// loads of a thread in flight together); the two floats past an odd end are read as 0 and written
// back as the kernel's result for 0 inputs, inside the padding.
constexpr int VQ = VEC_CH / 1024;
struct V16 { float v[4 * VQ]; };

typedef unsigned int vu32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __amdgpu_buffer_rsrc_t seg_rsrc(const float *base, const VecSeg &sg) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)(base + sg.off), (short)0, ((sg.n + 3) & ~3) * 4, 0x00020000);
}

__device__ __forceinline__ V16 ld16(const float *__restrict__ base, const VecSeg &sg) {
    const __amdgpu_buffer_rsrc_t rs = seg_rsrc(base, sg);
    V16 r;
#pragma unroll
    for (int q = 0; q < VQ; ++q) {
        const int e = (threadIdx.x + 256 * q) * 4;
        const vu32x4 x = __builtin_amdgcn_raw_buffer_load_b128(rs, e * 4, 0, 0);
        const bool full = e + 4 <= sg.n;   // else at most the first two floats are in the segment
        r.v[4 * q] = __uint_as_float(x.x);
        r.v[4 * q + 1] = __uint_as_float(x.y);
        r.v[4 * q + 2] = full ? __uint_as_float(x.z) : 0.f;
        r.v[4 * q + 3] = full ? __uint_as_float(x.w) : 0.f;
    }
    return r;
}

__device__ __forceinline__ void st16(float *__restrict__ base, const VecSeg &sg, const V16 &r) {
    const __amdgpu_buffer_rsrc_t rs = seg_rsrc(base, sg);
#pragma unroll
    for (int q = 0; q < VQ; ++q) {
        const int e = (threadIdx.x + 256 * q) * 4;
        const vu32x4 x = {__float_as_uint(r.v[4 * q]), __float_as_uint(r.v[4 * q + 1]),
                          __float_as_uint(r.v[4 * q + 2]), __float_as_uint(r.v[4 * q + 3])};
        __builtin_amdgcn_raw_buffer_store_b128(x, rs, e * 4, 0, 0);
    }
}

__device__ __forceinline__ double dot16(const V16 &x, const V16 &y) {
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < 4 * VQ; ++u) a = fma((double)x.v[u], (double)y.v[u], a);
    return a;
}

// N block sums at once (thread 0 gets the totals); same fixed order as block_sum
template <int N>
__device__ __forceinline__ void block_sums(double (&v)[N], double *red) {
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wave_sum64(v[k]);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) red[4 * k + w] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < N; ++k) v[k] = ((red[4 * k] + red[4 * k + 1]) + red[4 * k + 2]) + red[4 * k + 3];
    __syncthreads();
}

// Gram pass of the vector-free L-BFGS direction. With h = head (the slot of the newest step s_h,
// written by the previous update): y_h = g - g_prev into Y[h]; then the real inner products of the
// new vectors (s_h, y_h, g) with every stored one. Partials per segment, 6 per ring slot j:
//   j == h : <s_h,s_h> <s_h,y_h> <y_h,y_h> <g,s_h> <g,y_h> <g,g>
//   j valid: <s_j,s_h> <s_j,y_h> <s_j,g>   <y_j,s_h> <y_j,y_h> <y_j,g>
//   else   : zeros
__global__ __launch_bounds__(256) void gram_kernel(const VecSeg *__restrict__ segs, int m1,
                                                   const float *__restrict__ g, const float *__restrict__ gprev,
                                                   float *__restrict__ Yb, const float *__restrict__ Sb,
                                                   int64_t stride2, const SolveScalars *__restrict__ sc,
                                                   double *__restrict__ part) {
    __shared__ double red[4 * 6];
    const VecSeg sg = segs[blockIdx.x];
    const SolveScalars &s = sc[sg.prob];
    const int h = s.head, count = s.count;
    double *pp = part + (int64_t)sg.part * 6 * m1;
    const V16 vg = ld16(g, sg);
    const V16 vs = ld16(Sb + h * stride2, sg);
    V16 vy = ld16(gprev, sg);
    // the first held pair is loaded with the new vectors (an empty range when there is none)
    VecSeg sg0 = sg;
    if (count == 0) sg0.n = 0;
    const int j0 = ring_slot(s, 0, m1);
    V16 sj = ld16(Sb + j0 * stride2, sg0);
    V16 yj = ld16(Yb + j0 * stride2, sg0);
#pragma unroll
    for (int u = 0; u < 4 * VQ; ++u) vy.v[u] = vg.v[u] - vy.v[u];
    st16(Yb + h * stride2, sg, vy);
    {
        double a[6] = {dot16(vs, vs), dot16(vs, vy), dot16(vy, vy), dot16(vg, vs), dot16(vg, vy), dot16(vg, vg)};
        block_sums<6>(a, red);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < 6; ++k) pp[6 * h + k] = a[k];
    }
    // the held pairs, each one's loads issued before the block reduction of the previous one
    for (int i = 0; i < count; ++i) {
        const int j = ring_slot(s, i, m1);
        VecSeg sgn = sg;   // past the last pair: an empty range, the loads return 0 and move no data
        if (i + 1 >= count) sgn.n = 0;
        const int jn = ring_slot(s, i + 1, m1);
        const V16 sn = ld16(Sb + jn * stride2, sgn);
        const V16 yn = ld16(Yb + jn * stride2, sgn);
        double a[6] = {dot16(sj, vs), dot16(sj, vy), dot16(sj, vg), dot16(yj, vs), dot16(yj, vy), dot16(yj, vg)};
        block_sums<6>(a, red);
        if (threadIdx.x == 0)
#pragma unroll
            for (int k = 0; k < 6; ++k) pp[6 * j + k] = a[k];
        sj = sn;
        yj = yn;
    }
    if (threadIdx.x < 6 * m1) {   // slots that are neither h nor valid
        const int j = threadIdx.x / 6;
        bool used = (j == h);
        for (int i = 0; i < count; ++i) used = used || (ring_slot(s, i, m1) == j);
        if (!used) pp[threadIdx.x] = 0.0;
    }
}

// p = sum_b c_b v_b over the active basis {g, s_j, y_j : valid j} with the coefficients that the
// finalisation of the Gram pass left in coef[] (index 2 m1 for g, j for s_j, m1 + j for y_j).
__global__ __launch_bounds__(256) void combine_kernel(const VecSeg *__restrict__ segs, int m1,
                                                      float *__restrict__ p, const float *__restrict__ g,
                                                      const float *__restrict__ Sb, const float *__restrict__ Yb,
                                                      int64_t stride2, const SolveScalars *__restrict__ sc,
                                                      const double *__restrict__ coef, int64_t cstride) {
    const VecSeg sg = segs[blockIdx.x];
    const SolveScalars &s = sc[sg.prob];
    const double *c = coef + (int64_t)sg.prob * cstride;
    const int count = s.count;
    // FP32 vectors and FP32 accumulation (the coefficients come from the FP64 two-loop on the Gram
    // matrix and are rounded once to FP32), fixed order: g, then the pairs newest first
    V16 r;
    {
        const V16 vg = ld16(g, sg);
        const float cg = (float)c[2 * m1];
#pragma unroll
        for (int u = 0; u < 4 * VQ; ++u) r.v[u] = cg * vg.v[u];
    }
    for (int i = 0; i < count; ++i) {
        const int j = ring_slot(s, i, m1);
        const float cs = (float)c[j], cy = (float)c[m1 + j];
        const V16 sj = ld16(Sb + j * stride2, sg);
        const V16 yj = ld16(Yb + j * stride2, sg);
#pragma unroll
        for (int u = 0; u < 4 * VQ; ++u) r.v[u] = fmaf(cy, yj.v[u], fmaf(cs, sj.v[u], r.v[u]));
    }
    st16(p, sg, r);
}

// p = -g (steepest descent: first iteration, restarts of plain gradient descent)
__global__ __launch_bounds__(256) void negate_kernel(const VecSeg *__restrict__ segs, float *__restrict__ p,
                                                     const float *__restrict__ g) {
    const VecSeg sg = segs[blockIdx.x];
    V16 v = ld16(g, sg);
#pragma unroll
    for (int u = 0; u < 4 * VQ; ++u) v.v[u] = -v.v[u];
    st16(p, sg, v);
}

// g += 2 lambda (theta - c)   (c = 0 when cen is NULL)
__global__ __launch_bounds__(256) void reg_grad_kernel(const VecSeg *__restrict__ segs, float *__restrict__ g,
                                                       const float *__restrict__ th, const float *__restrict__ cen,
                                                       float lam2) {
    const VecSeg sg = segs[blockIdx.x];
    V16 v = ld16(g, sg);
    V16 t = ld16(th, sg);
    if (cen) {
        const V16 c = ld16(cen, sg);
#pragma unroll
        for (int u = 0; u < 4 * VQ; ++u) t.v[u] -= c.v[u];
    }
#pragma unroll
    for (int u = 0; u < 4 * VQ; ++u) v.v[u] += lam2 * t.v[u];
    st16(g, sg, v);
}

// penalty sums with d = theta - c (c = 0 when cen is NULL):
//   p == NULL: partial ||d||^2 ;   else partials Re<d, p>, ||p||^2
__global__ __launch_bounds__(256) void pen_kernel(const VecSeg *__restrict__ segs, const float *__restrict__ th,
                                                  const float *__restrict__ cen, const float *__restrict__ p,
                                                  double *__restrict__ part) {
    __shared__ double red[4 * 2];
    const VecSeg sg = segs[blockIdx.x];
    V16 d = ld16(th, sg);
    if (cen) {
        const V16 c = ld16(cen, sg);
#pragma unroll
        for (int u = 0; u < 4 * VQ; ++u) d.v[u] -= c.v[u];
    }
    if (!p) {
        double a[1] = {dot16(d, d)};
        block_sums<1>(a, red);
        if (threadIdx.x == 0) part[sg.part] = a[0];
        return;
    }
    const V16 vp = ld16(p, sg);
    double a[2] = {dot16(d, vp), dot16(vp, vp)};
    block_sums<2>(a, red);
    if (threadIdx.x == 0) { part[2 * sg.part] = a[0]; part[2 * sg.part + 1] = a[1]; }
}

// ADMM split and scaled dual (init: z = theta, u = 0), then the next X-update's center c = z - u:
//   z = (theta + u) * scale with scale = 1 / (1 + 2 lambda / rho);  u = u + theta - z
__global__ __launch_bounds__(256) void admm_update_kernel(const VecSeg *__restrict__ segs, int init,
                                                          const float *__restrict__ th, float *__restrict__ z,
                                                          float *__restrict__ uu, float *__restrict__ cen,
                                                          float scale) {
    const VecSeg sg = segs[blockIdx.x];
    const V16 t = ld16(th, sg);
    V16 vz, vu;
    if (init) {
        vz = t;
#pragma unroll
        for (int q = 0; q < 4 * VQ; ++q) vu.v[q] = 0.f;
    } else {
        vu = ld16(uu, sg);
#pragma unroll
        for (int q = 0; q < 4 * VQ; ++q) {
            vz.v[q] = (t.v[q] + vu.v[q]) * scale;
            vu.v[q] = vu.v[q] + t.v[q] - vz.v[q];
        }
    }
    st16(z, sg, vz);
    st16(uu, sg, vu);
#pragma unroll
    for (int q = 0; q < 4 * VQ; ++q) vz.v[q] -= vu.v[q];
    st16(cen, sg, vz);
}

// theta += step p ; S[head] = step p ; partial ||theta - c||^2 (c = 0 when cen is NULL)
__global__ __launch_bounds__(256) void theta_update_kernel(const VecSeg *__restrict__ segs, float *__restrict__ th,
                                                           const float *__restrict__ p, float *__restrict__ Sb,
                                                           int64_t stride2, const float *__restrict__ cen,
                                                           const SolveScalars *__restrict__ sc,
                                                           double *__restrict__ part) {
    __shared__ double red[4];
    const VecSeg sg = segs[blockIdx.x];
    // the vector loads need the segment only: they are in flight while the step is read
    V16 v = ld16(th, sg);
    V16 sp = ld16(p, sg);
    const SolveScalars &s = sc[sg.prob];
    const float a = (float)s.step;
    const bool frozen = s.frozen != 0;   // a non-finite step froze this problem: theta stays as is
#pragma unroll
    for (int u = 0; u < 4 * VQ; ++u) {
        sp.v[u] = a * sp.v[u];
        const float nv = v.v[u] + sp.v[u];
        v.v[u] = frozen ? v.v[u] : nv;
    }
    if (!frozen) {
        st16(th, sg, v);
        if (Sb) st16(Sb + s.head * stride2, sg, sp);
    }
    if (cen) {
        const V16 c = ld16(cen, sg);
#pragma unroll
        for (int u = 0; u < 4 * VQ; ++u) v.v[u] -= c.v[u];
    }
    double acc[1] = {dot16(v, v)};
    block_sums<1>(acc, red);
    if (threadIdx.x == 0) part[sg.part] = acc[0];
}

// r += step a + step^2 b ; partial ||r||^2
__global__ __launch_bounds__(256) void resid_update_kernel(const VecSeg *__restrict__ segs, float *__restrict__ r,
                                                           const float *__restrict__ a, const float *__restrict__ b,
                                                           const SolveScalars *__restrict__ sc,
                                                           double *__restrict__ part) {
    __shared__ double red[4];
    const VecSeg sg = segs[blockIdx.x];
    // the vector loads need the segment only: they are in flight while the step is read
    V16 v = ld16(r, sg);
    const V16 va = ld16(a, sg), vb = ld16(b, sg);
    const SolveScalars &s = sc[sg.prob];
    // a non-finite step froze this problem: r stays as is (the update is discarded, nothing written)
    const bool frozen = s.frozen != 0;
    const float al = (float)s.step;
    const float al2 = (float)(s.step * s.step);
#pragma unroll
    for (int u = 0; u < 4 * VQ; ++u) {
        const float nv = v.v[u] + (al * va.v[u] + al2 * vb.v[u]);
        v.v[u] = frozen ? v.v[u] : nv;
    }
    if (!frozen) st16(r, sg, v);
    double acc[1] = {dot16(v, v)};
    block_sums<1>(acc, red);
    if (threadIdx.x == 0) part[sg.part] = acc[0];
}

// ---------------------------------------------------------------------------
// per-problem finalisation (one block per problem)
// ---------------------------------------------------------------------------
// the scalar work of one problem (thread 0); G: the staged Gram matrix and coefficients (FIN_GRAM)
__device__ __forceinline__ void finalize_scalars(const FinArgs &fa, int prob, const double *tot, double *Gs) {
    SolveScalars &s = fa.sc[prob];
    const int m1 = fa.m1;
    switch (fa.op) {
        case FIN_INIT:
            s.head = 0; s.count = 0; s.restart = 0; s.frozen = 0; s.gamma = 1.0; s.step = 0.0;
            s.f = 0.0; s.fdata = 0.0; s.thnorm2 = 0.0; s.tp = 0.0; s.pnorm2 = 0.0;
            break;
        case FIN_F: {  // tot[0] = ||r||^2
            const double f = 0.5 * tot[0] + fa.lam * s.thnorm2;
            s.f = f;
            s.fdata = 0.5 * tot[0];
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
        case FIN_RECORD:  // data misfit of the tracked residual into the history at index t
            if (fa.fhist) fa.fhist[prob][fa.t] = s.fdata;
            else if (fa.fhist0) fa.fhist0[fa.t] = s.fdata;
            break;
        case FIN_RESET:  // fresh pair memory (a new sub-problem starts from the current theta)
            s.head = 0; s.count = 0; s.restart = 0; s.gamma = 1.0;
            break;
        case FIN_GRAM: {  // Gram entries of the newest pair and of g; direction coefficients
            const int nb = 2 * m1 + 1, ig = 2 * m1;
            double *G = Gs;   // nb x nb, then nb coefficients
            double *cf = G + nb * nb;
            const int h = s.head;
            const double *th = tot + 6 * h;
            const double sy = th[1], yy = th[2];
            // g against the pairs already held (before the newest one is taken in)
            for (int i = 0; i < s.count; ++i) {
                const int j = ring_slot(s, i, m1);
                G[ig * nb + j] = G[j * nb + ig] = tot[6 * j + 2];
                G[ig * nb + m1 + j] = G[(m1 + j) * nb + ig] = tot[6 * j + 5];
            }
            G[ig * nb + ig] = th[5];
            s.sy = sy; s.yy = yy;
            if (sy > 0.0 && yy > 0.0 && isfinite(sy) && isfinite(yy) && !s.frozen) {
                for (int i = 0; i < s.count; ++i) {
                    const int j = ring_slot(s, i, m1);
                    const double *tj = tot + 6 * j;
                    G[j * nb + h] = G[h * nb + j] = tj[0];
                    G[j * nb + m1 + h] = G[(m1 + h) * nb + j] = tj[1];
                    G[(m1 + j) * nb + h] = G[h * nb + m1 + j] = tj[3];
                    G[(m1 + j) * nb + m1 + h] = G[(m1 + h) * nb + m1 + j] = tj[4];
                }
                G[h * nb + h] = th[0];
                G[h * nb + m1 + h] = G[(m1 + h) * nb + h] = sy;
                G[(m1 + h) * nb + m1 + h] = yy;
                G[ig * nb + h] = G[h * nb + ig] = th[3];
                G[ig * nb + m1 + h] = G[(m1 + h) * nb + ig] = th[4];
                s.rho[h] = 1.0 / sy;
                s.gamma = sy / yy;
                s.head = (h + 1) % m1;
                s.count = min(s.count + 1, m1 - 1);
            }
            // two-loop recursion on coefficient vectors over the basis (s_j, y_j, g):
            // q = sum_b d_b v_b, so <v_a, q> = sum_b G_ab d_b
            for (int b2 = 0; b2 < nb; ++b2) cf[b2] = 0.0;
            cf[ig] = 1.0;
            const int cnt = s.count;
            auto dotG = [&](int a_) {
                double v = G[a_ * nb + ig] * cf[ig];
                for (int i = 0; i < cnt; ++i) {
                    const int j = ring_slot(s, i, m1);
                    v += G[a_ * nb + j] * cf[j] + G[a_ * nb + m1 + j] * cf[m1 + j];
                }
                return v;
            };
            for (int i = 0; i < cnt; ++i) {   // newest first
                const int j = ring_slot(s, i, m1);
                s.alpha[i] = s.rho[j] * dotG(j);
                cf[m1 + j] -= s.alpha[i];
            }
            if (cnt > 0)
                for (int b2 = 0; b2 < nb; ++b2) cf[b2] *= s.gamma;
            for (int i = cnt - 1; i >= 0; --i) {   // oldest first
                const int j = ring_slot(s, i, m1);
                const double beta = s.rho[j] * dotG(m1 + j);
                cf[j] += s.alpha[i] - beta;
            }
            for (int b2 = 0; b2 < nb; ++b2) cf[b2] = -cf[b2];
            const double gp = dotG(ig);
            s.gp = gp;
            s.restart = (gp >= 0.0 || !isfinite(gp)) ? 1 : 0;
            if (s.restart) {   // not a descent direction: p = -g and the history is dropped
                s.count = 0;
                s.gamma = 1.0;
                for (int b2 = 0; b2 < nb; ++b2) cf[b2] = 0.0;
                cf[ig] = -1.0;
                s.gp = -G[ig * nb + ig];
            }
            break;
        }
        case FIN_LAMTERMS:  // (Re<theta - c, p>, ||p||^2)
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

// The scalar work runs on one thread and is a chain of dependent steps, so everything it touches sits
// in LDS first: the partial sums are reduced by the four waves at once (wave w takes sums w, w + 4,
// ...: lanes stride over the slots, then one DPP wave reduction, a fixed order), and the Gram pass
// stages the problem's Gram matrix and coefficient vector, which are written back afterwards.
constexpr int FIN_NB = 2 * (MAX_LBFGS_M + 1) + 1;
__global__ __launch_bounds__(256) void finalize_kernel(FinArgs fa) {
    __shared__ double tot[6 * (MAX_LBFGS_M + 1)];
    __shared__ double sG[FIN_NB * FIN_NB + FIN_NB];
    const int prob = blockIdx.x;
    const int count = fa.counts ? fa.counts[prob] : fa.ucount;
    const double *base = fa.partials + (int64_t)prob * fa.pstride * fa.nsum;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    for (int k = wv; k < fa.nsum; k += 4) {
        double v = 0.0;
        for (int i = lane; i < count; i += 64) v += base[(int64_t)i * fa.nsum + k];
        v = wave_sum64(v);
        if (lane == 0) tot[k] = v;
    }
    const int m1 = fa.m1;
    const int gwords = (2 * m1 + 1) * (2 * m1 + 1) + 2 * m1 + 1;
    double *Gg = fa.op == FIN_GRAM ? fa.gram + (int64_t)prob * fa.gstride : nullptr;
    if (Gg)
        for (int i = threadIdx.x; i < gwords; i += 256) sG[i] = Gg[i];
    __syncthreads();
    if (threadIdx.x == 0) finalize_scalars(fa, prob, tot, sG);
    if (Gg) {
        __syncthreads();
        for (int i = threadIdx.x; i < gwords; i += 256) Gg[i] = sG[i];
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
    const unsigned gy = (unsigned)std::min<int64_t>(rows, 65535);
    hipLaunchKernelGGL(copy2d_kernel, dim3(gx, gy), dim3(256), 0, s, src, lds, dst, ldd, rows, cols);
    return hipGetLastError();
}

hipError_t launch_permute_cols(const float2 *in, const int64_t *perm, float2 *out, int64_t rows,
                               int64_t cols, int32_t *bad, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::min<int64_t>((cols + 255) / 256, 64);
    const unsigned gy = (unsigned)std::min<int64_t>(rows, 65535);
    hipLaunchKernelGGL(permute_kernel, dim3(gx, gy), dim3(256), 0, s, in, perm, out, rows, cols, bad);
    return hipGetLastError();
}

hipError_t launch_fill_zero(void *p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (((uintptr_t)p & 3) || (bytes & 3)) return hipErrorInvalidValue;
    const int64_t words = (int64_t)(bytes / 4);
    const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((words / 4 + 255) / 256, 4096));
    hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(256), 0, s, (uint32_t *)p, words);
    return hipGetLastError();
}

#define SEGS_LAUNCH(kern, nseg, s, ...)                                              \
    do {                                                                             \
        if ((nseg) <= 0) return hipSuccess;                                          \
        hipLaunchKernelGGL(kern, dim3((unsigned)(nseg)), dim3(256), 0, s, __VA_ARGS__); \
        return hipGetLastError();                                                    \
    } while (0)

hipError_t launch_gram(const VecSeg *segs, int nseg, int m1, const float *g, const float *gprev, float *Yb,
                       const float *Sb, int64_t stride2, const SolveScalars *sc, double *part, hipStream_t s) {
    SEGS_LAUNCH(gram_kernel, nseg, s, segs, m1, g, gprev, Yb, Sb, stride2, sc, part);
}
hipError_t launch_combine(const VecSeg *segs, int nseg, int m1, float *p, const float *g, const float *Sb,
                          const float *Yb, int64_t stride2, const SolveScalars *sc, const double *coef,
                          int64_t cstride, hipStream_t s) {
    SEGS_LAUNCH(combine_kernel, nseg, s, segs, m1, p, g, Sb, Yb, stride2, sc, coef, cstride);
}
hipError_t launch_negate(const VecSeg *segs, int nseg, float *p, const float *g, hipStream_t s) {
    SEGS_LAUNCH(negate_kernel, nseg, s, segs, p, g);
}
hipError_t launch_reg_grad(const VecSeg *segs, int nseg, float *g, const float *th, const float *cen, float lam2,
                           hipStream_t s) {
    SEGS_LAUNCH(reg_grad_kernel, nseg, s, segs, g, th, cen, lam2);
}
hipError_t launch_pen(const VecSeg *segs, int nseg, const float *th, const float *cen, const float *p, double *part,
                      hipStream_t s) {
    SEGS_LAUNCH(pen_kernel, nseg, s, segs, th, cen, p, part);
}
hipError_t launch_admm_update(const VecSeg *segs, int nseg, int init, const float *th, float *z, float *u, float *cen,
                              float scale, hipStream_t s) {
    SEGS_LAUNCH(admm_update_kernel, nseg, s, segs, init, th, z, u, cen, scale);
}
hipError_t launch_theta_update(const VecSeg *segs, int nseg, float *th, const float *p, float *Sb,
                               int64_t stride2, const float *cen, const SolveScalars *sc, double *part,
                               hipStream_t s) {
    SEGS_LAUNCH(theta_update_kernel, nseg, s, segs, th, p, Sb, stride2, cen, sc, part);
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
