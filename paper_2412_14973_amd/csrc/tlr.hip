// Tile low-rank matrix product D C(theta) without the dense X (the paper's
// Discussion section names it as the way to cut the cost of the dense products).
//
// Column block j of D X is sum_i D_:,i X_ij with every tile a product of two
// factors, X_ij = A_ij B_ij:
//   i > j: A = L_ij, B = R_ij;   i < j: A = R_ji^T, B = L_ji^T  (X_ij = X_ji^T);
//   i = j: A = Q_ii, B = Q_ii^T, or (dense) A = I, B = (Z_ii + Z_ii^T)/2.
// Stage 1 (one GEMM per tile row i): P_i = D_:,i [A_i0 | A_i1 | ...].
// Stage 2 (one GEMM per tile column j): r_:,j = [P_0j | P_1j | ...] [B_0j; B_1j; ...] - U_:,j,
// where P_ij is the column block of P_i that multiplies B_ij. The kernels below pack the
// factor blocks into the GEMM operands and gather the P blocks; the products themselves run
// on the FP32 MFMA GEMM. The solver's tile forms of the line search and the gradient use the
// same factorisation (their stage 1 stores its blocks regrouped in its epilogue instead of a
// gather); for them this file also holds the summation of the gradient's partial planes into
// the factor gradients and the update of the carried theta half of stage 1.
#include <algorithm>

#include "common.hpp"
#include "tlr.hpp"

namespace tlr {
namespace {

// one packed block per work item: dst[r * ldd + c] = op(src) for r < rows, c < cols
__global__ __launch_bounds__(256) void tlr_pack_kernel(const PackItem *__restrict__ items,
                                                       const float2 *__restrict__ theta,
                                                       const float2 *__restrict__ theta2,
                                                       float2 *__restrict__ dst_base) {
    const PackItem it = items[blockIdx.x];
    float2 *dst = dst_base + it.dst;
    const float2 *src = (it.from ? theta2 : theta) + it.src;
    if (it.op == PACK_TRANS || it.op == PACK_CTRANS) {
        // transposes through LDS in 32 x 32 tiles: reads along the source rows, writes along dst rows
        __shared__ float2 tile[32][33];
        const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
        const int ntr = (it.rows + 31) / 32, ntc = (it.cols + 31) / 32;
        const float sgn = it.op == PACK_CTRANS ? -1.f : 1.f;
        for (int q = blockIdx.y; q < ntr * ntc; q += gridDim.y) {
            const int r0 = (q / ntc) * 32, c0 = (q % ntc) * 32;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = c0 + ty + 8 * j, r = r0 + tx;
                if (c < it.cols && r < it.rows) tile[ty + 8 * j][tx] = src[(int64_t)c * it.lds + r];
            }
            __syncthreads();
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = r0 + ty + 8 * j, c = c0 + tx;
                if (c < it.cols && r < it.rows) {
                    const float2 v = tile[tx][ty + 8 * j];
                    dst[(int64_t)r * it.ldd + c] = make_float2(v.x, sgn * v.y);
                }
            }
            __syncthreads();
        }
        return;
    }
    const int64_t n = (int64_t)it.rows * it.cols;
    for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.y * blockDim.x) {
        const int r = (int)(e / it.cols), c = (int)(e % it.cols);
        float2 v;
        switch (it.op) {
            case PACK_COPY: v = src[(int64_t)r * it.lds + c]; break;            // src rows x cols
            case PACK_CONJ: v = src[(int64_t)r * it.lds + c]; v.y = -v.y; break;
            case PACK_IDENT: v = make_float2(r == c ? 1.f : 0.f, 0.f); break;
            default: {                                                           // (Z + Z^T)/2
                const float2 a = src[(int64_t)r * it.lds + c], b = src[(int64_t)c * it.lds + r];
                v = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y + b.y));
            }
        }
        dst[(int64_t)r * it.ldd + c] = v;
    }
}

// Pcol_j[:, roff + c] = P_i[:, coff + c] for c < k, every source row (lds rows)
__global__ __launch_bounds__(256) void tlr_gather_kernel(const GatherItem *__restrict__ items,
                                                         const float2 *__restrict__ P, float2 *__restrict__ Pcol,
                                                         int64_t rows) {
    const GatherItem it = items[blockIdx.x];
    for (int64_t s = blockIdx.y; s < rows; s += gridDim.y)
        for (int c = threadIdx.x; c < it.k; c += blockDim.x)
            Pcol[it.dst + s * it.ldd + c] = P[it.src + s * it.lds + c];
}

// Gradient blocks of the tile form from the partial planes of its two products (fixed summation
// order: the H1 planes, then the H2 planes) in 32 x 32 tiles: every thread reads along the rows of H
// (c fastest); transposed blocks pass through LDS so that they are written along the rows of g too.
__global__ __launch_bounds__(256) void tlr_grad_kernel(const TGradItem *__restrict__ items,
                                                       const float2 *__restrict__ H1,
                                                       const float2 *__restrict__ H2, int nparts,
                                                       int64_t part_stride, int64_t ldh, int conj1,
                                                       float2 *__restrict__ g) {
    __shared__ float2 tile[32][33];
    const TGradItem it = items[blockIdx.x];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    const int ntr = (it.rows + 31) / 32, ntc = (it.cols + 31) / 32;
    for (int q = blockIdx.y; q < ntr * ntc; q += gridDim.y) {
        const int r0 = (q / ntc) * 32, c0 = (q % ntc) * 32;
        float2 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int r = r0 + ty + 8 * j, c = c0 + tx;
            float sx = 0.f, sy = 0.f;
            if (r < it.rows && c < it.cols) {
                const int64_t h = it.src + (int64_t)r * ldh + c;
                for (int p = 0; p < nparts; ++p) {
                    const float2 a = H1[h + p * part_stride];
                    sx += a.x;
                    sy += a.y;
                }
                if (conj1) sy = -sy;
                for (int p = 0; p < nparts; ++p) {
                    const float2 a = H2[h + p * part_stride];
                    sx += a.x;
                    sy += a.y;
                }
            }
            v[j] = make_float2(sx, sy);
        }
        if (!it.trans) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int r = r0 + ty + 8 * j, c = c0 + tx;
                if (r < it.rows && c < it.cols) g[it.dst + (int64_t)r * it.ldd + c] = v[j];
            }
            continue;   // uniform per block: it.trans is the item's
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) tile[ty + 8 * j][tx] = v[j];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 4; ++j) {   // g[dst + c * ldd + r], r fastest
            const int c = c0 + ty + 8 * j, r = r0 + tx;
            if (r < it.rows && c < it.cols) g[it.dst + (int64_t)c * it.ldd + r] = tile[tx][ty + 8 * j];
        }
        __syncthreads();
    }
}

// Pcol theta half += step * direction half (float4 = two complex per thread; half_cols and ld even)
__global__ __launch_bounds__(256) void tlr_paxpy_kernel(float2 *__restrict__ Pcol, int nt, int64_t entry_stride,
                                                        int64_t rows, int64_t ld, int64_t half_cols,
                                                        const SolveScalars *__restrict__ sc) {
    const int e = blockIdx.x;
    const SolveScalars &st = sc[e / nt];
    if (st.frozen) return;   // theta was not updated
    const float a = (float)st.step;
    float2 *base = Pcol + e * entry_stride;
    const int64_t h = half_cols >> 1;   // float4 per row and half
    const int64_t n = rows * h;
    for (int64_t i = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.y * blockDim.x) {
        const int64_t row = i / h, c2 = i - row * h;
        const float4 pv = *reinterpret_cast<const float4 *>(base + row * ld + 2 * c2);
        float4 *tp = reinterpret_cast<float4 *>(base + row * ld + half_cols + 2 * c2);
        float4 tv = *tp;
        tv.x += a * pv.x;
        tv.y += a * pv.y;
        tv.z += a * pv.z;
        tv.w += a * pv.w;
        *tp = tv;
    }
}

}  // namespace

hipError_t launch_tlr_grad(const TGradItem *items, int nitems, const float2 *H1, const float2 *H2, int nparts,
                           int64_t part_stride, int64_t ldh, bool conj1, float2 *g, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    hipLaunchKernelGGL(tlr_grad_kernel, dim3((unsigned)nitems, 8), dim3(256), 0, s, items, H1, H2, nparts,
                       part_stride, ldh, conj1 ? 1 : 0, g);
    return hipGetLastError();
}

hipError_t launch_tlr_paxpy(float2 *Pcol, int nentries, int nt, int64_t entry_stride, int64_t rows, int64_t ld,
                            int64_t half_cols, const SolveScalars *sc, hipStream_t s) {
    if (nentries <= 0 || rows <= 0) return hipSuccess;
    if ((half_cols & 1) || (ld & 1) || (entry_stride & 1)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tlr_paxpy_kernel, dim3((unsigned)nentries, 16), dim3(256), 0, s, Pcol, nt, entry_stride,
                       rows, ld, half_cols, sc);
    return hipGetLastError();
}

hipError_t launch_tlr_pack(const PackItem *items, int nitems, const float2 *theta, float2 *dst, hipStream_t s,
                           const float2 *theta2, int blocks_per_item) {
    if (nitems <= 0) return hipSuccess;
    if (blocks_per_item < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(tlr_pack_kernel, dim3((unsigned)nitems, (unsigned)blocks_per_item), dim3(256), 0, s, items,
                       theta, theta2 ? theta2 : theta, dst);
    return hipGetLastError();
}

hipError_t launch_tlr_gather(const GatherItem *items, int nitems, const float2 *P, float2 *Pcol, int64_t rows,
                             hipStream_t s) {
    if (nitems <= 0 || rows <= 0) return hipSuccess;
    const unsigned gy = (unsigned)std::min<int64_t>(rows, 256);
    hipLaunchKernelGGL(tlr_gather_kernel, dim3((unsigned)nitems, gy), dim3(256), 0, s, items, P, Pcol, rows);
    return hipGetLastError();
}

}  // namespace tlr
