// Operand packing for the tile low-rank product (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace tlr {

enum PackOp : int32_t { PACK_COPY = 0, PACK_TRANS = 1, PACK_IDENT = 2, PACK_SYM = 3, PACK_CONJ = 4, PACK_CTRANS = 5 };

// dst[r * ldd + c] (r < rows, c < cols) from the theta block at src:
// COPY src[r * lds + c]; TRANS src[c * lds + r]; IDENT delta_rc; SYM (src[r][c] + src[c][r]) / 2;
// CONJ conj(src[r * lds + c]); CTRANS conj(src[c * lds + r])
// (from = 1: the block is read from the second source vector, e.g. the search direction p)
struct PackItem {
    int32_t op;
    int32_t rows, cols;
    int32_t from;
    int64_t src, lds;   // theta offset and row pitch of the source block
    int64_t dst, ldd;   // operand-buffer offset and row pitch of the destination
};

// copy k columns (all rows) from P at src (row pitch lds) to Pcol at dst (row pitch ldd)
struct GatherItem {
    int32_t k;
    int32_t pad;
    int64_t src, lds;
    int64_t dst, ldd;
};

// One block of the tile-form gradient: g[dst + r * ldd + c] (or g[dst + c * ldd + r] with trans) =
// sum over the partial planes of H1 (conjugated when conj1) and H2 at src + r * ldh + c, for r < rows,
// c < cols.
struct TGradItem {
    int32_t rows, cols;
    int32_t trans;
    int32_t pad;
    int64_t src, dst, ldd;
};

hipError_t launch_tlr_grad(const TGradItem *items, int nitems, const float2 *H1, const float2 *H2, int nparts,
                           int64_t part_stride, int64_t ldh, bool conj1, float2 *g, hipStream_t s);

// Pcol theta half += step * direction half for every (problem, tile column) of a tile range: rows x
// (nt kpad) per entry at Pcol + e * entry_stride (direction half at column 0, theta half at column
// half_cols, row pitch ld); entry e belongs to problem e / nt, whose step and frozen flag are in sc.
struct SolveScalars;
hipError_t launch_tlr_paxpy(float2 *Pcol, int nentries, int nt, int64_t entry_stride, int64_t rows, int64_t ld,
                            int64_t half_cols, const SolveScalars *sc, hipStream_t s);

// blocks_per_item: workgroups that share one item (grid-stride over its elements or 32 x 32 tiles)
hipError_t launch_tlr_pack(const PackItem *items, int nitems, const float2 *theta, float2 *dst, hipStream_t s,
                           const float2 *theta2 = nullptr, int blocks_per_item = 16);
hipError_t launch_tlr_gather(const GatherItem *items, int nitems, const float2 *P, float2 *Pcol, int64_t rows,
                             hipStream_t s);

}  // namespace tlr
