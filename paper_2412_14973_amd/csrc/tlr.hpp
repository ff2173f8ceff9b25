// Operand packing for the tile low-rank product (internal).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace tlr {

enum PackOp : int32_t { PACK_COPY = 0, PACK_TRANS = 1, PACK_IDENT = 2, PACK_SYM = 3 };

// dst[r * ldd + c] (r < rows, c < cols) from the theta block at src:
// COPY src[r * lds + c]; TRANS src[c * lds + r]; IDENT delta_rc; SYM (src[r][c] + src[c][r]) / 2
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

hipError_t launch_tlr_pack(const PackItem *items, int nitems, const float2 *theta, float2 *dst, hipStream_t s,
                           const float2 *theta2 = nullptr);
hipError_t launch_tlr_gather(const GatherItem *items, int nitems, const float2 *P, float2 *Pcol, int64_t rows,
                             hipStream_t s);

}  // namespace tlr
