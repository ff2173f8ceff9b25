// Complex64 GEMM on CDNA4 BF16 matrix cores with a hi+lo split.
//
// Every FP32 operand x is carried as two BF16 numbers, hi = bf16(x) and
// lo = bf16(x - hi); a product is evaluated as hi*hi + hi*lo + lo*hi with FP32
// accumulation (the lo*lo term, about 2^-16 of the product, is dropped).
// The complex product is the same realified real GEMM as in the FP32 kernel
// (M x 2N x 2K, B expanded to [[Re b, Im b], [-Im b, Re b]] blocks), here on
// v_mfma_f32_32x32x16_bf16: one instruction consumes 8 complex k.
//
// Both operands are K-contiguous in memory ("NT" form): A is M x K complex
// (row-major), B is given TRANSPOSED, N x K complex. For the products of the
// method this is free: X, X1 and X2 are symmetric, and the adjoint operand
// r^T is written by the kernel that updates r. Operands are pre-split into
// separate hi and lo planes of interleaved complex BF16 (4 bytes per complex).
//
// Tiling: 512 threads = 8 waves (4 x 2), workgroup tile 256 rows x 128
// complex columns, one workgroup per CU, 8 complex k per stage. At the BF16
// rate a 128 x 128 tile needs about 13 TB/s of operand bandwidth from L2 and
// the memory-side cache; the 256-row tile shares each B panel between twice
// the rows and cuts that by a quarter. Operands go straight from global
// memory to LDS (buffer_load ... lds, no staging registers) into a 4-stage
// ring (four planes per stage: A hi/lo of 256 rows, B hi/lo of 128 rows,
// 16-byte chunks XOR-swizzled so operand reads are bank-conflict free; 96 KiB);
// loads run three stages ahead of the matrix cores. A stage's twelve fragment reads are one inline-asm group
// with its own LDS wait: as plain loads the compiler, unable to tell the ring
// buffers apart from the one the DMA just targeted, would wait for that DMA
// too and undo the prefetch. Per stage each wave issues 2 x 4 x 3 MFMAs,
// ordered so consecutive MFMAs accumulate into different tiles. Each
// lane's B fragment (4 complex b of one column) is turned into the realified
// row pair by one XOR (column parity 0: [Re, -Im]) or a 16-bit rotate
// (parity 1: [Im, Re]) per 32-bit word.
#include "gemm_common.hpp"

namespace tlr {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 2 * GEMM_BM, BN = GEMM_BN;   // 256 x 128 (complex) workgroup tile
constexpr int BKC = 8;                    // complex k per stage (= 16 real k = one MFMA)
constexpr int ROWB = 32;                  // bytes per LDS row of a plane (8 complex BF16)
constexpr int PLANE_A = BM * ROWB;        // 8 KiB per A plane
constexpr int PLANE_B = BN * ROWB;        // 4 KiB per B plane
constexpr int OFF_AL = PLANE_A, OFF_BH = 2 * PLANE_A, OFF_BL = 2 * PLANE_A + PLANE_B;
constexpr int STAGE = 2 * PLANE_A + 2 * PLANE_B;   // A hi, A lo, B hi, B lo: 24 KiB
constexpr int NSTAGE = 4;                 // LDS ring depth (96 KiB per workgroup)
constexpr int NTHREADS = 512;

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding)
template <int N>
__device__ __forceinline__ void wait_vm() {
    __builtin_amdgcn_s_waitcnt((N & 15) | (7 << 4) | (15 << 8) | (((N >> 4) & 3) << 14));
}

typedef __attribute__((address_space(3))) void *lds_ptr_t;

template <int MODE>
__global__ __launch_bounds__(NTHREADS, 1) void cgemm_bf16x3_kernel(GemmArgsB g) {
    // four distinct LDS objects (one per ring stage): reads of one stage and DMA into another are
    // then provably disjoint, so no conservative vmcnt wait is needed before the operand reads
    __shared__ __attribute__((aligned(1024))) unsigned char sm0[STAGE];
    __shared__ __attribute__((aligned(1024))) unsigned char sm1[STAGE];
    __shared__ __attribute__((aligned(1024))) unsigned char sm2[STAGE];
    __shared__ __attribute__((aligned(1024))) unsigned char sm3[STAGE];

    const int z = blockIdx.y;
    const int nb = gridDim.x;
    int pid = blockIdx.x;
    // contiguous tile ranges per XCD, grouped by 2 tile rows: an XCD's 8 tiles of a 1024-row problem
    // (4 row tiles of 256) are 2 rows x 4 columns, so it fetches half of A instead of all of it
    if ((nb & 7) == 0) pid = (pid & 7) * (nb >> 3) + (pid >> 3);
    const int group_rows = 2;
    const int per_group = group_rows * g.tiles_n;
    const int grp = pid / per_group;
    const int first_m = grp * group_rows;
    const int gsz = min(g.tiles_m - first_m, group_rows);
    const int tm = first_m + (pid % per_group) % gsz;
    const int tn = (pid % per_group) / gsz;
    const int m0 = tm * BM;
    const int n0 = (MODE == GM_LINE) ? tn * (BN / 2) : tn * BN;

    const int t = threadIdx.x;
    const int lane = t & 63;
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);   // wave-uniform (LDS DMA base in M0)
    const int wm = wave >> 1, wn = wave & 1;                   // wave rows 0..3, wave columns 0..1

    const __amdgpu_buffer_rsrc_t rAh = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(g.Ahi + z * g.sA * 2), (short)0, (int)g.bytesA, 0x00020000);
    const __amdgpu_buffer_rsrc_t rAl = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(g.Alo + z * g.sA * 2), (short)0, (int)g.bytesA, 0x00020000);
    const __amdgpu_buffer_rsrc_t rBh = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(g.Bhi + z * g.sB * 2), (short)0, (int)g.bytesB, 0x00020000);
    const __amdgpu_buffer_rsrc_t rBl = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(g.Blo + z * g.sB * 2), (short)0, (int)g.bytesB, 0x00020000);

    // Direct global -> LDS loads: lane l of wave w fills the 16 bytes at (w * 64 + l) * 16 of a
    // plane, i.e. row w*32 + l/2, stored chunk l&1. Chunks are XOR-swizzled by bit 3 of the row
    // (stored = actual ^ ((row >> 3) & 1)) so the 16-byte operand reads hit distinct banks. Every
    // wave loads its 32 rows of both A planes; waves 0-3 load the B hi plane, waves 4-7 the B lo
    // plane (32 rows each): three loads per wave and stage. Rows of A past M read as zero (buffer
    // range), so a 256-row tile may overhang a matrix of 128 * odd rows.
    const int lrow = wave * 32 + (lane >> 1);
    const int lchunk = (lane & 1) ^ ((lrow >> 3) & 1);
    const uint32_t offA = (uint32_t)(((int64_t)(m0 + lrow) * g.lda) * 4 + lchunk * 16);
    const int brow = (wave & 3) * 32 + (lane >> 1);
    const bool b_lo = wave >= 4;
    uint32_t offB;
    {
        int64_t row = n0 + brow;
        if (MODE == GM_LINE) {
            const int grp2 = brow >> 5;
            row = n0 + (grp2 >> 1) * 32 + (brow & 31) + ((grp2 & 1) ? g.b2_rows : 0);
        }
        offB = (uint32_t)(row * g.ldb * 4 + ((lane & 1) ^ ((brow >> 3) & 1)) * 16);
    }
    const __amdgpu_buffer_rsrc_t rB = b_lo ? rBl : rBh;
    const int dstB = (b_lo ? OFF_BL : OFF_BH) + (wave & 3) * 1024;
    auto issue = [&](unsigned char *buf, int kt) {
        const int so = kt * BKC * 4;
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rAh, (lds_ptr_t)(buf + wave * 1024), 16, (int)offA, so, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rAl, (lds_ptr_t)(buf + OFF_AL + wave * 1024), 16, (int)offA, so, 0, 0);
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rB, (lds_ptr_t)(buf + dstB), 16, (int)offB, so, 0, 0);
    };

    floatx16 acc[2][4];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

    const int j32 = lane & 31;
    const int half = lane >> 5;
    const bool odd = (j32 & 1) != 0;
    // fragment reads (swizzled chunk): A rows wm*64 + bm*32 + j32, B rows wn*64 + bn*16 + j32/2
    const int a_off = (wm * 64 + j32) * ROWB + ((half ^ ((j32 >> 3) & 1)) * 16);
    const int b_off = (wn * 64 + (j32 >> 1)) * ROWB + ((half ^ ((j32 >> 4) & 1)) * 16);

    // realified B row pair from 4 complex b: even column -> [Re, -Im] (flip the sign bit of the
    // high half), odd column -> [Im, Re] (rotate by 16); branch-free: rotr(x, sh) ^ msk
    const unsigned sh = odd ? 16u : 0u;
    const unsigned msk = odd ? 0u : 0x80000000u;
    auto xform = [&](u32x4 v) {
        u32x4 o;
#pragma unroll
        for (int w = 0; w < 4; ++w) o[w] = __builtin_amdgcn_alignbit(v[w], v[w], sh) ^ msk;
        return o;
    };

    // LDS addresses (32-bit) of this lane's fragments in each ring buffer
    auto lds_addr = [](const unsigned char *p) { return (uint32_t)(uintptr_t)(lds_ptr_t)p; };
    auto compute = [&](const unsigned char *st) {
        const uint32_t va = lds_addr(st) + a_off, vb = lds_addr(st) + b_off;
        u32x4 ah0, ah1, al0, al1, bh0, bh1, bh2, bh3, bl0, bl1, bl2, bl3;
        // all twelve fragment reads of the stage in flight together, waited in the same block
        // A hi rows +0 / +32 at 0 / 1024, A lo at 8192 / 9216; B hi (16 rows per block) at 16384 + 512 bn,
        // B lo at 20480 + 512 bn
        asm volatile(
            "ds_read_b128 %0, %12\n\t"
            "ds_read_b128 %1, %12 offset:1024\n\t"
            "ds_read_b128 %2, %12 offset:8192\n\t"
            "ds_read_b128 %3, %12 offset:9216\n\t"
            "ds_read_b128 %4, %13 offset:16384\n\t"
            "ds_read_b128 %5, %13 offset:16896\n\t"
            "ds_read_b128 %6, %13 offset:17408\n\t"
            "ds_read_b128 %7, %13 offset:17920\n\t"
            "ds_read_b128 %8, %13 offset:20480\n\t"
            "ds_read_b128 %9, %13 offset:20992\n\t"
            "ds_read_b128 %10, %13 offset:21504\n\t"
            "ds_read_b128 %11, %13 offset:22016\n\t"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(ah0), "=&v"(ah1), "=&v"(al0), "=&v"(al1), "=&v"(bh0), "=&v"(bh1), "=&v"(bh2), "=&v"(bh3),
              "=&v"(bl0), "=&v"(bl1), "=&v"(bl2), "=&v"(bl3)
            : "v"(va), "v"(vb));
        const bf16x8 ah[2] = {as_bf16x8(ah0), as_bf16x8(ah1)};
        const bf16x8 al[2] = {as_bf16x8(al0), as_bf16x8(al1)};
        const bf16x8 bh[4] = {as_bf16x8(xform(bh0)), as_bf16x8(xform(bh1)), as_bf16x8(xform(bh2)), as_bf16x8(xform(bh3))};
        const bf16x8 bl[4] = {as_bf16x8(xform(bl0)), as_bf16x8(xform(bl1)), as_bf16x8(xform(bl2)), as_bf16x8(xform(bl3))};
        // consecutive MFMAs accumulate into different tiles
#pragma unroll
        for (int bn = 0; bn < 4; ++bn)
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
                acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[bm], bh[bn], acc[bm][bn], 0, 0, 0);
#pragma unroll
        for (int bn = 0; bn < 4; ++bn)
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
                acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bm], bl[bn], acc[bm][bn], 0, 0, 0);
#pragma unroll
        for (int bn = 0; bn < 4; ++bn)
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
                acc[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[bm], bh[bn], acc[bm][bn], 0, 0, 0);
    };
    // one ring step: stage kt (in `cur`) has landed once at most the loads of the two stages
    // issued after it are outstanding; then the buffer of stage kt-1 (`nxt`) takes stage kt+3
    auto step = [&](int kt, int nk, const unsigned char *cur, unsigned char *nxt) {
        const int ahead = min(NSTAGE - 2, nk - 1 - kt);   // stages issued after kt (3 loads each)
        if (ahead >= 2) wait_vm<6>();
        else if (ahead == 1) wait_vm<3>();
        else wait_vm<0>();
        // Bare barrier: each wave has waited for its own DMA of stage kt above, so after the
        // barrier the whole stage is in LDS, and every wave has finished reading stage kt-1.
        // (A fenced barrier would drain all outstanding DMA and serialise the ring.)
        asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
        if (kt + NSTAGE - 1 < nk) issue(nxt, kt + NSTAGE - 1);
        compute(cur);
    };

    const int nk = g.K / BKC;   // a multiple of 16: K is padded to whole 128-tiles
    issue(sm0, 0);
    issue(sm1, 1);
    issue(sm2, 2);
    for (int kt = 0; kt < nk; kt += NSTAGE) {
        step(kt + 0, nk, sm0, sm3);
        step(kt + 1, nk, sm1, sm0);
        step(kt + 2, nk, sm2, sm1);
        step(kt + 3, nk, sm3, sm2);
    }
    __syncthreads();   // the LDS ring is reused by the epilogue's reduction scratch only after all reads

    EpiArgs ea;
    ea.C = g.C + z * g.sC;
    ea.C2 = (MODE == GM_LINE) ? g.C2 + z * g.sC : nullptr;
    ea.ldc = g.ldc;
    ea.E = (MODE == GM_STORE) ? nullptr : g.E + z * g.sE;
    ea.lde = g.lde;
    ea.Me = g.Me;
    ea.Ne = g.Ne;
    ea.partials = g.partials ? g.partials + z * g.sP : nullptr;
    ea.Mrows = g.M;
    ea.slot_step = g.tiles_n;
    // partial slots in the numbering of 128-row tiles (the finalisation sums M/128 x tiles_n slots)
    gemm_epilogue<MODE, 4>(acc, ea, m0, n0, 2 * tm * g.tiles_n + tn);
}

}  // namespace

hipError_t launch_cgemm_bf16(int mode, const GemmArgsB &a0, int batch, hipStream_t s) {
    GemmArgsB a = a0;
    a.tiles_m = (a.M + BM - 1) / BM;
    a.tiles_n = (mode == GM_LINE) ? a.N / (BN / 2) : a.N / BN;
    if (a.M <= 0 || a.N <= 0 || batch <= 0) return hipSuccess;
    if (a.M % GEMM_BM || a.N % BN || a.K % (BKC * NSTAGE) || a.K <= 0) return hipErrorInvalidValue;
    const int64_t bytesA = (int64_t)a.M * a.lda * 4;
    const int64_t rowsB = (mode == GM_LINE) ? a.b2_rows + a.N : a.N;
    const int64_t bytesB = rowsB * a.ldb * 4;
    if (bytesA >= (int64_t)1 << 32 || bytesB >= (int64_t)1 << 32) return hipErrorInvalidValue;
    a.bytesA = (uint32_t)bytesA;
    a.bytesB = (uint32_t)bytesB;
    dim3 grid(a.tiles_m * a.tiles_n, batch);
    switch (mode) {
        case GM_STORE: hipLaunchKernelGGL(cgemm_bf16x3_kernel<GM_STORE>, grid, dim3(NTHREADS), 0, s, a); break;
        case GM_RESID: hipLaunchKernelGGL(cgemm_bf16x3_kernel<GM_RESID>, grid, dim3(NTHREADS), 0, s, a); break;
        case GM_LINE:  hipLaunchKernelGGL(cgemm_bf16x3_kernel<GM_LINE>, grid, dim3(NTHREADS), 0, s, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace tlr
