// C ABI of the TLR-MDD library: validation, plans, workspace carving and the
// stream-ordered orchestration of the HIP kernels. No C++ exception crosses
// the ABI; every entry point returns a status code.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "tlrmdd.h"
#include "svd.hpp"
#include "tlr.hpp"
#include "vec.hpp"

using namespace tlr;

namespace {

thread_local std::string g_last_error;

int fail(int status, const std::string &msg) {
    g_last_error = msg;
    return status;
}

}  // namespace

int tlr::set_error(int status, const std::string &msg) { return fail(status, msg); }

namespace {

#define HIP_TRY(expr)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (expr);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(TLRMDD_HIP_ERROR, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

inline int64_t round_up(int64_t v, int64_t m) { return (v + m - 1) / m * m; }
inline size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// kernel timing: HIP events around launches of selected kinds, with each launch's algorithmic work
// ---------------------------------------------------------------------------
// Product forms of the complex GEMMs: real flops per complex flop (8 m n k) and the instruction type
enum Form : int32_t { F_4M = 0, F_3M = 1, F_BF16X3 = 2 };

// Work of one launch on the true (unpadded) sizes and ranks: complex flops counted 8 m n k, the real
// flops of the form that runs (four products 8 m n k, three products 6 m n k, BF16 hi+lo split 24 m n k
// in BF16), and HBM bytes with every operand read once and every output written once.
struct Work {
    double cflops = 0.0, flops = 0.0, bytes = 0.0;
    int dtype = TLRMDD_DT_NONE;
};

Work gemm_work(int form, double cflops, double bytes) {
    Work w;
    w.cflops = cflops;
    w.flops = cflops * (form == F_4M ? 1.0 : form == F_3M ? 0.75 : 3.0);
    w.bytes = bytes;
    w.dtype = form == F_BF16X3 ? TLRMDD_DT_BF16 : TLRMDD_DT_FP32;
    return w;
}

Work bytes_work(double bytes) {
    Work w;
    w.bytes = bytes;
    return w;
}

struct TimedLaunch {
    int kind;
    hipEvent_t a, b;
    Work work;
};
struct Recorder {
    std::mutex mu;
    std::atomic<uint32_t> kinds{0};   // bit k set: launches of kind k are timed (0: timing off)
    std::vector<TimedLaunch> ev;
    std::vector<hipEvent_t> pool;
} g_rec;

hipEvent_t rec_event() {
    if (!g_rec.pool.empty()) {
        hipEvent_t e = g_rec.pool.back();
        g_rec.pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// An open graph capture on this thread (tlrmdd_graph_begin .. tlrmdd_graph_end): launches are
// recorded, not timed, and host tables go to pinned buffers that the graph will own.
struct Capture {
    bool on = false;
    hipStream_t stream = nullptr;
    std::vector<char *> pinned;
};
thread_local Capture g_cap;

template <class F>
hipError_t timed(int kind, hipStream_t s, const Work &work, F &&launch) {
    if (!((g_rec.kinds.load(std::memory_order_relaxed) >> kind) & 1u) || g_cap.on) return launch();
    std::lock_guard<std::mutex> lk(g_rec.mu);
    // timing may have ended between the check and the lock: then the launch runs untimed
    if (!((g_rec.kinds.load(std::memory_order_relaxed) >> kind) & 1u)) return launch();
    hipEvent_t a = rec_event(), b = rec_event();
    if (a) (void)hipEventRecord(a, s);
    hipError_t e = launch();
    if (b) (void)hipEventRecord(b, s);
    if (a && b) g_rec.ev.push_back(TimedLaunch{kind, a, b, work});
    return e;
}

// ---------------------------------------------------------------------------
// host -> device uploads of host-built tables without waiting for the device
// ---------------------------------------------------------------------------
// A call's tables are gathered into one image, copied into a library-owned pinned buffer and sent
// to their device addresses on the caller's stream; an event recorded after the copies tells when
// the buffer may take another image. A call takes a buffer whose event has completed (or a new
// one), so no call blocks on the device and nothing the caller owns is read after it returns.
struct PinnedBuf {
    char *host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    int device = -1;
};
struct PinnedPool {
    std::mutex mu;
    std::vector<PinnedBuf> bufs;
} g_pinned;
constexpr size_t PINNED_MIN = size_t(64) << 10;
constexpr int PINNED_MAX_BUFS = 64;   // beyond this many buffers in flight a call waits for the oldest

class Upload {
  public:
    // queue `bytes` of host memory `src` for device address `dst`
    void add(void *dst, const void *src, size_t bytes) {
        if (!bytes) return;
        const size_t off = img_.size();
        img_.resize(off + ((bytes + 15) & ~size_t(15)));
        std::memcpy(img_.data() + off, src, bytes);
        pieces_.push_back(Piece{dst, off, bytes});
    }
    int commit(hipStream_t s);

  private:
    struct Piece {
        void *dst;
        size_t off, bytes;
    };
    std::vector<char> img_;
    std::vector<Piece> pieces_;
};

int Upload::commit(hipStream_t s) {
    if (img_.empty()) return TLRMDD_OK;
    if (g_cap.on) {
        // recorded copies read their source at every replay: a buffer of the graph's own
        char *host = nullptr;
        HIP_TRY(hipHostMalloc((void **)&host, img_.size(), hipHostMallocDefault));
        g_cap.pinned.push_back(host);
        std::memcpy(host, img_.data(), img_.size());
        for (const Piece &p : pieces_)
            if (p.bytes) HIP_TRY(hipMemcpyAsync(p.dst, host + p.off, p.bytes, hipMemcpyHostToDevice, s));
        return TLRMDD_OK;
    }
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_pinned.mu);
    PinnedBuf *pick = nullptr;
    int ndev = 0;
    for (PinnedBuf &b : g_pinned.bufs) {
        if (b.device != dev) continue;
        ++ndev;
        if (b.cap < img_.size() || hipEventQuery(b.done) != hipSuccess) continue;
        if (!pick || b.cap < pick->cap) pick = &b;
    }
    if (!pick && ndev >= PINNED_MAX_BUFS) {   // bounded: wait for a large enough buffer of this device
        for (PinnedBuf &b : g_pinned.bufs)
            if (b.device == dev && b.cap >= img_.size()) {
                HIP_TRY(hipEventSynchronize(b.done));
                pick = &b;
                break;
            }
    }
    if (!pick) {
        PinnedBuf b;
        b.device = dev;
        b.cap = PINNED_MIN;
        while (b.cap < img_.size()) b.cap *= 2;
        HIP_TRY(hipHostMalloc((void **)&b.host, b.cap, hipHostMallocDefault));
        hipError_t e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            (void)hipHostFree(b.host);
            return fail(TLRMDD_HIP_ERROR, std::string("upload event: ") + hipGetErrorString(e));
        }
        g_pinned.bufs.push_back(b);
        pick = &g_pinned.bufs.back();
    }
    std::memcpy(pick->host, img_.data(), img_.size());
    for (const Piece &p : pieces_)
        if (p.bytes) HIP_TRY(hipMemcpyAsync(p.dst, pick->host + p.off, p.bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(pick->done, s));
    return TLRMDD_OK;
}

// ---------------------------------------------------------------------------
// layout validation and tables
// ---------------------------------------------------------------------------
struct HostLayout {
    int64_t nr = 0, ns = 0;
    int N = 0;
    std::vector<int> d, start, kdiag;
    std::vector<int> koff;          // t order
    std::vector<TileDesc> tiles;    // diagonal tiles first, then sub-diagonal tiles in t order
    int64_t theta_size = 0;
    // complex flops (8 per complex multiply-add) of the tile products: assembly of X, of X1 and X2
    // (three products per tile), and the gradient contractions (two per sub-diagonal tile, one per
    // Q Q^T tile); a Q Q^T product counts its d (d + 1) / 2 distinct entries
    double asm_cflops = 0.0, asm_dir_cflops = 0.0, grad_cflops = 0.0;
};

int build_layout(const tlrmdd_layout *L, HostLayout &H) {
    if (!L) return fail(TLRMDD_INVALID_ARGUMENT, "layout is NULL");
    if (L->nr <= 0 || L->ns <= 0 || L->ntiles <= 0)
        return fail(TLRMDD_INVALID_ARGUMENT, "nr, ns and ntiles must be positive");
    if (L->nr > (int64_t)1 << 30 || L->ns > (int64_t)1 << 30)
        return fail(TLRMDD_INVALID_ARGUMENT, "nr / ns too large");
    if (!L->tile_size || !L->rank_diag || (L->ntiles > 1 && !L->rank_off))
        return fail(TLRMDD_INVALID_ARGUMENT, "tile_size / rank_off / rank_diag is NULL");
    H = HostLayout();
    H.nr = L->nr;
    H.ns = L->ns;
    H.N = L->ntiles;
    int64_t sum = 0;
    for (int i = 0; i < H.N; ++i) {
        const int di = L->tile_size[i];
        if (di <= 0) return fail(TLRMDD_INVALID_ARGUMENT, "tile size must be positive");
        H.start.push_back((int)sum);
        H.d.push_back(di);
        sum += di;
    }
    if (sum != H.nr) return fail(TLRMDD_INVALID_ARGUMENT, "sum of tile sizes differs from nr");
    for (int i = 0; i < H.N; ++i) {
        const int k = L->rank_diag[i];
        if (!(k == -1 || (k >= 1 && k <= H.d[i])))
            return fail(TLRMDD_INVALID_ARGUMENT, "diagonal rank must be -1 or in [1, d_i]");
        H.kdiag.push_back(k);
    }
    int t = 0;
    for (int i = 0; i < H.N; ++i)
        for (int j = 0; j < i; ++j, ++t) {
            const int k = L->rank_off[t];
            if (k < 1 || k > std::min(H.d[i], H.d[j]))
                return fail(TLRMDD_INVALID_ARGUMENT, "off-diagonal rank must be in [1, min(d_i, d_j)]");
            H.koff.push_back(k);
        }
    // theta packing: diagonal blocks, then all L_t, then all R_t
    int64_t pos = 0;
    for (int i = 0; i < H.N; ++i) {
        TileDesc td{};
        td.kind = H.kdiag[i] < 0 ? TILE_DENSE : TILE_QQ;
        td.di = td.dj = H.d[i];
        td.k = H.kdiag[i] < 0 ? H.d[i] : H.kdiag[i];
        td.row0 = td.col0 = H.start[i];
        td.offA = pos;
        td.offB = 0;
        pos += (int64_t)H.d[i] * td.k;
        H.tiles.push_back(td);
    }
    t = 0;
    for (int i = 0; i < H.N; ++i)
        for (int j = 0; j < i; ++j, ++t) {
            TileDesc td{};
            td.kind = TILE_LR;
            td.di = H.d[i];
            td.dj = H.d[j];
            td.k = H.koff[t];
            td.row0 = H.start[i];
            td.col0 = H.start[j];
            td.offA = pos;
            pos += (int64_t)td.di * td.k;
            H.tiles.push_back(td);
        }
    t = 0;
    for (int i = 0; i < H.N; ++i)
        for (int j = 0; j < i; ++j, ++t) {
            TileDesc &td = H.tiles[H.N + t];
            td.offB = pos;
            pos += (int64_t)td.k * td.dj;
        }
    H.theta_size = pos;
    for (const TileDesc &td : H.tiles) {
        const double di = td.di, dj = td.dj, k = td.k;
        if (td.kind == TILE_LR) {
            H.asm_cflops += 8.0 * di * dj * k;
            H.grad_cflops += 16.0 * di * dj * k;
        } else if (td.kind == TILE_QQ) {
            H.asm_cflops += 4.0 * di * (di + 1.0) * k;
            H.grad_cflops += 8.0 * di * dj * k;
        }
    }
    H.asm_dir_cflops = 3.0 * H.asm_cflops;
    return TLRMDD_OK;
}

// Work tables of one launch group (one problem, or a batch of problems).
struct Tables {
    std::vector<TileDesc> tiles;
    std::vector<AsmItem> asm_items;
    std::vector<int> asm_first;     // first assembly item of every problem (items are in problem order)
    std::vector<int> grad_first;    // first gradient item of every problem
    std::vector<GradItem> grad_items;
    std::vector<ProbOff> probs;
    std::vector<VecSeg> tsegs;      // theta-space segments
    std::vector<int32_t> tseg_count;
    std::vector<VecSeg> rsegs;      // residual-space segments (uniform per problem)
    int rseg_per_prob = 0;
    int tseg_max = 0;
    int64_t theta_total = 0;        // complex elements over all problems
};

// each problem's theta starts on a 16-byte boundary (vector kernels move 4 floats at a time)
int64_t theta_span(int64_t theta_size) { return (theta_size + 1) & ~int64_t(1); }

void append_problem(Tables &T, const HostLayout &H, int prob, int64_t x_off, int64_t ldk) {
    const int tile_base = (int)T.tiles.size();
    T.asm_first.push_back((int)T.asm_items.size());
    T.grad_first.push_back((int)T.grad_items.size());
    for (const TileDesc &td : H.tiles) T.tiles.push_back(td);
    for (int q = 0; q < (int)H.tiles.size(); ++q) {
        const TileDesc &td = H.tiles[q];
        // Q Q^T tiles: blocks on and below the diagonal only (the kernel mirrors them)
        for (int r0 = 0; r0 < td.di; r0 += ASM_B)
            for (int c0 = 0; c0 < (td.kind == TILE_QQ ? r0 + 1 : td.dj); c0 += ASM_B)
                T.asm_items.push_back(AsmItem{tile_base + q, r0, c0, prob});
        auto gi = [&](int kind, int a0, int b0) {
            const int kq = kind == G_Z ? 0 : (std::min(GR_KK, td.k - b0) + 15) / 16;
            T.grad_items.push_back(GradItem{tile_base + q, kind, a0, b0, prob, kq});
        };
        if (td.kind == TILE_DENSE) {
            for (int a0 = 0; a0 < td.di; a0 += GZ_BR)
                for (int b0 = 0; b0 < td.dj; b0 += GZ_BC) gi(G_Z, a0, b0);
        } else if (td.kind == TILE_QQ) {
            for (int a0 = 0; a0 < td.di; a0 += GR_ROWS)
                for (int b0 = 0; b0 < td.k; b0 += GR_KK) gi(G_Q, a0, b0);
        } else {
            for (int a0 = 0; a0 < td.di; a0 += GR_ROWS)
                for (int b0 = 0; b0 < td.k; b0 += GR_KK) gi(G_L, a0, b0);
            for (int a0 = 0; a0 < td.dj; a0 += GR_ROWS)
                for (int b0 = 0; b0 < td.k; b0 += GR_KK) gi(G_R, a0, b0);
        }
    }
    ProbOff po{};
    po.theta = T.theta_total;
    po.x = x_off;
    po.ldx = ldk;
    T.probs.push_back(po);
    T.theta_total += theta_span(H.theta_size);
}

// segments: called after all problems are appended; residual space is nsp x ldk per problem
void build_segments(Tables &T, const std::vector<const HostLayout *> &Hs, int64_t nsp, int64_t ldk) {
    const int np = (int)Hs.size();
    T.tseg_count.assign(np, 0);
    int maxseg = 0;
    for (int p = 0; p < np; ++p) {
        const int64_t n2 = 2 * Hs[p]->theta_size;
        maxseg = std::max<int>(maxseg, (int)((n2 + VEC_CH - 1) / VEC_CH));
    }
    const int64_t r2 = 2 * nsp * ldk;
    T.rseg_per_prob = (int)((r2 + VEC_CH - 1) / VEC_CH);
    T.tseg_max = maxseg;
    for (int p = 0; p < np; ++p) {
        const int64_t base = 2 * T.probs[p].theta;
        const int64_t n2 = 2 * Hs[p]->theta_size;
        int local = 0;
        for (int64_t o = 0; o < n2; o += VEC_CH, ++local)
            T.tsegs.push_back(VecSeg{base + o, (int32_t)std::min<int64_t>(VEC_CH, n2 - o), p, 0, 0});
        T.tseg_count[p] = local;
    }
    for (int p = 0; p < np; ++p) {
        int local = 0;
        for (int64_t o = 0; o < r2; o += VEC_CH, ++local)
            T.rsegs.push_back(VecSeg{p * r2 + o, (int32_t)std::min<int64_t>(VEC_CH, r2 - o), p, 0, 0});
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
namespace {
// Device tables of one launch group, carved from one buffer.
struct DevTables {
    TileDesc *tiles;
    AsmItem *asm_items;
    GradItem *grad_items;
    ProbOff *probs;
    VecSeg *tsegs;
    int32_t *tcount;
    VecSeg *rsegs;
    double **fhist;
    int n_asm, n_grad, n_tseg, n_rseg;
};
}  // namespace

struct tlrmdd_plan_s {
    HostLayout H;
    int64_t ldk = 0, lds = 0;   // padded sizes (complex): nr and ns rounded up to GEMM_PAD
    Tables T;
    int device = 0;
    DevTables D{};              // single-problem tables, uploaded once at plan creation
    void *d_block = nullptr;
};

namespace {

size_t tables_bytes(const Tables &T, int nprob) {
    size_t b = 0;
    b += align256(T.tiles.size() * sizeof(TileDesc));
    b += align256(T.asm_items.size() * sizeof(AsmItem));
    b += align256(T.grad_items.size() * sizeof(GradItem));
    b += align256(T.probs.size() * sizeof(ProbOff));
    b += align256(T.tsegs.size() * sizeof(VecSeg));
    b += align256(T.tseg_count.size() * sizeof(int32_t));
    b += align256(T.rsegs.size() * sizeof(VecSeg));
    b += align256(nprob * sizeof(double *));
    return b;
}

// Host image of the tables + their device addresses inside `dev`.
void pack_tables(const Tables &T, int nprob, char *dev, std::vector<char> &img, DevTables &D,
                 double *const *fhist) {
    img.assign(tables_bytes(T, nprob), 0);
    size_t o = 0;
    auto put = [&](const void *src, size_t bytes) -> char * {
        if (bytes) std::memcpy(img.data() + o, src, bytes);
        char *p = dev + o;
        o += align256(bytes);
        return p;
    };
    D.tiles = (TileDesc *)put(T.tiles.data(), T.tiles.size() * sizeof(TileDesc));
    D.asm_items = (AsmItem *)put(T.asm_items.data(), T.asm_items.size() * sizeof(AsmItem));
    D.grad_items = (GradItem *)put(T.grad_items.data(), T.grad_items.size() * sizeof(GradItem));
    D.probs = (ProbOff *)put(T.probs.data(), T.probs.size() * sizeof(ProbOff));
    D.tsegs = (VecSeg *)put(T.tsegs.data(), T.tsegs.size() * sizeof(VecSeg));
    D.tcount = (int32_t *)put(T.tseg_count.data(), T.tseg_count.size() * sizeof(int32_t));
    D.rsegs = (VecSeg *)put(T.rsegs.data(), T.rsegs.size() * sizeof(VecSeg));
    std::vector<double *> fh(nprob, nullptr);
    if (fhist)
        for (int p = 0; p < nprob; ++p) fh[p] = fhist[p];
    D.fhist = (double **)put(fh.data(), nprob * sizeof(double *));
    D.n_asm = (int)T.asm_items.size();
    D.n_grad = (int)T.grad_items.size();
    D.n_tseg = (int)T.tsegs.size();
    D.n_rseg = (int)T.rsegs.size();
}

// assign partial slots: part = prob * pstride + local
void assign_parts(Tables &T, int pstride) {
    std::vector<int> local(T.probs.size(), 0);
    for (VecSeg &s : T.tsegs) s.part = s.prob * pstride + local[s.prob]++;
    std::fill(local.begin(), local.end(), 0);
    for (VecSeg &s : T.rsegs) s.part = s.prob * pstride + local[s.prob]++;
}

int partial_stride(const Tables &T, int64_t nrp, int64_t nsp) {
    int ps = std::max(T.tseg_max, T.rseg_per_prob);
    ps = std::max(ps, gemm_partials_per_problem(GM_LINE, (int)nsp, (int)nrp) / 5);
    ps = std::max(ps, gemm_partials_per_problem(GM_RESID, (int)nsp, (int)nrp));
    return std::max(ps, 1);
}

// ---------------------------------------------------------------------------
// workspace layout
// ---------------------------------------------------------------------------
struct Ws {
    float2 *Ds = nullptr, *DHs = nullptr, *Us = nullptr, *XW = nullptr, *r = nullptr, *a = nullptr, *b = nullptr;
    float2 *Dc = nullptr;     // complex64 D for the tile-form products (Ds itself, or a copy in BF16 mode)
    uint32_t *rT = nullptr;   // BF16 split planes of r^T (hi, lo), ldk x lds each
    float *th = nullptr, *g0 = nullptr, *g1 = nullptr, *p = nullptr, *S = nullptr, *Y = nullptr;
    double *gram = nullptr;   // per problem: Gram matrix of the L-BFGS basis and direction coefficients
    float *z = nullptr, *u = nullptr, *cen = nullptr;   // ADMM
    double *partials = nullptr;
    SolveScalars *sc = nullptr;
    char *tables = nullptr;
    size_t bytes = 0;
};

// doubles per problem for the L-BFGS Gram matrix over (s_j, y_j, g) and the direction coefficients
int64_t gram_stride(int m1) { return (int64_t)(2 * m1 + 1) * (2 * m1 + 1) + 2 * m1 + 1; }

// op: 0 forward, 1 grad, 2 solve, 3 ADMM. Sizes for `nprob` problems of the same shape; every matrix is
// padded to whole GEMM tiles: ns x nr operands are lds x ldk (rows x cols), nr x nr ones ldk x ldk.
Ws carve(char *base, int op, int nprob, int64_t ldk, int64_t lds, int64_t theta_total, int m1, int pstride,
         size_t tbytes) {
    Ws w;
    size_t o = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + o : nullptr;
        o += align256(bytes);
        return p;
    };
    const size_t c8 = sizeof(float2);
    const size_t xsz = (size_t)nprob * ldk * ldk * c8;
    const size_t rsz = (size_t)nprob * lds * ldk * c8;
    w.Ds = (float2 *)take(rsz);
    if (op >= 1) w.DHs = (float2 *)take((size_t)nprob * ldk * lds * c8);
    w.XW = (float2 *)take(op >= 2 ? 2 * xsz : xsz);
    w.r = (float2 *)take(rsz);
    if (op >= 1) w.rT = (uint32_t *)take(rsz);
    if (op >= 2) {
        w.Us = (float2 *)take(rsz);
        w.a = (float2 *)take(rsz);
        w.b = (float2 *)take(rsz);
        const size_t tz = (size_t)theta_total * c8;
        w.th = (float *)take(tz);
        w.g0 = (float *)take(tz);
        w.g1 = (float *)take(tz);
        w.p = (float *)take(tz);
        w.S = (float *)take(tz * m1);
        w.Y = (float *)take(tz * m1);
        w.gram = (double *)take((size_t)nprob * gram_stride(m1) * sizeof(double));
    }
    if (op == 3) {   // ADMM: split variable, scaled dual, penalty center
        const size_t tz = (size_t)theta_total * c8;
        w.z = (float *)take(tz);
        w.u = (float *)take(tz);
        w.cen = (float *)take(tz);
    }
    w.partials = (double *)take((size_t)nprob * pstride * std::max(5, 6 * m1) * sizeof(double));
    w.sc = (SolveScalars *)take((size_t)nprob * sizeof(SolveScalars));
    w.tables = take(tbytes);
    w.bytes = o;
    return w;
}

// ---------------------------------------------------------------------------
// tile-form line search: [a | b] = D [X1 | X2] from the factors of theta and p, without X1, X2
// ---------------------------------------------------------------------------
// Every tile pair of X1 = C1(theta; p) and X2 = C2(p) is a product of packed factor blocks
//   X1_ij = A_p B_th + A_th B_p,  X2_ij = A_p B_p
// (i > j: A = L, B = R; i < j: A = R_ji^T, B = L_ji^T; i = j: A = Q, B = Q^T; the p-blocks are the
// same factors of the direction p). Stage 1 forms P_i = D_:,i [A_p(i0) | A_p(i1) | ... | A_th(i0) | ...]
// for every tile row (the nt direction blocks first, then the nt theta blocks) and stores its blocks
// regrouped by tile column, Pcol_j = [P_p(0j) | ... | P_th(0j) | ...], and stage 2 forms
//   a_:,j = Pcol_j [B_th(0j); ...; B_p(0j); ...],   b_:,j = Pcol_j[:, first half] [B_p(0j); ...]
// in one line-search product with the five line sums (b contracts over the first nt kpad columns only).
// Ranks are padded to kpad with zero columns. Flops relative to the dense pair D [X1 | X2]:
// stage 1 kpad / d, stage 2 kpad / d for a and kpad / 2d for b.
constexpr double LINE_TILE_FLOPS = 2.5;      // flops of the tile form per kpad / d of the dense pair
constexpr double LINE_TILE_MAX_COST = 0.6;   // tile form where its flops are at most this share

struct LineClass {
    int d = 0, nt = 0, kpad = 0;
    bool grad = false;               // the gradient in tile form too
    bool operator==(const LineClass &o) const {
        return d == o.d && nt == o.nt && kpad == o.kpad && grad == o.grad;
    }
};

// Gradient in tile form (TLRMDD_LINE_TILE_GRAD). With W = D^H r and every tile pair a factor product
// X_ij = A_ij B_ij, the gradient blocks are W_ij B_ij^H = D_:,i^H (r_:,j B_ij^H) and
// A_ij^H W_ij = (D_:,i A_ij)^H r_:,j (gradient equations; the sum over both orders of a tile pair
// forms W' = W + W^T). Three batched products of width Wg = nt kpad rounded up to 64:
//   G1: S_j = r_:,j [B_0j^H | B_1j^H | ...], stored regrouped by tile row (Scol_i = [S_i0 | S_i1 | ...]);
//   G2: GA_i = D_:,i^H Scol_i;   G3: GBT_j = r_:,j^T conj(P_th(:,j)), with P_th(ij) = D_:,i A_ij the theta
//   half of the line search's stage 1 (carried to the updated theta by P_th += step P_p);
// G2 and G3 split their ns-long contraction in GRAD_TILE_KS parts and run as one launch (G2 as its
// conjugate, D^T conj(Scol), in the transposed-A / conjugated-B role of G3), and
//   grad A_ij = GA_i[:, j kpad ..] + GBT_i[:, j kpad ..],  grad B_ij = (GA_j[:, i kpad ..] + GBT_j[:, i kpad ..])^T
// summed over the parts (Q: A = Q, B = Q^T; L, R: the pair (i > j) and its transpose (j, i)).
// Flops: 3 Wg / nr of the adjoint product D^H r.
constexpr double GRAD_TILE_MAX_COST = 0.6;
constexpr int GRAD_TILE_KS = 4;
static_assert(GEMM_PAD % (GRAD_TILE_KS * GEMM_BK) == 0, "every part of the padded ns is a whole number of k stages");
// (the product kernel's tile stages take a last column tile of 64)
int64_t grad_tile_width(const LineClass &lc) { return round_up((int64_t)lc.nt * lc.kpad, GEMM_BN / 2); }

// Tile form is possible when all tiles have one size d (a multiple of 128), nr needs no padding and the
// diagonal tiles are Q Q^T; problem_form decides whether the padded rank keeps the flops low enough.
bool line_class(const HostLayout &H, LineClass &lc) {
    if (H.nr % GEMM_PAD) return false;
    const int d = H.d[0];
    for (int i = 0; i < H.N; ++i)
        if (H.d[i] != d) return false;
    if (d % GEMM_BN) return false;
    int kmax = 1;
    for (const TileDesc &td : H.tiles) {
        if (td.kind == TILE_DENSE) return false;
        kmax = std::max(kmax, td.k);
    }
    const int nt = H.N;
    // stage-1 rows hold 2 nt blocks of kpad columns, a whole number of 128-column GEMM tiles:
    // nt * 2 * kpad divisible by 128 <=> kpad divisible by 64 / gcd(nt, 64); then nt kpad (the
    // k of b) is a multiple of 64
    int gcd = nt, b = 64;
    while (b) {
        const int r = gcd % b;
        gcd = b;
        b = r;
    }
    const int q = 64 / gcd;
    const int kpad = (int)round_up(kmax, q);
    lc = LineClass{d, nt, kpad};
    return true;
}


// Line-search (and gradient) form of one problem under opts: false = dense; lc.grad = gradient too.
// The tile-form products run on the three-product FP32 kernel; in BF16 mode the dense products they
// replace run at about twice its rate (measured: 340 against 171 TFLOP/s algorithmic on the bench
// workload), so there the flop shares must be half as large.
constexpr double BF16_DENSE_SPEED = 2.0;
bool tile_line_requested(int op, const tlrmdd_opts *opts);
bool problem_form(int op, const HostLayout &H, const tlrmdd_opts *opts, LineClass &lc) {
    if (!tile_line_requested(op, opts) || !line_class(H, lc)) return false;
    const double speed = opts->precision == TLRMDD_BF16X3 ? BF16_DENSE_SPEED : 1.0;
    if (LINE_TILE_FLOPS * lc.kpad * speed > LINE_TILE_MAX_COST * lc.d) return false;
    lc.grad = opts->line_products == TLRMDD_LINE_TILE_GRAD &&
              3.0 * (double)grad_tile_width(lc) * speed <= GRAD_TILE_MAX_COST * (double)H.nr;
    return true;
}

// Device state of the tile-form line search of one run (all problems of one class).
struct LineTile {
    bool on = false;
    LineClass lc;
    double ksum = 0.0;               // sum over the range's problems of the ranks of all ordered tile pairs
    int64_t NA = 0;                  // columns of a stage-1 row block: nt * 2 kpad (= rows of a stage-2 B)
    float2 *PA = nullptr, *PB = nullptr, *PB2 = nullptr, *Pcol = nullptr;
    PackItem *pack = nullptr;
    int npack = 0;
    // gradient in tile form (lc.grad): B^H blocks (per (p, j): d x Wg), S regrouped by tile row
    // (per (p, i): lds x NA, Wg columns used), the partial planes of G2 and G3 (per (p, x): KS planes
    // of d x Wg)
    int64_t Wg = 0;
    float2 *PBH = nullptr, *Scol = nullptr, *GA = nullptr, *GBT = nullptr;
    PackItem *gpack = nullptr;
    TGradItem *gitems = nullptr;
    int ngpack = 0, ngitems = 0;
    size_t gzero_off = 0, gzero_bytes = 0;   // PBH .. Scol, from the region's start
    size_t bytes = 0, zero_bytes = 0;   // zero_bytes: PA .. PB2 (their padding must read as zero)
};

// Workspace region of the tile-form line search for `nprob` problems of class lc (laid out at base).
LineTile line_tile_carve(char *base, int nprob, const LineClass &lc, int64_t lds, int npack) {
    const bool grad = lc.grad;
    LineTile L;
    L.on = true;
    L.lc = lc;
    L.NA = (int64_t)lc.nt * 2 * lc.kpad;
    size_t o = 0;
    auto take = [&](size_t bytes) -> char * {
        char *q = base ? base + o : nullptr;
        o += align256(bytes);
        return q;
    };
    const size_t c8 = sizeof(float2);
    const int64_t nrr = (int64_t)lc.nt * lc.d;
    // one block: PA (per (p, i): d x NA), PB and PB2 (per (p, j): NA x d); the packing items address
    // all three from PA (line_tile_tables)
    const int64_t blk = (int64_t)nprob * nrr * L.NA;
    L.PA = (float2 *)take((size_t)3 * blk * c8);
    L.PB = L.PA ? L.PA + blk : nullptr;
    L.PB2 = L.PA ? L.PA + 2 * blk : nullptr;
    L.zero_bytes = o;
    // the tile gradient's G3 reads Wg columns from the theta half of every row: Wg past the end
    L.Wg = grad ? grad_tile_width(lc) : 0;
    const int64_t npc = (int64_t)nprob * lc.nt * lds * L.NA + L.Wg;
    L.Pcol = (float2 *)take((size_t)npc * c8);                          // per (p, j): lds x NA
    if (grad) {
        const int64_t zb = o;   // PBH and Scol: their padding must read as zero
        L.PBH = (float2 *)take((size_t)nprob * lc.nt * lc.d * L.Wg * c8);
        L.Scol = (float2 *)take((size_t)nprob * lc.nt * lds * L.NA * c8);   // row pitch NA, like Pcol
        L.gzero_off = zb;
        L.gzero_bytes = o - zb;
        L.GA = (float2 *)take((size_t)nprob * lc.nt * GRAD_TILE_KS * lc.d * L.Wg * c8);
        L.GBT = (float2 *)take((size_t)nprob * lc.nt * GRAD_TILE_KS * lc.d * L.Wg * c8);
        L.ngpack = nprob * lc.nt * lc.nt;
        L.ngitems = nprob * lc.nt * lc.nt;
        L.gpack = (PackItem *)take((size_t)L.ngpack * sizeof(PackItem));
        L.gitems = (TGradItem *)take((size_t)L.ngitems * sizeof(TGradItem));
    }
    L.pack = (PackItem *)take((size_t)npack * sizeof(PackItem));
    L.npack = npack;
    L.bytes = o;
    return L;
}

// Packing items of the run; theta_off[p]: the problem's offset in the theta-space vectors.
void line_tile_tables(const std::vector<const HostLayout *> &Hs, const std::vector<int64_t> &theta_off,
                      const LineClass &lc, int64_t lds, std::vector<PackItem> &pack) {
    const int nt = lc.nt, d = lc.d, kp = lc.kpad;
    const int64_t NA = (int64_t)nt * 2 * kp, nrr = (int64_t)nt * d;
    const int64_t nprob = (int64_t)Hs.size();
    const int64_t pb = nprob * nrr * NA, pb2 = 2 * pb;   // PB - PA, PB2 - PA (line_tile_carve)
    for (int64_t p = 0; p < nprob; ++p) {
        const HostLayout &H = *Hs[p];
        // tile index of (i, j): diagonal tiles first, then the sub-diagonal ones in t order
        std::vector<int> tix(nt * nt, -1);
        for (int i = 0; i < nt; ++i) tix[i * nt + i] = i;
        for (int i = 0, t = 0; i < nt; ++i)
            for (int j = 0; j < i; ++j, ++t) tix[i * nt + j] = tix[j * nt + i] = nt + t;
        const int64_t th = theta_off[p];
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < nt; ++j) {
                const TileDesc &td = H.tiles[tix[i * nt + j]];
                const int k = td.k;
                for (int from = 0; from < 2; ++from) {   // 0: theta block, 1: p block
                    // A block of row i, column block j: A_p at columns j kp, A_th at nt kp + j kp
                    PackItem a{};
                    a.from = from;
                    a.rows = d; a.cols = k;
                    a.dst = (p * nt + i) * d * NA + (from ? 0 : nt * kp) + j * kp;
                    a.ldd = NA;
                    // B block of column j, row block i, facing the stage-2 A columns: in PB, B_th at
                    // rows i kp (facing P_p) and B_p at rows nt kp + i kp (facing P_th); in PB2, B_p at
                    // rows i kp
                    PackItem b{};
                    b.from = from;
                    b.rows = k; b.cols = d;
                    b.dst = pb + (p * nt + j) * NA * d + (int64_t)((from ? nt * kp : 0) + i * kp) * d;
                    b.ldd = d;
                    if (i > j) {          // L (d x k), R (k x d) of tile (i, j)
                        a.op = PACK_COPY; a.src = th + td.offA; a.lds = k;
                        b.op = PACK_COPY; b.src = th + td.offB; b.lds = d;
                    } else if (i < j) {   // tile (j, i): X_ij = R^T L^T
                        a.op = PACK_TRANS; a.src = th + td.offB; a.lds = d;
                        b.op = PACK_TRANS; b.src = th + td.offA; b.lds = k;
                    } else {              // Q Q^T
                        a.op = PACK_COPY; a.src = th + td.offA; a.lds = k;
                        b.op = PACK_TRANS; b.src = th + td.offA; b.lds = k;
                    }
                    pack.push_back(a);
                    pack.push_back(b);
                    if (from) {           // X2 = A_p B_p: B_p also in the first half of the PB2 block
                        PackItem b2 = b;
                        b2.dst = pb2 + (p * nt + j) * NA * d + (int64_t)(i * kp) * d;
                        pack.push_back(b2);
                    }
                }
            }
    }
}

// Gradient items of a tile range: B^H packing into PBH and the gradient blocks from the G2 / G3 planes.
void grad_tile_tables(const std::vector<const HostLayout *> &Hs, const std::vector<int64_t> &theta_off,
                      const LineTile &L, std::vector<PackItem> &pack, std::vector<TGradItem> &items) {
    const LineClass &lc = L.lc;
    const int nt = lc.nt, d = lc.d, kp = lc.kpad;
    const int64_t Wg = L.Wg, plane = (int64_t)d * Wg, blk = GRAD_TILE_KS * plane;
    for (int64_t p = 0; p < (int64_t)Hs.size(); ++p) {
        const HostLayout &H = *Hs[p];
        std::vector<int> tix(nt * nt, -1);
        for (int i = 0; i < nt; ++i) tix[i * nt + i] = i;
        for (int i = 0, t = 0; i < nt; ++i)
            for (int j = 0; j < i; ++j, ++t) tix[i * nt + j] = tix[j * nt + i] = nt + t;
        const int64_t th = theta_off[p];
        for (int i = 0; i < nt; ++i)
            for (int j = 0; j < nt; ++j) {
                const TileDesc &td = H.tiles[tix[i * nt + j]];
                const int k = td.k;
                PackItem b{};   // B_ij^H (d x k) into column block i of PBH_(p, j)
                b.rows = d; b.cols = k;
                b.dst = (p * nt + j) * d * Wg + (int64_t)i * kp;
                b.ldd = Wg;
                if (i > j) {            // B = R (k x d)
                    b.op = PACK_CTRANS; b.src = th + td.offB; b.lds = d;
                } else {                // B = L_ji^T or Q^T: B^H = conj(L_ji), conj(Q) (d x k)
                    b.op = PACK_CONJ; b.src = th + td.offA; b.lds = k;
                }
                pack.push_back(b);
                if (i < j) continue;
                // grad A_ij (Q or L: d x k) = H_(p,i)[:, j kp ..]; grad R_ij (k x d) = H_(p,j)[:, i kp ..]^T
                TGradItem a{};
                a.rows = d; a.cols = k; a.trans = 0;
                a.src = (p * nt + i) * blk + (int64_t)j * kp;
                a.dst = th + td.offA;
                a.ldd = k;
                items.push_back(a);
                if (i == j) continue;
                TGradItem r{};
                r.rows = d; r.cols = k; r.trans = 1;
                r.src = (p * nt + j) * blk + (int64_t)i * kp;
                r.dst = th + td.offB;
                r.ldd = d;
                items.push_back(r);
            }
    }
}

int line_tile_counts(int nprob, const LineClass &lc, int &npack) {
    npack = nprob * lc.nt * lc.nt * 5;
    return 0;
}

// A run's problems in maximal ranges of one line-search form: dense (X1, X2 assembled, one product
// D [X1 | X2]) or one tile class. Batched calls order their problems so that every form is one range.
struct LineSeg {
    int p0 = 0, np = 0;
    bool tile = false;
    LineTile lt;                     // tile ranges: device state of the stages
};

bool tile_line_requested(int op, const tlrmdd_opts *opts) {
    return op >= 2 && opts && opts->line_products != TLRMDD_LINE_DENSE &&
           (opts->precision == TLRMDD_FP32_3M || opts->precision == TLRMDD_BF16X3);
}

// Ranges of the run and the bytes of their tile regions (carved back to back from `base`, or sized
// only when base is NULL).
std::vector<LineSeg> line_segments(int op, int count, const tlrmdd_plan *plans, const tlrmdd_opts *opts,
                                   int64_t lds, char *base, size_t *bytes, float2 **dcopy = nullptr) {
    std::vector<LineSeg> segs;
    std::vector<LineClass> cls(count);
    std::vector<bool> tile(count, false);
    for (int p = 0; p < count; ++p) tile[p] = problem_form(op, plans[p]->H, opts, cls[p]);
    // the adjoint product runs on the problems before the tile-form gradient: those form a suffix
    int suffix = count;
    while (suffix > 0 && tile[suffix - 1] && cls[suffix - 1].grad) --suffix;
    for (int p = 0; p < suffix; ++p) cls[p].grad = false;
    size_t o = 0;
    // BF16 mode stages D as split planes; the tile-form products read a complex64 copy (every problem
    // of the run, so that problem p's copy sits at p lds ldk), carved first
    bool any_tile = false;
    for (int p = 0; p < count; ++p) any_tile = any_tile || tile[p];
    if (dcopy) *dcopy = nullptr;
    if (any_tile && opts->precision == TLRMDD_BF16X3) {
        const int64_t ldk = round_up(plans[0]->H.nr, GEMM_PAD);
        if (dcopy) *dcopy = base ? (float2 *)base : nullptr;
        o += align256((size_t)count * lds * ldk * sizeof(float2));
    }
    for (int p = 0; p < count;) {
        int q = p + 1;
        while (q < count && tile[q] == tile[p] && (!tile[p] || cls[q] == cls[p])) ++q;
        LineSeg sg;
        sg.p0 = p;
        sg.np = q - p;
        sg.tile = tile[p];
        if (sg.tile) {
            int npack = 0;
            line_tile_counts(sg.np, cls[p], npack);
            sg.lt = line_tile_carve(base ? base + o : nullptr, sg.np, cls[p], lds, npack);
            o += align256(sg.lt.bytes);
            for (int e = p; e < q; ++e)
                for (const TileDesc &td : plans[e]->H.tiles) sg.lt.ksum += td.kind == TILE_LR ? 2.0 * td.k : td.k;
        }
        segs.push_back(sg);
        p = q;
    }
    if (bytes) *bytes = o;
    return segs;
}

constexpr int MAX_STREAMS = 8;   // sub-batches of a batched call (tlrmdd_opts.streams)

int check_opts(const tlrmdd_opts *o) {
    if (!o) return fail(TLRMDD_INVALID_ARGUMENT, "opts is NULL");
    if (o->iters < 0) return fail(TLRMDD_INVALID_ARGUMENT, "iters must be >= 0");
    if (o->optimizer != TLRMDD_LBFGS && o->optimizer != TLRMDD_GD)
        return fail(TLRMDD_INVALID_ARGUMENT, "unknown optimizer");
    if (o->optimizer == TLRMDD_LBFGS && (o->lbfgs_m < 1 || o->lbfgs_m > MAX_LBFGS_M))
        return fail(TLRMDD_INVALID_ARGUMENT, "lbfgs_m must be in [1, 32]");
    if (o->precision != TLRMDD_FP32 && o->precision != TLRMDD_BF16X3 && o->precision != TLRMDD_FP32_3M)
        return fail(TLRMDD_INVALID_ARGUMENT, "unknown precision");
    if (!(o->lambda >= 0.0)) return fail(TLRMDD_INVALID_ARGUMENT, "lambda must be >= 0");
    if (o->resid_refresh < 0) return fail(TLRMDD_INVALID_ARGUMENT, "resid_refresh must be >= 0");
    if (o->streams < 0 || o->streams > MAX_STREAMS) return fail(TLRMDD_INVALID_ARGUMENT, "streams must be in [0, 8]");
    if (o->line_products != TLRMDD_LINE_DENSE && o->line_products != TLRMDD_LINE_TILE &&
        o->line_products != TLRMDD_LINE_TILE_GRAD)
        return fail(TLRMDD_INVALID_ARGUMENT, "unknown line_products");
    return TLRMDD_OK;
}

// ---------------------------------------------------------------------------
// sub-batches on their own streams
// ---------------------------------------------------------------------------

// Extra streams (default priority, non-blocking), created on first use per (device, caller stream) and
// kept for the life of the process, so calls on different caller streams never share them; fork /
// join events come from a free list and belong to one call while it enqueues its work (a wait that
// has been enqueued keeps referring to the record it was enqueued after, so an event may be recorded
// again once its waits are enqueued).
struct StreamPool {
    std::mutex mu;
    std::map<std::pair<int, hipStream_t>, std::vector<hipStream_t>> streams;
    std::map<int, std::vector<hipEvent_t>> free_events;   // by device
};
StreamPool g_pool;

// The call's side streams and events; the events return to the free list when it ends.
struct CallStreams {
    int device = 0;
    std::vector<hipStream_t> st;
    std::vector<hipEvent_t> ev;
    ~CallStreams() {
        if (ev.empty()) return;
        std::lock_guard<std::mutex> lk(g_pool.mu);
        auto &F = g_pool.free_events[device];
        F.insert(F.end(), ev.begin(), ev.end());
    }
};

int pool_get(int n, int nev, hipStream_t caller, CallStreams &cs) {
    HIP_TRY(hipGetDevice(&cs.device));
    std::lock_guard<std::mutex> lk(g_pool.mu);
    auto &S = g_pool.streams[{cs.device, caller}];
    while ((int)S.size() < n) {
        hipStream_t x;
        HIP_TRY(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
        S.push_back(x);
    }
    cs.st.assign(S.begin(), S.begin() + n);
    auto &F = g_pool.free_events[cs.device];
    while ((int)cs.ev.size() < nev) {
        hipEvent_t e;
        if (!F.empty()) {
            e = F.back();
            F.pop_back();
        } else {
            HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        }
        cs.ev.push_back(e);
    }
    return TLRMDD_OK;
}

int stream_groups(const tlrmdd_opts *o, int count) { return std::max(1, std::min(o ? o->streams : 1, count)); }

// problem indices of sub-batch g of G: g, g + G, g + 2G, ... (every sub-batch gets the same mix)
std::vector<int> group_members(int g, int G, int count) {
    std::vector<int> m;
    for (int i = g; i < count; i += G) m.push_back(i);
    return m;
}

// Sub-batches of a batched call and the number of streams they run on: `streams` interleaved
// sub-batches, one per stream (problem i in sub-batch i mod streams, so every sub-batch gets the same
// mix). With the tile-form line search requested, every sub-batch lists its problems by form (the
// dense-form problems, then every tile class in order of first appearance, those with the gradient in
// tile form last), so each form is one range of its run (one launch per phase for the whole
// sub-batch, a launch per range for the line-search products, the adjoint product on the problems
// before the tile-form gradient ranges).
std::vector<std::vector<int>> make_groups(int count, const tlrmdd_plan *plans, const tlrmdd_opts *opts,
                                          int *nstreams) {
    std::vector<std::vector<int>> groups;
    if (tile_line_requested(2, opts)) {
        std::vector<int> dense;
        std::vector<LineClass> keys;
        std::vector<std::vector<int>> cls;
        for (int i = 0; i < count; ++i) {
            LineClass lc;
            if (!problem_form(2, plans[i]->H, opts, lc)) {
                dense.push_back(i);
                continue;
            }
            size_t k = 0;
            while (k < keys.size() && !(keys[k] == lc)) ++k;
            if (k == keys.size()) {
                keys.push_back(lc);
                cls.emplace_back();
            }
            cls[k].push_back(i);
        }
        std::vector<int> rank(count);   // position of every problem in form order
        int r = 0;
        for (int i : dense) rank[i] = r++;
        for (int pass = 0; pass < 2; ++pass)   // classes with the dense gradient, then the tile-form gradient
            for (size_t k = 0; k < cls.size(); ++k)
                if (keys[k].grad == (pass == 1))
                    for (int i : cls[k]) rank[i] = r++;
        const int G = stream_groups(opts, count);
        for (int g = 0; g < G; ++g) {
            std::vector<int> m = group_members(g, G, count);
            std::sort(m.begin(), m.end(), [&](int a, int b) { return rank[a] < rank[b]; });
            groups.push_back(m);
        }
        *nstreams = G;
        return groups;
    }
    const int G = stream_groups(opts, count);
    for (int g = 0; g < G; ++g) groups.push_back(group_members(g, G, count));
    *nstreams = G;
    return groups;
}

// a batched call splits into sub-batches (streams or tile-form line search)
bool grouped_call(int count, const tlrmdd_opts *opts) {
    return count > 1 && (stream_groups(opts, count) > 1 ||
                         tile_line_requested(2, opts));
}

template <typename T> std::vector<T> pick(const T *a, const std::vector<int> &idx) {
    std::vector<T> r;
    for (int i : idx) r.push_back(a[i]);
    return r;
}

// Workspace of G sub-batches: their own workspaces back to back (256-byte aligned).
int ws_bytes_grouped(int op, int count, const tlrmdd_plan *plans, const tlrmdd_opts *opts, size_t *bytes,
                     std::vector<size_t> *parts = nullptr);

// A second stream with its fork / join events for a run (see Run::side), or none.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

// Runs impl(sub-batch arrays, workspace slice, bytes, stream, side stream) for every sub-batch: the first on
// `stream`, the others on pool streams that wait for `stream` first and are waited for at the end.
template <typename Impl>
int run_grouped(int op, int count, const tlrmdd_plan *plans, const void *const *D, const void *const *U,
                void *const *theta, const tlrmdd_opts *opts, double *const *fhist, void *workspace,
                size_t ws_bytes, hipStream_t stream, Impl impl) {
    int S = 1;
    const std::vector<std::vector<int>> groups = make_groups(count, plans, opts, &S);
    std::vector<size_t> parts;
    size_t need = 0;
    int st = ws_bytes_grouped(op, count, plans, opts, &need, &parts);
    if (st) return st;
    if (!workspace || ws_bytes < need) return fail(TLRMDD_WORKSPACE, "workspace too small");
    // S sub-batches: S - 1 pool streams forked with event S - 1 and joined with events 0 .. S - 2;
    // one sub-batch: a pool stream serves as the run's side stream (events S and S + 1 fork and join it)
    CallStreams cs;
    if ((st = pool_get(S == 1 ? 1 : S - 1, S + 2, stream, cs))) return st;
    const std::vector<hipStream_t> &ps = cs.st;
    const std::vector<hipEvent_t> &ev = cs.ev;
    SideStream side;
    if (S == 1) {
        side.s = ps[0];
        side.fork = ev[S];
        side.join = ev[S + 1];
    }
    HIP_TRY(hipEventRecord(ev[S - 1], stream));
    for (int k = 0; k < S - 1; ++k) HIP_TRY(hipStreamWaitEvent(ps[k], ev[S - 1], 0));
    char *base = static_cast<char *>(workspace);
    int first_err = TLRMDD_OK;
    for (size_t g = 0; g < groups.size(); ++g) {
        const std::vector<int> &m = groups[g];
        const std::vector<tlrmdd_plan> gp = pick(plans, m);
        const std::vector<const void *> gd = pick(D, m), gu = pick(U, m);
        const std::vector<void *> gt = pick(theta, m);
        const std::vector<double *> gf = pick(fhist, m);
        const int k = (int)(g % S);
        const int e = impl((int)m.size(), gp.data(), gd.data(), gu.data(), gt.data(), gf.data(), base, parts[g],
                           k == 0 ? stream : ps[k - 1], S == 1 ? &side : nullptr);
        if (e && !first_err) first_err = e;
        base += align256(parts[g]);
    }
    for (int k = 0; k < S - 1; ++k) {
        HIP_TRY(hipEventRecord(ev[k], ps[k]));
        HIP_TRY(hipStreamWaitEvent(stream, ev[k], 0));
    }
    return first_err;
}

int check_precision(int precision) {
    if (precision == TLRMDD_FP32 || precision == TLRMDD_BF16X3 || precision == TLRMDD_FP32_3M) return TLRMDD_OK;
    return fail(TLRMDD_INVALID_ARGUMENT, "unknown precision");
}

GemmArgs gemm_args() {
    GemmArgs g;
    std::memset(&g, 0, sizeof(g));
    return g;
}

FinArgs fin_args(int op, SolveScalars *sc) {
    FinArgs f;
    std::memset(&f, 0, sizeof(f));
    f.op = op;
    f.sc = sc;
    f.m1 = 1;
    return f;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *tlrmdd_status_string(int status) {
    switch (status) {
        case TLRMDD_OK: return "ok";
        case TLRMDD_INVALID_ARGUMENT: return "invalid argument";
        case TLRMDD_WORKSPACE: return "workspace too small or allocation failed";
        case TLRMDD_HIP_ERROR: return "HIP runtime error";
        case TLRMDD_NONFINITE: return "non-finite value";
        case TLRMDD_UNSUPPORTED: return "unsupported";
        case TLRMDD_NOT_CONVERGED: return "not converged";
        default: return "unknown status";
    }
}

const char *tlrmdd_last_error(void) { return g_last_error.c_str(); }

int64_t tlrmdd_theta_size(const tlrmdd_layout *layout) {
    HostLayout H;
    if (build_layout(layout, H) != TLRMDD_OK) return -1;
    return H.theta_size;
}

int tlrmdd_plan_create(const tlrmdd_layout *layout, tlrmdd_plan *plan_out) {
    g_last_error.clear();
    if (!plan_out) return fail(TLRMDD_INVALID_ARGUMENT, "plan_out is NULL");
    *plan_out = nullptr;
    tlrmdd_plan P = new (std::nothrow) tlrmdd_plan_s();
    if (!P) return fail(TLRMDD_WORKSPACE, "host allocation failed");
    int st = build_layout(layout, P->H);
    if (st != TLRMDD_OK) { delete P; return st; }
    P->ldk = round_up(P->H.nr, GEMM_PAD);
    P->lds = round_up(P->H.ns, GEMM_PAD);
    append_problem(P->T, P->H, 0, 0, P->ldk);
    build_segments(P->T, {&P->H}, P->lds, P->ldk);
    assign_parts(P->T, partial_stride(P->T, P->ldk, P->lds));
    hipError_t e = hipGetDevice(&P->device);
    if (e == hipSuccess) e = hipMalloc(&P->d_block, tables_bytes(P->T, 1));
    if (e == hipSuccess) {
        std::vector<char> img;
        pack_tables(P->T, 1, (char *)P->d_block, img, P->D, nullptr);
        e = hipMemcpy(P->d_block, img.data(), img.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        if (P->d_block) (void)hipFree(P->d_block);
        delete P;
        return fail(TLRMDD_HIP_ERROR, std::string("plan tables: ") + hipGetErrorString(e));
    }
    *plan_out = P;
    return TLRMDD_OK;
}

int tlrmdd_plan_destroy(tlrmdd_plan plan) {
    if (!plan) return TLRMDD_OK;
    if (plan->d_block) (void)hipFree(plan->d_block);
    delete plan;
    return TLRMDD_OK;
}

static size_t ws_bytes_single(const tlrmdd_plan P, int op, int m1) {
    const Tables &T = P->T;
    const int ps = partial_stride(T, P->ldk, P->lds);
    return carve(nullptr, op, 1, P->ldk, P->lds, theta_span(P->H.theta_size), m1, ps, 0).bytes;
}

int tlrmdd_workspace_bytes(tlrmdd_plan plan, int op, const tlrmdd_opts *opts, size_t *bytes) {
    g_last_error.clear();
    if (!plan || !bytes) return fail(TLRMDD_INVALID_ARGUMENT, "plan / bytes is NULL");
    if (op < 0 || op > 2) return fail(TLRMDD_INVALID_ARGUMENT, "unknown op");
    int m1 = 1;
    if (op == TLRMDD_OP_SOLVE) {
        int st = check_opts(opts);
        if (st != TLRMDD_OK) return st;
        m1 = (opts->optimizer == TLRMDD_LBFGS) ? opts->lbfgs_m + 1 : 1;
    }
    *bytes = ws_bytes_single(plan, op, m1);
    if (op == TLRMDD_OP_SOLVE) {
        size_t tb = 0;
        line_segments(op, 1, &plan, opts, plan->lds, nullptr, &tb);
        *bytes += tb;
    }
    return TLRMDD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// shared pieces of forward / grad / solve
// ---------------------------------------------------------------------------
namespace {

// the tables of a batch into the workspace (queued on `up`)
void upload_tables(const Tables &T, int nprob, const Ws &w, DevTables &D, double *const *fhist, Upload &up) {
    std::vector<char> img;
    pack_tables(T, nprob, w.tables, img, D, fhist);
    up.add(w.tables, img.data(), img.size());
}

struct Ctx {
    int nprob;
    int64_t nr, ns, ldk, lds;   // true sizes and padded sizes (ldk >= nr, lds >= ns)
    int pstride;
    Ws w;
    DevTables D;
    hipStream_t s;
    bool bf16 = false;          // BF16 hi+lo split products
    bool p3m = false;           // FP32 products in the three-real-product form
    int64_t xspace = 0;         // complex64 elements of X space per problem (1 or 2 ldk x ldk)

    int form() const { return bf16 ? F_BF16X3 : p3m ? F_3M : F_4M; }
    // split planes (uint32 words, one per complex): per problem [hi | lo]
    uint32_t *dsw() const { return reinterpret_cast<uint32_t *>(w.Ds); }
    uint32_t *dhw() const { return reinterpret_cast<uint32_t *>(w.DHs); }
    uint32_t *xw() const { return reinterpret_cast<uint32_t *>(w.XW); }
    // X space in split form: X1 hi at 0, X2 hi at ldk^2, lo planes at + xspace words
    int64_t lo_words() const { return xspace; }
};

int fin(const Ctx &c, FinArgs f, const int32_t *counts, int ucount, int nsum) {
    f.partials = c.w.partials;
    f.pstride = c.pstride;
    f.counts = counts;
    f.ucount = ucount;
    f.nsum = nsum;
    HIP_TRY(launch_finalize(f, c.nprob, c.s));
    return TLRMDD_OK;
}

// The dense products contract over the true length rounded up to the kernel's k step (16 complex,
// 32 for the BF16 ring), not over the padded one: the padding is zero and would only add stages.
int gemm_resid(const Ctx &c, const float2 *X, int64_t sX, const float2 *U, int64_t ldu, int64_t sU, float2 *r) {
    const double np = c.nprob, ns = (double)c.ns, nr = (double)c.nr;
    const Work wk = gemm_work(c.form(), 8.0 * ns * nr * nr * np, 8.0 * np * (3.0 * ns * nr + nr * nr));
    if (c.bf16) {
        // X given as the split planes that start at the same place (word 2 * offset of X)
        const uint32_t *xh = reinterpret_cast<const uint32_t *>(X);
        GemmArgsB g;
        std::memset(&g, 0, sizeof(g));
        g.Ahi = reinterpret_cast<const uint16_t *>(c.dsw());
        g.Alo = reinterpret_cast<const uint16_t *>(c.dsw() + c.lds * c.ldk);
        g.lda = c.ldk; g.sA = 2 * c.lds * c.ldk;
        g.Bhi = reinterpret_cast<const uint16_t *>(xh);
        g.Blo = reinterpret_cast<const uint16_t *>(xh + c.lo_words());
        g.ldb = c.ldk; g.sB = 2 * sX;
        g.C = r; g.ldc = c.ldk; g.sC = c.lds * c.ldk;
        g.E = U; g.lde = ldu; g.sE = sU;
        g.partials = c.w.partials; g.sP = (int64_t)c.pstride;
        g.M = (int)c.lds; g.N = (int)c.ldk; g.K = (int)round_up(c.nr, 32);
        g.Me = (int)c.ns; g.Ne = (int)c.nr;
        HIP_TRY(timed(TLRMDD_K_GEMM_RESID, c.s, wk, [&] { return launch_cgemm_bf16(GM_RESID, g, c.nprob, c.s); }));
        return TLRMDD_OK;
    }
    GemmArgs g = gemm_args();
    g.A = c.w.Ds; g.lda = c.ldk; g.sA = c.lds * c.ldk;
    g.B = X; g.ldb = c.ldk; g.sB = sX;
    g.C = r; g.ldc = c.ldk; g.sC = c.lds * c.ldk;
    g.E = U; g.lde = ldu; g.sE = sU;
    g.partials = c.w.partials; g.sP = (int64_t)c.pstride;   // one sum per workgroup
    g.M = (int)c.lds; g.N = (int)c.ldk; g.K = (int)round_up(c.nr, GEMM_BK);
    g.Me = (int)c.ns; g.Ne = (int)c.nr;
    HIP_TRY(timed(TLRMDD_K_GEMM_RESID, c.s, wk, [&] {
        return c.p3m ? launch_cgemm3m(GM_RESID, g, c.nprob, c.s) : launch_cgemm(GM_RESID, g, c.nprob, c.s);
    }));
    return TLRMDD_OK;
}

int gemm_adjoint(const Ctx &c, const float2 *r, float2 *W, int64_t sW) {
    const double np = c.nprob, ns = (double)c.ns, nr = (double)c.nr;
    const Work wk = gemm_work(c.form(), 8.0 * nr * ns * nr * np, 8.0 * np * (2.0 * ns * nr + nr * nr));
    if (c.bf16) {
        // r^T split planes (written by split_r_transpose) are the transposed B operand
        GemmArgsB g;
        std::memset(&g, 0, sizeof(g));
        g.Ahi = reinterpret_cast<const uint16_t *>(c.dhw());
        g.Alo = reinterpret_cast<const uint16_t *>(c.dhw() + c.ldk * c.lds);
        g.lda = c.lds; g.sA = 2 * c.ldk * c.lds;
        g.Bhi = reinterpret_cast<const uint16_t *>(c.w.rT);
        g.Blo = reinterpret_cast<const uint16_t *>(c.w.rT + c.ldk * c.lds);
        g.ldb = c.lds; g.sB = 2 * c.ldk * c.lds;
        g.C = W; g.ldc = c.ldk; g.sC = sW;
        g.M = (int)c.ldk; g.N = (int)c.ldk; g.K = (int)round_up(c.ns, 32);
        HIP_TRY(timed(TLRMDD_K_GEMM_ADJOINT, c.s, wk, [&] { return launch_cgemm_bf16(GM_STORE, g, c.nprob, c.s); }));
        return TLRMDD_OK;
    }
    GemmArgs g = gemm_args();
    g.A = c.w.DHs; g.lda = c.lds; g.sA = c.ldk * c.lds;
    g.B = r; g.ldb = c.ldk; g.sB = c.lds * c.ldk;
    g.C = W; g.ldc = c.ldk; g.sC = sW;
    g.M = (int)c.ldk; g.N = (int)c.ldk; g.K = (int)round_up(c.ns, GEMM_BK);
    HIP_TRY(timed(TLRMDD_K_GEMM_ADJOINT, c.s, wk, [&] {
        return c.p3m ? launch_cgemm3m(GM_STORE, g, c.nprob, c.s) : launch_cgemm(GM_STORE, g, c.nprob, c.s);
    }));
    return TLRMDD_OK;
}

int gemm_line(const Ctx &c, const float2 *X1, const float2 *X2, int64_t sX) {
    const double np = c.nprob, ns = (double)c.ns, nr = (double)c.nr;
    const Work wk = gemm_work(c.form(), 16.0 * ns * nr * nr * np, 8.0 * np * (4.0 * ns * nr + 2.0 * nr * nr));
    if (c.bf16) {
        const uint32_t *xh = reinterpret_cast<const uint32_t *>(X1);
        GemmArgsB g;
        std::memset(&g, 0, sizeof(g));
        g.Ahi = reinterpret_cast<const uint16_t *>(c.dsw());
        g.Alo = reinterpret_cast<const uint16_t *>(c.dsw() + c.lds * c.ldk);
        g.lda = c.ldk; g.sA = 2 * c.lds * c.ldk;
        g.Bhi = reinterpret_cast<const uint16_t *>(xh);
        g.Blo = reinterpret_cast<const uint16_t *>(xh + c.lo_words());
        g.ldb = c.ldk; g.sB = 2 * sX; g.b2_rows = c.ldk;   // X2 planes follow X1's ldk rows
        g.C = c.w.a; g.C2 = c.w.b; g.ldc = c.ldk; g.sC = c.lds * c.ldk;
        g.E = c.w.r; g.lde = c.ldk; g.sE = c.lds * c.ldk;
        g.partials = c.w.partials; g.sP = (int64_t)c.pstride * 5;
        g.M = (int)c.lds; g.N = (int)c.ldk; g.K = (int)round_up(c.nr, 32);
        HIP_TRY(timed(TLRMDD_K_GEMM_LINE, c.s, wk, [&] { return launch_cgemm_bf16(GM_LINE, g, c.nprob, c.s); }));
        return TLRMDD_OK;
    }
    GemmArgs g = gemm_args();
    g.A = c.w.Ds; g.lda = c.ldk; g.sA = c.lds * c.ldk;
    g.B = X1; g.B2 = X2; g.ldb = c.ldk; g.sB = sX;
    g.C = c.w.a; g.C2 = c.w.b; g.ldc = c.ldk; g.sC = c.lds * c.ldk;
    g.E = c.w.r; g.lde = c.ldk; g.sE = c.lds * c.ldk;
    g.partials = c.w.partials; g.sP = (int64_t)c.pstride * 5;
    g.M = (int)c.lds; g.N = (int)c.ldk; g.K = (int)round_up(c.nr, GEMM_BK);
    HIP_TRY(timed(TLRMDD_K_GEMM_LINE, c.s, wk, [&] {
        return c.p3m ? launch_cgemm3m(GM_LINE, g, c.nprob, c.s) : launch_cgemm(GM_LINE, g, c.nprob, c.s);
    }));
    return TLRMDD_OK;
}

// r^T split planes for the BF16 adjoint product
int split_r_transpose(const Ctx &c) {
    if (!c.bf16) return TLRMDD_OK;
    HIP_TRY(launch_split_transpose(c.w.r, c.ldk, c.lds, c.ldk, c.w.rT, c.w.rT + c.ldk * c.lds, c.lds, c.nprob,
                                   c.lds * c.ldk, 2 * c.ldk * c.lds, c.s));
    return TLRMDD_OK;
}

// staging of D for problem p (padded; split planes in BF16 mode): reads D, writes D and D^H
int stage(const Ctx &c, int p, const float2 *D, bool with_dh) {
    const Work wk = bytes_work((with_dh ? 24.0 : 16.0) * (double)c.ns * (double)c.nr);
    if (c.bf16) {
        uint32_t *dh = c.dsw() + (int64_t)p * 2 * c.lds * c.ldk;
        uint32_t *hh = with_dh ? c.dhw() + (int64_t)p * 2 * c.ldk * c.lds : nullptr;
        HIP_TRY(timed(TLRMDD_K_STAGE, c.s, wk, [&] {
            return launch_stage_d_split(D, c.ns, c.nr, dh, dh + c.lds * c.ldk, c.ldk, hh,
                                        hh ? hh + c.ldk * c.lds : nullptr, c.lds, c.s);
        }));
    } else {
        HIP_TRY(timed(TLRMDD_K_STAGE, c.s, wk, [&] {
            return launch_stage_d(D, c.ns, c.nr, c.w.Ds + (int64_t)p * c.lds * c.ldk, c.ldk,
                                  with_dh ? c.w.DHs + (int64_t)p * c.ldk * c.lds : nullptr, c.lds, c.s);
        }));
    }
    return TLRMDD_OK;
}

int resid_tiles(const Ctx &c) { return gemm_partials_per_problem(GM_RESID, (int)c.lds, (int)c.ldk); }
int line_tiles(const Ctx &c) { return gemm_partials_per_problem(GM_LINE, (int)c.lds, (int)c.ldk) / 5; }

// The whole solve, for one problem or a batch of equal-shape problems.
// One run of the solver over `nprob` problems of one shape: tables, workspace views, staged operands
// and the tracked residual. Setup stages D and U, copies theta in and forms r = D C(theta) - U; then
// any number of iterate() calls continue from the current theta and residual.
struct Run {
    Ctx c;
    Tables T;
    bool single = true, lbfgs = true;
    int m = 0, m1 = 1;
    int64_t xstride = 0, rstride = 0, x2w = 0, stride2 = 0;
    float2 *X1 = nullptr, *X2 = nullptr;
    int nt = 0, nrs = 0;
    float *gcur = nullptr, *gprev = nullptr;
    double *fhist0 = nullptr;
    const tlrmdd_opts *opts = nullptr;
    // ADMM state (op 3): split variable, scaled dual, penalty center
    float *z = nullptr, *u = nullptr, *cen = nullptr;
    std::vector<LineSeg> segs;       // line-search form of every problem range
    std::vector<int> asm_first;      // first assembly item of every problem, and the total
    std::vector<int> grad_first;     // first gradient item of every problem, and the total
    int n_adj = 0;                   // problems before the tile-form gradient ranges (adjoint product)
    std::vector<double> theta_pre;   // complex unknowns of problems 0 .. p - 1 (true sizes)
    std::vector<double> asm_pre, asm_dir_pre, grad_pre;   // tile-product complex flops, likewise
    // a second stream (default priority) on which the tile-form gradient runs beside the adjoint
    // product of the other problems, and the events that fork it from and join it to c.s
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};

// The context of problems p0 .. p0 + np - 1 of a run for the line-search products (complex64 operands
// and the line-search partial slots offset to the first problem).
Ctx line_ctx(const Ctx &c, int p0, int np) {
    Ctx s = c;
    const int64_t rs = c.lds * c.ldk;
    s.nprob = np;
    s.w.Ds += p0 * rs;
    if (s.w.Dc) s.w.Dc += p0 * rs;
    if (s.w.DHs) s.w.DHs += p0 * rs;
    s.w.r += p0 * rs;
    s.w.a += p0 * rs;
    s.w.b += p0 * rs;
    s.w.partials += (int64_t)p0 * c.pstride * 5;
    return s;
}

// Stage 1 of a tile range: pack the factor blocks of theta and of the direction `dir`, then
// Pcol_(p,j) = [D_:,i A_dir(ij) ... | D_:,i A_th(ij) ...] (see LineTile), or the direction half only
// (dir_only: the theta half is carried by P_th += step P_p in ranges with the tile-form gradient)
int tile_stage1(Run &R, const LineSeg &sg, const float *dir, bool dir_only = false, bool theta_only = false,
                hipStream_t stream = nullptr) {
    Ctx c = line_ctx(R.c, sg.p0, sg.np);
    if (stream) c.s = stream;
    const LineTile &L = sg.lt;
    const LineClass &lc = L.lc;
    const int64_t NA = L.NA, d = lc.d, nt = lc.nt;
    const double ks = L.ksum, dd = (double)d, ns = (double)c.ns, nr = (double)c.nr, np = c.nprob;
    // the A and B blocks of theta and of the direction, and B_p once more: 5 d ksum entries
    HIP_TRY(timed(TLRMDD_K_LINE_PACK, c.s, bytes_work(16.0 * 5.0 * dd * ks), [&] {
        return launch_tlr_pack(L.pack, L.npack, (const float2 *)c.w.th, L.PA, c.s, (const float2 *)dir, 2);
    }));
    GemmArgs g1 = gemm_args();   // stage 1: P_(p,i) = D_p[:, i d ...] PA_(p,i)
    const int64_t half = theta_only ? nt * lc.kpad : 0;   // the theta half starts nt kpad columns in
    g1.A = c.w.Dc; g1.lda = c.ldk; g1.sA = c.lds * c.ldk; g1.sA2 = d;
    g1.B = L.PA + half; g1.ldb = NA; g1.sB = nt * d * NA; g1.sB2 = d * NA;
    // stored regrouped by tile column: block j of row i -> Pcol_(p,j) at columns i kpad (each half)
    g1.C = L.Pcol + half; g1.ldc = NA; g1.sC = nt * c.lds * NA; g1.sC2 = lc.kpad;
    const int N = (dir_only || theta_only) ? (int)(nt * lc.kpad) : (int)NA;
    g1.scat_kp = lc.kpad; g1.scat_w = (int)(nt * lc.kpad); g1.scat_lim = N; g1.scat_js = c.lds * NA - lc.kpad;
    g1.M = (int)c.lds; g1.N = N; g1.K = (int)d;
    g1.nz2 = (int)nt;
    const double h = (dir_only || theta_only) ? 1.0 : 2.0;   // halves formed
    const Work wk = gemm_work(F_3M, 8.0 * ns * dd * ks * h, 8.0 * (ns * nr * np + dd * ks * h + ns * ks * h));
    HIP_TRY(timed(TLRMDD_K_LINE_TILE, c.s, wk, [&] {
        return launch_cgemm3m(GM_STORE, g1, (int)(c.nprob * nt), c.s, GR_TILE);
    }));
    return TLRMDD_OK;
}

// [a | b] = D [X1 | X2] with the five line-search sums for the problems of a tile range (see LineTile).
// dir_only: stage 1 forms the direction half only (the theta half is current, see tile_pcol_update).
int line_products_tile(Run &R, const LineSeg &sg, bool dir_only = false, hipStream_t stream = nullptr) {
    int st = tile_stage1(R, sg, R.c.w.p, dir_only, false, stream);
    if (st) return st;
    Ctx c = line_ctx(R.c, sg.p0, sg.np);
    if (stream) c.s = stream;
    const LineTile &L = sg.lt;
    const LineClass &lc = L.lc;
    const int64_t NA = L.NA, d = lc.d, nt = lc.nt;
    GemmArgs g2 = gemm_args();   // stage 2: [a | b]_(p, columns of tile j) = Pcol_(p,j) [PB | PB2]_(p,j)
    g2.A = L.Pcol; g2.lda = NA; g2.sA = nt * c.lds * NA; g2.sA2 = c.lds * NA;
    g2.B = L.PB; g2.B2 = L.PB2; g2.ldb = d; g2.sB = nt * NA * d; g2.sB2 = NA * d;
    g2.C = c.w.a; g2.C2 = c.w.b; g2.ldc = c.ldk; g2.sC = c.lds * c.ldk; g2.sC2 = d;
    g2.E = c.w.r; g2.lde = c.ldk; g2.sE = c.lds * c.ldk; g2.sE2 = d;
    g2.partials = c.w.partials; g2.sP = (int64_t)c.pstride * 5;
    g2.sP2 = (c.lds / GEMM_BM) * (d / (GEMM_BN / 2)) * 5;   // the line tiles of one tile column
    g2.M = (int)c.lds; g2.N = (int)d; g2.K = (int)NA;
    g2.K2 = (int)(nt * lc.kpad);   // b: the direction half of Pcol only
    g2.nz2 = (int)nt;
    {   // a: K = 2 ksum, b: K = ksum per tile column; reads Pcol, the B blocks of theta and p, r; writes a, b
        const double ks = L.ksum, dd = (double)d, ns = (double)c.ns, nr = (double)c.nr, np = c.nprob;
        const Work wk = gemm_work(F_3M, 24.0 * ns * dd * ks,
                                  8.0 * (2.0 * ns * ks + 2.0 * ks * dd + 3.0 * ns * nr * np));
        HIP_TRY(timed(TLRMDD_K_LINE_TILE, c.s, wk, [&] {
            return launch_cgemm3m(GM_LINE, g2, (int)(c.nprob * nt), c.s, GR_TILE);
        }));
    }
    return TLRMDD_OK;
}

// Gradient of the problems of a tile range in tile form (see GRAD_TILE_MAX_COST), into g. Needs the
// theta half of Pcol for the current theta.
int tile_gradient(Run &R, const LineSeg &sg, float *g, hipStream_t stream) {
    Ctx c = line_ctx(R.c, sg.p0, sg.np);
    c.s = stream;
    const LineTile &L = sg.lt;
    const LineClass &lc = L.lc;
    const int64_t NA = L.NA, d = lc.d, nt = lc.nt, kp = lc.kpad, Wg = L.Wg;
    const int KS = GRAD_TILE_KS;
    const int64_t Kc = c.lds / KS;
    const double ks = L.ksum, dd = (double)d, ns = (double)c.ns, nr = (double)c.nr, np = c.nprob;
    HIP_TRY(timed(TLRMDD_K_LINE_PACK, c.s, bytes_work(16.0 * dd * ks), [&] {
        return launch_tlr_pack(L.gpack, L.ngpack, (const float2 *)c.w.th, L.PBH, c.s, nullptr, 2);
    }));
    GemmArgs g1 = gemm_args();   // G1: S_(p,j) = r_p[:, j d ...] PBH_(p,j), stored as Scol_(p,i)[:, j kp ...]
    g1.A = c.w.r; g1.lda = c.ldk; g1.sA = c.lds * c.ldk; g1.sA2 = d;
    g1.B = L.PBH; g1.ldb = Wg; g1.sB = nt * d * Wg; g1.sB2 = d * Wg;
    g1.C = L.Scol; g1.ldc = NA; g1.sC = nt * c.lds * NA; g1.sC2 = kp;
    g1.scat_kp = (int)kp; g1.scat_w = (int)(nt * kp); g1.scat_lim = (int)(nt * kp); g1.scat_js = c.lds * NA - kp;
    g1.M = (int)c.lds; g1.N = (int)Wg; g1.K = (int)d;
    g1.nz2 = (int)nt;
    HIP_TRY(timed(TLRMDD_K_GRAD_TILE, c.s,
                  gemm_work(F_3M, 8.0 * ns * dd * ks, 8.0 * (ns * nr * np + dd * ks + ns * ks)), [&] {
                      return launch_cgemm3m(GM_STORE, g1, (int)(c.nprob * nt), c.s, GR_TILE);
                  }));
    // G2 and G3 in one launch of the transposed-A / conjugated-B role, per (p, tile x, part q):
    //   set 0: GBT_(p,x,q) = r_p[q Kc ..., x d ...]^T conj(Pcol_th(p,x)[q Kc ...])
    //   set 1: conj(GA_(p,x,q)) = D_p[q Kc ..., x d ...]^T conj(Scol_(p,x)[q Kc ...])
    // (the same strides: D and r, Pcol and Scol share their layouts)
    GemmArgs g3 = gemm_args();
    g3.A = c.w.r; g3.lda = c.ldk; g3.sA = c.lds * c.ldk; g3.sA2 = d; g3.sA3 = Kc * c.ldk; g3.sA4 = c.w.Dc - c.w.r;
    g3.B = L.Pcol + nt * kp; g3.ldb = NA; g3.sB = nt * c.lds * NA; g3.sB2 = c.lds * NA; g3.sB3 = Kc * NA;
    g3.sB4 = L.Scol - (L.Pcol + nt * kp);
    g3.C = L.GBT; g3.ldc = Wg; g3.sC = nt * KS * d * Wg; g3.sC2 = KS * d * Wg; g3.sC3 = d * Wg; g3.sC4 = L.GA - L.GBT;
    g3.M = (int)d; g3.N = (int)Wg; g3.K = (int)Kc;
    g3.nz2 = (int)(nt * KS * 2); g3.nz3 = KS; g3.nz4 = 2;
    HIP_TRY(timed(TLRMDD_K_GRAD_TILE, c.s,
                  gemm_work(F_3M, 16.0 * ns * dd * ks, 8.0 * (2.0 * ns * nr * np + 2.0 * ns * ks + 2.0 * dd * ks)),
                  [&] { return launch_cgemm3m(GM_STORE, g3, (int)(c.nprob * nt * KS * 2), c.s, GR_TILE_TA_CB); }));
    // every gradient entry (d ksum of them) from 2 KS partial planes
    HIP_TRY(timed(TLRMDD_K_LINE_PACK, c.s, bytes_work(8.0 * (2.0 * KS + 1.0) * dd * ks), [&] {
        return launch_tlr_grad(L.gitems, L.ngitems, L.GA, L.GBT, KS, d * Wg, Wg, true, (float2 *)g, c.s);
    }));
    return TLRMDD_OK;
}

// r = D C(theta) - U for the problems of a range with the tile-form gradient, from the factors
// (the tile low-rank product): P_th afresh by stage 1 on theta, then per tile column
// r_:,j = sum_i P_th(ij) B_th(ij) - U_:,j with the FP64 partial sums of |r|^2 (K = nt kpad instead of nr).
int tile_resid(Run &R, const LineSeg &sg) {
    const LineTile &L = sg.lt;
    const LineClass &lc = L.lc;
    const int64_t NA = L.NA, d = lc.d, nt = lc.nt, kp = lc.kpad;
    const bool halves = (nt * kp) % GEMM_BN == 0;
    int st = tile_stage1(R, sg, R.c.w.th, false, halves);
    if (st) return st;
    const Ctx &c0 = R.c;
    const int64_t rs = c0.lds * c0.ldk;
    GemmArgs g = gemm_args();
    g.A = L.Pcol + nt * kp; g.lda = NA; g.sA = nt * c0.lds * NA; g.sA2 = c0.lds * NA;
    g.B = L.PB; g.ldb = d; g.sB = nt * NA * d; g.sB2 = NA * d;   // rows i kpad: B_th(ij)
    g.C = c0.w.r + sg.p0 * rs; g.ldc = c0.ldk; g.sC = rs; g.sC2 = d;
    g.E = c0.w.Us + sg.p0 * rs; g.lde = c0.ldk; g.sE = rs; g.sE2 = d;
    g.partials = c0.w.partials + (int64_t)sg.p0 * c0.pstride; g.sP = c0.pstride;
    g.sP2 = (c0.lds / GEMM_BM) * (d / GEMM_BN);   // the residual tiles of one tile column
    g.M = (int)c0.lds; g.N = (int)d; g.K = (int)(nt * kp);
    g.Me = (int)c0.ns; g.Ne = (int)d;             // E's columns are local to the tile column
    g.nz2 = (int)nt;
    const double ks = L.ksum, dd = (double)d, ns = (double)c0.ns, nr = (double)c0.nr, np = sg.np;
    const Work wk = gemm_work(F_3M, 8.0 * ns * dd * ks, 8.0 * (ns * ks + dd * ks + 2.0 * ns * nr * np));
    HIP_TRY(timed(TLRMDD_K_RESID_TILE, c0.s, wk, [&] {
        return launch_cgemm3m(GM_RESID, g, (int)(sg.np * nt), c0.s, GR_TILE);
    }));
    return TLRMDD_OK;
}

// After the update theta += step p: the theta half of Pcol follows (P_th += step P_p).
int tile_pcol_update(Run &R, const LineSeg &sg) {
    const Ctx c = line_ctx(R.c, sg.p0, sg.np);
    const LineTile &L = sg.lt;
    const int64_t nt = L.lc.nt;
    HIP_TRY(timed(TLRMDD_K_LINE_PACK, c.s, bytes_work(24.0 * (double)c.ns * L.ksum), [&] {
        return launch_tlr_paxpy(L.Pcol, (int)(c.nprob * nt), (int)nt, c.lds * L.NA, c.lds, L.NA, nt * L.lc.kpad,
                                c.w.sc + sg.p0, c.s);
    }));
    return TLRMDD_OK;
}

// Split planes of the X space: W (complex64, written by the adjoint product) overlays them with a
// different element layout, so their padding must be re-zeroed before each assembly.
int clear_plane_padding(Run &R) {
    Ctx &c = R.c;
    if (!c.bf16 || c.ldk == c.nr) return TLRMDD_OK;
    HIP_TRY(launch_zero_pad(c.xw(), c.ldk, c.nr, 4, c.ldk * c.ldk, c.nprob, 2 * R.xstride, c.s));
    return TLRMDD_OK;
}

// record < 0: no f-history entry
int fin_f(Run &R, int record, double lam, int nsum_parts) {
    FinArgs f = fin_args(FIN_F, R.c.w.sc);
    if (record >= 0) {
        f.fhist = R.single ? nullptr : R.c.D.fhist;
        f.fhist0 = R.fhist0;
        f.t = record;
    }
    f.lam = lam;
    return fin(R.c, f, nullptr, nsum_parts, 1);
}

// r = D C(theta) - U afresh: assembly and the dense product for the problems before the tile-form
// gradient ranges, the tile low-rank product for those
int objective_fresh(Run &R, int record, double lam) {
    Ctx &c = R.c;
    int e = 0;
    if (R.n_adj > 0) {
        if ((e = clear_plane_padding(R))) return e;
        const int na = (R.single || R.n_adj == c.nprob) ? c.D.n_asm : R.asm_first[R.n_adj];
        const double nr = (double)c.nr;
        const Work wk = gemm_work(F_4M, R.asm_pre[R.n_adj], 8.0 * (nr * nr * R.n_adj + R.theta_pre[R.n_adj]));
        HIP_TRY(timed(TLRMDD_K_ASSEMBLE, c.s, wk, [&] {
            return launch_assemble(false, c.D.tiles, c.D.asm_items, na, c.D.probs, (const float2 *)c.w.th,
                                   nullptr, R.X1, nullptr, c.s, c.bf16, R.x2w, c.lo_words());
        }));
        Ctx ca = c;
        ca.nprob = R.n_adj;
        if ((e = gemm_resid(ca, R.X1, R.xstride, c.w.Us, c.ldk, R.rstride, c.w.r))) return e;
    }
    for (const LineSeg &sg : R.segs)
        if (sg.tile && sg.lt.lc.grad)
            if ((e = tile_resid(R, sg))) return e;
    if ((e = split_r_transpose(c))) return e;
    return fin_f(R, record, lam, resid_tiles(c));
}

int run_setup(Run &R, int op, int nprob, const tlrmdd_plan *plans, const void *const *D, const void *const *U,
              void *const *theta, const tlrmdd_opts *opts, double *const *fhist, void *workspace, size_t ws_bytes,
              hipStream_t s) {
    int st = check_opts(opts);
    if (st != TLRMDD_OK) return st;
    const int64_t nr = plans[0]->H.nr, ns = plans[0]->H.ns;
    for (int p = 0; p < nprob; ++p) {
        if (!plans[p]) return fail(TLRMDD_INVALID_ARGUMENT, "plan is NULL");
        if (plans[p]->H.nr != nr || plans[p]->H.ns != ns)
            return fail(TLRMDD_INVALID_ARGUMENT, "batched problems must share nr and ns");
        if (!D[p] || !U[p] || !theta[p] || !fhist[p]) return fail(TLRMDD_INVALID_ARGUMENT, "NULL data pointer");
    }
    if (!workspace) return fail(TLRMDD_INVALID_ARGUMENT, "workspace is NULL");
    R.opts = opts;
    R.lbfgs = opts->optimizer == TLRMDD_LBFGS;
    R.m = R.lbfgs ? opts->lbfgs_m : 0;
    R.m1 = R.lbfgs ? R.m + 1 : 1;

    Ctx &c = R.c;
    c.nprob = nprob;
    c.nr = nr;
    c.ns = ns;
    c.ldk = round_up(nr, GEMM_PAD);
    c.lds = round_up(ns, GEMM_PAD);
    c.s = s;
    std::vector<const HostLayout *> Hs;
    R.theta_pre.assign(1, 0.0);
    R.asm_pre.assign(1, 0.0);
    R.asm_dir_pre.assign(1, 0.0);
    R.grad_pre.assign(1, 0.0);
    for (int p = 0; p < nprob; ++p) {
        append_problem(R.T, plans[p]->H, p, (int64_t)p * 2 * c.ldk * c.ldk, c.ldk);
        Hs.push_back(&plans[p]->H);
        R.theta_pre.push_back(R.theta_pre.back() + (double)plans[p]->H.theta_size);
        R.asm_pre.push_back(R.asm_pre.back() + plans[p]->H.asm_cflops);
        R.asm_dir_pre.push_back(R.asm_dir_pre.back() + plans[p]->H.asm_dir_cflops);
        R.grad_pre.push_back(R.grad_pre.back() + plans[p]->H.grad_cflops);
    }
    build_segments(R.T, Hs, c.lds, c.ldk);
    c.pstride = partial_stride(R.T, c.ldk, c.lds);
    assign_parts(R.T, c.pstride);
    R.single = (nprob == 1);
    c.w = carve((char *)workspace, op, nprob, c.ldk, c.lds, R.T.theta_total, R.m1, c.pstride,
                R.single ? 0 : tables_bytes(R.T, nprob));
    if (c.w.bytes > ws_bytes) return fail(TLRMDD_WORKSPACE, "workspace too small");
    size_t tbytes = 0;
    float2 *dcopy = nullptr;
    R.segs = line_segments(op, nprob, plans, opts, c.lds, (char *)workspace + c.w.bytes, &tbytes, &dcopy);
    if (c.w.bytes + tbytes > ws_bytes) return fail(TLRMDD_WORKSPACE, "workspace too small");
    c.w.Dc = dcopy ? dcopy : c.w.Ds;
    R.asm_first = R.T.asm_first;
    R.asm_first.push_back((int)R.T.asm_items.size());
    R.grad_first = R.T.grad_first;
    R.grad_first.push_back((int)R.T.grad_items.size());
    R.n_adj = nprob;
    for (const LineSeg &sg : R.segs)
        if (sg.tile && sg.lt.lc.grad) R.n_adj = std::min(R.n_adj, sg.p0);
    Upload up;
    for (LineSeg &sg : R.segs) {
        if (!sg.tile) continue;
        std::vector<PackItem> pack;
        std::vector<int64_t> toff;
        std::vector<const HostLayout *> Hseg;
        for (int p = sg.p0; p < sg.p0 + sg.np; ++p) {
            toff.push_back(R.T.probs[p].theta);
            Hseg.push_back(Hs[p]);
        }
        line_tile_tables(Hseg, toff, sg.lt.lc, c.lds, pack);
        if ((int)pack.size() != sg.lt.npack)
            return fail(TLRMDD_UNSUPPORTED, "tile-form line search tables");
        up.add(sg.lt.pack, pack.data(), pack.size() * sizeof(PackItem));
        HIP_TRY(launch_fill_zero(sg.lt.PA, sg.lt.zero_bytes, s));   // rank padding reads as zero
        if (sg.lt.lc.grad) {
            std::vector<PackItem> gpack;
            std::vector<TGradItem> gitems;
            grad_tile_tables(Hseg, toff, sg.lt, gpack, gitems);
            if ((int)gpack.size() != sg.lt.ngpack || (int)gitems.size() > sg.lt.ngitems)
                return fail(TLRMDD_UNSUPPORTED, "tile-form gradient tables");
            sg.lt.ngitems = (int)gitems.size();
            up.add(sg.lt.gpack, gpack.data(), gpack.size() * sizeof(PackItem));
            up.add(sg.lt.gitems, gitems.data(), gitems.size() * sizeof(TGradItem));
            // B^H padding and the unused columns of S read as zero
            HIP_TRY(launch_fill_zero((char *)sg.lt.PA + sg.lt.gzero_off, sg.lt.gzero_bytes, s));
        }
    }
    if (R.single) c.D = plans[0]->D;
    else upload_tables(R.T, nprob, c.w, c.D, fhist, up);
    if ((st = up.commit(s))) return st;
    R.fhist0 = R.single ? fhist[0] : nullptr;
    R.xstride = 2 * c.ldk * c.ldk;   // per-problem X-space stride
    R.rstride = c.lds * c.ldk;
    c.bf16 = opts->precision == TLRMDD_BF16X3;
    c.p3m = opts->precision == TLRMDD_FP32_3M;
    c.xspace = R.xstride;
    R.X1 = c.w.XW;
    R.X2 = c.w.XW + c.ldk * c.ldk;
    R.x2w = c.ldk * c.ldk;               // split form: X2 planes start ldk rows after X1's
    R.stride2 = 2 * R.T.theta_total;     // floats between ring slots
    R.nt = c.D.n_tseg;
    R.nrs = c.D.n_rseg;
    R.gcur = c.w.g0;
    R.gprev = c.w.g1;
    R.z = c.w.z;
    R.u = c.w.u;
    R.cen = c.w.cen;

    // padding of the X space must read as zero (the assembly writes only the true nr x nr block)
    if (c.ldk != nr) HIP_TRY(launch_fill_zero(c.w.XW, (size_t)nprob * R.xstride * sizeof(float2), s));
    const double snr = (double)ns * (double)nr;
    for (int p = 0; p < nprob; ++p) {
        if ((st = stage(c, p, (const float2 *)D[p], true))) return st;
        if (c.w.Dc != c.w.Ds)   // BF16 mode with tile-form ranges: their complex64 D
            HIP_TRY(timed(TLRMDD_K_STAGE, s, bytes_work(16.0 * snr), [&] {
                return launch_stage_d((const float2 *)D[p], c.ns, c.nr, c.w.Dc + p * c.lds * c.ldk, c.ldk, nullptr,
                                      c.lds, s);
            }));
        HIP_TRY(timed(TLRMDD_K_STAGE, s, bytes_work(16.0 * snr), [&] {
            return launch_copy2d((const float2 *)U[p], nr, c.w.Us + p * R.rstride, c.ldk, ns, nr, s);
        }));
        HIP_TRY(hipMemcpyAsync(c.w.th + 2 * R.T.probs[p].theta, theta[p],
                               plans[p]->H.theta_size * sizeof(float2), hipMemcpyDeviceToDevice, s));
    }
    FinArgs f0 = fin_args(FIN_INIT, c.w.sc);
    return fin(c, f0, nullptr, 0, 1);
}

// `iters` iterations of L-BFGS (or steepest descent) with exact line search on
//   f(theta) + lam ||theta - cen||^2     (cen == NULL: the plain Frobenius term; lam == 0: f alone)
// from the current theta and tracked residual, with fresh pair memory. f-history entries go to
// index record_base + t (none when record_base < 0).
int run_iterate(Run &R, int iters, double lam, const float *cen, int record_base) {
    Ctx &c = R.c;
    hipStream_t s = c.s;
    const int m1 = R.m1, nt = R.nt;
    int st;
    if ((st = fin(c, fin_args(FIN_RESET, c.w.sc), nullptr, 0, 1))) return st;
    if (lam != 0.0) {
        HIP_TRY(launch_pen(c.D.tsegs, nt, c.w.th, cen, nullptr, c.w.partials, s));
        if ((st = fin(c, fin_args(FIN_THNORM, c.w.sc), c.D.tcount, 0, 1))) return st;
    }
    // tile-form gradient ranges: the theta half of Pcol for the current theta (the direction half is
    // theta too here, and unused)
    for (const LineSeg &sg : R.segs)
        if (sg.tile && sg.lt.lc.grad && iters > 0)
            if ((st = tile_stage1(R, sg, c.w.th))) return st;
    for (int t = 0; t < iters; ++t) {
        // gradient from the tracked residual (eqs. DXLR): W = D^H r and the tile blocks of W' for the
        // problems before the tile-form gradient ranges, the tile form for those
        // (the two parts write disjoint problems' gradients; with a side stream they run side by side)
        const bool overlap = R.side && R.n_adj > 0 && R.n_adj < c.nprob;
        hipStream_t gs = s;
        if (overlap) {
            HIP_TRY(hipEventRecord(R.fork, s));
            HIP_TRY(hipStreamWaitEvent(R.side, R.fork, 0));
            gs = R.side;
        }
        for (const LineSeg &sg : R.segs)
            if (sg.tile && sg.lt.lc.grad)
                if ((st = tile_gradient(R, sg, R.gcur, gs))) return st;
        if (R.n_adj > 0) {
            const Ctx ca = R.n_adj == c.nprob ? c : line_ctx(c, 0, R.n_adj);
            if ((st = gemm_adjoint(ca, c.w.r, R.X1, R.xstride))) return st;
            const int ng = (R.single || R.n_adj == c.nprob) ? c.D.n_grad : R.grad_first[R.n_adj];
            const double nr = (double)c.nr;
            const Work wk = gemm_work(F_4M, R.grad_pre[R.n_adj], 8.0 * (nr * nr * R.n_adj + 2.0 * R.theta_pre[R.n_adj]));
            HIP_TRY(timed(TLRMDD_K_GRAD, s, wk, [&] {
                return launch_grad(c.D.tiles, c.D.grad_items, ng, c.D.probs, R.X1, (const float2 *)c.w.th,
                                   (float2 *)R.gcur, s);
            }));
        }
        if (overlap) {
            HIP_TRY(hipEventRecord(R.join, R.side));
            HIP_TRY(hipStreamWaitEvent(s, R.join, 0));
        }
        if (lam != 0.0) HIP_TRY(launch_reg_grad(c.D.tsegs, nt, R.gcur, c.w.th, cen, (float)(2.0 * lam), s));
        // direction: steepest descent first, then L-BFGS in vector-free form (Gram pass, two-loop
        // recursion on the (2 m + 1)-term coefficient vectors on the device, one combination pass)
        if (!R.lbfgs || t == 0) {
            HIP_TRY(launch_negate(c.D.tsegs, nt, c.w.p, R.gcur, s));
        } else {
            // held pairs besides the newest (a run without restarts): min(t - 1, m) in the Gram pass,
            // min(t, m) in the combination
            const double th_all = R.theta_pre.back();
            const double held = std::min(t - 1, R.m);
            HIP_TRY(timed(TLRMDD_K_GRAM, s, bytes_work(8.0 * th_all * (4.0 + 2.0 * held)), [&] {
                return launch_gram(c.D.tsegs, nt, m1, R.gcur, R.gprev, c.w.Y, c.w.S, R.stride2, c.w.sc, c.w.partials,
                                   s);
            }));
            FinArgs f = fin_args(FIN_GRAM, c.w.sc);
            f.m1 = m1;
            f.gram = c.w.gram;
            f.gstride = gram_stride(m1);
            if ((st = fin(c, f, c.D.tcount, 0, 6 * m1))) return st;
            HIP_TRY(timed(TLRMDD_K_COMBINE, s, bytes_work(8.0 * th_all * (2.0 + 2.0 * std::min(t, R.m))), [&] {
                return launch_combine(c.D.tsegs, nt, m1, c.w.p, R.gcur, c.w.S, c.w.Y, R.stride2, c.w.sc,
                                      c.w.gram + (2 * m1 + 1) * (2 * m1 + 1), gram_stride(m1), s);
            }));
        }
        // exact line search: a = D C1(theta;p), b = D C2(p)
        for (const LineSeg &sg : R.segs) {
            if (sg.tile) continue;
            if ((st = clear_plane_padding(R))) return st;
            const int a0 = R.single ? 0 : R.asm_first[sg.p0];
            const int na = R.single ? c.D.n_asm : R.asm_first[sg.p0 + sg.np] - a0;
            const double nr = (double)c.nr;
            const Work wk = gemm_work(F_4M, R.asm_dir_pre[sg.p0 + sg.np] - R.asm_dir_pre[sg.p0],
                                      16.0 * (nr * nr * sg.np + R.theta_pre[sg.p0 + sg.np] - R.theta_pre[sg.p0]));
            HIP_TRY(timed(TLRMDD_K_ASSEMBLE_DIR, s, wk, [&] {
                return launch_assemble(true, c.D.tiles, c.D.asm_items + a0, na, c.D.probs,
                                       (const float2 *)c.w.th, (const float2 *)c.w.p, R.X1, R.X2, s, c.bf16, R.x2w,
                                       c.lo_words());
            }));
        }
        if (lam != 0.0) {
            HIP_TRY(launch_pen(c.D.tsegs, nt, c.w.th, cen, c.w.p, c.w.partials, s));
            if ((st = fin(c, fin_args(FIN_LAMTERMS, c.w.sc), c.D.tcount, 0, 2))) return st;
        }
        // With a side stream and several tile ranges, the tile ranges alternate between it and s once
        // the dense ranges' product is enqueued, so that the small launches of two tile classes fill
        // each other's last rounds of workgroups; the side stream is joined before the line sums.
        int ntile = 0;
        for (const LineSeg &sg : R.segs) ntile += sg.tile ? 1 : 0;
        const bool tile_overlap = R.side && ntile > 1;
        bool forked = false;
        int itile = 0;
        for (const LineSeg &sg : R.segs) {
            // ranges with the tile-form gradient carry P_th from step to step (formed afresh with every
            // residual recompute, so its rounding accumulates over no more iterations than the tracked
            // residual's): stage 1 forms the direction half only where the halves fill whole tiles
            const bool dir_only = sg.tile && sg.lt.lc.grad && (sg.lt.lc.nt * sg.lt.lc.kpad) % GEMM_BN == 0;
            if (sg.tile && tile_overlap && !forked) {
                HIP_TRY(hipEventRecord(R.fork, s));
                HIP_TRY(hipStreamWaitEvent(R.side, R.fork, 0));
                forked = true;
            }
            if (sg.tile) st = line_products_tile(R, sg, dir_only, (tile_overlap && (itile++ & 1) == 0) ? R.side : s);
            else if (sg.np == c.nprob) st = gemm_line(c, R.X1, R.X2, R.xstride);
            else st = gemm_line(line_ctx(c, sg.p0, sg.np), R.X1 + sg.p0 * R.xstride, R.X2 + sg.p0 * R.xstride,
                                R.xstride);
            if (st) return st;
        }
        if (forked) {
            HIP_TRY(hipEventRecord(R.join, R.side));
            HIP_TRY(hipStreamWaitEvent(s, R.join, 0));
        }
        {
            FinArgs f = fin_args(FIN_LINE, c.w.sc);
            f.lam = lam;
            if ((st = fin(c, f, nullptr, line_tiles(c), 5))) return st;
        }
        // updates
        HIP_TRY(timed(TLRMDD_K_THETA_UPDATE, s,
                      bytes_work(8.0 * R.theta_pre.back() * ((R.lbfgs ? 4.0 : 3.0) + (cen ? 1.0 : 0.0))), [&] {
                          return launch_theta_update(c.D.tsegs, nt, c.w.th, c.w.p, R.lbfgs ? c.w.S : nullptr,
                                                     R.stride2, cen, c.w.sc, c.w.partials, s);
                      }));
        for (const LineSeg &sg : R.segs)
            if (sg.tile && sg.lt.lc.grad)
                if ((st = tile_pcol_update(R, sg))) return st;
        if (lam != 0.0)
            if ((st = fin(c, fin_args(FIN_THNORM, c.w.sc), c.D.tcount, 0, 1))) return st;
        // residual: recomputed from theta every resid_refresh iterations, else updated in place
        const bool refresh = R.opts->resid_refresh > 0 && (t + 1) % R.opts->resid_refresh == 0;
        if (refresh) {
            if ((st = objective_fresh(R, record_base >= 0 ? record_base + t + 1 : -1, lam))) return st;
        } else {
            HIP_TRY(timed(TLRMDD_K_RESID_UPDATE, s, bytes_work(32.0 * (double)c.ns * (double)c.nr * c.nprob), [&] {
                return launch_resid_update(c.D.rsegs, R.nrs, (float *)c.w.r, (const float *)c.w.a,
                                           (const float *)c.w.b, c.w.sc, c.w.partials, s);
            }));
            if ((st = split_r_transpose(c))) return st;
            if ((st = fin_f(R, record_base >= 0 ? record_base + t + 1 : -1, lam, R.T.rseg_per_prob))) return st;
        }
        std::swap(R.gcur, R.gprev);
    }
    return TLRMDD_OK;
}

int run_finish(Run &R, const tlrmdd_plan *plans, void *const *theta) {
    for (int p = 0; p < R.c.nprob; ++p)
        HIP_TRY(hipMemcpyAsync(theta[p], R.c.w.th + 2 * R.T.probs[p].theta, plans[p]->H.theta_size * sizeof(float2),
                               hipMemcpyDeviceToDevice, R.c.s));
    return TLRMDD_OK;
}

int solve_impl(int nprob, const tlrmdd_plan *plans, const void *const *D, const void *const *U,
               void *const *theta, const tlrmdd_opts *opts, double *const *fhist, void *workspace,
               size_t ws_bytes, hipStream_t s, const SideStream *side = nullptr) {
    Run R;
    int st = run_setup(R, 2, nprob, plans, D, U, theta, opts, fhist, workspace, ws_bytes, s);
    if (st) return st;
    if (side) {
        R.side = side->s;
        R.fork = side->fork;
        R.join = side->join;
    }
    const double lam = opts->lambda;
    if (lam != 0.0) {
        HIP_TRY(launch_pen(R.c.D.tsegs, R.nt, R.c.w.th, nullptr, nullptr, R.c.w.partials, s));
        if ((st = fin(R.c, fin_args(FIN_THNORM, R.c.w.sc), R.c.D.tcount, 0, 1))) return st;
    }
    if ((st = objective_fresh(R, 0, lam))) return st;
    if ((st = run_iterate(R, opts->iters, lam, nullptr, 0))) return st;
    return run_finish(R, plans, theta);
}

int check_admm(const tlrmdd_admm_opts *a) {
    if (!a) return fail(TLRMDD_INVALID_ARGUMENT, "admm opts is NULL");
    if (a->nstages < 1 || !a->lambdas) return fail(TLRMDD_INVALID_ARGUMENT, "need at least one lambda");
    if (a->outer < 0) return fail(TLRMDD_INVALID_ARGUMENT, "outer must be >= 0");
    if (!(a->rho > 0.0) || !std::isfinite(a->rho)) return fail(TLRMDD_INVALID_ARGUMENT, "rho must be > 0");
    for (int k = 0; k < a->nstages; ++k)
        if (!(a->lambdas[k] >= 0.0) || !std::isfinite(a->lambdas[k]))
            return fail(TLRMDD_INVALID_ARGUMENT, "lambdas must be finite and >= 0");
    return check_opts(&a->inner);
}

// Scaled ADMM with lambda continuation: per stage and outer step, inner.iters L-BFGS iterations of
// the X-update on f + rho/2 ||theta - (z - u)||^2, then the Z-update and the dual update on the
// device. f-history: data misfit at the start and after every X-update.
int admm_impl(int nprob, const tlrmdd_plan *plans, const void *const *D, const void *const *U,
              void *const *theta, const tlrmdd_admm_opts *aopts, double *const *fhist, void *workspace,
              size_t ws_bytes, hipStream_t s, const SideStream *side = nullptr) {
    int st = check_admm(aopts);
    if (st) return st;
    Run R;
    if ((st = run_setup(R, 3, nprob, plans, D, U, theta, &aopts->inner, fhist, workspace, ws_bytes, s))) return st;
    if (side) {
        R.side = side->s;
        R.fork = side->fork;
        R.join = side->join;
    }
    Ctx &c = R.c;
    if ((st = objective_fresh(R, -1, 0.0))) return st;
    auto record = [&](int k) -> int {
        FinArgs f = fin_args(FIN_RECORD, c.w.sc);
        f.fhist = R.single ? nullptr : c.D.fhist;
        f.fhist0 = R.fhist0;
        f.t = k;
        return fin(c, f, nullptr, 0, 1);
    };
    if ((st = record(0))) return st;
    HIP_TRY(launch_admm_update(c.D.tsegs, R.nt, 1, c.w.th, R.z, R.u, R.cen, 1.0f, s));
    const double rho = aopts->rho;
    int k = 0;
    for (int stg = 0; stg < aopts->nstages; ++stg) {
        const float scale = (float)(1.0 / (1.0 + 2.0 * aopts->lambdas[stg] / rho));
        for (int o = 0; o < aopts->outer; ++o) {
            if ((st = run_iterate(R, aopts->inner.iters, 0.5 * rho, R.cen, -1))) return st;
            if ((st = record(++k))) return st;
            HIP_TRY(launch_admm_update(c.D.tsegs, R.nt, 0, c.w.th, R.z, R.u, R.cen, scale, s));
        }
    }
    return run_finish(R, plans, theta);
}

}  // namespace

extern "C" {

int tlrmdd_forward(tlrmdd_plan plan, const void *D, const void *U, const void *theta, double *f_dev, void *r_out,
                   void *X_out, int precision, void *workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!plan || !D || !U || !theta || !f_dev || !workspace)
        return fail(TLRMDD_INVALID_ARGUMENT, "NULL argument");
    int st = check_precision(precision);
    if (st) return st;
    Ctx c;
    c.nprob = 1;
    c.nr = plan->H.nr;
    c.ns = plan->H.ns;
    c.ldk = plan->ldk;
    c.lds = plan->lds;
    c.s = stream;
    c.pstride = partial_stride(plan->T, c.ldk, c.lds);
    c.w = carve((char *)workspace, 0, 1, c.ldk, c.lds, theta_span(plan->H.theta_size), 1, c.pstride, 0);
    if (c.w.bytes > ws_bytes) return fail(TLRMDD_WORKSPACE, "workspace too small");
    c.D = plan->D;
    c.bf16 = precision == TLRMDD_BF16X3;
    c.p3m = precision == TLRMDD_FP32_3M;
    c.xspace = c.ldk * c.ldk;
    if (c.ldk != c.nr) HIP_TRY(launch_fill_zero(c.w.XW, (size_t)c.ldk * c.ldk * sizeof(float2), stream));
    if ((st = stage(c, 0, (const float2 *)D, false))) return st;
    const double nr2 = (double)c.nr * (double)c.nr, thn = (double)plan->H.theta_size;
    HIP_TRY(timed(TLRMDD_K_ASSEMBLE, stream, gemm_work(F_4M, plan->H.asm_cflops, 8.0 * (nr2 + thn)), [&] { return launch_assemble(false, c.D.tiles, c.D.asm_items, c.D.n_asm, c.D.probs, (const float2 *)theta, nullptr,
                            c.w.XW, nullptr, stream, c.bf16, 0, c.lo_words()); }));
    if ((st = gemm_resid(c, c.w.XW, 0, (const float2 *)U, c.nr, 0, c.w.r))) return st;
    FinArgs f = fin_args(FIN_F_OUT, c.w.sc);
    f.fout = f_dev;
    if ((st = fin(c, f, nullptr, resid_tiles(c), 1))) return st;
    if (r_out) HIP_TRY(launch_copy2d(c.w.r, c.ldk, (float2 *)r_out, c.nr, c.ns, c.nr, stream));
    if (X_out) {
        if (c.bf16)   // the X space holds split planes: re-assemble X in complex64 for the caller
            HIP_TRY(launch_assemble(false, c.D.tiles, c.D.asm_items, c.D.n_asm, c.D.probs, (const float2 *)theta,
                                    nullptr, c.w.XW, nullptr, stream));
        HIP_TRY(launch_copy2d(c.w.XW, c.ldk, (float2 *)X_out, c.nr, c.nr, c.nr, stream));
    }
    return TLRMDD_OK;
}

int tlrmdd_grad(tlrmdd_plan plan, const void *D, const void *U, const void *theta, double *f_dev, void *grad_out,
                int precision, void *workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!plan || !D || !U || !theta || !grad_out || !workspace)
        return fail(TLRMDD_INVALID_ARGUMENT, "NULL argument");
    int st = check_precision(precision);
    if (st) return st;
    Ctx c;
    c.nprob = 1;
    c.nr = plan->H.nr;
    c.ns = plan->H.ns;
    c.ldk = plan->ldk;
    c.lds = plan->lds;
    c.s = stream;
    c.pstride = partial_stride(plan->T, c.ldk, c.lds);
    c.w = carve((char *)workspace, 1, 1, c.ldk, c.lds, theta_span(plan->H.theta_size), 1, c.pstride, 0);
    if (c.w.bytes > ws_bytes) return fail(TLRMDD_WORKSPACE, "workspace too small");
    c.D = plan->D;
    c.bf16 = precision == TLRMDD_BF16X3;
    c.p3m = precision == TLRMDD_FP32_3M;
    c.xspace = c.ldk * c.ldk;
    if (c.ldk != c.nr) HIP_TRY(launch_fill_zero(c.w.XW, (size_t)c.ldk * c.ldk * sizeof(float2), stream));
    if ((st = stage(c, 0, (const float2 *)D, true))) return st;
    const double nr2 = (double)c.nr * (double)c.nr, thn = (double)plan->H.theta_size;
    HIP_TRY(timed(TLRMDD_K_ASSEMBLE, stream, gemm_work(F_4M, plan->H.asm_cflops, 8.0 * (nr2 + thn)), [&] { return launch_assemble(false, c.D.tiles, c.D.asm_items, c.D.n_asm, c.D.probs, (const float2 *)theta, nullptr,
                            c.w.XW, nullptr, stream, c.bf16, 0, c.lo_words()); }));
    if ((st = gemm_resid(c, c.w.XW, 0, (const float2 *)U, c.nr, 0, c.w.r))) return st;
    if ((st = split_r_transpose(c))) return st;
    if (f_dev) {
        FinArgs f = fin_args(FIN_F_OUT, c.w.sc);
        f.fout = f_dev;
        if ((st = fin(c, f, nullptr, resid_tiles(c), 1))) return st;
    }
    // the assembled X is dead once r exists: W = D^H r reuses its storage
    if ((st = gemm_adjoint(c, c.w.r, c.w.XW, 0))) return st;
    HIP_TRY(timed(TLRMDD_K_GRAD, stream, gemm_work(F_4M, plan->H.grad_cflops, 8.0 * (nr2 + 2.0 * thn)), [&] { return launch_grad(c.D.tiles, c.D.grad_items, c.D.n_grad, c.D.probs, c.w.XW, (const float2 *)theta,
                        (float2 *)grad_out, stream); }));
    return TLRMDD_OK;
}

int tlrmdd_adjoint(tlrmdd_plan plan, const void *D, const void *U, void *X_out, int precision, void *workspace,
                   size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!plan || !D || !U || !X_out || !workspace) return fail(TLRMDD_INVALID_ARGUMENT, "NULL argument");
    int st = check_precision(precision);
    if (st) return st;
    Ctx c;
    c.nprob = 1;
    c.nr = plan->H.nr;
    c.ns = plan->H.ns;
    c.ldk = plan->ldk;
    c.lds = plan->lds;
    c.s = stream;
    c.pstride = partial_stride(plan->T, c.ldk, c.lds);
    c.w = carve((char *)workspace, 1, 1, c.ldk, c.lds, theta_span(plan->H.theta_size), 1, c.pstride, 0);
    if (c.w.bytes > ws_bytes) return fail(TLRMDD_WORKSPACE, "workspace too small");
    c.D = plan->D;
    c.bf16 = precision == TLRMDD_BF16X3;
    c.p3m = precision == TLRMDD_FP32_3M;
    c.xspace = c.ldk * c.ldk;
    if ((st = stage(c, 0, (const float2 *)D, true))) return st;
    // U takes the place of the residual: padded copy with zero padding, then W = D^H U
    HIP_TRY(launch_stage_d((const float2 *)U, c.ns, c.nr, c.w.r, c.ldk, nullptr, c.lds, stream));
    if ((st = split_r_transpose(c))) return st;
    if ((st = gemm_adjoint(c, c.w.r, c.w.XW, 0))) return st;
    HIP_TRY(launch_copy2d(c.w.XW, c.ldk, (float2 *)X_out, c.nr, c.nr, c.nr, stream));
    return TLRMDD_OK;
}

int tlrmdd_solve(tlrmdd_plan plan, const void *D, const void *U, void *theta_inout, const tlrmdd_opts *opts,
                 double *f_hist_dev, void *workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!plan) return fail(TLRMDD_INVALID_ARGUMENT, "plan is NULL");
    const void *Dp[1] = {D};
    const void *Up[1] = {U};
    void *Tp[1] = {theta_inout};
    double *Fp[1] = {f_hist_dev};
    return solve_impl(1, &plan, Dp, Up, Tp, opts, Fp, workspace, ws_bytes, stream);
}

}  // extern "C"

namespace {
int ws_bytes_group(int op, int count, const tlrmdd_plan *plans, const tlrmdd_opts *opts, size_t *bytes) {
    if (count <= 0 || !plans || !bytes) return fail(TLRMDD_INVALID_ARGUMENT, "bad arguments");
    int st = check_opts(opts);
    if (st) return st;
    for (int p = 0; p < count; ++p)
        if (!plans[p]) return fail(TLRMDD_INVALID_ARGUMENT, "plan is NULL");
    const int64_t nr = plans[0]->H.nr, ns = plans[0]->H.ns;
    const int64_t ldk = round_up(nr, GEMM_PAD), lds = round_up(ns, GEMM_PAD);
    Tables T;
    std::vector<const HostLayout *> Hs;
    for (int p = 0; p < count; ++p) {
        if (plans[p]->H.nr != nr || plans[p]->H.ns != ns)
            return fail(TLRMDD_INVALID_ARGUMENT, "batched problems must share nr and ns");
        append_problem(T, plans[p]->H, p, (int64_t)p * 2 * ldk * ldk, ldk);
        Hs.push_back(&plans[p]->H);
    }
    build_segments(T, Hs, lds, ldk);
    const int m1 = opts->optimizer == TLRMDD_LBFGS ? opts->lbfgs_m + 1 : 1;
    *bytes = carve(nullptr, op, count, ldk, lds, T.theta_total, m1, partial_stride(T, ldk, lds),
                   count == 1 ? 0 : tables_bytes(T, count)).bytes;
    size_t tb = 0;
    line_segments(op, count, plans, opts, lds, nullptr, &tb);
    *bytes += tb;
    return TLRMDD_OK;
}

int ws_bytes_grouped(int op, int count, const tlrmdd_plan *plans, const tlrmdd_opts *opts, size_t *bytes,
                     std::vector<size_t> *parts) {
    if (count <= 0 || !plans || !bytes) return fail(TLRMDD_INVALID_ARGUMENT, "bad arguments");
    int st = check_opts(opts);
    if (st) return st;
    for (int p = 0; p < count; ++p)
        if (!plans[p]) return fail(TLRMDD_INVALID_ARGUMENT, "plan is NULL");
    int S = 1;
    size_t total = 0;
    for (const std::vector<int> &m : make_groups(count, plans, opts, &S)) {
        const std::vector<tlrmdd_plan> gp = pick(plans, m);
        size_t b = 0;
        if ((st = ws_bytes_group(op, (int)gp.size(), gp.data(), opts, &b))) return st;
        if (parts) parts->push_back(b);
        total += align256(b);
    }
    *bytes = total;
    return TLRMDD_OK;
}

}  // namespace

extern "C" {

int tlrmdd_line_form(tlrmdd_plan plan, const tlrmdd_opts *opts, int *tile_form, int *kpad) {
    g_last_error.clear();
    if (!plan || !tile_form) return fail(TLRMDD_INVALID_ARGUMENT, "plan / tile_form is NULL");
    int st = check_opts(opts);
    if (st) return st;
    LineClass lc;
    const bool on = problem_form(2, plan->H, opts, lc);
    *tile_form = on ? (lc.grad ? 2 : 1) : 0;
    if (kpad) *kpad = on ? lc.kpad : 0;
    return TLRMDD_OK;
}

int tlrmdd_workspace_bytes_batched(int count, const tlrmdd_plan *plans, const tlrmdd_opts *opts, size_t *bytes) {
    g_last_error.clear();
    return ws_bytes_grouped(2, count, plans, opts, bytes);
}

int tlrmdd_workspace_bytes_admm(int count, const tlrmdd_plan *plans, const tlrmdd_admm_opts *opts, size_t *bytes) {
    g_last_error.clear();
    int st = check_admm(opts);
    if (st) return st;
    return ws_bytes_grouped(3, count, plans, &opts->inner, bytes);
}

int tlrmdd_admm(tlrmdd_plan plan, const void *D, const void *U, void *theta_inout, const tlrmdd_admm_opts *opts,
                double *f_hist_dev, void *workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!plan) return fail(TLRMDD_INVALID_ARGUMENT, "plan is NULL");
    const void *Dp[1] = {D};
    const void *Up[1] = {U};
    void *Tp[1] = {theta_inout};
    double *Fp[1] = {f_hist_dev};
    return admm_impl(1, &plan, Dp, Up, Tp, opts, Fp, workspace, ws_bytes, stream);
}

int tlrmdd_admm_batched(int count, const tlrmdd_plan *plans, const void *const *D, const void *const *U,
                        void *const *theta_inout, const tlrmdd_admm_opts *opts, double *const *f_hist_dev,
                        void *workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (count <= 0 || !plans || !D || !U || !theta_inout || !f_hist_dev)
        return fail(TLRMDD_INVALID_ARGUMENT, "bad arguments");
    int st = check_admm(opts);
    if (st) return st;
    if (!grouped_call(count, &opts->inner))
        return admm_impl(count, plans, D, U, theta_inout, opts, f_hist_dev, workspace, ws_bytes, stream);
    return run_grouped(3, count, plans, D, U, theta_inout, &opts->inner, f_hist_dev, workspace, ws_bytes, stream,
                       [&](int n, const tlrmdd_plan *p, const void *const *d, const void *const *u, void *const *t,
                           double *const *f, void *w, size_t b, hipStream_t s, const SideStream *side) {
                           return admm_impl(n, p, d, u, t, opts, f, w, b, s, side);
                       });
}

int tlrmdd_solve_batched(int count, const tlrmdd_plan *plans, const void *const *D, const void *const *U,
                         void *const *theta_inout, const tlrmdd_opts *opts, double *const *f_hist_dev,
                         void *workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (count <= 0 || !plans || !D || !U || !theta_inout || !f_hist_dev)
        return fail(TLRMDD_INVALID_ARGUMENT, "bad arguments");
    int st = check_opts(opts);
    if (st) return st;
    if (!grouped_call(count, opts))
        return solve_impl(count, plans, D, U, theta_inout, opts, f_hist_dev, workspace, ws_bytes, stream);
    return run_grouped(2, count, plans, D, U, theta_inout, opts, f_hist_dev, workspace, ws_bytes, stream,
                       [&](int n, const tlrmdd_plan *p, const void *const *d, const void *const *u, void *const *t,
                           double *const *f, void *w, size_t b, hipStream_t s, const SideStream *side) {
                           return solve_impl(n, p, d, u, t, opts, f, w, b, s, side);
                       });
}

int tlrmdd_timing_begin_kinds(uint32_t kinds) {
    g_last_error.clear();
    if (kinds == 0 || (kinds >> TLRMDD_K_NKINDS) != 0)
        return fail(TLRMDD_INVALID_ARGUMENT, "kinds: a non-empty set of bits below 1 << TLRMDD_K_NKINDS");
    std::lock_guard<std::mutex> lk(g_rec.mu);
    for (TimedLaunch &t : g_rec.ev) {
        g_rec.pool.push_back(t.a);
        g_rec.pool.push_back(t.b);
    }
    g_rec.ev.clear();
    g_rec.kinds.store(kinds, std::memory_order_relaxed);
    return TLRMDD_OK;
}

int tlrmdd_timing_begin(void) { return tlrmdd_timing_begin_kinds((1u << TLRMDD_K_NKINDS) - 1u); }

int tlrmdd_timing_end(tlrmdd_kernel_stats *stats) {
    g_last_error.clear();
    std::lock_guard<std::mutex> lk(g_rec.mu);
    g_rec.kinds.store(0, std::memory_order_relaxed);
    tlrmdd_kernel_stats acc[TLRMDD_K_NKINDS];
    for (int k = 0; k < TLRMDD_K_NKINDS; ++k) {
        std::memset(&acc[k], 0, sizeof(acc[k]));
        acc[k].flop_dtype = TLRMDD_DT_NONE;
    }
    int status = TLRMDD_OK;
    for (TimedLaunch &t : g_rec.ev) {
        float v = 0.f;
        hipError_t e = hipEventSynchronize(t.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&v, t.a, t.b);
        if (e != hipSuccess) {
            status = fail(TLRMDD_HIP_ERROR, std::string("timing events: ") + hipGetErrorString(e));
            continue;
        }
        if (t.kind >= 0 && t.kind < TLRMDD_K_NKINDS) {
            tlrmdd_kernel_stats &a = acc[t.kind];
            a.ms += v;
            a.launches += 1;
            a.cflops += t.work.cflops;
            a.flops += t.work.flops;
            a.bytes += t.work.bytes;
            if (t.work.dtype != TLRMDD_DT_NONE) {
                if (a.flop_dtype == TLRMDD_DT_NONE) a.flop_dtype = t.work.dtype;
                else if (a.flop_dtype != t.work.dtype) a.flop_dtype = TLRMDD_DT_MIXED;
            }
        }
        g_rec.pool.push_back(t.a);
        g_rec.pool.push_back(t.b);
    }
    g_rec.ev.clear();
    if (stats)
        for (int k = 0; k < TLRMDD_K_NKINDS; ++k) stats[k] = acc[k];
    return status;
}

// ---- HIP graphs of library calls ----
struct tlrmdd_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<char *> pinned;   // host images read by the graph's copy nodes
};

static void graph_free(tlrmdd_graph g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    for (char *h : g->pinned) (void)hipHostFree(h);
    delete g;
}

int tlrmdd_graph_begin(hipStream_t stream) {
    g_last_error.clear();
    if (!stream) return fail(TLRMDD_INVALID_ARGUMENT, "graph capture needs a created stream (not the null stream)");
    if (g_cap.on) return fail(TLRMDD_INVALID_ARGUMENT, "a graph capture is already open on this thread");
    HIP_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed));
    g_cap.on = true;
    g_cap.stream = stream;
    g_cap.pinned.clear();
    return TLRMDD_OK;
}

int tlrmdd_graph_end(hipStream_t stream, tlrmdd_graph *graph_out) {
    g_last_error.clear();
    if (graph_out) *graph_out = nullptr;
    if (!g_cap.on || g_cap.stream != stream)
        return fail(TLRMDD_INVALID_ARGUMENT, "no graph capture open on this stream in this thread");
    // the capture is closed in every case below
    g_cap.on = false;
    tlrmdd_graph g = new tlrmdd_graph_s;
    g->pinned.swap(g_cap.pinned);
    hipError_t e = hipStreamEndCapture(stream, &g->graph);
    if (!graph_out) {
        graph_free(g);
        return fail(TLRMDD_INVALID_ARGUMENT, "graph_out is NULL (the capture is closed, its graph dropped)");
    }
    if (e == hipSuccess && !g->graph) e = hipErrorStreamCaptureInvalidated;
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        graph_free(g);
        return fail(TLRMDD_HIP_ERROR, std::string("graph capture: ") + hipGetErrorString(e));
    }
    *graph_out = g;
    return TLRMDD_OK;
}

int tlrmdd_graph_launch(tlrmdd_graph graph, hipStream_t stream) {
    g_last_error.clear();
    if (!graph) return fail(TLRMDD_INVALID_ARGUMENT, "graph is NULL");
    HIP_TRY(hipGraphLaunch(graph->exec, stream));
    return TLRMDD_OK;
}

int tlrmdd_graph_destroy(tlrmdd_graph graph) {
    g_last_error.clear();
    if (graph) graph_free(graph);
    return TLRMDD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// per-tile SVD: rank / tile-size estimate and warm start
// ---------------------------------------------------------------------------
namespace {

struct SvdHost {
    std::vector<SvdTile> tiles;
    std::vector<int32_t> pair_tile;
    int64_t nW = 0, nV = 0, nS = 0;
    int maxnp = 2;
};

// jacobi == false: the tile is only gathered (no rotations, no V), e.g. a dense diagonal tile of a warm start
void svd_add_tile(SvdHost &S, int m, int n, int64_t row0, int64_t col0, bool with_v, bool jacobi = true) {
    SvdTile t;
    t.trans = m < n ? 1 : 0;   // decompose the transpose of a wide tile: A is never wider than tall
    t.pad = 0;
    if (t.trans) std::swap(m, n);
    t.m = m;
    t.n = n;
    t.row0 = row0;
    t.col0 = col0;
    t.offW = S.nW;
    t.offV = with_v ? S.nV : -1;
    t.offS = S.nS;
    t.npad = n + (n & 1);
    t.pair0 = (int32_t)S.pair_tile.size();
    S.nW += (int64_t)m * n;
    if (with_v) S.nV += (int64_t)n * n;
    S.nS += n;
    if (jacobi) {
        S.maxnp = std::max(S.maxnp, t.npad);
        for (int k = 0; k < t.npad / 2; ++k) S.pair_tile.push_back((int32_t)S.tiles.size());
    }
    S.tiles.push_back(t);
}

std::vector<int> split_sizes(int64_t nr, int d) {
    std::vector<int> sz((size_t)(nr / d), d);
    if (nr % d) sz.push_back((int)(nr % d));
    return sz;
}

// tiles (i, j), i >= j, in the order i(i+1)/2 + j
SvdHost svd_grid(int64_t nr, int d, bool with_v) {
    SvdHost S;
    const std::vector<int> sz = split_sizes(nr, d);
    std::vector<int64_t> st(sz.size() + 1, 0);
    for (size_t i = 0; i < sz.size(); ++i) st[i + 1] = st[i] + sz[i];
    for (size_t i = 0; i < sz.size(); ++i)
        for (size_t j = 0; j <= i; ++j) svd_add_tile(S, sz[i], sz[j], st[i], st[j], with_v);
    return S;
}

struct SvdWs {
    double2 *W = nullptr, *V = nullptr;
    double *sig = nullptr, *v0 = nullptr;
    int32_t *order = nullptr, *kout = nullptr, *flags = nullptr, *pair_tile = nullptr;
    SvdTile *tiles = nullptr;
    WarmItem *items = nullptr;
    size_t bytes = 0;
};

SvdWs svd_carve(char *base, const SvdHost &S, int nitems) {
    SvdWs w;
    size_t o = 0;
    auto take = [&](size_t b) -> char * {
        char *p = base ? base + o : nullptr;
        o += align256(b);
        return p;
    };
    w.W = (double2 *)take((size_t)S.nW * sizeof(double2));
    if (S.nV) w.V = (double2 *)take((size_t)S.nV * sizeof(double2));
    w.sig = (double *)take((size_t)S.nS * sizeof(double));
    w.order = (int32_t *)take((size_t)S.nS * sizeof(int32_t));
    w.kout = (int32_t *)take(S.tiles.size() * sizeof(int32_t));
    w.v0 = (double *)take(sizeof(double));
    w.flags = (int32_t *)take(2 * sizeof(int32_t));
    w.tiles = (SvdTile *)take(S.tiles.size() * sizeof(SvdTile));
    w.pair_tile = (int32_t *)take(S.pair_tile.size() * sizeof(int32_t));
    w.items = (WarmItem *)take((size_t)std::max(nitems, 1) * sizeof(WarmItem));
    w.bytes = o;
    return w;
}

// Jacobi sweeps on the gathered tiles, then sigma per column. Tables must already be on the device.
// Sweeps are enqueued two at a time; the host reads the convergence flag in between and stops
// enqueueing once no pair was rotated (synchronises the stream).
int svd_run(const SvdHost &S, const SvdWs &w, const float2 *X, int64_t ldx, hipStream_t s) {
    const int nt = (int)S.tiles.size();
    const int npairs = (int)S.pair_tile.size();
    HIP_TRY(launch_svd_gather(w.tiles, nt, X, ldx, w.W, w.V, s));
    HIP_TRY(launch_fill_zero(w.flags, 2 * sizeof(int32_t), s));
    bool converged = npairs == 0;
    for (int sw = 0; sw < SVD_MAX_SWEEPS && !converged; ++sw) {
        for (int r = 0; r < S.maxnp - 1; ++r)
            HIP_TRY(launch_svd_round(w.tiles, w.pair_tile, npairs, r, w.W, w.V, w.flags, w.flags + 1, SVD_TOL, s));
        HIP_TRY(launch_svd_sweep_end(w.flags, w.flags + 1, s));
        if (sw % 2 == 1 || sw + 1 == SVD_MAX_SWEEPS) {
            int32_t done = 0;
            HIP_TRY(hipMemcpyAsync(&done, w.flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            converged = done != 0;
        }
    }
    if (!converged)
        return fail(TLRMDD_NOT_CONVERGED, "per-tile Jacobi SVD: pairs still rotated after the sweep limit");
    HIP_TRY(launch_svd_sigma(w.tiles, nt, w.W, w.sig, s));
    return TLRMDD_OK;
}

int svd_upload(const SvdHost &S, const SvdWs &w, const std::vector<WarmItem> *items, hipStream_t s) {
    Upload up;
    up.add(w.tiles, S.tiles.data(), S.tiles.size() * sizeof(SvdTile));
    up.add(w.pair_tile, S.pair_tile.data(), S.pair_tile.size() * sizeof(int32_t));
    if (items) up.add(w.items, items->data(), items->size() * sizeof(WarmItem));
    return up.commit(s);
}

int check_rank_args(const void *X, int64_t nr, int32_t d, double eps) {
    if (!X) return fail(TLRMDD_INVALID_ARGUMENT, "X is NULL");
    if (nr <= 0 || nr > ((int64_t)1 << 20)) return fail(TLRMDD_INVALID_ARGUMENT, "nr out of range");
    if (d < 1 || d > SVD_MAX_N) return fail(TLRMDD_INVALID_ARGUMENT, "tile size must be in [1, 1024]");
    if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(TLRMDD_INVALID_ARGUMENT, "eps must be finite and >= 0");
    return TLRMDD_OK;
}

// ranks of all tiles at size d into host vectors (t order / diagonal order); synchronises the stream
int tile_ranks_impl(const void *X, int64_t nr, int32_t d, double eps, std::vector<int32_t> &koff,
                    std::vector<int32_t> &kdiag, double *v0, void *workspace, size_t ws_bytes, hipStream_t s) {
    int st = check_rank_args(X, nr, d, eps);
    if (st) return st;
    if (!workspace) return fail(TLRMDD_INVALID_ARGUMENT, "workspace is NULL");
    const SvdHost S = svd_grid(nr, d, false);
    const SvdWs w = svd_carve((char *)workspace, S, 0);
    if (w.bytes > ws_bytes) return fail(TLRMDD_WORKSPACE, "workspace too small");
    if ((st = svd_upload(S, w, nullptr, s))) return st;
    if ((st = svd_run(S, w, (const float2 *)X, nr, s))) return st;
    HIP_TRY(launch_svd_rank(w.tiles, (int)S.tiles.size(), w.sig, S.nS, eps, w.kout, w.v0, s));
    std::vector<int32_t> k(S.tiles.size());
    double v = 0.0;
    HIP_TRY(hipMemcpyAsync(k.data(), w.kout, k.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&v, w.v0, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const int N = (int)split_sizes(nr, d).size();
    koff.clear();
    kdiag.assign(N, 0);
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < i; ++j) koff.push_back(k[(size_t)i * (i + 1) / 2 + j]);
        kdiag[i] = k[(size_t)i * (i + 1) / 2 + i];
    }
    if (v0) *v0 = v;
    return TLRMDD_OK;
}

}  // namespace

extern "C" {

int tlrmdd_workspace_bytes_ranks(int64_t nr, int32_t d, size_t *bytes) {
    g_last_error.clear();
    if (!bytes) return fail(TLRMDD_INVALID_ARGUMENT, "bytes is NULL");
    if (nr <= 0 || nr > ((int64_t)1 << 20) || d < 1 || d > SVD_MAX_N)
        return fail(TLRMDD_INVALID_ARGUMENT, "nr or tile size out of range");
    *bytes = svd_carve(nullptr, svd_grid(nr, d, false), 0).bytes;
    return TLRMDD_OK;
}

int tlrmdd_tile_ranks(const void *X, int64_t nr, int32_t d, double eps, int32_t *k_off_out, int32_t *k_diag_out,
                      double *v0_out, void *workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!k_off_out || !k_diag_out) return fail(TLRMDD_INVALID_ARGUMENT, "output arrays are NULL");
    std::vector<int32_t> ko, kd;
    int st = tile_ranks_impl(X, nr, d, eps, ko, kd, v0_out, workspace, ws_bytes, stream);
    if (st) return st;
    std::copy(ko.begin(), ko.end(), k_off_out);
    std::copy(kd.begin(), kd.end(), k_diag_out);
    return TLRMDD_OK;
}

int tlrmdd_choose_layout(const void *X, int64_t nr, const int32_t *candidates, int32_t ncand, double eps,
                         int32_t *d_out, int64_t *entries_out, int32_t *rank_off_out, int64_t off_capacity,
                         int32_t *rank_diag_out, int64_t diag_capacity, void *workspace, size_t ws_bytes,
                         hipStream_t stream) {
    g_last_error.clear();
    if (!candidates || ncand < 1 || !d_out || !rank_off_out || !rank_diag_out)
        return fail(TLRMDD_INVALID_ARGUMENT, "bad arguments");
    int64_t best = -1;
    for (int c = 0; c < ncand; ++c) {
        std::vector<int32_t> ko, kd;
        int st = tile_ranks_impl(X, nr, candidates[c], eps, ko, kd, nullptr, workspace, ws_bytes, stream);
        if (st) return st;
        const std::vector<int> sz = split_sizes(nr, candidates[c]);
        // layout of the estimate: ranks >= 1; dense diagonal when k_ii >= d_i / 2
        int64_t n = 0;
        size_t t = 0;
        for (size_t i = 0; i < sz.size(); ++i) {
            for (size_t j = 0; j < i; ++j, ++t) {
                ko[t] = std::max(1, ko[t]);
                n += (int64_t)ko[t] * (sz[i] + sz[j]);
            }
            kd[i] = (kd[i] >= (sz[i] + 1) / 2) ? -1 : std::max(1, kd[i]);
            n += (int64_t)sz[i] * (kd[i] < 0 ? sz[i] : kd[i]);
        }
        if (entries_out) entries_out[c] = n;
        if (best < 0 || n < best) {
            if ((int64_t)ko.size() > off_capacity || (int64_t)kd.size() > diag_capacity)
                return fail(TLRMDD_INVALID_ARGUMENT, "rank arrays too small for a candidate tile size");
            best = n;
            *d_out = candidates[c];
            std::copy(ko.begin(), ko.end(), rank_off_out);
            std::copy(kd.begin(), kd.end(), rank_diag_out);
        }
    }
    return TLRMDD_OK;
}

}  // extern "C"

namespace {
SvdHost warm_grid(const HostLayout &H, std::vector<WarmItem> &items) {
    SvdHost S;
    items.clear();
    for (const TileDesc &td : H.tiles) {
        WarmItem it{};
        it.tile = (int32_t)S.tiles.size();
        it.kind = td.kind == TILE_LR ? WARM_LR : (td.kind == TILE_QQ ? WARM_QQ : WARM_DENSE);
        it.k = td.k;
        it.offA = td.offA;
        it.offB = td.offB;
        items.push_back(it);
        // a dense diagonal tile is copied as is (gathered, never rotated)
        svd_add_tile(S, td.di, td.dj, td.row0, td.col0, td.kind != TILE_DENSE, td.kind != TILE_DENSE);
    }
    return S;
}
}  // namespace

extern "C" {

int tlrmdd_workspace_bytes_warm(tlrmdd_plan plan, size_t *bytes) {
    g_last_error.clear();
    if (!plan || !bytes) return fail(TLRMDD_INVALID_ARGUMENT, "plan / bytes is NULL");
    for (int d : plan->H.d)
        if (d > SVD_MAX_N) return fail(TLRMDD_INVALID_ARGUMENT, "tile sizes above 1024 are not supported");
    std::vector<WarmItem> items;
    const SvdHost S = warm_grid(plan->H, items);
    *bytes = svd_carve(nullptr, S, (int)items.size()).bytes;
    return TLRMDD_OK;
}

int tlrmdd_warm_start(tlrmdd_plan plan, const void *X, void *theta_out, void *workspace, size_t ws_bytes,
                      hipStream_t stream) {
    g_last_error.clear();
    if (!plan || !X || !theta_out || !workspace) return fail(TLRMDD_INVALID_ARGUMENT, "NULL argument");
    for (int d : plan->H.d)
        if (d > SVD_MAX_N) return fail(TLRMDD_INVALID_ARGUMENT, "tile sizes above 1024 are not supported");
    std::vector<WarmItem> items;
    const SvdHost S = warm_grid(plan->H, items);
    const SvdWs w = svd_carve((char *)workspace, S, (int)items.size());
    if (w.bytes > ws_bytes) return fail(TLRMDD_WORKSPACE, "workspace too small");
    int st = svd_upload(S, w, &items, stream);
    if (st) return st;
    if ((st = svd_run(S, w, (const float2 *)X, plan->H.nr, stream))) return st;
    HIP_TRY(launch_svd_order(w.tiles, (int)S.tiles.size(), w.sig, w.order, stream));
    HIP_TRY(launch_svd_factors(w.tiles, w.items, (int)items.size(), w.W, w.V, w.sig, w.order, (const float2 *)X,
                               plan->H.nr, (float2 *)theta_out, stream));
    return TLRMDD_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// tile low-rank product D C(theta) without the dense X
// ---------------------------------------------------------------------------
namespace {

struct TlrHost {
    int N = 0;
    int64_t Kpmax = 0, K1p = 0, K2p = 0, dp = 0;   // padded operand shapes (uniform per tile)
    std::vector<PackItem> packA, packB;
    std::vector<GatherItem> gather;
    std::vector<std::pair<int, int>> runs;          // [first, last] tiles of equal size
};

struct TlrWs {
    float2 *Ds, *A, *P, *B, *Pcol, *R;
    double *partials;
    SolveScalars *sc;
    PackItem *pa, *pb;
    GatherItem *gi;
    size_t bytes;
};

TlrHost tlr_plan(const HostLayout &H, int64_t lds) {
    TlrHost T;
    const int N = H.N;
    T.N = N;
    // rank of tile (i, j) as a product of two factors, and the TileDesc of its factors
    std::vector<int> tix(N * N, -1);   // index into H.tiles: diagonal tiles first, then t order
    for (int i = 0; i < N; ++i) tix[i * N + i] = i;
    {
        int t = 0;
        for (int i = 0; i < N; ++i)
            for (int j = 0; j < i; ++j, ++t) tix[i * N + j] = tix[j * N + i] = N + t;
    }
    auto kk = [&](int i, int j) -> int {
        const TileDesc &td = H.tiles[tix[i * N + j]];
        return (i == j && td.kind == TILE_DENSE) ? H.d[i] : td.k;
    };
    std::vector<int64_t> K1(N, 0);
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) K1[i] += kk(i, j);
    int64_t kmax = 0, dmax = 0;
    for (int i = 0; i < N; ++i) {
        kmax = std::max(kmax, K1[i]);
        dmax = std::max<int64_t>(dmax, H.d[i]);
    }
    T.Kpmax = round_up(dmax, GEMM_BK);
    T.K1p = round_up(kmax, GEMM_PAD);
    T.K2p = round_up(kmax, GEMM_BK);   // sum over i of k(i, j) equals K1[j] (ranks are symmetric)
    T.dp = round_up(dmax, GEMM_PAD);
    const int64_t sA = T.Kpmax * T.K1p, sP = lds * T.K1p, sB = T.K2p * T.dp, sPc = lds * T.K2p;
    std::vector<int64_t> roff(N, 0);   // running row offset inside B_j / column offset inside Pcol_j
    for (int i = 0; i < N; ++i) {
        int64_t coff = 0;
        for (int j = 0; j < N; ++j) {
            const TileDesc &td = H.tiles[tix[i * N + j]];
            const int k = kk(i, j), di = H.d[i], dj = H.d[j];
            PackItem a{}, b{};
            a.rows = di; a.cols = k; a.dst = i * sA + coff; a.ldd = T.K1p;
            b.rows = k; b.cols = dj; b.dst = j * sB + roff[j] * T.dp; b.ldd = T.dp;
            if (i == j && td.kind == TILE_DENSE) {
                a.op = PACK_IDENT;
                b.op = PACK_SYM; b.src = td.offA; b.lds = di;
            } else if (i == j) {   // Q Q^T
                a.op = PACK_COPY; a.src = td.offA; a.lds = k;
                b.op = PACK_TRANS; b.src = td.offA; b.lds = k;
            } else if (i > j) {    // tile (i, j): L (d_i x k) R (k x d_j)
                a.op = PACK_COPY; a.src = td.offA; a.lds = k;
                b.op = PACK_COPY; b.src = td.offB; b.lds = dj;
            } else {               // tile (j, i) holds L (d_j x k), R (k x d_i): X_ij = R^T L^T
                a.op = PACK_TRANS; a.src = td.offB; a.lds = di;
                b.op = PACK_TRANS; b.src = td.offA; b.lds = k;
            }
            T.packA.push_back(a);
            T.packB.push_back(b);
            GatherItem g{};
            g.k = k;
            g.src = i * sP + coff; g.lds = T.K1p;
            g.dst = j * sPc + roff[j]; g.ldd = T.K2p;
            T.gather.push_back(g);
            coff += k;
            roff[j] += k;
        }
    }
    for (int i = 0; i < N;) {   // runs of equal tile size share one batched launch per stage
        int e = i;
        while (e + 1 < N && H.d[e + 1] == H.d[i]) ++e;
        T.runs.push_back({i, e});
        i = e + 1;
    }
    return T;
}

TlrWs tlr_carve(char *base, const TlrHost &T, int64_t lds, int64_t ldk) {
    TlrWs w{};
    size_t o = 0;
    auto take = [&](size_t b) -> char * {
        char *p = base ? base + o : nullptr;
        o += align256(b);
        return p;
    };
    const size_t c8 = sizeof(float2);
    const int64_t N = T.N;
    w.Ds = (float2 *)take((size_t)lds * ldk * c8);
    w.A = (float2 *)take((size_t)N * T.Kpmax * T.K1p * c8);
    w.P = (float2 *)take((size_t)N * lds * T.K1p * c8);
    w.B = (float2 *)take((size_t)N * T.K2p * T.dp * c8);
    w.Pcol = (float2 *)take((size_t)N * lds * T.K2p * c8);
    w.R = (float2 *)take((size_t)N * lds * T.dp * c8);
    w.partials = (double *)take((size_t)N * (lds / GEMM_BM) * (T.dp / GEMM_BN) * sizeof(double));
    w.sc = (SolveScalars *)take(sizeof(SolveScalars));
    w.pa = (PackItem *)take(T.packA.size() * sizeof(PackItem));
    w.pb = (PackItem *)take(T.packB.size() * sizeof(PackItem));
    w.gi = (GatherItem *)take(T.gather.size() * sizeof(GatherItem));
    w.bytes = o;
    return w;
}

}  // namespace

extern "C" {

int tlrmdd_workspace_bytes_tlr(tlrmdd_plan plan, size_t *bytes) {
    g_last_error.clear();
    if (!plan || !bytes) return fail(TLRMDD_INVALID_ARGUMENT, "plan / bytes is NULL");
    const TlrHost T = tlr_plan(plan->H, plan->lds);
    *bytes = tlr_carve(nullptr, T, plan->lds, plan->ldk).bytes;
    return TLRMDD_OK;
}

int tlrmdd_forward_tlr(tlrmdd_plan plan, const void *D, const void *U, const void *theta, double *f_dev,
                       void *r_out, void *workspace, size_t ws_bytes, hipStream_t stream) {
    g_last_error.clear();
    if (!plan || !D || !U || !theta || !f_dev || !workspace) return fail(TLRMDD_INVALID_ARGUMENT, "NULL argument");
    const HostLayout &H = plan->H;
    const int64_t ns = H.ns, nr = H.nr, lds = plan->lds, ldk = plan->ldk;
    const TlrHost T = tlr_plan(H, lds);
    const TlrWs w = tlr_carve((char *)workspace, T, lds, ldk);
    if (w.bytes > ws_bytes) return fail(TLRMDD_WORKSPACE, "workspace too small");
    hipStream_t s = stream;
    Upload up;
    up.add(w.pa, T.packA.data(), T.packA.size() * sizeof(PackItem));
    up.add(w.pb, T.packB.data(), T.packB.size() * sizeof(PackItem));
    up.add(w.gi, T.gather.data(), T.gather.size() * sizeof(GatherItem));
    int st = up.commit(s);
    if (st) return st;
    const int64_t N = T.N;
    // padding of the packed operands must read as zero
    HIP_TRY(launch_fill_zero(w.A, (size_t)N * T.Kpmax * T.K1p * sizeof(float2), s));
    HIP_TRY(launch_fill_zero(w.B, (size_t)N * T.K2p * T.dp * sizeof(float2), s));
    HIP_TRY(launch_fill_zero(w.Pcol, (size_t)N * lds * T.K2p * sizeof(float2), s));
    HIP_TRY(launch_stage_d((const float2 *)D, ns, nr, w.Ds, ldk, nullptr, lds, s));
    HIP_TRY(launch_tlr_pack(w.pa, (int)T.packA.size(), (const float2 *)theta, w.A, s));
    HIP_TRY(launch_tlr_pack(w.pb, (int)T.packB.size(), (const float2 *)theta, w.B, s));
    const int64_t tiles2 = (lds / GEMM_BM) * (T.dp / GEMM_BN);
    for (const auto &run : T.runs) {   // stage 1: P_i = D_:,i A_i
        const int i0 = run.first, cnt = run.second - run.first + 1, di = H.d[i0];
        GemmArgs g = gemm_args();
        g.A = w.Ds + H.start[i0]; g.lda = ldk; g.sA = di;
        g.B = w.A + i0 * T.Kpmax * T.K1p; g.ldb = T.K1p; g.sB = T.Kpmax * T.K1p;
        g.C = w.P + i0 * lds * T.K1p; g.ldc = T.K1p; g.sC = lds * T.K1p;
        g.M = (int)lds; g.N = (int)T.K1p; g.K = (int)round_up(di, GEMM_BK);
        HIP_TRY(launch_cgemm(GM_STORE, g, cnt, s));
    }
    HIP_TRY(launch_tlr_gather(w.gi, (int)T.gather.size(), w.P, w.Pcol, lds, s));
    for (const auto &run : T.runs) {   // stage 2: r_:,j = Pcol_j B_j - U_:,j
        const int j0 = run.first, cnt = run.second - run.first + 1, dj = H.d[j0];
        GemmArgs g = gemm_args();
        g.A = w.Pcol + j0 * lds * T.K2p; g.lda = T.K2p; g.sA = lds * T.K2p;
        g.B = w.B + j0 * T.K2p * T.dp; g.ldb = T.dp; g.sB = T.K2p * T.dp;
        g.C = w.R + j0 * lds * T.dp; g.ldc = T.dp; g.sC = lds * T.dp;
        g.E = (const float2 *)U + H.start[j0]; g.lde = nr; g.sE = dj;
        g.partials = w.partials + j0 * tiles2; g.sP = tiles2;
        g.M = (int)lds; g.N = (int)T.dp; g.K = (int)T.K2p;
        g.Me = (int)ns; g.Ne = dj;
        HIP_TRY(launch_cgemm(GM_RESID, g, cnt, s));
    }
    FinArgs f = fin_args(FIN_F_OUT, w.sc);
    f.partials = w.partials;
    f.pstride = N * tiles2;
    f.counts = nullptr;
    f.ucount = (int32_t)(N * tiles2);
    f.nsum = 1;
    f.fout = f_dev;
    HIP_TRY(launch_finalize(f, 1, s));
    if (r_out)
        for (int j = 0; j < N; ++j)
            HIP_TRY(launch_copy2d(w.R + j * lds * T.dp, T.dp, (float2 *)r_out + H.start[j], nr, ns, H.d[j], s));
    return TLRMDD_OK;
}

int hilbert_order(const int32_t *ix, const int32_t *iy, int64_t n, int64_t *perm_out) {
    g_last_error.clear();
    if (n < 0) return fail(TLRMDD_INVALID_ARGUMENT, "n must be >= 0");
    if (n == 0) return TLRMDD_OK;
    if (!ix || !iy || !perm_out) return fail(TLRMDD_INVALID_ARGUMENT, "NULL pointer");
    int32_t mx = 0;
    for (int64_t q = 0; q < n; ++q) {
        if (ix[q] < 0 || iy[q] < 0) return fail(TLRMDD_INVALID_ARGUMENT, "negative grid coordinate");
        mx = std::max(mx, std::max(ix[q], iy[q]));
    }
    int m = 1;
    while (m < 31 && (int64_t(1) << m) <= mx) ++m;   // smallest 2^m > max coordinate
    const int64_t side = int64_t(1) << m;
    std::vector<int64_t> h(n);
    for (int64_t q = 0; q < n; ++q) {
        int64_t x = ix[q], y = iy[q], d = 0;
        for (int64_t s = side / 2; s > 0; s /= 2) {
            const int64_t rx = (x & s) ? 1 : 0;
            const int64_t ry = (y & s) ? 1 : 0;
            d += s * s * ((3 * rx) ^ ry);
            if (ry == 0) {   // rotate the quadrant into canonical orientation
                if (rx == 1) {
                    x = side - 1 - x;
                    y = side - 1 - y;
                }
                std::swap(x, y);
            }
        }
        h[q] = d;
    }
    std::vector<int64_t> idx(n);
    for (int64_t q = 0; q < n; ++q) idx[q] = q;
    std::stable_sort(idx.begin(), idx.end(), [&](int64_t a, int64_t b) { return h[a] < h[b]; });
    std::memcpy(perm_out, idx.data(), n * sizeof(int64_t));
    return TLRMDD_OK;
}

int tlrmdd_permute_columns(const void *in, const int64_t *perm, void *out, int64_t rows, int64_t cols,
                           int32_t *bad_dev, hipStream_t stream) {
    g_last_error.clear();
    if (rows < 0 || cols < 0) return fail(TLRMDD_INVALID_ARGUMENT, "negative size");
    if (rows == 0 || cols == 0) return TLRMDD_OK;
    if (!in || !perm || !out) return fail(TLRMDD_INVALID_ARGUMENT, "NULL pointer");
    const char *a = (const char *)in, *b = (const char *)out;
    const size_t bytes = (size_t)rows * (size_t)cols * sizeof(float2);
    if (a < b + bytes && b < a + bytes) return fail(TLRMDD_INVALID_ARGUMENT, "in and out must not overlap");
    HIP_TRY(timed(TLRMDD_K_PERMUTE, stream, bytes_work(16.0 * (double)rows * (double)cols + 8.0 * (double)cols), [&] {
        return launch_permute_cols((const float2 *)in, perm, (float2 *)out, rows, cols, bad_dev, stream);
    }));
    return TLRMDD_OK;
}

}  // extern "C"
