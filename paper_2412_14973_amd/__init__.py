"""MI355X (gfx950) tile low-rank multidimensional deconvolution (TLR-MDD).

Python binding of the C ABI in include/tlrmdd.h: arguments are torch device
tensors (complex64, contiguous) and the current torch stream; every step of
the computation runs in the library's HIP kernels. Method: Chen, Ravasi,
Keyes, arXiv 2412.14973 (objective eq. X2LQR_lst, gradients eqs. DXLR,
Hilbert receiver re-ordering eq. axb_sd).
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import BF16X3, FP32, FP32_3M, GD, LBFGS, TLRMDDError  # noqa: F401

__all__ = ["Plan", "hilbert_order", "permute_columns", "forward", "grad", "solve", "solve_batched", "adjoint",
           "benchmark_solve",
           "TLRMDDError", "FP32", "BF16X3", "LBFGS", "GD"]


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_tensor(t, name, dtype=torch.complex64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a torch device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Plan:
    """Validated tile layout of one frequency (tile sizes d_i, ranks k) plus device tables.

    tile_size: d_i (sum = nr); rank_off: k_t of tile (i, j), i > j, t = i(i-1)/2 + j;
    rank_diag: k_ii >= 1 (Q Q^T) or -1 (dense); ns: number of sources.
    """

    def __init__(self, tile_size, rank_off, rank_diag, ns):
        lib = _lib.load()
        self.tile_size = np.ascontiguousarray(tile_size, dtype=np.int32)
        self.rank_off = np.ascontiguousarray(rank_off, dtype=np.int32)
        self.rank_diag = np.ascontiguousarray(rank_diag, dtype=np.int32)
        self.nr = int(self.tile_size.sum())
        self.ns = int(ns)
        P = ctypes.POINTER(ctypes.c_int32)
        self._c = _lib.c_layout(self.nr, self.ns, int(self.tile_size.shape[0]),
                                self.tile_size.ctypes.data_as(P),
                                self.rank_off.ctypes.data_as(P) if self.rank_off.size else None,
                                self.rank_diag.ctypes.data_as(P))
        h = ctypes.c_void_p()
        _lib.check(lib.tlrmdd_plan_create(ctypes.byref(self._c), ctypes.byref(h)), "tlrmdd_plan_create")
        self._h = h
        self.theta_size = int(lib.tlrmdd_theta_size(ctypes.byref(self._c)))

    @classmethod
    def from_layout(cls, layout, ns):
        return cls(layout.tile_size, layout.rank_off, layout.rank_diag, ns)

    @property
    def handle(self):
        return self._h

    def workspace_bytes(self, op, opts=None):
        n = ctypes.c_size_t()
        _lib.check(_lib.load().tlrmdd_workspace_bytes(self._h, op, ctypes.byref(opts) if opts else None,
                                                      ctypes.byref(n)), "tlrmdd_workspace_bytes")
        return int(n.value)

    def workspace(self, op, opts=None, device=None):
        return torch.empty(max(self.workspace_bytes(op, opts), 1), dtype=torch.uint8,
                           device=device or torch.device("cuda"))

    def __del__(self):
        try:
            if getattr(self, "_h", None) and _lib._lib is not None:
                _lib._lib.tlrmdd_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass


def hilbert_order(ix, iy):
    """perm[k] = natural index of the k-th receiver along the Hilbert curve (host)."""
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    iy = np.ascontiguousarray(iy, dtype=np.int32)
    if ix.shape != iy.shape or ix.ndim != 1:
        raise ValueError("ix and iy must be 1-D arrays of equal length")
    out = np.empty(ix.shape[0], dtype=np.int64)
    _lib.check(_lib.load().hilbert_order(ix.ctypes.data, iy.ctypes.data, ix.shape[0], out.ctypes.data),
               "hilbert_order")
    return out


def permute_columns(A, perm, bad=None):
    """out[:, k] = A[:, perm[k]] on the device (Dhat = D S). bad: optional device int32 tensor (one
    element, cleared by the caller) that the kernel sets to 1 when a perm entry is outside [0, cols);
    such columns come out as zeros."""
    _dev_tensor(A, "A")
    _dev_tensor(perm, "perm", torch.int64)
    if bad is not None:
        _dev_tensor(bad, "bad", torch.int32)
    rows, cols = A.shape
    if perm.shape != (cols,):
        raise ValueError("perm must have one entry per column")
    out = torch.empty_like(A)
    _lib.check(_lib.load().tlrmdd_permute_columns(_ptr(A), _ptr(perm), _ptr(out), rows, cols, _ptr(bad), _stream()),
               "tlrmdd_permute_columns")
    return out


def _check_problem(plan, D, U, theta):
    _dev_tensor(D, "D")
    _dev_tensor(U, "U")
    _dev_tensor(theta, "theta")
    if tuple(D.shape) != (plan.ns, plan.nr) or tuple(U.shape) != (plan.ns, plan.nr):
        raise ValueError(f"D and U must be {plan.ns} x {plan.nr}")
    if theta.numel() != plan.theta_size:
        raise ValueError(f"theta must hold {plan.theta_size} complex entries")


def forward(plan, D, U, theta, precision=FP32, want_r=False, want_X=False, workspace=None):
    """f = 1/2 ||D C(theta) - U||^2 (device FP64 0-dim tensor), optionally r and X."""
    _check_problem(plan, D, U, theta)
    f = torch.empty((), dtype=torch.float64, device=D.device)
    r = torch.empty((plan.ns, plan.nr), dtype=torch.complex64, device=D.device) if want_r else None
    X = torch.empty((plan.nr, plan.nr), dtype=torch.complex64, device=D.device) if want_X else None
    ws = workspace if workspace is not None else plan.workspace(_lib.OP_FORWARD, device=D.device)
    _lib.check(_lib.load().tlrmdd_forward(plan.handle, _ptr(D), _ptr(U), _ptr(theta), _ptr(f), _ptr(r), _ptr(X),
                                          precision, _ptr(ws), ws.numel(), _stream()), "tlrmdd_forward")
    return f, r, X


def grad(plan, D, U, theta, precision=FP32, workspace=None):
    """(f, grad) with grad = df/dRe + i df/dIm of every packed factor."""
    _check_problem(plan, D, U, theta)
    f = torch.empty((), dtype=torch.float64, device=D.device)
    g = torch.empty_like(theta)
    ws = workspace if workspace is not None else plan.workspace(_lib.OP_GRAD, device=D.device)
    _lib.check(_lib.load().tlrmdd_grad(plan.handle, _ptr(D), _ptr(U), _ptr(theta), _ptr(f), _ptr(g), precision,
                                       _ptr(ws), ws.numel(), _stream()), "tlrmdd_grad")
    return f, g


def adjoint(plan, D, U, precision=FP32, workspace=None):
    """X_adj = D^H U (nr x nr complex64 on the device)."""
    _dev_tensor(D, "D")
    _dev_tensor(U, "U")
    X = torch.empty((plan.nr, plan.nr), dtype=torch.complex64, device=D.device)
    ws = workspace if workspace is not None else plan.workspace(_lib.OP_GRAD, device=D.device)
    _lib.check(_lib.load().tlrmdd_adjoint(plan.handle, _ptr(D), _ptr(U), _ptr(X), precision, _ptr(ws), ws.numel(),
                                          _stream()), "tlrmdd_adjoint")
    return X


def benchmark_solve(D, U, lam, iters, precision=FP32, lbfgs_m=5, Z0=None):
    """Benchmark (preconditioned Tikhonov) solver: min 1/2 ||D P Z - U||^2 + lam ||Z||^2 with
    P Z = (Z + Z^T)/2, then X = P Z. It is the tile solve with one dense diagonal tile of size
    nr; returns (X, f_hist)."""
    ns, nr = D.shape
    plan = Plan(np.array([nr]), np.zeros(0, dtype=np.int32), np.array([-1]), ns)
    Z = Z0 if Z0 is not None else torch.zeros(nr * nr, dtype=torch.complex64, device=D.device)
    Z, fh = solve(plan, D, U, Z, iters, lbfgs_m=lbfgs_m, precision=precision, lam=lam)
    _, _, X = forward(plan, D, U, Z, precision, want_X=True)
    return X, fh


# The residual is tracked as r += a a + a^2 b; its FP32 rounding accumulates over the iterations, so by
# default it is recomputed from theta every 20 iterations (keeps 100-iteration FP32 solves at nr = 4096
# within 1e-5 of the FP64 oracle in the factors; about 1 % more work).
RESID_REFRESH = 20


# line-search products from the assembled X1, X2 / in tile form where cheaper / and the gradient in tile form
# where cheaper too
LINE_DENSE, LINE_TILE, LINE_TILE_GRAD = 0, 1, 2


def make_opts(iters, optimizer=LBFGS, lbfgs_m=5, precision=FP32, lam=0.0, resid_refresh=RESID_REFRESH, streams=1,
              line_products=LINE_DENSE):
    return _lib.c_opts(int(iters), int(optimizer), int(lbfgs_m), int(precision), float(lam), int(resid_refresh),
                       int(streams), int(line_products), 0)


def line_form(plan, precision=FP32_3M, line_products=LINE_TILE):
    """(tile_form, kpad): 0 when the line search of this plan runs on the dense products under these
    options, 1 in tile form, 2 with the gradient in tile form as well."""
    tf, kp = ctypes.c_int(), ctypes.c_int()
    opts = make_opts(1, precision=precision, line_products=line_products)
    _lib.check(_lib.load().tlrmdd_line_form(plan.handle, ctypes.byref(opts), ctypes.byref(tf), ctypes.byref(kp)),
               "tlrmdd_line_form")
    return int(tf.value), int(kp.value)


def solve(plan, D, U, theta0, iters, optimizer=LBFGS, lbfgs_m=5, precision=FP32, lam=0.0, resid_refresh=RESID_REFRESH,
          workspace=None, line_products=LINE_DENSE):
    """Fixed-count solve from theta0; returns (theta_T, f_hist) with f_hist[t] (FP64, device)."""
    _check_problem(plan, D, U, theta0)
    opts = make_opts(iters, optimizer, lbfgs_m, precision, lam, resid_refresh, line_products=line_products)
    theta = theta0.clone()
    fh = torch.empty(iters + 1, dtype=torch.float64, device=D.device)
    ws = workspace if workspace is not None else plan.workspace(_lib.OP_SOLVE, opts, device=D.device)
    _lib.check(_lib.load().tlrmdd_solve(plan.handle, _ptr(D), _ptr(U), _ptr(theta), ctypes.byref(opts), _ptr(fh),
                                        _ptr(ws), ws.numel(), _stream()), "tlrmdd_solve")
    return theta, fh


def batched_workspace_bytes(plans, opts):
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    n = ctypes.c_size_t()
    _lib.check(_lib.load().tlrmdd_workspace_bytes_batched(len(plans), arr, ctypes.byref(opts), ctypes.byref(n)),
               "tlrmdd_workspace_bytes_batched")
    return int(n.value)


def solve_batched(plans, Ds, Us, thetas0, iters, optimizer=LBFGS, lbfgs_m=5, precision=FP32, lam=0.0,
                  resid_refresh=RESID_REFRESH, workspace=None, out_thetas=None, out_fhist=None, streams=1,
                  line_products=LINE_DENSE):
    """Solve independent frequencies of equal nr, ns with fused launches per phase (per sub-batch:
    streams > 1 runs problem i in sub-batch i % streams on its own stream; same results;
    line_products=LINE_TILE groups the problems by line-search form)."""
    n = len(plans)
    for p, D, U, th in zip(plans, Ds, Us, thetas0):
        _check_problem(p, D, U, th)
    opts = make_opts(iters, optimizer, lbfgs_m, precision, lam, resid_refresh, streams, line_products)
    thetas = out_thetas if out_thetas is not None else [t.clone() for t in thetas0]
    if out_thetas is not None:
        for dst, src in zip(thetas, thetas0):
            dst.copy_(src)
    fh = out_fhist if out_fhist is not None else [torch.empty(iters + 1, dtype=torch.float64, device=Ds[0].device)
                                                  for _ in range(n)]
    V = ctypes.c_void_p * n
    ws = workspace if workspace is not None else torch.empty(batched_workspace_bytes(plans, opts),
                                                             dtype=torch.uint8, device=Ds[0].device)
    _lib.check(_lib.load().tlrmdd_solve_batched(
        n, V(*[p.handle.value for p in plans]), V(*[d.data_ptr() for d in Ds]), V(*[u.data_ptr() for u in Us]),
        V(*[t.data_ptr() for t in thetas]), ctypes.byref(opts), V(*[f.data_ptr() for f in fh]),
        _ptr(ws), ws.numel(), _stream()), "tlrmdd_solve_batched")
    return thetas, fh


def make_admm_opts(lams=(10.0, 1.0, 0.1), outer=5, inner=10, rho=1.0, optimizer=LBFGS, lbfgs_m=5,
                   precision=FP32, streams=1, line_products=LINE_DENSE):
    """ADMM options; the returned struct keeps its lambda array alive."""
    lam_arr = (ctypes.c_double * len(lams))(*[float(v) for v in lams])
    o = _lib.c_admm_opts(make_opts(inner, optimizer, lbfgs_m, precision, streams=streams, line_products=line_products),
                         len(lams), int(outer),
                         ctypes.cast(lam_arr, ctypes.POINTER(ctypes.c_double)), float(rho))
    o._keep = lam_arr
    return o


def admm_workspace_bytes(plans, aopts):
    arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
    n = ctypes.c_size_t()
    _lib.check(_lib.load().tlrmdd_workspace_bytes_admm(len(plans), arr, ctypes.byref(aopts), ctypes.byref(n)),
               "tlrmdd_workspace_bytes_admm")
    return int(n.value)


def admm_batched(plans, Ds, Us, thetas0, lams=(10.0, 1.0, 0.1), outer=5, inner=10, rho=1.0, optimizer=LBFGS,
                 lbfgs_m=5, precision=FP32, workspace=None, streams=1, line_products=LINE_DENSE):
    """Scaled ADMM with lambda continuation over independent frequencies of equal nr, ns.

    Returns (thetas, f_hists); f_hist[k] is the data misfit at the start (k = 0) and after
    the k-th X-update (1 + len(lams) * outer entries, FP64, device)."""
    n = len(plans)
    for p, D, U, th in zip(plans, Ds, Us, thetas0):
        _check_problem(p, D, U, th)
    aopts = make_admm_opts(lams, outer, inner, rho, optimizer, lbfgs_m, precision, streams, line_products)
    thetas = [t.clone() for t in thetas0]
    fh = [torch.empty(1 + len(lams) * outer, dtype=torch.float64, device=Ds[0].device) for _ in range(n)]
    ws = workspace if workspace is not None else torch.empty(admm_workspace_bytes(plans, aopts),
                                                             dtype=torch.uint8, device=Ds[0].device)
    V = ctypes.c_void_p * n
    _lib.check(_lib.load().tlrmdd_admm_batched(
        n, V(*[p.handle.value for p in plans]), V(*[d.data_ptr() for d in Ds]), V(*[u.data_ptr() for u in Us]),
        V(*[t.data_ptr() for t in thetas]), ctypes.byref(aopts), V(*[f.data_ptr() for f in fh]),
        _ptr(ws), ws.numel(), _stream()), "tlrmdd_admm_batched")
    return thetas, fh


def admm(plan, D, U, theta0, lams=(10.0, 1.0, 0.1), outer=5, inner=10, rho=1.0, optimizer=LBFGS, lbfgs_m=5,
         precision=FP32, workspace=None, line_products=LINE_DENSE):
    """Scaled ADMM with lambda continuation on one frequency; returns (theta, f_hist)."""
    _check_problem(plan, D, U, theta0)
    aopts = make_admm_opts(lams, outer, inner, rho, optimizer, lbfgs_m, precision, line_products=line_products)
    theta = theta0.clone()
    fh = torch.empty(1 + len(lams) * outer, dtype=torch.float64, device=D.device)
    ws = workspace if workspace is not None else torch.empty(admm_workspace_bytes([plan], aopts),
                                                             dtype=torch.uint8, device=D.device)
    _lib.check(_lib.load().tlrmdd_admm(plan.handle, _ptr(D), _ptr(U), _ptr(theta), ctypes.byref(aopts), _ptr(fh),
                                       _ptr(ws), ws.numel(), _stream()), "tlrmdd_admm")
    return theta, fh


def forward_tlr(plan, D, U, theta, want_r=False, workspace=None):
    """f = 1/2 ||D C(theta) - U||^2 by the tile low-rank product (no dense X); returns (f, r or None)."""
    _check_problem(plan, D, U, theta)
    f = torch.empty((), dtype=torch.float64, device=D.device)
    r = torch.empty((plan.ns, plan.nr), dtype=torch.complex64, device=D.device) if want_r else None
    if workspace is None:
        n = ctypes.c_size_t()
        _lib.check(_lib.load().tlrmdd_workspace_bytes_tlr(plan.handle, ctypes.byref(n)), "tlrmdd_workspace_bytes_tlr")
        workspace = torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=D.device)
    _lib.check(_lib.load().tlrmdd_forward_tlr(plan.handle, _ptr(D), _ptr(U), _ptr(theta), _ptr(f),
                                              _ptr(r), _ptr(workspace),
                                              workspace.numel(), _stream()), "tlrmdd_forward_tlr")
    return f, r


def tlr_workspace_bytes(plan):
    n = ctypes.c_size_t()
    _lib.check(_lib.load().tlrmdd_workspace_bytes_tlr(plan.handle, ctypes.byref(n)), "tlrmdd_workspace_bytes_tlr")
    return int(n.value)


def tile_split(nr, d):
    """Tile sizes of size d covering nr (ragged last tile), as the estimate uses them."""
    return np.array([d] * (nr // d) + ([nr % d] if nr % d else []), dtype=np.int32)


def _ranks_workspace(nr, d, device):
    n = ctypes.c_size_t()
    _lib.check(_lib.load().tlrmdd_workspace_bytes_ranks(int(nr), int(d), ctypes.byref(n)),
               "tlrmdd_workspace_bytes_ranks")
    return torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=device)


def tile_ranks(X, d, eps=0.01):
    """Numerical ranks of the tiles of a symmetric X (device, nr x nr complex64) at tile size d:
    #{sigma >= eps v0} per tile, v0 the largest singular value of all tiles (FP64 Jacobi on the GPU).
    Returns (k_off in t order, k_diag, v0); synchronises the stream."""
    nr = int(X.shape[0])
    ws = _ranks_workspace(nr, d, X.device)   # validates nr and d
    N = len(tile_split(nr, d))
    ko = np.zeros(max(N * (N - 1) // 2, 1), dtype=np.int32)
    kd = np.zeros(N, dtype=np.int32)
    v0 = ctypes.c_double()
    _lib.check(_lib.load().tlrmdd_tile_ranks(_ptr(X), nr, int(d), float(eps), ko.ctypes.data, kd.ctypes.data,
                                             ctypes.byref(v0), _ptr(ws), ws.numel(), _stream()), "tlrmdd_tile_ranks")
    return ko[:N * (N - 1) // 2], kd, v0.value


def choose_layout(X, candidates, eps=0.01):
    """Tile size with the fewest factor entries among `candidates` and its layout (ranks >= 1, dense
    diagonal tiles where k_ii >= d_i / 2). Returns (d, tile_size, rank_off, rank_diag, entries)."""
    nr = int(X.shape[0])
    cand = np.ascontiguousarray(candidates, dtype=np.int32)
    nmax = max(len(tile_split(nr, int(d))) for d in cand)
    ro = np.zeros(max(nmax * (nmax - 1) // 2, 1), dtype=np.int32)
    rd = np.zeros(nmax, dtype=np.int32)
    ent = np.zeros(len(cand), dtype=np.int64)
    dsel = ctypes.c_int32()
    ws = _ranks_workspace(nr, int(cand.max()), X.device)
    _lib.check(_lib.load().tlrmdd_choose_layout(_ptr(X), nr, cand.ctypes.data, len(cand), float(eps),
                                                ctypes.byref(dsel), ent.ctypes.data, ro.ctypes.data, ro.size,
                                                rd.ctypes.data, rd.size, _ptr(ws), ws.numel(), _stream()),
               "tlrmdd_choose_layout")
    sizes = tile_split(nr, dsel.value)
    N = len(sizes)
    return dsel.value, sizes, ro[:N * (N - 1) // 2].copy(), rd[:N].copy(), ent


def warm_start(plan, X):
    """Factors of `plan`'s layout from a reference solution X (device, nr x nr complex64): truncated
    SVD of every off-diagonal tile, Takagi factor of every Q Q^T tile, Z = X_ii for dense ones."""
    n = ctypes.c_size_t()
    _lib.check(_lib.load().tlrmdd_workspace_bytes_warm(plan.handle, ctypes.byref(n)), "tlrmdd_workspace_bytes_warm")
    ws = torch.empty(max(int(n.value), 1), dtype=torch.uint8, device=X.device)
    theta = torch.zeros(plan.theta_size, dtype=torch.complex64, device=X.device)
    _lib.check(_lib.load().tlrmdd_warm_start(plan.handle, _ptr(X), _ptr(theta), _ptr(ws), ws.numel(), _stream()),
               "tlrmdd_warm_start")
    return theta


class Graph:
    """Library calls recorded into a HIP graph (tlrmdd_graph_*): launch() replays them on the current
    stream. The tensors the recorded calls use are held here, so their memory stays put."""

    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep

    def launch(self):
        _lib.check(_lib.load().tlrmdd_graph_launch(self._h, _stream()), "tlrmdd_graph_launch")

    def __del__(self):
        # as Plan: at interpreter exit the module globals may already be gone
        try:
            if getattr(self, "_h", None) is not None and self._h.value and _lib._lib is not None:
                _lib._lib.tlrmdd_graph_destroy(self._h)
                self._h = None
        except Exception:
            pass


def _record(call, keep):
    """Run `call` (library calls only, on the current stream) under a graph capture on a stream of
    its own, after the current stream's pending work; returns the Graph."""
    lib = _lib.load()
    cur = torch.cuda.current_stream()
    side = torch.cuda.Stream()   # default priority; the null stream cannot be captured
    side.wait_stream(cur)
    h = ctypes.c_void_p()
    with torch.cuda.stream(side):
        s = _stream()
        _lib.check(lib.tlrmdd_graph_begin(s), "tlrmdd_graph_begin")
        try:
            call()
        finally:
            st = lib.tlrmdd_graph_end(s, ctypes.byref(h))
    _lib.check(st, "tlrmdd_graph_end")
    cur.wait_stream(side)
    return Graph(h, keep + [side])


def solve_graph(plan, D, U, theta, fhist, iters, optimizer=LBFGS, lbfgs_m=5, precision=FP32, lam=0.0,
                resid_refresh=RESID_REFRESH, workspace=None, line_products=LINE_DENSE):
    """tlrmdd_solve recorded as a HIP graph: each launch() runs `iters` iterations from the current
    contents of `theta` (updated in place) and writes `fhist`; restore theta for a fresh solve."""
    _check_problem(plan, D, U, theta)
    opts = make_opts(iters, optimizer, lbfgs_m, precision, lam, resid_refresh, line_products=line_products)
    ws = workspace if workspace is not None else plan.workspace(_lib.OP_SOLVE, opts, device=D.device)

    def call():
        _lib.check(_lib.load().tlrmdd_solve(plan.handle, _ptr(D), _ptr(U), _ptr(theta), ctypes.byref(opts),
                                            _ptr(fhist), _ptr(ws), ws.numel(), _stream()), "tlrmdd_solve")
    return _record(call, [plan, D, U, theta, fhist, ws, opts])


def solve_batched_graph(plans, Ds, Us, thetas, fhists, iters, optimizer=LBFGS, lbfgs_m=5, precision=FP32, lam=0.0,
                        resid_refresh=RESID_REFRESH, workspace=None, streams=1, line_products=LINE_DENSE):
    """tlrmdd_solve_batched recorded as a HIP graph (thetas updated in place at every launch)."""
    n = len(plans)
    for p, D, U, th in zip(plans, Ds, Us, thetas):
        _check_problem(p, D, U, th)
    opts = make_opts(iters, optimizer, lbfgs_m, precision, lam, resid_refresh, streams, line_products)
    ws = workspace if workspace is not None else torch.empty(batched_workspace_bytes(plans, opts),
                                                             dtype=torch.uint8, device=Ds[0].device)
    V = ctypes.c_void_p * n
    args = (V(*[p.handle.value for p in plans]), V(*[d.data_ptr() for d in Ds]), V(*[u.data_ptr() for u in Us]),
            V(*[t.data_ptr() for t in thetas]), V(*[f.data_ptr() for f in fhists]))

    def call():
        _lib.check(_lib.load().tlrmdd_solve_batched(n, args[0], args[1], args[2], args[3], ctypes.byref(opts),
                                                    args[4], _ptr(ws), ws.numel(), _stream()),
                   "tlrmdd_solve_batched")
    return _record(call, [list(plans), list(Ds), list(Us), list(thetas), list(fhists), ws, opts, args])


class KernelTimer:
    """Context manager: per kernel kind the summed launch milliseconds (HIP events on the launch
    stream), launch count and the algorithmic work the library counted for those launches.

    kinds: names from KIND_NAMES to time (default: all); launches of the other kinds run untimed
    and read zero, and each timed launch costs two event records on its stream."""

    def __init__(self, kinds=None):
        self.kinds = None if kinds is None else list(kinds)

    def __enter__(self):
        if self.kinds is None:
            _lib.check(_lib.load().tlrmdd_timing_begin(), "tlrmdd_timing_begin")
        else:
            mask = 0
            for k in self.kinds:
                mask |= 1 << _lib.KIND_NAMES.index(k)
            _lib.check(_lib.load().tlrmdd_timing_begin_kinds(mask), "tlrmdd_timing_begin_kinds")
        return self

    def __exit__(self, *exc):
        st = (_lib.c_kernel_stats * _lib.K_NKINDS)()
        _lib.check(_lib.load().tlrmdd_timing_end(st), "tlrmdd_timing_end")
        names = _lib.KIND_NAMES
        self.ms = {k: st[i].ms for i, k in enumerate(names)}
        self.launches = {k: st[i].launches for i, k in enumerate(names)}
        self.cflops = {k: st[i].cflops for i, k in enumerate(names)}
        self.flops = {k: st[i].flops for i, k in enumerate(names)}
        self.bytes = {k: st[i].bytes for i, k in enumerate(names)}
        self.dtype = {k: {_lib.DT_NONE: None, _lib.DT_FP32: "f32", _lib.DT_BF16: "bf16",
                          _lib.DT_MIXED: "mixed"}[st[i].flop_dtype] for i, k in enumerate(names)}
        return False


class TLRMDDObjective(torch.autograd.Function):
    """f(theta) = 1/2 ||D C(theta) - U||^2 with a hand-written HIP backward.

    forward saves theta and references to D and U (never X); backward
    re-assembles X inside tlrmdd_grad and returns grad_output * grad, where
    grad = df/dRe + i df/dIm is torch's convention for complex leaves.
    """

    @staticmethod
    def forward(ctx, theta, D, U, plan, precision=FP32):
        f, _, _ = forward(plan, D, U, theta, precision)
        ctx.save_for_backward(theta)
        ctx.D, ctx.U, ctx.plan, ctx.precision = D, U, plan, precision
        return f

    @staticmethod
    def backward(ctx, gout):
        (theta,) = ctx.saved_tensors
        _, g = grad(ctx.plan, ctx.D, ctx.U, theta, ctx.precision)
        return (gout.to(torch.float32) * g), None, None, None, None


def objective(theta, D, U, plan, precision=FP32):
    """Differentiable TLR-MDD objective (see TLRMDDObjective)."""
    return TLRMDDObjective.apply(theta, D, U, plan, precision)
