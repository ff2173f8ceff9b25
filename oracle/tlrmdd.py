"""Plain FP64 CPU oracle for tile low-rank multidimensional deconvolution.

TEST INFRASTRUCTURE ONLY. Only the test-suite, the package smoke check and the
CPU-baseline leg of the benchmark may import this module; the product path
never does. It shares no code with the HIP library: every function below is
written directly from the paper (arXiv 2412.14973, "Reciprocity-aware adaptive
tile low-rank factorization for large-scale 3D multidimensional
deconvolution") in complex128 with plain NumPy, without blocking or fusion.

Section / equation map (names as in the paper):
  * Theory, eq. (axb) and eq. (standard_solver): D X = U, min 1/2 ||D X - U||_F^2
    solved for each frequency independently; X = X^T (reciprocity).
  * Tile Low-rank MDD: diagonal tiles X_ii = Q_ii Q_ii^T or X_ii = P Z_ii with
    P = (I + Gamma)/2; sub-diagonal X_ij = L_ij R_ij (i > j); super-diagonal
    X_ji = X_ij^T; stacks Zbar, Lbar, Rbar.
  * Receivers re-ordering, eqs. (hilbert)-(axb_sd): X_h = S^T X S, Dhat = D S,
    Uhat = U S, S from a Hilbert space-filling curve over the receiver grid.
  * ADMM solver, eq. (X2LQR_lst): f = 1/2 ||D C(Zbar, Lbar, Rbar) - U||_F^2.
  * ADMM solver, gradient equations (DXLR): W = D^H (D X - U), W' = W + W^T,
    grad L = W' R^H, grad R = L^H W', grad Z = W'/2, grad Q = W' conj(Q).
  * ADMM solver, X-update: limited-memory BFGS (Liu & Nocedal 1989); here with
    an exact line search along the quartic f(theta + alpha p).
  * Hyper-parameter selection: Frobenius regulariser lambda ||.||_F^2 whose
    gradient is 2 lambda theta; lambda continuation 10 -> 1 -> 0.1.
  * ADMM solver, X-update / Z-update (eq. proxofFro2) / dual update: scaled
    ADMM on min f(theta) + lambda ||theta||^2 with the split theta = z.
  * Hyper-parameter selection and the examples' rank study: per-tile SVD of a
    reference solution, numerical rank k = #{sigma >= eps v0} with v0 the
    largest singular value over all tiles of that size (eps = 0.01), the tile
    size with the fewest factor entries; warm start L = U_k S_k^(1/2),
    R = S_k^(1/2) V_k^H, Q Q^T = X_ii by the Takagi factorisation (eq. qqinit),
    Z_ii = X_ii for dense diagonal tiles.

Readings where the paper is silent (the same readings the GPU path follows):
  * gradient convention: 2 df/d(conj theta) = df/dRe + i df/dIm (the paper
    calls W the gradient w.r.t. X for f = 1/2||DX-U||^2);
  * Lbar / Rbar order: row-major lower triangle, t = i(i-1)/2 + j (0-based);
  * theta packing: all diagonal blocks (Q_ii d_i x k_ii, or Z_ii d_i x d_i),
    then all L_t (d_i x k_t), then all R_t (k_t x d_j), row-major each;
  * Hilbert curve: classic quadrant construction on the smallest enclosing
    2^m grid, starting at (0,0) and ending at (2^m - 1, 0); x = station along
    a line, y = line; natural index iy*nx + ix; stable ties.
  * L-BFGS: two-loop recursion with the real inner product Re<a,b>, memory m,
    H0 = gamma I with gamma = Re<s,y>/Re<y,y> of the newest pair (1 without
    pairs); steepest descent restart when Re<g,p> >= 0; pairs stored only when
    Re<s,y> > 0.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Tuple

import numpy as np


# ============================================================================
# Receivers re-ordering: Hilbert curve (Receivers re-ordering section)
# ============================================================================
def hilbert_index(x: int, y: int, n: int) -> int:
    """Position of grid cell (x, y) along the Hilbert curve filling an n x n grid.

    Quadrant construction: at each scale s = n/2, n/4, ..., 1 the quadrant
    (rx, ry) contributes s^2 * ((3 rx) xor ry) cells, after which the
    coordinates are reflected / swapped so that the sub-square is traversed
    in the canonical orientation.
    """
    h = 0
    s = n // 2
    while s > 0:
        rx = 1 if (x & s) else 0
        ry = 1 if (y & s) else 0
        h += s * s * ((3 * rx) ^ ry)
        if ry == 0:
            if rx == 1:
                x = n - 1 - x
                y = n - 1 - y
            x, y = y, x
        s //= 2
    return h


def hilbert_order(ix: np.ndarray, iy: np.ndarray) -> np.ndarray:
    """perm[k] = natural index of the k-th receiver along the Hilbert curve.

    ix, iy are 0-based grid coordinates of each receiver (receiver q has
    natural index q). The curve lives on the smallest 2^m x 2^m grid that
    encloses every point; points are stably sorted by their curve position.
    """
    ix = np.asarray(ix, dtype=np.int64)
    iy = np.asarray(iy, dtype=np.int64)
    if ix.size == 0:
        return np.zeros(0, dtype=np.int64)
    if ix.min() < 0 or iy.min() < 0:
        raise ValueError("grid coordinates must be non-negative")
    m = max(1, int(max(ix.max(), iy.max())).bit_length())
    n = 1 << m
    h = np.array([hilbert_index(int(a), int(b), n) for a, b in zip(ix, iy)], dtype=np.int64)
    return np.argsort(h, kind="stable").astype(np.int64)


def permute_columns(A: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """Dhat = D S: column k of the result is column perm[k] of A (eq. axb_sd)."""
    return A[:, perm]


def unpermute(Xh: np.ndarray, perm: np.ndarray) -> np.ndarray:
    """X = S X_h S^T (eq. hilbert1): X[perm[a], perm[b]] = X_h[a, b]."""
    X = np.empty_like(Xh)
    X[np.ix_(perm, perm)] = Xh
    return X


# ============================================================================
# Tile layout and the stacks Zbar, Lbar, Rbar (Tile Low-rank MDD section)
# ============================================================================
@dataclasses.dataclass
class Tiling:
    """Offsets of every factor inside the packed unknown vector theta."""
    d: List[int]           # tile sizes d_i
    start: List[int]       # first row/column of tile i
    kdiag: List[int]       # >=1: Q_ii rank; -1: dense Z_ii
    pairs: List[Tuple[int, int, int]]   # (i, j, k_ij) for i > j in t order
    off_diag: List[int]    # theta offset of Q_ii / Z_ii
    off_L: List[int]       # theta offset of L_t
    off_R: List[int]       # theta offset of R_t
    size: int              # total complex unknowns

    @property
    def n(self) -> int:
        return len(self.d)

    @property
    def nr(self) -> int:
        return sum(self.d)


def tiling(tile_size, rank_off, rank_diag) -> Tiling:
    d = [int(v) for v in tile_size]
    N = len(d)
    if N == 0 or any(v <= 0 for v in d):
        raise ValueError("tile sizes must be positive")
    start = [0] * N
    for i in range(1, N):
        start[i] = start[i - 1] + d[i - 1]
    kdiag = [int(v) for v in rank_diag]
    if len(kdiag) != N:
        raise ValueError("rank_diag needs one entry per tile")
    pairs = []
    t = 0
    rank_off = [int(v) for v in rank_off]
    if len(rank_off) != N * (N - 1) // 2:
        raise ValueError("rank_off needs N(N-1)/2 entries")
    for i in range(N):
        for j in range(i):
            k = rank_off[t]
            if k < 1 or k > min(d[i], d[j]):
                raise ValueError("off-diagonal rank out of range")
            pairs.append((i, j, k))
            t += 1
    pos = 0
    off_diag = []
    for i in range(N):
        if not (kdiag[i] == -1 or 1 <= kdiag[i] <= d[i]):
            raise ValueError("diagonal rank out of range")
        off_diag.append(pos)
        pos += d[i] * (d[i] if kdiag[i] < 0 else kdiag[i])
    off_L = []
    for (i, j, k) in pairs:
        off_L.append(pos)
        pos += d[i] * k
    off_R = []
    for (i, j, k) in pairs:
        off_R.append(pos)
        pos += k * d[j]
    return Tiling(d, start, kdiag, pairs, off_diag, off_L, off_R, pos)


def diag_block(T: Tiling, theta: np.ndarray, i: int) -> np.ndarray:
    """Q_ii (d_i x k_ii) or Z_ii (d_i x d_i) as a view into theta."""
    cols = T.d[i] if T.kdiag[i] < 0 else T.kdiag[i]
    o = T.off_diag[i]
    return theta[o:o + T.d[i] * cols].reshape(T.d[i], cols)


def L_block(T: Tiling, theta: np.ndarray, t: int) -> np.ndarray:
    i, j, k = T.pairs[t]
    o = T.off_L[t]
    return theta[o:o + T.d[i] * k].reshape(T.d[i], k)


def R_block(T: Tiling, theta: np.ndarray, t: int) -> np.ndarray:
    i, j, k = T.pairs[t]
    o = T.off_R[t]
    return theta[o:o + k * T.d[j]].reshape(k, T.d[j])


def _sl(T: Tiling, i: int) -> slice:
    return slice(T.start[i], T.start[i] + T.d[i])


# ============================================================================
# Assembly X = C(Zbar, Lbar, Rbar) (ADMM solver section, first equation)
# ============================================================================
def assemble(T: Tiling, theta: np.ndarray) -> np.ndarray:
    """Dense symmetric X from the tile factors."""
    X = np.zeros((T.nr, T.nr), dtype=np.complex128)
    for i in range(T.n):
        B = diag_block(T, theta, i)
        if T.kdiag[i] < 0:
            X[_sl(T, i), _sl(T, i)] = 0.5 * (B + B.T)        # X_ii = P Z_ii
        else:
            X[_sl(T, i), _sl(T, i)] = B @ B.T                # X_ii = Q Q^T
    for t, (i, j, k) in enumerate(T.pairs):
        Xij = L_block(T, theta, t) @ R_block(T, theta, t)    # X_ij = L R
        X[_sl(T, i), _sl(T, j)] = Xij
        X[_sl(T, j), _sl(T, i)] = Xij.T                      # X_ji = X_ij^T
    return X


def assemble_directional(T: Tiling, theta: np.ndarray, p: np.ndarray):
    """C(theta + alpha p) = C(theta) + alpha X1 + alpha^2 X2; returns (X1, X2).

    The assembly map is quadratic in the factors, so each tile expands exactly:
    L R -> (P_L R + L P_R), P_L P_R ; Q Q^T -> (P Q^T + Q P^T), P P^T ;
    (Z + Z^T)/2 -> (P + P^T)/2, 0.
    """
    X1 = np.zeros((T.nr, T.nr), dtype=np.complex128)
    X2 = np.zeros((T.nr, T.nr), dtype=np.complex128)
    for i in range(T.n):
        B = diag_block(T, theta, i)
        P = diag_block(T, p, i)
        s = _sl(T, i)
        if T.kdiag[i] < 0:
            X1[s, s] = 0.5 * (P + P.T)
        else:
            X1[s, s] = P @ B.T + B @ P.T
            X2[s, s] = P @ P.T
    for t, (i, j, k) in enumerate(T.pairs):
        L, R = L_block(T, theta, t), R_block(T, theta, t)
        PL, PR = L_block(T, p, t), R_block(T, p, t)
        A1 = PL @ R + L @ PR
        A2 = PL @ PR
        X1[_sl(T, i), _sl(T, j)] = A1
        X1[_sl(T, j), _sl(T, i)] = A1.T
        X2[_sl(T, i), _sl(T, j)] = A2
        X2[_sl(T, j), _sl(T, i)] = A2.T
    return X1, X2


# ============================================================================
# Objective and gradient (eq. X2LQR_lst and eqs. DXLR)
# ============================================================================
def residual(D: np.ndarray, X: np.ndarray, U: np.ndarray) -> np.ndarray:
    return D @ X - U


def objective(T: Tiling, D, U, theta) -> Tuple[float, np.ndarray]:
    """f = 1/2 ||D C(theta) - U||_F^2 and the residual r."""
    r = residual(D, assemble(T, theta), U)
    return 0.5 * float(np.vdot(r, r).real), r


def tile_gradient(T: Tiling, theta: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Gradient of f w.r.t. every factor given W = D^H r, packed like theta."""
    Wp = W + W.T                                            # W' = W + W^T
    g = np.zeros_like(theta, dtype=np.complex128)
    for i in range(T.n):
        s = _sl(T, i)
        G = diag_block(T, g, i)
        if T.kdiag[i] < 0:
            G[...] = 0.5 * Wp[s, s]                         # grad Z = W'_ii / 2
        else:
            G[...] = Wp[s, s] @ np.conj(diag_block(T, theta, i))   # grad Q = W' conj(Q)
    for t, (i, j, k) in enumerate(T.pairs):
        Wij = Wp[_sl(T, i), _sl(T, j)]
        L_block(T, g, t)[...] = Wij @ R_block(T, theta, t).conj().T   # W' R^H
        R_block(T, g, t)[...] = L_block(T, theta, t).conj().T @ Wij   # L^H W'
    return g


def gradient(T: Tiling, D, U, theta) -> Tuple[float, np.ndarray]:
    """(f, grad f) with grad = df/dRe + i df/dIm of every packed factor."""
    f, r = objective(T, D, U, theta)
    W = D.conj().T @ r
    return f, tile_gradient(T, theta, W)


def factor_of_entry(T: Tiling, q: int):
    """Locate packed entry q: (kind, tile index, row, col) with kind in
    {'Q', 'Z', 'L', 'R'} and (row, col) inside that factor."""
    for i in range(T.n):
        cols = T.d[i] if T.kdiag[i] < 0 else T.kdiag[i]
        o = T.off_diag[i]
        if o <= q < o + T.d[i] * cols:
            return ("Z" if T.kdiag[i] < 0 else "Q", i, (q - o) // cols, (q - o) % cols)
    for t, (i, j, k) in enumerate(T.pairs):
        o = T.off_L[t]
        if o <= q < o + T.d[i] * k:
            return ("L", t, (q - o) // k, (q - o) % k)
        o = T.off_R[t]
        if o <= q < o + k * T.d[j]:
            return ("R", t, (q - o) // T.d[j], (q - o) % T.d[j])
    raise IndexError(q)


def gradient_entries(T: Tiling, D: np.ndarray, r: np.ndarray, theta: np.ndarray, idx) -> np.ndarray:
    """Selected entries of the tile gradient, each from its definition
    (gradient equations DXLR) with only the entries of W = D^H r it needs:
    W'[p, q] = W[p, q] + W[q, p] and W[p, q] = conj(D[:, p]) . r[:, q]."""
    def Wblock(rows, cols):
        return D[:, rows].conj().T @ r[:, cols]

    out = np.zeros(len(idx), dtype=np.complex128)
    for n, q in enumerate(idx):
        kind, tix, a, b = factor_of_entry(T, int(q))
        if kind in ("Q", "Z"):
            rows = np.arange(T.start[tix], T.start[tix] + T.d[tix])
            p = T.start[tix] + a
            wrow = Wblock([p], rows)[0] + Wblock(rows, [p])[:, 0]     # W'[p, tile cols]
            if kind == "Z":
                c = T.start[tix] + b
                out[n] = 0.5 * (Wblock([p], [c])[0, 0] + Wblock([c], [p])[0, 0])
            else:
                Q = diag_block(T, theta, tix)
                out[n] = np.sum(wrow * np.conj(Q[:, b]))              # (W' conj(Q))[a, b]
        else:
            i, j, k = T.pairs[tix]
            ri = np.arange(T.start[i], T.start[i] + T.d[i])
            cj = np.arange(T.start[j], T.start[j] + T.d[j])
            if kind == "L":
                p = T.start[i] + a
                wrow = Wblock([p], cj)[0] + Wblock(cj, [p])[:, 0]      # W'_ij[a, :]
                out[n] = np.sum(wrow * np.conj(R_block(T, theta, tix)[b, :]))   # (W' R^H)[a, b]
            else:
                c = T.start[j] + b
                wcol = Wblock(ri, [c])[:, 0] + Wblock([c], ri)[0]      # W'_ij[:, b]
                out[n] = np.sum(np.conj(L_block(T, theta, tix)[:, a]) * wcol)   # (L^H W')[a, b]
    return out


def fd_entries_large(T: Tiling, D, U, theta, idx, h: float = 1e-6) -> np.ndarray:
    """Central differences of f along Re and Im of theta[idx] without forming
    D X for every shifted theta: r(theta') = r + D (C(theta') - C(theta)), where
    the difference is nonzero only in the rows/columns of the perturbed tiles
    (D times the rows of the difference that are nonzero)."""
    X = assemble(T, theta)
    r = D @ X - U

    def f_shift(e):
        dX = assemble(T, theta + e) - X
        nz = np.flatnonzero(np.any(dX != 0, axis=1))
        rr = r + D[:, nz] @ dX[nz, :]
        return 0.5 * float(np.vdot(rr, rr).real)

    out = np.zeros(len(idx), dtype=np.complex128)
    for n, q in enumerate(idx):
        e = np.zeros_like(theta)
        e[q] = h
        fr = (f_shift(e) - f_shift(-e)) / (2 * h)
        fi = (f_shift(1j * e) - f_shift(-1j * e)) / (2 * h)
        out[n] = fr + 1j * fi
    return out


def fd_gradient_entries(T: Tiling, D, U, theta, idx, h: float = 1e-6) -> np.ndarray:
    """Central differences of f along Re and Im of theta[idx] (complex128)."""
    out = np.zeros(len(idx), dtype=np.complex128)
    for n, q in enumerate(idx):
        e = np.zeros_like(theta)
        e[q] = h
        fr = (objective(T, D, U, theta + e)[0] - objective(T, D, U, theta - e)[0]) / (2 * h)
        fi = (objective(T, D, U, theta + 1j * e)[0] - objective(T, D, U, theta - 1j * e)[0]) / (2 * h)
        out[n] = fr + 1j * fi
    return out


def re_dot(a: np.ndarray, b: np.ndarray) -> float:
    """Real inner product Re sum conj(a) b (C^n viewed as R^2n)."""
    return float(np.vdot(a, b).real)


# ============================================================================
# Exact line search along the quartic  phi(alpha) = f(theta + alpha p)
# ============================================================================
def line_coefficients(r, a, b, theta=None, p=None, lam: float = 0.0, center=None):
    """phi'(alpha) = c0 + c1 alpha + c2 alpha^2 + c3 alpha^3 where
    phi(alpha) = 1/2 ||r + alpha a + alpha^2 b||^2 + lam ||theta + alpha p - center||^2
    (center = 0 unless given)."""
    c0 = re_dot(r, a)
    c1 = re_dot(a, a) + 2.0 * re_dot(r, b)
    c2 = 3.0 * re_dot(a, b)
    c3 = 2.0 * re_dot(b, b)
    if lam != 0.0:
        d = theta if center is None else theta - center
        c0 += 2.0 * lam * re_dot(d, p)
        c1 += 2.0 * lam * re_dot(p, p)
    return np.array([c0, c1, c2, c3], dtype=np.float64)


def phi_increment(c: np.ndarray, alpha: float) -> float:
    """phi(alpha) - phi(0) = c0 a + c1 a^2/2 + c2 a^3/3 + c3 a^4/4."""
    return c[0] * alpha + c[1] * alpha ** 2 / 2 + c[2] * alpha ** 3 / 3 + c[3] * alpha ** 4 / 4


def exact_step(c: np.ndarray) -> float:
    """Minimiser over alpha > 0 of the quartic phi whose derivative has coefficients c.

    Candidates are the positive real roots of phi' (numpy.roots on the
    companion matrix, each polished by Newton steps); the one with the lowest
    phi wins, ties to the smaller alpha. Returns 0 when no positive root exists.
    """
    c0, c1, c2, c3 = (float(v) for v in c)
    poly = np.array([c3, c2, c1, c0])
    nz = np.flatnonzero(np.abs(poly) > 0)
    if nz.size == 0:
        return 0.0
    poly = poly[nz[0]:]
    if poly.size < 2:
        return 0.0
    roots = np.roots(poly)
    cands = []
    for z in roots:
        if abs(z.imag) > 1e-6 * (1.0 + abs(z.real)):
            continue
        x = float(z.real)
        for _ in range(4):   # Newton polish on phi'
            fp = ((c3 * x + c2) * x + c1) * x + c0
            fpp = (3 * c3 * x + 2 * c2) * x + c1
            if fpp == 0:
                break
            x -= fp / fpp
        if x > 0 and np.isfinite(x):
            cands.append(x)
    if not cands:
        return 0.0
    best = None
    for x in sorted(cands):
        v = phi_increment(c, x)
        if best is None or v < best[0]:
            best = (v, x)
    return best[1]


# ============================================================================
# L-BFGS direction (two-loop recursion, Liu & Nocedal 1989)
# ============================================================================
def lbfgs_direction(g: np.ndarray, S: List[np.ndarray], Y: List[np.ndarray]) -> np.ndarray:
    """p = -H g from the stored pairs (oldest first in S, Y)."""
    q = g.copy()
    alphas = []
    for s, y in zip(reversed(S), reversed(Y)):
        rho = 1.0 / re_dot(y, s)
        al = rho * re_dot(s, q)
        q = q - al * y
        alphas.append(al)
    if S:
        gamma = re_dot(S[-1], Y[-1]) / re_dot(Y[-1], Y[-1])
    else:
        gamma = 1.0
    z = gamma * q
    for (s, y), al in zip(zip(S, Y), reversed(alphas)):
        rho = 1.0 / re_dot(y, s)
        beta = rho * re_dot(y, z)
        z = z + (al - beta) * s
    return -z


@dataclasses.dataclass
class SolveResult:
    theta: np.ndarray
    f_hist: np.ndarray      # f_hist[t] = objective tracked after t iterations
    alphas: np.ndarray      # step length of every iteration
    restarts: int


def solve(T: Tiling, D, U, theta0, iters: int, m: int = 5, optimizer: str = "lbfgs",
          lam: float = 0.0, record=None, center=None) -> SolveResult:
    """Fixed-count L-BFGS (or steepest descent) on f (+ lam ||theta - center||^2).

    Per iteration: gradient from the tracked residual r; direction; exact
    line search with a = D X1, b = D X2; theta += alpha p; r += alpha a +
    alpha^2 b. ``record(t, state)`` (optional) sees every iteration's state.
    ``center`` (default 0) is the point the Frobenius penalty pulls towards:
    0 for the plain regulariser, z - u in the ADMM X-update.
    """
    theta = np.array(theta0, dtype=np.complex128, copy=True)
    r = residual(D, assemble(T, theta), U)
    DH = D.conj().T
    cen = np.zeros_like(theta) if center is None else np.asarray(center, dtype=np.complex128)

    def fval(rr, th):
        v = 0.5 * re_dot(rr, rr)
        if lam != 0.0:
            v += lam * re_dot(th - cen, th - cen)
        return v

    f_hist = [fval(r, theta)]
    S: List[np.ndarray] = []
    Y: List[np.ndarray] = []
    alphas = []
    restarts = 0
    g_prev = None
    s_prev = None
    for t in range(iters):
        g = tile_gradient(T, theta, DH @ r)
        if lam != 0.0:
            g = g + 2.0 * lam * (theta - cen)
        if g_prev is not None and s_prev is not None:
            y = g - g_prev
            if re_dot(s_prev, y) > 0.0:
                S.append(s_prev)
                Y.append(y)
                if len(S) > m:
                    S.pop(0)
                    Y.pop(0)
        if optimizer == "gd":
            p = -g
        else:
            p = lbfgs_direction(g, S, Y)
            if re_dot(g, p) >= 0.0:
                p = -g
                S.clear()
                Y.clear()
                restarts += 1
        X1, X2 = assemble_directional(T, theta, p)
        a = D @ X1
        b = D @ X2
        c = line_coefficients(r, a, b, theta, p, lam, cen)
        alpha = exact_step(c)
        if record is not None:
            record(t, dict(theta=theta.copy(), r=r.copy(), g=g.copy(), p=p.copy(),
                           a=a, b=b, coeffs=c, alpha=alpha))
        theta = theta + alpha * p
        r = r + alpha * a + alpha * alpha * b
        s_prev = alpha * p
        g_prev = g
        alphas.append(alpha)
        f_hist.append(fval(r, theta))
    return SolveResult(theta, np.array(f_hist), np.array(alphas), restarts)


# ============================================================================
# ADMM with lambda continuation (ADMM solver section; hyper-parameter selection)
# ============================================================================
@dataclasses.dataclass
class AdmmResult:
    theta: np.ndarray       # the X-variable (the returned solution)
    z: np.ndarray           # the split variable after the last Z-update
    u: np.ndarray           # scaled dual after the last update
    f_hist: np.ndarray      # data misfit 1/2||D C(theta) - U||^2: start, then after every X-update
    stage_end: List[int]    # index into f_hist of the last X-update of each lambda stage


def admm(T: Tiling, D, U, theta0, lams=(10.0, 1.0, 0.1), outer: int = 5, inner: int = 10,
         rho: float = 1.0, m: int = 5, record=None) -> AdmmResult:
    """Scaled ADMM on min_theta f(theta) + lam ||theta||_F^2 with the split theta = z.

    For every lam of the continuation (each stage warm-started from the last)
    and `outer` times:
      X-update  theta <- argmin f(theta) + rho/2 ||theta - z + u||^2, by `inner`
                L-BFGS iterations from the current theta (fresh pair memory);
      Z-update  z <- (theta + u) / (1 + 2 lam / rho), the proximal point of
                lam ||.||^2 (closed form of the Frobenius prox);
      dual      u <- u + theta - z.
    Starts from z = theta0, u = 0.
    """
    theta = np.array(theta0, dtype=np.complex128, copy=True)
    z = theta.copy()
    u = np.zeros_like(theta)
    f_hist = [0.5 * float(np.linalg.norm(residual(D, assemble(T, theta), U)) ** 2)]
    stage_end = []
    for lam in lams:
        for k in range(outer):
            res = solve(T, D, U, theta, inner, m=m, lam=rho / 2.0, center=z - u)
            theta = res.theta
            z = (theta + u) / (1.0 + 2.0 * lam / rho)
            u = u + theta - z
            f_hist.append(0.5 * float(np.linalg.norm(residual(D, assemble(T, theta), U)) ** 2))
            if record is not None:
                record(lam, k, dict(theta=theta.copy(), z=z.copy(), u=u.copy()))
        stage_end.append(len(f_hist) - 1)
    return AdmmResult(theta, z, u, np.array(f_hist), stage_end)


# ============================================================================
# Rank / tile-size estimate and warm start (Hyper-parameter selection and
# initialization; the examples' entry-count study)
# ============================================================================
def split_sizes(nr: int, d: int) -> List[int]:
    """Tiles of size d covering nr receivers, the last one ragged when d does not divide nr."""
    sizes = [d] * (nr // d)
    if nr % d:
        sizes.append(nr % d)
    return sizes


def tile_ranks(X: np.ndarray, d: int, eps: float = 0.01):
    """Numerical ranks of the tiles of a symmetric X at tile size d.

    Every tile (i, j), i >= j, is decomposed by SVD; v0 is the largest singular
    value over all of them and a tile's rank is the number of its singular
    values >= eps v0 (0 possible; all of them = numerically full rank).
    Returns (sizes, k_off in t order, k_diag, v0)."""
    nr = X.shape[0]
    sizes = split_sizes(nr, d)
    start = np.concatenate([[0], np.cumsum(sizes)])
    sv = {}
    for i in range(len(sizes)):
        for j in range(i + 1):
            blk = X[start[i]:start[i + 1], start[j]:start[j + 1]]
            sv[(i, j)] = np.linalg.svd(blk, compute_uv=False)
    v0 = max(float(v[0]) for v in sv.values())
    k_off = [int(np.count_nonzero(sv[(i, j)] >= eps * v0)) for i in range(len(sizes)) for j in range(i)]
    k_diag = [int(np.count_nonzero(sv[(i, i)] >= eps * v0)) for i in range(len(sizes))]
    return sizes, k_off, k_diag, v0


def layout_from_ranks(sizes, k_off, k_diag):
    """Layout of the estimate: ranks of at least 1; a diagonal tile is dense when its rank is at
    least half its size (the symmetric part of a dense Z_ii then has no more degrees of freedom,
    d(d+1)/2, than Q_ii's d k), else Q Q^T.
    Returns (rank_off, rank_diag, entries), entries = complex unknowns of the layout."""
    rank_off = [max(1, int(k)) for k in k_off]
    rank_diag = [(-1 if k >= (sizes[i] + 1) // 2 else max(1, int(k))) for i, k in enumerate(k_diag)]
    entries = 0
    t = 0
    for i in range(len(sizes)):
        for j in range(i):
            entries += rank_off[t] * (sizes[i] + sizes[j])
            t += 1
        entries += sizes[i] * (sizes[i] if rank_diag[i] < 0 else rank_diag[i])
    return rank_off, rank_diag, entries


def choose_layout(X: np.ndarray, candidates, eps: float = 0.01):
    """The candidate tile size whose estimated layout has the fewest entries (first on ties).
    Returns (d, sizes, rank_off, rank_diag, entries_per_candidate)."""
    best = None
    entries = []
    for d in candidates:
        sizes, k_off, k_diag, _ = tile_ranks(X, int(d), eps)
        ro, rd, n = layout_from_ranks(sizes, k_off, k_diag)
        entries.append(n)
        if best is None or n < best[0]:
            best = (n, int(d), sizes, ro, rd)
    return best[1], best[2], best[3], best[4], entries


def takagi(Xs: np.ndarray, k: int) -> np.ndarray:
    """Q (n x k) with Q Q^T the rank-k Takagi truncation of a complex symmetric Xs.

    From the SVD Xs = U S V^H and symmetry, conj(V) = U D with D diagonal unitary
    (distinct singular values), so Xs = U S D U^T = W S W^T with W = U D^(1/2):
    Q = U_k D_k^(1/2) S_k^(1/2)."""
    U, S, Vh = np.linalg.svd(Xs)
    V = Vh.conj().T
    dph = np.einsum("ij,ij->j", U.conj(), V.conj())[:k]     # d_i = U_i^H conj(V_i)
    dph = dph / np.abs(dph)
    return U[:, :k] * (np.sqrt(dph) * np.sqrt(S[:k]))[None, :]


def warm_start(T: Tiling, X: np.ndarray) -> np.ndarray:
    """theta from a reference solution X tiled by T (Hyper-parameter selection and initialization):
    off-diagonal L = U_k S_k^(1/2), R = S_k^(1/2) V_k^H from the SVD of X_ij; diagonal
    Q_ii by the Takagi factorisation truncated to k_ii, or Z_ii = X_ii when dense."""
    theta = np.zeros(T.size, dtype=np.complex128)
    for i in range(T.n):
        blk = X[_sl(T, i), _sl(T, i)]
        if T.kdiag[i] < 0:
            theta[T.off_diag[i]:T.off_diag[i] + blk.size] = blk.ravel()
        else:
            k = T.kdiag[i]
            theta[T.off_diag[i]:T.off_diag[i] + T.d[i] * k] = takagi(blk, k).ravel()
    for t, (i, j, k) in enumerate(T.pairs):
        U, S, Vh = np.linalg.svd(X[_sl(T, i), _sl(T, j)])
        L = U[:, :k] * np.sqrt(S[:k])[None, :]
        R = np.sqrt(S[:k])[:, None] * Vh[:k, :]
        theta[T.off_L[t]:T.off_L[t] + L.size] = L.ravel()
        theta[T.off_R[t]:T.off_R[t] + R.size] = R.ravel()
    return theta


# ============================================================================
# Precision diagnostics
# ============================================================================
def predicted_objective_floor(D, X, r, unit_roundoff: float) -> float:
    """Expected relative error of f from rounding the products D X in a format
    with the given unit roundoff: about 2 sqrt(nr) u || |D||X| ||_F / ||r||_F."""
    nr = X.shape[0]
    num = np.linalg.norm(np.abs(D) @ np.abs(X))
    den = max(np.linalg.norm(r), 1e-300)
    return float(2.0 * np.sqrt(nr) * unit_roundoff * num / den)
