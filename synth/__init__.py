"""Seeded synthetic inputs for tile low-rank MDD (TLR-MDD).

This module produces *inputs only*: acquisition geometry, the down-going
wavefield D, the up-going wavefield U, a reference Green's function X_true,
tile layouts (tile sizes and ranks) and initial tile factors. It holds none of
the method's arithmetic (no tile assembly, objective, gradient, Hilbert
ordering or optimiser); both the FP64 CPU oracle and the GPU path consume what
it returns.

Stand-in for the paper's data (Numerical Examples, 3D survey setup): the paper
uses finite-difference data on the 3D Overthrust model, which is not available.
Here the wavefields are homogeneous-medium Green's functions on the same 20 m
receiver grids (scaled down), which give the value structure the method relies
on: smooth oscillatory kernels whose far-field tiles are numerically low rank
and a dominant diagonal once receivers are Hilbert ordered.

Recipe (all values float64 / complex128):
  * receivers: nx x ny grid, 20 m spacing, z = 0; natural index iy*nx + ix.
  * sources: same footprint, 40 m above the receivers; either the receiver
    grid itself (ns = nr) or every other line (ns = nr/2, 20 m x 40 m).
  * D_clean[s, r] = exp(-i w d_sr / c) / d_sr with c = 2000 m/s (d_sr >= 40 m).
  * X_true[a, b] = exp(-i w d_ab / c) / (d_ab + 10 m)  (exactly symmetric).
  * U = D_clean @ X_true + n_U, with n_U complex Gaussian rescaled so that
    ||D_clean X_true||^2 / ||n_U||^2 = 10^(SNR/10) exactly.
  * D = D_clean + n_D, ||n_D||_F = 0.05 ||D_clean||_F exactly.
  * both divided by alpha = max |D_clean| over all frequencies and entries
    (= 1 / min d_sr; the Green's function modulus does not depend on w).
  * initial factors: CN(0, 1e-2), i.e. Re and Im each N(0, 0.005).
Seeds: numpy SeedSequence(14973, spawn_key=(config, item, purpose)).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 14973
SPACING = 20.0          # receiver / source spacing in metres
SOURCE_HEIGHT = 40.0    # sources sit this far above the receiver datum
VELOCITY = 2000.0       # m/s
X_TRUE_OFFSET = 10.0    # metres added to the distance in X_true's denominator

# purpose codes for seed derivation
P_NOISE_D, P_NOISE_U, P_THETA, P_REQUEST, P_DIR = 1, 2, 3, 4, 5


def rng_for(config_id: int, item: int, purpose: int) -> np.random.Generator:
    """Independent, reproducible stream for (config, frequency/request, purpose)."""
    ss = np.random.SeedSequence(BASE_SEED, spawn_key=(int(config_id), int(item), int(purpose)))
    return np.random.default_rng(ss)


# ----------------------------------------------------------------------------
# layouts (plain data: tile sizes and ranks)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Layout:
    """Tile partition of the nr x nr Green's function.

    tile_size[i]  d_i, sum(d_i) = nr (a ragged last tile is allowed)
    rank_off[t]   k for sub-diagonal tile (i, j), i > j, t = i(i-1)/2 + j
    rank_diag[i]  k_ii >= 1 -> Q_ii Q_ii^T ;  -1 -> dense symmetrised Z_ii
    """
    tile_size: np.ndarray
    rank_off: np.ndarray
    rank_diag: np.ndarray

    def __post_init__(self):
        self.tile_size = np.ascontiguousarray(self.tile_size, dtype=np.int32)
        self.rank_off = np.ascontiguousarray(self.rank_off, dtype=np.int32)
        self.rank_diag = np.ascontiguousarray(self.rank_diag, dtype=np.int32)

    @property
    def ntiles(self) -> int:
        return int(self.tile_size.shape[0])

    @property
    def nr(self) -> int:
        return int(self.tile_size.sum())


def split_tiles(nr: int, d: int) -> np.ndarray:
    """Equal tiles of size d, the last one ragged when d does not divide nr."""
    n = -(-nr // d)
    sizes = np.full(n, d, dtype=np.int32)
    sizes[-1] = nr - d * (n - 1)
    return sizes


def uniform_layout(nr: int, d: int, k_off: int, k_diag: int) -> Layout:
    """Uniform tiles; k_diag = -1 gives dense diagonal tiles.

    Ranks are clipped to the tile sizes (a ragged last tile may be smaller).
    """
    sizes = split_tiles(nr, d)
    n = sizes.shape[0]
    ro = []
    for i in range(n):
        for j in range(i):
            ro.append(min(k_off, int(sizes[i]), int(sizes[j])))
    rd = [(-1 if k_diag < 0 else min(k_diag, int(sizes[i]))) for i in range(n)]
    return Layout(sizes, np.array(ro, dtype=np.int32), np.array(rd, dtype=np.int32))


def adaptive_layout(nr: int, k: int) -> Layout:
    """Batched-frequency tile rule: rank k -> tile 256 (k<=16), 128 (k<=32), else 64.

    Diagonal tiles are dense when k >= d/2, else Q Q^T of rank k.
    """
    d = 256 if k <= 16 else (128 if k <= 32 else 64)
    kd = -1 if k >= d // 2 else k
    return uniform_layout(nr, d, k, kd)


# ----------------------------------------------------------------------------
# geometry and wavefields
# ----------------------------------------------------------------------------
def grid(nx: int, ny: int, dx: float = SPACING, dy: float = SPACING, z: float = 0.0):
    """Points of an nx x ny grid, natural order idx = iy*nx + ix."""
    iy, ix = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    ix = ix.ravel().astype(np.int32)
    iy = iy.ravel().astype(np.int32)
    xyz = np.stack([ix * dx, iy * dy, np.full(ix.shape, z)], axis=1).astype(np.float64)
    return xyz, ix, iy


@dataclasses.dataclass
class Geometry:
    rec_xyz: np.ndarray
    rec_ix: np.ndarray
    rec_iy: np.ndarray
    src_xyz: np.ndarray

    @property
    def nr(self):
        return self.rec_xyz.shape[0]

    @property
    def ns(self):
        return self.src_xyz.shape[0]


def make_geometry(nx: int, ny: int, ns_mode: str = "full") -> Geometry:
    """ns_mode 'full': sources on the receiver grid; 'half': every other line (40 m)."""
    rec, ix, iy = grid(nx, ny)
    if ns_mode == "full":
        src, _, _ = grid(nx, ny, z=-SOURCE_HEIGHT)
    elif ns_mode == "half":
        src, _, _ = grid(nx, ny // 2, dx=SPACING, dy=2 * SPACING, z=-SOURCE_HEIGHT)
    else:
        raise ValueError(ns_mode)
    return Geometry(rec, ix, iy, src)


def _dist(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    d = a[:, None, :] - b[None, :, :]
    return np.sqrt(np.einsum("ijk,ijk->ij", d, d))


def normalisation(geom: Geometry) -> float:
    """alpha = max |D_clean| over all entries and frequencies = 1 / min distance."""
    return 1.0 / float(_dist(geom.src_xyz, geom.rec_xyz).min())


def _cgauss(rng: np.random.Generator, shape) -> np.ndarray:
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@dataclasses.dataclass
class Problem:
    """One frequency slice, natural receiver order, normalised."""
    D: np.ndarray        # ns x nr complex128 (noisy, what the solver sees)
    U: np.ndarray        # ns x nr complex128
    X_true: np.ndarray   # nr x nr complex128 (symmetric)
    freq: float
    geom: Geometry


def make_problem(geom: Geometry, freq: float, snr_db: Optional[float], d_noise: float,
                 config_id: int, item: int, alpha: Optional[float] = None) -> Problem:
    """D, U, X_true at one frequency (Hz); snr_db=None means noise-free U."""
    w = 2.0 * math.pi * freq
    dsr = _dist(geom.src_xyz, geom.rec_xyz)
    D_clean = np.exp(-1j * w * dsr / VELOCITY) / dsr
    drr = _dist(geom.rec_xyz, geom.rec_xyz)
    X_true = np.exp(-1j * w * drr / VELOCITY) / (drr + X_TRUE_OFFSET)
    X_true = 0.5 * (X_true + X_true.T)  # exact symmetry regardless of rounding in _dist
    U_clean = D_clean @ X_true
    U = U_clean
    if snr_db is not None:
        n_u = _cgauss(rng_for(config_id, item, P_NOISE_U), U.shape)
        scale = np.linalg.norm(U_clean) / (np.linalg.norm(n_u) * 10.0 ** (snr_db / 20.0))
        U = U_clean + scale * n_u
    D = D_clean
    if d_noise > 0:
        n_d = _cgauss(rng_for(config_id, item, P_NOISE_D), D.shape)
        D = D_clean + n_d * (d_noise * np.linalg.norm(D_clean) / np.linalg.norm(n_d))
    if alpha is None:
        alpha = normalisation(geom)
    return Problem(D / alpha, U / alpha, X_true, freq, geom)


def clean_problem_from_factors(D: np.ndarray, X: np.ndarray) -> np.ndarray:
    """U = D X for the zero-residual tests (X given explicitly by the caller)."""
    return D @ X


def init_theta(n: int, config_id: int, item: int, var: float = 1e-2,
               purpose: int = P_THETA) -> np.ndarray:
    """CN(0, var) complex vector of length n."""
    rng = rng_for(config_id, item, purpose)
    s = math.sqrt(var / 2.0)
    return s * rng.standard_normal(n) + 1j * s * rng.standard_normal(n)


def theta_length(layout: Layout) -> int:
    """Number of complex unknowns of a layout (a count, not arithmetic of the method)."""
    ts = layout.tile_size.astype(np.int64)
    n = 0
    for i in range(layout.ntiles):
        kd = int(layout.rank_diag[i])
        n += ts[i] * (ts[i] if kd < 0 else kd)
    t = 0
    for i in range(layout.ntiles):
        for j in range(i):
            k = int(layout.rank_off[t])
            n += ts[i] * k + k * ts[j]
            t += 1
    return int(n)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    name: str
    config_id: int
    nx: int
    ny: int
    ns_mode: str
    freqs: np.ndarray
    snr_db: Optional[float]
    d_noise: float
    iters: int

    def geometry(self) -> Geometry:
        return make_geometry(self.nx, self.ny, self.ns_mode)

    def layout(self, f_idx: int) -> Layout:
        raise NotImplementedError

    def problem(self, f_idx: int, geom: Optional[Geometry] = None) -> Problem:
        geom = geom or self.geometry()
        return make_problem(geom, float(self.freqs[f_idx]), self.snr_db, self.d_noise,
                            self.config_id, f_idx)

    def theta0(self, f_idx: int, layout: Optional[Layout] = None) -> np.ndarray:
        layout = layout or self.layout(f_idx)
        return init_theta(theta_length(layout), self.config_id, f_idx)


class SmallWorkload(Workload):
    """8x8 receivers, 64 sources, 8 frequencies 5-30 Hz, tile 16, k_off 4, QQ^T k 8."""
    def layout(self, f_idx):
        return uniform_layout(64, 16, 4, 8)


def small() -> SmallWorkload:
    return SmallWorkload("nr64_ns64_d16_k4_8freq", 1, 8, 8, "full",
                         np.linspace(5.0, 30.0, 8), 20.0, 0.05, 50)


def batched_rank(freq: float) -> int:
    return int(round(4 + 44 * (freq - 2.0) / 38.0))


class BatchedWorkload(Workload):
    """32x32 receivers, ns = nr = 1024, 64 frequencies 2-40 Hz, rank ramps 4..48."""
    def layout(self, f_idx):
        return adaptive_layout(1024, batched_rank(float(self.freqs[f_idx])))


def batched() -> BatchedWorkload:
    return BatchedWorkload("nr1024_ns1024_64freq_adaptive", 2, 32, 32, "full",
                           np.linspace(2.0, 40.0, 64), 20.0, 0.05, 100)


class LargeWorkload(Workload):
    """64x64 receivers (nr 4096), 2048 sources, 32 frequencies 5-35 Hz, tile 256, k 32."""
    def layout(self, f_idx):
        return uniform_layout(4096, 256, 32, 32)


def large(snr_db: float = 20.0, config_id: int = 3) -> LargeWorkload:
    return LargeWorkload("nr4096_ns2048_d256_k32_32freq", config_id, 64, 64, "half",
                         np.linspace(5.0, 35.0, 32), snr_db, 0.05, 100)


# ----------------------------------------------------------------------------
# serving stream
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    rid: int
    arrival: float       # seconds since stream start
    n_side: int          # receivers on an n_side x n_side grid
    ns_mode: str
    d: int
    k: int
    freq: float
    iters: int


def request_stream(n_requests: int, rate: float = 200.0, config_id: int = 5,
                   sides: Sequence[int] = (32, 48, 64, 96),
                   tiles: Sequence[int] = (128, 256, 512), kmin: int = 8, kmax: int = 64,
                   fmin: float = 5.0, fmax: float = 35.0, iters: int = 100) -> List[Request]:
    """Poisson arrivals of per-frequency solve requests with random shapes."""
    rng = rng_for(config_id, 0, P_REQUEST)
    t = 0.0
    out = []
    for rid in range(n_requests):
        t += float(rng.exponential(1.0 / rate))
        side = int(rng.choice(np.asarray(sides)))
        mode = "half" if rng.integers(2) == 0 else "full"
        d = int(rng.choice(np.asarray(tiles)))
        k = int(rng.integers(kmin, kmax + 1))
        f = float(rng.uniform(fmin, fmax))
        out.append(Request(rid, t, side, mode, d, k, f, iters))
    return out


def request_layout(req: Request) -> Layout:
    nr = req.n_side * req.n_side
    kd = -1 if req.k >= req.d // 2 else req.k
    return uniform_layout(nr, req.d, req.k, kd)


def request_problem(req: Request, config_id: int = 5) -> Tuple[Problem, Layout, np.ndarray]:
    geom = make_geometry(req.n_side, req.n_side, req.ns_mode)
    prob = make_problem(geom, req.freq, 20.0, 0.05, config_id, 1000 + req.rid)
    lay = request_layout(req)
    th = init_theta(theta_length(lay), config_id, 1000 + req.rid)
    return prob, lay, th


# ----------------------------------------------------------------------------
# device-side generation (same recipe, torch on the GPU) for large request sizes
# ----------------------------------------------------------------------------
def device_problem(req: Request, device, config_id: int = 5):
    """(D, U, theta0, layout, geometry) of a request, generated on `device` (see device_generate)."""
    geom = make_geometry(req.n_side, req.n_side, req.ns_mode)
    lay = request_layout(req)
    D, U, th = device_generate(geom, req.freq, 20.0, lay, config_id, 1000 + req.rid, device)
    return D, U, th, lay, geom


def device_generate_bytes(ns: int, nr: int) -> int:
    """Upper estimate of the device memory device_generate holds at its peak beyond the permuted
    complex64 D and U a caller keeps: distances, fields, noise and their temporaries (complex64),
    and the natural-order outputs."""
    return 64 * ns * nr + 28 * nr * nr


def device_workload_problem(wl: Workload, f_idx: int, device):
    """(D, U, theta0) of frequency f_idx of a workload, generated on `device` (see device_generate);
    the values differ from Workload.problem's (another generator) but follow the same recipe."""
    return device_generate(wl.geometry(), float(wl.freqs[f_idx]), wl.snr_db, wl.layout(f_idx), wl.config_id,
                           f_idx, device)


def device_generate(geom: Geometry, freq: float, snr_db: float, lay: Layout, config_id: int, item: int, device):
    """(D, U, theta0) generated on `device`.

    Same recipe as make_problem (homogeneous Green's functions, exact-SNR noise
    on U, 5 % noise on D, normalisation by 1/min distance), computed in
    complex64 with torch's device generator seeded from (config, item), in
    natural receiver order. Everything stays on the device and is queued on the
    current stream (no host synchronisation), so a server can make a request's
    inputs when it admits the request without stalling its loop.
    """
    import torch
    seed = int(np.random.SeedSequence(BASE_SEED, spawn_key=(config_id, item, P_REQUEST))
               .generate_state(1)[0])
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    rec = torch.as_tensor(geom.rec_xyz, device=device, dtype=torch.float32)
    src = torch.as_tensor(geom.src_xyz, device=device, dtype=torch.float32)
    k = 2.0 * math.pi * freq / VELOCITY
    dsr = torch.cdist(src, rec)
    D_clean = torch.polar(1.0 / dsr, -k * dsr)
    drr = torch.cdist(rec, rec)
    X_true = torch.polar(1.0 / (drr + X_TRUE_OFFSET), -k * drr)
    X_true = 0.5 * (X_true + X_true.T)
    U_clean = D_clean @ X_true
    del X_true, drr

    def cg(shape):
        return torch.complex(torch.randn(shape, generator=gen, device=device, dtype=torch.float32),
                             torch.randn(shape, generator=gen, device=device, dtype=torch.float32))
    n_u = cg(U_clean.shape)
    U = U_clean + n_u * (torch.linalg.norm(U_clean) / (torch.linalg.norm(n_u) * 10.0 ** (snr_db / 20.0)))
    del n_u, U_clean
    n_d = cg(D_clean.shape)
    D = D_clean + n_d * (0.05 * torch.linalg.norm(D_clean) / torch.linalg.norm(n_d))
    del n_d, D_clean
    dmin = dsr.min()   # the normalisation 1 / alpha = min distance, kept on the device
    n = theta_length(lay)
    s = math.sqrt(1e-2 / 2.0)
    th = torch.complex(s * torch.randn(n, generator=gen, device=device, dtype=torch.float32),
                       s * torch.randn(n, generator=gen, device=device, dtype=torch.float32))
    return (D * dmin).contiguous(), (U * dmin).contiguous(), th
