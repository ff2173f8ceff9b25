"""Shared construction of parity cases for the GPU tests.

Inputs come from the seeded generator (synth), are rounded once to complex64,
and both sides consume the rounded values: the oracle in complex128, the
HIP library in complex64 on the device. Each side applies its own Hilbert
ordering (oracle.hilbert_order on the CPU; the library's hilbert_order and its
device column gather on the GPU).
"""
import dataclasses

import numpy as np

import oracle as O
import synth

U32 = 2.0 ** -24


def c64(a):
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


@dataclasses.dataclass
class Case:
    name: str
    layout: synth.Layout
    T: O.Tiling
    D_nat: np.ndarray     # natural order, complex64-rounded (complex128 dtype)
    U_nat: np.ndarray
    D: np.ndarray         # Hilbert order (oracle side)
    U: np.ndarray
    theta: np.ndarray     # complex64-rounded
    ix: np.ndarray
    iy: np.ndarray


def from_workload(wl, f_idx, name=None):
    geom = wl.geometry()
    prob = wl.problem(f_idx, geom)
    lay = wl.layout(f_idx)
    return _finish(name or f"{wl.name}[{f_idx}]", lay, prob.D, prob.U, wl.theta0(f_idx, lay),
                   geom.rec_ix, geom.rec_iy)


def from_geometry(nx, ny, ns_mode, freq, layout, seed_item, name, snr=20.0, scale_theta=1.0):
    geom = synth.make_geometry(nx, ny, ns_mode)
    prob = synth.make_problem(geom, freq, snr, 0.05, 90, seed_item)
    th = synth.init_theta(synth.theta_length(layout), 90, seed_item) * scale_theta
    return _finish(name, layout, prob.D, prob.U, th, geom.rec_ix, geom.rec_iy)


def _finish(name, lay, D, U, th, ix, iy):
    T = O.tiling(lay.tile_size, lay.rank_off, lay.rank_diag)
    Dn, Un, th = c64(D), c64(U), c64(th)
    perm = O.hilbert_order(ix, iy)
    return Case(name, lay, T, Dn, Un, O.permute_columns(Dn, perm), O.permute_columns(Un, perm), th,
                np.asarray(ix), np.asarray(iy))


def to_device(case, tl, torch):
    """Device tensors in Hilbert order, built through the library."""
    perm = tl.hilbert_order(case.ix, case.iy)
    dev = torch.device("cuda")
    pd = torch.from_numpy(perm).to(dev)
    Dn = torch.from_numpy(case.D_nat.astype(np.complex64)).to(dev)
    Un = torch.from_numpy(case.U_nat.astype(np.complex64)).to(dev)
    D = tl.permute_columns(Dn, pd)
    U = tl.permute_columns(Un, pd)
    th = torch.from_numpy(case.theta.astype(np.complex64)).to(dev)
    plan = tl.Plan.from_layout(case.layout, case.D.shape[0])
    return plan, D, U, th, perm


def residual_bound(case, X):
    """Element-wise FP32 error scale of r = D X - U: sqrt(K) u (|D||X| + |U|)."""
    K = X.shape[0]
    return np.sqrt(K) * U32 * (np.abs(case.D) @ np.abs(X) + np.abs(case.U))


def gradient_bound(case, X, r):
    """Element-wise FP32 error scale of the tile gradient, propagated from r."""
    Er = residual_bound(case, X)
    ns = case.D.shape[0]
    aDH = np.abs(case.D).T
    EW = aDH @ Er + np.sqrt(ns) * U32 * (aDH @ np.abs(r))
    at = np.abs(case.theta).astype(np.complex128)
    dmax = max(case.T.d)
    W = case.D.conj().T @ r
    return (O.tile_gradient(case.T, at, EW.astype(np.complex128)).real
            + np.sqrt(dmax) * U32 * O.tile_gradient(case.T, at, np.abs(W).astype(np.complex128)).real)


BF16_SPLIT = 2.0 ** -15   # relative error per product of the hi+lo split (dropped lo*lo + lo rounding)


def residual_bound_bf16(case, X):
    """Element-wise error scale of r = D X - U with BF16 hi+lo split products."""
    aDX = np.abs(case.D) @ np.abs(X)
    K = X.shape[0]
    return BF16_SPLIT * aDX + np.sqrt(K) * U32 * (aDX + np.abs(case.U))


def gradient_bound_bf16(case, X, r):
    Er = residual_bound_bf16(case, X)
    ns = case.D.shape[0]
    aDH = np.abs(case.D).T
    EW = aDH @ Er + (BF16_SPLIT + np.sqrt(ns) * U32) * (aDH @ np.abs(r))
    at = np.abs(case.theta).astype(np.complex128)
    dmax = max(case.T.d)
    W = case.D.conj().T @ r
    return (O.tile_gradient(case.T, at, EW.astype(np.complex128)).real
            + np.sqrt(dmax) * U32 * O.tile_gradient(case.T, at, np.abs(W).astype(np.complex128)).real)
