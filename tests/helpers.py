"""Shared test helpers: oracle runs on light-cone windows and error metrics."""
import numpy as np
import torch

from oracle import qlg_oracle as O


def rel_l2(got, ref) -> float:
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.linalg.norm((got - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def oracle_qubits(a, b, nsteps, eps, g, split="interleaved"):
    """Run the oracle from numpy (a, b) planes; returns numpy (a, b)."""
    A, B = O.run(torch.from_numpy(np.ascontiguousarray(a)).to(torch.complex128),
                 torch.from_numpy(np.ascontiguousarray(b)).to(torch.complex128),
                 nsteps, eps, g, a.ndim - 1, split)
    return A.numpy(), B.numpy()


_CACHE = {}


def oracle_psi(psi, nsteps, eps, g, split="interleaved", key=None):
    """Oracle run from psi; results for a given `key` are computed once per session."""
    if key is not None and (key, nsteps, split) in _CACHE:
        return _CACHE[(key, nsteps, split)]
    a, b = O.run_psi(psi, nsteps, eps, g, split)
    out = (a.numpy(), b.numpy())
    if key is not None:
        _CACHE[(key, nsteps, split)] = out
    return out


def window_1d(field, center, half):
    """Periodic window field[..., center-half : center+half+1] of a (..., L) array."""
    L = field.shape[-1]
    idx = (np.arange(center - half, center + half + 1) % L)
    return field[..., idx]


def window_2d(field, cy, cx, half):
    ny, nx = field.shape[-2:]
    iy = (np.arange(cy - half, cy + half + 1) % ny)
    ix = (np.arange(cx - half, cx + half + 1) % nx)
    return field[..., iy[:, None], ix[None, :]]


def light_cone_oracle_1d(psi, center, nsteps, eps, g, split="interleaved"):
    """psi(center) after nsteps from the oracle on a window covering the light cone.

    One step has dependency radius 4 (four I' of radius 1), so a periodic
    window of half-width 4*nsteps + 2 reproduces the full-lattice value at its
    centre exactly: contamination from the artificial wrap moves at most 4
    sites per step.
    """
    half = 4 * nsteps + 2
    win = window_1d(psi, center, half)
    a, b = oracle_psi(win, nsteps, eps, g, split)
    return (a + b)[:, half]


def light_cone_oracle_2d(psi, cy, cx, nsteps, eps, g, half_out=0, split="interleaved"):
    """psi on the (2*half_out+1)^2 block around (cy, cx) after nsteps (2D light cone, radius 4/step/axis)."""
    half = 4 * nsteps + 2 + half_out
    win = window_2d(psi, cy, cx, half)
    a, b = oracle_psi(win, nsteps, eps, g, split)
    c = half
    return (a + b)[:, c - half_out:c + half_out + 1, c - half_out:c + half_out + 1]
