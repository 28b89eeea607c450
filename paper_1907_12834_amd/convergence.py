"""Plain vs interleaved convergence study (Sec. VII "Operator interleaving").

The paper measures the accuracy of the QLG step on stationary 1D eigenstates by
the unnormalised density error

    eps_L2 = sum over sites (n_exact - n_sim)^2,   n = sum_m |psi_m|^2,

after a fixed number of steps, for lattices of growing size, and compares the
power law eps_L2 ~ L^p of the plain split (one U per step) with the interleaved
one (U^{1/4} before each I').  The states are the Table I coefficients in the
bright form psi_m = c_m K sech(K X) (E = -2) and in the dark two-kink product
c_m K tanh(K(X - Lp/4)) tanh(K(3Lp/4 - X)) of Sec. IV (E = +2), with K = 1 and
X = eps x; a lattice of L = 40 w sites resolves the soliton width 1/K with
w = 1/eps sites.

Two protocols:
  * "fixed_steps": the paper's, a fixed number of steps (1000) at every size, so
    the physical time eps^2 * steps shrinks as 1/w^2 (diffusive scaling alone
    gives p = -2);
  * "fixed_time": a fixed physical time, where an O(eps^2) method gives an error
    that falls 8x per doubling of w (p = -3 for the sum over 2x the sites).

Every run goes through the HIP kernels (complex128 by default); `main` prints
the table and the fitted slopes as JSON.
"""
from __future__ import annotations

import argparse
import json
import math
import time
from typing import Dict, List, Sequence

import numpy as np
import torch

import qlg_inputs as qi
from .qlg import Lattice

# couplings for which Table I row 14 is real at E = -2 (bright) and at E = +2 (dark)
G_BRIGHT = (-1.0, 0.2, 1.0)
G_DARK = (1.0, 0.1, 0.7)
ROW = 14
SITES_PER_WIDTH = 40


def initial_state(kind: str, w: int) -> tuple:
    """(psi (5, L) complex128, eps, g) of the stationary state `kind` at resolution w."""
    eps = 1.0 / w
    L = SITES_PER_WIDTH * w
    if kind == "bright":
        c = qi.table1_coeffs(ROW, -2.0, *G_BRIGHT).real
        X = (np.arange(L) - L / 2) * eps
        return c[:, None] * (1.0 / np.cosh(X))[None, :], eps, G_BRIGHT
    if kind == "dark":
        c = qi.table1_coeffs(ROW, 2.0, *G_DARK).real
        return qi.dark_pair_1d(L, eps, c, K=1.0), eps, G_DARK
    raise ValueError("kind must be 'bright' or 'dark'")


def density_error(psi0: np.ndarray, psi: np.ndarray) -> float:
    """sum over sites (n_exact - n_sim)^2 with n = sum_m |psi_m|^2 (the stationary n is n(t = 0))."""
    n0 = (np.abs(psi0) ** 2).sum(axis=0)
    n1 = (np.abs(psi) ** 2).sum(axis=0)
    return float(np.sum((n0 - n1) ** 2))


def run_case(kind: str, split: str, w: int, nsteps: int, dtype: str = "c128") -> float:
    """eps_L2 after nsteps of the GPU step from the stationary state."""
    psi0, eps, g = initial_state(kind, w)
    lat = Lattice(1, [psi0.shape[1]], g=g, eps=eps, dtype=dtype, split=split)
    lat.set_psi([torch.from_numpy(psi0)])
    lat.step(nsteps)
    psi = lat.get_psi()[0].cpu().numpy().astype(np.complex128)
    lat.close()
    return density_error(psi0, psi)


def steps_for(protocol: str, w: int, nsteps: int, T: float) -> int:
    return nsteps if protocol == "fixed_steps" else int(round(T * w * w))


def slope(ws: Sequence[int], errs: Sequence[float]) -> float:
    """Least-squares exponent p of eps_L2 ~ L^p over the finite errors (L = 40 w)."""
    pts = [(math.log(SITES_PER_WIDTH * w), math.log(e)) for w, e in zip(ws, errs) if e > 0 and math.isfinite(e)]
    if len(pts) < 2:
        return float("nan")
    x, y = np.array(pts).T
    return float(np.polyfit(x, y, 1)[0])


def study(protocol: str = "fixed_steps", ws: Sequence[int] = (8, 12, 16, 24, 32, 48, 64), nsteps: int = 1000,
          T: float = 0.5, dtype: str = "c128") -> Dict:
    out: Dict = {"protocol": protocol, "w": list(ws), "lattice": [SITES_PER_WIDTH * w for w in ws],
                 "steps": [steps_for(protocol, w, nsteps, T) for w in ws], "dtype": dtype, "cases": {}}
    t0 = time.perf_counter()
    for kind in ("bright", "dark"):
        for split in ("interleaved", "plain"):
            errs: List[float] = [run_case(kind, split, w, steps_for(protocol, w, nsteps, T), dtype) for w in ws]
            out["cases"]["%s/%s" % (kind, split)] = {"eps_L2": errs, "slope": slope(ws, errs)}
    torch.cuda.synchronize()
    out["gpu_seconds"] = time.perf_counter() - t0
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description="plain vs interleaved convergence study on the GPU")
    ap.add_argument("--protocol", choices=["fixed_steps", "fixed_time"], default="fixed_steps")
    ap.add_argument("--steps", type=int, default=1000, help="steps of the fixed_steps protocol")
    ap.add_argument("--time", type=float, default=0.5, help="physical time of the fixed_time protocol")
    ap.add_argument("--w", type=int, nargs="+", default=[8, 12, 16, 24, 32, 48, 64])
    ap.add_argument("--dtype", choices=["c64", "c128"], default="c128")
    a = ap.parse_args(argv)
    print(json.dumps(study(a.protocol, a.w, a.steps, a.time, a.dtype)))


if __name__ == "__main__":
    main()
