"""Write the FP64 oracle's energy gradients for the 64 x 64 adjoint checks.

The oracle is differentiated by torch autograd, one step at a time: the forward run
stores (a, b) after every step without a graph, then the reverse walk rebuilds the
graph of one step from its stored input and pulls the cotangent back through it
(the same derivative as autograd through the whole run, with memory bounded by one
step's graph).  Stored per case: the objective L = E(psi_T) (the lattice energy of
Sec. II), dL/dpsi_0 (complex128, shape (5, 64, 64), cotangent convention
dL/dRe + i dL/dIm) and dL/d(g0, g1, g2); and the same three for an input that differs
from psi_0 at the rounding level (every amplitude times 1 + 1e-15 u, u a seeded
standard normal), whose distance from the first is the conditioning of the gradient:
the least difference any two FP64 implementations can be expected to show.

Cases (2D, interleaved split, g = (1, -0.3, 0.2), eps = 0.4):
  vortex_pair_T40, vortex_pair_T125: the vortex-pair construction (separation 16 sites,
      Pade coefficients drawn with default_rng(2019)) over 40 steps and over 125 steps,
      the physical time (eps^2 per step) of 2000 steps at eps = 0.1;
  spin_texture_T40, spin_texture_T125: the same state with a seeded random spinor of
      amplitude 0.05 added to every component, so that F != 0 at every site.
With g1 < 0 the vortex pair's m = +2 / m = -2 symmetry is dynamically unstable: an
asymmetry grows about 1e5-fold every 100 steps at eps = 0.4, so over much longer runs
rounding decides the trajectory and no FP64 gradient is reproducible.

Usage (from the repository root; about 10 minutes on 4 CPU threads):

    python tests/golden/make_adjoint_reference.py
"""
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import qlg_inputs as qi  # noqa: E402
from oracle import qlg_oracle as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "adjoint_64x64_oracle_grad.npz")
G = (1.0, -0.3, 0.2)
EPS = 0.4
CASES = {"vortex_pair_T40": 40, "vortex_pair_T125": 125, "spin_texture_T40": 40, "spin_texture_T125": 125}
PERTURB_SEED = 91


def initial_state(case):
    if case.startswith("vortex_pair"):
        return qi.adjoint_vortex_pair_2d_64()
    return qi.adjoint_spin_texture_2d_64()


def rounding_perturbed(psi0):
    u = np.random.default_rng(PERTURB_SEED).standard_normal(psi0.shape)
    return psi0 * (1.0 + 1e-15 * u)


def energy_grad(psi0, g, eps, nsteps, split="interleaved"):
    ndim = psi0.ndim - 1
    t0 = time.time()
    with torch.no_grad():
        a, b = O.encode(torch.from_numpy(psi0))
        states = [(a, b)]
        for k in range(nsteps):
            a, b = O.step(a, b, eps, g, ndim, split)
            states.append((a, b))
            if (k + 1) % 100 == 0:
                print("  forward %d (%.0f s)" % (k + 1, time.time() - t0), flush=True)
    gt = torch.tensor(g, dtype=torch.float64, requires_grad=True)
    gg = (gt[0], gt[1], gt[2])
    aT = states[-1][0].clone().requires_grad_(True)
    bT = states[-1][1].clone().requires_grad_(True)
    L = O.energy(aT + bT, eps, gg)
    la, lb, dg = torch.autograd.grad(L, (aT, bT, gt))
    for k in reversed(range(nsteps)):
        a0 = states[k][0].clone().requires_grad_(True)
        b0 = states[k][1].clone().requires_grad_(True)
        a1, b1 = O.step(a0, b0, eps, gg, ndim, split)
        la, lb, dgk = torch.autograd.grad((a1, b1), (a0, b0, gt), grad_outputs=(la, lb))
        dg = dg + dgk
        states[k + 1] = None
        if k % 100 == 0:
            print("  reverse %d (%.0f s)" % (k, time.time() - t0), flush=True)
    p = torch.from_numpy(psi0).clone().requires_grad_(True)
    a0, b0 = O.encode(p)
    (gp,) = torch.autograd.grad((a0, b0), (p,), grad_outputs=(la, lb))
    return float(L.detach()), gp.numpy(), dg.numpy()


def main():
    out = {}
    for case, nsteps in CASES.items():
        psi0 = initial_state(case)
        print("%s: %d steps" % (case, nsteps), flush=True)
        L, gp, gg = energy_grad(psi0, G, EPS, nsteps)
        out[case + "_L"] = np.float64(L)
        out[case + "_dpsi"] = gp
        out[case + "_dg"] = gg
        out[case + "_steps"] = np.int64(nsteps)
        print("  L = %.17g, dL/dg = %s" % (L, gg), flush=True)
        Lp, gpp, ggp = energy_grad(rounding_perturbed(psi0), G, EPS, nsteps)
        out[case + "_perturbed_L"] = np.float64(Lp)
        out[case + "_perturbed_dpsi"] = gpp
        out[case + "_perturbed_dg"] = ggp
        print("  rounding-level input change: dpsi rel %.3e, dg rel %.3e" %
              (np.linalg.norm(gpp - gp) / np.linalg.norm(gp), np.linalg.norm(ggp - gg) / np.linalg.norm(gg)),
              flush=True)
    np.savez_compressed(OUT, eps=EPS, g=np.array(G), **out)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
