"""GPU adjoint: gradients of a final-state objective through the HIP reverse sweep.

References: the FP64 oracle differentiated by torch autograd (tolerance 1e-10
relative), central finite differences of the GPU forward (1e-6), and exact
adjointness of the linear (g = 0) step.
"""
import numpy as np
import pytest
import torch

import qlg_inputs as qi
from oracle import qlg_oracle as O

pytestmark = pytest.mark.gpu


def lattice(*args, **kw):
    from paper_1907_12834_amd.qlg import Lattice
    return Lattice(*args, **kw)


def objective(*args, **kw):
    from paper_1907_12834_amd.autograd import qlg_objective
    return qlg_objective(*args, **kw)


def oracle_grad(psi0, g, eps, nsteps, split="interleaved", kind="energy", target=None, V=None, mu=0.0):
    p = torch.from_numpy(np.ascontiguousarray(psi0)).clone().requires_grad_(True)
    gt = torch.tensor(g, dtype=torch.float64, requires_grad=True)
    gg = (gt[0], gt[1], gt[2])
    a, b = O.encode(p)
    a, b = O.run(a, b, nsteps, eps, gg, p.dim() - 1, split, V=V, mu=mu)
    psi = a + b
    if kind == "energy":
        L = O.energy(psi, eps, gg, V, mu)
    else:
        t = torch.from_numpy(target)
        meas = eps ** (p.dim() - 1)
        L = (meas * (t.conj() * psi).sum()).abs() ** 2
    L.backward()
    return float(L.detach()), p.grad.numpy(), gt.grad.numpy()


def gpu_grad(psi0, g, eps, nsteps, K=4, dtype="c128", split="interleaved", kind="energy", target=None, V=None,
             mu=0.0):
    dev = "cuda:0"
    cdt = torch.complex64 if dtype == "c64" else torch.complex128
    p = torch.from_numpy(psi0).to(dev, cdt).requires_grad_(True)
    gt = torch.tensor(g, dtype=torch.float64, requires_grad=True)
    tg = torch.from_numpy(target).to(dev, cdt) if target is not None else None
    L = objective(p, gt, eps=eps, nsteps=nsteps, checkpoint_every=K, dtype=dtype, split=split, kind=kind,
                  target=tg, V=V, mu=mu)
    L.backward()
    return float(L.detach()), p.grad.detach().cpu().numpy().astype(np.complex128), gt.grad.numpy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


G = (1.1, -0.6, 0.8)


@pytest.mark.parametrize("split", ["interleaved", "plain"])
@pytest.mark.parametrize("shape", [(40,), (8, 10)])
def test_energy_gradient_matches_oracle_autograd(shape, split):
    psi0 = qi.random_field(shape, seed=41, scale=0.4)
    eps, nsteps = 0.3, 9
    L0, gp0, gg0 = oracle_grad(psi0, G, eps, nsteps, split)
    L1, gp1, gg1 = gpu_grad(psi0, G, eps, nsteps, K=4, split=split)
    assert abs(L1 - L0) <= 1e-12 * abs(L0)
    assert rel(gp1, gp0) <= 1e-10, rel(gp1, gp0)
    assert rel(gg1, gg0) <= 1e-10, (gg1, gg0)


@pytest.mark.parametrize("kind", ["energy", "fidelity"])
@pytest.mark.parametrize("split", ["interleaved", "plain"])
@pytest.mark.parametrize("shape", [(40,), (8, 10)])
def test_gradient_with_potential_matches_oracle_autograd(shape, split, kind):
    """An external potential V(x) and a chemical potential mu in the run (Sec. II "Additional terms"):
    the reverse sweep differentiates U with its (V + mu) phase, and the energy objective includes
    eps^d sum (V + mu) n."""
    psi0 = qi.random_field(shape, seed=45, scale=0.4)
    target = qi.random_field(shape, seed=46, scale=0.3) if kind == "fidelity" else None
    V = np.random.default_rng(47).uniform(0.0, 2.5, size=shape)
    eps, nsteps, mu = 0.3, 9, 0.7
    L0, gp0, gg0 = oracle_grad(psi0, G, eps, nsteps, split, kind, target, V=V, mu=mu)
    L1, gp1, gg1 = gpu_grad(psi0, G, eps, nsteps, K=4, split=split, kind=kind, target=target, V=V, mu=mu)
    assert abs(L1 - L0) <= 1e-12 * abs(L0), (L1, L0)
    assert rel(gp1, gp0) <= 1e-10, rel(gp1, gp0)
    assert rel(gg1, gg0) <= 1e-10, (gg1, gg0)
    # the potential changes the gradient (it is not silently ignored)
    _, gp2, _ = oracle_grad(psi0, G, eps, nsteps, split, kind, target)
    assert rel(gp2, gp0) > 1e-3


@pytest.mark.parametrize("kind,split,pot", [("energy", "interleaved", False), ("energy", "plain", False),
                                            ("fidelity", "interleaved", False), ("energy", "interleaved", True)])
def test_3d_gradient_matches_oracle_autograd(kind, split, pot):
    """3D (Lie product n = 12): the reverse sweep walks z, y, x substeps; against oracle autograd."""
    shape = (3, 4, 6)
    psi0 = qi.random_field(shape, seed=51, scale=0.4)
    target = qi.random_field(shape, seed=52, scale=0.3) if kind == "fidelity" else None
    V = np.random.default_rng(53).uniform(0.0, 2.0, size=shape) if pot else None
    mu = 0.4 if pot else 0.0
    eps, nsteps = 0.35, 7
    L0, gp0, gg0 = oracle_grad(psi0, G, eps, nsteps, split, kind, target, V=V, mu=mu)
    L1, gp1, gg1 = gpu_grad(psi0, G, eps, nsteps, K=3, split=split, kind=kind, target=target, V=V, mu=mu)
    assert abs(L1 - L0) <= 1e-12 * abs(L0), (L1, L0)
    assert rel(gp1, gp0) <= 1e-10, rel(gp1, gp0)
    assert rel(gg1, gg0) <= 1e-10, (gg1, gg0)


def test_fidelity_gradient_matches_oracle_autograd():
    psi0 = qi.random_field((33,), seed=42, scale=0.4)
    target = qi.random_field((33,), seed=43, scale=0.3)
    eps, nsteps = 0.3, 7
    L0, gp0, gg0 = oracle_grad(psi0, G, eps, nsteps, kind="fidelity", target=target)
    L1, gp1, gg1 = gpu_grad(psi0, G, eps, nsteps, kind="fidelity", target=target)
    assert abs(L1 - L0) <= 1e-12 * abs(L0)
    assert rel(gp1, gp0) <= 1e-10
    assert rel(gg1, gg0) <= 1e-10


def test_checkpoint_interval_does_not_change_gradient():
    """The checkpoint interval changes which states the reverse sweep regenerates (a chain of
    per-substep kernels) and which it takes from the fused forward kernel.  Both evaluate the same
    formulas, but the compiler contracts them into FMAs differently, so FP64 states can differ in
    the last bit; summed over every site and substep, dL/dg then moves by ~1e-14 relative.  The
    bound, 1e-13, stays ten times under the FP64 parity bar."""
    psi0 = qi.random_field((50,), seed=44, scale=0.4)
    ref = gpu_grad(psi0, G, 0.3, 12, K=1)
    for K in (3, 5, 12, 50):
        got = gpu_grad(psi0, G, 0.3, 12, K=K)
        assert rel(got[1], ref[1]) <= 1e-13 and rel(got[2], ref[2]) <= 1e-13, K


def test_finite_differences_fp64():
    psi0 = qi.random_field((36,), seed=45, scale=0.4)
    eps, nsteps, h = 0.3, 10, 1e-6
    L, gp, gg = gpu_grad(psi0, G, eps, nsteps)
    rng = np.random.default_rng(46)
    d = rng.normal(size=psi0.shape) + 1j * rng.normal(size=psi0.shape)

    def Lof(p, g):
        with torch.no_grad():
            return float(objective(torch.from_numpy(p).cuda(), torch.tensor(g, dtype=torch.float64), eps=eps,
                                   nsteps=nsteps, checkpoint_every=4))
    fd = (Lof(psi0 + h * d, G) - Lof(psi0 - h * d, G)) / (2 * h)
    an = float(np.real(np.sum(np.conj(gp) * d)))
    assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-8), (fd, an)
    for k in range(3):
        gp_, gm_ = list(G), list(G)
        gp_[k] += h
        gm_[k] -= h
        fdg = (Lof(psi0, gp_) - Lof(psi0, gm_)) / (2 * h)
        assert abs(fdg - gg[k]) <= 1e-6 * max(abs(gg[k]), 1e-8), (k, fdg, gg[k])


@pytest.mark.parametrize("ndim", [1, 2])
def test_linear_step_adjointness(ndim):
    """g = 0: the step is linear and unitary; <y, M z0> = <M^H y, z0> exactly."""
    shape = (45,) if ndim == 1 else (9, 13)
    a, b = qi.random_qubits(shape, seed=47, scale=0.5)
    lat = lattice(ndim, [shape[-1]], [shape[0]] if ndim == 2 else None, g=(0.0, 0.0, 0.0), eps=0.3,
                  dtype="c128")
    z0 = np.stack([a, b])
    lat.set_qubits([torch.from_numpy(z0)])
    nsteps, K = 7, 3
    ckpt = lat.forward_record(nsteps, K)
    zT = lat.get_qubits()[0].cpu().numpy()
    y = qi.random_qubits(shape, seed=48, scale=1.0)
    y = np.stack(y)
    lam = torch.from_numpy(y.reshape(-1).copy()).cuda()
    dg = lat.adjoint_step(nsteps, K, ckpt, lam)
    lam0 = lam.cpu().numpy().reshape(z0.shape)
    lhs = np.vdot(y, zT)
    rhs = np.vdot(lam0, z0)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    assert all(np.isfinite(dg))   # dL/dg at g = 0 is not zero: the objective depends on g


def test_batched_adjoint_matches_single_instances():
    from paper_1907_12834_amd.qlg import Lattice
    f = [qi.random_field((30,), seed=50, scale=0.4), qi.random_field((47,), seed=51, scale=0.4)]
    eps, nsteps, K = 0.3, 6, 4
    lat = Lattice(1, [30, 47], g=G, eps=eps, dtype="c128")
    lat.set_psi([torch.from_numpy(x) for x in f])
    ck = lat.forward_record(nsteps, K)
    val, lam, dg0 = lat.objective_grad("energy")
    dg = lat.adjoint_step(nsteps, K, ck, lam)
    lam = lam.cpu().numpy()
    off, tot_dg, tot_val = 0, np.zeros(3), 0.0
    for x in f:
        one = Lattice(1, [x.shape[1]], g=G, eps=eps, dtype="c128")
        one.set_psi([torch.from_numpy(x)])
        c1 = one.forward_record(nsteps, K)
        v1, l1, e1 = one.objective_grad("energy")
        d1 = one.adjoint_step(nsteps, K, c1, l1)
        n = 10 * x.shape[1]
        assert rel(lam[off:off + n], l1.cpu().numpy()) <= 1e-14
        off += n
        tot_dg += np.array(d1) + np.array(e1)
        tot_val += v1
    assert abs(val - tot_val) <= 1e-13 * abs(tot_val)
    assert rel(np.array(dg) + np.array(dg0), tot_dg) <= 1e-13


def test_adjoint_independent_of_forward_plan():
    """The checkpoints come from the fused forward kernels of the context's plan: a site's qubits
    on one lane, on two wavefronts or on two lanes give the same gradient (the plans round the
    forward states in different orders, FP64)."""
    from paper_1907_12834_amd.qlg import Lattice
    x = qi.random_field((83,), seed=52, scale=0.4)
    eps, nsteps, K = 0.3, 7, 3
    res = []
    for S, qs in ((1, 0), (3, 1), (2, 2), (3, 2)):
        lat = Lattice(1, [83], g=G, eps=eps, dtype="c128")
        lat.set_tuning(steps_per_pass=S, qubit_split=qs)
        lat.set_psi([torch.from_numpy(x)])
        ck = lat.forward_record(nsteps, K)
        val, lam, dg0 = lat.objective_grad("energy")
        dg = lat.adjoint_step(nsteps, K, ck, lam)
        res.append((val, lam.cpu().numpy(), np.array(dg) + np.array(dg0)))
    for val, lam, dg in res[1:]:
        assert abs(val - res[0][0]) <= 1e-13 * abs(res[0][0])
        assert rel(lam, res[0][1]) <= 1e-12 and rel(dg, res[0][2]) <= 1e-12


def test_c64_forward_fp64_jacobian_close_to_oracle():
    psi0 = qi.random_field((40,), seed=52, scale=0.4)
    eps, nsteps = 0.3, 9
    L0, gp0, gg0 = oracle_grad(psi0, G, eps, nsteps)
    L1, gp1, gg1 = gpu_grad(psi0, G, eps, nsteps, dtype="c64")
    assert abs(L1 - L0) <= 1e-5 * abs(L0)
    assert rel(gp1, gp0) <= 1e-4
    assert rel(gg1, gg0) <= 1e-4


def test_adjoint_vortex_pair_512_full_size():
    """The adjoint workload at full size (the 512^2 vortex pair, checkpoints every 64), 128 steps.
    Complex64 forward with the FP64 Jacobian: the energy is invariant under a global phase, so
    the gradient is orthogonal to i psi0.  Complex128: dL/dg0 and a directional derivative against
    central differences of the GPU forward."""
    w = qi.adjoint_vortex_pair_2d_512(nsteps=128)
    psi0, g, eps, nsteps, K = w.psi[0], w.g, w.eps, 128, 64
    L, gp, gg = gpu_grad(psi0, g, eps, nsteps, K=K, dtype="c64")
    dphase = float(np.real(np.sum(np.conj(gp) * (1j * psi0))))
    assert abs(dphase) <= 1e-4 * np.linalg.norm(gp) * np.linalg.norm(psi0), dphase
    L, gp, gg = gpu_grad(psi0, g, eps, nsteps, K=K, dtype="c128")
    h = 1e-6

    def Lof(p, gv):
        with torch.no_grad():
            return float(objective(torch.from_numpy(p).cuda(), torch.tensor(gv, dtype=torch.float64), eps=eps,
                                   nsteps=nsteps, checkpoint_every=K))
    gp_, gm_ = list(g), list(g)
    gp_[0] += h
    gm_[0] -= h
    fdg = (Lof(psi0, gp_) - Lof(psi0, gm_)) / (2 * h)
    assert abs(fdg - gg[0]) <= 1e-6 * abs(gg[0]), (fdg, gg[0])
    d = qi.random_field(psi0.shape[1:], seed=54, scale=1.0)
    fd = (Lof(psi0 + h * d, g) - Lof(psi0 - h * d, g)) / (2 * h)
    an = float(np.real(np.sum(np.conj(gp) * d)))
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)


def test_vortex_pair_2d_fd_check():
    """The 2D vortex-pair construction on 64^2 (eps = 0.4, separation 16) in FP64: FD vs adjoint."""
    rng = np.random.default_rng(2019)
    psi0 = qi.vortex_pair_2d(64, 64, 16.0, 0.4, rng)
    g, eps, nsteps, K, h = (1.0, -0.3, 0.2), 0.4, 40, 16, 1e-6
    L, gp, gg = gpu_grad(psi0, g, eps, nsteps, K=K)

    def Lof(p, gv):
        with torch.no_grad():
            return float(objective(torch.from_numpy(p).cuda(), torch.tensor(gv, dtype=torch.float64), eps=eps,
                                   nsteps=nsteps, checkpoint_every=K))
    d = qi.random_field((64, 64), seed=53, scale=1.0)
    fd = (Lof(psi0 + h * d, g) - Lof(psi0 - h * d, g)) / (2 * h)
    an = float(np.real(np.sum(np.conj(gp) * d)))
    assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    for k in range(3):
        gp_, gm_ = list(g), list(g)
        gp_[k] += h
        gm_[k] -= h
        fdg = (Lof(psi0, gp_) - Lof(psi0, gm_)) / (2 * h)
        assert abs(fdg - gg[k]) <= 1e-6 * max(abs(gg[k]), 1e-6), (k, fdg, gg[k])


@pytest.mark.parametrize("split", ["interleaved", "plain"])
def test_3d_gradient_multi_chunk_matches_oracle_autograd(split):
    """A 3D lattice of several 256-site chunks (16 x 12 x 10 = 1920 sites, 8 chunks; ragged
    extents): every substep kernel of the reverse sweep writes its dL/dg partials for all
    chunks, so the workspace must be sized by the whole lattice, not by one x row."""
    shape = (16, 12, 10)
    psi0 = qi.random_field(shape, seed=57, scale=0.4)
    eps, nsteps = 0.35, 5
    L0, gp0, gg0 = oracle_grad(psi0, G, eps, nsteps, split)
    L1, gp1, gg1 = gpu_grad(psi0, G, eps, nsteps, K=2, split=split)
    assert abs(L1 - L0) <= 1e-12 * abs(L0), (L1, L0)
    assert rel(gp1, gp0) <= 1e-10, rel(gp1, gp0)
    assert rel(gg1, gg0) <= 1e-10, (gg1, gg0)
