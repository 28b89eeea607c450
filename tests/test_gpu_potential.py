"""GPU parity of the external potential V(x) and chemical potential mu (Sec. II "Additional terms").

The HIP path (qlg_set_potential + qlg_step, through the C ABI) against the FP64
oracle's step with the same V and mu: FP64 rel-L2 <= 1e-12, FP32 <= 1e-4, on
ragged 1D and 2D lattices in every launch plan (1D: one- and two-wave tiles,
1..7 steps per pass; 2D: several band heights), both splits, batches of
instances with their own potentials; the energy observable with the (V + mu) n
term; harmonic-trap physics on the GPU; removal of the potential restoring the
plain kernels bit for bit; and graph replay and potentials whose values change
between calls.  (Gradients with a potential: tests/test_gpu_adjoint.py.)
"""
import numpy as np
import pytest
import torch

import qlg_inputs as qi
from helpers import rel_l2
from oracle import qlg_oracle as O

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-4}


def lattice(*args, **kw):
    from paper_1907_12834_amd.qlg import Lattice
    return Lattice(*args, **kw)


def smooth_potential(shape, seed, amp=3.0):
    """A seeded smooth periodic potential (a few low Fourier modes) plus a small random part."""
    rng = np.random.default_rng(seed)
    grids = np.meshgrid(*[np.arange(n) / n for n in shape], indexing="ij")
    V = np.zeros(shape)
    for _ in range(3):
        k = [int(v) for v in rng.integers(0, 3, size=len(shape))]
        V += rng.uniform(0.2, 1.0) * np.cos(2 * np.pi * sum(ki * g for ki, g in zip(k, grids)) + rng.uniform(0, 6))
    return amp * (V + 0.1 * rng.normal(size=shape))


def oracle_qubits_ext(a, b, nsteps, eps, g, split, V, mu):
    A, B = O.run(torch.from_numpy(np.ascontiguousarray(a)), torch.from_numpy(np.ascontiguousarray(b)),
                 nsteps, eps, g, a.ndim - 1, split, V=V, mu=mu)
    return A.numpy(), B.numpy()


def qubits_tensor(a, b):
    return torch.from_numpy(np.stack([a, b]))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("split", ["interleaved", "plain"])
@pytest.mark.parametrize("plan", [(1, 0), (3, 0), (7, 0), (2, 1), (4, 1), (1, 2), (3, 2)])
def test_1d_potential_random_qubits(dtype, split, plan):
    """(steps per pass, qubit split): V + mu on a ragged lattice, element-wise against the oracle."""
    S, qsplit = plan
    L, nsteps = 437, 13
    g, eps, mu = (1.2, -0.7, 0.9), 0.35, 0.6
    # amplitude 0.4: the plain split's large nonlinear phases amplify a relative perturbation
    # of the initial state 44x over these 13 steps (387x at amplitude 0.5, where FP32 rounding
    # alone reaches the 1e-4 bar with or without a potential)
    a, b = qi.random_qubits((L,), seed=31, scale=0.4)
    V = smooth_potential((L,), seed=3)
    lat = lattice(1, [L], g=g, eps=eps, dtype=dtype, split=split)
    lat.set_tuning(steps_per_pass=S, qubit_split=qsplit)
    lat.set_potential(V, mu)
    lat.set_qubits([qubits_tensor(a, b)])
    lat.step(nsteps)
    got = lat.get_qubits()[0].cpu().numpy()
    ra, rb = oracle_qubits_ext(a, b, nsteps, eps, g, split, V, mu)
    err = rel_l2(got, np.stack([ra, rb]))
    assert err <= TOL[dtype], err


@pytest.mark.parametrize("ysplit", [0, 1])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("split", ["interleaved", "plain"])
@pytest.mark.parametrize("shape,rows", [((37, 130), 16), ((23, 57), 8), ((5, 200), 64), ((1, 1), 8)])
def test_2d_potential_random_qubits(dtype, split, shape, rows, ysplit):
    """V + mu on ragged 2D lattices in several band heights (the y pipeline's row ring), the y
    half in one launch or two."""
    ny, nx = shape
    g, eps, mu, nsteps = (1.1, -0.6, 0.7), 0.4, -0.8, 5
    a, b = qi.random_qubits(shape, seed=ny * 7 + nx, scale=0.4)
    V = smooth_potential(shape, seed=ny + nx)
    lat = lattice(2, [nx], [ny], g=g, eps=eps, dtype=dtype, split=split)
    lat.set_tuning(tile_rows=rows, qubit_split=ysplit)
    lat.set_potential(V, mu)
    lat.set_qubits([qubits_tensor(a, b)])
    lat.step(nsteps)
    got = lat.get_qubits()[0].cpu().numpy()
    ra, rb = oracle_qubits_ext(a, b, nsteps, eps, g, split, V, mu)
    err = rel_l2(got, np.stack([ra, rb]))
    assert err <= TOL[dtype], err


@pytest.mark.parametrize("ndim", [1, 2])
def test_batched_instances_own_potentials(ndim):
    """Each instance of a batch uses its own V (canonical scalar layout), FP64, with the energy."""
    g, eps, mu, nsteps = (1.0, -0.4, 0.6), 0.3, 0.25, 7
    shapes = [(300,), (64,), (129,)] if ndim == 1 else [(20, 70), (33, 17), (8, 130)]
    lat = lattice(ndim, [s[-1] for s in shapes], [s[0] for s in shapes] if ndim == 2 else None,
                  g=g, eps=eps, dtype="c128")
    psis = [qi.random_field(s, seed=50 + i, scale=0.4) for i, s in enumerate(shapes)]
    Vs = [smooth_potential(s, seed=60 + i) for i, s in enumerate(shapes)]
    lat.set_potential(Vs, mu)
    lat.set_psi([torch.from_numpy(p) for p in psis])
    lat.step(nsteps)
    obs = lat.observables()
    for i, (p, V) in enumerate(zip(psis, Vs)):
        A, B = O.run_psi(p, nsteps, eps, g, V=V, mu=mu)
        got = lat.get_psi()[i].cpu().numpy()
        assert rel_l2(got, (A + B).numpy()) <= 1e-12, i
        ref = O.observables(A, B, eps, g, V=V, mu=mu)
        assert abs(obs[i]["energy"] - ref["energy"]) <= 1e-11 * abs(ref["energy"]), (i, obs[i]["energy"], ref)


def test_harmonic_trap_on_gpu():
    """Free spinor in V = X^2/4 (omega = 1): the ground state's overlap energy is omega/2 and a
    displaced packet swings to -X0 after half a period, as in the oracle."""
    eps, X0 = 0.1, 2.0
    L = 200
    X = eps * (np.arange(L) - L / 2)
    V = X ** 2 / 4
    rng = np.random.default_rng(5)
    c = rng.normal(size=5) + 1j * rng.normal(size=5)
    lat = lattice(1, [L], g=(0.0, 0.0, 0.0), eps=eps, dtype="c128")
    lat.set_potential(V)
    lat.set_psi([torch.from_numpy(c[:, None] * np.exp(-X ** 2 / 4)[None, :])])
    lat.step(1)
    assert abs(lat.observables()[0]["e_overlap"].real / eps ** 2 - 0.5) < 1e-4
    lat.set_psi([torch.from_numpy(c[:, None] * np.exp(-(X - X0) ** 2 / 4)[None, :])])
    nhalf = int(round(np.pi / eps ** 2))
    lat.step(nhalf)
    n = (lat.get_psi()[0].abs() ** 2).sum(0).cpu().numpy()
    xm = float((n * X).sum() / n.sum())
    assert abs(xm - X0 * np.cos(nhalf * eps ** 2)) < 1e-3, xm


@pytest.mark.parametrize("ndim", [1, 2])
def test_chemical_potential_alone_is_a_global_phase(ndim):
    """mu without V (the kernels' uniform path): the run equals the mu = 0 run times e^{-i mu eps^2 n}."""
    shape = (150,) if ndim == 1 else (24, 70)
    g, eps, mu, nsteps = (1.1, -0.6, 0.7), 0.3, 1.3, 9
    psi = torch.from_numpy(qi.random_field(shape, seed=4, scale=0.5))
    runs = []
    for m in (0.0, mu):
        lat = lattice(ndim, [shape[-1]], [shape[0]] if ndim == 2 else None, g=g, eps=eps, dtype="c128")
        lat.set_potential(None, m)
        lat.set_psi([psi])
        lat.step(nsteps)
        runs.append(lat.get_qubits()[0].cpu().numpy())
    assert rel_l2(runs[1], runs[0] * np.exp(-1j * mu * eps ** 2 * nsteps)) <= 1e-12


@pytest.mark.parametrize("ndim", [1, 2])
def test_removing_the_potential_restores_plain_kernels(ndim):
    """After set_potential(None, 0) the step is bit-identical to a context that never had one."""
    shape = (300,) if ndim == 1 else (40, 90)
    g, eps = (1.1, -0.6, 0.7), 0.3
    psi = torch.from_numpy(qi.random_field(shape, seed=8, scale=0.5))
    out = []
    for with_pot in (False, True):
        lat = lattice(ndim, [shape[-1]], [shape[0]] if ndim == 2 else None, g=g, eps=eps, dtype="c64")
        if with_pot:
            lat.set_potential(smooth_potential(shape, seed=1), 0.4)
            lat.set_potential(None, 0.0)
        lat.set_psi([psi])
        lat.step(11)
        out.append(lat.get_qubits()[0].cpu())
    assert torch.equal(out[0], out[1])


def test_graph_replay_and_changing_values():
    """Graph replay with a potential equals direct launches; new values written into the same
    device array take effect at the next step (the pointer is kept, not the values)."""
    shape = (30, 80)
    g, eps = (1.0, -0.3, 0.5), 0.3
    psi = torch.from_numpy(qi.random_field(shape, seed=12, scale=0.5))
    V1, V2 = smooth_potential(shape, seed=21), smooth_potential(shape, seed=22)
    res = []
    for graph in (False, True):
        lat = lattice(2, [shape[1]], [shape[0]], g=g, eps=eps, dtype="c128")
        lat.set_tuning(use_graph=graph)
        lat.set_potential(V1, 0.2)
        lat.set_psi([psi])
        lat.step(4)
        lat.step(4)                                  # replays a captured graph when graph = True
        lat._pot.copy_(torch.from_numpy(V2).reshape(-1))
        lat.step(4)
        res.append(lat.get_qubits()[0].cpu().numpy())
    assert np.array_equal(res[0], res[1])
    A, B = O.run_psi(psi.numpy(), 8, eps, g, V=V1, mu=0.2)
    A, B = O.run(A, B, 4, eps, g, 2, V=V2, mu=0.2)
    assert rel_l2(res[0], np.stack([A.numpy(), B.numpy()])) <= 1e-12


def test_set_potential_argument_errors():
    from paper_1907_12834_amd.qlg import QLGError
    lat = lattice(1, [64], g=(1.0, -0.3, 0.5), eps=0.3, dtype="c128")
    with pytest.raises(QLGError, match="QLG_ERR_ARG"):
        lat.set_potential(None, float("nan"))
    with pytest.raises(ValueError):
        lat.set_potential(np.zeros(63))
