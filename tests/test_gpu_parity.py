"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances: FP64 kernels rel-L2 <= 1e-12; FP32 kernels rel-L2 <= 1e-4 and
qubit-norm drift <= 1e-5.  Sizes span several wave tiles and ragged tails;
full-size workloads are checked on light-cone windows the oracle can afford.
"""
import math
import os

import numpy as np
import pytest
import torch

import qlg_inputs as qi
from helpers import (light_cone_oracle_1d, light_cone_oracle_2d, oracle_psi, oracle_qubits, rel_l2)
from oracle import qlg_oracle as O

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-4}


def lattice(*args, **kw):
    from paper_1907_12834_amd.qlg import Lattice
    return Lattice(*args, **kw)


def qubits_tensor(a, b):
    return torch.from_numpy(np.stack([a, b]))


# ---------------------------------------------------------------------------
# 1D
# ---------------------------------------------------------------------------
def test_single_bright_L1024_fp64_1000_steps():
    """1D L=1024 bright soliton, complex128, 1000 steps: rel-L2 <= 1e-12, N_q to 1e-12."""
    w = qi.single_bright_1d_L1024()
    lat = lattice(1, [1024], g=w.g, eps=w.eps, dtype="c128")
    lat.set_psi([torch.from_numpy(w.psi[0])])
    obs0 = lat.observables()[0]
    lat.step(w.nsteps)
    got = lat.get_qubits()[0].cpu().numpy()
    a, b = oracle_psi(w.psi[0], w.nsteps, w.eps, w.g)
    err = rel_l2(got, np.stack([a, b]))
    obs = lat.observables()[0]
    print("single bright L=1024 fp64 rel-L2 after 1000 steps: %.3e" % err)
    assert err <= 1e-12
    assert abs(obs["norm_q"] / obs0["norm_q"] - 1) <= 1e-12


@pytest.mark.parametrize("qsplit", [0, 1, 2])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("split", ["interleaved", "plain"])
@pytest.mark.parametrize("steps_per_pass", [1, 2, 3, 4, 5, 6, 7])
def test_1d_random_qubits_ragged(dtype, split, steps_per_pass, qsplit):
    """Off-manifold random (a, b) on a ragged lattice (several tiles + tail), element-wise,
    with both qubits of a site in one lane, on two wavefronts and on two lanes (whose
    32-site tiles take at most 3 steps per pass)."""
    from paper_1907_12834_amd.qlg import QLGError
    L, nsteps = 437, 13
    g, eps = (1.2, -0.7, 0.9), 0.35
    a, b = qi.random_qubits((L,), seed=21, scale=0.5)
    lat = lattice(1, [L], g=g, eps=eps, dtype=dtype, split=split)
    if qsplit == 2 and steps_per_pass > 3:
        with pytest.raises(QLGError, match="QLG_ERR_ARG"):
            lat.set_tuning(steps_per_pass=steps_per_pass, qubit_split=qsplit)
        return
    lat.set_tuning(steps_per_pass=steps_per_pass, qubit_split=qsplit)
    lat.set_qubits([qubits_tensor(a, b)])
    lat.step(nsteps)
    got = lat.get_qubits()[0].cpu().numpy()
    ra, rb = oracle_qubits(a, b, nsteps, eps, g, split)
    err = rel_l2(got, np.stack([ra, rb]))
    assert err <= TOL[dtype], err


@pytest.mark.parametrize("qsplit", [0, 1, 2])
@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 15, 16, 17, 31, 32, 33, 63, 64, 65, 129])
def test_1d_tiny_and_edge_sizes(L, qsplit):
    """Lattices smaller than a tile wrap several times inside one wavefront."""
    g, eps, nsteps = (0.8, -0.4, 1.1), 0.3, 7
    a, b = qi.random_qubits((L,), seed=L, scale=0.6)
    lat = lattice(1, [L], g=g, eps=eps, dtype="c128")
    lat.set_tuning(steps_per_pass=2, qubit_split=qsplit)
    lat.set_qubits([qubits_tensor(a, b)])
    lat.step(nsteps)
    got = lat.get_qubits()[0].cpu().numpy()
    ra, rb = oracle_qubits(a, b, nsteps, eps, g)
    assert rel_l2(got, np.stack([ra, rb])) <= 1e-12


def test_1d_zero_steps_and_empty_field():
    lat = lattice(1, [100], g=(1, -0.5, 0.5), eps=0.1, dtype="c128")
    z = np.zeros((5, 100), complex)
    lat.set_psi([torch.from_numpy(z)])
    lat.step(0)
    lat.step(5)
    assert np.abs(lat.get_psi()[0].cpu().numpy()).max() == 0.0
    obs = lat.observables()[0]
    assert obs["norm_q"] == 0.0 and obs["energy"] == 0.0


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_two_solitons_reduced(dtype):
    """1D L=16384 two-soliton scattering workload, 100 steps, whole lattice vs the oracle."""
    w = qi.two_solitons_1d_L16384(nsteps=100)
    lat = lattice(1, [w.nx[0]], g=w.g, eps=w.eps, dtype=dtype)
    lat.set_psi([torch.from_numpy(w.psi[0])])
    o0 = lat.observables()[0]
    lat.step(w.nsteps)
    got = lat.get_psi()[0].cpu().numpy()
    a, b = oracle_psi(w.psi[0], w.nsteps, w.eps, w.g, key="two-solitons-L16384")
    err = rel_l2(got, a + b)
    o1 = lat.observables()[0]
    drift = abs(o1["norm_q"] / o0["norm_q"] - 1)
    print("two solitons L=16384 %s rel-L2 %.3e drift %.3e" % (dtype, err, drift))
    assert err <= TOL[dtype]
    assert drift <= (1e-12 if dtype == "c128" else 1e-5)


TWO_SOLITONS_REFERENCE = {
    -0.5: os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "two_solitons_L16384_oracle_psi.npz"),
    0.5: os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "two_solitons_L16384_c1_plus05_oracle_psi.npz")}


@pytest.mark.parametrize("c1", [-0.5, 0.5])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_two_solitons_L16384_parity_at_stated_lengths(dtype, c1):
    """The two-soliton workload in the autotuned launch plan, for both spin couplings c1 = -0.5
    and +0.5, against the oracle's own states after 2000 and 20000 steps (written by
    tests/golden/make_two_solitons_reference.py from the oracle alone)."""
    ref = np.load(TWO_SOLITONS_REFERENCE[c1])
    w = qi.two_solitons_1d_L16384(c1=c1)
    assert int(ref["L"]) == w.nx[0] and float(ref["eps"]) == w.eps and tuple(ref["g"]) == tuple(w.g)
    lat = lattice(1, [w.nx[0]], g=w.g, eps=w.eps, dtype=dtype)
    lat.autotune()
    lat.set_tuning(use_graph=True)
    lat.set_psi([torch.from_numpy(w.psi[0])])
    o0 = lat.observables()[0]
    done = 0
    for n in [int(v) for v in ref["steps"]]:
        trace = lat.run(n - done, every=100)
        done = n
        got = lat.get_psi()[0].cpu().numpy()
        err = rel_l2(got, ref["psi_%d" % n])
        drift = max(abs(o["norm_q"] / o0["norm_q"] - 1) for (o,) in trace)
        print("two solitons L=16384 %s plan %s: %d steps rel-L2 %.3e, worst norm drift %.3e" % (dtype, lat.tuning(), n, err, drift))
        assert err <= TOL[dtype], (n, err)
        assert drift <= (1e-11 if dtype == "c128" else 1e-5), (n, drift)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_two_solitons_L16384_full_length_invariants(dtype):
    """The full length of the L = 16384 two-soliton run (20000 steps) on the GPU: qubit norm and energy are tracked every 100 steps."""
    w = qi.two_solitons_1d_L16384()
    lat = lattice(1, [w.nx[0]], g=w.g, eps=w.eps, dtype=dtype)
    lat.autotune()
    lat.set_psi([torch.from_numpy(w.psi[0])])
    o0 = lat.observables()[0]
    worst = 0.0
    energies = []
    for _ in range(w.nsteps // 100):
        lat.step(100)
        o = lat.observables()[0]
        worst = max(worst, abs(o["norm_q"] / o0["norm_q"] - 1))
        energies.append(o["energy"])
    print("two solitons L=16384 %s 20000 steps: worst norm drift %.3e, energy %.6f -> %.6f" %
          (dtype, worst, o0["energy"], energies[-1]))
    assert worst <= (1e-11 if dtype == "c128" else 1e-5)
    assert all(math.isfinite(e) for e in energies)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_two_solitons_L16384_light_cone_samples(dtype):
    """Full-size lattice in the autotuned launch configuration, sampled sites vs light-cone oracle."""
    w = qi.two_solitons_1d_L16384()
    nsteps = 40
    lat = lattice(1, [w.nx[0]], g=w.g, eps=w.eps, dtype=dtype)
    lat.autotune()
    lat.set_psi([torch.from_numpy(w.psi[0])])
    lat.step(nsteps)
    got = lat.get_psi()[0].cpu().numpy()
    L = w.nx[0]
    for xc in (L // 2 - L // 8, L // 2 + L // 8 + 17, 0, L - 1):
        ref = light_cone_oracle_1d(w.psi[0], xc, nsteps, w.eps, w.g)
        scale = max(np.abs(ref).max(), 1e-3)
        assert np.abs(got[:, xc] - ref).max() / scale <= (1e-12 if dtype == "c128" else 1e-4)


# ---------------------------------------------------------------------------
# Observables
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ndim,plan", [(1, None), (1, (3, 1)), (1, (2, 2)), (1, (3, 2)), (2, None), (2, (1, 1))])
def test_observables_match_oracle(ndim, plan):
    """Observables and the overlap energy of the last step (recorded by the step kernel of the
    plan: steps per pass, qubit split; in 2D qubit split 1 is the y half over two launches)
    against the oracle."""
    g, eps, nsteps = (1.0, -0.5, 0.5), 0.2, 9
    shape = (300,) if ndim == 1 else (19, 70)
    a, b = qi.random_qubits(shape, seed=33, scale=0.4)
    lat = lattice(ndim, [shape[-1]], [shape[0]] if ndim == 2 else None, g=g, eps=eps, dtype="c128")
    if plan:
        lat.set_tuning(steps_per_pass=plan[0], qubit_split=plan[1])
    lat.set_qubits([qubits_tensor(a, b)])
    lat.step(nsteps)
    got = lat.observables()[0]
    ra, rb = oracle_qubits(a, b, nsteps - 1, eps, g)
    prev = torch.from_numpy(ra + rb)
    A, B = O.step(torch.from_numpy(ra), torch.from_numpy(rb), eps, g, ndim)
    ref = O.observables(A, B, eps, g, prev_psi=prev)
    for k in ("norm_q", "norm_psi", "energy"):
        assert abs(got[k] - ref[k]) <= 1e-12 * abs(ref[k]), k
    assert np.allclose(got["pop"], ref["pop"], rtol=1e-12, atol=0)
    ovr = ref["e_overlap"]
    assert abs(got["e_overlap"] - ovr) <= 1e-12 * max(abs(ovr), 1e-3)


@pytest.mark.parametrize("ndim", [1, 2])
def test_recorded_observables_equal_synchronous_ones(ndim):
    """Device-side records, decoded later, give exactly qlg_observables' values and flags."""
    g, eps = (1.0, -0.5, 0.5), 0.2
    shapes = [(300,), (77,)] if ndim == 1 else [(19, 70), (9, 33)]
    qbs = [qubits_tensor(*qi.random_qubits(sh, seed=60 + i, scale=0.4)) for i, sh in enumerate(shapes)]
    nx = [sh[-1] for sh in shapes]
    ny = [sh[0] for sh in shapes] if ndim == 2 else None
    lat = lattice(ndim, nx, ny, g=g, eps=eps, dtype="c128")
    lat.set_qubits(qbs)
    rec = lat.new_records(4)
    lat.record_observables(rec, 0)
    sync = [lat.observables()]
    for k, n in enumerate((3, 1, 5), start=1):
        lat.step(n)
        lat.record_observables(rec, k)
        sync.append(lat.observables())
    dec = lat.decode_records(rec)
    assert [o["step"] for o in dec[0]] == [0, 0] and not any("e_overlap" in o for o in dec[0])
    assert [o["step"] for o in dec[3]] == [9, 9] and all("e_overlap" in o for o in dec[3])
    for r in range(4):
        for i in range(2):
            a, b = dec[r][i], sync[r][i]
            assert a.keys() == b.keys()
            for key in a:
                assert np.array_equal(np.asarray(a[key]), np.asarray(b[key])), (r, i, key)
    # `run` records every k steps with one synchronisation; same values as stepping by hand
    lat.set_qubits(qbs)
    trace = lat.run(10, every=5)
    lat.set_qubits(qbs)
    lat.step(5)
    lat.step(5)
    ref = lat.observables()
    assert len(trace) == 2 and trace[1][0]["energy"] == ref[0]["energy"] and trace[1][1]["step"] == 10
    # a non-finite record is reported by the decoder
    bad = rec.cpu().clone()
    bad[2, 1, 0] = float("nan")
    from paper_1907_12834_amd.qlg import QLGError
    with pytest.raises(QLGError):
        lat.decode_records(bad)


def test_bright_soliton_overlap_energy_on_gpu():
    """Re E_ov / eps^2 -> -K^2 for the Table I row-1 bright soliton (dispersion at p = 0)."""
    wdt = 24
    eps = 1.0 / wdt
    L = 40 * wdt
    X = (np.arange(L) - L / 2) * eps
    c = qi.table1_coeffs(1, -2.0, 1.0, -0.5, 0.5).real
    psi = c[:, None] * (1.0 / np.cosh(X))[None, :]
    lat = lattice(1, [L], g=(1.0, -0.5, 0.5), eps=eps, dtype="c128")
    lat.set_psi([torch.from_numpy(psi)])
    lat.step(41)
    e = lat.observables()[0]["e_overlap"].real / eps ** 2
    assert abs(e + 1.0) < 0.01


# ---------------------------------------------------------------------------
# 2D
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("ysplit", [0, 1])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("split", ["interleaved", "plain"])
@pytest.mark.parametrize("shape,rows", [((37, 130), 16), ((23, 57), 8), ((70, 9), 32), ((2, 4), 8),
                                        ((1, 1), 8), ((5, 200), 64)])
def test_2d_random_qubits(dtype, split, shape, rows, ysplit):
    """Ragged 2D lattices in several band heights, the y half in one launch or two."""
    ny, nx = shape
    g, eps, nsteps = (1.1, -0.6, 0.7), 0.4, 5
    a, b = qi.random_qubits(shape, seed=ny * 1000 + nx, scale=0.5)
    lat = lattice(2, [nx], [ny], g=g, eps=eps, dtype=dtype, split=split)
    lat.set_tuning(tile_rows=rows, qubit_split=ysplit)
    lat.set_qubits([qubits_tensor(a, b)])
    lat.step(nsteps)
    got = lat.get_qubits()[0].cpu().numpy()
    ra, rb = oracle_qubits(a, b, nsteps, eps, g, split)
    err = rel_l2(got, np.stack([ra, rb]))
    assert err <= TOL[dtype], err


@pytest.mark.parametrize("use_graph", [False, True])
def test_y_split_switched_mid_run(use_graph):
    """The y half in one launch or two leaves the state in different copies of the ping-pong
    pair; switching the plan between steps keeps the state (against the oracle)."""
    shape = (30, 50)
    g, eps = (1.0, -0.5, 0.5), 0.3
    a, b = qi.random_qubits(shape, seed=17, scale=0.5)
    lat = lattice(2, [shape[1]], [shape[0]], g=g, eps=eps, dtype="c128")
    lat.set_tuning(tile_rows=8, use_graph=use_graph)
    lat.set_qubits([qubits_tensor(a, b)])
    for n, ysplit in ((3, 0), (4, 1), (1, 1), (2, 0), (5, 1)):
        lat.set_tuning(qubit_split=ysplit)
        lat.step(n)
    got = lat.get_qubits()[0].cpu().numpy()
    ra, rb = oracle_qubits(a, b, 15, eps, g)
    assert rel_l2(got, np.stack([ra, rb])) <= 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_vortex_pair_256_reduced(dtype):
    """2D vortex-pair workload on 256^2 (the 2048^2 construction: separation 128, eps = 0.1,
    seeded Pade cores), 200 steps in the autotuned plan, the whole lattice vs the oracle."""
    rng = np.random.default_rng(2019)
    psi = qi.vortex_pair_2d(256, 256, 128.0, 0.1, rng)
    g, eps, nsteps = (1.0, -0.3, 0.2), 0.1, 200
    lat = lattice(2, [256], [256], g=g, eps=eps, dtype=dtype)
    lat.autotune()
    lat.set_psi([torch.from_numpy(psi)])
    o0 = lat.observables()[0]
    lat.step(nsteps)
    got = lat.get_psi()[0].cpu().numpy()
    a, b = oracle_psi(psi, nsteps, eps, g, key="vortex-pair-256")
    err = rel_l2(got, a + b)
    drift = abs(lat.observables()[0]["norm_q"] / o0["norm_q"] - 1)
    print("vortex pair 256^2 %s plan %s rel-L2 %.3e drift %.3e" % (dtype, lat.tuning(), err, drift))
    assert err <= TOL[dtype]
    assert drift <= (1e-12 if dtype == "c128" else 1e-5)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_vortex_pair_2048_light_cone_samples(dtype):
    """2048^2 in the autotuned configuration (the benchmark's launch configuration for each
    storage type, hipGraph replay included), 20 steps, light-cone windows vs the oracle: the
    vortex cores, the lattice's corners and wrap, and a window across a band boundary and a
    column-tile boundary of the plan."""
    w = qi.vortex_pair_2d_2048()
    nsteps = 20
    lat = lattice(2, [2048], [2048], g=w.g, eps=w.eps, dtype=dtype)
    lat.autotune()
    rows = lat.tuning()["tile_rows"]
    lat.set_psi([torch.from_numpy(w.psi[0])])
    lat.step(nsteps)
    got = lat.get_psi()[0].cpu().numpy()
    band = rows * (2048 // rows // 2)            # the first row of a band in the middle
    for cy, cx in ((1024, 1024 - 64), (1024, 1024 + 64), (0, 0), (2047, 1500), (band, 56 * 18)):
        ref = light_cone_oracle_2d(w.psi[0], cy, cx, nsteps, w.eps, w.g, half_out=2)
        sub = got[:, (np.arange(cy - 2, cy + 3) % 2048)[:, None], (np.arange(cx - 2, cx + 3) % 2048)[None, :]]
        assert rel_l2(sub, ref) <= (1e-12 if dtype == "c128" else 1e-4), (cy, cx, rel_l2(sub, ref))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_spin_texture_2048_light_cone_samples(dtype):
    """The 2048^2 workload with a seeded complex Gaussian spinor of amplitude 0.05 added to every
    component (the adjoint's spin-texture recipe): m = +-1 are populated and F != 0 at every site,
    so the spin rotation of the self-interaction acts everywhere (the vortex pair alone keeps
    F = 0).  Autotuned configuration, 20 steps, light-cone windows vs the oracle."""
    w = qi.vortex_pair_2d_2048()
    psi = w.psi[0] + qi.random_field((2048, 2048), seed=79, scale=0.05)
    nsteps = 20
    lat = lattice(2, [2048], [2048], g=w.g, eps=w.eps, dtype=dtype)
    lat.autotune()
    lat.set_psi([torch.from_numpy(psi)])
    lat.step(nsteps)
    got = lat.get_psi()[0].cpu().numpy()
    for cy, cx in ((1024, 1024 - 64), (300, 1700), (2047, 0)):
        ref = light_cone_oracle_2d(psi, cy, cx, nsteps, w.eps, w.g, half_out=2)
        fz = 2 * (np.abs(ref[0]) ** 2 - np.abs(ref[4]) ** 2) + np.abs(ref[1]) ** 2 - np.abs(ref[3]) ** 2
        fp = 2 * np.conj(ref[0]) * ref[1] + 6 ** 0.5 * (np.conj(ref[1]) * ref[2] + np.conj(ref[2]) * ref[3]) \
            + 2 * np.conj(ref[3]) * ref[4]
        assert np.min(np.sqrt(fz ** 2 + np.abs(fp) ** 2)) > 1e-3     # the spin factor is not the identity
        sub = got[:, (np.arange(cy - 2, cy + 3) % 2048)[:, None], (np.arange(cx - 2, cx + 3) % 2048)[None, :]]
        assert rel_l2(sub, ref) <= TOL[dtype], (cy, cx, rel_l2(sub, ref))


# ---------------------------------------------------------------------------
# Batched, graphs, autotune
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("plan", [(3, 0), (2, 1), (2, 2)])
def test_batched_equals_individual_and_oracle(dtype, plan):
    """Batched and one-at-a-time runs under the same plan (steps per pass, kernel variant) are
    bit-identical; the two kernel variants round in different orders, so the plan is pinned."""
    S, qsplit = plan
    w = qi.batched_two_solitons_1d_256(nbatch=8, nsteps=1000)
    lat = lattice(1, w.nx, g=w.g, eps=w.eps, dtype=dtype)
    lat.set_tuning(steps_per_pass=S, qubit_split=qsplit)
    lat.set_psi([torch.from_numpy(p) for p in w.psi])
    lat.step(w.nsteps)
    got = [t.cpu().numpy() for t in lat.get_psi()]
    for i in (0, 3, 7):
        one = lattice(1, [w.nx[i]], g=w.g, eps=w.eps, dtype=dtype)
        one.set_tuning(steps_per_pass=S, qubit_split=qsplit)
        one.set_psi([torch.from_numpy(w.psi[i])])
        one.step(w.nsteps)
        alone = one.get_psi()[0].cpu().numpy()
        assert np.array_equal(alone, got[i]), i    # same kernels, same arithmetic: bit-identical
    i = int(np.argmin(w.nx))
    a, b = oracle_psi(w.psi[i], w.nsteps, w.eps, w.g, key="batched-smallest")
    assert rel_l2(got[i], a + b) <= TOL[dtype]


def test_batched_256_full_size_light_cone_samples():
    """The full 256-instance batch (2.3 M sites) in the autotuned plan, 40 steps: sites of the
    smallest, the largest and random instances (on the solitons, random, at the periodic seam)
    against the oracle on light-cone windows (radius 4 per step), and every qubit norm kept."""
    w = qi.batched_two_solitons_1d_256(nsteps=40)
    nsteps = 40
    lat = lattice(1, w.nx, g=w.g, eps=w.eps, dtype="c64")
    lat.set_psi([torch.from_numpy(p) for p in w.psi])
    lat.autotune()
    o0 = lat.observables()
    lat.step(nsteps)
    o1 = lat.observables()
    got = lat.get_psi()
    half = 4 * nsteps + 2
    rng = np.random.default_rng(7)
    inst = [int(np.argmin(w.nx)), int(np.argmax(w.nx))] + [int(v) for v in rng.integers(0, w.nbatch, size=3)]
    for i in inst:
        L = w.nx[i]
        peak = np.abs(w.psi[i]).max()
        for c in (L // 2 - L // 8, L // 2 + L // 8, int(rng.integers(0, L)), 0, L - 1):
            idx = np.arange(c - half, c + half + 1) % L
            A, B = O.run_psi(w.psi[i][:, idx], nsteps, w.eps, w.g)
            ref = (A + B).numpy()[:, half]
            g_ = got[i][:, c].cpu().numpy()
            assert np.abs(g_ - ref).max() <= 1e-5 * peak, (i, c, g_, ref)
    for i in range(w.nbatch):
        assert abs(o1[i]["norm_q"] / o0[i]["norm_q"] - 1) <= 1e-5, i


def test_batched_2d_uneven():
    g, eps, nsteps = (1.0, -0.3, 0.2), 0.3, 4
    shapes = [(20, 33), (9, 70), (64, 64)]
    fields = [qi.random_qubits(s, seed=i, scale=0.5) for i, s in enumerate(shapes)]
    lat = lattice(2, [s[1] for s in shapes], [s[0] for s in shapes], g=g, eps=eps, dtype="c128")
    lat.set_qubits([qubits_tensor(a, b) for a, b in fields])
    lat.step(nsteps)
    got = [t.cpu().numpy() for t in lat.get_qubits()]
    for (a, b), gq in zip(fields, got):
        ra, rb = oracle_qubits(a, b, nsteps, eps, g)
        assert rel_l2(gq, np.stack([ra, rb])) <= 1e-12


@pytest.mark.parametrize("ndim,qsplit", [(1, 0), (1, 1), (1, 2), (2, 0), (2, 1)])
def test_graph_replay_equals_eager(ndim, qsplit):
    shape = (777,) if ndim == 1 else (40, 90)
    a, b = qi.random_qubits(shape, seed=5, scale=0.5)
    res = []
    for use_graph in (False, True):
        lat = lattice(ndim, [shape[-1]], [shape[0]] if ndim == 2 else None, g=(1, -0.5, 0.5), eps=0.3,
                      dtype="c64")
        lat.set_tuning(use_graph=use_graph, steps_per_pass=2 if ndim == 1 else None, qubit_split=qsplit)
        lat.set_qubits([qubits_tensor(a, b)])
        outs = []
        for rep in range(3):   # replay the same captured graph several times, with eager work between
            lat.step(6)
            outs.append(lat.get_qubits()[0].cpu().numpy())
            _ = lat.observables()
        res.append(outs)
    for e, gr in zip(res[0], res[1]):
        assert np.array_equal(e, gr)


def test_autotune_keeps_state():
    w = qi.single_bright_1d_L1024(L=2048)
    lat = lattice(1, [2048], g=w.g, eps=w.eps, dtype="c64")
    lat.set_psi([torch.from_numpy(w.psi[0])])
    before = lat.get_qubits()[0].cpu().numpy()
    t = lat.autotune()
    after = lat.get_qubits()[0].cpu().numpy()
    assert np.array_equal(before, after)
    assert 1 <= t["steps_per_pass"] <= 7
