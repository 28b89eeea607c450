"""GPU parity of the 3D step (Lie product n = 12; a z pass and a y-x pass per step).

The HIP path through the C ABI against the FP64 oracle's 3D step: FP64 rel-L2
<= 1e-12, FP32 <= 1e-4, element by element on ragged lattices (several 64-lane
tiles along x with a tail, bands with a tail along y and z, 1-site extents) in
several band heights, both splits; batched 3D instances of different sizes;
observables and the overlap energy; a potential; graph replay; the exact
reduction of a z-uniform free field to the 2D step; the 256^3 and 512^3
vortex-line states at full size on light-cone windows; and the lattice
vorticity of the three plane families and their vortex-core lists.
"""
import numpy as np
import pytest
import torch

import qlg_inputs as qi
from helpers import rel_l2
from oracle import qlg_oracle as O

pytestmark = pytest.mark.gpu

TOL = {"c128": 1e-12, "c64": 1e-4}


def lattice3(shapes, **kw):
    from paper_1907_12834_amd.qlg import Lattice
    return Lattice(3, [s[2] for s in shapes], [s[1] for s in shapes], [s[0] for s in shapes], **kw)


def oracle_qubits3(a, b, nsteps, eps, g, split="interleaved", V=None, mu=0.0):
    A, B = O.run(torch.from_numpy(np.ascontiguousarray(a)), torch.from_numpy(np.ascontiguousarray(b)),
                 nsteps, eps, g, 3, split, V=V, mu=mu)
    return A.numpy(), B.numpy()


@pytest.mark.parametrize("ysplit", [0, 1])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("split", ["interleaved", "plain"])
@pytest.mark.parametrize("shape,rows", [((5, 7, 70), 8), ((9, 3, 130), 16), ((17, 2, 9), 8),
                                        ((3, 20, 64), 16), ((1, 1, 1), 8), ((2, 1, 65), 8)])
def test_3d_random_qubits(dtype, split, shape, rows, ysplit):
    """Ragged 3D lattices; ysplit 1: the z and the y half each over two launches."""
    g, eps, nsteps = (1.1, -0.6, 0.7), 0.45, 3
    a, b = qi.random_qubits(shape, seed=sum(shape) * 13 + rows, scale=0.4)
    lat = lattice3([shape], g=g, eps=eps, dtype=dtype, split=split)
    lat.set_tuning(tile_rows=rows, qubit_split=ysplit)
    lat.set_qubits([torch.from_numpy(np.stack([a, b]))])
    lat.step(nsteps)
    got = lat.get_qubits()[0].cpu().numpy()
    ra, rb = oracle_qubits3(a, b, nsteps, eps, g, split)
    err = rel_l2(got, np.stack([ra, rb]))
    assert err <= TOL[dtype], err


@pytest.mark.parametrize("ysplit", [0, 1])
def test_3d_batched_instances_and_observables(ysplit):
    """Three 3D instances of different shape in one context; every state and every observable
    (norms, populations, energy, overlap energy) against the oracle."""
    shapes = [(6, 5, 70), (3, 9, 20), (11, 2, 3)]
    g, eps, nsteps = (1.0, -0.4, 0.6), 0.4, 4
    psis = [qi.random_field(s, seed=70 + i, scale=0.4) for i, s in enumerate(shapes)]
    lat = lattice3(shapes, g=g, eps=eps, dtype="c128")
    lat.set_tuning(tile_rows=8, qubit_split=ysplit)
    lat.set_psi([torch.from_numpy(p) for p in psis])
    lat.step(nsteps - 1)
    prev = [p.cpu().numpy() for p in lat.get_psi()]
    lat.step(1)
    obs = lat.observables()
    got = [p.cpu().numpy() for p in lat.get_psi()]
    for i, p in enumerate(psis):
        A, B = O.run_psi(p, nsteps, eps, g)
        assert rel_l2(got[i], (A + B).numpy()) <= 1e-12, i
        ref = O.observables(A, B, eps, g, prev_psi=torch.from_numpy(prev[i]))
        o = obs[i]
        assert abs(o["norm_q"] - ref["norm_q"]) <= 1e-12 * ref["norm_q"]
        assert np.allclose(o["pop"], ref["pop"], rtol=1e-12, atol=0)
        assert abs(o["energy"] - ref["energy"]) <= 1e-11 * abs(ref["energy"]), (o["energy"], ref["energy"])
        assert abs(o["e_overlap"] - ref["e_overlap"]) <= 1e-10 * abs(ref["e_overlap"]), i


def test_3d_uniform_state_pure_phase():
    """A uniform Table I state: each step is the pure phase e^{-i E eps^2} (Sec. IV), in the overlap energy."""
    E, eps, g = 2.0, 0.1, (1.0, 0.1, 0.7)
    c = qi.table1_coeffs(6, E, *g).real
    shape = (9, 5, 70)
    lat = lattice3([shape], g=g, eps=eps, dtype="c128")
    lat.set_psi([torch.from_numpy(np.tile(c[:, None, None, None], (1,) + shape).astype(complex))])
    lat.step(10)
    e = lat.observables()[0]["e_overlap"]
    # <psi_t|psi_{t-1}> = e^{i E eps^2} <psi_t|psi_t> exactly, so E_ov = i (1 - e^{i E eps^2})
    assert abs(e - 1j * (1 - np.exp(1j * E * eps ** 2))) < 1e-12, e


def test_3d_free_z_uniform_equals_2d():
    """Free (g = 0) z-uniform field: the 3D step is the 2D step (four SWAPs along z)."""
    from paper_1907_12834_amd.qlg import Lattice
    ny, nx, nz, eps, nsteps = 13, 75, 4, 0.3, 6
    a, b = qi.random_qubits((ny, nx), seed=17, scale=0.5)
    lat2 = Lattice(2, [nx], [ny], g=(0.0, 0.0, 0.0), eps=eps, dtype="c128")
    lat2.set_qubits([torch.from_numpy(np.stack([a, b]))])
    lat2.step(nsteps)
    ref = lat2.get_qubits()[0].cpu().numpy()
    lat3 = lattice3([(nz, ny, nx)], g=(0.0, 0.0, 0.0), eps=eps, dtype="c128")
    lat3.set_qubits([torch.from_numpy(np.stack([np.repeat(a[:, None], nz, 1), np.repeat(b[:, None], nz, 1)]))])
    lat3.step(nsteps)
    got = lat3.get_qubits()[0].cpu().numpy()
    for k in range(nz):
        assert np.abs(got[:, :, k] - ref).max() < 1e-13


def test_3d_harmonic_trap_and_mu():
    """3D potential: parity with the oracle, and an isotropic trap's ground state E = 3 omega/2 + mu."""
    shape, g, eps, mu = (6, 7, 66), (1.0, -0.5, 0.4), 0.4, 0.3
    a, b = qi.random_qubits(shape, seed=23, scale=0.4)
    V = np.random.default_rng(4).uniform(0.0, 2.0, size=shape)
    lat = lattice3([shape], g=g, eps=eps, dtype="c128")
    lat.set_potential(V, mu)
    lat.set_qubits([torch.from_numpy(np.stack([a, b]))])
    lat.step(3)
    ra, rb = oracle_qubits3(a, b, 3, eps, g, V=V, mu=mu)
    assert rel_l2(lat.get_qubits()[0].cpu().numpy(), np.stack([ra, rb])) <= 1e-12
    n, eps = 40, 0.25
    X = eps * (np.arange(n) - n / 2)
    r2 = X[:, None, None] ** 2 + X[None, :, None] ** 2 + X[None, None, :] ** 2
    lat = lattice3([(n, n, n)], g=(0.0, 0.0, 0.0), eps=eps, dtype="c128")
    lat.set_potential(r2 / 4, mu)
    c = np.random.default_rng(6).normal(size=5) + 0j
    lat.set_psi([torch.from_numpy(c[:, None, None, None] * np.exp(-r2 / 4)[None])])
    lat.step(1)
    e = lat.observables()[0]["e_overlap"].real / eps ** 2
    assert abs(e - (1.5 + mu)) < 2e-2, e     # second order in eps (the 2D trap pins the order)


def test_3d_graph_replay_and_autotune_keep_results():
    """Graph replay and an autotune between steps change nothing: every plan computes each site
    with the same arithmetic, and the autotuner's timing passes leave the state alone."""
    shape = (10, 12, 70)
    g, eps = (1.0, -0.3, 0.5), 0.4
    psi = torch.from_numpy(qi.random_field(shape, seed=31, scale=0.4))
    res = []
    for variant in ("direct", "graph", "autotune"):
        lat = lattice3([shape], g=g, eps=eps, dtype="c64")
        lat.set_tuning(tile_rows=16, use_graph=(variant == "graph"))
        lat.set_psi([psi])
        lat.step(3)
        if variant == "autotune":
            lat.autotune()
            assert lat.tuning()["steps_per_pass"] == 1
        lat.step(3)
        lat.step(3)
        res.append(lat.get_qubits()[0].cpu())
    assert torch.equal(res[0], res[1]) and torch.equal(res[0], res[2])


def test_3d_vortex_lines_full_size_light_cone():
    """The 256^3 vortex-line workload (complex64) after 3 steps in the autotuned plan: sampled
    sites against the oracle on periodic light-cone windows (radius 4 per step per axis)."""
    w = qi.vortex_lines_3d_256(nsteps=3)
    n = w.nx[0]
    lat = lattice3([(n, n, n)], g=w.g, eps=w.eps, dtype="c64")
    lat.set_psi([torch.from_numpy(w.psi[0])])
    lat.autotune()
    lat.step(3)
    got = lat.get_psi()[0]
    half = 4 * 3 + 2
    rng = np.random.default_rng(0)
    pts = [(n // 2, n // 2, n // 2 - 32), (0, 0, 0), (n - 1, 17, n - 1)] + \
          [tuple(int(v) for v in rng.integers(0, n, size=3)) for _ in range(2)]
    for (cz, cy, cx) in pts:
        idx = [np.arange(c - half, c + half + 1) % n for c in (cz, cy, cx)]
        win = w.psi[0][:, idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]]
        A, B = O.run_psi(win, 3, w.eps, w.g)
        ref = (A + B).numpy()[:, half, half, half]
        g_ = got[:, cz, cy, cx].cpu().numpy()
        assert np.abs(g_ - ref).max() <= 1e-5 * np.abs(ref).max(), (cz, cy, cx, g_, ref)
    o = lat.observables()[0]
    # encoded as a = b = psi / 2, so the conserved qubit norm is eps^3 sum |psi|^2 / 2
    assert abs(o["norm_q"] / (0.5 * w.eps ** 3 * (np.abs(w.psi[0]) ** 2).sum()) - 1) < 1e-5


def test_3d_vortex_lines_512_light_cone():
    """The largest cube the paper names, 512^3 (the vortex-line state; complex64, 21.5 GB of qubit
    state in two copies): 2 steps in the autotuned plan, sampled sites against the oracle on
    periodic light-cone windows, and the qubit norm."""
    w = qi.vortex_lines_3d_512(nsteps=2)
    n = w.nx[0]
    lat = lattice3([(n, n, n)], g=w.g, eps=w.eps, dtype="c64")
    lat.set_psi([torch.from_numpy(w.psi[0])])
    lat.autotune()
    lat.step(2)
    got = lat.get_psi()[0]
    half = 4 * 2 + 2
    rng = np.random.default_rng(1)
    pts = [(n // 2, n // 2, n // 2 - 64), (n - 1, n - 1, n - 1), (3, n // 2, n // 2 + 64)] + \
          [tuple(int(v) for v in rng.integers(0, n, size=3)) for _ in range(2)]
    for (cz, cy, cx) in pts:
        idx = [np.arange(c - half, c + half + 1) % n for c in (cz, cy, cx)]
        win = w.psi[0][:, idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]]
        A, B = O.run_psi(win, 2, w.eps, w.g)
        ref = (A + B).numpy()[:, half, half, half]
        g_ = got[:, cz, cy, cx].cpu().numpy()
        assert np.abs(g_ - ref).max() <= 1e-5 * np.abs(ref).max(), (cz, cy, cx, g_, ref)
    o = lat.observables()[0]
    assert abs(o["norm_q"] / (0.5 * w.eps ** 3 * (np.abs(w.psi[0]) ** 2).sum()) - 1) < 1e-5
    # the fused vorticity pass at 8192 workgroups (tiles regrouped by XCD): sampled planes of
    # each family against the oracle's 2D rule on the GPU's own psi of m = +2, sliced on the device
    r = lat.vorticity(0)[0]
    psi0 = got[0]
    for k in (0, 257, n - 1):
        for c, sel in ((0, lambda a: a[..., k]), (1, lambda a: a[:, k, :].T), (2, lambda a: a[k])):
            o2, w2 = O.vorticity(sel(psi0).cpu().numpy())
            assert np.array_equal(sel(r["winding"][c]).cpu().numpy(), w2), (c, k)
            assert np.abs(sel(r["omega"][c]).cpu().numpy() - o2).max() <= 1e-12, (c, k)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_3d_vorticity_random_ragged_batch(dtype):
    """The three plane families of a 3D state (instances of different shapes, 1- and 2-site
    extents included) against the oracle on the GPU's own psi: windings exact, omega to rounding
    (both sides take the same FP64 differences of the same phases in the same order).  The
    shapes put ragged 64-site x tiles, 16-row y tiles and 16-slice z runs at the edges; the
    17 x 17 x 65 instance has eight workgroups, the case whose tiles are regrouped by XCD."""
    shapes = [(5, 7, 70), (3, 20, 9), (1, 1, 1), (2, 1, 65), (34, 3, 2), (17, 17, 65)]
    lat = lattice3(shapes, g=(1.0, -0.3, 0.5), eps=0.4, dtype=dtype)
    lat.set_psi([torch.from_numpy(qi.random_field(sh, seed=80 + i)) for i, sh in enumerate(shapes)])
    lat.step(2)
    psi = [p.cpu().numpy() for p in lat.get_psi()]
    for m in (0, 3):
        res = lat.vorticity(m)
        for i, sh in enumerate(shapes):
            om, wd = O.vorticity(psi[i][m])
            assert res[i]["omega"].shape == (3,) + sh and res[i]["winding"].shape == (3,) + sh
            assert np.array_equal(res[i]["winding"].cpu().numpy(), wd), (m, i)
            assert np.abs(res[i]["omega"].cpu().numpy() - om).max() <= 1e-12, (m, i)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_3d_vortex_lines_vorticity_full_size(dtype):
    """The 256^3 vortex-line workload after 3 steps: windings and omega of sampled planes of each
    family against the oracle's lattice vorticity of that plane."""
    w = qi.vortex_lines_3d_256(nsteps=3)
    n = w.nx[0]
    lat = lattice3([(n, n, n)], g=w.g, eps=w.eps, dtype=dtype)
    lat.set_psi([torch.from_numpy(w.psi[0])])
    lat.step(3)
    psi0 = lat.get_psi()[0][0].cpu().numpy()          # m = +2, [z][y][x]
    r = lat.vorticity(0)[0]
    om, wd = r["omega"].cpu().numpy(), r["winding"].cpu().numpy()
    for k in (0, 100, 255):
        # normal x: the (z, y) plane circulated y -> z; normal y: (x, z) circulated z -> x;
        # normal z: (y, x) circulated x -> y -- the oracle's 2D rule with u = axis 1, v = axis 0
        for c, plane, back in ((0, psi0[:, :, k], lambda a: a[:, :, k]),
                               (1, psi0[:, k, :].T, lambda a: a[:, k, :].T),
                               (2, psi0[k], lambda a: a[k])):
            o2, w2 = O.vorticity(plane)
            assert np.array_equal(back(wd[c]), w2), (c, k)
            assert np.abs(back(om[c]) - o2).max() <= 1e-12, (c, k)
    # the +1 line of m = +2 crosses every z plane; the periodic lattice's windings sum to zero
    for z in (0, 64, 128, 255):
        assert (wd[2, z] == 1).any() and int(wd[2, z].sum()) == 0


def oracle_cores3(psis, m_index):
    """(instance, family, z, y, x, winding) of every non-zero winding of the oracle's three plane
    families, in (family, instance, z, y, x) order."""
    per = [O.vorticity(p[m_index])[1] for p in psis]
    rows = []
    for c in range(3):
        for i, wd in enumerate(per):
            rows += [(i, c, int(z), int(y), int(x), int(wd[c, z, y, x])) for z, y, x in np.argwhere(wd[c])]
    return np.array(rows, dtype=np.int64).reshape(-1, 6)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_3d_find_vortices_ragged_batch(dtype):
    """Core lists of the three plane families of random fields on ragged 3D instances (1-site
    extents included) equal the oracle's, entry by entry and in order; a capacity below the count
    writes the first entries and reports the full count; the winding output holds all three
    families."""
    from paper_1907_12834_amd.qlg import lib
    shapes = [(5, 7, 70), (3, 20, 9), (1, 1, 1), (2, 1, 65), (17, 17, 65)]
    lat = lattice3(shapes, g=(1.0, -0.3, 0.5), eps=0.4, dtype=dtype)
    lat.set_psi([torch.from_numpy(qi.random_field(sh, seed=90 + i)) for i, sh in enumerate(shapes)])
    lat.step(2)
    psis = [p.cpu().numpy() for p in lat.get_psi()]
    for m in (0, 3):
        ref = oracle_cores3(psis, m)
        assert len(ref) > 1000 and set(ref[:, 1]) == {0, 1, 2}
        got = lat.find_vortices(m, capacity=64).cpu().numpy()       # grows to the count by itself
        assert got.shape == ref.shape and np.array_equal(got, ref), (m, got[:5], ref[:5])
    wind = torch.empty(3 * lat.sites, dtype=torch.int32, device="cuda")
    cores = torch.full((10, 6), -7, dtype=torch.int32, device="cuda")
    count = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert lib().qlg_find_vortices(lat.ctx, 0, wind.data_ptr(), cores.data_ptr(), 10, count.data_ptr()) == 0
    ref = oracle_cores3(psis, 0)
    assert int(count.item()) == len(ref) and np.array_equal(cores.cpu().numpy(), ref[:10])
    r = lat.vorticity(0, omega=False)
    flat = torch.cat([r[i]["winding"].reshape(3, -1) for i in range(len(shapes))], dim=1).reshape(-1)
    assert torch.equal(wind, flat)


def test_3d_vortex_lines_cores_full_size():
    """The 256^3 vortex-line state after 3 steps (complex64): the core list of m = +2 equals the
    non-zero windings of the vorticity output, and every z plane holds a core of the line that
    crosses it, with windings of both signs summing to zero per plane."""
    w = qi.vortex_lines_3d_256(nsteps=3)
    n = w.nx[0]
    lat = lattice3([(n, n, n)], g=w.g, eps=w.eps, dtype="c64")
    lat.set_psi([torch.from_numpy(w.psi[0])])
    lat.step(3)
    wd = lat.vorticity(0, omega=False)[0]["winding"]
    cores = lat.find_vortices(0).cpu().numpy()
    nz = torch.nonzero(wd).cpu().numpy()                              # (family, z, y, x), row-major
    assert np.array_equal(cores[:, 1:5], nz) and (cores[:, 0] == 0).all()
    assert np.array_equal(cores[:, 5], wd[tuple(torch.from_numpy(nz).T.to(wd.device))].cpu().numpy())
    zc = cores[cores[:, 1] == 2]
    assert set(zc[:, 2]) == set(range(n))
    for z in (0, 128, 255):
        sel = zc[zc[:, 2] == z]
        assert (sel[:, 5] == 1).any() and sel[:, 5].sum() == 0


def test_3d_track_vortices_against_oracle_steps():
    """Core lists of the three plane families every 2 steps of a 3D run (complex128) equal those
    of the oracle's own run from the same initial field."""
    shape = (6, 10, 14)
    g, eps = (1.0, -0.3, 0.5), 0.4
    psi0 = qi.random_field(shape, seed=33)
    lat = lattice3([shape], g=g, eps=eps, dtype="c128")
    lat.set_psi([torch.from_numpy(psi0)])
    tracks = lat.track_vortices(3, 6, 2)
    assert [t for t, _ in tracks] == [0, 2, 4, 6]
    for t, cores in tracks:
        A, B = O.run_psi(psi0, t, eps, g)
        ref = oracle_cores3([(A + B).numpy()], 3)
        assert len(ref) > 50
        assert np.array_equal(cores.cpu().numpy(), ref), t


def test_3d_fields_and_core_errors():
    from paper_1907_12834_amd.qlg import QLGError
    lat = lattice3([(4, 5, 6)], g=(1.0, -0.3, 0.5), eps=0.4, dtype="c128")
    lat.set_psi([torch.from_numpy(qi.random_field((4, 5, 6), seed=2))])
    with pytest.raises(QLGError, match="QLG_ERR_ARG"):
        lat.find_vortices(5)
    f = lat.fields(("n",))[0]["n"]
    assert f.shape == (4, 5, 6)
    ref = (np.abs(lat.get_psi()[0].cpu().numpy()) ** 2).sum(0)
    assert np.abs(f.cpu().numpy() - ref).max() < 1e-12
