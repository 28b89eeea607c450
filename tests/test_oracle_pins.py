"""Pins for the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle (oracle/qlg_oracle.py) against something other than
itself: printed closed forms (Table I, Table II), an FFT solution of the free
lattice, the continuum Schroedinger flow, dense brute-force matrices built with
scipy.linalg.expm, exact eigenstates, and reductions to scalar GP.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl
import torch

import qlg_inputs as qi
from oracle import qlg_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# independent numpy constructions (not imported from the oracle)
# ---------------------------------------------------------------------------
def np_spin2():
    r = math.sqrt(1.5)
    fx = np.array([[0, 1, 0, 0, 0], [1, 0, r, 0, 0], [0, r, 0, r, 0], [0, 0, r, 0, 1],
                   [0, 0, 0, 1, 0]], complex)
    fy = 1j * np.array([[0, -1, 0, 0, 0], [1, 0, -r, 0, 0], [0, r, 0, -r, 0],
                        [0, 0, r, 0, -1], [0, 0, 0, 1, 0]], complex)
    fz = np.diag([2, 1, 0, -1, -2]).astype(complex)
    return fx, fy, fz


def np_singlet_matrix():
    """S with (S psi)_m = (-1)^m psi_{-m}, rows/cols ordered m = 2..-2."""
    S = np.zeros((5, 5))
    for m in range(-2, 3):
        S[2 - m, 2 + m] = (-1) ** m
    return S


def np_hloc(c, g):
    """Right-hand side of eq. (eomspin2) without the kinetic term, for one site."""
    g0, g1, g2 = g
    fx, fy, fz = np_spin2()
    S = np_singlet_matrix()
    n = np.vdot(c, c).real
    F = [np.vdot(c, f @ c).real for f in (fx, fy, fz)]
    sigma = c @ S @ c
    return g0 * n * c + g1 * sum(Fi * (f @ c) for Fi, f in zip(F, (fx, fy, fz))) \
        + (g2 / 5) * sigma * (S @ c.conj())


def t(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(torch.complex128)


# ---------------------------------------------------------------------------
# The oracle's matrix exponential against scipy's (independent Pade algorithm)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("batch", [1, 2, 7])
@pytest.mark.parametrize("scale", [1e-6, 0.005, 0.013, 0.02, 0.1, 0.7, 3.0, 40.0])
def test_expm_matches_scipy(batch, scale):
    rng = np.random.default_rng(int(scale * 1000) + batch)
    H = rng.normal(size=(batch, 5, 5)) + 1j * rng.normal(size=(batch, 5, 5))
    H = H + H.conj().transpose(0, 2, 1)
    M = -1j * scale * H / np.abs(H).sum(-2).max()
    got = O.expm(torch.from_numpy(M)).numpy()
    for i in range(batch):
        want = sl.expm(M[i])
        assert np.abs(got[i] - want).max() < 2e-15 * max(1.0, np.abs(want).max()) * (1 + scale)


# ---------------------------------------------------------------------------
# P1: unitarity of every operator and norm conservation
# ---------------------------------------------------------------------------
def test_collide_is_sqrt_swap():
    a, b = qi.random_qubits((7,), seed=1)
    a2, b2 = O.collide(*O.collide(t(a), t(b)))
    assert torch.allclose(a2, t(b), atol=1e-15) and torch.allclose(b2, t(a), atol=1e-15)
    # eigenvalue +1 on a = b (bosonic manifold), -i on a = -b
    ab, bb = O.collide(t(a), t(a))
    assert torch.allclose(ab, t(a), atol=1e-15) and torch.allclose(bb, t(a), atol=1e-15)
    am, bm = O.collide(t(a), t(-a))
    assert torch.allclose(am, -1j * t(a), atol=1e-15)


@pytest.mark.parametrize("shape", [(16,), (6, 10)])
def test_norm_conserved_each_operator(shape):
    a, b = qi.random_qubits(shape, seed=2)
    a, b = t(a), t(b)
    n0 = float((a.abs() ** 2).sum() + (b.abs() ** 2).sum())
    g = (1.3, -0.7, 0.9)
    for op in ("collide", "iprime_x", "potential"):
        if op == "collide":
            a1, b1 = O.collide(a, b)
        elif op == "iprime_x":
            a1, b1 = O.iprime(a, b, "x", "a")
        else:
            a1, b1 = O.potential(a, b, 0.37, g)
        n1 = float((a1.abs() ** 2).sum() + (b1.abs() ** 2).sum())
        assert abs(n1 - n0) / n0 < 1e-14, op


def test_norm_conserved_long_run():
    w = qi.single_bright_1d_L1024(L=256, width=16.0)
    a, b = O.run_psi(w.psi[0], 200, w.eps, w.g)
    n = O.observables(a, b, w.eps, w.g)["norm_q"]
    # on the bosonic manifold a = b = psi/2, so N_q = N_psi / 2 = 1/2 initially
    assert abs(n - 0.5) < 1e-12


# ---------------------------------------------------------------------------
# P2: free limit (g = 0) is linear; FFT + per-k 2x2 transfer matrices
# ---------------------------------------------------------------------------
def _kin_matrix(kappa, q):
    """2x2 Fourier symbol of I'_q for one axis: C, S_q^T (e^{+i kappa}), C, S_q (e^{-i kappa})."""
    al, be = (1 - 1j) / 2, (1 + 1j) / 2
    C = np.array([[al, be], [be, al]])
    i = 0 if q == "a" else 1
    Dp = np.eye(2, dtype=complex)
    Dp[i, i] = np.exp(1j * kappa)
    Dm = Dp.conj()
    return Dm @ C @ Dp @ C


def _step_symbol(kappas, ndim):
    """Free-step symbol for wave numbers kappas = (..., k_y, k_x); axes in time order z, y, x."""
    M = np.eye(2, dtype=complex)
    axes = list(zip("zyx"[3 - ndim:], kappas[-ndim:]))
    for _, kap in axes:
        for q in ("b", "b", "a", "a"):
            M = _kin_matrix(kap, q) @ M
    return M


@pytest.mark.parametrize("split", ["interleaved", "plain"])
def test_free_limit_fft_1d(split):
    L, nsteps = 64, 25
    a, b = qi.random_qubits((L,), seed=3)
    A, B = O.run(t(a), t(b), nsteps, 0.1, (0.0, 0.0, 0.0), 1, split)
    ah, bh = np.fft.fft(a, axis=-1), np.fft.fft(b, axis=-1)
    kap = 2 * np.pi * np.fft.fftfreq(L)
    ref_a, ref_b = np.empty_like(ah), np.empty_like(bh)
    for j, kk in enumerate(kap):
        M = np.linalg.matrix_power(_step_symbol([kk], 1), nsteps)
        v = M @ np.stack([ah[:, j], bh[:, j]])
        ref_a[:, j], ref_b[:, j] = v[0], v[1]
    ref_a, ref_b = np.fft.ifft(ref_a, axis=-1), np.fft.ifft(ref_b, axis=-1)
    err = max(np.abs(A.numpy() - ref_a).max(), np.abs(B.numpy() - ref_b).max())
    assert err < 1e-12


def test_free_limit_fft_2d():
    ny, nx, nsteps = 8, 12, 10
    a, b = qi.random_qubits((ny, nx), seed=4)
    A, B = O.run(t(a), t(b), nsteps, 0.1, (0.0, 0.0, 0.0), 2)
    ah, bh = np.fft.fft2(a), np.fft.fft2(b)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    ra, rb = np.empty_like(ah), np.empty_like(bh)
    for iy, vy in enumerate(ky):
        for ix, vx in enumerate(kx):
            M = np.linalg.matrix_power(_step_symbol([vy, vx], 2), nsteps)
            v = M @ np.stack([ah[:, iy, ix], bh[:, iy, ix]])
            ra[:, iy, ix], rb[:, iy, ix] = v[0], v[1]
    ra, rb = np.fft.ifft2(ra), np.fft.ifft2(rb)
    err = max(np.abs(A.numpy() - ra).max(), np.abs(B.numpy() - rb).max())
    assert err < 1e-12


def test_free_limit_fft_3d():
    nz, ny, nx, nsteps = 4, 5, 6, 6
    a, b = qi.random_qubits((nz, ny, nx), seed=14)
    A, B = O.run(t(a), t(b), nsteps, 0.1, (0.0, 0.0, 0.0), 3)
    ah, bh = np.fft.fftn(a, axes=(1, 2, 3)), np.fft.fftn(b, axes=(1, 2, 3))
    ks = [2 * np.pi * np.fft.fftfreq(n) for n in (nz, ny, nx)]
    ra, rb = np.empty_like(ah), np.empty_like(bh)
    for iz, vz in enumerate(ks[0]):
        for iy, vy in enumerate(ks[1]):
            for ix, vx in enumerate(ks[2]):
                M = np.linalg.matrix_power(_step_symbol([vz, vy, vx], 3), nsteps)
                v = M @ np.stack([ah[:, iz, iy, ix], bh[:, iz, iy, ix]])
                ra[:, iz, iy, ix], rb[:, iz, iy, ix] = v[0], v[1]
    ra, rb = np.fft.ifftn(ra, axes=(1, 2, 3)), np.fft.ifftn(rb, axes=(1, 2, 3))
    err = max(np.abs(A.numpy() - ra).max(), np.abs(B.numpy() - rb).max())
    assert err < 1e-12


def test_free_3d_reduces_to_2d_and_1d():
    """On a field uniform along an axis, S along it is the identity, so each I' of that axis is
    C^2 = SWAP and its four I' multiply to 1: a free (g = 0) z-uniform 3D field evolves exactly as
    the 2D field, and an (x, y)-uniform one as the 1D field along z."""
    nsteps, eps = 7, 0.2
    a, b = qi.random_qubits((6, 9), seed=15)
    A2, B2 = O.run(t(a), t(b), nsteps, eps, (0.0, 0.0, 0.0), 2)
    A3, B3 = O.run(t(np.repeat(a[:, None], 3, axis=1)), t(np.repeat(b[:, None], 3, axis=1)), nsteps, eps,
                   (0.0, 0.0, 0.0), 3)
    for k in range(3):
        assert torch.allclose(A3[:, k], A2, atol=1e-13) and torch.allclose(B3[:, k], B2, atol=1e-13)
    a1, b1 = qi.random_qubits((11,), seed=16)
    A1, B1 = O.run(t(a1), t(b1), nsteps, eps, (0.0, 0.0, 0.0), 1)
    A3, B3 = O.run(t(np.tile(a1[:, :, None, None], (1, 1, 2, 3))), t(np.tile(b1[:, :, None, None], (1, 1, 2, 3))),
                   nsteps, eps, (0.0, 0.0, 0.0), 3)
    assert torch.allclose(A3, A1[:, :, None, None].expand_as(A3), atol=1e-13)
    assert torch.allclose(B3, B1[:, :, None, None].expand_as(B3), atol=1e-13)


def test_uniform_tf_state_3d_pure_phase():
    """P4 in 3D: a uniform real Table I state acquires exactly e^{-i E eps^2} per step."""
    E, eps, nsteps = 2.0, 0.1, 30
    c = qi.table1_coeffs(6, E, *TABLE_G).real
    psi = np.tile(c[:, None, None, None], (1, 3, 2, 4)).astype(complex)
    A, B = O.run_psi(psi, nsteps, eps, TABLE_G)
    assert np.abs((A + B).numpy() - psi * np.exp(-1j * E * eps ** 2 * nsteps)).max() < 1e-12


def test_bosonic_dispersion_sign():
    """The a = b mode acquires phase -k^2 + O(k^4) per step: I'I'I'I' = 1 - i p^2 (Sec. VII)."""
    for k in (0.02, 0.05, 0.1):
        M = _step_symbol([k], 1)
        w, V = np.linalg.eig(M)
        j = np.argmax(np.abs(V.conj().T @ np.array([1, 1]) / math.sqrt(2)))
        ph = np.angle(w[j])
        assert abs(ph - (-k * k + k ** 4 / 3)) < 5 * k ** 6
    # and the oracle reproduces it on a plane wave on the bosonic manifold
    L, k = 128, 2 * np.pi * 3 / 128
    psi = np.tile(np.exp(1j * k * np.arange(L)), (5, 1))
    A, B = O.run_psi(psi, 1, 0.1, (0.0, 0.0, 0.0))
    ratio = (A + B).numpy()[:, 5] / psi[:, 5]
    assert abs(np.angle(ratio[0]) - (-k * k + k ** 4 / 3)) < 1e-5


# ---------------------------------------------------------------------------
# P3: free limit converges to the continuum e^{-i K^2 T} at O(eps^2)
# ---------------------------------------------------------------------------
def test_free_limit_continuum_second_order():
    T, errs = 0.5, []
    for w in (8, 16, 32):
        eps = 1.0 / w
        L = 16 * w
        X = (np.arange(L) - L / 2) * eps
        g0 = np.exp(-X ** 2 / 2) * np.exp(1j * 1.0 * X)
        psi = np.tile(g0, (5, 1))
        nsteps = int(round(T / eps ** 2))
        A, B = O.run_psi(psi, nsteps, eps, (0.0, 0.0, 0.0))
        K = 2 * np.pi * np.fft.fftfreq(L, d=eps)
        exact = np.fft.ifft(np.fft.fft(g0) * np.exp(-1j * K ** 2 * nsteps * eps ** 2))
        sim = (A + B).numpy()[0]
        errs.append(np.linalg.norm(sim - exact) / np.linalg.norm(exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.6 < r1 < 4.4 and 3.6 < r2 < 4.4, errs


# ---------------------------------------------------------------------------
# Table I / Table II: printed closed forms; the singlet sign reading
# ---------------------------------------------------------------------------
TABLE_G = (1.0, 0.1, 0.7)
FAMILY = {11: dict(c2=0.5), 12: dict(c1=0.5), 16: dict(c1=0.4, c2=0.3)}


@pytest.mark.parametrize("row", list(range(1, 17)))
def test_table1_rows_solve_tf_system(row):
    """Every Table I row satisfies H_loc c = E c with the (-1)^m singlet reading."""
    E = 2.0
    c = qi.table1_coeffs(row, E, *TABLE_G, **FAMILY.get(row, {}))
    assert np.abs(c.imag).max() == 0.0
    res = np_hloc(c, TABLE_G) - E * c
    assert np.abs(res).max() < 1e-12


@pytest.mark.parametrize("row", list(range(1, 17)))
def test_oracle_potential_phase_on_tf_states(row):
    """U(theta) on a uniform Table I state is the pure phase e^{-i theta E} (P4, one site)."""
    E, theta = 2.0, 0.173
    c = qi.table1_coeffs(row, E, *TABLE_G, **FAMILY.get(row, {}))
    psi = t(np.tile(c[:, None], (1, 3)))
    a, b = O.encode(psi)
    a1, b1 = O.potential(a, b, theta, TABLE_G)
    assert torch.allclose(a1 + b1, psi * np.exp(-1j * theta * E), atol=1e-14)


def test_table2_characteristics_golden():
    with open(os.path.join(GOLDEN, "table2_characteristics.json")) as fh:
        gold = json.load(fh)
    E = 2.0
    g0, g1, g2 = TABLE_G
    env = dict(E=E, g0=g0, g1=g1, g2=g2, sqrt=math.sqrt)
    for row, exprs in gold["rows"].items():
        row = int(row)
        c = qi.table1_coeffs(row, E, *TABLE_G, **FAMILY.get(row, {}))
        psi = t(c[:, None])
        n, F, v = O.invariants(psi)
        sigma = complex((v.conj() * psi).sum())
        got = [abs(float(F[2])), math.hypot(float(F[0]), float(F[1])), abs(sigma) / math.sqrt(5)]
        want = [eval(e, {}, env) for e in exprs]  # noqa: S307 - fixed fixture strings
        assert np.allclose(got, want, atol=1e-12), (row, got, want)


def test_uniform_tf_state_whole_step_is_pure_phase():
    """P4: on a uniform real Table I state the whole interleaved step is e^{-i E eps^2}."""
    E, eps, nsteps = 2.0, 0.1, 1000
    for row in (6, 14, 16):
        c = qi.table1_coeffs(row, E, *TABLE_G, **FAMILY.get(row, {})).real
        psi = np.tile(c[:, None], (1, 8))
        A, B = O.run_psi(psi, nsteps, eps, TABLE_G)
        want = psi * np.exp(-1j * E * eps * eps * nsteps)
        # 4000 U applications: the phase carries ~6e-16 of rounding per application
        assert np.abs((A + B).numpy() - want).max() < 1e-11, row
    # also in 2D (n = 8 Lie product)
    c = qi.table1_coeffs(14, E, *TABLE_G).real
    psi = np.tile(c[:, None, None], (1, 4, 4))
    A, B = O.run_psi(psi, 200, eps, TABLE_G)
    assert np.abs((A + B).numpy() - psi * np.exp(-1j * E * eps * eps * 200)).max() < 1e-12


# ---------------------------------------------------------------------------
# P5: dense brute force on <= 8 sites (80 x 80 matrices, scipy expm factors)
# ---------------------------------------------------------------------------
class Dense:
    """State z = [a(5 x N), b(5 x N)] flattened m-major; all operators as dense matrices."""

    def __init__(self, shape):
        self.shape = shape
        self.N = int(np.prod(shape))
        self.dim = 10 * self.N

    def idx(self, q, m, site):
        return q * 5 * self.N + m * self.N + site

    def collide(self):
        al, be = (1 - 1j) / 2, (1 + 1j) / 2
        M = np.zeros((self.dim, self.dim), complex)
        for m in range(5):
            for s in range(self.N):
                ia, ib = self.idx(0, m, s), self.idx(1, m, s)
                M[ia, ia], M[ia, ib], M[ib, ia], M[ib, ib] = al, be, be, al
        return M

    def shift(self, axis, q, transpose):
        """Permutation: q(r) <- q(r - e) (S), or q(r) <- q(r + e) (S^T)."""
        M = np.eye(self.dim, dtype=complex)
        coords = list(np.ndindex(*self.shape))
        ax = len(self.shape) - 1 - {"x": 0, "y": 1, "z": 2}[axis]
        qi_ = 0 if q == "a" else 1
        for m in range(5):
            for s, r in enumerate(coords):
                src = list(r)
                src[ax] = (src[ax] + (1 if transpose else -1)) % self.shape[ax]
                ssrc = int(np.ravel_multi_index(src, self.shape))
                M[self.idx(qi_, m, s), :] = 0
                M[self.idx(qi_, m, s), self.idx(qi_, m, ssrc)] = 1
        return M

    def potential(self, z, theta, g):
        g0, g1, g2 = g
        fx, fy, fz = np_spin2()
        S = np_singlet_matrix()
        W = np.zeros((self.dim, self.dim), complex)
        for s in range(self.N):
            ia = [self.idx(0, m, s) for m in range(5)]
            ib = [self.idx(1, m, s) for m in range(5)]
            psi = z[ia] + z[ib]
            n = np.vdot(psi, psi).real
            F = [np.vdot(psi, f @ psi).real for f in (fx, fy, fz)]
            v = S @ psi.conj()
            Hs = (g2 / 5) * np.outer(v, v.conj())
            Hf = g1 * (F[0] * fx + F[1] * fy + F[2] * fz)
            w = sl.expm(-1j * theta * g0 * n * np.eye(5)) @ sl.expm(-1j * theta * Hf) \
                @ sl.expm(-1j * theta * Hs)
            W[np.ix_(ia, ia)] = w
            W[np.ix_(ib, ib)] = w
        return W @ z


@pytest.mark.parametrize("shape,split", [((8,), "interleaved"), ((5,), "interleaved"),
                                         ((8,), "plain"), ((2, 4), "interleaved"),
                                         ((2, 2), "interleaved"), ((2, 2, 2), "interleaved"),
                                         ((2, 1, 3), "plain"), ((1, 3, 2), "interleaved")])
def test_dense_brute_force(shape, split):
    g, eps, nsteps = (0.8, -0.6, 1.1), 0.7, 3
    a, b = qi.random_qubits(shape, seed=5, scale=0.6)
    D = Dense(shape)
    z = np.concatenate([a.reshape(-1), b.reshape(-1)])
    C = D.collide()
    ndim = len(shape)
    seq = [(ax, q) for ax in "zyx"[3 - ndim:] for q in "bbaa"]
    Ip = {}
    for ax, q in set(seq):
        Ip[(ax, q)] = D.shift(ax, q, False) @ C @ D.shift(ax, q, True) @ C
    for _ in range(nsteps):
        if split == "interleaved":
            for ax, q in seq:
                z = D.potential(z, eps * eps / len(seq), g)
                z = Ip[(ax, q)] @ z
        else:
            z = D.potential(z, eps * eps, g)
            for ax, q in seq:
                z = Ip[(ax, q)] @ z
    A, B = O.run(t(a), t(b), nsteps, eps, g, ndim, split)
    got = np.concatenate([A.numpy().reshape(-1), B.numpy().reshape(-1)])
    # strongly nonlinear (theta*g*n ~ 0.1 per substep): scipy vs torch expm rounding
    # differences grow to ~2e-13; any mistake in stencil, wrap or order is O(1e-2)
    assert np.abs(got - z).max() < 1e-12


def test_dense_detects_planted_mistakes():
    """The brute force separates the readings: wrong shift direction / order change results."""
    g, eps = (0.8, -0.6, 1.1), 0.7
    a, b = qi.random_qubits((6,), seed=6, scale=0.6)
    A, B = O.run(t(a), t(b), 2, eps, g, 1)
    # swapped qubit order (I'_1 first) must give a different answer
    orig = O.kinetic_sequence
    try:
        O.kinetic_sequence = lambda ndim: [("x", "a"), ("x", "a"), ("x", "b"), ("x", "b")]
        A2, B2 = O.run(t(a), t(b), 2, eps, g, 1)
    finally:
        O.kinetic_sequence = orig
    assert (A - A2).abs().max() > 1e-3


# ---------------------------------------------------------------------------
# P6, P8: bright soliton stationarity and dispersion E = p^2 - K^2
# ---------------------------------------------------------------------------
G_BRIGHT = (1.0, -0.5, 0.5)   # g0 + 4 g1 = -1: Table I row 1 is real with E = -2


def _bright(w, p=0.0, K=1.0):
    eps = 1.0 / w
    L = 40 * w
    X = (np.arange(L) - L / 2) * eps
    c = qi.table1_coeffs(1, -2.0, *G_BRIGHT).real
    f = K / np.cosh(K * X) * np.exp(1j * p * X)
    return c[:, None] * f[None, :], eps


def test_bright_soliton_stationary_converges():
    T, errs = 0.5, []
    for w in (8, 16):
        psi, eps = _bright(w)
        nsteps = int(round(T / eps ** 2))
        A, B = O.run_psi(psi, nsteps, eps, G_BRIGHT)
        errs.append(O.density_l2_error(t(psi), A + B))
    assert errs[1] < errs[0] / 6, errs
    assert errs[1] < 5e-4


def test_bright_soliton_overlap_energy():
    w = 24
    for p in (0.0, 0.5):
        psi, eps = _bright(w, p=p)
        A, B = O.run_psi(psi, 40, eps, G_BRIGHT)
        prev = A + B
        a1, b1 = O.step(A, B, eps, G_BRIGHT, 1)
        obs = O.observables(a1, b1, eps, G_BRIGHT, prev_psi=prev)
        e = obs["e_overlap"].real / eps ** 2
        assert abs(e - (p * p - 1.0)) < 0.01 * max(1.0, abs(p * p - 1.0)), (p, e)


def test_moving_bright_soliton_velocity():
    """A kicked bright soliton moves with velocity 2p (Sec. III, eq. timedependentsoliton) and keeps
    its shape."""
    w, T = 16, 2.0
    for p in (0.5, -0.8):
        psi, eps = _bright(w, p=p)
        L = psi.shape[1]
        X = (np.arange(L) - L / 2) * eps
        nsteps = int(round(T / eps ** 2))
        A, B = O.run_psi(psi, nsteps, eps, G_BRIGHT)
        d0 = (np.abs(psi) ** 2).sum(0)
        d1 = (np.abs((A + B).numpy()) ** 2).sum(0)
        shift = (X * d1).sum() / d1.sum() - (X * d0).sum() / d0.sum()
        expect = 2 * p * nsteps * eps ** 2
        assert abs(shift / expect - 1) < 0.01, (p, shift, expect)
        moved = np.interp(X - expect, X, d0)
        assert np.linalg.norm(d1 - moved) / np.linalg.norm(d0) < 0.03


# ---------------------------------------------------------------------------
# P7, P8: dark solitons (Table I with E = +2, psi = c K tanh(K x)) in the periodic
# product form of Sec. IV; dispersion E = p^2 + 2 K^2 (eq. darkdispersion)
# ---------------------------------------------------------------------------
G_DARK = (1.0, 0.1, 0.7)   # repulsive in every channel: all Table I rows real at E = +2


def _dark(w, p=0.0, row=16):
    eps = 1.0 / w
    c = qi.table1_coeffs(row, 2.0, *G_DARK, c1=0.5, c2=0.5).real
    return qi.dark_pair_1d(40 * w, eps, c, K=1.0, p=p), eps


@pytest.mark.parametrize("row", [6, 16])
def test_dark_soliton_stationary_converges(row):
    """Density of the two-kink state stays put; the error falls ~8x per doubling of resolution
    (sum over twice the sites of an O(eps^2) error), and the plain split is worse than the
    interleaved one (Sec. VII)."""
    T, errs = 0.5, {}
    for split in ("interleaved", "plain"):
        for w in (8, 16):
            psi, eps = _dark(w, row=row)
            A, B = O.run_psi(psi, int(round(T / eps ** 2)), eps, G_DARK, split)
            errs[split, w] = O.density_l2_error(t(psi), A + B)
    assert errs["interleaved", 16] < errs["interleaved", 8] / 6, errs
    assert errs["interleaved", 16] < 5e-4, errs
    assert errs["plain", 8] > 1.5 * errs["interleaved", 8], errs


def test_dark_soliton_overlap_energy():
    """Re E_ov / eps^2 -> p^2 + 2 K^2 for resting and kicked dark solitons (p = 2 pi n / Lp keeps
    the product state periodic)."""
    w = 24
    for p in (0.0, 2 * np.pi * 3 / 40.0):
        psi, eps = _dark(w, p=p)
        A, B = O.run_psi(psi, 40, eps, G_DARK)
        prev = A + B
        a1, b1 = O.step(A, B, eps, G_DARK, 1)
        e = O.observables(a1, b1, eps, G_DARK, prev_psi=prev)["e_overlap"].real / eps ** 2
        assert abs(e - (p * p + 2.0)) < 1e-3 * (p * p + 2.0), (p, e)


# ---------------------------------------------------------------------------
# P10: Pade vortices (Sec. V, Table III; calibration quadrupole of Sec. VI)
# ---------------------------------------------------------------------------
def _table3(m, E, g0, g1, g2):
    """Table III closed forms as printed, for channel m, with the root that gives a1 > 0."""
    if abs(m) == 2:
        G = g0 + 4 * g1
        gam = E * E * math.sqrt(361 * E * E - 8 * G * (4 * G + 13 * E))
        a1 = max((19 * E ** 3 - 12 * G * E * E + s * gam) / (64 * G * (2 * E - G)) for s in (1, -1))
        b1 = (16 * a1 * (G - 3 * E) + 5 * E * E) / (48 * (E - 4 * a1))
    elif abs(m) == 1:
        G = g0 + g1
        gam = E * E * math.sqrt(361 * E * E - 8 * G * (4 * G + 13 * E))
        a1 = max(-11 * E ** 4 / (76 * E ** 3 - 48 * G * E * E + s * 4 * gam) for s in (1, -1))
        b1 = (16 * a1 * (G - 3 * E) + 5 * E * E) / (48 * (E - 4 * a1))
    else:
        G5 = 5 * g0 + g2
        gam = E * E * math.sqrt(9025 * E * E - 8 * G5 * (20 * g0 + 4 * g2 + 65 * E))
        a1 = max(5 * (95 * E ** 3 - 12 * G5 * E * E + s * gam) / (64 * G5 * (10 * E - G5)) for s in (1, -1))
        b1 = (16 * a1 * (G5 - 15 * E) + 25 * E * E) / (240 * (E - 4 * a1))
    return a1, a1 * (b1 - E / 4), b1


GEFF = {2: lambda g: g[0] + 4 * g[1], 1: lambda g: g[0] + g[1], 0: lambda g: g[0] + g[2] / 5}


@pytest.mark.parametrize("m", [2, 1, 0])
@pytest.mark.parametrize("g", [(1.0, -0.1, 0.2), (1.3, 0.2, -0.5)])
def test_pade_coefficients_match_table3(m, g):
    """On a unit background (E = g_eff) the Pade coefficients equal Table III's closed forms."""
    G = GEFF[m](g)
    ours = qi.pade_coefficients(G)
    assert np.allclose(ours, _table3(m, G, *g), rtol=1e-12, atol=0), (ours, _table3(m, G, *g))


@pytest.mark.parametrize("G", [0.7, 1.04])
def test_pade_profile_solves_radial_equation_to_r7(G):
    """The radial residual E f + (f'' + f'/r - f/r^2) - G f^3 of f = sqrt(pade) vanishes through
    r^5 (accurate to O(r^7), Sec. V): residual / r^7 stays bounded as r -> 0.  Derivatives by
    high-order central differences, independent of the series used to find the coefficients."""
    a1, a2, b1 = qi.pade_coefficients(G)
    f = lambda r: np.sqrt(qi.pade_density(r, a1, a2, b1))   # noqa: E731
    h = 1e-3
    ratios = []
    for r in (0.2, 0.1, 0.05):
        d1 = (f(r - 2 * h) - 8 * f(r - h) + 8 * f(r + h) - f(r + 2 * h)) / (12 * h)
        d2 = (-f(r - 2 * h) + 16 * f(r - h) - 30 * f(r) + 16 * f(r + h) - f(r + 2 * h)) / (12 * h * h)
        res = G * f(r) + d2 + d1 / r - f(r) / r ** 2 - G * f(r) ** 3
        ratios.append(abs(res) / r ** 7)
    assert max(ratios) < 10 * G ** 4, ratios   # an O(r^3) or O(r^5) residual would blow up here
    # a wrong coefficient leaves an O(r^3) residual
    f = lambda r: np.sqrt(qi.pade_density(r, a1 * 1.05, a2, b1))   # noqa: E731
    r = 0.05
    d1 = (f(r - 2 * h) - 8 * f(r - h) + 8 * f(r + h) - f(r + 2 * h)) / (12 * h)
    d2 = (-f(r - 2 * h) + 16 * f(r - h) - 30 * f(r) + 16 * f(r + h) - f(r + 2 * h)) / (12 * h * h)
    assert abs(G * f(r) + d2 + d1 / r - f(r) / r ** 2 - G * f(r) ** 3) / r ** 7 > 1e3 * max(ratios)


def _core_profile(nfield, cy, cx, R=14):
    """Azimuthal average of the density in unit rings around the density minimum near (cy, cx)."""
    win = nfield[cy - 6:cy + 7, cx - 6:cx + 7]
    iy, ix = np.unravel_index(np.argmin(win), win.shape)
    y0, x0 = cy - 6 + iy, cx - 6 + ix
    yy, xx = np.mgrid[-R:R + 1, -R:R + 1]
    rr = np.sqrt(yy ** 2 + xx ** 2)
    vals = nfield[y0 - R:y0 + R + 1, x0 - R:x0 + R + 1]
    return np.array([vals[(rr >= k) & (rr < k + 1)].mean() for k in range(R)])


def _winding(field, cy, cx, rad):
    """Phase winding of field along the square contour of half-size rad around (cy, cx)."""
    pts = [(cy - rad, x) for x in range(cx - rad, cx + rad)] + [(y, cx + rad) for y in range(cy - rad, cy + rad)]
    pts += [(cy + rad, x) for x in range(cx + rad, cx - rad, -1)] + [(y, cx - rad) for y in range(cy + rad, cy - rad, -1)]
    ph = np.angle(np.array([field[q] for q in pts + pts[:1]]))
    return float(np.sum(np.angle(np.exp(1j * np.diff(ph)))) / (2 * np.pi))


@pytest.mark.parametrize("m_index", [2, 1])
def test_pade_quadrupole_cores_stationary(m_index):
    """Single-channel Pade quadrupole (m = 0 or m = +1) under the 2D step: each core keeps its radial
    density profile (about 1 % change over unit time) where a free evolution or a core of the wrong
    size changes it several times more; every winding number is conserved, and the other four
    components stay exactly zero."""
    g = (1.0, -0.3, 0.2)
    G = GEFF[2 - m_index](g)
    n, eps, d, T = 128, 0.25, 32, 1.0
    nsteps = int(round(T / eps ** 2))
    centres = [(n // 2 + sy * d, n // 2 + sx * d) for sx, sy in ((-1, -1), (1, -1), (-1, 1), (1, 1))]
    change = {}
    for label, gg, scale in (("pade", g, 1.0), ("free", (0.0, 0.0, 0.0), 1.0),
                             ("core x1.5", g, 1.5), ("core x0.7", g, 0.7)):
        psi = qi.pade_quadrupole_2d(n, eps, d, G, m_index, core_scale=scale)
        A, B = O.run_psi(psi, nsteps, eps, gg)
        out = (A + B).numpy()
        n0, n1 = (np.abs(psi) ** 2).sum(0), (np.abs(out) ** 2).sum(0)
        change[label] = np.mean([np.linalg.norm(_core_profile(n1, *c) - _core_profile(n0, *c)) /
                                 np.linalg.norm(1 - _core_profile(n0, *c)) for c in centres])
        if label == "pade":
            assert [round(_winding(out[m_index], cy, cx, 8), 9) for cy, cx in centres] == [1.0, -1.0, -1.0, 1.0]
            assert all(np.abs(out[k]).max() == 0.0 for k in range(5) if k != m_index)
    assert change["pade"] < 0.03, change
    for label in ("free", "core x1.5", "core x0.7"):
        assert change["pade"] < 0.25 * change[label], change


# ---------------------------------------------------------------------------
# P9: reductions to scalar GP (pure m = 0: g0 + g2/5; pure m = +-2: g0 + 4 g1)
# ---------------------------------------------------------------------------
def scalar_qlg(u, nsteps, eps, geff):
    """Independent single-component QLG in numpy (same reading of C, S; U = e^{-i th geff |psi|^2})."""
    al, be = (1 - 1j) / 2, (1 + 1j) / 2
    a, b = u / 2, u / 2
    th = eps * eps / 4
    for _ in range(nsteps):
        for q in "bbaa":
            p = a + b
            ph = np.exp(-1j * th * geff * np.abs(p) ** 2)
            a, b = ph * a, ph * b
            a, b = al * a + be * b, be * a + al * b
            if q == "a":
                a = np.roll(a, -1)
            else:
                b = np.roll(b, -1)
            a, b = al * a + be * b, be * a + al * b
            if q == "a":
                a = np.roll(a, 1)
            else:
                b = np.roll(b, 1)
    return a + b


@pytest.mark.parametrize("m_index,geff", [(2, 1.0 + 0.9 / 5), (0, 1.0 + 4 * -0.35),
                                          (4, 1.0 + 4 * -0.35)])
def test_reduction_to_scalar_gp(m_index, geff):
    g, eps, L, nsteps = (1.0, -0.35, 0.9), 0.2, 64, 150
    rng = np.random.default_rng(7)
    u = (1.0 + 0.3 * np.cos(2 * np.pi * np.arange(L) / L)) * np.exp(1j * rng.uniform(0, 0.2, L))
    psi = np.zeros((5, L), complex)
    psi[m_index] = u
    A, B = O.run_psi(psi, nsteps, eps, g)
    out = (A + B).numpy()
    others = [i for i in range(5) if i != m_index]
    assert np.abs(out[others]).max() == 0.0
    ref = scalar_qlg(u, nsteps, eps, geff)
    assert np.abs(out[m_index] - ref).max() < 1e-12


# ---------------------------------------------------------------------------
# Observables: energy definition against an independent numpy evaluation
# ---------------------------------------------------------------------------
def test_energy_matches_numpy_definition():
    psi = qi.random_field((12,), seed=8, scale=0.5)
    g, eps = (1.0, -0.5, 0.5), 0.1
    fx, fy, fz = np_spin2()
    S = np_singlet_matrix()
    kin = np.sum(np.abs(np.roll(psi, -1, axis=1) - psi) ** 2) / eps ** 2
    pot = 0.0
    for x in range(psi.shape[1]):
        c = psi[:, x]
        n = np.vdot(c, c).real
        F = np.array([np.vdot(c, f @ c).real for f in (fx, fy, fz)])
        sig = c @ S @ c
        pot += 0.5 * (g[0] * n * n + g[1] * F @ F + g[2] * abs(sig) ** 2 / 5)
    want = eps * (kin + pot)
    got = float(O.energy(t(psi), eps, g))
    assert abs(got - want) < 1e-12 * abs(want)


def test_energy_3d_plane_waves():
    """Free energy of a plane wave along each axis of a 3D lattice: eps^3 N |c|^2 4 sin^2(k/2) / eps^2
    (forward differences), and a z-uniform field has eps * nz times its 2D energy."""
    nz, ny, nx, eps = 4, 6, 5, 0.3
    c = qi.random_field((1,), seed=3, scale=0.7)[:, 0]
    N = nz * ny * nx
    for axis, n_ax in ((1, nz), (2, ny), (3, nx)):
        k = 2 * np.pi * 1 / n_ax
        shape = [1, 1, 1]
        shape[axis - 1] = n_ax
        ph = np.exp(1j * k * np.arange(n_ax)).reshape(shape)
        psi = c[:, None, None, None] * np.broadcast_to(ph, (nz, ny, nx))[None]
        want = eps ** 3 * N * np.vdot(c, c).real * 4 * math.sin(k / 2) ** 2 / eps ** 2
        assert abs(float(O.energy(t(psi), eps, (0.0, 0.0, 0.0))) - want) < 1e-12 * want
    p2 = qi.random_field((ny, nx), seed=4, scale=0.5)
    e2 = float(O.energy(t(p2), eps, TABLE_G))
    e3 = float(O.energy(t(np.repeat(p2[:, None], nz, axis=1)), eps, TABLE_G))
    assert abs(e3 - eps * nz * e2) < 1e-12 * abs(e3)


def test_energy_gradient_is_hloc():
    """dE/dpsi* = eps^d (-lap_fd psi / eps^2 + H_loc psi): the energy and the EOM agree."""
    psi = qi.random_field((10,), seed=9, scale=0.5)
    g, eps = (1.0, -0.5, 0.5), 0.1
    p = t(psi).clone().requires_grad_(True)
    E = O.energy(p, eps, g)
    E.backward()
    grad = p.grad.numpy() / 2            # torch gives 2 dE/dpsi*
    lap = (np.roll(psi, -1, 1) - 2 * psi + np.roll(psi, 1, 1)) / eps ** 2
    hl = np.stack([np_hloc(psi[:, x], g) for x in range(psi.shape[1])], axis=1)
    want = eps * (-lap + hl)
    assert np.abs(grad - want).max() < 1e-10 * np.abs(want).max()


# ---------------------------------------------------------------------------
# P11: per-site fields (Sec. III eq. cmap) and lattice vorticity (Sec. VI)
# ---------------------------------------------------------------------------
def test_fields_table2_golden():
    """fields() reproduces Table II's F_par, F_perp and |A00| for the Table I states."""
    with open(os.path.join(GOLDEN, "table2_characteristics.json")) as fh:
        gold = json.load(fh)
    E = 2.0
    g0, g1, g2 = TABLE_G
    env = dict(E=E, g0=g0, g1=g1, g2=g2, sqrt=math.sqrt)
    for row, exprs in gold["rows"].items():
        c = qi.table1_coeffs(int(row), E, *TABLE_G, **FAMILY.get(int(row), {}))
        fl = O.fields(t(np.tile(c[:, None], (1, 3))))
        got = [abs(float(fl["f_par"][1])), float(fl["f_perp"][1]), float(fl["a00"][1])]
        want = [eval(e, {}, env) for e in exprs]  # noqa: S307 - fixed fixture strings
        assert np.allclose(got, want, atol=1e-12), (row, got, want)
        assert abs(float(fl["n"][1]) - np.vdot(c, c).real) < 1e-12


def test_fields_spin_rotations():
    """Spin rotations: a rotated |m=2> has F_par = 2 cos b, F_perp = 2 |sin b|; n and |A00| are
    invariant under any rotation (|A00| is the singlet amplitude), F_par and F_perp under rotations
    about z, and |F| under all.  A wrong sign or a dropped pairing in sigma breaks the invariance."""
    fx, fy, fz = np_spin2()
    rng = np.random.default_rng(11)
    psi = rng.normal(size=(5, 6)) + 1j * rng.normal(size=(5, 6))
    base = O.fields(t(psi))
    for beta in (0.3, 1.1, 2.5):
        Ry = sl.expm(-1j * beta * fy)
        Rz = sl.expm(-1j * 0.7 * beta * fz)
        top = O.fields(t(Ry @ np.eye(5)[:, :1]))
        assert abs(float(top["f_par"][0]) - 2 * math.cos(beta)) < 1e-12
        assert abs(float(top["f_perp"][0]) - 2 * abs(math.sin(beta))) < 1e-12
        assert abs(float(top["a00"][0]) - 0.0) < 1e-12
        for R, same in ((Ry, ("n", "a00")), (Rz, ("n", "a00", "f_par", "f_perp"))):
            rot = O.fields(t(R @ psi))
            for k in same:
                assert torch.allclose(rot[k], base[k], atol=1e-12, rtol=1e-12), (beta, k)
            F2 = lambda f: f["f_par"] ** 2 + f["f_perp"] ** 2   # noqa: E731
            assert torch.allclose(F2(rot), F2(base), rtol=1e-12)
    # the polar m = 0 state and the m = +-2 "cyclic" pair: |A00| = 1/sqrt(5) at unit density
    assert abs(float(O.fields(t(np.eye(5)[:, 2:3]))["a00"][0]) - 1 / math.sqrt(5)) < 1e-15
    assert abs(float(O.fields(t((np.eye(5)[:, 0] + np.eye(5)[:, 4])[:, None] / math.sqrt(2)))["a00"][0])
               - 1 / math.sqrt(5)) < 1e-15


def _vortex_field(ny, nx, cores, kx=0.0, ky=0.0):
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    out = np.exp(1j * (kx * x + ky * y))
    for cy, cx, w in cores:
        out = out * np.exp(1j * w * np.arctan2(y - cy, x - cx))
    return out


def test_vorticity_plaquette_windings():
    """Winding +1 / -1 on exactly the plaquettes that enclose a +1 / -1 core, 0 elsewhere in the
    interior, also on top of a uniform flow.  (The test field, a product of atan2 phases, is not
    periodic, so the seam plaquettes carry windings of their own.)  Over the whole periodic lattice
    the windings sum to zero: every wrapped edge difference enters two plaquettes with opposite
    signs."""
    cores = [(20.5, 14.5, 1), (20.5, 45.5, -1), (44.5, 30.5, 1), (44.5, 50.5, -1)]
    for kx, ky in ((0.0, 0.0), (2 * np.pi * 3 / 64, -2 * np.pi / 64)):
        _, wind = O.vorticity(_vortex_field(64, 64, cores, kx, ky))
        inner = wind[:-1, :-1]
        nz = {(int(a), int(b)): int(inner[a, b]) for a, b in zip(*np.nonzero(inner))}
        want = {(int(cy), int(cx)): w for cy, cx, w in cores}
        assert wind.dtype == np.int32
        assert nz == want, nz
        assert int(wind.sum()) == 0


def test_vorticity_uniform_flow_and_circulation():
    """omega vanishes for a uniform flow (a plane wave, any wrap of the phase); summed over a box
    around one core it equals the circulation 2 pi w (discrete Stokes), and away from the cores it
    decays like the continuum curl of grad(arg), which is zero."""
    y, x = np.mgrid[0:48, 0:64].astype(float)
    om, wind = O.vorticity(np.exp(1j * (2 * np.pi * 5 / 64 * x - 2 * np.pi * 7 / 48 * y)))
    assert np.abs(om).max() < 1e-14 and not wind.any()
    cores = [(32.5, 20.5, 1), (32.5, 44.5, -1)]
    om, _ = O.vorticity(_vortex_field(64, 64, cores))
    for cy, cx, w in cores:
        box = om[int(cy) - 10:int(cy) + 12, int(cx) - 10:int(cx) + 12]
        assert abs(box.sum() - 2 * np.pi * w) < 1e-9, box.sum()
    far = np.ones_like(om, bool)
    for cy, cx, _ in cores:
        far[int(cy) - 4:int(cy) + 6, int(cx) - 4:int(cx) + 6] = False
    assert np.abs(om[far]).max() < 0.05 * np.abs(om).max()


def test_vorticity_zero_component_and_signed_zeros():
    """A component that is identically zero (also as -0.0) has phase 0: omega = 0, no windings."""
    z = np.zeros((8, 8), complex)
    z.real[::2] = -0.0
    z.imag[:, ::3] = -0.0
    om, wind = O.vorticity(z)
    assert not om.any() and not wind.any()


def test_vorticity_small_lattices():
    """On a 1 x N or 2 x N periodic lattice the stencils wrap onto the site itself (np.roll reading)."""
    rng = np.random.default_rng(3)
    for shape in ((1, 7), (2, 5), (3, 3)):
        psi = np.exp(1j * rng.uniform(-np.pi, np.pi, size=shape))
        om, wind = O.vorticity(psi)
        assert om.shape == shape and np.isfinite(om).all()
        # the total winding of a periodic lattice is zero
        assert int(wind.sum()) == 0


def test_vorticity_3d_z_uniform_reduces_to_2d():
    """A field uniform along z: the z components are the 2D vorticity and windings of every plane,
    the x and y components vanish (no phase changes along z)."""
    cores = [(20.5, 14.5, 1), (20.5, 45.5, -1)]
    f2 = _vortex_field(40, 64, cores, kx=2 * np.pi * 3 / 64)
    om2, w2 = O.vorticity(f2)
    om3, w3 = O.vorticity(np.repeat(f2[None], 5, axis=0))
    assert om3.shape == (3, 5, 40, 64) and w3.dtype == np.int32
    for z in range(5):
        assert np.array_equal(om3[2, z], om2) and np.array_equal(w3[2, z], w2)
    assert not om3[:2].any() and not w3[:2].any()


def test_vorticity_3d_line_along_x_is_right_handed():
    """A straight vortex line along x (phase atan2(z - z0, y - y0), which turns from y to z): winding
    +1 on the x-normal plaquette around the core in every x plane (circulation y -> z, right-handed
    about +x), none in the interior elsewhere, none on y- or z-normal plaquettes (the field does not
    change along x), and omega_x sums to 2 pi around the core (discrete Stokes)."""
    nz, ny, nx, z0, y0 = 40, 48, 6, 20.5, 23.5
    z, y, _ = np.mgrid[0:nz, 0:ny, 0:nx].astype(float)
    om, w = O.vorticity(np.exp(1j * np.arctan2(z - z0, y - y0)))
    for x in range(nx):
        inner = w[0, :-1, :-1, x]
        assert {(int(a), int(b)): int(inner[a, b]) for a, b in zip(*np.nonzero(inner))} == {(20, 23): 1}
        box = om[0, 10:32, 13:35, x]
        assert abs(box.sum() - 2 * np.pi) < 1e-9, box.sum()
    assert not w[1:].any() and not om[1:].any()


def test_vorticity_3d_cyclic_relabelling_of_axes():
    """Relabelling the axes cyclically (x, y, z) -> (z, x, y) is a rotation: the components follow
    the axes, value for value (the same arithmetic on the same phases), which fixes the orientation
    and sign conventions of all three plane families together."""
    rng = np.random.default_rng(12)
    psi = np.exp(1j * rng.uniform(-np.pi, np.pi, size=(5, 6, 7)))
    om, w = O.vorticity(psi)
    P = np.transpose(psi, (1, 2, 0))              # P[i, j, k] = psi[k, i, j]: P's x, y, z = psi's z, x, y
    omP, wP = O.vorticity(P)
    for cP, c in ((0, 2), (1, 0), (2, 1)):
        assert np.array_equal(omP[cP], np.transpose(om[c], (1, 2, 0)))
        assert np.array_equal(wP[cP], np.transpose(w[c], (1, 2, 0)))
    # and on a periodic lattice every plane family's windings sum to zero
    assert not w.sum(axis=(1, 2, 3)).any()


# ---------------------------------------------------------------------------
# P12: external potential and chemical potential (Sec. II "Additional terms"; Sec. IV dispersion)
# ---------------------------------------------------------------------------
def _trap_1d(eps, omega=1.0, half_width=10.0):
    """Lattice X = eps (i - L/2) and the harmonic trap V = omega^2 X^2 / 4 (m = 1/2: V = m omega^2 X^2 / 2)."""
    L = int(round(2 * half_width / eps))
    X = eps * (np.arange(L) - L / 2)
    return X, omega ** 2 * X ** 2 / 4


def _spinor(profile, seed=5):
    rng = np.random.default_rng(seed)
    c = rng.normal(size=5) + 1j * rng.normal(size=5)
    return c.reshape((5,) + (1,) * profile.ndim) * profile[None]


def test_harmonic_trap_ground_state_energy():
    """Free spinor in a harmonic trap: the ground state exp(-omega X^2/4) in every component has
    E = omega/2 (overlap energy of one step, which converges fast) and the lattice energy per
    particle tends to omega/2 at second order.  A wrong factor or sign of V, or V applied with the
    wrong theta, moves E by O(1)."""
    errs = []
    for eps in (0.2, 0.1):
        X, V = _trap_1d(eps)
        psi = _spinor(np.exp(-X ** 2 / 4))
        a, b = O.encode(t(psi))
        a1, b1 = O.step(a, b, eps, (0.0, 0.0, 0.0), 1, V=V)
        ob = O.observables(a1, b1, eps, (0.0, 0.0, 0.0), prev_psi=a + b, V=V)
        assert abs(ob["e_overlap"].real / eps ** 2 - 0.5) < 1e-4, (eps, ob["e_overlap"])
        errs.append(abs(ob["energy"] / ob["norm_psi"] - 0.5))
    assert errs[1] < 1e-3 and 3.0 < errs[0] / errs[1] < 5.0, errs


def test_harmonic_trap_oscillation():
    """A displaced ground state oscillates as <X>(t) = X0 cos(omega t) (exact in the continuum for a
    quadratic potential); the lattice error falls faster than 4x per halving of eps."""
    X0, errs = 2.0, []
    for eps in (0.2, 0.1):
        X, V = _trap_1d(eps)
        psi = _spinor(np.exp(-(X - X0) ** 2 / 4))
        n_half = int(round(np.pi / eps ** 2))
        out = psi
        for nst in (n_half // 2, n_half - n_half // 2):     # quarter and half period
            A, B = O.run_psi(out, nst, eps, (0.0, 0.0, 0.0), V=V)
            out = (A + B).numpy()
        n = (np.abs(out) ** 2).sum(0)
        xm = float((n * X).sum() / n.sum())
        errs.append(abs(xm - X0 * np.cos(n_half * eps ** 2)))
    assert errs[1] < 5e-4 and errs[0] / errs[1] > 4.0, errs


def test_harmonic_trap_2d_anisotropic():
    """2D trap V = (wx^2 X^2 + wy^2 Y^2)/4: the product ground state has E = (wx + wy)/2 (here 1.5),
    reached at second order in eps, so the potential enters both axes' substeps with the right theta."""
    wx, wy, errs = 1.0, 2.0, []
    for eps in (0.2, 0.1):
        n = int(round(16 / eps))
        X = eps * (np.arange(n) - n / 2)
        Y = X[:, None]
        V = (wx ** 2 * X[None, :] ** 2 + wy ** 2 * Y ** 2) / 4
        psi = _spinor(np.exp(-wx * X[None, :] ** 2 / 4 - wy * Y ** 2 / 4))
        a, b = O.encode(t(psi))
        a1, b1 = O.step(a, b, eps, (0.0, 0.0, 0.0), 2, V=V)
        ob = O.observables(a1, b1, eps, (0.0, 0.0, 0.0), prev_psi=a + b, V=V)
        errs.append(abs(ob["e_overlap"].real / eps ** 2 - (wx + wy) / 2))
    assert errs[1] < 2e-3 and 3.5 < errs[0] / errs[1] < 4.5, errs


@pytest.mark.parametrize("split", ["interleaved", "plain"])
@pytest.mark.parametrize("ndim", [1, 2])
def test_chemical_potential_is_a_global_phase(split, ndim):
    """mu psi_m in the equation of motion multiplies the state by e^{-i mu t}: after n steps the
    run with mu equals the run without it times e^{-i mu eps^2 n}, also with interactions and a trap."""
    shape = (24,) if ndim == 1 else (12, 10)
    psi = qi.random_field(shape, seed=9, scale=0.5)
    V = np.random.default_rng(2).uniform(0, 3, size=shape)
    g, eps, mu, nst = (1.1, -0.6, 0.8), 0.3, 1.7, 6
    A0, B0 = O.run_psi(psi, nst, eps, g, split, V=V)
    A1, B1 = O.run_psi(psi, nst, eps, g, split, V=V, mu=mu)
    ph = np.exp(-1j * mu * eps ** 2 * nst)
    assert torch.allclose(A1, A0 * ph, atol=1e-12) and torch.allclose(B1, B0 * ph, atol=1e-12)


def test_bright_soliton_dispersion_with_chemical_potential():
    """Sec. IV: with a chemical potential the bright-soliton dispersion is E = mu + p^2 - k^2."""
    w, mu = 24, 0.7
    for p in (0.0, 0.5):
        psi, eps = _bright(w, p=p)
        A, B = O.run_psi(psi, 40, eps, G_BRIGHT, mu=mu)
        prev = A + B
        a1, b1 = O.step(A, B, eps, G_BRIGHT, 1, mu=mu)
        obs = O.observables(a1, b1, eps, G_BRIGHT, prev_psi=prev, mu=mu)
        e = obs["e_overlap"].real / eps ** 2
        assert abs(e - (mu + p * p - 1.0)) < 0.01 * max(1.0, abs(mu + p * p - 1.0)), (p, e)
