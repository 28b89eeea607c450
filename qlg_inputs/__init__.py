"""Seeded synthetic input fields for the spin-2 QLG workloads.

This module is the only code shared by the FP64 oracle (``oracle/``) and the
GPU path (``paper_1907_12834_amd``).  It builds initial spinor fields
psi[m][y][x] (m ordered 2, 1, 0, -1, -2) as numpy complex128 arrays and holds
none of the lattice-gas arithmetic: no collide, stream or self-interaction
operator appears here.

Field shapes follow the paper's analytic states:

* bright solitons psi_m = c_m k sech(k x) (Sec. III "Bright soliton solutions"),
  kicked by a phase e^{i p x} (Sec. IV "Kicked solitons");
* dark solitons psi_m = c_m k tanh(k x) and the periodic product of two of them
  (Sec. III "Dark soliton solutions", Sec. IV "Dark solitons");
* Thomas-Fermi coefficients c_m of Table I;
* Pade-profile vortices |psi|^2 = (a2 r^4 + a1 r^2)/(a2 r^4 + b1 r^2 + 1) with
  winding e^{+-i theta} (Sec. V, eq. pade_form).

Lattice units: site index x = 0..L-1; a physical coordinate is X = eps * x
(the paper's scaling x -> a x, Sec. VII "Scaling").  Norms use the measure
eps^d, so "normalised to int n = 1" means eps^d * sum_x sum_m |psi_m|^2 = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

M_VALUES = (2, 1, 0, -1, -2)


# ---------------------------------------------------------------------------
# Table I: Thomas-Fermi coefficients (Sec. III, Table I)
# ---------------------------------------------------------------------------
def table1_coeffs(row: int, E: float, g0: float, g1: float, g2: float,
                  c1: Optional[float] = None, c2: Optional[float] = None) -> np.ndarray:
    """Return c = (c_2, c_1, c_0, c_-1, c_-2) of Table I, row ``row`` (1..16).

    Rows 11, 12 and 16 are one- or two-parameter families; their free
    coefficients are passed as ``c2``/``c1``.  The square roots are taken of
    possibly negative numbers, so the result is complex in general; a row is a
    real solution only where its radicands are non-negative (Table I caption).
    """
    s = lambda z: np.sqrt(complex(z))  # noqa: E731
    z = 0.0
    if row == 1:
        return np.array([s(E / (g0 + 4 * g1)), z, z, z, z])
    if row == 2:
        return np.array([z, z, z, z, s(E / (g0 + 4 * g1))])
    if row == 3:
        return np.array([z, s(E / (g0 + g1)), z, z, z])
    if row == 4:
        return np.array([z, z, z, s(E / (g0 + g1)), z])
    if row == 5:
        return np.array([z, z, s(5 * E / (5 * g0 + g2)), z, z])
    if row == 6:
        c = s(5 * E / (10 * g0 + 2 * g2))
        return np.array([c, z, z, z, c])
    if row == 7:
        c = s(5 * E / (10 * g0 + 2 * g2))
        return np.array([z, c, z, c, z])
    if row == 8:
        return np.array([s(E / (3 * g0)), z, z, s(2 * E / (3 * g0)), z])
    if row == 9:
        return np.array([z, s(2 * E / (3 * g0)), z, z, s(E / (3 * g0))])
    if row == 10:
        c = s(E / (4 * g0))
        return np.array([c, z, s(E / (2 * g0)), z, -c])
    if row == 11:
        assert c2 is not None
        c0 = s((5 * E - 10 * c2 ** 2 * g0 - 2 * c2 ** 2 * g2) / (5 * g0 + g2))
        return np.array([c2, z, c0, z, c2], dtype=complex)
    if row == 12:
        assert c1 is not None
        c0 = s((5 * E - 10 * c1 ** 2 * g0 - 2 * c1 ** 2 * g2) / (5 * g0 + g2))
        return np.array([z, c1, c0, -c1, z], dtype=complex)
    if row == 13:
        c = s(E / (4 * g0 + 4 * g1))
        return np.array([c, c, z, -c, -c])
    if row == 14:
        return np.array([s(3 * E / (16 * g0)), s(E / (4 * g0)), -s(E / (8 * g0)),
                         s(E / (4 * g0)), s(3 * E / (16 * g0))])
    if row == 15:
        c = s(E / (g0 + 4 * g1))
        return np.array([c / 4, c / 2, 0.5 * s(3 * E / (2 * g0 + 8 * g1)), c / 2, c / 4])
    if row == 16:
        assert c1 is not None and c2 is not None
        c0 = s((5 * E - (c2 ** 2 + c1 ** 2) * (10 * g0 + 2 * g2)) / (5 * g0 + g2))
        return np.array([c2, c1, c0, -c1, c2], dtype=complex)
    raise ValueError(f"Table I has rows 1..16, got {row}")


# ---------------------------------------------------------------------------
# 1D soliton fields
# ---------------------------------------------------------------------------
def sech(x):
    return 1.0 / np.cosh(x)


def soliton_1d(L: int, center: float, width: float, k: float, weights: Sequence[complex],
               kind: str = "bright") -> np.ndarray:
    """psi_m(x) = w_m f((x - center)/width) e^{i k (x - center)}, shape (5, L).

    ``k`` is in radians per site, ``width`` and ``center`` in sites; f is sech
    (bright) or tanh (dark).  The lattice is periodic, so the nearest periodic
    image of the centre is used for every site.
    """
    x = np.arange(L, dtype=np.float64)
    d = x - center
    d = d - L * np.round(d / L)
    f = sech(d / width) if kind == "bright" else np.tanh(d / width)
    w = np.asarray(weights, dtype=np.complex128).reshape(5, 1)
    return w * (f * np.exp(1j * k * d))[None, :]


def normalise(psi: np.ndarray, eps: float, target: float = 1.0) -> np.ndarray:
    """Scale psi so that eps^d * sum |psi|^2 == target (d = psi.ndim - 1)."""
    d = psi.ndim - 1
    nrm = (eps ** d) * float(np.sum(np.abs(psi) ** 2))
    return psi * math.sqrt(target / nrm)


def random_weights(rng: np.random.Generator) -> np.ndarray:
    """Five complex spinor weights, each N(0,1) + i N(0,1)."""
    return rng.normal(size=5) + 1j * rng.normal(size=5)


# ---------------------------------------------------------------------------
# 2D Pade vortices (Sec. V)
# ---------------------------------------------------------------------------
def pade_density(r: np.ndarray, a1: float, a2: float, b1: float) -> np.ndarray:
    """(a2 r^4 + a1 r^2)/(a2 r^4 + b1 r^2 + 1), eq. pade_form squared."""
    r2 = r * r
    return (a2 * r2 * r2 + a1 * r2) / (a2 * r2 * r2 + b1 * r2 + 1.0)


def pade_coefficients(geff: float) -> tuple:
    """(a1, a2, b1) of the single-channel winding-1 Pade vortex on a unit background.

    For psi = sqrt(pade(r)) e^{i theta} in a channel with effective coupling
    geff (g0 + 4 g1 for m = +-2, g0 + g1 for m = +-1, g0 + g2/5 for m = 0), the
    background density is 1, so E = geff, and the three lowest orders (r, r^3,
    r^5) of the radial equation E f = -(f'' + f'/r - f/r^2) + geff f^3 vanish for
    a1 = 11 geff / 32, b1 = geff / 3, a2 = a1 (b1 - E / 4) = 11 geff^2 / 384
    (Sec. V; the root of Table III with a1 > 0).
    """
    g = float(geff)
    return 11.0 * g / 32.0, 11.0 * g * g / 384.0, g / 3.0


def pade_quadrupole_2d(n: int, eps: float, d: float, geff: float, m_index: int,
                       core_scale: float = 1.0) -> np.ndarray:
    """Four single-channel Pade vortices at (n/2 +- d, n/2 +- d) (sites), windings +1, -1, -1, +1,
    in component m_index of an (5, n, n) field: the periodic calibration state of Sec. VI.
    core_scale != 1 stretches every core by that factor (a non-eigenstate control)."""
    a1, a2, b1 = pade_coefficients(geff)
    f = np.ones((n, n), dtype=np.complex128)
    c = n / 2.0
    for sx, sy, wnd in ((-1, -1, 1), (1, -1, -1), (-1, 1, -1), (1, 1, 1)):
        f = f * vortex_2d(n, n, c + sx * d, c + sy * d, wnd, eps / core_scale, a1, a2, b1)
    psi = np.zeros((5, n, n), dtype=np.complex128)
    psi[m_index] = f
    return psi


def dark_pair_1d(L: int, eps: float, coeffs: Sequence[float], K: float = 1.0, p: float = 0.0) -> np.ndarray:
    """c_m K tanh(K(X - Lp/4)) tanh(K(3Lp/4 - X)) e^{i p X}, X = eps x, Lp = eps L: two dark
    solitons in the periodic product form of Sec. IV (the amplitude c_m K appears once)."""
    X = np.arange(L, dtype=np.float64) * eps
    Lp = L * eps
    f = K * np.tanh(K * (X - Lp / 4)) * np.tanh(K * (3 * Lp / 4 - X)) * np.exp(1j * p * X)
    return np.asarray(coeffs, dtype=np.complex128).reshape(5, 1) * f[None, :]


def vortex_2d(nx: int, ny: int, cx: float, cy: float, winding: int, eps: float,
              a1: float, a2: float, b1: float) -> np.ndarray:
    """sqrt(pade(r)) e^{i winding theta} on an (ny, nx) grid; r = eps * distance."""
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    dx = x - cx
    dy = y - cy
    r = eps * np.sqrt(dx * dx + dy * dy)
    return np.sqrt(pade_density(r, a1, a2, b1)) * np.exp(1j * winding * np.arctan2(dy, dx))


# ---------------------------------------------------------------------------
# Workload presets (shapes and distributions of the paper's 1D and 2D runs)
# ---------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    ndim: int
    nx: List[int]
    ny: List[int]
    psi: List[np.ndarray]             # one complex128 array per instance, (5, [nz,] [ny,] nx)
    g: tuple
    eps: float
    nsteps: int
    meta: dict = field(default_factory=dict)
    nz: List[int] = field(default_factory=lambda: [1])

    @property
    def nbatch(self) -> int:
        return len(self.psi)

    @property
    def sites(self) -> int:
        return int(sum(a * b * c for a, b, c in zip(self.nx, self.ny, self.nz * len(self.nx)
                                                      if len(self.nz) == 1 else self.nz)))


def single_bright_1d_L1024(L: int = 1024, width: float = 32.0, eps: float = 0.1, seed: int = 1907,
                     nsteps: int = 1000) -> Workload:
    """1D periodic lattice, one stationary bright soliton with seeded weights, int n = 1."""
    rng = np.random.default_rng(seed)
    psi = soliton_1d(L, L / 2, width, 0.0, random_weights(rng))
    psi = normalise(psi, eps)
    return Workload("1d_bright_L%d" % L, 1, [L], [1], [psi], (1.0, -0.5, 0.5), eps, nsteps,
                    {"width": width, "seed": seed})


def two_solitons_1d(L: int, width: float, k: float, rng: np.random.Generator, eps: float,
                    rel_phase: float = 0.0) -> np.ndarray:
    """Two bright solitons at L/2 -+ L/8 moving towards each other (+k on the left one)."""
    left = normalise(soliton_1d(L, L / 2 - L / 8, width, +k, random_weights(rng)), eps)
    right = normalise(soliton_1d(L, L / 2 + L / 8, width, -k, random_weights(rng)), eps)
    return left + right * np.exp(1j * rel_phase)


def two_solitons_1d_L16384(L: int = 16384, width: float = 48.0, k: float = 0.05 * math.pi,
                    c1: float = -0.5, eps: float = 0.1, seed: int = 12834,
                    nsteps: int = 20000, rel_phase: float = 0.0) -> Workload:
    rng = np.random.default_rng(seed)
    psi = two_solitons_1d(L, width, k, rng, eps, rel_phase)
    return Workload("1d_two_solitons_L%d" % L, 1, [L], [1], [psi], (1.0, c1, 0.5), eps, nsteps,
                    {"width": width, "k": k, "seed": seed, "obs_every": 100})


def vortex_pair_2d(nx: int, ny: int, sep: float, eps: float, rng: np.random.Generator,
                   n0: float = 1.0, coeffs=(0.3, 0.05, 0.4), jitter: float = 0.05) -> np.ndarray:
    """Background n0 shared by m = +2, 0, -2; winding +1 vortex in m = +-2, winding -1 in m = 0.

    The Pade coefficients (a1, a2, b1) are drawn as coeffs * (1 + jitter * U[-1, 1]).
    """
    a1, a2, b1 = (c * (1.0 + jitter * rng.uniform(-1.0, 1.0)) for c in coeffs)
    cxa, cxb, cy = nx / 2 - sep / 2, nx / 2 + sep / 2, ny / 2
    va = vortex_2d(nx, ny, cxa, cy, +1, eps, a1, a2, b1)
    vb = vortex_2d(nx, ny, cxb, cy, -1, eps, a1, a2, b1)
    amp = math.sqrt(n0 / 3.0)
    psi = np.zeros((5, ny, nx), dtype=np.complex128)
    psi[0] = amp * va
    psi[4] = amp * va
    psi[2] = amp * vb
    return psi


def vortex_pair_2d_2048(n: int = 2048, sep: float = 128.0, eps: float = 0.1, seed: int = 2019,
                   nsteps: int = 10000) -> Workload:
    rng = np.random.default_rng(seed)
    psi = vortex_pair_2d(n, n, sep, eps, rng)
    return Workload("2d_vortex_pair_%dx%d" % (n, n), 2, [n], [n], [psi], (1.0, -0.3, 0.2), eps,
                    nsteps, {"sep": sep, "seed": seed})


def batched_two_solitons_1d_256(nbatch: int = 256, seed: int = 4, eps: float = 0.1, nsteps: int = 5000,
               lmax_units: int = 16, unit: int = 1024) -> Workload:
    """Independent 1D two-soliton scattering runs of uneven size.

    Draw order: L (1024 * U{1..16}), k (U[0.01, 0.1] * pi), width (U[24, 64]), then weights.
    """
    rng = np.random.default_rng(seed)
    Ls = [int(unit * v) for v in rng.integers(1, lmax_units + 1, size=nbatch)]
    ks = rng.uniform(0.01, 0.1, size=nbatch) * math.pi
    ws = rng.uniform(24.0, 64.0, size=nbatch)
    psis = [two_solitons_1d(L, float(w), float(k), rng, eps) for L, k, w in zip(Ls, ks, ws)]
    return Workload("1d_batched_%d" % nbatch, 1, Ls, [1] * nbatch, psis, (1.0, -0.5, 0.5), eps,
                    nsteps, {"seed": seed, "k": ks.tolist(), "width": ws.tolist()})


def adjoint_vortex_pair_2d_512(n: int = 512, sep: float = 128.0, eps: float = 0.1, seed: int = 2019,
               nsteps: int = 2000, checkpoint_every: int = 64) -> Workload:
    rng = np.random.default_rng(seed)
    psi = vortex_pair_2d(n, n, sep, eps, rng)
    return Workload("2d_adjoint_%dx%d" % (n, n), 2, [n], [n], [psi], (1.0, -0.3, 0.2), eps,
                    nsteps, {"sep": sep, "seed": seed, "checkpoint_every": checkpoint_every})


def adjoint_spin_texture_2d_512(n: int = 512, sep: float = 128.0, eps: float = 0.1, seed: int = 2019,
                                noise_seed: int = 78, noise: float = 0.05, nsteps: int = 2000,
                                checkpoint_every: int = 64) -> Workload:
    """The 512^2 adjoint workload's vortex pair plus a seeded complex Gaussian spinor of amplitude
    `noise` in every component, so that F != 0 at every site and the spin factor of the
    self-interaction and its derivative act everywhere (in the vortex pair m = +-1 are empty and
    F = 0 for the whole run)."""
    w = adjoint_vortex_pair_2d_512(n, sep, eps, seed, nsteps, checkpoint_every)
    psi = w.psi[0] + random_field((n, n), noise_seed, noise)
    return Workload("2d_adjoint_spin_texture_%dx%d" % (n, n), 2, [n], [n], [psi], w.g, eps, nsteps,
                    dict(w.meta, noise=noise, noise_seed=noise_seed))


def adjoint_vortex_pair_2d_64(n: int = 64, sep: float = 16.0, eps: float = 0.4, seed: int = 2019) -> np.ndarray:
    """The vortex-pair construction on the 64^2 lattice of the adjoint's finite-difference and
    reference-gradient checks: separation 16 sites and eps = 0.4, so the cores fit the box."""
    return vortex_pair_2d(n, n, sep, eps, np.random.default_rng(seed))


def adjoint_spin_texture_2d_64(n: int = 64, sep: float = 16.0, eps: float = 0.4, seed: int = 2019,
                               noise_seed: int = 77, noise: float = 0.05) -> np.ndarray:
    """adjoint_vortex_pair_2d_64 plus a seeded complex Gaussian spinor of amplitude `noise` in
    every component: m = +-1 are populated and F != 0 at every site, so the spin factor of
    the self-interaction (and its derivative) acts everywhere."""
    return adjoint_vortex_pair_2d_64(n, sep, eps, seed) + random_field((n, n), noise_seed, noise)


def vortex_lines_3d(n: int, sep: float, eps: float, rng: np.random.Generator, amp: float = 4.0,
                    coeffs=(0.3, 0.05, 0.4), jitter: float = 0.05) -> np.ndarray:
    """The 2D vortex pair of vortex_pair_2d extruded along z into two vortex lines on an n^3
    lattice, each line displaced along x by amp * sin(2 pi z / n + phase) (one period over the
    lattice, seeded phases), so that the lines bend and move in 3D."""
    a1, a2, b1 = (c * (1.0 + jitter * rng.uniform(-1.0, 1.0)) for c in coeffs)
    pha, phb = rng.uniform(0.0, 2 * math.pi, size=2)
    amp0 = math.sqrt(1.0 / 3.0)
    psi = np.zeros((5, n, n, n), dtype=np.complex128)
    for z in range(n):
        cxa = n / 2 - sep / 2 + amp * math.sin(2 * math.pi * z / n + pha)
        cxb = n / 2 + sep / 2 + amp * math.sin(2 * math.pi * z / n + phb)
        va = vortex_2d(n, n, cxa, n / 2, +1, eps, a1, a2, b1)
        vb = vortex_2d(n, n, cxb, n / 2, -1, eps, a1, a2, b1)
        psi[0, z] = amp0 * va
        psi[4, z] = amp0 * va
        psi[2, z] = amp0 * vb
    return psi


def vortex_lines_3d_256(n: int = 256, sep: float = 64.0, eps: float = 0.1, seed: int = 2020,
                    nsteps: int = 1000) -> Workload:
    rng = np.random.default_rng(seed)
    psi = vortex_lines_3d(n, sep, eps, rng)
    return Workload("3d_vortex_lines_%d" % n, 3, [n], [n], [psi], (1.0, -0.3, 0.2), eps, nsteps,
                    {"sep": sep, "seed": seed}, nz=[n])


def vortex_lines_3d_512(n: int = 512, sep: float = 128.0, eps: float = 0.1, seed: int = 2021,
                        nsteps: int = 1000) -> Workload:
    """The 3D vortex-line state on the largest cube the paper names (512^3): lines 128 sites
    apart, as in the 2D vortex pair, bending by 8 sites along x."""
    rng = np.random.default_rng(seed)
    psi = vortex_lines_3d(n, sep, eps, rng, amp=8.0)
    return Workload("3d_vortex_lines_%d" % n, 3, [n], [n], [psi], (1.0, -0.3, 0.2), eps, nsteps,
                    {"sep": sep, "seed": seed}, nz=[n])


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Generic seeded complex field of shape (5, *spatial) for stress tests."""
    rng = np.random.default_rng(seed)
    return scale * (rng.normal(size=(5,) + tuple(shape)) + 1j * rng.normal(size=(5,) + tuple(shape)))


def random_qubits(shape, seed: int, scale: float = 1.0):
    """Independent seeded (a, b) qubit planes, each (5, *spatial), off the a = b manifold."""
    rng = np.random.default_rng(seed)
    sh = (5,) + tuple(shape)
    a = scale * (rng.normal(size=sh) + 1j * rng.normal(size=sh))
    b = scale * (rng.normal(size=sh) + 1j * rng.normal(size=sh))
    return a, b
