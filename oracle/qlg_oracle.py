"""FP64 CPU oracle for the spin-2 quantum-lattice-gas (QLG) step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, calls or links this file; only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may.
It shares no code with the HIP path: the only common module is
``qlg_inputs`` (seeded initial fields, which hold none of the arithmetic).

Everything is plain torch CPU code in complex128, written to be read against
the paper (Taylor, Smith, Yepez, arXiv:1907.12834):

* spin-2 matrices f_x, f_y, f_z and the spin-2 equation of motion: Sec. II,
  eqs. (hamspin2), (eomspin2), (spinsinglet);
* collide C, stream S, I'_q = S_q C S_q^T C, the plain split
  psi(t+tau) = I'_1 I'_1 I'_2 I'_2 U psi(t) and the interleaved split
  I'_1 U^{1/4} I'_1 U^{1/4} I'_2 U^{1/4} I'_2 U^{1/4} (Lie product n = 4 in
  1D, n = 8 in 2D, n = 12 in 3D): Sec. VII "Operator interleaving";
* scaling x -> a x, t -> a^2 t: Sec. VII "Scaling";
* overlap energy E = i(<psi_t|psi_t> - <psi_t|psi_{t-1}>)/<psi_t|psi_t>: Sec. IV,
  eq. (disecrete_energy);
* the optional psi-independent term (V(x) + mu) psi_m of Sec. II "Additional
  terms" (external trap, chemical potential), a per-site phase inside U, and its
  energy eps^d sum (V + mu) n;
* per-site F_par, F_perp, |A00| (Sec. III, eq. cmap) and the lattice vorticity
  of one component from central differences of its phase, with plaquette
  winding numbers (Sec. VI, "Calculating quantum vorticity on a lattice"); on
  3D lattices the same in each family of lattice planes (three components).

The paper defers C, S and U to earlier work, so the definitions below are
readings, each pinned by the tests of this oracle:

* C is the sqrt(SWAP) gate [[alpha, beta], [beta, alpha]] with
  alpha = (1 - i)/2, beta = (1 + i)/2 acting on the qubit pair (a_m, b_m) of
  each m; the bosonic field is psi = a + b.
* S_{axis,q} moves qubit q (q = a for the paper's subscript 1, b for 2) one
  site in the +axis direction, q(x) <- q(x - e); S^T moves it back.
* U(theta) is the per-site frozen-field unitary
  W = exp(-i theta g0 n) exp(-i theta g1 F.f) (I + (exp(-i theta g2 n / 5) - 1) v v^H / n),
  v = S psi*, (S psi)_m = (-1)^m psi_{-m}, applied to a and to b with the
  invariants n, F, v of psi = a + b taken before the update.  Its generator is
  the right-hand side of eq. (eomspin2) with |A00|^2 read as sigma/5 and the
  singlet term as (g2/5) sigma (-1)^m psi*_{-m}.
* One step advances physical time eps^2; U^{1/(4d)} uses theta = eps^2/(4d),
  the plain split theta = eps^2.

Layout: a, b are complex128 tensors of shape (5, L), (5, Ny, Nx) or (5, Nz, Ny, Nx),
component index 0..4 <-> m = 2, 1, 0, -1, -2; x is the last axis, y the one before,
z the one before that.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence, Tuple

import numpy as np
import torch

CDT = torch.complex128
RDT = torch.float64

ALPHA = complex(0.5, -0.5)   # collide coefficient (1 - i)/2
BETA = complex(0.5, 0.5)     # collide coefficient (1 + i)/2


# ---------------------------------------------------------------------------
# Spin-2 matrices (Sec. II, spin-2 f_x, f_y, f_z), ordering m = 2, 1, 0, -1, -2
# ---------------------------------------------------------------------------
def spin2_matrices() -> Tuple[torch.Tensor, torch.Tensor, torch.Tensor]:
    r = math.sqrt(1.5)
    fx = torch.tensor([[0, 1, 0, 0, 0],
                       [1, 0, r, 0, 0],
                       [0, r, 0, r, 0],
                       [0, 0, r, 0, 1],
                       [0, 0, 0, 1, 0]], dtype=CDT)
    fy = 1j * torch.tensor([[0, -1, 0, 0, 0],
                            [1, 0, -r, 0, 0],
                            [0, r, 0, -r, 0],
                            [0, 0, r, 0, -1],
                            [0, 0, 0, 1, 0]], dtype=CDT)
    fz = torch.diag(torch.tensor([2, 1, 0, -1, -2], dtype=CDT))
    return fx, fy, fz


FX, FY, FZ = spin2_matrices()
M_SIGN = torch.tensor([1.0, -1.0, 1.0, -1.0, 1.0], dtype=RDT)   # (-1)^m for m = 2..-2


def time_reverse(psi: torch.Tensor) -> torch.Tensor:
    """v = S psi*, v_m = (-1)^m conj(psi_{-m}) (the singlet partner, eq. spinsinglet)."""
    flipped = torch.flip(psi, dims=[0]).conj()
    shape = (5,) + (1,) * (psi.dim() - 1)
    return M_SIGN.reshape(shape).to(psi.dtype) * flipped


# ---------------------------------------------------------------------------
# Encode / decode (two qubit amplitudes per m_f; psi = a + b)
# ---------------------------------------------------------------------------
def encode(psi: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    """a = b = psi / 2: the state on the bosonic manifold where I' is ~ identity."""
    return psi / 2, psi / 2


def decode(a: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    return a + b


# ---------------------------------------------------------------------------
# Kinetic operators (Sec. VII, I'_q = S_q C S_q^T C)
# ---------------------------------------------------------------------------
def collide(a: torch.Tensor, b: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
    """sqrt(SWAP) on every (a_m, b_m) pair: a' = alpha a + beta b, b' = beta a + alpha b."""
    return ALPHA * a + BETA * b, BETA * a + ALPHA * b


def _dim(x: torch.Tensor, axis: str) -> int:
    """Tensor dimension of a lattice axis: x is the last, y the one before, z the one before that."""
    return x.dim() - 1 - "xyz".index(axis)


def stream(x: torch.Tensor, axis: str, transpose: bool) -> torch.Tensor:
    """S: x(r) <- x(r - e_axis); S^T: x(r) <- x(r + e_axis); periodic."""
    return torch.roll(x, shifts=-1 if transpose else 1, dims=_dim(x, axis))


def iprime(a: torch.Tensor, b: torch.Tensor, axis: str, q: str):
    """I'_{axis,q} = S_q C S_q^T C: in time order C, S_q^T, C, S_q."""
    a, b = collide(a, b)
    if q == "a":
        a = stream(a, axis, transpose=True)
    else:
        b = stream(b, axis, transpose=True)
    a, b = collide(a, b)
    if q == "a":
        a = stream(a, axis, transpose=False)
    else:
        b = stream(b, axis, transpose=False)
    return a, b


# ---------------------------------------------------------------------------
# Self-interaction U(theta) (Sec. II eq. eomspin2; frozen-field reading)
# ---------------------------------------------------------------------------
def invariants(psi: torch.Tensor):
    """n = sum |psi_m|^2, F_nu = psi^H f_nu psi, v = S psi*."""
    n = (psi.abs() ** 2).sum(0)
    F = [torch.einsum("m...,mk,k...->...", psi.conj(), f, psi).real for f in (FX, FY, FZ)]
    return n, F, time_reverse(psi)


def expm(M: torch.Tensor, max_terms: int = 18) -> torch.Tensor:
    """Matrix exponential of a batch (..., k, k) by its power series.

    exp(M) = (sum_{j<=N} (M/2^s)^j / j!)^(2^s), with s chosen so that
    r = ||M/2^s||_1 <= 1/2 for every matrix of the batch and N the smallest
    number of terms whose remainder bound r^(N+1)/(N+1)! * 2 is below 1e-18.
    (torch.linalg.matrix_exp was not used: for a batch of one matrix of norm
    ~0.01-0.02 it is only accurate to ~1e-12.)
    """
    norm = float(M.detach().abs().sum(-2).amax()) if M.numel() else 0.0
    s = max(0, int(math.ceil(math.log2(norm / 0.5)))) if norm > 0.5 else 0
    r = norm / (2.0 ** s)
    N, term = 1, r
    while N < max_terms and 2.0 * term * r / (N + 1) > 1e-18:
        N += 1
        term *= r / N
    A = M / (2.0 ** s)
    eye = torch.eye(M.shape[-1], dtype=M.dtype).expand_as(M)
    T = eye
    for j in range(N, 0, -1):              # Horner: I + A/1 (I + A/2 (I + ... ))
        T = eye + (A @ T) / j
    for _ in range(s):
        T = T @ T
    return T


def potential(a: torch.Tensor, b: torch.Tensor, theta: float, g: Sequence[float], ext=None):
    """Apply W = e^{-i th (g0 n + ext)} exp(-i th g1 F.f) P_A to a and b (same frozen W).

    ext (optional) is the m-independent term of the equation of motion that does not
    depend on psi (Sec. II "Additional terms"): an external potential V(x) plus a
    chemical potential mu, a real array of the spatial shape or a scalar."""
    g0, g1, g2 = g
    psi = a + b
    n, F, v = invariants(psi)
    spatial = n.shape
    # singlet factor P_A = I + (e^{-i th g2 n/5} - 1) v v^H / n   (identity where n = 0)
    safe_n = torch.where(n > 0, n, torch.ones_like(n))
    lam = torch.where(n > 0, (torch.exp(-1j * theta * g2 * n / 5) - 1) / safe_n,
                      torch.zeros_like(n, dtype=CDT))
    # spin factor R = exp(-i th g1 F.f), one 5x5 matrix exponential per site
    H = (F[0].reshape(-1, 1, 1) * FX + F[1].reshape(-1, 1, 1) * FY + F[2].reshape(-1, 1, 1) * FZ)
    R = expm(-1j * theta * g1 * H)                               # (sites, 5, 5)
    phase = g0 * n if ext is None else g0 * n + torch.as_tensor(ext, dtype=RDT)
    dens = torch.exp(-1j * theta * phase).reshape(-1)

    out = []
    for x in (a, b):
        proj = (v.conj() * x).sum(0)                             # v^H x per site
        y = x + lam * proj * v                                   # P_A x
        yf = y.reshape(5, -1).transpose(0, 1).unsqueeze(-1)      # (sites, 5, 1)
        z = (R @ yf).squeeze(-1).transpose(0, 1)                 # R y
        out.append((dens * z).reshape((5,) + tuple(spatial)))
    return out[0], out[1]


# ---------------------------------------------------------------------------
# Steps and schedules (Sec. VII; readings for the 2D order)
# ---------------------------------------------------------------------------
def kinetic_sequence(ndim: int):
    """The I' factors of one step in time order (rightmost operator acts first).

    1D: I'_2 I'_2 then I'_1 I'_1, i.e. (x,b), (x,b), (x,a), (x,a).
    2D: the same four for y, then the same four for x (n = 8 Lie product).
    3D: z, then y, then x (n = 12), the same reading extended to the third axis.
    """
    one = [("b",), ("b",), ("a",), ("a",)]
    axes = ["x", "y", "z"][:ndim][::-1]
    return [(ax, q[0]) for ax in axes for q in one]


def external(V=None, mu: float = 0.0):
    """The psi-independent diagonal term V(x) + mu (None when both are absent)."""
    if V is None:
        return None if mu == 0.0 else mu
    return torch.as_tensor(np.asarray(V, dtype=np.float64)) + mu


def step(a, b, eps: float, g, ndim: int, split: str = "interleaved", V=None, mu: float = 0.0):
    """One step; V (spatial shape, real) and mu add the term (V(x) + mu) psi_m to the
    equation of motion, so U gains the phase e^{-i theta (V + mu)} per site."""
    seq = kinetic_sequence(ndim)
    ext = external(V, mu)
    if split == "interleaved":
        theta = eps * eps / len(seq)
        for ax, q in seq:
            a, b = potential(a, b, theta, g, ext)
            a, b = iprime(a, b, ax, q)
    elif split == "plain":
        a, b = potential(a, b, eps * eps, g, ext)
        for ax, q in seq:
            a, b = iprime(a, b, ax, q)
    else:
        raise ValueError(split)
    return a, b


def run(a, b, nsteps: int, eps: float, g, ndim: int, split: str = "interleaved", V=None, mu: float = 0.0):
    for _ in range(nsteps):
        a, b = step(a, b, eps, g, ndim, split, V, mu)
    return a, b


def run_psi(psi: np.ndarray, nsteps: int, eps: float, g, split: str = "interleaved", V=None, mu: float = 0.0):
    """Convenience: encode a numpy psi (5, ...) field, run, return (a, b) tensors."""
    p = torch.from_numpy(np.ascontiguousarray(psi)).to(CDT)
    a, b = encode(p)
    ndim = p.dim() - 1
    with torch.no_grad():
        return run(a, b, nsteps, eps, g, ndim, split, V, mu)


# ---------------------------------------------------------------------------
# Observables (Sec. IV overlap energy; continuum energy of eq. hamspin2)
# ---------------------------------------------------------------------------
def energy(psi: torch.Tensor, eps: float, g, V=None, mu: float = 0.0) -> torch.Tensor:
    """E = eps^d sum_x [ sum_axis |psi(x+e) - psi(x)|^2 / eps^2 + (V + mu) n
                         + (g0 n^2 + g1 |F|^2 + g2 |sigma|^2 / 5) / 2 ].

    The kinetic term is the forward-difference form of psi^H (-lap) psi with
    hbar = 1, m = 1/2; sigma = psi^T S psi = 2 psi_2 psi_-2 - 2 psi_1 psi_-1 + psi_0^2.
    """
    g0, g1, g2 = g
    d = psi.dim() - 1
    kin = torch.zeros((), dtype=RDT)
    for ax in ["x", "y", "z"][:d]:
        diff = torch.roll(psi, shifts=-1, dims=_dim(psi, ax)) - psi
        kin = kin + (diff.abs() ** 2).sum() / (eps * eps)
    n, F, v = invariants(psi)
    sigma = (v.conj() * psi).sum(0)
    f2 = F[0] ** 2 + F[1] ** 2 + F[2] ** 2
    pot = 0.5 * (g0 * n * n + g1 * f2 + g2 * sigma.abs() ** 2 / 5).sum()
    ext = external(V, mu)
    if ext is not None:
        pot = pot + (ext * n).sum()
    return (eps ** d) * (kin + pot)


def observables(a, b, eps: float, g, prev_psi: Optional[torch.Tensor] = None, V=None,
                mu: float = 0.0) -> Dict[str, float]:
    d = a.dim() - 1
    meas = eps ** d
    psi = a + b
    out = {
        "norm_q": float(meas * ((a.abs() ** 2).sum() + (b.abs() ** 2).sum())),
        "norm_psi": float(meas * (psi.abs() ** 2).sum()),
        "pop": [float(meas * (psi[i].abs() ** 2).sum()) for i in range(5)],
        "energy": float(energy(psi, eps, g, V, mu)),
    }
    if prev_psi is not None:
        nn = (psi.abs() ** 2).sum()
        ov = (psi.conj() * prev_psi).sum()
        e_ov = 1j * (nn - ov) / nn
        out["e_overlap"] = complex(e_ov)
    return out


def density_l2_error(psi_exact: torch.Tensor, psi_sim: torch.Tensor) -> float:
    """Sec. VII: sum over the lattice of (psi psi^H - psi_sim psi_sim^H)^2."""
    n1 = (psi_exact.abs() ** 2).sum(0)
    n2 = (psi_sim.abs() ** 2).sum(0)
    return float(((n1 - n2) ** 2).sum())


# ---------------------------------------------------------------------------
# Diagnostic fields (Sec. III eq. cmap) and lattice vorticity (Sec. VI)
# ---------------------------------------------------------------------------
def fields(psi: torch.Tensor) -> Dict[str, torch.Tensor]:
    """Per-site n, F_par = F_z, F_perp = sqrt(F_x^2 + F_y^2) and |A00| = |sigma| / sqrt(5),
    sigma = psi^T S psi = 2 psi_2 psi_-2 - 2 psi_1 psi_-1 + psi_0^2 (the general forms: the
    printed component formulas hold for real psi only)."""
    n, F, _ = invariants(psi)
    sigma = 2 * psi[0] * psi[4] - 2 * psi[1] * psi[3] + psi[2] * psi[2]
    return {"n": n, "f_par": F[2], "f_perp": torch.sqrt(F[0] ** 2 + F[1] ** 2),
            "a00": sigma.abs() / math.sqrt(5.0)}


def _wrap(d: np.ndarray) -> np.ndarray:
    """A difference of two phases in [-pi, pi] (so d in [-2 pi, 2 pi]) reduced to (-pi, pi]."""
    return np.where(d > np.pi, d - 2 * np.pi, np.where(d <= -np.pi, d + 2 * np.pi, d))


def _plane_vorticity(S: np.ndarray, ua: int, va: int) -> Tuple[np.ndarray, np.ndarray]:
    """omega = d_u v_v - d_v v_u and the windings of the plaquettes c -> c+u -> c+u+v -> c+v, in the
    planes spanned by array axes ua (u) and va (v), for a periodic phase field S."""
    su = lambda f, k: np.roll(f, -k, axis=ua)   # noqa: E731  f(c + k u)
    sv = lambda f, k: np.roll(f, -k, axis=va)   # noqa: E731  f(c + k v)
    vu = _wrap(su(S, 1) - su(S, -1)) / 2
    vv = _wrap(sv(S, 1) - sv(S, -1)) / 2
    omega = (su(vv, 1) - su(vv, -1) - sv(vu, 1) + sv(vu, -1)) / 2
    s10, s11, s01 = su(S, 1), su(sv(S, 1), 1), sv(S, 1)
    circ = _wrap(s10 - S) + _wrap(s11 - s10) + _wrap(s01 - s11) + _wrap(S - s01)
    return omega, np.rint(circ / (2 * np.pi)).astype(np.int32)


def vorticity(psi_m: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Vorticity of one component on a periodic (Ny, Nx) lattice, Sec. VI: S = arg psi_m (0 where
    psi_m = 0); v_x = (S(x+1) - S(x-1)) / 2 and v_y likewise, each difference wrapped to (-pi, pi];
    omega = (v_y(x+1, y) - v_y(x-1, y) - v_x(x, y+1) + v_x(x, y-1)) / 2, the central-difference curl
    (the printed stencil swaps v_x and v_y in two terms).  Also the winding number of every
    plaquette (x, y) -> (x+1, y) -> (x+1, y+1) -> (x, y+1): the sum of its four wrapped phase
    differences over 2 pi, an integer, indexed by its corner (x, y).

    On a periodic (Nz, Ny, Nx) lattice (the paper's method in 3D, which it names as future work):
    the same in each family of lattice planes, the three components of the curl omega = curl v
    and the windings of the plaquettes normal to x, y and z, circulated y -> z, z -> x and x -> y
    (right-handed about the normal); both arrays have shape (3, Nz, Ny, Nx), components x, y, z."""
    psi_m = np.asarray(psi_m, dtype=np.complex128)
    S = np.where(psi_m == 0, 0.0, np.angle(psi_m))
    if S.ndim == 2:
        return _plane_vorticity(S, 1, 0)          # u = x, v = y
    planes = [_plane_vorticity(S, 1, 0),          # normal x: u = y, v = z
              _plane_vorticity(S, 0, 2),          # normal y: u = z, v = x
              _plane_vorticity(S, 2, 1)]          # normal z: u = x, v = y
    return np.stack([o for o, _ in planes]), np.stack([w for _, w in planes])
