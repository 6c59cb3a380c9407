"""Vidal/Hastings-form MPS and the TEBD two-site update (oracle, complex128).

State layout (0-based):
  B[i]   : array [chi_i][d][chi_{i+1}], right-canonical (B = Gamma Lambda)
  lam[j] : Schmidt values on virtual bond j (left of site j), j = 0..L;
           lam[0] = lam[L] = [1]
The wave function is lam[0] B[0] B[1] ... B[L-1] (Eq. mps with the Schmidt
values of Eq. schmidt kept on the bonds).

Bond b joins sites b and b+1 and owns the Schmidt values lam[b+1].

The update of bond b with gate G (a d^2 x d^2 unitary) follows the
contraction / gate / split description of Sec. "Basic concepts" (two-site
tensor Theta, SVD split with truncation) and App. "Details of the Krylov
method" (steps 1, 3, 4 of the plain TEBD update), in the Hastings form that
never divides by Schmidt values:
  1. theta~  = B_b . B_{b+1}                      (contract over the bond)
  2. theta~' = G theta~                           (gate on the two sites)
  3. theta'  = lam[b] * theta~'                   (left Schmidt values)
  4. theta'  = U S V^dag                           (SVD, (chi d) x (d chi))
  5. k by the count rule; w = sum_{j>k} s_j^2; n_k = sqrt(sum_{j<=k} s_j^2)
  6. lam[b+1] = s_{1..k} / n_k                     (App. Auxiliary calculations)
  7. B_{b+1}  = V^dag_{1..k}
  8. B_b      = theta~' V_{1..k} / n_k

Count rule: k = min(chi_max, min{k >= 1 : sum_{j>k} s_j^2 <= eps * sum_j s_j^2}),
the local-tolerance truncation of Sec. "Basic concepts" (discarded weight
bounds 1 - <psi'|psi>, Eq. elocal).  eps < 0 keeps min(chi_max, rank-dim)
values, zeros included.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np
import scipy.linalg

from . import models

P4 = 1.0 / (4.0 - 4.0 ** (1.0 / 3.0))   # Suzuki fractal weight for TEBD4


@dataclass
class MPS:
    B: List[np.ndarray]
    lam: List[np.ndarray]
    d: int
    disc: List[float] = field(default_factory=list)   # discarded weight log

    @property
    def L(self):
        return len(self.B)

    def chis(self):
        return [len(x) for x in self.lam]

    def copy(self):
        return MPS([b.copy() for b in self.B], [l.copy() for l in self.lam], self.d, list(self.disc))


def product_mps(vectors: np.ndarray) -> MPS:
    """Product state from (L, d) local vectors (normalised)."""
    L, d = vectors.shape
    B = []
    for i in range(L):
        v = vectors[i] / np.linalg.norm(vectors[i])
        B.append(v.reshape(1, d, 1).astype(np.complex128))
    lam = [np.ones(1) for _ in range(L + 1)]
    return MPS(B, lam, d)


def gate(h: np.ndarray, tau: complex) -> np.ndarray:
    """exp(-i tau h) for Hermitian h by eigendecomposition (real tau)."""
    e, V = np.linalg.eigh(h)
    return (V * np.exp(-1j * tau * e)) @ V.conj().T


def svd(theta: np.ndarray):
    """Full reduced SVD, LAPACK gesdd with gesvd as fallback."""
    try:
        return scipy.linalg.svd(theta, full_matrices=False, lapack_driver="gesdd")
    except np.linalg.LinAlgError:
        return scipy.linalg.svd(theta, full_matrices=False, lapack_driver="gesvd")


def count_rule(s: np.ndarray, chi_max: int, eps: float) -> int:
    r = len(s)
    if eps < 0:
        return min(chi_max, r)
    s2 = s.astype(np.float64) ** 2
    total = s2.sum()
    k = r
    for kk in range(1, r + 1):
        if s2[kk:].sum() <= eps * total:
            k = kk
            break
    return max(1, min(chi_max, k))


def truncate(theta_mat: np.ndarray, chi_max: int, eps: float):
    """SVD split with truncation.  Returns U_k, s_k (unnormalised), Vh_k,
    discarded weight w = sum_{j>k} s_j^2, norm n_k and the full spectrum."""
    U, s, Vh = svd(theta_mat)
    k = count_rule(s, chi_max, eps)
    w = float(np.sum(s[k:] ** 2))
    nk = float(np.sqrt(np.sum(s[:k] ** 2)))
    return U[:, :k], s[:k], Vh[:k], w, nk, s


def truncate_eig(theta_mat: np.ndarray, chi_max: int, eps: float):
    """The eigendecomposition split of Sec. "Basic concepts" (Eq. AAD_ULLUD):
    the Hermitian A A^dag = U lambda^2 U^dag gives U and the squared singular
    values; U^dag A = lambda V^dag then gives the right factor, so the kept
    rows of V^dag are (U^dag A)_j / lambda_j.  Same count rule and outputs as
    ``truncate`` (eigenvalues sorted descending, negative round-off set to 0;
    a kept row with lambda_j = 0, possible only with eps < 0, is left zero).
    The squared values carry an absolute error of order eps_mach lambda_1^2, so
    a singular value s_j comes out with relative error ~ eps_mach (s_1/s_j)^2."""
    A = theta_mat
    ev, U = np.linalg.eigh(A @ A.conj().T)
    order = np.argsort(ev)[::-1]
    lam2 = np.maximum(ev[order], 0.0)
    U = U[:, order]
    s = np.sqrt(lam2)
    k = count_rule(s, chi_max, eps)
    w = float(np.sum(lam2[k:]))
    nk = float(np.sqrt(np.sum(lam2[:k])))
    inv = np.divide(1.0, s[:k], out=np.zeros(k), where=s[:k] > 0)
    Vh = (U[:, :k].conj().T @ A) * inv[:, None]
    return U[:, :k], s[:k], Vh, w, nk, s


def apply_bond(psi: MPS, b: int, G: np.ndarray, chi_max: int, eps: float) -> float:
    """One Hastings-form two-site update of bond b.  Returns discarded weight."""
    d = psi.d
    Bl, Br = psi.B[b], psi.B[b + 1]
    chl, chr_ = Bl.shape[0], Br.shape[2]
    theta_t = np.einsum("asb,btc->astc", Bl, Br)
    G4 = G.reshape(d, d, d, d)
    theta_tp = np.einsum("uvst,astc->auvc", G4, theta_t)
    theta_p = psi.lam[b][:, None, None, None] * theta_tp
    mat = theta_p.reshape(chl * d, d * chr_)
    _, s, Vh, w, nk, _ = truncate(mat, chi_max, eps)
    k = len(s)
    psi.lam[b + 1] = s / nk
    psi.B[b + 1] = Vh.reshape(k, d, chr_)
    psi.B[b] = (theta_tp.reshape(chl * d, d * chr_) @ Vh.conj().T / nk).reshape(chl, d, k)
    psi.disc.append(w)
    return w


# ---------------------------------------------------------------------------
# Schedules
# ---------------------------------------------------------------------------

def strang_layers(L: int, tau: float):
    """TEBD2 (Strang even/odd) for one step tau: list of (bonds, tau_layer).

    Odd bonds in the paper's 1-based numbering (b = 1, 3, 5, ...; 0-based
    0, 2, 4, ...) with tau/2, then even bonds with tau, then odd with tau/2.
    This is the Suzuki-Trotter even/odd alternative the paper names next to
    the Sornborger-Stewart sweep (Sec. Sornborger-Stewart decomposition).
    """
    odd = list(range(0, L - 1, 2))
    even = list(range(1, L - 1, 2))
    return [(odd, 0.5 * tau), (even, tau), (odd, 0.5 * tau)]


def tebd4_layers(L: int, dt: float):
    """TEBD4 as Suzuki's 5-stage fractal of TEBD2 steps:
    U4(dt) = U2(p dt) U2(p dt) U2((1-4p) dt) U2(p dt) U2(p dt),
    p = 1/(4 - 4^(1/3)).  Error O(dt^4) (Sec. Sornborger-Stewart)."""
    layers = []
    for c in (P4, P4, 1.0 - 4.0 * P4, P4, P4):
        layers += strang_layers(L, c * dt)
    return layers


def sweep_layers(L: int, dt: float):
    """Sornborger-Stewart second-order sweep, Eq. sornborger2: left-to-right
    over every bond with dt/2, then right-to-left with dt/2 (the rightmost
    product factor acts first)."""
    return [([b], 0.5 * dt) for b in range(L - 1)] + [([b], 0.5 * dt) for b in range(L - 2, -1, -1)]


def step_layers(method: str, L: int, dt: float):
    if method == "tebd2":
        return strang_layers(L, dt)
    if method == "tebd4":
        return tebd4_layers(L, dt)
    if method == "sweep":
        return sweep_layers(L, dt)
    raise ValueError(method)


class GateCache:
    def __init__(self, hs):
        self.hs = hs
        self.cache = {}

    def __call__(self, b, tau):
        key = (b, float(tau))
        if key not in self.cache:
            self.cache[key] = gate(self.hs[b], tau)
        return self.cache[key]


def tebd_run(spec, method: str, dt: float, n_steps: int, eps: float, chi_max=None,
             observe=None, psi=None):
    """Evolve the product state of ``spec`` for n_steps.  ``observe(psi, step)``
    is called after every step (and at step 0)."""
    chi_max = spec.chi_max if chi_max is None else chi_max
    from workloads import initial_vectors
    psi = product_mps(initial_vectors(spec)) if psi is None else psi
    gates = GateCache(models.bond_hamiltonians(spec))
    layers = step_layers(method, spec.L, dt)
    if observe:
        observe(psi, 0)
    for n in range(1, n_steps + 1):
        for bonds, tau in layers:
            for b in bonds:
                apply_bond(psi, b, gates(b, tau), chi_max, eps)
        if observe:
            observe(psi, n)
    return psi


# ---------------------------------------------------------------------------
# Observables (Sec. Observables; reduced density matrices Eq. reducedrho)
# ---------------------------------------------------------------------------

def site_rdm(psi: MPS, i: int) -> np.ndarray:
    """rho_i[s, s'] = sum_{a,c} lam_i[a]^2 B_i[a,s,c] conj(B_i[a,s',c])."""
    B = psi.B[i]
    l2 = psi.lam[i] ** 2
    return np.einsum("a,asc,arc->sr", l2, B, B.conj())


def local_expect(psi: MPS, op: np.ndarray) -> np.ndarray:
    return np.array([np.real(np.trace(site_rdm(psi, i) @ op.T)) for i in range(psi.L)])


def theta_bond(psi: MPS, b: int) -> np.ndarray:
    return psi.lam[b][:, None, None, None] * np.einsum("asb,btc->astc", psi.B[b], psi.B[b + 1])


def bond_expect(psi: MPS, b: int, h: np.ndarray) -> float:
    th = theta_bond(psi, b)
    d = psi.d
    th2 = th.transpose(1, 2, 0, 3).reshape(d * d, -1)
    return float(np.real(np.vdot(th2, h @ th2)))


def energy(psi: MPS, hs) -> float:
    return sum(bond_expect(psi, b, hs[b]) for b in range(psi.L - 1))


def szsz(psi: MPS) -> np.ndarray:
    sz = 0.5 * models.SZ
    o = np.kron(sz, sz)
    return np.array([bond_expect(psi, b, o) for b in range(psi.L - 1)])


def entropies(psi: MPS) -> np.ndarray:
    out = []
    for l in psi.lam[1:-1]:
        p = l ** 2
        p = p[p > 0]
        out.append(float(-np.sum(p * np.log(p))))
    return np.array(out)


def norm2(psi: MPS) -> float:
    """<psi|psi> by contraction of the transfer matrices from the left."""
    E = np.diag(psi.lam[0] ** 2).astype(np.complex128)
    for B in psi.B:
        E = np.einsum("ab,asc,bsd->cd", E, B.conj(), B)
    return float(np.real(np.trace(E)))


def to_vector(psi: MPS) -> np.ndarray:
    """Dense state vector (small L), index order site 0 most significant."""
    v = psi.lam[0][:, None] * psi.B[0].reshape(psi.B[0].shape[0], -1)
    v = v.reshape(-1, psi.B[0].shape[2])
    for B in psi.B[1:]:
        v = v @ B.reshape(B.shape[0], -1)
        v = v.reshape(-1, B.shape[2])
    return v.reshape(-1)


def from_vector(vec: np.ndarray, L: int, d: int, chi_max=10 ** 9, eps=-1.0) -> MPS:
    """Exact MPS of a state vector by successive SVDs (Eq. mps), brought to
    Hastings form.  eps < 0 keeps all Schmidt values."""
    lam = [np.ones(1)]
    As = []
    rest = vec.reshape(1, -1)
    for i in range(L - 1):
        chl = rest.shape[0]
        mat = rest.reshape(chl * d, -1)
        U, s, Vh = svd(mat)
        k = count_rule(s, chi_max, eps)
        As.append(U[:, :k].reshape(chl, d, k))
        lam.append(s[:k] / np.linalg.norm(s[:k]))
        rest = s[:k, None] * Vh[:k]
    As.append(rest.reshape(rest.shape[0], d, 1) / np.linalg.norm(rest))
    lam.append(np.ones(1))
    # left-canonical A_i -> Hastings B_i = lam_i^{-1} A_i lam_{i+1}
    B = []
    for i in range(L):
        li = lam[i]
        inv = np.where(li > 1e-300, 1.0 / np.where(li > 0, li, 1.0), 0.0)
        Bi = inv[:, None, None] * As[i]
        if i < L - 1:
            Bi = Bi * lam[i + 1][None, None, :]
        B.append(Bi)
    return MPS(B, lam, d)
