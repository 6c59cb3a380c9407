"""State-vector references (oracle): exact propagation, the exact Trotter
circuit, reduced density matrices and the paper's error measures.

* exact propagation exp(-i H T) psi0 by dense eigendecomposition (small L) or
  scipy's expm_multiply; for a time-independent H this is the paper's exact
  diagonalisation reference (Sec. Computational error and convergence) with
  no time-ordering error.
* the exact Trotter circuit applies the very gate sequence TEBD applies, to a
  d^L state vector, so it is the exact target of an untruncated TEBD run.
* error measures: maximal single-site and two-site trace distances
  (Eqs. erhoi and the two-site variant), energy error, and the half-chain
  entropy error (Eq. eentr).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse.linalg

from . import models


def product_vector(vectors: np.ndarray) -> np.ndarray:
    v = np.ones(1, dtype=np.complex128)
    for x in vectors:
        v = np.kron(v, x / np.linalg.norm(x))
    return v


def apply_two_site(psi: np.ndarray, G: np.ndarray, b: int, L: int, d: int) -> np.ndarray:
    t = psi.reshape(d ** b, d * d, d ** (L - b - 2))
    t = np.einsum("ij,ajc->aic", G, t)
    return t.reshape(-1)


def _suzuki_p() -> float:
    """Weight p of the five-stage fourth-order fractal U2(p)U2(p)U2(1-4p)U2(p)U2(p):
    the third-order error cancels when 4 p^3 + (1 - 4p)^3 = 0.  Taken here as
    the real root of that cubic, so the circuit does not share the closed
    form the MPS schedule uses."""
    roots = np.roots([4.0 - 64.0, 48.0, -12.0, 1.0])   # 4p^3 + (1-4p)^3 expanded
    real = roots[np.abs(roots.imag) < 1e-12].real
    return float(real[0])


def circuit_schedule(method: str, L: int, dt: float):
    """The ordered list of (bond, tau) exponentials of one time step, written
    from the definitions independently of the MPS code: Strang splitting with
    the bonds b = 0, 2, 4, ... (the paper's odd bonds, 1-based) applied first
    and last with tau/2 and the others with tau in between; the fourth-order
    fractal of five Strang steps; the Sornborger-Stewart sweep (every bond
    left to right, then right to left, each with dt/2; Eq. sornborger2)."""
    def strang(tau):
        first = [(b, 0.5 * tau) for b in range(L - 1) if b % 2 == 0]
        middle = [(b, tau) for b in range(L - 1) if b % 2 == 1]
        return first + middle + list(first)
    if method == "tebd2":
        return strang(dt)
    if method == "tebd4":
        p = _suzuki_p()
        out = []
        for w in (p, p, 1.0 - 4.0 * p, p, p):
            out += strang(w * dt)
        return out
    if method == "sweep":
        right = [(b, 0.5 * dt) for b in range(L - 1)]
        return right + right[::-1]
    raise ValueError(method)


def trotter_circuit(spec, method: str, dt: float, n_steps: int, psi0=None, observe=None):
    """Apply the TEBD gate sequence of ``method`` to the state vector.  The
    two-site propagators are matrix exponentials (scipy's Pade expm), not the
    eigendecomposition the MPS code uses, and the schedule is
    ``circuit_schedule``: nothing of the MPS update is shared."""
    from workloads import initial_vectors
    L, d = spec.L, spec.d
    psi = product_vector(initial_vectors(spec)) if psi0 is None else psi0.copy()
    hs = models.bond_hamiltonians(spec)
    cache = {}
    if observe:
        observe(psi, 0)
    for n in range(1, n_steps + 1):
        for b, tau in circuit_schedule(method, L, dt):
            key = (b, tau)
            if key not in cache:
                cache[key] = scipy.linalg.expm(-1j * tau * hs[b])
            psi = apply_two_site(psi, cache[key], b, L, d)
        if observe:
            observe(psi, n)
    return psi


def exact_evolve(H: np.ndarray, psi0: np.ndarray, t: float) -> np.ndarray:
    if H.shape[0] <= 4096:
        e, V = np.linalg.eigh(H)
        return V @ (np.exp(-1j * t * e) * (V.conj().T @ psi0))
    return scipy.sparse.linalg.expm_multiply(-1j * t * scipy.sparse.csr_matrix(H), psi0)


def expect_local(psi: np.ndarray, op: np.ndarray, L: int, d: int) -> np.ndarray:
    out = []
    for i in range(L):
        t = psi.reshape(d ** i, d, d ** (L - i - 1))
        out.append(float(np.real(np.einsum("asc,st,atc->", t.conj(), op, t))))
    return np.array(out)


def expect_bond(psi: np.ndarray, op2: np.ndarray, b: int, L: int, d: int) -> float:
    t = psi.reshape(d ** b, d * d, d ** (L - b - 2))
    return float(np.real(np.einsum("asc,st,atc->", t.conj(), op2, t)))


def rdm1(psi: np.ndarray, i: int, L: int, d: int) -> np.ndarray:
    t = psi.reshape(d ** i, d, d ** (L - i - 1))
    return np.einsum("asc,arc->sr", t, t.conj())


def rdm2(psi: np.ndarray, i: int, j: int, L: int, d: int) -> np.ndarray:
    t = psi.reshape([d] * L)
    rest = [k for k in range(L) if k not in (i, j)]
    t = np.transpose(t, [i, j] + rest).reshape(d * d, -1)
    return t @ t.conj().T


def trace_distance(r1: np.ndarray, r2: np.ndarray) -> float:
    """D = 1/2 |r1 - r2|, |A| = sqrt(A^dag A) (Eq. erhoi)."""
    ev = np.linalg.eigvalsh(r1 - r2)
    return 0.5 * float(np.sum(np.abs(ev)))


def half_chain_entropy(psi: np.ndarray, L: int, d: int) -> float:
    s = np.linalg.svd(psi.reshape(d ** (L // 2), -1), compute_uv=False)
    p = s ** 2
    p = p[p > 1e-300]
    return float(-np.sum(p * np.log(p)))


def error_measures(psi: np.ndarray, ref: np.ndarray, H: np.ndarray, L: int, d: int) -> dict:
    """The four error measures of Sec. Computational error and convergence."""
    e_loc = max(trace_distance(rdm1(psi, i, L, d), rdm1(ref, i, L, d)) for i in range(L))
    e_cor = max(trace_distance(rdm2(psi, i, j, L, d), rdm2(ref, i, j, L, d))
                for i in range(L) for j in range(i + 1, L))
    e_E = abs(float(np.real(np.vdot(psi, H @ psi))) - float(np.real(np.vdot(ref, H @ ref))))
    e_S = abs(half_chain_entropy(psi, L, d) - half_chain_entropy(ref, L, d))
    return {"eps_local": e_loc, "eps_corr": e_cor, "eps_E": e_E, "eps_S": e_S}


def ground_state(H: np.ndarray) -> np.ndarray:
    e, V = np.linalg.eigh(H)
    return V[:, 0]
