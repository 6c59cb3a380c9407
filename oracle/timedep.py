"""Time-dependent Hamiltonians by commutator-free Magnus expansions (oracle,
complex128).

Sec. "Time evolution methods" (time ordering of the propagators): for
H(t) = sum_k f_k(t) H_k the propagator over [t, t + dt] is a product of s
exponentials, each of a linear combination of the Hamiltonian at a few nodes
t + c_j dt.  Unitarity is explicit and no commutator or nested integral
appears.  The paper's default (order N = 2, s = 1) is the midpoint rule,
    U(t + dt, t) = exp(-i dt H(t + dt/2)).
The fourth-order scheme with two exponentials is the one of the cited
commutator-free expansions:
    nodes c_{1,2} = 1/2 -+ sqrt(3)/6, weights a_1 = (3 - 2 sqrt 3)/12,
    a_2 = (3 + 2 sqrt 3)/12,
    U = exp(-i dt (a_1 H_1 + a_2 H_2)) exp(-i dt (a_2 H_1 + a_1 H_2)),
with H_j = H(t + c_j dt) and the right factor acting first.  Each
exponential exp(-i dt A) with A = sum_k w_k H_k is taken as one Trotter step
of ``mps`` (TEBD2, TEBD4 or the sweep) whose bond Hamiltonians are
h_b = sum_k w_k h_b^(k), the bond split of every H_k.

The paper's exact-diagonalisation reference for its Ising quench applies
exp(-i H(t_n + dt/2) dt) to the state vector for every step n: the midpoint
rule without the Trotter splitting (``exact_midpoint``).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import mps

_S3 = np.sqrt(3.0)
# scheme -> (nodes c_j, weights W[e][j] of node j in exponential e, in the
# order the exponentials are applied)
SCHEMES = {
    2: (np.array([0.5]), np.array([[1.0]])),
    4: (np.array([0.5 - _S3 / 6.0, 0.5 + _S3 / 6.0]),
        np.array([[(3.0 + 2.0 * _S3) / 12.0, (3.0 - 2.0 * _S3) / 12.0],
                  [(3.0 - 2.0 * _S3) / 12.0, (3.0 + 2.0 * _S3) / 12.0]])),
}


def step_coefficients(scheme: int, f, t: float, dt: float) -> np.ndarray:
    """coef[e][k]: weight of H_k in exponential e (application order) of the
    step [t, t + dt]; ``f(t)`` returns the K values f_k(t)."""
    nodes, W = SCHEMES[scheme]
    F = np.array([np.asarray(f(t + c * dt), dtype=np.float64) for c in nodes])   # [node][k]
    return W @ F


def combine(term_hs, coef) -> list:
    """Bond Hamiltonians h_b = sum_k coef[k] h_b^(k) of one exponential."""
    return [sum(c * hk[b] for c, hk in zip(coef, term_hs)) for b in range(len(term_hs[0]))]


def td_tebd_run(psi: mps.MPS, term_hs, f, method: str, dt: float, n_steps: int, eps: float, chi_max: int,
                scheme: int = 2, t0: float = 0.0, observe=None, charges=None) -> mps.MPS:
    """n_steps steps from time t0: every exponential of the scheme is one
    Trotter step of ``method`` with its combined bond Hamiltonians.
    ``charges`` = (q, qsite, modulus) of a charge-carrying chain: every
    update by ``u1.apply_bond_u1`` (q is updated in place)."""
    L = psi.L
    layers = mps.step_layers(method, L, dt)
    if observe:
        observe(psi, 0)
    for n in range(n_steps):
        for coef in step_coefficients(scheme, f, t0 + n * dt, dt):
            hs = combine(term_hs, coef)
            for bonds, tau in layers:
                for b in bonds:
                    if charges is None:
                        mps.apply_bond(psi, b, mps.gate(hs[b], tau), chi_max, eps)
                    else:
                        from .u1 import apply_bond_u1
                        q, qsite, modulus = charges
                        apply_bond_u1(psi, q, qsite, b, mps.gate(hs[b], tau), chi_max, eps, modulus)
        if observe:
            observe(psi, n + 1)
    return psi


def exact_midpoint(H_terms, f, psi0: np.ndarray, dt: float, n_steps: int, t0: float = 0.0) -> np.ndarray:
    """prod_n exp(-i dt H(t_n + dt/2)) psi0 with dense H(t) = sum_k f_k(t) H_k."""
    psi = psi0.astype(np.complex128).copy()
    for n in range(n_steps):
        fk = np.asarray(f(t0 + (n + 0.5) * dt), dtype=np.float64)
        H = sum(c * Hk for c, Hk in zip(fk, H_terms))
        e, V = np.linalg.eigh(H)
        psi = V @ (np.exp(-1j * dt * e) * (V.conj().T @ psi))
    return psi


def exact_cfme(H_terms, f, psi0: np.ndarray, dt: float, n_steps: int, scheme: int, t0: float = 0.0) -> np.ndarray:
    """The scheme's product of exponentials of the dense H (no Trotter splitting)."""
    psi = psi0.astype(np.complex128).copy()
    for n in range(n_steps):
        for coef in step_coefficients(scheme, f, t0 + n * dt, dt):
            A = sum(c * Hk for c, Hk in zip(coef, H_terms))
            psi = scipy.linalg.expm(-1j * dt * A) @ psi
    return psi
