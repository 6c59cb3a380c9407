"""Free-fermion reference for the XX chain (oracle).

For Jz = 0 the XXZ chain H = sum_b J_b Jxy (Sx Sx + Sy Sy) maps, by the
Jordan-Wigner transformation (the fermion mapping the paper uses for its
fermionic operators, App. Convenient features), to free fermions hopping
with amplitude J_b Jxy / 2 between neighbours:
    H = sum_b (J_b Jxy / 2) (c_b^dag c_{b+1} + h.c.),
with n_i = c_i^dag c_i = S^z_i + 1/2 (spin up = occupied).

The correlation matrix C_ij = <c_i^dag c_j> of a Gaussian state evolves as
C(t) = U(t)^* C(0) U(t)^T with U = exp(-i h t) (single-particle h), so
<S^z_i>(t) = C_ii(t) - 1/2.

A nearest-neighbour XX gate exp(-i tau h_b) is itself the exponential of a
fermion bilinear on two adjacent sites (no Jordan-Wigner string), so a
Trotterized TEBD circuit of XX gates is exactly the product of the 2x2 blocks
exp(-i tau h^(b)) embedded in the L x L single-particle space.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def hopping_matrix(J_b, Jxy=1.0) -> np.ndarray:
    L = len(J_b) + 1
    h = np.zeros((L, L))
    for b, J in enumerate(J_b):
        h[b, b + 1] = h[b + 1, b] = 0.5 * J * Jxy
    return h


def neel_correlation(L: int) -> np.ndarray:
    """C(0) of the Neel state up, down, up, ...: occupied on even sites."""
    return np.diag([1.0 if i % 2 == 0 else 0.0 for i in range(L)]).astype(np.complex128)


def evolve_exact(C0: np.ndarray, h: np.ndarray, t: float) -> np.ndarray:
    U = scipy.linalg.expm(-1j * t * h)
    return U.conj() @ C0 @ U.T


def bond_unitary(L: int, b: int, amp: float, tau: float) -> np.ndarray:
    """Single-particle unitary of the two-site gate exp(-i tau amp (c_b^dag
    c_{b+1} + h.c.)) embedded in L x L."""
    U = np.eye(L, dtype=np.complex128)
    blk = scipy.linalg.expm(-1j * tau * amp * np.array([[0, 1], [1, 0]]))
    U[b:b + 2, b:b + 2] = blk
    return U


def evolve_trotter(C0: np.ndarray, J_b, Jxy: float, layers_per_step, n_steps: int):
    """Apply the gate layers [(bonds, tau), ...] n_steps times.  Returns the
    list of C after every step (index 0 = initial)."""
    L = C0.shape[0]
    Ustep = np.eye(L, dtype=np.complex128)
    for bonds, tau in layers_per_step:
        for b in bonds:
            Ustep = bond_unitary(L, b, 0.5 * J_b[b] * Jxy, tau) @ Ustep
    out = [C0]
    C = C0
    for _ in range(n_steps):
        C = Ustep.conj() @ C @ Ustep.T
        out.append(C)
    return out


def sz_from_C(C: np.ndarray) -> np.ndarray:
    return np.real(np.diag(C)) - 0.5
