"""Model definitions for the GPU path: two-site bond Hamiltonians.

These matrices are the *input* of the method (the Hamiltonian the state is
evolved with), built once on the host in FP64 and uploaded; every step of the
update itself runs in the HIP kernels.

Spin-1/2 basis index 0 = up (sigma^z = +1); bosons in the Fock basis.
Two-site index (s_out*d + t_out, s_in*d + t_in), s = left site.
Transverse Ising (Eq. Ising): h_b = -J sz sz - J g (wl sx x 1 + wr 1 x sx);
XXZ: h_b = J_b [Jxy (Sx Sx + Sy Sy) + Jz_b Sz Sz], S = sigma/2;
Bose-Hubbard (Eq. bosehubbard, mu = 0): h_b = -t (b^dag x b + b x b^dag)
  + (U/2) (wl n(n-1) x 1 + wr 1 x n(n-1)).
A site term is shared half/half by the two bonds of an interior site and
carried whole by the single bond of an end site (wl, wr).
"""
from __future__ import annotations

import numpy as np


def _pauli():
    x = np.array([[0.0, 1.0], [1.0, 0.0]], dtype=np.complex128)
    y = np.array([[0.0, -1.0j], [1.0j, 0.0]], dtype=np.complex128)
    z = np.array([[1.0, 0.0], [0.0, -1.0]], dtype=np.complex128)
    return x, y, z


def _weights(b, L):
    return (1.0 if b == 0 else 0.5), (1.0 if b == L - 2 else 0.5)


def bond_hamiltonians(spec) -> np.ndarray:
    """(L-1, d*d, d*d) complex128 array of bond Hamiltonians of a ChainSpec."""
    L, d = spec.L, spec.d
    out = np.zeros((L - 1, d * d, d * d), dtype=np.complex128)
    if spec.model == "tfim":
        x, _, z = _pauli()
        one = np.eye(2)
        J, g = spec.params["J"], spec.params["g"]
        for b in range(L - 1):
            wl, wr = _weights(b, L)
            out[b] = -J * np.kron(z, z) - J * g * (wl * np.kron(x, one) + wr * np.kron(one, x))
    elif spec.model == "xxz":
        x, y, z = _pauli()
        Jxy = spec.params["Jxy"]
        for b in range(L - 1):
            out[b] = spec.J_b[b] * 0.25 * (Jxy * (np.kron(x, x) + np.kron(y, y)) + spec.Jz_b[b] * np.kron(z, z))
    elif spec.model == "bh":
        n = np.arange(d, dtype=np.float64)
        a = np.diag(np.sqrt(n[1:]), 1).astype(np.complex128)     # annihilation
        ad = a.conj().T
        onsite = np.diag(0.5 * spec.params["U"] * n * (n - 1)).astype(np.complex128)
        one = np.eye(d)
        t = spec.params["t"]
        for b in range(L - 1):
            wl, wr = _weights(b, L)
            out[b] = -t * (np.kron(ad, a) + np.kron(a, ad)) + wl * np.kron(onsite, one) + wr * np.kron(one, onsite)
    else:
        raise ValueError(spec.model)
    return out


def sz_operator() -> np.ndarray:
    return np.array([[0.5, 0.0], [0.0, -0.5]], dtype=np.complex128)


def number_operator(d: int) -> np.ndarray:
    return np.diag(np.arange(d)).astype(np.complex128)


def mpo(spec) -> np.ndarray:
    """MPO matrices W[k] as an (L, w, w, d, d) complex128 array, [b_l][b_r][s_out][s_in].

    Lower-triangular MPO-matrix form (Eq. MPOdef): identity at the top-left
    (terms finished) and bottom-right (terms not started); the last row opens a
    term, the first column closes it.  The left boundary selects row w-1 and
    the right boundary column 0.
    """
    L, d = spec.L, spec.d
    if spec.model == "tfim":
        x, _, z = _pauli()
        one = np.eye(2)
        J, g = spec.params["J"], spec.params["g"]
        W = np.zeros((L, 3, 3, 2, 2), dtype=np.complex128)
        W[:, 0, 0] = one
        W[:, 1, 0] = z
        W[:, 2, 0] = -J * g * x
        W[:, 2, 1] = -J * z
        W[:, 2, 2] = one
        return W
    if spec.model == "xxz":
        sp = np.array([[0.0, 1.0], [0.0, 0.0]], dtype=np.complex128)
        sm = sp.T.copy()
        sz = np.diag([0.5, -0.5]).astype(np.complex128)
        one = np.eye(2)
        Jxy = spec.params["Jxy"]
        W = np.zeros((L, 5, 5, 2, 2), dtype=np.complex128)
        W[:, 0, 0] = one
        W[:, 1, 0] = sp
        W[:, 2, 0] = sm
        W[:, 3, 0] = sz
        W[:, 4, 4] = one
        for k in range(L - 1):
            W[k, 4, 1] = 0.5 * spec.J_b[k] * Jxy * sm
            W[k, 4, 2] = 0.5 * spec.J_b[k] * Jxy * sp
            W[k, 4, 3] = spec.J_b[k] * spec.Jz_b[k] * sz
        return W
    if spec.model == "bh":
        n = np.arange(d, dtype=np.float64)
        a = np.diag(np.sqrt(n[1:]), 1).astype(np.complex128)
        ad = a.conj().T
        one = np.eye(d)
        t, U = spec.params["t"], spec.params["U"]
        W = np.zeros((L, 4, 4, d, d), dtype=np.complex128)
        W[:, 0, 0] = one
        W[:, 1, 0] = ad
        W[:, 2, 0] = a
        W[:, 3, 0] = np.diag(0.5 * U * n * (n - 1))
        W[:, 3, 1] = -t * a
        W[:, 3, 2] = -t * ad
        W[:, 3, 3] = one
        return W
    raise ValueError(spec.model)
