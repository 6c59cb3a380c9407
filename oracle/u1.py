"""U(1)-symmetric truncated SVD (oracle, complex128).  TEST INFRASTRUCTURE
ONLY (see the package docstring).

App. "Convenient features" (symmetry conservation): with a diagonal symmetry
generator (a conserved charge such as the particle number or 2 S^z), a
two-site tensor cut at a bond is block diagonal in the charge carried by that
bond, and the decomposition can run on each block, a smaller subspace.  Here
a row r of theta (the left indices) carries the charge row_q[r] and a column
c (the right indices) the charge col_q[c]; theta[r, c] vanishes unless the
two agree.  The singular values of theta are the union of those of the
blocks theta[rows of charge q, columns of charge q]; the truncation (count
rule of Sec. "Basic concepts", the same as ``mps.truncate``) is applied to
that union, and every kept singular vector carries the charge of its block.

Ties between equal singular values of different blocks are ordered by charge,
then by position in the block, so the kept set is well defined.  Rows or
columns whose charge has no partner on the other side, and the rank deficit
of rectangular blocks, are structural zeros and not part of the spectrum: a
dense SVD returns them as rounding-level values, which only a tolerance of
exactly 0 (keep every nonzero value) can tell apart.
"""
from __future__ import annotations

import numpy as np

from .mps import count_rule


def charge_blocks(row_q, col_q):
    """[(q, rows, cols)] for every charge present on both sides, ascending q."""
    row_q = np.asarray(row_q)
    col_q = np.asarray(col_q)
    out = []
    for q in sorted(set(row_q.tolist()) & set(col_q.tolist())):
        out.append((int(q), np.flatnonzero(row_q == q), np.flatnonzero(col_q == q)))
    return out


def truncate_u1(theta: np.ndarray, row_q, col_q, chi_max: int, eps: float):
    """Blockwise SVD and global truncation.  Returns U_k [m][k], s_k, Vh_k
    [k][n], the charges q_k of the kept vectors, the discarded weight w, n_k
    and the full sorted spectrum, like ``mps.truncate`` plus the charges."""
    m, n = theta.shape
    vals = []  # (s, q, index in block, block number)
    vecs = []
    for bi, (q, rows, cols) in enumerate(charge_blocks(row_q, col_q)):
        U, s, Vh = np.linalg.svd(theta[np.ix_(rows, cols)], full_matrices=False)
        vecs.append((rows, cols, U, Vh))
        for j, sv in enumerate(s):
            vals.append((float(sv), q, j, bi))
    if not vals:
        raise ValueError("no charge is shared by rows and columns")
    vals.sort(key=lambda t: (-t[0], t[1], t[2]))
    s_all = np.array([v[0] for v in vals])
    k = count_rule(s_all, chi_max, eps)
    Uk = np.zeros((m, k), dtype=np.complex128)
    Vk = np.zeros((k, n), dtype=np.complex128)
    qk = np.zeros(k, dtype=np.int64)
    for j, (sv, q, jj, bi) in enumerate(vals[:k]):
        rows, cols, U, Vh = vecs[bi]
        Uk[rows, j] = U[:, jj]
        Vk[j, cols] = Vh[jj]
        qk[j] = q
    w = float(np.sum(s_all[k:] ** 2))
    nk = float(np.sqrt(np.sum(s_all[:k] ** 2)))
    return Uk, s_all[:k], Vk, qk, w, nk, s_all


# ---------------------------------------------------------------------------
# Charge-carrying chains: TEBD with the blockwise truncation.  The charge is
# additive: U(1) (modulus 0) or Z_n (modulus n, charges taken modulo n, as
# for the parity of a particle number with n = 2).
# ---------------------------------------------------------------------------

def _reduce(q, modulus: int):
    """Charges of U(1) (modulus 0) as they are; of Z_n (modulus n) in 0..n-1."""
    q = np.asarray(q, dtype=np.int64)
    return q if modulus == 0 else np.mod(q, modulus)


def product_charges(vectors: np.ndarray, qsite, modulus: int = 0) -> list:
    """Bond charges of a product of basis states: q[b] holds, for the single
    Schmidt state of bond b, the total charge of sites 0..b-1 (modulo n for a
    Z_n symmetry, modulus n).  ``vectors`` (L, d) must be basis vectors up to
    a phase."""
    qsite = np.asarray(qsite)
    q = [np.zeros(1, dtype=np.int64)]
    for v in vectors:
        s = int(np.argmax(np.abs(v)))
        if np.count_nonzero(v) != 1:
            raise ValueError("a charge-carrying product state needs basis states on every site")
        q.append(_reduce([q[-1][0] + qsite[s]], modulus))
    return q


def bond_charges(q_left, q_right, qsite, modulus: int = 0):
    """Row and column charges of theta at the bond between two sites: row
    (alpha, s1) carries q_left[alpha] + qsite[s1] (the charge left of the new
    bond), column (s2, gamma) carries q_right[gamma] - qsite[s2] (the charge
    left of the right bond minus that of the second site); modulo n for Z_n."""
    qsite = np.asarray(qsite)
    row_q = (np.asarray(q_left)[:, None] + qsite[None, :]).reshape(-1)
    col_q = (np.asarray(q_right)[None, :] - qsite[:, None]).reshape(-1)
    return _reduce(row_q, modulus), _reduce(col_q, modulus)


def apply_bond_u1(psi, q: list, qsite, b: int, G: np.ndarray, chi_max: int, eps: float,
                  modulus: int = 0) -> float:
    """The Hastings-form update of ``mps.apply_bond`` with the blockwise
    truncation: theta' is cut at bond b+1 by ``truncate_u1`` with the charges
    of ``bond_charges``, and q[b+1] becomes the charges of the kept vectors.
    Returns the discarded weight."""
    d = psi.d
    Bl, Br = psi.B[b], psi.B[b + 1]
    chl, chr_ = Bl.shape[0], Br.shape[2]
    theta_t = np.einsum("asb,btc->astc", Bl, Br)
    theta_tp = np.einsum("uvst,astc->auvc", G.reshape(d, d, d, d), theta_t)
    mat = (psi.lam[b][:, None, None, None] * theta_tp).reshape(chl * d, d * chr_)
    row_q, col_q = bond_charges(q[b], q[b + 2], qsite, modulus)
    _, s, Vh, qk, w, nk, _ = truncate_u1(mat, row_q, col_q, chi_max, eps)
    k = len(s)
    psi.lam[b + 1] = s / nk
    psi.B[b + 1] = Vh.reshape(k, d, chr_)
    psi.B[b] = (theta_tp.reshape(chl * d, d * chr_) @ Vh.conj().T / nk).reshape(chl, d, k)
    q[b + 1] = qk
    psi.disc.append(w)
    return w


def tebd_run_u1(spec, method: str, dt: float, n_steps: int, eps: float, qsite, chi_max=None, modulus: int = 0,
                hs=None):
    """``mps.tebd_run`` on a charge-carrying chain: the product state of
    ``spec`` (basis states), every update by ``apply_bond_u1``; bond terms
    ``hs`` (default: those of ``spec``).  Returns the state and its bond
    charges."""
    from workloads import initial_vectors
    from . import models
    from .mps import GateCache, product_mps, step_layers
    chi_max = spec.chi_max if chi_max is None else chi_max
    vecs = initial_vectors(spec)
    psi = product_mps(vecs)
    q = product_charges(vecs, qsite, modulus)
    gates = GateCache(models.bond_hamiltonians(spec) if hs is None else hs)
    for _ in range(n_steps):
        for bonds, tau in step_layers(method, spec.L, dt):
            for b in bonds:
                apply_bond_u1(psi, q, qsite, b, gates(b, tau), chi_max, eps, modulus)
    return psi, q


def ktebd_run_u1(spec, dt: float, n_steps: int, eps: float, qsite, n_max: int = 20, tol: float = 1e-10,
                 modulus: int = 0):
    """``ktebd.ktebd_run`` on a charge-carrying chain (every cut on the
    charge blocks of its bond).  Returns the state and its bond charges."""
    from workloads import initial_vectors
    from . import models
    from .ktebd import ktebd_step
    from .mps import product_mps
    vecs = initial_vectors(spec)
    psi = product_mps(vecs)
    q = product_charges(vecs, qsite, modulus)
    hs = models.bond_hamiltonians(spec)
    for _ in range(n_steps):
        ktebd_step(psi, hs, dt, spec.chi_max, eps, n_max, tol, charges=(q, qsite, modulus))
    return psi, q


def sector_spectra(lam, q) -> dict:
    """{charge: Schmidt values of that charge, descending} of one bond."""
    out = {}
    for c in sorted(set(np.asarray(q).tolist())):
        out[int(c)] = np.sort(np.asarray(lam)[np.asarray(q) == c])[::-1]
    return out
