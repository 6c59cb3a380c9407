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
