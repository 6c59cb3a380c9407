"""Local operators, bond Hamiltonians, MPOs and dense Hamiltonians (oracle).

Conventions
-----------
* Spin-1/2 basis: index 0 = up (sigma^z=+1), index 1 = down.  S = sigma/2.
* Bosons: Fock basis n = 0..n_max, b|n> = sqrt(n)|n-1>.
* Sites are 0-based, i = 0..L-1; bond b joins sites b and b+1, b = 0..L-2.
* A two-site operator is a (d*d, d*d) matrix with row index (s_out*d + t_out)
  and column index (s_in*d + t_in), s = left site.

Models
------
* Transverse Ising, Eq. Ising: H = -J sum sz_i sz_{i+1} - J g sum sx_i.
* XXZ: H = sum_b J_b [Jxy (Sx Sx + Sy Sy) + Jz_b Sz Sz].
* Bose-Hubbard, Eq. bosehubbard with mu = 0:
  H = -t sum (b_i^dag b_{i+1} + h.c.) + U/2 sum n_i (n_i - 1).

Site terms are split between bonds for the bond Hamiltonians used by TEBD:
an interior site gives half of its term to each of its two bonds; an end site
gives its whole term to its only bond.  (The paper writes the bond sum only,
Eq. sornborger2; this split is the reading taken here.)

MPOs follow the lower-triangular MPO-matrix form of Eq. MPOdef: the bulk
matrix M^[k] has the identity in the top-left and bottom-right corners, the
first column closes terms, the last row opens them.  The first site uses the
last row and the last site the first column.
"""
from __future__ import annotations

import numpy as np

SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SY = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)
SP = np.array([[0, 1], [0, 0]], dtype=np.complex128)  # sigma^+ = |up><down|
SM = SP.T.copy()
I2 = np.eye(2, dtype=np.complex128)


def boson_ops(n_max: int):
    d = n_max + 1
    b = np.zeros((d, d), dtype=np.complex128)
    for n in range(1, d):
        b[n - 1, n] = np.sqrt(n)
    nop = np.diag(np.arange(d)).astype(np.complex128)
    return b, b.conj().T.copy(), nop, np.eye(d, dtype=np.complex128)


def _site_weights(b: int, L: int):
    cl = 1.0 if b == 0 else 0.5
    cr = 1.0 if b == L - 2 else 0.5
    return cl, cr


def bond_hamiltonians(spec) -> list:
    """List of L-1 two-site matrices h_b (complex128) for a ChainSpec."""
    L = spec.L
    hs = []
    if spec.model == "tfim":
        J, g = spec.params["J"], spec.params["g"]
        for b in range(L - 1):
            cl, cr = _site_weights(b, L)
            h = -J * np.kron(SZ, SZ) - J * g * (cl * np.kron(SX, I2) + cr * np.kron(I2, SX))
            hs.append(h)
    elif spec.model == "xxz":
        Jxy = spec.params["Jxy"]
        for b in range(L - 1):
            h = spec.J_b[b] * (Jxy * 0.25 * (np.kron(SX, SX) + np.kron(SY, SY))
                               + spec.Jz_b[b] * 0.25 * np.kron(SZ, SZ))
            hs.append(h)
    elif spec.model == "bh":
        t, U = spec.params["t"], spec.params["U"]
        bb, bd, nop, Id = boson_ops(spec.d - 1)
        onsite = 0.5 * U * nop @ (nop - Id)
        for b in range(L - 1):
            cl, cr = _site_weights(b, L)
            h = -t * (np.kron(bd, bb) + np.kron(bb, bd)) + cl * np.kron(onsite, Id) + cr * np.kron(Id, onsite)
            hs.append(h)
    else:
        raise ValueError(spec.model)
    return hs


def xxz_unit_bond(spec, b: int) -> np.ndarray:
    """The XXZ bond term with J_b factored out: h_b = J_b * h0_b."""
    Jxy = spec.params["Jxy"]
    return (Jxy * 0.25 * (np.kron(SX, SX) + np.kron(SY, SY))
            + spec.Jz_b[b] * 0.25 * np.kron(SZ, SZ))


def embed_two_site(h: np.ndarray, b: int, L: int, d: int) -> np.ndarray:
    """Dense d^L x d^L matrix of a two-site operator on sites b, b+1."""
    left = np.eye(d ** b, dtype=np.complex128)
    right = np.eye(d ** (L - b - 2), dtype=np.complex128)
    return np.kron(np.kron(left, h), right)


def embed_one_site(o: np.ndarray, i: int, L: int, d: int) -> np.ndarray:
    left = np.eye(d ** i, dtype=np.complex128)
    right = np.eye(d ** (L - i - 1), dtype=np.complex128)
    return np.kron(np.kron(left, o), right)


def dense_hamiltonian(spec) -> np.ndarray:
    """H = sum_b h_b embedded in the full Hilbert space (small L only)."""
    hs = bond_hamiltonians(spec)
    D = spec.d ** spec.L
    H = np.zeros((D, D), dtype=np.complex128)
    for b, h in enumerate(hs):
        H += embed_two_site(h, b, spec.L, spec.d)
    return H


def dense_hamiltonian_from_sites(spec) -> np.ndarray:
    """H assembled term by term from local operators, without the bond split.

    Independent of ``bond_hamiltonians``; used to pin it.
    """
    L, d = spec.L, spec.d
    D = d ** L
    H = np.zeros((D, D), dtype=np.complex128)
    if spec.model == "tfim":
        J, g = spec.params["J"], spec.params["g"]
        for i in range(L - 1):
            H -= J * embed_one_site(SZ, i, L, d) @ embed_one_site(SZ, i + 1, L, d)
        for i in range(L):
            H -= J * g * embed_one_site(SX, i, L, d)
    elif spec.model == "xxz":
        Jxy = spec.params["Jxy"]
        for i in range(L - 1):
            for op, c in ((SX, Jxy), (SY, Jxy), (SZ, spec.Jz_b[i])):
                H += spec.J_b[i] * c * 0.25 * embed_one_site(op, i, L, d) @ embed_one_site(op, i + 1, L, d)
    elif spec.model == "bh":
        t, U = spec.params["t"], spec.params["U"]
        bb, bd, nop, Id = boson_ops(d - 1)
        for i in range(L - 1):
            hop = embed_one_site(bd, i, L, d) @ embed_one_site(bb, i + 1, L, d)
            H -= t * (hop + hop.conj().T)
        for i in range(L):
            n = embed_one_site(nop, i, L, d)
            H += 0.5 * U * n @ (n - np.eye(D))
    return H


def mpo(spec) -> list:
    """Bulk MPO matrices W[k] as arrays [w_l][w_r][s_out][s_in], one per site.

    The boundary vectors are handled by the environments: the left boundary
    selects the last row (index w-1) and the right boundary the first column
    (index 0), which reproduces the paper's row/column vectors M^[1], M^[L].
    """
    L, d = spec.L, spec.d
    Ws = []
    if spec.model == "tfim":
        J, g = spec.params["J"], spec.params["g"]
        for k in range(L):
            W = np.zeros((3, 3, 2, 2), dtype=np.complex128)
            W[0, 0] = I2
            W[1, 0] = SZ
            W[2, 0] = -J * g * SX
            W[2, 1] = -J * SZ
            W[2, 2] = I2
            Ws.append(W)
    elif spec.model == "xxz":
        Jxy = spec.params["Jxy"]
        Sp, Sm, Sz = SP, SM, 0.5 * SZ
        for k in range(L):
            W = np.zeros((5, 5, 2, 2), dtype=np.complex128)
            W[0, 0] = I2
            W[1, 0] = Sp
            W[2, 0] = Sm
            W[3, 0] = Sz
            if k < L - 1:
                W[4, 1] = 0.5 * spec.J_b[k] * Jxy * Sm
                W[4, 2] = 0.5 * spec.J_b[k] * Jxy * Sp
                W[4, 3] = spec.J_b[k] * spec.Jz_b[k] * Sz
            W[4, 4] = I2
            Ws.append(W)
    elif spec.model == "bh":
        t, U = spec.params["t"], spec.params["U"]
        bb, bd, nop, Id = boson_ops(d - 1)
        for k in range(L):
            W = np.zeros((4, 4, d, d), dtype=np.complex128)
            W[0, 0] = Id
            W[1, 0] = bd
            W[2, 0] = bb
            W[3, 0] = 0.5 * U * nop @ (nop - Id)
            W[3, 1] = -t * bb
            W[3, 2] = -t * bd
            W[3, 3] = Id
            Ws.append(W)
    else:
        raise ValueError(spec.model)
    return Ws


def mpo_to_dense(Ws: list) -> np.ndarray:
    """Contract the MPO (with the boundary selections) into a dense matrix.

    Multiplies the MPO matrices in the auxiliary indices and takes tensor
    products in the physical ones, as in the paper's three-site example.
    """
    w = Ws[0].shape[0]
    # running operator-valued row vector: list over aux index of dense ops
    cur = [None] * w
    row = Ws[0][w - 1]              # last row of the first site: shape [w_r][d][d]
    for a in range(w):
        cur[a] = row[a].copy()
    for W in Ws[1:]:
        wr = W.shape[1]
        nxt = [None] * wr
        for b in range(wr):
            acc = None
            for a in range(len(cur)):
                if not np.any(W[a, b]):
                    continue
                term = np.kron(cur[a], W[a, b])
                acc = term if acc is None else acc + term
            if acc is None:
                D = cur[0].shape[0] * W.shape[2]
                acc = np.zeros((D, D), dtype=np.complex128)
            nxt[b] = acc
        cur = nxt
    return cur[0]


def local_sz(d: int) -> np.ndarray:
    """S^z = sigma^z / 2 for spins."""
    assert d == 2
    return 0.5 * SZ


def number_op(d: int) -> np.ndarray:
    return np.diag(np.arange(d)).astype(np.complex128)
