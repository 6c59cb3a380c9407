"""Environments, the structured effective Hamiltonian, and two-site TDVP
(oracle, complex128).

Effective Hamiltonian (Sec. "Fundamentals of the library", Fig. LanczosMPS):
the sites left and right of the two active sites are contracted with their
MPO matrices into one left tensor and one right tensor; with the two MPO
matrices of the active sites they form H_eff, which is applied to a vector
step by step (O(chi^3) instead of building the chi^2 d^2 square matrix).

Index conventions (shared with the C-ABI documentation, not with its code):
  Lenv[a_out][beta][a_in], W[beta_l][beta_r][s_out][s_in],
  Renv[c_out][beta][c_in], x[a][s][t][c].
  y[a',s',t',c'] = sum L[a',b,a] W1[b,g,s',s] W2[g,e,t',t] R[c',e,c] x[a,s,t,c]

Two-site TDVP (Sec. TDVP; the algorithm of the cited Haegeman et al. 2016,
whose steps the paper does not print): symmetric second order, each
half-sweep with tau = dt/2.  Left-to-right over bonds b = 0..L-2: evolve the
two-site tensor forward with H2_eff(b), split by truncated SVD (A_b = U,
C = S V^dag), update the left environment, and, unless b is the last bond,
evolve C backward with the one-site H1_eff(b+1).  The right-to-left
half-sweep mirrors it.  The exponentials are the Lanczos approximation of
``krylov.lanczos_expm`` (the local Krylov step of App. Details of the Krylov
method).
"""
from __future__ import annotations

import numpy as np

from . import models
from .krylov import lanczos_expm
from .mps import truncate


def left_boundary(w: int) -> np.ndarray:
    Lb = np.zeros((1, w, 1), dtype=np.complex128)
    Lb[0, w - 1, 0] = 1.0
    return Lb


def right_boundary(w: int) -> np.ndarray:
    Rb = np.zeros((1, w, 1), dtype=np.complex128)
    Rb[0, 0, 0] = 1.0
    return Rb


def update_left(Lenv, A, W):
    """L'[a',b',c'] = sum conj(A[a,s',a']) L[a,b,c] W[b,b',s',s] A[c,s,c']."""
    return np.einsum("apx,abc,bypq,cqz->xyz", A.conj(), Lenv, W, A)


def update_right(Renv, B, W):
    """R'[a',b,c'] = sum conj(B[a',t',a]) W[b,b',t',t] R[a,b',c] B[c',t,c]."""
    return np.einsum("xpa,bypq,ayc,zqc->xbz", B.conj(), W, Renv, B)


# Each stage below contracts two tensors over the indices its subscripts name;
# optimize=True only lets NumPy evaluate that pairwise sum through BLAS
# (tensordot) instead of its element loop, the same contraction.
def heff2_apply(Lenv, W1, W2, Renv, x):
    X1 = np.einsum("xba,astc->xbstc", Lenv, x, optimize=True)
    X2 = np.einsum("bgus,xbstc->xgutc", W1, X1, optimize=True)
    X3 = np.einsum("gevt,xgutc->xuevc", W2, X2, optimize=True)
    return np.einsum("xuevc,yec->xuvy", X3, Renv, optimize=True)


def heff1_apply(Lenv, W, Renv, x):
    X1 = np.einsum("xba,asc->xbsc", Lenv, x, optimize=True)
    X2 = np.einsum("bgus,xbsc->xguc", W, X1, optimize=True)
    return np.einsum("xguc,ygc->xuy", X2, Renv, optimize=True)


def heff2_dense(Lenv, W1, W2, Renv) -> np.ndarray:
    """Dense chi^2 d^2 square H_eff (brute force, tiny sizes only)."""
    H = np.einsum("xba,bgus,gevt,yec->xuvyastc", Lenv, W1, W2, Renv)
    n = Lenv.shape[0] * W1.shape[2] * W2.shape[2] * Renv.shape[0]
    return H.reshape(n, n)


class OCMPS:
    """MPS in mixed-canonical form: tensors M[i] = [chi_i][d][chi_{i+1}]."""

    def __init__(self, M):
        self.M = M

    @property
    def L(self):
        return len(self.M)

    def to_vector(self):
        v = self.M[0].reshape(self.M[0].shape[0] * self.M[0].shape[1], -1)
        for T in self.M[1:]:
            v = (v @ T.reshape(T.shape[0], -1)).reshape(-1, T.shape[2])
        return v.reshape(-1)


def product_oc(vectors) -> OCMPS:
    return OCMPS([(v / np.linalg.norm(v)).reshape(1, -1, 1).astype(np.complex128) for v in vectors])


def full_dimension_oc(vec: np.ndarray, L: int, d: int) -> OCMPS:
    """Exact MPS of ``vec`` with every virtual bond i at its full dimension
    min(d^i, d^(L-i)), zero Schmidt values kept (full SVDs supply the
    orthonormal completion).  Sites 1..L-1 right-canonical, centre on site 0."""
    rest = vec.reshape(-1, 1)
    Ms = [None] * L
    for i in range(L - 1, 0, -1):
        chr_ = rest.shape[1]
        mat = rest.reshape(d ** i, d * chr_)
        U, s, Vh = np.linalg.svd(mat, full_matrices=True)
        k = min(d ** i, d * chr_)
        Ms[i] = Vh[:k].reshape(k, d, chr_)
        rest = U[:, :k] * s[None, :k]
    Ms[0] = rest.reshape(1, d, -1)
    return OCMPS(Ms)


def _right_envs(psi: OCMPS, Ws):
    L = psi.L
    w = Ws[0].shape[0]
    R = [None] * (L + 1)
    R[L] = right_boundary(w)
    for i in range(L - 1, 0, -1):
        R[i] = update_right(R[i + 1], psi.M[i], Ws[i])
    return R


def _split(th2, b, chi_max, eps, charges):
    """Truncated SVD of the two-site matrix of bond b: dense, or on the charge
    blocks of a charge-carrying chain (charges = (q, qsite, modulus); q[b+1]
    becomes the charges of the kept vectors)."""
    if charges is None:
        return truncate(th2, chi_max, eps)
    from .u1 import bond_charges, truncate_u1
    q, qsite, modulus = charges
    rq, cq = bond_charges(q[b], q[b + 2], qsite, modulus)
    U, s, Vh, qk, w, nk, s_all = truncate_u1(th2, rq, cq, chi_max, eps)
    q[b + 1] = qk
    return U, s, Vh, w, nk, s_all


def tdvp2_step(psi: OCMPS, Ws, dt: float, chi_max: int, eps: float, n_max=20, tol=1e-10,
               log=None, charges=None):
    """One symmetric 2TDVP step.  psi must have its orthogonality centre on
    site 0 with all other sites right-canonical; on return the same holds.
    ``charges`` = (q, qsite, modulus): every split on the charge blocks of
    its bond (App. "Convenient features"), q updated in place."""
    L = psi.L
    w = Ws[0].shape[0]
    tau = 0.5 * dt
    Lenv = [None] * (L + 1)
    Lenv[0] = left_boundary(w)
    R = _right_envs(psi, Ws)
    R[L] = right_boundary(w)
    # left to right
    for b in range(L - 1):
        A, B = psi.M[b], psi.M[b + 1]
        th = np.einsum("asb,btc->astc", A, B)
        sh = th.shape
        f = lambda v: heff2_apply(Lenv[b], Ws[b], Ws[b + 1], R[b + 2], v.reshape(sh)).reshape(-1)
        th, n, err, conv = lanczos_expm(f, th.reshape(-1), tau, n_max, tol)
        if log is not None:
            log.append(("2f", b, n, err, conv))
        U, s, Vh, wdisc, nk, _ = _split(th.reshape(sh[0] * sh[1], sh[2] * sh[3]), b, chi_max, eps, charges)
        k = len(s)
        psi.M[b] = U.reshape(sh[0], sh[1], k)
        C = (s[:, None] * Vh).reshape(k, sh[2], sh[3])
        Lenv[b + 1] = update_left(Lenv[b], psi.M[b], Ws[b])
        if b < L - 2:
            g = lambda v: heff1_apply(Lenv[b + 1], Ws[b + 1], R[b + 2], v.reshape(C.shape)).reshape(-1)
            C, n, err, conv = lanczos_expm(g, C.reshape(-1), -tau, n_max, tol)
            C = C.reshape(k, sh[2], sh[3])
            if log is not None:
                log.append(("1b", b + 1, n, err, conv))
        psi.M[b + 1] = C
    # right to left
    for b in range(L - 2, -1, -1):
        A, B = psi.M[b], psi.M[b + 1]
        th = np.einsum("asb,btc->astc", A, B)
        sh = th.shape
        f = lambda v: heff2_apply(Lenv[b], Ws[b], Ws[b + 1], R[b + 2], v.reshape(sh)).reshape(-1)
        th, n, err, conv = lanczos_expm(f, th.reshape(-1), tau, n_max, tol)
        if log is not None:
            log.append(("2f", b, n, err, conv))
        U, s, Vh, wdisc, nk, _ = _split(th.reshape(sh[0] * sh[1], sh[2] * sh[3]), b, chi_max, eps, charges)
        k = len(s)
        psi.M[b + 1] = Vh.reshape(k, sh[2], sh[3])
        C = (U * s[None, :]).reshape(sh[0], sh[1], k)
        R[b + 1] = update_right(R[b + 2], psi.M[b + 1], Ws[b + 1])
        if b > 0:
            g = lambda v: heff1_apply(Lenv[b], Ws[b], R[b + 1], v.reshape(C.shape)).reshape(-1)
            C, n, err, conv = lanczos_expm(g, C.reshape(-1), -tau, n_max, tol)
            C = C.reshape(sh[0], sh[1], k)
            if log is not None:
                log.append(("1b", b, n, err, conv))
        psi.M[b] = C
    return psi


def right_canonicalize(psi: OCMPS) -> OCMPS:
    """Bring all sites but site 0 into right-canonical form (exact, no truncation)."""
    for i in range(psi.L - 1, 0, -1):
        T = psi.M[i]
        chl, d, chr_ = T.shape
        U, s, Vh = np.linalg.svd(T.reshape(chl, d * chr_), full_matrices=False)
        psi.M[i] = Vh.reshape(-1, d, chr_)
        psi.M[i - 1] = np.einsum("asb,bc->asc", psi.M[i - 1], U * s[None, :])
    return psi


def oc_site_expect(psi: OCMPS, op: np.ndarray) -> np.ndarray:
    """<O_i> for a product-free general OC-MPS by full left/right contraction."""
    L = psi.L
    out = []
    for i in range(L):
        E = np.ones((1, 1), dtype=np.complex128)
        for j, T in enumerate(psi.M):
            if j == i:
                E = np.einsum("ab,asc,st,btd->cd", E, T.conj(), op, T)
            else:
                E = np.einsum("ab,asc,bsd->cd", E, T.conj(), T)
        out.append(float(np.real(E[0, 0])))
    return np.array(out)
