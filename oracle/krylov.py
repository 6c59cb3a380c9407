"""Lanczos approximation of exp(-i tau A) v (oracle, complex128).

Sec. "Krylov time evolution": build an orthonormal Krylov basis
V = [v_1 .. v_n] from v_1 = psi/|psi|; for Hermitian A the projection
T = V^dag A V is real symmetric tridiagonal, and
    exp(-i tau A) psi ~= |psi| V exp(-i tau T) e_1         (Eq. krylov:approx).
App. "Details of the Krylov method" shows that, with the orthogonality centre
inside the two sites, every Krylov vector and the sum over them live on those
two sites only, so the whole iteration acts on the two-site tensor.

Steps per iteration j (all in complex128):
  r = A v_j;  alpha_j = Re<v_j|r>;  r -= alpha_j v_j + beta_{j-1} v_{j-1};
  full re-orthogonalisation of r against all v, done twice;  beta_j = |r|;
  T_j = Q diag(theta) Q^T;  u = Q (exp(-i tau theta) * Q^T e_1);
  err_j = |psi| beta_j |u_j|   (a-posteriori estimate of the residual);
  stop when err_j <= tol or beta_j <= 1e-14 |psi| (invariant subspace).
The result is |psi| V u.  tau may be complex (imaginary time for tests).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg


def tridiag_expm_e1(alpha, beta, tau):
    """u = exp(-i tau T) e_1 for the real symmetric tridiagonal T."""
    n = len(alpha)
    T = np.diag(alpha) + np.diag(beta[: n - 1], 1) + np.diag(beta[: n - 1], -1)
    th, Q = np.linalg.eigh(T)
    return Q @ (np.exp(-1j * tau * th) * Q[0, :])


def lanczos_expm(apply_A, psi: np.ndarray, tau: complex, n_max=20, tol=1e-10, history=None):
    """Returns (result, n_used, err_est, converged).  If ``history`` is a list,
    the estimate err_j of every iteration is appended to it."""
    nrm = np.linalg.norm(psi)
    if nrm == 0:
        return psi.copy(), 0, 0.0, True
    V = [psi / nrm]
    alpha, beta = [], []
    u = np.array([1.0 + 0j])
    err = np.inf
    conv = False
    for j in range(n_max):
        r = apply_A(V[j])
        a = float(np.real(np.vdot(V[j], r)))
        alpha.append(a)
        r = r - a * V[j]
        if j > 0:
            r = r - beta[j - 1] * V[j - 1]
        for _ in range(2):
            for v in V:
                r = r - np.vdot(v, r) * v
        bj = float(np.linalg.norm(r))
        beta.append(bj)
        u = tridiag_expm_e1(np.array(alpha), np.array(beta), tau)
        err = nrm * bj * abs(u[-1])
        if history is not None:
            history.append(float(err))
        if err <= tol or bj <= 1e-14 * nrm:
            conv = True
            break
        V.append(r / bj)
    n = len(alpha)
    out = nrm * sum(u[i] * V[i] for i in range(n))
    return out, n, float(err), conv


def dense_expm_apply(A: np.ndarray, psi: np.ndarray, tau: complex) -> np.ndarray:
    return scipy.linalg.expm(-1j * tau * A) @ psi
