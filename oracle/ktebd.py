"""Krylov TEBD: the Sornborger-Stewart sweep with the Lanczos exponential of
every bond term (oracle, complex128).

Sec. "Sornborger-Stewart decomposition" and App. "Details of the Krylov
method": with the orthogonality centre on one of the two sites of bond b, the
parts of the chain left and right of the bond are orthonormal sets, so the
Krylov basis built with the local Hamiltonian H_C = h_b, the overlaps between
its vectors and their weighted sum all live on the two-site tensor.  The
paper's KTEBD replaces the propagator matrix exp(-i tau h_b) of plain TEBD by
this local Lanczos approximation (the six steps of its cost analysis in the
appendix: contract, build Krylov vectors, orthogonalise, exponentiate the
tridiagonal matrix, sum the weighted vectors, split).

One step of length dt (Eq. sornborger2, the rightmost product acting first):
  left to right, b = 0 .. L-2, tau = dt/2:
      theta = C_b B_{b+1}                       (C_b carries the centre)
      theta <- Lanczos approximation of exp(-i tau h_b) theta,
               h_b acting on the two physical indices only
      SVD with the count rule;  A_b = U_k;  C_{b+1} = S_k V_k^dag / n_k
  right to left, b = L-2 .. 0, tau = dt/2:
      theta = A_b C_{b+1}
      the same Krylov step;  B_{b+1} = V_k^dag;  C_b = U_k S_k / n_k
n_k = (sum_{j<=k} s_j^2)^(1/2) renormalises the kept values, as in the
Hastings-form update of ``mps``, and lam[b+1] = s_k / n_k.

After the right-to-left half every B_{b+1} = V_k^dag is right-canonical and
the centre C_0 on site 0 is lam_0 B_0 with lam_0 = 1, so the state vector is
lam_0 B_0 B_1 ... B_{L-1} as for a Hastings-form ``mps.MPS``.  When every
local propagator is unitary (the Krylov space reached an invariant subspace)
lam[j] is also the Schmidt spectrum of the final state at every cut.  An
approximate Krylov propagator is not unitary on the whole two-site space, so
updates of bonds left of j made later in the right-to-left half move that
spectrum by the size of the Krylov error; the next step never reads those
values (its left-to-right half sets lam[b] before bond b uses it), but
observables weighted by lam carry that error.  A step must start from a
chain whose sites 1..L-1 are right-canonical (a product state is).
"""
from __future__ import annotations

import numpy as np

from . import models
from .krylov import lanczos_expm
from .mps import MPS, product_mps, truncate


def bond_krylov_update(psi: MPS, b: int, h: np.ndarray, tau: float, chi_max: int, eps: float, n_max: int,
                       tol: float, moving_right: bool, log=None, charges=None) -> float:
    """One KTEBD update of bond b with the centre inside the two sites.
    Returns the discarded weight; appends (b, n_used, err, history, conv) to log.
    ``charges`` = (q, qsite, modulus) of a charge-carrying chain: the cut
    runs on the charge blocks (``u1.truncate_u1``) and q[b+1] is updated."""
    Ml, Mr = psi.B[b], psi.B[b + 1]
    chl, d, _ = Ml.shape
    chr_ = Mr.shape[2]
    D = d * d
    theta = np.einsum("asb,btc->astc", Ml, Mr).reshape(chl, D, chr_)

    def apply_h(x):
        # H_C acts on the pair (s, t) of physical indices: (h x)[a,p,c] = sum_q h[p,q] x[a,q,c]
        return np.einsum("pq,aqc->apc", h, x.reshape(chl, D, chr_)).reshape(-1)

    hist = []
    out, n, err, conv = lanczos_expm(apply_h, theta.reshape(-1), tau, n_max, tol, history=hist)
    if charges is None:
        U, s, Vh, w, nk, _ = truncate(out.reshape(chl * d, d * chr_), chi_max, eps)
    else:
        from .u1 import bond_charges, truncate_u1
        q, qsite, modulus = charges
        rq, cq = bond_charges(q[b], q[b + 2], qsite, modulus)
        U, s, Vh, qk, w, nk, _ = truncate_u1(out.reshape(chl * d, d * chr_), rq, cq, chi_max, eps)
        q[b + 1] = qk
    k = len(s)
    lam = s / nk
    psi.lam[b + 1] = lam
    if moving_right:
        psi.B[b] = U.reshape(chl, d, k)
        psi.B[b + 1] = (lam[:, None] * Vh).reshape(k, d, chr_)
    else:
        psi.B[b + 1] = Vh.reshape(k, d, chr_)
        psi.B[b] = (U * lam[None, :]).reshape(chl, d, k)
    psi.disc.append(w)
    if log is not None:
        log.append((b, n, err, hist, conv))
    return w


def ktebd_step(psi: MPS, hs, dt: float, chi_max: int, eps: float, n_max: int, tol: float, log=None,
               charges=None) -> MPS:
    """One Sornborger-Stewart step with local Krylov propagation (module docstring)."""
    L = psi.L
    tau = 0.5 * dt
    for b in range(L - 1):
        bond_krylov_update(psi, b, hs[b], tau, chi_max, eps, n_max, tol, True, log, charges)
    for b in range(L - 2, -1, -1):
        bond_krylov_update(psi, b, hs[b], tau, chi_max, eps, n_max, tol, False, log, charges)
    return psi


def ktebd_run(spec, dt: float, n_steps: int, eps: float, n_max: int = 20, tol: float = 1e-10, chi_max=None,
              observe=None, psi=None, log=None) -> MPS:
    """Evolve the product state of ``spec`` (or ``psi``) for n_steps KTEBD steps.
    ``observe(psi, step)`` is called at step 0 and after every step."""
    chi_max = spec.chi_max if chi_max is None else chi_max
    from workloads import initial_vectors
    psi = product_mps(initial_vectors(spec)) if psi is None else psi
    hs = models.bond_hamiltonians(spec)
    if observe:
        observe(psi, 0)
    for n in range(1, n_steps + 1):
        ktebd_step(psi, hs, dt, chi_max, eps, n_max, tol, log)
        if observe:
            observe(psi, n)
    return psi
