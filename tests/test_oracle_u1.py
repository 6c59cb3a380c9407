"""Pins of the U(1)-symmetric truncated SVD oracle (oracle/u1.py) against the
dense SVD and against the charge structure of a number-conserving state.

* A random theta that is block diagonal in charge: the blockwise spectrum is
  the dense spectrum without its structural zeros; k, the discarded weight,
  n_k and the truncated theta agree with ``mps.truncate``; U_k and Vh_k are
  block sparse and orthonormal.
* The exact state of an XXZ chain evolved from a Neel state (conserved total
  S^z): cut into left and right halves, its coefficient matrix vanishes
  outside the blocks where the left charge plus the right charge is the
  total, and the blockwise and dense decompositions agree.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ed, models as om, mps as omps, u1


def _block_theta(rng, row_q, col_q):
    m, n = len(row_q), len(col_q)
    T = rng.normal(size=(m, n)) + 1j * rng.normal(size=(m, n))
    T[np.asarray(row_q)[:, None] != np.asarray(col_q)[None, :]] = 0.0
    # graded values so that the count rule cuts inside the spectrum
    T *= np.exp(-0.15 * np.arange(m))[:, None]
    return T / np.linalg.norm(T)


@pytest.mark.parametrize("seed,m,n,chi,eps", [(1, 40, 30, 12, 1e-6), (2, 64, 64, 64, 0.0), (3, 25, 50, 8, 1e-3)])
def test_blockwise_equals_dense(seed, m, n, chi, eps):
    rng = np.random.default_rng(170300387 + seed)
    row_q = rng.integers(-3, 4, size=m)
    col_q = rng.integers(-2, 5, size=n)
    T = _block_theta(rng, row_q, col_q)
    Uk, sk, Vk, qk, w, nk, s_all = u1.truncate_u1(T, row_q, col_q, chi, eps)
    Ud, sd, Vd, wd, nkd, sd_all = omps.truncate(T, chi, eps)
    nz = sd_all[sd_all > 1e-13]
    assert np.allclose(s_all[:len(nz)], nz, rtol=0, atol=1e-14)
    assert np.all(s_all[len(nz):] <= 1e-13)
    if eps > 0:
        assert len(sk) == len(sd)
    else:  # eps = 0 keeps every value; the dense SVD adds rounding-level values for the structural zeros
        assert len(sk) == min(chi, len(nz)) and np.all(sd[len(sk):] <= 1e-13)
    assert abs(w - wd) <= 1e-14 and abs(nk - nkd) <= 1e-14
    assert np.abs((Uk * sk) @ Vk - (Ud * sd) @ Vd).max() <= 1e-12
    k = len(sk)
    assert np.abs(Uk.conj().T @ Uk - np.eye(k)).max() <= 1e-13
    assert np.abs(Vk @ Vk.conj().T - np.eye(k)).max() <= 1e-13
    assert np.all(Uk[row_q[:, None] != qk[None, :]] == 0)
    assert np.all(Vk[qk[:, None] != col_q[None, :]] == 0)


def test_neel_state_splits_by_charge():
    L, d = 10, 2
    spec = W.xxz_chain(L, 32, 1.0, 0.5)
    psi0 = ed.product_vector(W.initial_vectors(spec))
    psi = ed.exact_evolve(om.dense_hamiltonian(spec), psi0, 1.3)
    cut = 4
    theta = psi.reshape(d ** cut, d ** (L - cut))
    # charge of a configuration: number of up spins (basis index 0 = up)
    def ups(idx, nsites):
        digits = [(idx // d ** (nsites - 1 - i)) % d for i in range(nsites)]
        return sum(1 for x in digits if x == 0)
    qL = np.array([ups(r, cut) for r in range(d ** cut)])
    qR = np.array([ups(c, L - cut) for c in range(d ** (L - cut))])
    Q = L // 2
    off = theta[qL[:, None] + qR[None, :] != Q]
    assert np.abs(off).max() <= 1e-13
    Uk, sk, Vk, qk, w, nk, s_all = u1.truncate_u1(theta, qL, Q - qR, 64, 0.0)
    Ud, sd, Vd, wd, nkd, sd_all = omps.truncate(theta, 64, 0.0)
    assert np.allclose(np.sort(s_all)[::-1][:len(sd)], sd, atol=1e-13)
    assert np.abs((Uk * sk) @ Vk - theta).max() <= 1e-12
