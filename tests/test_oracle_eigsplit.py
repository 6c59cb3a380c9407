"""Pins of the oracle's eigendecomposition split (Sec. "Basic concepts",
Eq. AAD_ULLUD: A A^dag = U lambda^2 U^dag, U^dag A = lambda V^dag) and of its
accuracy against the SVD.

E1  on a well-conditioned matrix it reproduces the SVD: values, discarded
    weight, the projector V_k^dag V_k and the reconstruction
E2  accuracy law: the split's singular values carry a relative error
    <= 20 eps_mach (s_1/s_j)^2 (the Gram squares the condition number), the
    SVD's <= 20 eps_mach (s_1/s_j); at s_j/s_1 = 1e-6 (the square root of
    eps_local = 1e-12) the split keeps only about 4 digits
E3  with eps_local = 1e-12 the truncation keeps the same count, the
    discarded weight agrees to 1e-14; the kept subspace (projector
    V_k^dag V_k) differs at the 1e-5 level along the directions with
    s_j ~ 1e-6 s_1, which moves the truncated matrix U_k S_k V_k^dag by about
    5e-11 (bound 1e-9), far below the truncation's own sqrt(w) ~ 1e-6
"""
import numpy as np
import pytest

import workloads as W
from oracle import mps

EPS = np.finfo(np.float64).eps


def _graded(m, n, s, key):
    Uq, _ = np.linalg.qr(W.random_complex((m, m), key + (1,)))
    Vq, _ = np.linalg.qr(W.random_complex((n, n), key + (2,)))
    r = len(s)
    return (Uq[:, :r] * s) @ Vq[:, :r].conj().T


@pytest.mark.parametrize("m,n", [(24, 24), (16, 40), (40, 16)])
def test_eig_split_equals_svd_when_well_conditioned(m, n):
    r = min(m, n)
    A = _graded(m, n, np.linspace(1.0, 0.05, r), (61, m, n))
    Ue, se, Vhe, we, nke, sfe = mps.truncate_eig(A, 10, 0.0)
    Us, ss, Vhs, ws, nks, sfs = mps.truncate(A, 10, 0.0)
    np.testing.assert_allclose(se, ss, rtol=1e-13)
    assert abs(we - ws) < 1e-13
    np.testing.assert_allclose(Vhe.conj().T @ Vhe, Vhs.conj().T @ Vhs, atol=1e-12)
    np.testing.assert_allclose((Ue * se) @ Vhe, (Us * ss) @ Vhs, atol=1e-12)


def test_eig_split_accuracy_law():
    m = n = 48
    s = np.logspace(0, -7, m)
    A = _graded(m, n, s, (62,))
    _, se, _, _, _, _ = mps.truncate_eig(A, m, -1.0)
    _, ss, _, _, _, _ = mps.truncate(A, m, -1.0)
    rel_e = np.abs(se - s) / s
    rel_s = np.abs(ss - s) / s
    assert np.all(rel_e <= 20 * EPS * (s[0] / s) ** 2), rel_e
    assert np.all(rel_s <= 20 * EPS * (s[0] / s)), rel_s
    near = np.argmin(np.abs(s - 1e-6))
    print(f"s = {s[near]:.2e}: eig split rel. error {rel_e[near]:.1e}, SVD {rel_s[near]:.1e}")
    assert rel_e[near] > 100 * rel_s[near]     # the split is measurably worse there


def test_eig_split_truncation_at_eps_local():
    m = n = 64
    s = np.exp(-0.45 * np.arange(m))            # crosses sqrt(1e-12) s_1 near j = 31
    A = _graded(m, n, s, (63,))
    A /= np.linalg.norm(A)
    Ue, se, Vhe, we, _, _ = mps.truncate_eig(A, m, 1e-12)
    Us, ss, Vhs, ws, _, _ = mps.truncate(A, m, 1e-12)
    assert len(se) == len(ss)
    assert abs(we - ws) < 1e-14
    assert np.abs((Ue * se) @ Vhe - (Us * ss) @ Vhs).max() < 1e-9
    dP = np.abs(Vhe.conj().T @ Vhe - Vhs.conj().T @ Vhs).max()
    assert 1e-9 < dP < 1e-4, dP
