"""Pins of the oracle's Lanczos exponential, structured H_eff and 2TDVP.

P6a Lanczos vs dense expm;  P6b exact once the Krylov space is invariant;
P6c full-bond-dimension 2TDVP == exp(-i dt H) (local projectors are
identities);  P7 structured H_eff == brute-force dense H_eff, and with
environments of the whole chain <theta|H_eff|theta> = <psi|H|psi>;
T6 the local-Krylov lemma: h11 = <C|H_C|C> on the two sites.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ed, krylov, models, tdvp


def _herm(n, seed):
    r = np.random.default_rng(seed)
    A = r.normal(size=(n, n)) + 1j * r.normal(size=(n, n))
    return A + A.conj().T


@pytest.mark.parametrize("tau", [0.05, 0.2, -0.1, 0.1 - 0.05j])
def test_lanczos_vs_dense(tau):
    A = _herm(80, 1)
    v = W.random_complex(80, (5,))
    out, n, err, conv = krylov.lanczos_expm(lambda x: A @ x, v, tau, 30, 1e-11)
    ref = krylov.dense_expm_apply(A, v, tau)
    assert conv
    assert np.linalg.norm(out - ref) <= 10 * max(err, 1e-13)


def test_lanczos_exact_in_invariant_subspace():
    A = _herm(12, 2)
    v = W.random_complex(12, (6,))
    out, n, err, conv = krylov.lanczos_expm(lambda x: A @ x, v, 0.7, 12, 0.0)
    assert np.linalg.norm(out - krylov.dense_expm_apply(A, v, 0.7)) < 1e-12


def test_lanczos_nonconvergence_flag():
    A = _herm(40, 3)
    v = W.random_complex(40, (7,))
    out, n, err, conv = krylov.lanczos_expm(lambda x: A @ x, v, 1.0, 2, 1e-14)
    assert not conv and n == 2 and err > 1e-14


def test_heff_structured_equals_dense():
    spec = W.bh_chain(4, 2, 64, 1.0, 4.0)
    Ws = models.mpo(spec)
    chi, w, d = 3, 4, 3
    Lenv = W.random_complex((chi, w, chi), (10,))
    Renv = W.random_complex((chi, w, chi), (11,))
    x = W.random_complex((chi, d, d, chi), (12,))
    y1 = tdvp.heff2_apply(Lenv, Ws[1], Ws[2], Renv, x).reshape(-1)
    y2 = tdvp.heff2_dense(Lenv, Ws[1], Ws[2], Renv) @ x.reshape(-1)
    np.testing.assert_allclose(y1, y2, atol=1e-13)


@pytest.mark.parametrize("spec", [W.xxz_chain(6, 64, 1.0, 0.5), W.bh_chain(4, 2, 64, 1.0, 4.0),
                                  W.tfim_chain(6, 64, 1.0, 1.2)], ids=lambda s: s.model)
def test_heff_with_full_environments_gives_energy(spec):
    L, d = spec.L, spec.d
    H = models.dense_hamiltonian(spec)
    v = W.random_complex(d ** L, (20, L))
    v /= np.linalg.norm(v)
    psi = tdvp.full_dimension_oc(v, L, d)
    Ws = models.mpo(spec)
    R = [None] * (L + 1)
    R[L] = tdvp.right_boundary(Ws[0].shape[0])
    for i in range(L - 1, 1, -1):
        R[i] = tdvp.update_right(R[i + 1], psi.M[i], Ws[i])
    Lb = tdvp.left_boundary(Ws[0].shape[0])
    th = np.einsum("asb,btc->astc", psi.M[0], psi.M[1])
    e_local = np.vdot(th.reshape(-1), tdvp.heff2_apply(Lb, Ws[0], Ws[1], R[2], th).reshape(-1))
    assert abs(e_local - np.vdot(v, H @ v)) < 1e-12
    # T6: the first Lanczos coefficient h11 is this same local expectation
    out, n, err, conv = krylov.lanczos_expm(
        lambda x: tdvp.heff2_apply(Lb, Ws[0], Ws[1], R[2], x.reshape(th.shape)).reshape(-1),
        th.reshape(-1), 0.01, 1, 0.0)
    assert n == 1


@pytest.mark.parametrize("spec", [W.xxz_chain(6, 64, 1.0, 0.5), W.bh_chain(4, 2, 64, 1.0, 4.0),
                                  W.tfim_chain(6, 64, 1.0, 1.2)], ids=lambda s: s.model)
def test_full_dimension_tdvp2_is_exact(spec):
    L, d = spec.L, spec.d
    H = models.dense_hamiltonian(spec)
    v0 = ed.product_vector(W.initial_vectors(spec))
    psi = tdvp.full_dimension_oc(v0, L, d)
    Ws = models.mpo(spec)
    dt, n = 0.05, 8
    for _ in range(n):
        tdvp.tdvp2_step(psi, Ws, dt, 10 ** 6, -1.0, 30, 1e-13)
    ref = ed.exact_evolve(H, v0, n * dt)
    assert np.linalg.norm(psi.to_vector() - ref) < 1e-10


def test_truncated_tdvp2_conserves_particles_and_energy():
    spec = W.bh_chain(6, 4, 64, 1.0, 4.0)
    H = models.dense_hamiltonian(spec)
    psi = tdvp.product_oc(W.initial_vectors(spec))
    Ws = models.mpo(spec)
    E0 = np.vdot(psi.to_vector(), H @ psi.to_vector()).real
    for _ in range(5):
        tdvp.tdvp2_step(psi, Ws, 0.02, 64, 1e-12, 20, 1e-10)
    v = psi.to_vector()
    assert abs(np.linalg.norm(v) - 1) < 1e-9
    assert abs(np.vdot(v, H @ v).real - E0) < 1e-8
    n_tot = tdvp.oc_site_expect(psi, models.number_op(5)).sum()
    assert abs(n_tot - spec.L) < 1e-8
    ref = ed.exact_evolve(H, ed.product_vector(W.initial_vectors(spec)), 0.1)
    assert 1 - abs(np.vdot(v, ref)) < 1e-8
