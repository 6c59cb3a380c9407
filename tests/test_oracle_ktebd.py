"""Pins of the oracle's Krylov TEBD (Sornborger-Stewart sweep, local Lanczos).

K1  one Krylov vector: every bond update multiplies the state by the phase
    exp(-i tau <h_b>), so a step maps psi to exp(-i dt <H>) psi, and the
    update's error estimate is the standard deviation of h_b in the state
    (both from exact diagonalisation, with H assembled site by site)
K2  enough Krylov vectors to span the invariant subspace: KTEBD equals the
    exact Trotter circuit of the sweep (exact propagators on the state vector)
K3  the local Krylov error with n vectors falls as tau^n
K4  closed form: free-field Ising precession <sz_i>(t) = cos(2 h t)
K5  after every step B is right-canonical and the norm is 1; with unitary
    (converged) local propagators lam equals the Schmidt values of the state
    vector at every cut
"""
import numpy as np
import pytest

import workloads as W
from oracle import ed, ktebd, models, mps


def _random_state(L, d, key):
    v = W.random_complex(d ** L, key)
    return v / np.linalg.norm(v)


def _mixed_vector(psi):
    """State vector of a chain whose centre sits in the tensors themselves (lam_0 = 1)."""
    v = psi.B[0].reshape(-1, psi.B[0].shape[2])
    for T in psi.B[1:]:
        v = (v @ T.reshape(T.shape[0], -1)).reshape(-1, T.shape[2])
    return v.reshape(-1)


@pytest.mark.parametrize("spec", [
    W.xxz_chain(6, 64, 1.0, 0.5, J_b=np.linspace(0.8, 1.2, 5), Jz_b=np.linspace(0.5, 1.5, 5)),
    W.tfim_chain(6, 64, 1.0, 1.3),
    W.bh_chain(4, 2, 64, 1.0, 4.0),
], ids=lambda s: s.model)
def test_one_krylov_vector_gives_the_energy_phase(spec):
    L, d = spec.L, spec.d
    v = _random_state(L, d, (71, L, d))
    H = models.dense_hamiltonian_from_sites(spec)
    E0 = float(np.vdot(v, H @ v).real)
    dt, n_steps = 0.07, 3
    log = []
    psi = ktebd.ktebd_run(spec, dt, n_steps, -1.0, n_max=1, tol=0.0, chi_max=10 ** 6,
                          psi=mps.from_vector(v, L, d), log=log)
    out = mps.to_vector(psi)
    np.testing.assert_allclose(out, np.exp(-1j * n_steps * dt * E0) * v, atol=1e-12)
    assert all(n == 1 for (_, n, _, _, _) in log)
    # first update (bond 0): err = |psi| beta_0 |u_0| = sqrt(<h^2> - <h>^2)
    h = models.bond_hamiltonians(spec)[0]
    r2 = ed.rdm2(v, 0, 1, L, d)
    std = np.sqrt(np.trace(r2 @ h @ h).real - np.trace(r2 @ h).real ** 2)
    assert abs(log[0][2] - std) < 1e-12


@pytest.mark.parametrize("spec", [
    W.xxz_chain(8, 256, 1.0, 0.5),
    W.tfim_chain(8, 256, 1.0, 1.0),
    W.bh_chain(5, 2, 256, 1.0, 4.0),
    W.xxz_chain(7, 256, 1.0, 0.5, J_b=np.linspace(0.8, 1.2, 6), Jz_b=np.linspace(0.5, 1.5, 6),
                init="random_product", local_states=W.random_complex((7, 2), (99, 1))),
], ids=lambda s: f"{s.model}-L{s.L}")
def test_converged_ktebd_equals_sweep_trotter_circuit(spec):
    dt, n_steps = 0.05, 4
    psi = ktebd.ktebd_run(spec, dt, n_steps, 0.0, n_max=spec.d ** 2 + 1, tol=0.0, chi_max=10 ** 6)
    ref = ed.trotter_circuit(spec, "sweep", dt, n_steps)
    np.testing.assert_allclose(mps.to_vector(psi), ref, atol=1e-12)


@pytest.mark.parametrize("n_max", [1, 2, 3])
def test_local_krylov_error_order(n_max):
    # TFIM bond terms with unequal site weights have four distinct eigenvalues,
    # so no Krylov space below dimension 4 is invariant
    spec = W.tfim_chain(6, 64, 1.0, 1.3)
    L, d = spec.L, spec.d
    v = _random_state(L, d, (72,))
    h = models.bond_hamiltonians(spec)[0]
    errs = []
    for tau in (0.04, 0.02, 0.01):
        psi = mps.from_vector(v, L, d)
        ktebd.bond_krylov_update(psi, 0, h, tau, 10 ** 6, -1.0, n_max, 0.0, True)
        ref = ed.apply_two_site(v, mps.gate(h, tau), 0, L, d)
        errs.append(np.linalg.norm(_mixed_vector(psi) - ref))
    for a, b in zip(errs, errs[1:]):
        assert 2 ** n_max * 0.95 < a / b < 2 ** n_max * 1.05, errs


def test_free_field_ising_precession_ktebd():
    spec = W.tfim_chain(6, 64, 1.0, 1.0)
    zz = -1.0 * np.kron(models.SZ, models.SZ)
    hs = [h - zz for h in models.bond_hamiltonians(spec)]
    psi = mps.product_mps(W.initial_vectors(spec))
    dt = 0.07
    for n in range(1, 16):
        ktebd.ktebd_step(psi, hs, dt, 64, 1e-12, 8, 1e-14)
        np.testing.assert_allclose(mps.local_expect(psi, models.SZ), np.cos(2 * n * dt), atol=1e-13)


@pytest.mark.parametrize("n_max", [2, 5])
def test_chain_form_after_each_step(n_max):
    # n_max = 2 is an approximate propagator; 5 spans the invariant subspace
    spec = W.xxz_chain(7, 10 ** 6, 1.0, 0.5, J_b=np.linspace(0.8, 1.2, 6))
    hs = models.bond_hamiltonians(spec)
    psi = mps.product_mps(W.initial_vectors(spec))
    L, d = spec.L, spec.d
    for _ in range(5):
        ktebd.ktebd_step(psi, hs, 0.1, 10 ** 6, 0.0, n_max, 0.0)
        for B in psi.B:
            M = B.reshape(B.shape[0], -1)
            np.testing.assert_allclose(M @ M.conj().T, np.eye(B.shape[0]), atol=1e-12)
        vec = mps.to_vector(psi)
        assert abs(np.linalg.norm(vec) - 1.0) < 1e-13
        if n_max < 5:
            continue
        for j in range(1, L):
            s = np.linalg.svd(vec.reshape(d ** j, -1), compute_uv=False)
            lam = psi.lam[j]
            np.testing.assert_allclose(lam, s[:len(lam)], atol=1e-12)
            assert np.sum(s[len(lam):] ** 2) < 1e-24


@pytest.mark.parametrize("d", [2, 3])
def test_converged_update_with_complex_bond_term(d):
    # a complex Hermitian bond term tells h from its transpose (h^T = conj h)
    L, D = 5, d * d
    A = W.random_complex((D, D), (73, d))
    h = A + A.conj().T
    v = _random_state(L, d, (74, d))
    for b, right in ((0, True), (2, True), (3, False)):
        psi = mps.from_vector(v, L, d)
        if b > 0:   # move the centre onto site b by exact (untruncated) updates
            for bb in range(b):
                ktebd.bond_krylov_update(psi, bb, np.zeros((D, D)), 0.0, 10 ** 6, -1.0, 1, 0.0, True)
        ktebd.bond_krylov_update(psi, b, h, 0.3, 10 ** 6, -1.0, D + 1, 0.0, right)
        ref = ed.apply_two_site(v, mps.gate(h, 0.3), b, L, d)
        np.testing.assert_allclose(_mixed_vector(psi), ref, atol=1e-12)
