"""Pins of the oracle's TEBD update, schedules, truncation and observables.

P1  untruncated Hastings-form TEBD == exact Trotter circuit (state vector)
P2  Trotter order: error ratio at dt vs dt/2 ~ 4 (TEBD2), ~ 16 (TEBD4)
P3  closed forms: free-field Ising precession, g=0 eigenstate, XX free
    fermions at L=64 (Trotterized and exact), Bose-Hubbard t=0 stationary
P4  conservation of norm and particle number
P5/T2 truncation: Eckart-Young, overlap identity and elocal bound
T7  GHZ entropy = log 2
"""
import numpy as np
import pytest

import workloads as W
from oracle import ed, freefermion as ff, models, mps


def _ovl_err(a, b):
    return 1.0 - abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))


@pytest.mark.parametrize("method", ["tebd2", "tebd4", "sweep"])
@pytest.mark.parametrize("spec", [
    W.xxz_chain(8, 256, 1.0, 0.5),
    W.tfim_chain(8, 256, 1.0, 1.0),
    W.bh_chain(5, 2, 256, 1.0, 4.0),
    W.xxz_chain(7, 256, 1.0, 0.5, J_b=np.linspace(0.8, 1.2, 6), Jz_b=np.linspace(0.5, 1.5, 6),
                init="random_product",
                local_states=W.random_complex((7, 2), (99, 1))),
], ids=lambda s: f"{s.model}-L{s.L}")
def test_untruncated_tebd_equals_trotter_circuit(spec, method):
    if spec.init == "random_product":
        spec.local_states = spec.local_states / np.linalg.norm(spec.local_states, axis=1, keepdims=True)
    psi = mps.tebd_run(spec, method, 0.1, 6, 0.0, 10 ** 6)
    v = ed.trotter_circuit(spec, method, 0.1, 6)
    assert _ovl_err(mps.to_vector(psi), v) < 1e-12
    sz = ed.expect_local(v, models.number_op(spec.d) if spec.model == "bh" else 0.5 * models.SZ,
                         spec.L, spec.d)
    got = mps.local_expect(psi, models.number_op(spec.d) if spec.model == "bh" else 0.5 * models.SZ)
    np.testing.assert_allclose(got, sz, atol=1e-12)


@pytest.mark.parametrize("method,lo,hi", [("tebd2", 3.5, 4.5), ("tebd4", 13.0, 19.0), ("sweep", 3.5, 4.5)])
def test_trotter_order(method, lo, hi):
    spec = W.xxz_chain(8, 256, 1.0, 0.5)
    H = models.dense_hamiltonian(spec)
    psi0 = ed.product_vector(W.initial_vectors(spec))
    T = 1.0
    ref = ed.exact_evolve(H, psi0, T)
    errs = []
    for dt in (0.2, 0.1, 0.05, 0.025):
        psi = mps.tebd_run(spec, method, dt, int(round(T / dt)), 0.0, 10 ** 6)
        errs.append(np.linalg.norm(mps.to_vector(psi) - ref))
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    for r in ratios:
        assert lo <= r <= hi, (errs, ratios)


def test_free_field_ising_precession():
    # coupling off, field h = J g = 1: every site precesses, <sz>(t) = cos(2 h t)
    spec = W.tfim_chain(6, 64, 1.0, 1.0)
    spec.params = {"J": 1.0, "g": 1.0}
    hs = models.bond_hamiltonians(spec)
    # rebuild without the zz term: subtract it from each bond Hamiltonian
    zz = -1.0 * np.kron(models.SZ, models.SZ)
    hs = [h - zz for h in hs]
    psi = mps.product_mps(W.initial_vectors(spec))
    dt = 0.07
    for n in range(1, 21):
        for bonds, tau in mps.strang_layers(spec.L, dt):
            for b in bonds:
                mps.apply_bond(psi, b, mps.gate(hs[b], tau), 64, 1e-12)
        np.testing.assert_allclose(mps.local_expect(psi, models.SZ), np.cos(2 * n * dt), atol=1e-13)


def test_ising_g0_eigenstate():
    spec = W.tfim_chain(8, 64, 1.0, 0.0)
    hs = models.bond_hamiltonians(spec)
    E0 = []
    psi = mps.tebd_run(spec, "tebd2", 0.1, 10, 1e-12,
                       observe=lambda p, n: E0.append((mps.energy(p, hs), mps.local_expect(p, models.SZ))))
    for E, sz in E0:
        assert abs(E - (-(spec.L - 1))) < 1e-13
        np.testing.assert_allclose(sz, 1.0, atol=1e-13)


def test_bose_hubbard_t0_stationary():
    spec = W.bh_chain(6, 4, 64, 0.0, 4.0)
    psi = mps.tebd_run(spec, "tebd4", 0.05, 5, 1e-12)
    np.testing.assert_allclose(mps.local_expect(psi, models.number_op(5)), 1.0, atol=1e-13)
    assert max(psi.chis()) == 1


@pytest.mark.parametrize("method", ["tebd2", "tebd4"])
def test_xx_free_fermions_L64(method):
    L, dt, n = 64, 0.05, 20
    spec = W.xxz_chain(L, 256, 1.0, 0.0)
    out = []
    # Each truncation with discarded weight w moves the state by trace
    # distance <= sqrt(w); |Delta<O>| <= 2 |O| D (App. Bounding measurement with
    # the trace distance), |S^z| = 1/2, so the bound is sum_i sqrt(w_i).
    psi = mps.tebd_run(spec, method, dt, n, 1e-14,
                       observe=lambda p, k: out.append((mps.local_expect(p, 0.5 * models.SZ),
                                                        float(np.sum(np.sqrt(p.disc))))))
    sched = [([b], tau) for b, tau in ed.circuit_schedule(method, L, dt)]
    Cs = ff.evolve_trotter(ff.neel_correlation(L), spec.J_b, 1.0, sched, n)
    for k, (sz, bound) in enumerate(out):
        err = np.abs(sz - ff.sz_from_C(Cs[k])).max()
        assert err <= max(1e-12, bound), (k, err, bound)
    # Trotter error of the circuit against the exact single-particle propagator
    Cex = ff.evolve_exact(ff.neel_correlation(L), ff.hopping_matrix(spec.J_b), n * dt)
    d_trot = np.abs(ff.sz_from_C(Cs[-1]) - ff.sz_from_C(Cex)).max()
    assert d_trot < (2e-3 if method == "tebd2" else 1e-5)


def test_norm_and_particle_number_conservation():
    # untruncated: the gates conserve N and the norm exactly
    spec = W.bh_chain(5, 4, 10 ** 6, 1.0, 4.0)
    psi = mps.tebd_run(spec, "tebd2", 0.05, 20, 0.0)
    assert abs(mps.norm2(psi) - 1.0) < 1e-12
    assert abs(mps.local_expect(psi, models.number_op(5)).sum() - spec.L) < 1e-12
    # truncated: Schmidt values are renormalised after every cut, so the norm
    # deviates from 1 by no more than the accumulated discarded weight
    spec = W.bh_chain(8, 4, 12, 1.0, 4.0)
    psi = mps.tebd_run(spec, "tebd2", 0.05, 20, 1e-10)
    assert sum(psi.disc) > 0
    assert abs(mps.norm2(psi) - 1.0) <= sum(psi.disc)


def test_truncation_identities():
    # Eckart-Young and the overlap identity (Eqs. overlap, elocal, App. aux)
    rng = np.random.default_rng(3)
    L, d = 8, 2
    v = rng.normal(size=d ** L) + 1j * rng.normal(size=d ** L)
    v /= np.linalg.norm(v)
    M = v.reshape(d ** 4, -1)
    for chi in (1, 3, 8, 15):
        U, s, Vh, w, nk, sfull = mps.truncate(M, chi, 0.0)
        approx = (U * s) @ Vh
        assert abs(np.linalg.norm(M - approx) ** 2 - w) < 1e-13
        assert abs(w - np.sum(sfull[chi:] ** 2)) < 1e-14
        vt = (approx / nk).reshape(-1)
        ov = np.vdot(vt, v).real
        assert abs(ov - nk) < 1e-13                       # <psi'|psi> = sqrt(sum kept lambda^2)
        assert 1 - ov <= w + 1e-15                         # elocal <= discarded weight


def test_count_rule():
    s = np.array([0.9, 0.4, 1e-3, 1e-7, 1e-9])
    tot = np.sum(s ** 2)
    assert mps.count_rule(s, 10, 0.0) == 5
    assert mps.count_rule(s, 10, 1.5e-14 / tot) == 3       # drops 1e-7 and 1e-9
    assert mps.count_rule(s, 2, 0.0) == 2
    assert mps.count_rule(s, 10, 1.0) == 1                  # k >= 1 always
    assert mps.count_rule(s, 4, -1.0) == 4


def test_ghz_entropy_log2():
    L = 6
    v = np.zeros(2 ** L, dtype=complex)
    v[0] = v[-1] = 1 / np.sqrt(2)
    psi = mps.from_vector(v, L, 2, eps=1e-14)
    np.testing.assert_allclose(mps.entropies(psi), np.log(2), atol=1e-14)


def test_hastings_form_is_right_canonical_after_evolution():
    # exact when nothing is cut: B_b = theta~' V / n_k inherits right-canonicity
    spec = W.xxz_chain(10, 10 ** 6, 1.0, 0.5)
    psi = mps.tebd_run(spec, "tebd2", 0.1, 15, 0.0)
    for B in psi.B:
        chl = B.shape[0]
        M = B.reshape(chl, -1)
        np.testing.assert_allclose(M @ M.conj().T, np.eye(chl), atol=1e-12)


def test_energy_conservation_scaling():
    spec = W.xxz_chain(8, 256, 1.0, 0.5)
    hs = models.bond_hamiltonians(spec)
    drift = {}
    for method in ("tebd2", "tebd4"):
        for dt in (0.1, 0.05):
            E = []
            mps.tebd_run(spec, method, dt, int(round(2.0 / dt)), 0.0, 10 ** 6,
                         observe=lambda p, n: E.append(mps.energy(p, hs)))
            drift[(method, dt)] = max(abs(e - E[0]) for e in E)
    assert 2.5 < drift[("tebd2", 0.1)] / drift[("tebd2", 0.05)] < 5.5
    assert drift[("tebd4", 0.1)] / drift[("tebd4", 0.05)] > 8.0
