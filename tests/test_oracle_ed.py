"""Pins of the oracle's state-vector references: reduced density matrices,
the trace distance and half-chain entropy, the four error measures of Sec.
"Computational error and convergence", and the circuit schedule.

Each value below is fixed by elementary quantum mechanics, not by the code:
* two orthogonal pure states are at trace distance 1; |0> and |+> at
  sqrt(1 - |<0|+>|^2) = 1/sqrt(2) (pure states: D = sqrt(1 - |<a|b>|^2));
* the two-site reduced density matrix of a product state is the Kronecker
  product of its one-site matrices, in the order of the sites asked for;
* a Bell pair cut in the middle has entropy ln 2 (natural log, Eq. eentr), a
  product state 0, and a cut of Schmidt weights (p, 1 - p) has the binary
  entropy -p ln p - (1 - p) ln(1 - p).
"""
import numpy as np
import pytest

import workloads as W
from oracle import ed, models


def _basis(L, d, digits):
    v = np.zeros(d ** L, dtype=np.complex128)
    v[int("".join(str(x) for x in digits), d)] = 1.0
    return v


def _prod(*vs):
    out = np.ones(1, dtype=np.complex128)
    for v in vs:
        out = np.kron(out, v)
    return out


def test_trace_distance_closed_forms():
    z0 = np.array([[1, 0], [0, 0]], dtype=np.complex128)
    z1 = np.array([[0, 0], [0, 1]], dtype=np.complex128)
    plus = 0.5 * np.ones((2, 2), dtype=np.complex128)
    assert ed.trace_distance(z0, z1) == pytest.approx(1.0, abs=1e-15)
    assert ed.trace_distance(z0, plus) == pytest.approx(1.0 / np.sqrt(2.0), abs=1e-15)
    assert ed.trace_distance(z0, z0) == pytest.approx(0.0, abs=1e-15)
    # maximally mixed against a pure state: 1/2 |diag(1/2, -1/2)| = 1/2
    assert ed.trace_distance(0.5 * np.eye(2), z0) == pytest.approx(0.5, abs=1e-15)
    # pure states in general: D = sqrt(1 - |<a|b>|^2)
    rng = np.random.default_rng(1)
    for _ in range(5):
        a = rng.normal(size=4) + 1j * rng.normal(size=4)
        b = rng.normal(size=4) + 1j * rng.normal(size=4)
        a /= np.linalg.norm(a)
        b /= np.linalg.norm(b)
        want = np.sqrt(1.0 - abs(np.vdot(a, b)) ** 2)
        got = ed.trace_distance(np.outer(a, a.conj()), np.outer(b, b.conj()))
        assert got == pytest.approx(want, abs=1e-13)


def test_rdm1_rdm2_of_product_states():
    rng = np.random.default_rng(2)
    L, d = 4, 3
    vs = [rng.normal(size=d) + 1j * rng.normal(size=d) for _ in range(L)]
    vs = [v / np.linalg.norm(v) for v in vs]
    psi = _prod(*vs)
    rho = [np.outer(v, v.conj()) for v in vs]
    for i in range(L):
        np.testing.assert_allclose(ed.rdm1(psi, i, L, d), rho[i], atol=1e-14)
        for j in range(i + 1, L):
            np.testing.assert_allclose(ed.rdm2(psi, i, j, L, d), np.kron(rho[i], rho[j]), atol=1e-14)
    # the order of the two sites is (i, j): a distinguishable pair tells it
    psi = _basis(3, 2, [0, 0, 1])
    r = ed.rdm2(psi, 0, 2, 3, 2)
    assert r[1, 1] == pytest.approx(1.0)      # |0>_0 |1>_2  -> index 0*2 + 1
    assert abs(np.trace(r)) == pytest.approx(1.0)


def test_rdm2_of_a_bell_pair_between_distant_sites():
    # (|0 x 0> + |1 x 1>)/sqrt 2 on sites 0 and 2 with site 1 in |1>
    L, d = 3, 2
    psi = (_basis(L, d, [0, 1, 0]) + _basis(L, d, [1, 1, 1])) / np.sqrt(2.0)
    r = ed.rdm2(psi, 0, 2, L, d)
    bell = np.array([1, 0, 0, 1], dtype=np.complex128) / np.sqrt(2.0)
    np.testing.assert_allclose(r, np.outer(bell, bell.conj()), atol=1e-15)
    # its single sites are maximally mixed
    np.testing.assert_allclose(ed.rdm1(psi, 0, L, d), 0.5 * np.eye(2), atol=1e-15)
    np.testing.assert_allclose(ed.rdm1(psi, 1, L, d), np.diag([0.0, 1.0]), atol=1e-15)


def test_half_chain_entropy_closed_forms():
    L, d = 4, 2
    assert ed.half_chain_entropy(_basis(L, d, [0, 1, 1, 0]), L, d) == pytest.approx(0.0, abs=1e-15)
    # Bell pair across the middle cut (sites 1 and 2), the other sites product
    bell = (_basis(L, d, [0, 0, 0, 0]) + _basis(L, d, [0, 1, 1, 0])) / np.sqrt(2.0)
    assert ed.half_chain_entropy(bell, L, d) == pytest.approx(np.log(2.0), abs=1e-14)
    # Bell pair inside the left half: no entanglement across the cut
    inside = (_basis(L, d, [0, 0, 0, 0]) + _basis(L, d, [1, 1, 0, 0])) / np.sqrt(2.0)
    assert ed.half_chain_entropy(inside, L, d) == pytest.approx(0.0, abs=1e-14)
    # unequal Schmidt weights p, 1 - p: the binary entropy
    p = 0.2
    psi = np.sqrt(p) * _basis(L, d, [0, 0, 0, 0]) + np.sqrt(1 - p) * _basis(L, d, [0, 1, 1, 0])
    want = -p * np.log(p) - (1 - p) * np.log(1 - p)
    assert ed.half_chain_entropy(psi, L, d) == pytest.approx(want, abs=1e-14)


def test_error_measures_closed_forms():
    L, d = 4, 2
    H = sum(models.embed_one_site(models.SZ, i, L, d) for i in range(L))   # sum of sigma^z
    ref = _basis(L, d, [0, 0, 0, 0])              # all sigma^z = +1: energy 4
    flipped = _basis(L, d, [0, 0, 1, 0])          # one site flipped: energy 2
    m = ed.error_measures(flipped, ref, H, L, d)
    assert m["eps_local"] == pytest.approx(1.0, abs=1e-14)    # orthogonal states of site 2
    assert m["eps_corr"] == pytest.approx(1.0, abs=1e-14)     # any pair containing site 2
    assert m["eps_E"] == pytest.approx(2.0, abs=1e-14)
    assert m["eps_S"] == pytest.approx(0.0, abs=1e-14)
    # a Bell pair across the middle against the product state it grew from
    bell = (_basis(L, d, [0, 0, 0, 0]) + _basis(L, d, [0, 1, 1, 0])) / np.sqrt(2.0)
    m = ed.error_measures(bell, ref, H, L, d)
    assert m["eps_S"] == pytest.approx(np.log(2.0), abs=1e-14)
    assert m["eps_local"] == pytest.approx(0.5, abs=1e-14)    # rho = 1/2 against |0><0|
    # two-site: the Bell pair (1,2) against |00><00|: eigenvalues of
    # |B><B| - |00><00| are +-1/sqrt(2), so D = 1/sqrt(2)
    assert m["eps_corr"] == pytest.approx(1.0 / np.sqrt(2.0), abs=1e-14)
    # <H>_bell = 1/2 * 4 + 1/2 * 0 = 2 against <H>_ref = 4
    assert m["eps_E"] == pytest.approx(2.0, abs=1e-14)


@pytest.mark.parametrize("method", ["tebd2", "tebd4", "sweep"])
def test_circuit_schedule_definitions(method):
    L, dt = 7, 0.1
    sched = ed.circuit_schedule(method, L, dt)
    # each bond's exponents add up to dt within one step (a consistent splitting)
    tot = np.zeros(L - 1)
    for b, tau in sched:
        tot[b] += tau
    np.testing.assert_allclose(tot, dt, atol=1e-15)
    if method == "tebd2":
        assert [b for b, _ in sched] == [0, 2, 4, 1, 3, 5, 0, 2, 4]
    if method == "tebd4":
        p = ed._suzuki_p()
        assert 4 * p ** 3 + (1 - 4 * p) ** 3 == pytest.approx(0.0, abs=1e-15)
        assert 4 * p + (1 - 4 * p) == pytest.approx(1.0)
        assert len(sched) == 45
    if method == "sweep":
        assert [b for b, _ in sched] == [0, 1, 2, 3, 4, 5, 5, 4, 3, 2, 1, 0]


def test_circuit_schedule_matches_tebd_order_on_a_random_chain():
    # the circuit (its own schedule and exponentials) reproduces the exact
    # evolution to the Trotter order: a schedule with a misplaced bond would
    # break the ratio of the errors at dt and dt/2
    spec = W.xxz_chain(6, 64, 1.0, 0.5)
    H = models.dense_hamiltonian(spec)
    psi0 = ed.product_vector(W.initial_vectors(spec))
    errs = []
    for dt in (0.1, 0.05):
        v = ed.trotter_circuit(spec, "tebd4", dt, int(round(0.5 / dt)))
        errs.append(np.linalg.norm(v - ed.exact_evolve(H, psi0, 0.5)))
    assert 13.0 <= errs[0] / errs[1] <= 19.0, errs
