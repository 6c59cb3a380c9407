"""Pins of the oracle's time-dependent propagation (commutator-free Magnus
expansions on top of the Trotter steps).

D1  commuting terms (transverse field only, g(t) ramped): every spin precesses
    by the quadrature of g over each step, <sz_i>(T) = cos(2 sum_n dt gbar_n)
    with gbar_n = g(t_n + dt/2) (midpoint) or the two-node Gauss-Legendre mean
    (fourth-order scheme)
D2  global order against the exact time-ordered evolution (adaptive ODE
    solver on the dense Hamiltonian): midpoint + TEBD2 ~ dt^2, the
    fourth-order scheme + TEBD4 ~ dt^4 (error ratios 4 and 16)
D3  against the paper's exact-diagonalisation midpoint reference for its
    Ising quench (g from 5 to 4.5 over T = 0.5): the TEBD4 midpoint run differs
    only by the Trotter error, ratio 16 when dt halves
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import workloads as W
from oracle import ed, models, mps, timedep


def ising_terms(L, J=1.0):
    """Bond split of the coupling (weight 1) and of the unit transverse field."""
    hz = models.bond_hamiltonians(W.tfim_chain(L, 64, J, 0.0))
    hf = [a - b for a, b in zip(models.bond_hamiltonians(W.tfim_chain(L, 64, J, 1.0)), hz)]
    return [hz, hf]


def ising_dense(L, J=1.0):
    Hz = models.dense_hamiltonian_from_sites(W.tfim_chain(L, 64, J, 0.0))
    Hf = models.dense_hamiltonian_from_sites(W.tfim_chain(L, 64, J, 1.0)) - Hz
    return [Hz, Hf]


@pytest.mark.parametrize("scheme", [2, 4])
@pytest.mark.parametrize("method", ["tebd2", "sweep"])
def test_field_ramp_precession_closed_form(scheme, method):
    L = 6
    hz, hf = ising_terms(L)
    terms = [[0.0 * h for h in hz], hf]          # coupling off: commuting field terms
    g = lambda t: 5.0 - 3.0 * t + 2.0 * t * t
    f = lambda t: np.array([1.0, g(t)])
    dt, n = 0.03, 17
    psi = mps.product_mps(W.initial_vectors(W.tfim_chain(L, 64, 1.0, 1.0)))
    timedep.td_tebd_run(psi, terms, f, method, dt, n, 1e-12, 64, scheme)
    nodes, W_ = timedep.SCHEMES[scheme]
    phi = 0.0
    for k in range(n):
        phi += dt * np.sum(W_ @ np.array([g(k * dt + c * dt) for c in nodes]))
    np.testing.assert_allclose(mps.local_expect(psi, models.SZ), np.cos(2 * phi), atol=1e-13)


def _exact_ode(H_terms, f, psi0, T):
    H = lambda t: sum(c * Hk for c, Hk in zip(f(t), H_terms))
    sol = solve_ivp(lambda t, y: -1j * (H(t) @ y), (0.0, T), psi0.astype(np.complex128), method="DOP853",
                    rtol=1e-13, atol=1e-14)
    return sol.y[:, -1]


@pytest.mark.parametrize("scheme,method,lo,hi", [(2, "tebd2", 3.5, 4.5), (4, "tebd4", 13.0, 19.0)])
def test_global_order_against_time_ordered_evolution(scheme, method, lo, hi):
    L = 6
    terms, Hd = ising_terms(L), ising_dense(L)
    f = lambda t: np.array([1.0, 1.0 + np.sin(3.0 * t)])
    spec = W.tfim_chain(L, 64, 1.0, 1.0)
    psi0 = ed.product_vector(W.initial_vectors(spec))
    T = 0.6
    ref = _exact_ode(Hd, f, psi0, T)
    errs = []
    for n in (6, 12, 24):
        psi = mps.product_mps(W.initial_vectors(spec))
        timedep.td_tebd_run(psi, terms, f, method, T / n, n, 0.0, 10 ** 6, scheme)
        errs.append(np.linalg.norm(mps.to_vector(psi) - ref))
    ratios = [a / b for a, b in zip(errs, errs[1:])]
    assert all(lo < r < hi for r in ratios), (errs, ratios)


def test_quench_against_exact_midpoint_reference():
    L = 8
    terms, Hd = ising_terms(L), ising_dense(L)
    g = lambda t: 5.0 - t                        # g(0) = 5 to g(0.5) = 4.5
    f = lambda t: np.array([1.0, g(t)])
    H0 = Hd[0] + 5.0 * Hd[1]
    v0 = ed.ground_state(H0)
    T = 0.5
    errs = []
    for n in (5, 10, 20):
        ref = timedep.exact_midpoint(Hd, f, v0, T / n, n)
        psi = mps.from_vector(v0, L, 2)
        timedep.td_tebd_run(psi, terms, f, "tebd4", T / n, n, 0.0, 10 ** 6, 2)
        errs.append(np.linalg.norm(mps.to_vector(psi) - ref))
    ratios = [a / b for a, b in zip(errs, errs[1:])]
    assert all(13.0 < r < 19.0 for r in ratios), (errs, ratios)
