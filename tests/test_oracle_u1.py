"""Pins of the U(1)-symmetric truncated SVD and TEBD oracle (oracle/u1.py)
against the dense SVD, the exact Trotter circuit and the charge structure of
number-conserving states.

* A random theta that is block diagonal in charge: the blockwise spectrum is
  the dense spectrum without its structural zeros; k, the discarded weight,
  n_k and the truncated theta agree with ``mps.truncate``; U_k and Vh_k are
  block sparse and orthonormal.
* The exact state of an XXZ chain evolved from a Neel state (conserved total
  S^z): cut into left and right halves, its coefficient matrix vanishes
  outside the blocks where the left charge plus the right charge is the
  total, and the blockwise and dense decompositions agree.
* TEBD of charge-carrying chains (XXZ from a Neel state with charges n_up or
  2 S^z, Bose-Hubbard at unit filling with the particle number): untruncated,
  the state is the Trotter circuit's and every bond's Schmidt values split by
  charge as the exact vector's do; truncated, the run equals the dense TEBD
  (same bond dimensions, discarded weight and state).
* Z_2 charges (the parity of n_up) on an XYZ chain, where n_up itself is not
  conserved: untruncated, the Trotter circuit and its parity-resolved
  spectra; the U(1) run misses the circuit; truncated, the dense TEBD.
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


# ---------------------------------------------------------------------------
# TEBD of charge-carrying chains (apply_bond_u1 / tebd_run_u1)
# ---------------------------------------------------------------------------

def _left_charges(nsites, d, qsite):
    """Charge of every configuration of nsites sites (first site most significant)."""
    q = np.zeros(1, dtype=np.int64)
    for _ in range(nsites):
        q = (q[:, None] + np.asarray(qsite)[None, :]).reshape(-1)
    return q


@pytest.mark.parametrize("spec,qsite,method", [
    (W.xxz_chain(10, 32, 1.0, 0.5), [1, 0], "tebd2"),
    (W.xxz_chain(9, 16, 1.0, 0.7), [1, -1], "sweep"),
    (W.bh_chain(6, 2, 27, 1.0, 3.0), [0, 1, 2], "tebd4"),
])
def test_untruncated_u1_tebd_equals_trotter_circuit(spec, qsite, method):
    """At full bond dimension the blockwise update loses nothing: the state is
    the exact Trotter circuit's, and every bond's Schmidt values split by
    charge as the exact vector's coefficient matrix does (the charge labels
    come out right: a wrong label moves a value to another sector)."""
    L, d = spec.L, spec.d
    psi, q = u1.tebd_run_u1(spec, method, 0.1, 5, -1.0, qsite)   # keep everything
    v = ed.trotter_circuit(spec, method, 0.1, 5)
    got = omps.to_vector(psi)
    assert 1.0 - abs(np.vdot(got, v)) <= 1e-12
    for b in range(1, L):
        M = v.reshape(d ** b, d ** (L - b))
        qL = _left_charges(b, d, qsite)
        exact = {}
        for c in sorted(set(qL.tolist())):
            s = np.linalg.svd(M[qL == c], compute_uv=False)
            s = s[s > 1e-6]
            if len(s):
                exact[int(c)] = s
        ours = {c: s[s > 1e-6] for c, s in u1.sector_spectra(psi.lam[b], q[b]).items()}
        ours = {c: s for c, s in ours.items() if len(s)}
        assert sorted(exact) == sorted(ours), b
        for c in exact:
            assert len(exact[c]) == len(ours[c]) and np.abs(exact[c] - ours[c]).max() <= 1e-10, (b, c)


def test_truncated_u1_tebd_equals_dense_tebd():
    """With truncation the blockwise and the dense update keep the same
    values (the spectrum is the same set; no two sectors tie at the cut), so
    the two runs give the same state, bond dimensions and discarded weight."""
    spec = W.xxz_chain(12, 6, 1.0, 0.5)
    psi, q = u1.tebd_run_u1(spec, "tebd2", 0.05, 30, 1e-10, [1, 0])
    ref = omps.tebd_run(spec, "tebd2", 0.05, 30, 1e-10)
    assert psi.chis() == ref.chis()
    assert abs(sum(psi.disc) - sum(ref.disc)) <= 1e-12 + 1e-8 * sum(ref.disc)
    assert sum(ref.disc) > 1e-6                       # the cut is inside the spectrum
    a, r = omps.to_vector(psi), omps.to_vector(ref)
    assert 1.0 - abs(np.vdot(a, r)) / (np.linalg.norm(a) * np.linalg.norm(r)) <= 1e-10
    # total charge: every configuration in the support has L/2 up spins
    qs = _left_charges(12, 2, [1, 0])
    assert np.abs(a[qs != 6]).max() == 0.0


def test_product_charges_need_basis_states():
    spec = W.xxz_chain(4, 4, 1.0, 0.5, init="random_product", local_states=W.random_complex((4, 2), (5,)))
    with pytest.raises(ValueError):
        u1.product_charges(W.initial_vectors(spec), [1, 0])
    q = u1.product_charges(W.product_state_vectors("neel", 5, 2), [1, 0])
    assert [int(x[0]) for x in q] == [0, 1, 1, 2, 2, 3]


# ---------------------------------------------------------------------------
# Z_n charges (modulus n): the parity of n_up on an XYZ chain
# ---------------------------------------------------------------------------

def _xyz_terms(L, jx=1.0, jy=0.6, jz=0.4):
    """XYZ bond terms: with jx != jy the pair terms s+s+ and s-s- change n_up
    by 2, so only its parity (Z_2) is conserved."""
    X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
    Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
    Z = np.diag([1.0, -1.0]).astype(np.complex128)
    h = 0.25 * (jx * np.kron(X, X) + jy * np.kron(Y, Y) + jz * np.kron(Z, Z))
    return [h.copy() for _ in range(L - 1)]


def _circuit(spec, hs, method, dt, n_steps):
    v = ed.product_vector(W.initial_vectors(spec))
    for _ in range(n_steps):
        for bonds, tau in omps.step_layers(method, spec.L, dt):
            for b in bonds:
                v = ed.apply_two_site(v, omps.gate(hs[b], tau), b, spec.L, spec.d)
    return v


def test_z2_tebd_of_an_xyz_chain():
    """Untruncated, the Z_2 run is the Trotter circuit and each bond's Schmidt
    values split by the parity of the left n_up as the exact vector's do; a
    U(1) run on the same chain projects out the n_up-changing terms and
    misses the circuit (the modulus matters); truncated, Z_2 equals the dense
    TEBD."""
    L, d = 10, 2
    spec = W.xxz_chain(L, 32, 1.0, 0.5)
    hs = _xyz_terms(L)
    psi, q = u1.tebd_run_u1(spec, "tebd2", 0.1, 5, -1.0, [1, 0], modulus=2, hs=hs)
    v = _circuit(spec, hs, "tebd2", 0.1, 5)
    assert 1.0 - abs(np.vdot(omps.to_vector(psi), v)) <= 1e-12
    for b in range(1, L):
        M = v.reshape(d ** b, d ** (L - b))
        par = _left_charges(b, d, [1, 0]) % 2
        for c in (0, 1):
            s = np.linalg.svd(M[par == c], compute_uv=False)
            s = s[s > 1e-6]
            ours = u1.sector_spectra(psi.lam[b], q[b]).get(c, np.zeros(0))
            ours = ours[ours > 1e-6]
            assert len(s) == len(ours) and (len(s) == 0 or np.abs(s - ours).max() <= 1e-10), (b, c)
        assert set(np.asarray(q[b]).tolist()) <= {0, 1}
    pu, _ = u1.tebd_run_u1(spec, "tebd2", 0.1, 5, -1.0, [1, 0], modulus=0, hs=hs)
    assert 1.0 - abs(np.vdot(omps.to_vector(pu), v)) / np.linalg.norm(omps.to_vector(pu)) > 1e-4
    spec = W.xxz_chain(12, 6, 1.0, 0.5)
    hs = _xyz_terms(12)
    pz, _ = u1.tebd_run_u1(spec, "tebd2", 0.05, 30, 1e-10, [1, 0], modulus=2, hs=hs)
    ref = omps.product_mps(W.initial_vectors(spec))
    for _ in range(30):
        for bonds, tau in omps.strang_layers(12, 0.05):
            for b in bonds:
                omps.apply_bond(ref, b, omps.gate(hs[b], tau), 6, 1e-10)
    assert pz.chis() == ref.chis() and sum(ref.disc) > 1e-7
    a, r = omps.to_vector(pz), omps.to_vector(ref)
    assert 1.0 - abs(np.vdot(a, r)) / (np.linalg.norm(a) * np.linalg.norm(r)) <= 1e-10


def test_krylov_tebd_on_charge_blocks_equals_dense_krylov_tebd():
    """The Krylov sweep with the blockwise cut equals the dense Krylov sweep
    under truncation (same bond dimensions and state), and its bond charges
    split the Schmidt values as at the start of the next update."""
    from oracle import ktebd
    spec = W.xxz_chain(10, 6, 1.0, 0.5)
    psi, q = u1.ktebd_run_u1(spec, 0.05, 20, 1e-10, [1, 0], n_max=20, tol=1e-12)
    ref = ktebd.ktebd_run(spec, 0.05, 20, 1e-10, n_max=20, tol=1e-12)
    assert psi.chis() == ref.chis() and sum(ref.disc) > 1e-8
    a, r = omps.to_vector(psi), omps.to_vector(ref)
    assert 1.0 - abs(np.vdot(a, r)) / (np.linalg.norm(a) * np.linalg.norm(r)) <= 1e-10
    assert all(len(q[b]) == len(psi.lam[b]) for b in range(spec.L + 1))


def test_time_dependent_run_on_charge_blocks_equals_dense():
    """The Magnus-scheme run with the blockwise cut (H(t) = H_xy + f(t) H_zz,
    both conserving n_up) equals the dense run under truncation."""
    from oracle import models as om, timedep
    L, chi = 10, 8
    spec = W.xxz_chain(L, chi, 1.0, 0.5)
    hxy = om.bond_hamiltonians(W.xxz_chain(L, chi, 1.0, 0.0))
    hzz = [om.bond_hamiltonians(W.xxz_chain(L, chi, 1.0, 1.0))[b] - hxy[b] for b in range(L - 1)]
    f = lambda t: np.array([1.0, 0.5 + 0.5 * np.sin(2.0 * t)])
    v = W.initial_vectors(spec)
    q = u1.product_charges(v, [1, 0])
    a = timedep.td_tebd_run(omps.product_mps(v), [hxy, hzz], f, "tebd4", 0.05, 16, 1e-10, chi, 4,
                            charges=(q, [1, 0], 0))
    r = timedep.td_tebd_run(omps.product_mps(v), [hxy, hzz], f, "tebd4", 0.05, 16, 1e-10, chi, 4)
    assert a.chis() == r.chis() and sum(r.disc) > 1e-9
    va, vr = omps.to_vector(a), omps.to_vector(r)
    assert 1.0 - abs(np.vdot(va, vr)) / (np.linalg.norm(va) * np.linalg.norm(vr)) <= 1e-10


@pytest.mark.parametrize("spec,qsite", [(W.xxz_chain(8, 6, 1.0, 0.5), [1, 0]),
                                        (W.bh_chain(6, 2, 9, 1.0, 3.0), [0, 1, 2])], ids=["xxz", "bh"])
def test_tdvp_on_charge_blocks_equals_dense_tdvp(spec, qsite):
    """Two-site TDVP with every split on the charge blocks equals the dense
    TDVP under truncation, and the bond charges follow the bond dimensions."""
    from oracle import models as om, tdvp as ot
    Ws = om.mpo(spec)
    v = W.initial_vectors(spec)
    a = ot.product_oc(v)
    r = ot.product_oc(v)
    q = u1.product_charges(v, qsite)
    for _ in range(10):
        ot.tdvp2_step(a, Ws, 0.05, spec.chi_max, 1e-10, 20, 1e-12, charges=(q, qsite, 0))
        ot.tdvp2_step(r, Ws, 0.05, spec.chi_max, 1e-10, 20, 1e-12)
    chis = [T.shape[0] for T in a.M] + [1]
    assert chis == [T.shape[0] for T in r.M] + [1]
    assert max(chis) > 2
    assert all(len(q[b]) == chis[b] for b in range(spec.L + 1))
    va, vr = a.to_vector(), r.to_vector()
    assert 1.0 - abs(np.vdot(va, vr)) / (np.linalg.norm(va) * np.linalg.norm(vr)) <= 1e-10
