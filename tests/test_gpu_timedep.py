"""GPU parity of time-dependent propagation (commutator-free Magnus
expansions over the Trotter steps, mps_tebd_td_step) against the oracle.

Tolerances as for the TEBD runs: complex128 chains |Delta <S^z_i>| <= 1e-6 and
1 - |<psi_gpu|psi_oracle>| <= 1e-9; complex64 |Delta <S^z_i>| <= 2e-7
sqrt(#updates).  The closed-form precession is held to 1e-12.
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_1703_00387_amd import api
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    h = api.Handle(0)
    yield h
    h.close()


def _ising_terms(L):
    from oracle import models as om
    hz = om.bond_hamiltonians(W.tfim_chain(L, 64, 1.0, 0.0))
    hf = [a - b for a, b in zip(om.bond_hamiltonians(W.tfim_chain(L, 64, 1.0, 1.0)), hz)]
    return [hz, hf]


def _chain_from_mps(psi, chi_max, terms, dtype="c128"):
    """Device chain holding an oracle Hastings-form MPS; hbond holds the term sets."""
    from paper_1703_00387_amd import api
    L, d = psi.L, psi.d
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    B = torch.zeros((L, chi_max, d, chi_max), dtype=tdt)
    lam = torch.zeros((L + 1, chi_max), dtype=torch.float64)
    chi = torch.ones(L + 1, dtype=torch.int32)
    for i, T in enumerate(psi.B):
        B[i, :T.shape[0], :, :T.shape[2]] = torch.from_numpy(T).to(tdt)
    for j, l in enumerate(psi.lam):
        lam[j, :len(l)] = torch.from_numpy(l)
        chi[j] = len(l)
    hb = torch.from_numpy(np.ascontiguousarray(np.array(terms)))
    return api.Chain(L, d, chi_max, B.cuda(), lam.cuda(), chi.cuda(), hb.cuda(),
                     torch.zeros(L - 1, dtype=torch.float64, device="cuda"))


def _gpu_vector(chain):
    B, lam, chi = chain.to_host()
    v = lam[0][:, None] * B[0].reshape(B[0].shape[0], -1)
    v = v.reshape(-1, B[0].shape[2])
    for T in B[1:]:
        v = (v @ T.reshape(T.shape[0], -1)).reshape(-1, T.shape[2])
    return v.reshape(-1)


def _f_nodes(f, scheme, dt, n_steps, t0=0.0):
    from paper_1703_00387_amd import api
    nodes = api.cfme_nodes(scheme)
    return np.array([[f(t0 + n * dt + c * dt) for c in nodes] for n in range(n_steps)])


def _compare(H, psi0, terms, f, order, method, scheme, dt, n_steps, check_every, chi_max, eps, dtype="c128"):
    from oracle import mps as omps, models as om, timedep
    from paper_1703_00387_amd import api, models
    ref = {}

    def obs(p, n):
        if n % check_every == 0:
            ref[n] = (omps.local_expect(p, om.SZ), omps.to_vector(p) if p.L <= 12 else None, len(p.disc))

    timedep.td_tebd_run(psi0.copy(), terms, f, method, dt, n_steps, eps, chi_max, scheme, observe=obs)
    ch = _chain_from_mps(psi0, chi_max, terms, dtype)
    fn = _f_nodes(f, scheme, dt, n_steps)
    sz = 2.0 * models.sz_operator()
    worst = 0.0
    for n in range(0, n_steps + 1, check_every):
        if n > 0:
            api.tebd_td_step(H, [ch], order, dt, check_every, eps, fn[n - check_every:n], scheme)
            code, word = H.device_status()
            assert code == 0 and word == 0, (code, word)
        site, _, _ = api.observe(H, ch, sz)
        sz_o, v_o, nupd = ref[n]
        d = np.abs(site.cpu().numpy() - sz_o).max()
        worst = max(worst, d)
        bar = 1e-6 if dtype == "c128" else max(1e-6, 2e-7 * np.sqrt(max(nupd, 1)))
        assert d <= bar, (n, d, bar)
        if v_o is not None and dtype == "c128":
            vg = _gpu_vector(ch)
            ov = abs(np.vdot(vg, v_o)) / (np.linalg.norm(vg) * np.linalg.norm(v_o))
            assert 1 - ov <= 1e-9, (n, 1 - ov)
    return worst, ch


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_paper_ising_quench_L10(H, dtype):
    """The paper's quench: Ising L = 10 from the ground state at g = 5, g ramped
    linearly to 4.5 over T = 0.5, TEBD4 with the midpoint rule (its default),
    dt = 0.01.  Also prints the paper's error measures against its exact
    midpoint reference."""
    from oracle import ed, models as om, mps as omps, timedep
    L = 10
    terms = _ising_terms(L)
    Hz = om.dense_hamiltonian_from_sites(W.tfim_chain(L, 64, 1.0, 0.0))
    Hf = om.dense_hamiltonian_from_sites(W.tfim_chain(L, 64, 1.0, 1.0)) - Hz
    v0 = ed.ground_state(Hz + 5.0 * Hf)
    psi0 = omps.from_vector(v0, L, 2)
    f = lambda t: np.array([1.0, 5.0 - t])
    # chi_max = 32 holds every Schmidt value at L = 10 and nothing is cut
    # (eps_local = 0), as in the paper's study; a cut at 1e-12 would already
    # move the two-site density matrices of distant pairs by ~1e-5 (square
    # root of the discarded weight)
    worst, ch = _compare(H, psi0, terms, f, 4, "tebd4", 2, 0.01, 50, 10, 32, 0.0, dtype)
    if dtype == "c128":
        ref = timedep.exact_midpoint([Hz, Hf], f, v0, 0.01, 50)
        meas = ed.error_measures(_gpu_vector(ch), ref, Hz + 4.5 * Hf, L, 2)
        print(f"quench L10 worst |dsz| {worst:.2e}; error measures vs exact midpoint: {meas}")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_fourth_order_scheme_and_sweep(H, dtype):
    from oracle import mps as omps
    L = 8
    terms = _ising_terms(L)
    f = lambda t: np.array([1.0, 1.0 + np.sin(3.0 * t)])
    psi0 = omps.product_mps(W.initial_vectors(W.tfim_chain(L, 64, 1.0, 1.0)))
    _compare(H, psi0, terms, f, 4, "tebd4", 4, 0.05, 12, 4, 16, 1e-12, dtype)
    psi0 = omps.product_mps(W.initial_vectors(W.tfim_chain(L, 64, 1.0, 1.0)))
    _compare(H, psi0, terms, f, 0, "sweep", 2, 0.05, 12, 4, 16, 1e-12, dtype)


def test_ramped_field_precession_closed_form(H):
    """Coupling off: <sz_i>(T) = cos(2 sum_n dt gbar_n), gbar_n the scheme's
    quadrature of g over step n."""
    from oracle import mps as omps, timedep
    from paper_1703_00387_amd import api, models
    L = 6
    hz, hf = _ising_terms(L)
    terms = [[0.0 * h for h in hz], hf]
    g = lambda t: 5.0 - 3.0 * t + 2.0 * t * t
    f = lambda t: np.array([1.0, g(t)])
    dt, n = 0.03, 17
    for scheme in (2, 4):
        psi0 = omps.product_mps(W.initial_vectors(W.tfim_chain(L, 64, 1.0, 1.0)))
        ch = _chain_from_mps(psi0, 8, terms)
        api.tebd_td_step(H, [ch], 2, dt, n, 1e-12, _f_nodes(f, scheme, dt, n), scheme)
        nodes, Wt = timedep.SCHEMES[scheme]
        phi = sum(dt * np.sum(Wt @ np.array([g(k * dt + c * dt) for c in nodes])) for k in range(n))
        site, _, _ = api.observe(H, ch, 2.0 * models.sz_operator())
        np.testing.assert_allclose(site.cpu().numpy(), np.cos(2 * phi), atol=1e-12)


def test_batch_of_chains_and_errors(H):
    """Chains of different length in one call match the oracle per chain; bad
    arguments are refused."""
    from oracle import mps as omps, models as om, timedep
    from paper_1703_00387_amd import api, models, _lib
    f = lambda t: np.array([1.0, 0.8 + 0.5 * np.cos(2.0 * t)])
    specs = [W.tfim_chain(L, 16, 1.0, 1.0) for L in (6, 9, 12)]
    chains, refs = [], []
    for sp in specs:
        terms = _ising_terms(sp.L)
        psi0 = omps.product_mps(W.initial_vectors(sp))
        chains.append(_chain_from_mps(psi0, 16, terms))
        refs.append(timedep.td_tebd_run(psi0.copy(), terms, f, "tebd2", 0.04, 10, 1e-12, 16, 4))
    api.tebd_td_step(H, chains, 2, 0.04, 10, 1e-12, _f_nodes(f, 4, 0.04, 10), 4)
    for ch, ref in zip(chains, refs):
        site, _, _ = api.observe(H, ch, 2.0 * models.sz_operator())
        assert np.abs(site.cpu().numpy() - omps.local_expect(ref, om.SZ)).max() <= 1e-6
    with pytest.raises(ValueError):
        api.tebd_td_step(H, chains, 2, 0.04, 2, 1e-12, _f_nodes(f, 4, 0.04, 10), 4)   # wrong step count
    fbad = _f_nodes(f, 4, 0.04, 2)
    fbad[1, 0, 1] = np.nan
    with pytest.raises(_lib.MPSError) as e:
        api.tebd_td_step(H, chains, 2, 0.04, 2, 1e-12, fbad, 4)
    assert e.value.code == _lib.MPS_ERR_INVALID
