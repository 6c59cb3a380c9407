"""GPU parity of the two-site update against the oracle (through the C ABI).

Tolerances (FP32 contractions, FP64 SVD; stated per result):
  propagators: complex128 output within 1e-12 of the oracle's, complex64 1e-6
  truncated SVD (FP64 Jacobi; absolute floor 1e-15 |theta|^2 on inner products):
    squared singular values within 1e-13 |theta|^2, values >= 1e-3 s_1 within
    1e-12 s_1, discarded weight within 1e-12 + 1e-6 w, count k identical,
    reconstruction error^2 = w within 1e-12, kept rows p, q of V^dag
    orthogonal to 1e-10 + 1e-14 |theta|^2 / (s_p s_q)
  TEBD runs, complex128 chains (FP64 MFMA contractions): |Delta <S^z_i>| <= 1e-6
    at every checked step, |Delta E|/L <= 1e-6, 1 - |<psi_gpu|psi_oracle>| <=
    1e-9 (state check at L <= 16), over the window where the oracle's summed
    discarded weight is below 1e-8.
  complex64 chains (FP32 MFMA, FP32 storage): the rounding floor of FP32
    storage is ~6e-8 per update, accumulating like a random walk, so the bar
    is |Delta <S^z_i>| <= 2e-7 sqrt(#updates) (measured and printed).
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


def _herm(n, key):
    A = W.random_complex((n, n), key)
    return A + A.conj().T


# ---------------------------------------------------------------- propagators
@pytest.mark.parametrize("dd", [4, 9, 16, 25])
def test_gates_match_oracle(H, dd):
    from oracle import mps as omps
    hs = np.stack([_herm(dd, (1, dd, i)) for i in range(5)])
    taus = np.array([0.01, 0.05, -0.3, 1.7, 0.0])
    G64, G128 = H.gates(torch.from_numpy(hs).cuda(), torch.from_numpy(taus).cuda())
    G128 = G128.cpu().numpy()
    G64 = G64.cpu().numpy()
    for i in range(5):
        ref = omps.gate(hs[i], taus[i])
        assert np.abs(G128[i] - ref).max() < 1e-12
        assert np.abs(G64[i] - ref).max() < 1e-6


# ------------------------------------------------------------- truncated SVD
def _graded(m, n, key, decay):
    r = min(m, n)
    Uq, _ = np.linalg.qr(W.random_complex((m, r), key + (1,)))
    Vq, _ = np.linalg.qr(W.random_complex((n, r), key + (2,)))
    s = np.exp(-decay * np.arange(r))
    return (Uq * s) @ Vq.conj().T


@pytest.mark.parametrize("m,n,chi,eps,kind", [
    (8, 8, 8, 0.0, "rand"),
    (64, 64, 32, 1e-12, "graded"),
    (37, 91, 40, 1e-10, "graded"),        # ragged, several blocks and a tail
    (130, 70, 50, 1e-12, "rand"),
    (256, 256, 128, 1e-12, "graded"),
    (512, 512, 256, 1e-12, "graded"),
    (1280, 1280, 256, 1e-12, "graded"),    # 20 panel pairs: each split over 12 column ranges
    (100, 100, 100, 1e-20, "rank5"),
    (1, 16, 4, 0.0, "rand"),
])
def test_truncate_matches_oracle(H, m, n, chi, eps, kind):
    from oracle import mps as omps
    if kind == "rand":
        A = W.random_complex((m, n), (2, m, n))
    elif kind == "graded":
        A = _graded(m, n, (3, m, n), 0.08)
    else:
        A = W.random_complex((m, 5), (4, m)) @ W.random_complex((5, n), (5, n))
    A = A / np.linalg.norm(A)
    U, S, Vh, k, disc, norm2 = H.truncate(torch.from_numpy(A).cuda(), chi, eps)
    U, S, Vh = U.cpu().numpy(), S.cpu().numpy(), Vh.cpu().numpy()
    Uo, so, Vho, wo, nko, sfull = omps.truncate(A, chi, eps)
    print(f"m={m} n={n} k={k}/{len(so)} max|ds2|={np.abs(S**2 - so**2).max():.2e} "
          f"disc={disc:.3e}/{wo:.3e}")
    assert k == len(so)
    assert np.abs(S ** 2 - so ** 2).max() <= 1e-13
    big = so >= 1e-3 * sfull[0]
    assert np.abs(S[big] - so[big]).max() <= 1e-12 * sfull[0]
    assert abs(disc - wo) <= 1e-12 + 1e-6 * wo
    assert abs(norm2 - 1.0) < 1e-12
    R = (U * S) @ Vh
    assert abs(np.linalg.norm(A - R) ** 2 - wo) < 1e-12
    # right singular vectors: rows p, q are orthogonal up to the Jacobi floor,
    # |<v_p, v_q>| <= 1e-10 + 10 * abs_tol |A|^2 / (s_p s_q), abs_tol = 1e-15
    ov = np.abs(Vh @ Vh.conj().T - np.eye(k))
    bound = 1e-10 + 10 * 1e-15 / np.outer(S, S)
    assert (ov <= bound).all(), float((ov / bound).max())


# ---------------------------------------------------------------- TEBD runs
def _gpu_chain(spec, dtype="c128"):
    from paper_1703_00387_amd import api, models
    return api.Chain.product(W.initial_vectors(spec), spec.chi_max, models.bond_hamiltonians(spec), dtype=dtype)


def _gpu_vector(chain):
    B, lam, chi = chain.to_host()
    v = lam[0][:, None] * B[0].reshape(B[0].shape[0], -1)
    v = v.reshape(-1, B[0].shape[2])
    for T in B[1:]:
        v = (v @ T.reshape(T.shape[0], -1)).reshape(-1, T.shape[2])
    return v.reshape(-1)


def _run_compare(H, spec, method, dt, n_steps, eps, check_every, state_check=False, flags=0, dtype="c128"):
    from oracle import mps as omps, models as om
    from paper_1703_00387_amd import api, models
    order = {"tebd2": 2, "tebd4": 4, "sweep": 0}[method]
    hs = om.bond_hamiltonians(spec)
    ref = {}
    op_o = om.number_op(spec.d) if spec.model == "bh" else 0.5 * om.SZ

    def obs(p, n):
        if n % check_every == 0:
            ref[n] = (omps.local_expect(p, op_o), omps.energy(p, hs), p.copy(), sum(p.disc), len(p.disc))

    omps.tebd_run(spec, method, dt, n_steps, eps, observe=obs)
    ch = _gpu_chain(spec, dtype)
    sz = models.number_operator(spec.d) if spec.model == "bh" else models.sz_operator()
    hb = models.bond_hamiltonians(spec)
    worst = 0.0
    for n in range(0, n_steps + 1, check_every):
        if n > 0:
            api.tebd_step(H, [ch], order, dt, check_every, eps, flags)
        site, bond, _ = api.observe(H, ch, sz, hb, per_bond=True)
        code, word = H.device_status()
        assert code == 0, (n, word)
        sz_g = site.cpu().numpy()
        E_g = bond.cpu().numpy().sum()
        sz_o, E_o, p_o, wsum, nupd = ref[n]
        if wsum < 1e-8:
            dsz = np.abs(sz_g - sz_o).max()
            worst = max(worst, dsz)
            bar = 1e-6 if dtype == "c128" else max(1e-6, 2e-7 * np.sqrt(max(nupd, 1)))
            assert dsz <= bar, (n, dsz, bar)
            assert abs(E_g - E_o) / spec.L <= bar, (n, E_g, E_o)
            if state_check and dtype == "c128":
                vg = _gpu_vector(ch)
                vo = omps.to_vector(p_o)
                ov = abs(np.vdot(vg, vo)) / (np.linalg.norm(vg) * np.linalg.norm(vo))
                assert 1 - ov <= 1e-9, (n, 1 - ov)
    return worst, ch


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_tfim_tebd2_L16_full_run(H, dtype):
    """TEBD2 transverse Ising, L=16, J=g=1, all up, dt=0.01, 100 steps, chi_max=32."""
    spec = W.tfim_tebd2_L16().chains[0]
    worst, ch = _run_compare(H, spec, "tebd2", 0.01, 100, 1e-12, 10, state_check=True, dtype=dtype)
    print(f"tfim L16 {dtype} worst |dSz| {worst:.3e} chi {ch.chi.cpu().numpy().max()}")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_xxz_tebd4_small(H, dtype):
    spec = W.xxz_chain(12, 64, 1.0, 0.5)
    worst, _ = _run_compare(H, spec, "tebd4", 0.05, 20, 1e-12, 5, state_check=True, dtype=dtype)
    print(f"xxz L12 tebd4 {dtype} worst |dSz| {worst:.3e}")


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_sweep_tfim_and_xxz(H, dtype):
    """The paper's own second-order sweep (one bond at a time, left to right
    then back, dt/2 each) against the oracle's sweep."""
    spec = W.tfim_chain(12, 32, 1.0, 1.0, "all_up")
    worst, _ = _run_compare(H, spec, "sweep", 0.02, 30, 1e-12, 10, state_check=True, dtype=dtype)
    spec = W.xxz_chain(10, 16, 1.0, 0.5)
    worst2, _ = _run_compare(H, spec, "sweep", 0.05, 20, 1e-12, 5, state_check=True, dtype=dtype)
    print(f"sweep {dtype} worst |dSz| tfim {worst:.3e} xxz {worst2:.3e}")


def test_sweep_batch_of_chains_and_graph(H):
    """Sweeps of chains of different length in one call (each chain runs its own
    left-to-right-and-back order) match the oracle per chain; graph replay equals eager."""
    from oracle import mps as omps, models as om
    from paper_1703_00387_amd import api, models, _lib
    wl = W.xxz_batch256(n_chains=3)
    specs = [W.xxz_chain(L, 16, 1.0, 0.5, None, c.Jz_b[:L - 1], "random_product", c.local_states[:L])
             for L, c in zip((8, 11, 14), wl.chains)]
    a = [_gpu_chain(sp) for sp in specs]
    b = [_gpu_chain(sp) for sp in specs]
    api.tebd_step(H, a, 0, 0.05, 6, 1e-12)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        api.tebd_step(H, b, 0, 0.05, 6, 1e-12, flags=_lib.MPS_FLAG_GRAPH)
    s.synchronize()
    for sp, x, y in zip(specs, a, b):
        ref = omps.tebd_run(sp, "sweep", 0.05, 6, 1e-12)
        site, _, _ = api.observe(H, x, models.sz_operator())
        dd = np.abs(site.cpu().numpy() - omps.local_expect(ref, 0.5 * om.SZ)).max()
        assert dd <= 1e-6, (sp.L, dd)
        site_g, _, _ = api.observe(H, y, models.sz_operator())
        assert np.abs(site_g.cpu().numpy() - site.cpu().numpy()).max() <= 1e-9


def test_bh_tebd2_d5(H):
    spec = W.bh_chain(6, 4, 40, 1.0, 4.0)
    _run_compare(H, spec, "tebd2", 0.02, 10, 1e-12, 5, state_check=True)


def test_xxz_random_product_couplings(H):
    wl = W.xxz_batch256(n_chains=3)
    spec = wl.chains[0]
    spec = W.xxz_chain(10, 32, 1.0, 0.5, J_b=None, Jz_b=spec.Jz_b[:9], init="random_product",
                       local_states=spec.local_states[:10])
    _run_compare(H, spec, "tebd2", 0.05, 10, 1e-12, 5, state_check=True)


def test_batched_equals_unbatched(H):
    """Each chain's result must not depend on what else is in the batch."""
    from paper_1703_00387_amd import api
    wl = W.xxz_batch256(n_chains=5)
    specs = [W.xxz_chain(min(c.L, 20), min(c.chi_max, 64), 1.0, 0.5, None, c.Jz_b[:min(c.L, 20) - 1],
                         "random_product", c.local_states[:min(c.L, 20)]) for c in wl.chains]
    alone = []
    for sp in specs:
        ch = _gpu_chain(sp)
        api.tebd_step(H, [ch], 2, 0.05, 4, 1e-12)
        alone.append(ch)
    batch = [_gpu_chain(sp) for sp in specs]
    api.tebd_step(H, batch, 2, 0.05, 4, 1e-12)
    torch.cuda.synchronize()
    for a, b in zip(alone, batch):
        assert torch.equal(a.chi, b.chi)
        assert torch.equal(a.B, b.B)
        assert torch.equal(a.lam, b.lam)


def test_graph_replay_equals_eager(H):
    from paper_1703_00387_amd import api
    spec = W.xxz_chain(12, 32, 1.0, 0.5)
    eager = _gpu_chain(spec)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        api.tebd_step(H, [eager], 2, 0.05, 6, 1e-12, flags=0x2)  # fixed sweeps, no host sync
        g = _gpu_chain(spec)
        api.tebd_step(H, [g], 2, 0.05, 6, 1e-12, flags=0x1)      # captured step, replayed 6 times
    s.synchronize()
    assert torch.equal(eager.chi, g.chi)
    assert torch.equal(eager.B, g.B)
    assert torch.equal(eager.lam, g.lam)
    # the handle keeps the captured step: a second call with the same chain,
    # schedule and options replays it without a new capture; a changed option
    # (or another chain) captures anew
    with torch.cuda.stream(s):
        api.tebd_step(H, [eager], 2, 0.05, 3, 1e-12, flags=0x2)
        api.tebd_step(H, [g], 2, 0.05, 3, 1e-12, flags=0x1)
        H.set_option(4, 2)
        try:
            api.tebd_step(H, [eager], 2, 0.05, 2, 1e-12, flags=0x2)
            api.tebd_step(H, [g], 2, 0.05, 2, 1e-12, flags=0x1)
        finally:
            H.set_option(4, 1)
        other = _gpu_chain(spec)
        ref = _gpu_chain(spec)
        api.tebd_step(H, [ref], 2, 0.05, 4, 1e-12, flags=0x2)
        api.tebd_step(H, [other], 2, 0.05, 4, 1e-12, flags=0x1)
    s.synchronize()
    for a, b in ((eager, g), (ref, other)):
        assert torch.equal(a.chi, b.chi)
        assert torch.equal(a.B, b.B)
        assert torch.equal(a.lam, b.lam)


def test_argument_errors(H):
    from paper_1703_00387_amd import api, _lib
    spec = W.xxz_chain(6, 8, 1.0, 0.5)
    ch = _gpu_chain(spec)
    with pytest.raises(_lib.MPSError) as e:
        api.tebd_step(H, [ch], 3, 0.05, 1, 1e-12)
    assert e.value.code == _lib.MPS_ERR_INVALID
    with pytest.raises(_lib.MPSError) as e:
        H.truncate(torch.zeros((5000, 2), dtype=torch.complex128, device="cuda"), 2, 0.0)
    assert e.value.code == _lib.MPS_ERR_CAPACITY


def test_nonfinite_flag(H):
    A = torch.full((8, 8), float("nan"), dtype=torch.complex128, device="cuda")
    H.truncate(A, 4, 0.0)
    code, word = H.device_status()
    from paper_1703_00387_amd import _lib
    assert code == _lib.MPS_ERR_NONFINITE and word & _lib.MPS_DEV_NONFINITE


def test_batch_of_chains_matches_oracle(H):
    """Several chains of different L and chi_max in one call: each matches the
    oracle run of that chain alone (the batched workload at reduced size)."""
    from oracle import mps as omps, models as om
    from paper_1703_00387_amd import api, models
    wl = W.xxz_batch256(n_chains=6)
    specs = []
    for i, c in enumerate(wl.chains):
        L = 12 + 2 * i
        specs.append(W.xxz_chain(L, [16, 32][i % 2], 1.0, 0.5, None, c.Jz_b[:L - 1], "random_product",
                                 c.local_states[:L]))
    chains = [_gpu_chain(sp) for sp in specs]
    api.tebd_step(H, chains, 2, 0.05, 12, 1e-12)
    for sp, ch in zip(specs, chains):
        ref = omps.tebd_run(sp, "tebd2", 0.05, 12, 1e-12)
        site, _, _ = api.observe(H, ch, models.sz_operator())
        d = np.abs(site.cpu().numpy() - omps.local_expect(ref, 0.5 * om.SZ)).max()
        assert d <= 1e-6 or sum(ref.disc) >= 1e-8, (sp.L, d)


def test_plain_form_equals_batched(H):
    from paper_1703_00387_amd import api, _lib
    wl = W.xxz_batch256(n_chains=4)
    specs = [W.xxz_chain(14, 32, 1.0, 0.5, None, c.Jz_b[:13], "random_product", c.local_states[:14])
             for c in wl.chains]
    a = [_gpu_chain(sp) for sp in specs]
    b = [_gpu_chain(sp) for sp in specs]
    api.tebd_step(H, a, 2, 0.05, 5, 1e-12)
    api.tebd_step(H, b, 2, 0.05, 5, 1e-12, flags=_lib.MPS_FLAG_PLAIN)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x.chi, y.chi) and torch.equal(x.B, y.B) and torch.equal(x.lam, y.lam)


def _canonical_bh_chain(dtype):
    """A seeded random Bose-Hubbard state (L = 6, d = 5) in Hastings form from
    the oracle (bond dimensions 1, 5, 25, 125, 25, 5, 1) as a GPU chain of
    chi_max = 128, and the oracle's tensors (rounded to the chain precision)."""
    from oracle import mps as omps
    from paper_1703_00387_amd import api, models
    L, nmax, cm = 6, 4, 128
    spec = W.bh_chain(L, nmax, cm)
    d = spec.d
    vec = W.random_complex((d ** L,), (85, 1))
    psi0 = omps.from_vector(vec / np.linalg.norm(vec), L, d)
    prof = psi0.chis()
    assert prof == [1, 5, 25, 125, 25, 5, 1], prof
    tdt = torch.complex128 if dtype == "c128" else torch.complex64
    Bd = np.zeros((L, cm, d, cm), np.complex128)
    lam = np.zeros((L + 1, cm))
    Bs = []
    for i in range(L):
        t = torch.from_numpy(psi0.B[i]).to(tdt).to(torch.complex128).numpy()  # the oracle starts from the rounded tensors
        Bd[i, :prof[i], :, :prof[i + 1]] = t
        Bs.append(t)
    for j in range(L + 1):
        lam[j, :prof[j]] = psi0.lam[j]
    ch = api.Chain(L, d, cm, torch.from_numpy(Bd).to(tdt).cuda(), torch.from_numpy(lam).cuda(),
                   torch.tensor(prof, dtype=torch.int32).cuda(),
                   torch.from_numpy(np.ascontiguousarray(models.bond_hamiltonians(spec))).cuda(),
                   torch.zeros(L - 1, dtype=torch.float64).cuda())
    return spec, ch, Bs, [l.copy() for l in psi0.lam]


@pytest.mark.parametrize("warm", [1, 0])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_long_contractions_canonical_chain(H, dtype, warm):
    """One TEBD2 step of a seeded random Bose-Hubbard state (L = 6, d = 5) put
    into Hastings form by the oracle: bond dimensions 1, 5, 25, 125, 25, 5, 1,
    so the middle update contracts over 125 = 7 * 16 + 13 (many K-chunks and a
    ragged last one, which the product-state runs above do not reach) and its
    125 x 125 theta' gets the Jacobi's warm start (Q from the QR of
    Lambda_l B_b, a partial last panel), here on and off.  Bond dimensions
    identical, Schmidt values within 1e-11 (c128) or 2e-6 (c64) of the
    oracle's."""
    from oracle import mps as omps, models as om
    from paper_1703_00387_amd import api
    spec, ch, Bs, lams = _canonical_bh_chain(dtype)
    L, d, cm = spec.L, spec.d, spec.chi_max
    H.set_option(9, warm)
    try:
        api.tebd_step(H, [ch], 2, 0.05, 1, 1e-14)
        torch.cuda.synchronize()
    finally:
        H.set_option(9, 0)
    code, word = H.device_status()
    assert code == 0, word
    psi = omps.MPS(Bs, lams, d)
    hs = om.bond_hamiltonians(spec)
    for bonds, tau in omps.strang_layers(L, 0.05):
        for b in bonds:
            omps.apply_bond(psi, b, omps.gate(hs[b], tau), cm, 1e-14)
    _, lam1, chi1 = ch.to_host()
    assert list(chi1) == psi.chis()
    dl = max(np.abs(lam1[j] - psi.lam[j]).max() for j in range(L + 1))
    print(f"long contractions {dtype} warm {warm}: chis {list(chi1)} max|dlam| {dl:.2e}")
    assert dl <= (1e-11 if dtype == "c128" else 2e-6), dl


def test_graph_replay_with_warm_start(H):
    """The warm start's launches (the QR of Lambda_l B_b and Q^dag theta',
    sized from capacities, no host synchronisation) captured in the kept
    graph: two captured TEBD2 steps and a replay equal the same steps run
    eagerly with fixed sweeps, bit for bit."""
    from paper_1703_00387_amd import api
    _, eager, _, _ = _canonical_bh_chain("c128")
    _, g, _, _ = _canonical_bh_chain("c128")
    H.set_option(9, 1)
    try:
        s = torch.cuda.Stream()
        with torch.cuda.stream(s):
            api.tebd_step(H, [eager], 2, 0.05, 2, 1e-14, flags=0x2)  # fixed sweeps, no host sync
            api.tebd_step(H, [g], 2, 0.05, 2, 1e-14, flags=0x1)      # captured, replayed
            api.tebd_step(H, [eager], 2, 0.05, 1, 1e-14, flags=0x2)
            api.tebd_step(H, [g], 2, 0.05, 1, 1e-14, flags=0x1)      # the kept graph again
        s.synchronize()
    finally:
        H.set_option(9, 0)
    code, word = H.device_status()
    assert code == 0, word
    assert torch.equal(eager.chi, g.chi)
    assert torch.equal(eager.B, g.B)
    assert torch.equal(eager.lam, g.lam)
