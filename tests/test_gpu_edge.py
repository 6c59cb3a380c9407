"""Edge cases of the GPU path against the oracle, closed forms or exact
constructions: the shortest chain (one bond), chi_max = 1, zero steps,
complex bond terms, the capacity limits, and a truncated SVD at the largest
size the boundary accepts (4096 x 4096) with an exactly known spectrum.
Bars as in the TEBD tests: |Delta <S^z_i>| <= 1e-6 and 1 - overlap <= 1e-9 for
complex128 chains; the known-spectrum SVD to the truncation test's bars.
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


def _chain(spec, hb=None, dtype="c128"):
    from paper_1703_00387_amd import api, models
    hb = models.bond_hamiltonians(spec) if hb is None else hb
    return api.Chain.product(W.initial_vectors(spec), spec.chi_max, hb, dtype=dtype)


def _vector(chain):
    B, lam, chi = chain.to_host()
    v = lam[0][:, None] * B[0].reshape(B[0].shape[0], -1)
    v = v.reshape(-1, B[0].shape[2])
    for T in B[1:]:
        v = (v @ T.reshape(T.shape[0], -1)).reshape(-1, T.shape[2])
    return v.reshape(-1)


def _overlap_err(a, b):
    return 1.0 - abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))


@pytest.mark.parametrize("method,order", [("tebd2", 2), ("tebd4", 4), ("sweep", 0)])
def test_single_bond_chain(H, method, order):
    """L = 2: every layer is the one bond (or empty for even bonds)."""
    from oracle import mps as omps
    from paper_1703_00387_amd import api
    spec = W.xxz_chain(2, 4, 1.0, 0.5, init="random_product", local_states=W.random_complex((2, 2), (91,)))
    ref = omps.tebd_run(spec, method, 0.1, 7, 1e-12)
    ch = _chain(spec)
    api.tebd_step(H, [ch], order, 0.1, 7, 1e-12)
    assert _overlap_err(_vector(ch), omps.to_vector(ref)) <= 1e-12


def test_single_bond_chain_krylov(H):
    from oracle import ktebd, mps as omps
    from paper_1703_00387_amd import api
    spec = W.tfim_chain(2, 4, 1.0, 1.3)
    ref = ktebd.ktebd_run(spec, 0.1, 5, 1e-12, n_max=3, tol=1e-14)
    ch = _chain(spec)
    api.ktebd_step(H, [ch], 0.1, 5, 1e-12, 3, 1e-14)
    code, word = H.device_status()        # three vectors never meet tol = 1e-14 here
    assert word & ~0x2 == 0, word
    assert _overlap_err(_vector(ch), omps.to_vector(ref)) <= 1e-12


def test_chi_max_one(H):
    """Every update keeps one Schmidt value (the state stays a product)."""
    from oracle import mps as omps, models as om
    from paper_1703_00387_amd import api, models
    spec = W.xxz_chain(8, 1, 1.0, 0.5, init="random_product", local_states=W.random_complex((8, 2), (92,)))
    ref = omps.tebd_run(spec, "tebd2", 0.05, 10, 1e-12)
    ch = _chain(spec)
    api.tebd_step(H, [ch], 2, 0.05, 10, 1e-12)
    assert int(ch.chi.max().item()) == 1
    site, _, _ = api.observe(H, ch, models.sz_operator())
    assert np.abs(site.cpu().numpy() - omps.local_expect(ref, 0.5 * om.SZ)).max() <= 1e-9
    assert abs(float(ch.disc.sum().item()) - sum(ref.disc)) <= 1e-12 + 1e-6 * sum(ref.disc)


def test_zero_steps_leave_the_chain_unchanged(H):
    from paper_1703_00387_amd import api
    spec = W.xxz_chain(10, 16, 1.0, 0.5)
    ch = _chain(spec)
    api.tebd_step(H, [ch], 4, 0.05, 5, 1e-12)
    before = (ch.B.clone(), ch.lam.clone(), ch.chi.clone(), ch.disc.clone())
    api.tebd_step(H, [ch], 4, 0.05, 0, 1e-12)
    api.ktebd_step(H, [ch], 0.05, 0, 1e-12)
    for a, b in zip(before, (ch.B, ch.lam, ch.chi, ch.disc)):
        assert torch.equal(a, b)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_complex_bond_terms_tebd(H, dtype):
    """Random complex Hermitian two-site terms tell G from its transpose in the
    fused gate epilogue."""
    from oracle import mps as omps
    from paper_1703_00387_amd import api, models
    spec = W.xxz_chain(9, 16, 1.0, 0.5, init="random_product", local_states=W.random_complex((9, 2), (93,)))
    hs = []
    for b in range(spec.L - 1):
        A = W.random_complex((4, 4), (94, b))
        hs.append(0.5 * (A + A.conj().T))
    psi = omps.product_mps(W.initial_vectors(spec))
    for _ in range(6):
        for bonds, tau in omps.strang_layers(spec.L, 0.05):
            for b in bonds:
                omps.apply_bond(psi, b, omps.gate(hs[b], tau), spec.chi_max, 1e-12)
    ch = _chain(spec, hs, dtype)
    api.tebd_step(H, [ch], 2, 0.05, 6, 1e-12)
    site, _, _ = api.observe(H, ch, models.sz_operator())
    from oracle import models as om
    d = np.abs(site.cpu().numpy() - omps.local_expect(psi, 0.5 * om.SZ)).max()
    assert d <= (1e-9 if dtype == "c128" else 2e-6), d
    if dtype == "c128":
        assert _overlap_err(_vector(ch), omps.to_vector(psi)) <= 1e-9


def test_capacity_limits(H):
    from paper_1703_00387_amd import api, _lib
    ch = _chain(W.xxz_chain(4, 4, 1.0, 0.5))
    ch.chi_max = 2049                                 # d * chi_max = 4098 > 4096: refused before any access
    with pytest.raises(_lib.MPSError) as e:
        api.tebd_step(H, [ch], 2, 0.05, 1, 1e-12)
    assert e.value.code == _lib.MPS_ERR_CAPACITY
    with pytest.raises(_lib.MPSError) as e:
        H.truncate(torch.zeros((4097, 4), dtype=torch.complex128, device="cuda"), 4, 1e-12)
    assert e.value.code == _lib.MPS_ERR_CAPACITY


def test_truncate_at_the_size_limit_with_known_spectrum(H):
    """A = R3 diag(s) R1 R2 with Householder reflectors R (unitary) has singular
    values exactly s; at 4096 x 4096 (the boundary's limit) the Jacobi runs
    with split rounds.  Kept values, count, discarded weight and the
    reconstruction error are checked against the exact spectrum."""
    n = 4096
    dev = "cuda"
    s = torch.exp(-0.004 * torch.arange(n, dtype=torch.float64, device=dev))
    s = s / torch.linalg.vector_norm(s)
    gen = np.random.default_rng(170300387 + 95)

    def refl(M, left):
        v = torch.from_numpy(gen.normal(size=n) + 1j * gen.normal(size=n)).to(dev)
        v = v / torch.linalg.vector_norm(v)
        if left:    # (I - 2 v v^dag) M
            return M - 2.0 * torch.outer(v, v.conj() @ M)
        return M - 2.0 * torch.outer(M @ v, v.conj())   # M (I - 2 v v^dag)

    H.device_status()                      # clear what earlier calls left
    A = torch.diag(s).to(torch.complex128)
    A = refl(refl(A, False), False)
    A = refl(A, True)
    chi, eps = 512, 1e-12
    U, S, Vh, k, disc, norm2 = H.truncate(A, chi, eps)
    code, word = H.device_status()
    assert code == 0, word
    s_np = s.cpu().numpy()
    s2 = s_np ** 2
    tail = np.cumsum(s2[::-1])[::-1]                  # tail[j] = sum_{i>=j} s_i^2
    k_ref = next(kk for kk in range(1, n + 1) if kk == n or tail[kk] <= eps * s2.sum())
    k_ref = min(k_ref, chi)
    assert k == k_ref
    Sg = S.cpu().numpy()
    assert np.abs(Sg ** 2 - s2[:k]).max() <= 1e-13
    assert abs(disc - s2[k:].sum()) <= 1e-12 + 1e-6 * s2[k:].sum()
    R = (U * S.to(torch.complex128)) @ Vh
    err2 = float(torch.linalg.vector_norm(A - R) ** 2)
    assert abs(err2 - s2[k:].sum()) <= 1e-12


def test_nonfinite_bond_in_a_batched_layer_is_flagged(H):
    """A NaN in one chain's tensor reaches the Jacobi preparation of its bond:
    the layer finishes (every kernel exits) and the device status says
    non-finite, while a second, finite chain in the same call still matches
    the oracle."""
    from oracle import mps as omps, models as om
    from paper_1703_00387_amd import api, models, _lib
    good = W.xxz_chain(10, 16, 1.0, 0.5, init="random_product", local_states=W.random_complex((10, 2), (96,)))
    ref = omps.tebd_run(good, "tebd2", 0.05, 4, 1e-12)
    bad = W.xxz_chain(10, 16, 1.0, 0.5)
    cg, cb = _chain(good), _chain(bad)
    cb.B[3].view(torch.float64)[0] = float("nan")
    H.device_status()
    api.tebd_step(H, [cb, cg], 2, 0.05, 4, 1e-12)
    code, word = H.device_status()
    assert code == _lib.MPS_ERR_NONFINITE and word & _lib.MPS_DEV_NONFINITE, (code, word)
    site, _, _ = api.observe(H, cg, models.sz_operator())
    assert np.abs(site.cpu().numpy() - omps.local_expect(ref, 0.5 * om.SZ)).max() <= 1e-9


def test_persistent_wait_timeout_reported_and_handle_recovers(H):
    """The persistent Jacobi's bounded waits, forced to run out from the host
    (option 10 = one poll; option 6 = 0, so that no round takes the column
    split and the batch runs in the persistent launch): the call returns, every
    workgroup having left; the status word carries MPS_DEV_SCHED_TIMEOUT,
    reported as MPS_ERR_NOCONV (MPS_ERR_NONFINITE where the incomplete
    rotations also left a non-finite value); with the options restored the same handle
    steps a fresh chain cleanly.  Chain: the canonical Bose-Hubbard state of
    the long-contraction test (a 125-row bond of four row blocks)."""
    from paper_1703_00387_amd import api, _lib
    from test_gpu_tebd import _canonical_bh_chain
    for opt, val in [(10, 0), (10, 2e8), (11, 1)]:   # out of range, and no option 11
        with pytest.raises(_lib.MPSError) as e:
            H.set_option(opt, val)
        assert e.value.code == _lib.MPS_ERR_INVALID
    H.device_status()
    H.set_option(6, 0)
    H.set_option(10, 1)
    try:
        _, ch, _, _ = _canonical_bh_chain("c128")
        api.tebd_step(H, [ch], 2, 0.05, 1, 1e-14)
        torch.cuda.synchronize()
        code, word = H.device_status()
    finally:
        H.set_option(10, 1e6)
        H.set_option(6, 32)
    print(f"[edge] forced wait timeout: code {code} word {word:#x}", flush=True)
    assert word & _lib.MPS_DEV_SCHED_TIMEOUT, word
    assert code in (_lib.MPS_ERR_NOCONV, _lib.MPS_ERR_NONFINITE), code   # the results are incomplete
    _, ch, _, _ = _canonical_bh_chain("c128")
    api.tebd_step(H, [ch], 2, 0.05, 1, 1e-14)
    torch.cuda.synchronize()
    code, word = H.device_status()
    assert code == 0 and word == 0, (code, word)
    _, lam, chi = ch.to_host()
    assert int(max(chi)) <= 128
    assert all(np.isfinite(l).all() for l in lam)
