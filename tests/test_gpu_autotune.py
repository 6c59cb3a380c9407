"""The Jacobi autotuner: valid choices, the JSON cache, and unchanged results
(every candidate computes the same split to the truncation test's bars)."""
import json

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


@pytest.mark.parametrize("n_mats,m,n,n_cand", [(8, 64, 64, 12), (4, 256, 256, 6), (1, 512, 512, 6)])
def test_autotune_choices_and_cache(H, tmp_path, n_mats, m, n, n_cand):
    from paper_1703_00387_amd import api
    cache = str(tmp_path / "tune.json")
    r = api.autotune(H, n_mats, m, n, apply=True, cache=cache)
    print(f"[autotune] {n_mats} x {m}x{n}: threads {r['threads']} split_below {r['split_below']} "
          f"method {r['method']} times {r['times_ms']}")
    assert not r["cached"] and len(r["times_ms"]) == n_cand
    assert r["threads"] in (256, 512) and r["split_below"] in (0, 32, 128) and r["method"] in (0, 1)
    assert all(t > 0 for t in r["times_ms"])
    table = json.load(open(cache))
    assert len(table) == 1
    r2 = api.autotune(H, n_mats, m, n, apply=True, cache=cache)
    assert r2["cached"] and r2["threads"] == r["threads"] and r2["method"] == r["method"]
    # the tuned handle still splits to the oracle's bars
    from oracle import mps as omps
    A = W.random_complex((m, n), (97, m))
    A /= np.linalg.norm(A)
    U, S, Vh, k, disc, norm2 = H.truncate(torch.from_numpy(A).cuda(), min(m, n), 1e-12)
    Uo, so, Vho, wo, nko, sfull = omps.truncate(A, min(m, n), 1e-12)
    assert k == len(so)
    assert np.abs(S.cpu().numpy() ** 2 - so ** 2).max() <= 1e-13
    H.set_option(5, 512)
    H.set_option(6, 32)
    H.set_option(7, 0)


def _set_all_tiles(kind, cand):
    from paper_1703_00387_amd import api
    # one (M, N) per shape class: few tiles, tall, wide, square
    for dt in ("c64", "c128"):
        for M, N in ((16, 16), (1024, 128), (128, 1024), (512, 512)):
            api.gemm_tile(kind, dt, M, N, cand)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_gemm_tile_shapes_give_identical_results(H, dtype):
    """Every MFMA tile candidate sums each output element over K in the same
    order: the H_eff apply (strided GEMMs) and a batched TEBD run (write-back
    GEMMs) come out bit for bit the same under every candidate."""
    from paper_1703_00387_amd import api, models
    npdt = np.complex128 if dtype == "c128" else np.complex64
    chi, d, w = 150, 3, 4
    Lenv = torch.from_numpy(W.random_complex((chi, w, chi), (71,)).astype(npdt)).cuda()
    Wm = torch.from_numpy(W.random_complex((w, w, d, d), (72,)).astype(npdt)).cuda()
    Renv = torch.from_numpy(W.random_complex((chi, w, chi), (73,)).astype(npdt)).cuda()
    x = torch.from_numpy(W.random_complex((chi, d, d, chi), (74,)).astype(npdt)).cuda()
    specs = [W.xxz_chain(L, 48, 1.0, 0.5) for L in (12, 14)]
    ref_y, ref_chains = None, None
    try:
        for cand in range(6):
            _set_all_tiles(0, cand)
            _set_all_tiles(1, cand)
            print(f"[gemm tiles] {dtype} candidate {cand}", flush=True)
            y = api.heff_apply(H, Lenv, Wm, Wm, Renv, x)
            chains = [api.Chain.product(W.initial_vectors(sp), sp.chi_max, models.bond_hamiltonians(sp),
                                        dtype=dtype) for sp in specs]
            api.tebd_step(H, chains, 2, 0.05, 6, 1e-12)
            torch.cuda.synchronize()
            if ref_y is None:
                ref_y, ref_chains = y, chains
                continue
            assert torch.equal(y, ref_y), cand
            for a, b in zip(chains, ref_chains):
                assert torch.equal(a.chi, b.chi) and torch.equal(a.B, b.B) and torch.equal(a.lam, b.lam), cand
    finally:
        _set_all_tiles(0, 0)
        _set_all_tiles(1, 0)


@pytest.mark.parametrize("kind,dtype,batch,M,N,K", [(0, "c128", 1, 1280, 1280, 2560), (0, "c64", 1, 1024, 2048, 512),
                                                    (1, "c128", 32, 512, 256, 512), (1, "c64", 32, 512, 256, 512)])
def test_gemm_autotune(H, kind, dtype, batch, M, N, K):
    from paper_1703_00387_amd import api
    try:
        r = api.autotune_gemm(H, kind, dtype, M, N, K, batch=batch, apply=True)
        flops = 8.0 * batch * M * N * K
        rates = [flops / (t * 1e-3) / 1e12 for t in r["times_ms"]]
        print(f"[gemm tune] kind {kind} {dtype} {batch}x{M}x{N}x{K}: best {r['tiles'][r['best']]} "
              f"TFLOP/s {[round(x, 1) for x in rates]}", flush=True)
        assert len(r["times_ms"]) == 6 and all(t > 0 for t in r["times_ms"])
        assert 0 <= r["best"] < 6 and api.gemm_tile(kind, dtype, M, N) == r["best"]
        assert r["tiles"][0] == (64, 64)
    finally:
        api.gemm_tile(kind, dtype, M, N, 0)
