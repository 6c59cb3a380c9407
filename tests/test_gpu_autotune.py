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
