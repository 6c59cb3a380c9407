"""The truncated SVD entry point that allocates nothing (mps_truncate_noalloc)
against mps_truncate on the same inputs, through the C ABI: two calls in a
row, the second with a smaller input, both equal to the allocating entry
point's results (same kernels and launch shapes, so the bar is identity of
k and agreement of every output to 1e-14), and no device memory taken by the
second call.  Sizes beyond the fixed scratch are refused."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _graded(m, n, key, decay):
    r = min(m, n)
    Uq, _ = np.linalg.qr(W.random_complex((m, r), key + (1,)))
    Vq, _ = np.linalg.qr(W.random_complex((n, r), key + (2,)))
    s = np.exp(-decay * np.arange(r))
    A = (Uq * s) @ Vq.conj().T
    return A / np.linalg.norm(A)


def _compare(a, b):
    Ua, Sa, Va, ka, da, na = a
    Ub, Sb, Vb, kb, db, nb = b
    assert ka == kb
    assert abs(da - db) <= 1e-14 and abs(na - nb) <= 1e-14
    for x, y in ((Ua, Ub), (Sa, Sb), (Va, Vb)):
        assert (x - y).abs().max().item() <= 1e-14


def test_noalloc_truncate_equals_truncate_twice():
    from paper_1703_00387_amd import api
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    h = api.Handle(0)
    try:
        cases = [(512, 512, 256, 1e-12, (71,)), (200, 136, 64, 1e-10, (72,))]
        mats = [torch.from_numpy(_graded(m, n, key, 0.05)).cuda() for m, n, _, _, key in cases]
        torch.cuda.synchronize()
        for (m, n, chi, eps, _), A in zip(cases, mats):
            print(f"[noalloc] m={m} n={n} chi={chi}", flush=True)
            free0 = torch.cuda.mem_get_info()[0]
            got = h.truncate(A, chi, eps, noalloc=True)
            torch.cuda.synchronize()
            free1 = torch.cuda.mem_get_info()[0]
            ref = h.truncate(A, chi, eps)
            torch.cuda.synchronize()
            code, word = h.device_status()
            assert code == 0, word
            _compare(got, ref)
            if m < 512:      # the second, smaller call: every module is loaded by now
                assert free1 == free0, (free0, free1)
            print(f"[noalloc] m={m} n={n}: k={got[3]} equal to mps_truncate", flush=True)
    finally:
        h.close()


def test_noalloc_truncate_refuses_sizes_beyond_its_scratch():
    from paper_1703_00387_amd import api, _lib
    h = api.Handle(0)
    try:
        A = torch.zeros((600, 8), dtype=torch.complex128, device="cuda")
        with pytest.raises(_lib.MPSError) as e:
            h.truncate(A, 4, 0.0, noalloc=True)
        assert e.value.code == _lib.MPS_ERR_CAPACITY
    finally:
        h.close()
