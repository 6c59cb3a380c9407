"""U(1)-symmetric truncated SVD on the GPU (mps_truncate_u1) against the
oracle's blockwise SVD (oracle/u1.py), at the bars of the dense truncation
test: squared singular values within 1e-13 |theta|^2, the kept count and the
charges of the kept vectors identical, discarded weight within
1e-12 + 1e-6 w, the truncated theta within 1e-12 + k 1e-14 / s_k (the
Jacobi's vector accuracy for small kept values), and U, Vh exactly zero off
their charge blocks.
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


def _block_theta(seed, row_q, col_q, grade):
    rng = np.random.default_rng(170300387 + seed)
    m, n = len(row_q), len(col_q)
    T = rng.normal(size=(m, n)) + 1j * rng.normal(size=(m, n))
    T[np.asarray(row_q)[:, None] != np.asarray(col_q)[None, :]] = 0.0
    T *= np.exp(-grade * np.arange(m))[:, None]
    return T / np.linalg.norm(T)


def _check(H, T, row_q, col_q, chi, eps):
    from oracle import u1
    Ug, Sg, Vg, qg, k, disc, norm2 = H.truncate_u1(torch.from_numpy(T).cuda(), row_q, col_q, chi, eps)
    Uo, so, Vo, qo, wo, nko, s_all = u1.truncate_u1(T, row_q, col_q, chi, eps)
    Ug, Sg, Vg, qg = Ug.cpu().numpy(), Sg.cpu().numpy(), Vg.cpu().numpy(), qg.cpu().numpy()
    print(f"m={T.shape[0]} n={T.shape[1]} k={k}/{len(so)} max|ds2|={np.abs(Sg ** 2 - so ** 2).max():.2e}")
    assert k == len(so)
    assert np.abs(Sg ** 2 - so ** 2).max() <= 1e-13
    assert np.array_equal(qg, qo)
    assert abs(disc - wo) <= 1e-12 + 1e-6 * wo
    assert abs(norm2 - 1.0) < 1e-12
    # kept rows of V^dag are orthogonal to 1e-10 + 1e-14 |theta|^2 / (s_p s_q)
    # (the Jacobi's accuracy contract), so the term s_j u_j v_j^dag of a small
    # kept value is fixed to about 1e-14 / s_k
    bar = 1e-12 + len(so) * 1e-14 / so[-1]
    assert np.abs((Ug * Sg) @ Vg - (Uo * so) @ Vo).max() <= bar
    rq, cq = np.asarray(row_q), np.asarray(col_q)
    assert np.all(Ug[rq[:, None] != qg[None, :]] == 0)
    assert np.all(Vg[qg[:, None] != cq[None, :]] == 0)


@pytest.mark.parametrize("seed,m,n,qr,chi,eps,grade", [
    (1, 40, 30, (-3, 4), 12, 1e-6, 0.15),
    (2, 130, 70, (-2, 3), 50, 1e-12, 0.08),
    (3, 512, 512, (-6, 7), 256, 1e-12, 0.02),     # 13 sectors, blocks of about 40 rows
    (4, 1024, 1024, (-2, 3), 300, 1e-12, 0.01),   # 5 sectors of about 200 rows: round-based sweeps
    (5, 9, 300, (0, 3), 9, 0.0, 0.0),
])
def test_random_blocks_match_oracle(H, seed, m, n, qr, chi, eps, grade):
    rng = np.random.default_rng(seed)
    row_q = rng.integers(qr[0], qr[1], size=m)
    col_q = rng.integers(qr[0], qr[1], size=n)
    _check(H, _block_theta(seed, row_q, col_q, grade), row_q, col_q, chi, eps)


def test_neel_state_cut(H):
    """The exactly evolved Neel state of an XXZ chain, cut after 5 of 10 sites:
    left charge = up spins on the left, right charge = total - up spins on the
    right."""
    from oracle import ed, models as om
    L, d, cut = 10, 2, 5
    spec = W.xxz_chain(L, 32, 1.0, 0.5)
    psi = ed.exact_evolve(om.dense_hamiltonian(spec), ed.product_vector(W.initial_vectors(spec)), 1.3)
    theta = psi.reshape(d ** cut, d ** (L - cut))

    def ups(idx, nsites):
        return sum(1 for i in range(nsites) if (idx // d ** (nsites - 1 - i)) % d == 0)
    qL = [ups(r, cut) for r in range(d ** cut)]
    qR = [L // 2 - ups(c, L - cut) for c in range(d ** (L - cut))]
    _check(H, theta, qL, qR, 20, 1e-10)


def test_no_shared_charge_is_an_error(H):
    from paper_1703_00387_amd import _lib
    T = torch.zeros((4, 4), dtype=torch.complex128, device="cuda")
    with pytest.raises(_lib.MPSError) as e:
        H.truncate_u1(T, [0, 0, 1, 1], [2, 2, 3, 3], 4, 1e-12)
    assert e.value.code == _lib.MPS_ERR_SHAPE
