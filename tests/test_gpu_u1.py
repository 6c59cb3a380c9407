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


def test_u1_truncate_at_the_size_limit_with_known_spectrum(H):
    """4096 x 4096 (the boundary's limit) with four charges interleaved over
    rows and columns (row r and column c carry r mod 4 and c mod 4): block q is
    R_q diag(s_q) R'_q with Householder reflectors, so the singular values are
    exactly the union of the s_q.  Kept values, their charges, the discarded
    weight, the block structure of U and Vh and the reconstruction error
    against the exact spectrum."""
    n, nq = 4096, 4
    nb = n // nq
    dev = "cuda"
    gen = np.random.default_rng(170300387 + 97)
    rates = [0.004, 0.005, 0.006, 0.007]
    s_blocks = [torch.exp(-rates[q] * torch.arange(nb, dtype=torch.float64, device=dev)) * (1.0 + 0.1 * q)
                for q in range(nq)]
    tot = torch.sqrt(sum((sq ** 2).sum() for sq in s_blocks))
    s_blocks = [sq / tot for sq in s_blocks]

    def refl(M, left):
        v = torch.from_numpy(gen.normal(size=nb) + 1j * gen.normal(size=nb)).to(dev)
        v = v / torch.linalg.vector_norm(v)
        if left:
            return M - 2.0 * torch.outer(v, v.conj() @ M)
        return M - 2.0 * torch.outer(M @ v, v.conj())

    A = torch.zeros((n, n), dtype=torch.complex128, device=dev)
    for q in range(nq):
        Bq = refl(refl(torch.diag(s_blocks[q]).to(torch.complex128), True), False)
        A[q::nq, q::nq] = Bq
    row_q = np.arange(n) % nq
    col_q = np.arange(n) % nq
    H.device_status()
    chi, eps = 256, 1e-12
    U, S, Vh, qo, k, disc, norm2 = H.truncate_u1(A, row_q, col_q, chi, eps)
    code, word = H.device_status()
    assert code == 0, word
    allv = np.concatenate([sq.cpu().numpy() for sq in s_blocks])
    owner = np.repeat(np.arange(nq), nb)
    order = np.argsort(-allv, kind="stable")
    s2 = allv[order] ** 2
    tail = np.cumsum(s2[::-1])[::-1]
    k_ref = min(chi, next(kk for kk in range(1, n + 1) if kk == n or tail[kk] <= eps * s2.sum()))
    print(f"4096 x 4096 U(1): k={k} (ref {k_ref}) disc={disc:.3e}")
    assert k == k_ref
    assert np.abs(S.cpu().numpy() ** 2 - s2[:k]).max() <= 1e-13
    assert np.array_equal(qo.cpu().numpy(), owner[order][:k])
    assert abs(disc - s2[k:].sum()) <= 1e-12 + 1e-6 * s2[k:].sum()
    Uc, Vc, qn = U.cpu().numpy(), Vh.cpu().numpy(), qo.cpu().numpy()
    assert np.all(Uc[row_q[:, None] != qn[None, :]] == 0)
    assert np.all(Vc[qn[:, None] != col_q[None, :]] == 0)
    R = (U * S.to(torch.complex128)) @ Vh
    err2 = float(torch.linalg.vector_norm(A - R) ** 2)
    assert abs(err2 - s2[k:].sum()) <= 1e-12
