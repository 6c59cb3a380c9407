"""Pins of the oracle's gradients (reverse mode, ED adjoint, finite differences).

P8: reverse-mode TEBD2 gradient with the truncated-SVD backward agrees with
central finite differences (h=1e-5) and with the exact-diagonalisation
adjoint gradient of the untruncated Trotter circuit.  The truncated-SVD
backward itself agrees with PyTorch's own SVD backward on a
non-degenerate untruncated case with a gauge-invariant loss.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import grad


def test_truncsvd_backward_matches_torch_untruncated():
    rng = np.random.default_rng(0)
    A0 = rng.normal(size=(7, 5)) + 1j * rng.normal(size=(7, 5))
    M = torch.tensor(rng.normal(size=(7, 7)) + 1j * rng.normal(size=(7, 7)))
    N = torch.tensor(rng.normal(size=(5, 5)) + 1j * rng.normal(size=(5, 5)))

    def loss_from(U, s, Vh):
        # gauge invariant: depends on U diag(s) V^dag and on |U|, |V| products
        X = (U * s[None, :]) @ Vh
        return torch.real(torch.sum(X.conj() * (M[:, :7] @ X @ N))) + torch.sum(s ** 3)

    A = torch.tensor(A0, requires_grad=True)
    U, s, Vh = grad.TruncSVD.apply(A, 5, 0.0)
    loss_from(U, s, Vh).backward()
    g1 = A.grad.clone()
    A2 = torch.tensor(A0, requires_grad=True)
    U, s, Vh = torch.linalg.svd(A2, full_matrices=False)
    loss_from(U, s, Vh).backward()
    np.testing.assert_allclose(g1.numpy(), A2.grad.numpy(), atol=1e-10)


def test_truncsvd_backward_projector_terms_fd():
    # truncated, uses U and V separately (gauge-invariant via U_k U_k^dag A V_k V_k^dag)
    rng = np.random.default_rng(1)
    A0 = rng.normal(size=(6, 8)) + 1j * rng.normal(size=(6, 8))
    P = rng.normal(size=(6, 8)) + 1j * rng.normal(size=(6, 8))

    def f(Anp):
        A = torch.tensor(Anp)
        U, s, Vh = grad.TruncSVD.apply(A, 3, 0.0)
        Y = U @ U.conj().T @ A @ Vh.conj().T @ Vh
        return float(torch.real(torch.sum(Y * torch.tensor(P).conj())))

    A = torch.tensor(A0, requires_grad=True)
    U, s, Vh = grad.TruncSVD.apply(A, 3, 0.0)
    Y = U @ U.conj().T @ A @ Vh.conj().T @ Vh
    torch.real(torch.sum(Y * torch.tensor(P).conj())).backward()
    g = A.grad.numpy()
    h = 1e-6
    for (i, j) in [(0, 0), (2, 5), (5, 7), (3, 1)]:
        for unit in (1.0, 1j):
            E = np.zeros_like(A0)
            E[i, j] = unit * h
            fd = (f(A0 + E) - f(A0 - E)) / (2 * h)
            an = np.real(np.conj(g[i, j]) * unit)
            assert abs(fd - an) < 1e-6, (i, j, unit, fd, an)


@pytest.mark.parametrize("L,steps,chi", [(6, 10, 8), (8, 8, 6)])
def test_reverse_vs_fd_and_ed(L, steps, chi):
    spec = W.xxz_chain(L, chi, 1.0, 0.5, J_b=W.xxz_grad_couplings(L))
    loss, g_rev = grad.reverse_gradient(spec, 0.05, steps, chi, 1e-12)
    g_fd = grad.fd_gradient(spec, 0.05, steps, chi, 1e-12)
    assert np.linalg.norm(g_rev - g_fd) / np.linalg.norm(g_fd) < 1e-7
    if chi >= 2 ** (L // 2):
        loss_ed, g_ed = grad.ed_gradient(spec, 0.05, steps)
        assert abs(loss - loss_ed) < 1e-8
        assert np.linalg.norm(g_rev - g_ed) / np.linalg.norm(g_ed) < 1e-7


def test_reverse_tebd4_vs_fd_and_ed():
    """The reverse mode through a TEBD4 run (15 layers per step, four time-step
    classes) against central differences and the exact circuit's adjoint
    (nothing cut at chi = 8 on L = 6)."""
    spec = W.xxz_chain(6, 8, 1.0, 0.5, J_b=W.xxz_grad_couplings(6))
    loss, g_rev = grad.reverse_gradient(spec, 0.1, 3, 8, 1e-12, method="tebd4")
    g_fd = grad.fd_gradient(spec, 0.1, 3, 8, 1e-12, method="tebd4")
    assert np.linalg.norm(g_rev - g_fd) / np.linalg.norm(g_fd) < 1e-7
    loss_ed, g_ed = grad.ed_gradient(spec, 0.1, 3, method="tebd4")
    assert abs(loss - loss_ed) < 1e-8
    assert np.linalg.norm(g_rev - g_ed) / np.linalg.norm(g_ed) < 1e-7
    # and it is not the TEBD2 gradient of the same run
    _, g2 = grad.reverse_gradient(spec, 0.1, 3, 8, 1e-12, method="tebd2")
    assert np.linalg.norm(g2 - g_rev) / np.linalg.norm(g_rev) > 1e-6


def test_broadening_sensitivity_small():
    spec = W.xxz_chain(6, 8, 1.0, 0.5, J_b=W.xxz_grad_couplings(6))
    gs = [grad.reverse_gradient(spec, 0.05, 6, 8, 1e-12, eta=eta)[1] for eta in (1e-10, 1e-12, 1e-14)]
    for g in gs[1:]:
        assert np.linalg.norm(g - gs[0]) / np.linalg.norm(gs[0]) < 1e-6


def test_truncsvd_backward_all_cotangents_fd():
    # truncated (k = 3 of 5), m > n, a loss that uses U, s and Vh each on
    # their own (gauge invariant): every cotangent of the backward is exercised
    rng = np.random.default_rng(2)
    A0 = rng.normal(size=(9, 5)) + 1j * rng.normal(size=(9, 5))
    M = rng.normal(size=(9, 9)) + 1j * rng.normal(size=(9, 9))
    N = rng.normal(size=(5, 5)) + 1j * rng.normal(size=(5, 5))
    K = rng.normal(size=(9, 5)) + 1j * rng.normal(size=(9, 5))
    c = np.array([0.7, -1.3, 0.4])

    def loss(U, s, Vh):
        t = torch.tensor
        return (torch.real(torch.einsum("rj,rq,qj->", U.conj(), t(M), U))
                + torch.sum(s ** 3)
                + torch.real(torch.einsum("jc,cd,jd->", Vh, t(N), Vh.conj()))
                + torch.real(torch.sum(t(K).conj() * ((U * t(c)[None, :]) @ Vh))))

    def f(Anp):
        return float(loss(*grad.TruncSVD.apply(torch.tensor(Anp), 3, 0.0)))

    A = torch.tensor(A0, requires_grad=True)
    loss(*grad.TruncSVD.apply(A, 3, 0.0)).backward()
    g = A.grad.numpy()
    h = 1e-6
    for (i, j) in [(0, 0), (4, 2), (8, 4), (6, 1)]:
        for unit in (1.0, 1j):
            E = np.zeros_like(A0)
            E[i, j] = unit * h
            fd = (f(A0 + E) - f(A0 - E)) / (2 * h)
            an = np.real(np.conj(g[i, j]) * unit)
            assert abs(fd - an) < 1e-6 * max(1.0, abs(fd)), (i, j, unit, fd, an)


def test_theta_gate_vjp_fd():
    # the reverse mode of the theta' definition against central differences of
    # L = Re <W, theta'> in every input (real and imaginary directions)
    rng = np.random.default_rng(3)
    chl, d, chm, chr_ = 3, 2, 4, 2
    cplx = lambda *sh: rng.normal(size=sh) + 1j * rng.normal(size=sh)
    Bl, Br, G, Wt = cplx(chl, d, chm), cplx(chm, d, chr_), cplx(d * d, d * d), cplx(chl * d, d * chr_)
    lam = rng.uniform(0.2, 1.0, size=chl)
    got = grad.theta_gate_vjp(Bl, Br, lam, G, Wt)

    def f(args):
        tp = grad.theta_gate_torch(*[torch.tensor(a) for a in args]).numpy()
        return float(np.real(np.sum(np.conj(Wt) * tp)))

    base = [Bl, Br, lam, G]
    h = 1e-6
    for which, idx in [(0, (2, 1, 3)), (0, (0, 0, 0)), (1, (3, 1, 1)), (1, (1, 0, 0)), (2, (1,)), (3, (2, 1)),
                       (3, (0, 3))]:
        units = (1.0,) if which == 2 else (1.0, 1j)
        for unit in units:
            plus = [x.copy() for x in base]
            minus = [x.copy() for x in base]
            plus[which] = plus[which].astype(np.complex128 if which != 2 else np.float64)
            minus[which] = minus[which].astype(plus[which].dtype)
            plus[which][idx] += unit * h
            minus[which][idx] -= unit * h
            fd = (f(plus) - f(minus)) / (2 * h)
            an = np.real(np.conj(got[which][idx]) * unit)
            assert abs(fd - an) < 1e-7 * max(1.0, abs(fd)), (which, idx, unit, fd, an)
