"""Gradients of final-time observables with respect to per-bond couplings
(oracle, complex128).

Three independent routes:

(i)  reverse mode through the truncated TEBD2 run (PyTorch autograd on CPU in
     complex128) with a hand-written truncated-SVD backward: the full reduced
     SVD backward with the adjoints of the discarded singular triplets set to
     zero, so kept/discarded coupling terms are retained.  With the cotangent
     convention dL = Re tr(Xbar^dag dX), for A = U S V^dag (r = min(m,n)):
       Abar = U X V^dag + (1 - U U^dag) Ubar S^-1 V^dag + U S^-1 Vbar^dag (1 - V V^dag)
       X_ij = F_ij [ s_j (Ju - Ju^dag)_ij + s_i (Jv - Jv^dag)_ij ]   (i != j)
       X_ii = Sbar_i + i Im(Ju_ii - Jv_ii) / (2 s_i)                 (gauge term)
       Ju = U^dag Ubar,  Jv = V^dag Vbar,  F_ij = 1 / (s_j^2 - s_i^2)
     Lorentzian broadening: F_ij -> (s_j^2 - s_i^2) / ((s_j^2 - s_i^2)^2 + eta)
     and 1/s -> s / (s^2 + eta).  The derivation (from U^dag dA V) is in the
     design notes; finite differences and route (ii) pin it.
(ii) the adjoint-state gradient of the exact Trotter circuit (no truncation):
     dL/dJ_b = sum over occurrences of bond b of 2 Re <lambda| dG/dJ_b |psi_before>.
(iii) central finite differences of the complete oracle run.

For the XXZ chain the coupling J_b multiplies the whole bond term, so
G_b(tau) = exp(-i tau J_b h0_b) and dG/dJ_b = -i tau h0_b G_b.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import torch

from . import models, mps as omps, ed

torch.set_default_dtype(torch.float64)


class TruncSVD(torch.autograd.Function):
    @staticmethod
    def forward(ctx, A, k: int, eta: float):
        U, s, Vh = torch.linalg.svd(A, full_matrices=False)
        ctx.save_for_backward(U, s, Vh)
        ctx.k, ctx.eta = k, eta
        return U[:, :k].clone(), s[:k].clone(), Vh[:k].clone()

    @staticmethod
    def backward(ctx, gU, gs, gVh):
        U, s, Vh = ctx.saved_tensors
        k, eta = ctx.k, ctx.eta
        r = s.shape[0]
        m, n = U.shape[0], Vh.shape[1]
        V = Vh.conj().transpose(0, 1)
        Ub = torch.zeros_like(U)
        Vb = torch.zeros_like(V)
        Sb = torch.zeros(r, dtype=s.dtype)
        if gU is not None:
            Ub[:, :k] = gU
        if gVh is not None:
            Vb[:, :k] = gVh.conj().transpose(0, 1)
        if gs is not None:
            Sb[:k] = gs
        Ju = U.conj().transpose(0, 1) @ Ub
        Jv = V.conj().transpose(0, 1) @ Vb
        s2 = s * s
        D = s2[None, :] - s2[:, None]                 # D_ij = s_j^2 - s_i^2
        F = D / (D * D + eta)
        F.fill_diagonal_(0.0)
        Ku = Ju - Ju.conj().transpose(0, 1)
        Kv = Jv - Jv.conj().transpose(0, 1)
        X = F * (s[None, :] * Ku + s[:, None] * Kv)
        sinv = s / (s2 + eta)
        diag = Sb.to(X.dtype) + 1j * torch.imag(torch.diagonal(Ju) - torch.diagonal(Jv)) * sinv * 0.5
        X = X + torch.diag(diag)
        gA = U @ X @ Vh
        if m > r:
            gA = gA + (Ub - U @ (U.conj().transpose(0, 1) @ Ub)) * sinv[None, :] @ Vh
        if n > r:
            gA = gA + (U * sinv[None, :]) @ (Vb.conj().transpose(0, 1) - (Vb.conj().transpose(0, 1) @ V) @ Vh)
        return gA, None, None


def theta_gate_torch(Bl, Br, lam_l, G):
    """theta' of one two-site update (App. "Details of the Krylov method", the
    plain two-site update: contract the two sites over their shared bond, apply
    the two-site propagator to the physical pair; rows scaled by the left
    Schmidt values, Hastings form).  Bl [chl][d][chm], Br [chm][d][chr],
    lam_l [chl], G [d*d][d*d] with G[(s,t)][(u,v)] mapping (u,v) to (s,t);
    returns theta' [chl*d][d*chr]."""
    chl, d, _ = Bl.shape
    chr_ = Br.shape[2]
    th = torch.einsum("aub,bvc->auvc", Bl, Br).reshape(chl, d * d, chr_)
    thp = torch.einsum("xy,ayc->axc", G, th)
    return (lam_l.to(thp.dtype)[:, None, None] * thp).reshape(chl * d, d * chr_)


def theta_gate_vjp(Bl, Br, lam_l, G, theta_bar):
    """(dBl, dBr, dlam_l, dG) of theta_gate_torch for the cotangent theta_bar,
    with dL = Re sum conj(Xbar) dX (reverse mode of the definition above)."""
    xs = [torch.tensor(np.asarray(x), requires_grad=True) for x in (Bl, Br, lam_l, G)]
    tp = theta_gate_torch(*xs)
    torch.real(torch.sum(torch.tensor(np.asarray(theta_bar)).conj() * tp)).backward()
    return tuple(x.grad.numpy() for x in xs)


def _gate_factors(spec, b):
    e, V = np.linalg.eigh(models.xxz_unit_bond(spec, b))
    return torch.tensor(e), torch.tensor(V)


def torch_gate(e, V, Jb, tau):
    ph = torch.exp(-1j * tau * Jb * e)
    return (V * ph[None, :]) @ V.conj().transpose(0, 1)


def tebd2_state_torch(spec, J: torch.Tensor, dt: float, n_steps: int, chi_max: int, eps: float,
                      eta: float = 1e-12, method="tebd2"):
    """The final Hastings-form state (B, lam lists of tensors) of the truncated
    TEBD run, as a differentiable function of the per-bond couplings J."""
    from workloads import initial_vectors
    L, d = spec.L, spec.d
    psi0 = omps.product_mps(initial_vectors(spec))
    B = [torch.tensor(x) for x in psi0.B]
    lam = [torch.tensor(x) for x in psi0.lam]
    fac = [_gate_factors(spec, b) for b in range(L - 1)]
    layers = omps.step_layers(method, L, dt)
    for _ in range(n_steps):
        for bonds, tau in layers:
            for b in bonds:
                G = torch_gate(*fac[b], J[b], tau).reshape(d, d, d, d)
                th = torch.einsum("asb,btc->astc", B[b], B[b + 1])
                thp = torch.einsum("uvst,astc->auvc", G, th)
                chl, chr_ = thp.shape[0], thp.shape[3]
                mat = (lam[b].to(thp.dtype)[:, None, None, None] * thp).reshape(chl * d, d * chr_)
                with torch.no_grad():
                    s_all = torch.linalg.svdvals(mat)
                k = omps.count_rule(s_all.numpy(), chi_max, eps)
                U, s, Vh = TruncSVD.apply(mat, k, eta)
                nk = torch.sqrt(torch.sum(s * s))
                lam[b + 1] = s / nk
                B[b + 1] = Vh.reshape(k, d, chr_)
                B[b] = (thp.reshape(chl * d, d * chr_) @ Vh.conj().transpose(0, 1) / nk).reshape(chl, d, k)
    return B, lam


def site_expect_torch(B, lam, op: np.ndarray, i: int):
    """<op at site i> = sum_a lam_i[a]^2 <B_i[a]| op |B_i[a]> of a Hastings-form state."""
    Bi = B[i]
    l2 = (lam[i] ** 2).to(Bi.dtype)
    return torch.real(torch.einsum("a,asc,st,atc->", l2, Bi.conj(), torch.tensor(op), Bi))


def tebd2_loss_torch(spec, J: torch.Tensor, dt: float, n_steps: int, chi_max: int, eps: float,
                     eta: float = 1e-12, site=None, method="tebd2"):
    """Loss <S^z_site>(T) + sum_b <S^z_b S^z_{b+1}>(T) of the truncated TEBD
    run, as a differentiable function of the per-bond couplings J."""
    L, d = spec.L, spec.d
    site = L // 2 - 1 if site is None else site
    B, lam = tebd2_state_torch(spec, J, dt, n_steps, chi_max, eps, eta, method)
    sz = torch.tensor(0.5 * models.SZ)
    Bi = B[site]
    l2 = (lam[site] ** 2).to(Bi.dtype)
    loss = torch.real(torch.einsum("a,asc,st,atc->", l2, Bi.conj(), sz, Bi))
    szsz = torch.kron(sz, sz).reshape(d, d, d, d)
    for b in range(L - 1):
        th = lam[b].to(Bi.dtype)[:, None, None, None] * torch.einsum("asb,btc->astc", B[b], B[b + 1])
        loss = loss + torch.real(torch.einsum("auvc,uvst,astc->", th.conj(), szsz, th))
    return loss


def reverse_gradient(spec, dt, n_steps, chi_max, eps, eta=1e-12, method="tebd2"):
    J = torch.tensor(np.asarray(spec.J_b, dtype=np.float64), requires_grad=True)
    loss = tebd2_loss_torch(spec, J, dt, n_steps, chi_max, eps, eta, method=method)
    loss.backward()
    return float(loss.detach()), J.grad.numpy().copy()


def oracle_loss(spec, J, dt, n_steps, chi_max, eps, method="tebd2"):
    """Plain NumPy forward of the same loss (no autograd), for differences."""
    import copy
    sp = copy.copy(spec)
    sp.J_b = np.asarray(J, dtype=np.float64)
    psi = omps.tebd_run(sp, method, dt, n_steps, eps, chi_max)
    L = sp.L
    site = L // 2 - 1
    return float(omps.local_expect(psi, 0.5 * models.SZ)[site] + omps.szsz(psi).sum())


def fd_gradient(spec, dt, n_steps, chi_max, eps, h=1e-5, bonds=None, method="tebd2"):
    J0 = np.asarray(spec.J_b, dtype=np.float64)
    bonds = range(len(J0)) if bonds is None else bonds
    g = np.zeros(len(J0))
    for b in bonds:
        Jp, Jm = J0.copy(), J0.copy()
        Jp[b] += h
        Jm[b] -= h
        g[b] = (oracle_loss(spec, Jp, dt, n_steps, chi_max, eps, method)
                - oracle_loss(spec, Jm, dt, n_steps, chi_max, eps, method)) / (2 * h)
    return g


def ed_gradient(spec, dt, n_steps, method="tebd2"):
    """Adjoint-state gradient of the exact Trotter circuit (no truncation)."""
    from workloads import initial_vectors
    L, d = spec.L, spec.d
    psi = ed.product_vector(initial_vectors(spec))
    # the circuit's own schedule and Pade exponentials: nothing shared with
    # the MPS run whose gradient this checks
    seq = ed.circuit_schedule(method, L, dt) * n_steps
    h0 = [models.xxz_unit_bond(spec, b) for b in range(L - 1)]
    G = {}
    for b, tau in seq:
        if (b, tau) not in G:
            G[(b, tau)] = scipy.linalg.expm(-1j * tau * spec.J_b[b] * h0[b])
    for b, tau in seq:
        psi = ed.apply_two_site(psi, G[(b, tau)], b, L, d)
    site = L // 2 - 1
    O = models.embed_one_site(0.5 * models.SZ, site, L, d)
    zz = np.kron(0.5 * models.SZ, 0.5 * models.SZ)
    for b in range(L - 1):
        O = O + models.embed_two_site(zz, b, L, d)
    loss = float(np.real(np.vdot(psi, O @ psi)))
    lam = O @ psi
    grad = np.zeros(L - 1)
    for b, tau in reversed(seq):
        Gb = G[(b, tau)]
        psi = ed.apply_two_site(psi, Gb.conj().T, b, L, d)
        dG = -1j * tau * h0[b] @ Gb
        grad[b] += 2.0 * np.real(np.vdot(lam, ed.apply_two_site(psi, dG, b, L, d)))
        lam = ed.apply_two_site(lam, Gb.conj().T, b, L, d)
    return loss, grad
