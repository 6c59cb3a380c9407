"""GPU tests of the boundary's workspace, record and adjoint entry points,
through the C ABI.

* A handle on a caller-owned workspace (mps_create_ws) sized by
  mps_workspace_size gives bit-identical TEBD results to a handle that owns
  its workspace, takes no device memory during the calls, and a workspace
  that is too small is refused with MPS_ERR_CAPACITY.
* The per-update discarded-weight log of mps_tebd_step_ex equals the oracle's
  discarded weight of every update in order (R10: |dw| <= 1e-12 + 1e-6 w),
  adds up to the chains' per-bond accumulators, and a captured step logs the
  same as the eager one.
* mps_theta_gate_vjp and mps_truncate_vjp (the two pieces of one update's
  reverse pass) against the oracle's reverse mode of the theta' definition
  (1e-13 of the largest entry) and its truncated-SVD backward (1e-10
  relative), the latter with the cotangents of a gauge-invariant loss of
  (U, S, Vh) taken by each side in its own gauge.
* mps_tebd_step_vjp after a checkpointed batched TEBD2 run: for state
  cotangents built from a weighted sum of <S^z_i> of each chain's final
  state, dL/dJ equals the oracle's reverse-mode gradient of that loss
  (1e-6 relative) and the single-chain adjoint mps_tebd_vjp (1e-10 relative);
  api.TebdStep gives the same gradient through torch.autograd for a loss
  that torch computes from the final states.
"""
import copy

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


def _chain(spec, dtype="c128"):
    from paper_1703_00387_amd import api, models
    return api.Chain.product(W.initial_vectors(spec), spec.chi_max, models.bond_hamiltonians(spec), dtype=dtype)


def _batch_specs(n, L0, chi):
    wl = W.xxz_batch256(n_chains=n)
    return [W.xxz_chain(L0 + 2 * i, chi, 1.0, 0.5, None, c.Jz_b[:L0 + 2 * i - 1], "random_product",
                        c.local_states[:L0 + 2 * i]) for i, c in enumerate(wl.chains)]


def test_caller_owned_workspace(H):
    from paper_1703_00387_amd import api, _lib
    specs = _batch_specs(3, 12, 32)
    need = api.workspace_size(_lib.MPS_OP_TEBD, "c128", 3, 16, 2, 32)
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    hw = api.Handle(0, workspace=ws)
    try:
        a = [_chain(sp) for sp in specs]
        b = [_chain(sp) for sp in specs]
        print(f"[boundary] caller workspace {need} bytes", flush=True)
        api.tebd_step(hw, a, 4, 0.05, 2, 1e-12)          # loads every module once
        api.tebd_step(H, b, 4, 0.05, 2, 1e-12)
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        api.tebd_step(hw, a, 4, 0.05, 3, 1e-12)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        api.tebd_step(H, b, 4, 0.05, 3, 1e-12)
        torch.cuda.synchronize()
        assert free1 == free0, (free0, free1)
        for x, y in zip(a, b):
            assert torch.equal(x.chi, y.chi) and torch.equal(x.B, y.B) and torch.equal(x.lam, y.lam)
        assert 0 < hw.workspace_needed() <= need
        # a single large matrix: the column split keeps its partial Grams behind the plan
        A = torch.from_numpy(W.random_complex((256, 256), (81,))).cuda()
        r1 = hw.truncate(A, 64, 1e-12)
        r2 = H.truncate(A, 64, 1e-12)
        assert r1[3] == r2[3] and (r1[1] - r2[1]).abs().max().item() <= 1e-14
    finally:
        hw.close()
    small = torch.empty(4096, dtype=torch.uint8, device="cuda")
    hs = api.Handle(0, workspace=small)
    try:
        c = [_chain(specs[0])]
        with pytest.raises(_lib.MPSError) as e:
            api.tebd_step(hs, c, 2, 0.05, 1, 1e-12)
        assert e.value.code == _lib.MPS_ERR_CAPACITY
        assert hs.workspace_needed() > 4096
    finally:
        hs.close()


@pytest.mark.parametrize("order,method", [(2, "tebd2"), (4, "tebd4")])
def test_disc_log_matches_oracle(H, order, method):
    from oracle import mps as omps
    from paper_1703_00387_amd import api
    specs = _batch_specs(2, 8, 2)     # chi_max = 2: the cap cuts
    n_steps, dt, eps = 4, 0.1, 1e-10
    n_layers = 3 if order == 2 else 15
    l_max = max(sp.L for sp in specs)
    chains = [_chain(sp) for sp in specs]
    log = torch.zeros((n_steps, n_layers, len(chains), l_max - 1), dtype=torch.float64, device="cuda")
    print(f"[boundary] disc log order {order}", flush=True)
    api.tebd_step_ex(H, chains, order, dt, n_steps, eps, disc_log=log)
    torch.cuda.synchronize()
    code, word = H.device_status()
    assert code == 0, word
    lg = log.cpu().numpy()
    for c, (sp, ch) in enumerate(zip(specs, chains)):
        ref = omps.tebd_run(sp, method, dt, n_steps, eps)
        got = []
        layers = omps.step_layers(method, sp.L, dt)
        for st in range(n_steps):
            for li, (bonds, _) in enumerate(layers):
                got += [lg[st, li, c, b] for b in bonds]
        got, want = np.array(got), np.array(ref.disc)
        assert len(got) == len(want)
        assert (np.abs(got - want) <= 1e-12 + 1e-6 * want).all(), np.abs(got - want).max()
        assert want.max() > 1e-6                  # the cap cut
        acc = ch.disc.cpu().numpy()
        np.testing.assert_allclose(lg[:, :, c, :sp.L - 1].sum(axis=(0, 1)), acc, rtol=1e-12, atol=1e-18)
    # the captured step logs the same
    g = [_chain(sp) for sp in specs]
    log2 = torch.zeros_like(log)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        api.tebd_step_ex(H, g, order, dt, n_steps, eps, flags=0x1, disc_log=log2)
    s.synchronize()
    assert torch.equal(log, log2)


def test_checkpointed_vjp_matches_oracle_and_single_chain(H):
    from oracle import grad, models as om
    from paper_1703_00387_amd import api, _lib, models
    dt, n_steps, chi, eps = 0.05, 6, 8, 1e-12
    specs = []
    for L in (6, 8):
        sp = W.xxz_chain(L, chi, 1.0, 0.5, J_b=W.xxz_grad_couplings(L))
        specs.append(sp)
    h0s = []
    for sp in specs:
        unit = copy.copy(sp)
        unit.J_b = np.ones(sp.L - 1)
        h0s.append(torch.from_numpy(np.ascontiguousarray(models.bond_hamiltonians(unit))).cuda())
    chains = [_chain(sp) for sp in specs]
    ck = torch.zeros(api.tebd_ckpt_bytes(chains, n_steps), dtype=torch.uint8, device="cuda")
    print("[boundary] checkpointed forward", flush=True)
    api.tebd_step_ex(H, chains, 2, dt, n_steps, eps, flags=_lib.MPS_FLAG_CHECKPOINT, ckpt=ck)
    torch.cuda.synchronize()
    # cotangents of L = sum_i w_i <S^z_i> at the final state (dL = Re<dB, dB'> + <dlam, dlam'>):
    # dB_i = 2 w_i lam_i^2 (S^z B_i), dlam_i[a] = 2 w_i lam_i[a] Re<B_i[a], S^z B_i[a]>
    sz = 0.5 * om.SZ
    weights, dBs, dls = [], [], []
    for c, (sp, ch) in enumerate(zip(specs, chains)):
        w = W.random_real((sp.L,), (91, c), -1.0, 1.0)
        weights.append(w)
        B = ch.B.cpu().numpy()
        lam = ch.lam.cpu().numpy()
        chis = ch.chi.cpu().numpy()
        dB = np.zeros_like(B)
        dl = np.zeros_like(lam)
        for i in range(sp.L):
            a, r = chis[i], chis[i + 1]
            Bi = B[i, :a, :, :r]
            OB = np.einsum("st,atc->asc", sz, Bi)
            l = lam[i, :a]
            dB[i, :a, :, :r] = 2 * w[i] * (l ** 2)[:, None, None] * OB
            dl[i, :a] += 2 * w[i] * l * np.real(np.einsum("asc,asc->a", Bi.conj(), OB))
        dBs.append(torch.from_numpy(dB).cuda())
        dls.append(torch.from_numpy(dl).cuda())
    print("[boundary] tebd_step_vjp", flush=True)
    dJ = api.tebd_step_vjp(H, chains, h0s, ck, dBs, dls, eta=1e-12).cpu().numpy()
    code, word = H.device_status()
    assert code == 0, word
    for c, sp in enumerate(specs):
        # oracle: reverse mode through the same truncated run, loss from its own final state
        J = torch.tensor(np.asarray(sp.J_b, dtype=np.float64), requires_grad=True)
        Bt, lt = grad.tebd2_state_torch(sp, J, dt, n_steps, chi, eps, 1e-12)
        loss = sum(weights[c][i] * grad.site_expect_torch(Bt, lt, sz, i) for i in range(sp.L))
        loss.backward()
        g_or = J.grad.numpy()
        rel = np.linalg.norm(dJ[c, :sp.L - 1] - g_or) / np.linalg.norm(g_or)
        # the single-chain adjoint with the same weights
        one = _chain(sp)
        _, dJ1 = api.tebd_vjp(H, one, h0s[c], dt, n_steps, eps, models.sz_operator(),
                              np.kron(models.sz_operator(), models.sz_operator()), weights[c], np.zeros(sp.L - 1))
        dJ1 = dJ1.cpu().numpy()
        rel1 = np.linalg.norm(dJ[c, :sp.L - 1] - dJ1) / np.linalg.norm(dJ1)
        print(f"[boundary] chain L={sp.L}: rel vs oracle {rel:.2e}, vs single-chain adjoint {rel1:.2e}", flush=True)
        assert rel <= 1e-6 and rel1 <= 1e-10
        assert np.all(dJ[c, sp.L - 1:] == 0.0)


def test_checkpointed_vjp_tebd4_matches_oracle(H):
    """mps_tebd_step_vjp after a checkpointed batched TEBD4 run (15 layers a
    step) against the oracle's reverse mode through its own TEBD4 run, for
    L = sum_i w_i <S^z_i> of the final states; chi_max = 4 cuts on L = 8.
    Also api.TebdStep with order 4 under torch.autograd."""
    from oracle import grad, models as om
    from paper_1703_00387_amd import api, _lib, models
    dt, n_steps, eps = 0.1, 3, 1e-12
    specs = [W.xxz_chain(L, chi, 1.0, 0.5, J_b=W.xxz_grad_couplings(L)) for L, chi in ((6, 8), (8, 4))]
    h0s = []
    for sp in specs:
        unit = copy.copy(sp)
        unit.J_b = np.ones(sp.L - 1)
        h0s.append(torch.from_numpy(np.ascontiguousarray(models.bond_hamiltonians(unit))).cuda())
    chains = [_chain(sp) for sp in specs]
    ck = torch.zeros(api.tebd_ckpt_bytes(chains, n_steps), dtype=torch.uint8, device="cuda")
    print("[boundary] checkpointed TEBD4 forward", flush=True)
    api.tebd_step_ex(H, chains, 4, dt, n_steps, eps, flags=_lib.MPS_FLAG_CHECKPOINT, ckpt=ck)
    torch.cuda.synchronize()
    sz = 0.5 * om.SZ
    weights, dBs, dls = [], [], []
    for c, (sp, ch) in enumerate(zip(specs, chains)):
        w = W.random_real((sp.L,), (95, c), -1.0, 1.0)
        weights.append(w)
        B, lam, chis = ch.B.cpu().numpy(), ch.lam.cpu().numpy(), ch.chi.cpu().numpy()
        dB, dl = np.zeros_like(B), np.zeros_like(lam)
        for i in range(sp.L):
            a, r = chis[i], chis[i + 1]
            Bi = B[i, :a, :, :r]
            OB = np.einsum("st,atc->asc", sz, Bi)
            l = lam[i, :a]
            dB[i, :a, :, :r] = 2 * w[i] * (l ** 2)[:, None, None] * OB
            dl[i, :a] += 2 * w[i] * l * np.real(np.einsum("asc,asc->a", Bi.conj(), OB))
        dBs.append(torch.from_numpy(dB).cuda())
        dls.append(torch.from_numpy(dl).cuda())
    print("[boundary] tebd_step_vjp TEBD4", flush=True)
    dJ = api.tebd_step_vjp(H, chains, h0s, ck, dBs, dls, eta=1e-12).cpu().numpy()
    code, word = H.device_status()
    assert code == 0, word
    refs = []
    for c, sp in enumerate(specs):
        J = torch.tensor(np.asarray(sp.J_b, dtype=np.float64), requires_grad=True)
        Bt, lt = grad.tebd2_state_torch(sp, J, dt, n_steps, sp.chi_max, eps, 1e-12, method="tebd4")
        loss = sum(weights[c][i] * grad.site_expect_torch(Bt, lt, sz, i) for i in range(sp.L))
        loss.backward()
        g_or = J.grad.numpy()
        refs.append(g_or)
        rel = np.linalg.norm(dJ[c, :sp.L - 1] - g_or) / np.linalg.norm(g_or)
        print(f"[boundary] TEBD4 chain L={sp.L} chi={sp.chi_max}: rel vs oracle {rel:.2e}", flush=True)
        assert rel <= 1e-6
        assert np.all(dJ[c, sp.L - 1:] == 0.0)
    # the same through the autograd Function with order 4
    Jn = np.zeros((2, 7))
    for c, sp in enumerate(specs):
        Jn[c, :sp.L - 1] = sp.J_b
    Jt = torch.tensor(Jn, device="cuda", requires_grad=True)
    szt = torch.from_numpy(sz.astype(np.complex128)).cuda()
    outs = []
    for c, sp in enumerate(specs):
        o = api.TebdStep.apply(Jt[c:c + 1], H, [W.initial_vectors(sp)], sp.chi_max, [h0s[c].cpu().numpy()], dt,
                               n_steps, eps, 1e-12, 4)
        outs.append(o)
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    for c, sp in enumerate(specs):
        B, lam, chis = outs[c][0], outs[c][1], outs[c][2].cpu().numpy()
        for i in range(sp.L):
            a, r = int(chis[i]), int(chis[i + 1])
            Bi = B[i, :a, :, :r]
            OB = torch.einsum("st,atc->asc", szt.to(Bi.dtype), Bi)
            loss = loss + weights[c][i] * torch.sum(lam[i, :a] ** 2 * torch.real(torch.einsum("asc,asc->a",
                                                                                              Bi.conj(), OB)))
    loss.backward()
    g = Jt.grad.cpu().numpy()
    for c, sp in enumerate(specs):
        rel = np.linalg.norm(g[c, :sp.L - 1] - refs[c]) / np.linalg.norm(refs[c])
        print(f"[boundary] TebdStep order 4 chain L={sp.L}: rel {rel:.2e}", flush=True)
        assert rel <= 1e-6


def _unitary(n, seed):
    q, _ = np.linalg.qr(W.random_complex((n, n), seed))
    return q


@pytest.mark.parametrize("chl,d,chm,chr_", [(37, 2, 50, 29), (8, 3, 21, 13), (64, 2, 128, 64)])
def test_theta_gate_vjp_matches_oracle(H, chl, d, chm, chr_):
    from oracle import grad
    from paper_1703_00387_amd import api
    seed = (101, chl, d, chm)
    Bl = W.random_complex((chl, d, chm), seed + (0,))
    Br = W.random_complex((chm, d, chr_), seed + (1,))
    G = W.random_complex((d * d, d * d), seed + (2,))
    tb = W.random_complex((chl * d, d * chr_), seed + (3,))
    lam = W.random_real((chl,), seed + (4,), 0.1, 1.0)
    want = grad.theta_gate_vjp(Bl, Br, lam, G, tb)
    cu = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
    print(f"[boundary] theta_gate_vjp {chl}x{d}x{chm}x{chr_}", flush=True)
    got = api.theta_gate_vjp(H, cu(Bl), cu(Br), cu(lam), cu(G), cu(tb))
    torch.cuda.synchronize()
    for name, g, w in zip(("dBl", "dBr", "dlam", "dG"), got, want):
        g = g.cpu().numpy()
        err = np.abs(g - w).max() / np.abs(w).max()
        assert err <= 1e-13, (name, err)


def _spectral(m, n, s, seed):
    r = len(s)
    return (_unitary(m, seed + (0,))[:, :r] * s[None, :]) @ _unitary(n, seed + (1,))[:r, :]


@pytest.mark.parametrize("m,n,k,cots,eta", [(96, 64, 20, "usv", 0.0), (64, 150, 30, "usv", 0.0),
                                            (130, 130, 130, "usv", 0.0), (200, 120, 1, "usv", 0.0),
                                            (160, 96, 40, "sv", 1e-12), (80, 200, 24, "v", 0.0)])
def test_truncate_vjp_matches_oracle(H, m, n, k, cots, eta):
    """mps_truncate_vjp against the oracle's truncated-SVD backward, each side
    taking the cotangents of one gauge-invariant loss in its own gauge."""
    from oracle import grad
    from paper_1703_00387_amd import api
    seed = (111, m, n, k)
    r = min(m, n)
    s = np.geomspace(1.0, 1e-2, r)          # gaps s_i^2 - s_{i+1}^2 >= 0.07 s_i^2
    A0 = _spectral(m, n, s, seed)
    M = W.random_complex((m, m), seed + (2,))
    N = W.random_complex((n, n), seed + (3,))
    K = W.random_complex((m, n), seed + (4,))
    c = W.random_real((k,), seed + (5,), -1.0, 1.0)
    w = W.random_real((k,), seed + (6,), -1.0, 1.0)

    def loss(U, sv, Vh):
        t = torch.tensor
        out = torch.zeros((), dtype=torch.float64)
        if "u" in cots:
            out = out + torch.real(torch.einsum("rj,rq,qj->", U.conj(), t(M), U))
            out = out + torch.real(torch.sum(t(K).conj() * ((U * t(c)[None, :]) @ Vh)))
        if "s" in cots:
            out = out + torch.sum(t(w) * sv ** 3)
        if "v" in cots:
            out = out + torch.real(torch.einsum("jc,cd,jd->", Vh, t(N), Vh.conj()))
        return out

    A = torch.tensor(A0, requires_grad=True)
    loss(*grad.TruncSVD.apply(A, k, eta)).backward()
    want = A.grad.numpy()
    Ad = torch.from_numpy(A0).cuda()
    print(f"[boundary] truncate_vjp {m}x{n} k={k} cotangents {cots} eta {eta}", flush=True)
    U, S, Vh, kk, _, _ = H.truncate(Ad, k, -1.0)
    assert kk == k
    leaves = [x.detach().cpu().clone().requires_grad_(True) for x in (U, S, Vh)]
    loss(*leaves).backward()
    bars = [x.grad.cuda().contiguous() if x.grad is not None else None for x in leaves]
    got = api.truncate_vjp(H, Ad, S.contiguous(), Vh.contiguous(), bars[0] if "u" in cots else None,
                           bars[1] if "s" in cots else None, bars[2], eta=eta).cpu().numpy()
    code, word = H.device_status()
    assert code == 0 and word == 0, (code, word)
    assert np.isfinite(got).all()
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    # the backward divides by the gaps s_i^2 - s_j^2 >= 0.07 s_i^2 (s >= 1e-2):
    # SVD errors of 1e-16 |theta| grow to about 1e-16 / (0.07e-4) = 1.4e-11
    print(f"[boundary]   rel {err:.2e}", flush=True)
    assert err <= 1e-9


def test_jacobi_absolute_tolerance_floor(H):
    from paper_1703_00387_amd import _lib
    with pytest.raises(_lib.MPSError) as e:
        H.set_option(2, 0.0)
    assert e.value.code == _lib.MPS_ERR_INVALID
    H.set_option(2, 1e-30)
    # a residual with more rows than columns: every row comes back finite
    m, n, k = 96, 64, 20
    A0 = _spectral(m, n, np.geomspace(1.0, 1e-2, n), (113,))
    _, _, Vh = np.linalg.svd(A0, full_matrices=False)
    R = A0 - (A0 @ Vh[:k].conj().T) @ Vh[:k]
    try:
        U, S, V, kk, _, _ = H.truncate(torch.from_numpy(R).cuda(), n - k, -1.0)
        assert kk == n - k and torch.isfinite(torch.view_as_real(V)).all().item()
        np.testing.assert_allclose(S.cpu().numpy(), np.linalg.svd(R, compute_uv=False)[:n - k], rtol=1e-12,
                                   atol=1e-15)
    finally:
        H.set_option(2, 1e-15)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_tebd_step_autograd_function(H, dtype):
    """api.TebdStep (forward: checkpointed batched TEBD2, backward:
    mps_tebd_step_vjp) under torch.autograd, for a loss computed by torch
    from the final states, against the oracle's reverse-mode gradient:
    1e-6 relative for complex128 chains, 1e-4 for complex64 ones (forward on
    FP32 MFMA, reverse pass in FP64; the bar of the complex64 gradient test;
    measured 1.9e-5 and 3.9e-5)."""
    from oracle import grad, models as om
    from paper_1703_00387_amd import api, models
    dt, n_steps, chi, eps = 0.05, 5, 8, 1e-12
    specs = [W.xxz_chain(L, chi, 1.0, 0.5, J_b=W.xxz_grad_couplings(L)) for L in (8, 6)]
    h0s = []
    for sp in specs:
        unit = copy.copy(sp)
        unit.J_b = np.ones(sp.L - 1)
        h0s.append(np.ascontiguousarray(models.bond_hamiltonians(unit)))
    Jn = np.zeros((2, 7))
    for c, sp in enumerate(specs):
        Jn[c, :sp.L - 1] = sp.J_b
    J = torch.tensor(Jn, device="cuda", requires_grad=True)
    sz = 0.5 * om.SZ
    szt = torch.from_numpy(sz.astype(np.complex128)).cuda()
    weights = [W.random_real((sp.L,), (93, c), -1.0, 1.0) for c, sp in enumerate(specs)]
    print("[boundary] TebdStep forward", flush=True)
    outs = api.TebdStep.apply(J, H, [W.initial_vectors(sp) for sp in specs], chi, h0s, dt, n_steps, eps, 1e-12, 2,
                              dtype)
    loss = torch.zeros((), dtype=torch.float64, device="cuda")
    for c, sp in enumerate(specs):
        B, lam, chis = outs[3 * c], outs[3 * c + 1], outs[3 * c + 2].cpu().numpy()
        for i in range(sp.L):
            a, r = int(chis[i]), int(chis[i + 1])
            Bi = B[i, :a, :, :r]
            OB = torch.einsum("st,atc->asc", szt.to(Bi.dtype), Bi)
            loss = loss + weights[c][i] * torch.sum(lam[i, :a] ** 2 * torch.real(torch.einsum("asc,asc->a",
                                                                                              Bi.conj(), OB)))
    print("[boundary] TebdStep backward", flush=True)
    loss.backward()
    g = J.grad.cpu().numpy()
    for c, sp in enumerate(specs):
        Jt = torch.tensor(np.asarray(sp.J_b, dtype=np.float64), requires_grad=True)
        Bt, lt = grad.tebd2_state_torch(sp, Jt, dt, n_steps, chi, eps, 1e-12)
        lo = sum(weights[c][i] * grad.site_expect_torch(Bt, lt, sz, i) for i in range(sp.L))
        lo.backward()
        rel = np.linalg.norm(g[c, :sp.L - 1] - Jt.grad.numpy()) / np.linalg.norm(Jt.grad.numpy())
        print(f"[boundary] TebdStep {dtype} chain L={sp.L}: rel {rel:.2e}", flush=True)
        assert rel <= (1e-6 if dtype == "c128" else 1e-4)
        assert np.all(g[c, sp.L - 1:] == 0.0)


def test_truncate_ex_dtypes_and_renormalize(H):
    """mps_truncate_ex: complex128 equals mps_truncate bit for bit (renormalised
    S = S / |S|); complex64 input is split in FP64 on the exactly up-converted
    matrix (values against the oracle's SVD of it, 1e-13), factors in complex64."""
    from oracle import mps as omps
    m, n, chi = 200, 160, 64
    s = np.geomspace(1.0, 1e-5, min(m, n))
    A0 = _spectral(m, n, s, (121,))
    A0 /= np.linalg.norm(A0)
    A = torch.from_numpy(A0).cuda()
    U1, S1, V1, k1, w1, n1 = H.truncate(A, chi, 1e-12)
    U2, S2, V2, k2, w2, n2 = H.truncate_ex(A, chi, 1e-12, renormalize=True)
    assert k1 == k2 and torch.equal(U1, U2) and torch.equal(V1, V2) and w1 == w2 and n1 == n2
    np.testing.assert_allclose(S2.cpu().numpy(), (S1 / torch.linalg.vector_norm(S1)).cpu().numpy(), rtol=1e-14)
    A64 = A.to(torch.complex64)
    Ar = A64.to(torch.complex128).cpu().numpy()
    U, S, V, k, w, nrm = H.truncate_ex(A64, chi, 1e-12)
    assert U.dtype == torch.complex64 and V.dtype == torch.complex64
    Uo, so, Vho, wo, nko, sfull = omps.truncate(Ar, chi, 1e-12)
    assert k == len(so)
    assert np.abs(S.cpu().numpy() ** 2 - so ** 2).max() <= 1e-13
    R = (U.cpu().numpy().astype(np.complex128) * S.cpu().numpy()) @ V.cpu().numpy().astype(np.complex128)
    Ro = (Uo * so) @ Vho
    assert np.abs(R - Ro).max() <= 2e-6
    with pytest.raises(Exception):
        H.truncate_ex(A.real.contiguous(), chi, 1e-12)


def test_observation_log_matches_oracle(H):
    """MPS_FLAG_OBSERVE: <S^z_i> of every chain after every step, eager and
    under graph replay, against the oracle's runs of 1..n steps."""
    from oracle import mps as omps, models as om
    from paper_1703_00387_amd import api, models, _lib
    specs = _batch_specs(2, 8, 16)
    n_steps, dt, eps = 4, 0.05, 1e-12
    l_max = max(sp.L for sp in specs)
    sz = torch.from_numpy((0.5 * om.SZ).astype(np.complex128)).cuda()
    a = [_chain(sp) for sp in specs]
    log = torch.full((n_steps, len(a), l_max), -7.0, dtype=torch.float64, device="cuda")
    print("[boundary] observation log", flush=True)
    api.tebd_step_ex(H, a, 2, dt, n_steps, eps, obs_op=sz, obs_log=log)
    b = [_chain(sp) for sp in specs]
    log2 = torch.full_like(log, -7.0)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        api.tebd_step_ex(H, b, 2, dt, n_steps, eps, flags=_lib.MPS_FLAG_GRAPH, obs_op=sz, obs_log=log2)
    st.synchronize()
    code, word = H.device_status()
    assert code == 0 and word == 0, (code, word)
    lg, lg2 = log.cpu().numpy(), log2.cpu().numpy()
    for c, sp in enumerate(specs):
        for stp in range(n_steps):
            ref = omps.tebd_run(sp, "tebd2", dt, stp + 1, eps)
            want = omps.local_expect(ref, 0.5 * om.SZ)
            assert np.abs(lg[stp, c, :sp.L] - want).max() <= 1e-10
            assert np.abs(lg2[stp, c, :sp.L] - want).max() <= 1e-10
        assert np.all(lg[:, c, sp.L:] == -7.0)
