"""Host-only size queries of the C ABI (no GPU work): mps_workspace_size
plans through the entry points' own argument checks and workspace plans, and
mps_tebd_ckpt_bytes is the header plus one adjoint arena block per chain."""
import numpy as np
import pytest

import workloads as W
from paper_1703_00387_amd import _lib, api, models


def test_workspace_size_grows_with_the_problem_and_refuses_bad_arguments():
    op = _lib.MPS_OP_TEBD
    one = api.workspace_size(op, "c128", 1, 64, 2, 256)
    many = api.workspace_size(op, "c128", 4, 64, 2, 256)
    small = api.workspace_size(op, "c128", 1, 64, 2, 64)
    assert 0 < small < one < many
    assert api.workspace_size(op, "c64", 1, 64, 2, 256) < one          # complex64 theta~ slots
    t = api.workspace_size(_lib.MPS_OP_TRUNCATE, "c128", 1, 2, 2, 256)   # a 512 x 512 matrix
    assert t >= 512 * 512 * 16
    k = api.workspace_size(_lib.MPS_OP_KRYLOV, "c128", 1, 2, 5, 512, 4, 20)
    assert k >= 21 * 512 * 25 * 512 * 16                                # 21 FP64 Krylov vectors
    assert api.workspace_size(_lib.MPS_OP_TDVP, "c128", 1, 32, 5, 512, 4, 20) > k
    # refused: unknown op, d > 5 for TEBD, d * chi_max beyond 4096, n_max beyond 30
    assert api.workspace_size(99, "c128", 1, 64, 2, 256) == 0
    assert api.workspace_size(op, "c128", 1, 64, 9, 16) == 0
    assert api.workspace_size(op, "c128", 1, 64, 2, 4096) == 0
    assert api.workspace_size(_lib.MPS_OP_KRYLOV, "c128", 1, 2, 5, 64, 4, 40) == 0


def test_checkpoint_arena_bytes():
    specs = [W.xxz_chain(L, 16, 1.0, 0.5) for L in (6, 9)]
    chains = [api.Chain.product(W.initial_vectors(sp), 16, models.bond_hamiltonians(sp), device="cpu")
              for sp in specs]
    per = [_lib.lib().mps_tebd_grad_arena_bytes(sp.L, 2, 16, 5) for sp in specs]
    # a chain's block is the TEBD2 adjoint arena plus what a TEBD4 reverse pass
    # needs besides: 12 more layer snapshots (B, lam, chi of the chain each)
    # and the gates and their derivatives of two more time-step classes
    extra = []
    for sp in specs:
        al = lambda x: (x + 255) // 256 * 256
        snap = al(sp.L * 16 * 2 * 16 * 16) + al((sp.L + 1) * 16 * 8) + al((sp.L + 1) * 4)
        gates = 2 * 2 * (sp.L - 1) * 4 * 4 * 16        # two classes, G and dG, (d^2)^2 complex128
        extra.append(12 * snap + gates)
    total = api.tebd_ckpt_bytes(chains, 5)
    lo = 256 + sum((b + e + 255) // 256 * 256 for b, e in zip(per, extra))
    assert lo <= total <= lo + len(specs) * 4096   # alignment and the gate jobs
    assert api.tebd_ckpt_bytes(chains, 0) == 0
