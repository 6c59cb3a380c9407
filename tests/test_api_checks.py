"""Host-side argument checks of the binding (no GPU): bond charges handed to
the charge-carrying entry points and matrices handed to the truncations are
refused with ValueError before any pointer reaches the library, since the
kernels would read or write them with the chain's chi_max stride, or read
them as complex128 device memory."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_1703_00387_amd import api, models


def _chain():
    spec = W.xxz_chain(6, 8, 1.0, 0.5)
    return spec, api.Chain.product(W.initial_vectors(spec), spec.chi_max, models.bond_hamiltonians(spec),
                                   device="cpu")


def _bad_charges(spec, ch):
    good = api.Charges.product(W.initial_vectors(spec), [1, 0], spec.chi_max, device="cpu")
    out = {
        "int64": api.Charges(good.qbond.to(torch.int64), good.qsite),
        "undersized": api.Charges(good.qbond[:, :4].contiguous(), good.qsite),
        "short": api.Charges(good.qbond[:-1].contiguous(), good.qsite),
        "strided": api.Charges(torch.zeros((spec.chi_max, spec.L + 1), dtype=torch.int32).t(), good.qsite),
        "other_device": api.Charges(torch.zeros((spec.L + 1, spec.chi_max), dtype=torch.int32, device="meta"),
                                    good.qsite),
        "qsite": api.Charges(good.qbond, (1, 0, 2)),
    }
    return out


@pytest.mark.parametrize("case", ["int64", "undersized", "short", "strided", "other_device", "qsite"])
def test_tebd_and_ktebd_u1_refuse_bad_charges(case):
    spec, ch = _chain()
    q = _bad_charges(spec, ch)[case]
    with pytest.raises(ValueError):
        api.tebd_step_u1(None, [ch], [q], 2, 0.05, 1, 1e-12)
    with pytest.raises(ValueError):
        api.ktebd_step_u1(None, [ch], [q], 0.05, 1, 1e-12)


@pytest.mark.parametrize("case", ["int64", "undersized", "strided", "other_device"])
def test_time_dependent_u1_refuses_bad_charges(case):
    spec, ch = _chain()
    q = _bad_charges(spec, ch)[case]
    f = np.ones((1, 1, 1))
    with pytest.raises(ValueError):
        api.tebd_td_step(None, [ch], 2, 0.05, 1, 1e-12, f, scheme=2, charges=[q])


def test_charge_count_must_match_chains():
    spec, ch = _chain()
    good = api.Charges.product(W.initial_vectors(spec), [1, 0], spec.chi_max, device="cpu")
    with pytest.raises(ValueError):
        api.tebd_step_u1(None, [ch, ch], [good], 2, 0.05, 1, 1e-12)


@pytest.mark.parametrize("case", ["int64", "undersized", "other_device"])
def test_tdvp_u1_refuses_bad_charges(case):
    from oracle import models as om
    spec = W.xxz_chain(6, 8, 1.0, 0.5)
    oc = api.OCChain.product(W.initial_vectors(spec), spec.chi_max, np.stack(om.mpo(spec)), device="cpu")
    q = _bad_charges(spec, None)[case]
    with pytest.raises(ValueError):
        api.tdvp2_step(None, oc, 0.05, 1, 1e-12, charges=q)


@pytest.mark.parametrize("theta", [
    torch.zeros((4, 4), dtype=torch.complex64),            # wrong element type
    torch.zeros((4, 4), dtype=torch.complex128),           # host memory
    torch.zeros((2, 4, 4), dtype=torch.complex128),        # not a matrix
])
def test_truncations_refuse_bad_matrices(theta):
    with pytest.raises(ValueError):
        api.Handle.truncate(None, theta, 2, 0.0)
    with pytest.raises(ValueError):
        api.Handle.truncate_u1(None, theta, [0] * 4, [0] * 4, 2, 0.0)
