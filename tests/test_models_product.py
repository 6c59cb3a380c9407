"""The GPU path's model inputs (bond Hamiltonians, MPOs) equal the oracle's.

Both sides build them independently from the model definitions; this CPU test
checks they describe the same Hamiltonians."""
import numpy as np
import pytest

import workloads as W
from oracle import models as om
from paper_1703_00387_amd import models as pm


@pytest.mark.parametrize("spec", [
    W.tfim_chain(7, 8, 1.3, 0.7),
    W.xxz_chain(7, 8, 0.9, 0.5, J_b=np.linspace(0.8, 1.2, 6), Jz_b=np.linspace(0.5, 1.5, 6)),
    W.bh_chain(5, 4, 8, 1.0, 4.0),
], ids=lambda s: s.model)
def test_product_models_equal_oracle(spec):
    np.testing.assert_allclose(pm.bond_hamiltonians(spec), np.stack(om.bond_hamiltonians(spec)), atol=1e-15)
    np.testing.assert_allclose(pm.mpo(spec), np.stack(om.mpo(spec)), atol=1e-15)
