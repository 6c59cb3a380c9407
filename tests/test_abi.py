"""The C-ABI library loads and exports every symbol include/mps.h declares
(no device call: runs without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for f in os.listdir(inc):
        if f.endswith(".h"):
            src = open(os.path.join(inc, f)).read()
            names |= set(re.findall(r"^\s*(?:mps_status|const char\*|size_t)\s+(mps_\w+)\s*\(", src, re.M))
    return names


def test_header_declares_entry_points():
    names = _declared()
    for must in ("mps_create", "mps_destroy", "mps_truncate", "mps_tebd_step", "mps_gates", "mps_observe"):
        assert must in names


def test_library_exports_declared_symbols():
    from paper_1703_00387_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmps.so not built (run __graft_entry__.build())")
    L = ctypes.CDLL(_lib.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_lib.EXPORTS) == _declared()


def test_product_package_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1703_00387_amd")
    for dp, _, fs in os.walk(pkg):
        for f in fs:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dp, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", src, re.M), f


def test_cfme_nodes_match_the_scheme_definition():
    """Host-only query of the commutator-free Magnus nodes (no GPU needed)."""
    from oracle import timedep
    from paper_1703_00387_amd import api
    for scheme in (2, 4):
        np.testing.assert_allclose(api.cfme_nodes(scheme), timedep.SCHEMES[scheme][0], rtol=0, atol=1e-15)
    with pytest.raises(ValueError):
        api.cfme_nodes(3)
