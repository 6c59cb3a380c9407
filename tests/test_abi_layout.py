"""The ctypes descriptors of the binding have the layout of the C structs in
include/mps.h: a C program built with gcc prints sizeof and offsetof of every
field, compared with the ctypes Structure fields.  Host logic of the
charge-carrying chains' Charges.product (no GPU)."""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "mps_chain_desc": ("ChainDesc", ["L", "d", "chi_max", "dtype", "B", "lam", "chi", "hbond", "disc"]),
    "mps_oc_chain": ("OCChainDesc", ["L", "d", "chi_max", "dtype", "w", "reserved", "M", "chi", "W"]),
    "mps_u1_chain": ("U1ChainDesc", ["qbond", "qsite", "modulus", "reserved"]),
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_descriptor_layouts_match_the_header(tmp_path):
    from paper_1703_00387_amd import _lib
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{ROOT}/include/mps.h"', 'int main(void) {']
    for cname, (_, fields) in STRUCTS.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ['  return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln.strip():
            name, field, val = ln.split()
            got[(name, field)] = int(val)
    for cname, (pyname, fields) in STRUCTS.items():
        cls = getattr(_lib, pyname)
        assert C.sizeof(cls) == got[(cname, "size")], cname
        for f in fields:
            assert getattr(cls, f).offset == got[(cname, f)], (cname, f)


def test_charges_of_a_product_state():
    torch = pytest.importorskip("torch")
    from paper_1703_00387_amd import api
    import workloads as W
    v = W.product_state_vectors("neel", 6, 2)
    q = api.Charges.product(v, [1, 0], 4, device="cpu")
    assert q.qbond.dtype == torch.int32 and tuple(q.qbond.shape) == (7, 4)
    assert q.qbond[:, 0].tolist() == [0, 1, 1, 2, 2, 3, 3]
    q2 = api.Charges.product(v, [1, 0], 4, device="cpu", modulus=2)
    assert q2.qbond[:, 0].tolist() == [0, 1, 1, 0, 0, 1, 1] and q2.modulus == 2
    d = q2.desc()
    assert list(d.qsite)[:2] == [1, 0] and d.modulus == 2
    with pytest.raises(ValueError):
        api.Charges.product(v, [1, 0, 2], 4, device="cpu")
    with pytest.raises(ValueError):
        api.Charges.product(np.full((6, 2), 2 ** -0.5), [1, 0], 4, device="cpu")
