"""Pins of the oracle's model layer: MPO construction and bond Hamiltonians.

T1: the paper's worked three-site Ising MPO product (Sec. Hamiltonians) is
read from tests/golden/ising_mpo_3site.txt and compared term by term; the MPO
contraction, the split bond Hamiltonians and the term-by-term dense H agree
for every model at small L.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import models

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAULI = {"I": models.I2, "X": models.SX, "Z": models.SZ}


def _golden_ising(J, g):
    H = 0
    for line in open(os.path.join(GOLD, "ising_mpo_3site.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        unit, sign, a, b, c = line.split()
        coef = float(sign) * (J if unit == "J" else J * g)
        H = H + coef * np.kron(np.kron(PAULI[a], PAULI[b]), PAULI[c])
    return H


@pytest.mark.parametrize("J,g", [(1.0, 1.0), (0.7, 2.3), (-1.3, 0.4)])
def test_ising_three_site_mpo_matches_paper(J, g):
    spec = W.tfim_chain(3, 8, J, g)
    H_mpo = models.mpo_to_dense(models.mpo(spec))
    np.testing.assert_allclose(H_mpo, _golden_ising(J, g), atol=1e-15)


def _specs():
    return [
        W.tfim_chain(6, 64, 1.0, 1.3),
        W.xxz_chain(6, 64, 1.0, 0.7, J_b=np.linspace(0.8, 1.2, 5), Jz_b=np.linspace(0.5, 1.5, 5)),
        W.bh_chain(4, 2, 64, 1.0, 4.0),
        W.bh_chain(3, 4, 64, 0.6, 3.0),
    ]


@pytest.mark.parametrize("spec", _specs(), ids=lambda s: f"{s.model}-L{s.L}-d{s.d}")
def test_mpo_and_bond_split_equal_site_sum(spec):
    Hs = models.dense_hamiltonian_from_sites(spec)
    assert np.abs(Hs - Hs.conj().T).max() < 1e-14
    np.testing.assert_allclose(models.mpo_to_dense(models.mpo(spec)), Hs, atol=1e-13)
    np.testing.assert_allclose(models.dense_hamiltonian(spec), Hs, atol=1e-13)


def test_xxz_two_site_spectrum():
    # Heisenberg point: S.S on two spins-1/2 has eigenvalues -3/4 (singlet), 1/4 x3.
    spec = W.xxz_chain(2, 4, 1.0, 1.0)
    e = np.linalg.eigvalsh(models.bond_hamiltonians(spec)[0])
    np.testing.assert_allclose(e, [-0.75, 0.25, 0.25, 0.25], atol=1e-15)


def test_boson_ops():
    b, bd, n, I = models.boson_ops(4)
    np.testing.assert_allclose(bd @ b, n, atol=1e-15)
    comm = b @ bd - bd @ b
    np.testing.assert_allclose(np.diag(comm)[:-1], np.ones(4), atol=1e-14)   # [b, b^dag] = 1 below cutoff
