"""Seeded synthetic workloads for the two-site MPS update.

This module is the only code shared by the oracle (``oracle/``) and the HIP
path (``paper_1703_00387_amd``).  It holds workload *parameters* and seeded
random draws only: chain lengths, bond dimensions, couplings, time steps and
the local vectors of initial product states.  It holds none of the method's
arithmetic (no operators, Hamiltonians, gates, contractions or
decompositions); each side builds those itself from the parameters.

The five workloads follow the paper's time-evolution setting (Sec. "Time
evolution methods", Sornborger-Stewart/Trotter decompositions and TDVP) on the
models the paper defines: the transverse Ising chain (Eq. Ising), an XXZ spin
chain, and the Bose-Hubbard chain (Eq. bosehubbard).

Random numbers come from ``numpy.random.SeedSequence(MASTER_SEED)`` spawned
per purpose, with the PCG64 generator.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

MASTER_SEED = 170300387


@dataclass
class ChainSpec:
    """One chain: model name, length, local dimension, couplings and state.

    model    : "tfim", "xxz" or "bh"
    L        : number of sites
    d        : local dimension (2 for spins, n_max+1 for bosons)
    chi_max  : bond-dimension cap
    params   : model scalars (J, g for tfim; Jxy for xxz; t, U for bh)
    J_b      : per-bond overall coupling, length L-1 (xxz; ones otherwise)
    Jz_b     : per-bond zz anisotropy, length L-1 (xxz)
    init     : "all_up", "neel", "unit_filling" or "random_product"
    local_states : (L, d) complex array of normalised site vectors when
               init == "random_product", else None
    """
    model: str
    L: int
    d: int
    chi_max: int
    params: dict
    J_b: np.ndarray
    Jz_b: np.ndarray
    init: str
    local_states: Optional[np.ndarray] = None


@dataclass
class Workload:
    name: str
    method: str            # "tebd2", "tebd4" or "tdvp2"
    dt: float
    n_steps: int
    eps_local: float
    chains: List[ChainSpec] = field(default_factory=list)
    n_krylov: int = 20
    krylov_tol: float = 1e-10
    mpo_w: int = 0


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([MASTER_SEED, *key])))


def product_state_vectors(init: str, L: int, d: int) -> np.ndarray:
    """Local site vectors (L, d) of a deterministic product state.

    Basis convention: for spins index 0 is up (sigma^z = +1), index 1 down;
    for bosons index n is the Fock state with n particles.
    """
    v = np.zeros((L, d), dtype=np.complex128)
    if init == "all_up":
        v[:, 0] = 1.0
    elif init == "neel":
        v[0::2, 0] = 1.0
        v[1::2, 1] = 1.0
    elif init == "unit_filling":
        v[:, 1] = 1.0
    else:
        raise ValueError(init)
    return v


def tfim_chain(L=16, chi_max=32, J=1.0, g=1.0, init="all_up") -> ChainSpec:
    return ChainSpec("tfim", L, 2, chi_max, {"J": J, "g": g},
                     np.ones(L - 1), np.zeros(L - 1), init)


def xxz_chain(L=64, chi_max=256, Jxy=1.0, Jz=0.5, J_b=None, Jz_b=None,
              init="neel", local_states=None) -> ChainSpec:
    J_b = np.ones(L - 1) if J_b is None else np.asarray(J_b, dtype=np.float64)
    Jz_b = np.full(L - 1, Jz) if Jz_b is None else np.asarray(Jz_b, dtype=np.float64)
    return ChainSpec("xxz", L, 2, chi_max, {"Jxy": Jxy}, J_b, Jz_b, init, local_states)


def bh_chain(L=32, n_max=4, chi_max=512, t=1.0, U=4.0, init="unit_filling") -> ChainSpec:
    return ChainSpec("bh", L, n_max + 1, chi_max, {"t": t, "U": U},
                     np.ones(L - 1), np.zeros(L - 1), init)


def initial_vectors(c: ChainSpec) -> np.ndarray:
    if c.init == "random_product":
        return c.local_states
    return product_state_vectors(c.init, c.L, c.d)


# --------------------------------------------------------------------------
# The five workloads
# --------------------------------------------------------------------------

def tfim_tebd2_L16() -> Workload:
    """TEBD2 on the transverse Ising chain, L=16, J=g=1, all up, dt=0.01,
    100 steps, chi_max=32."""
    return Workload("tfim_tebd2_L16", "tebd2", 0.01, 100, 1e-12,
                    [tfim_chain(16, 32, 1.0, 1.0, "all_up")])


def xxz_tebd4_L64() -> Workload:
    """TEBD4 on the XXZ chain, L=64, Jxy=1, Jz=0.5, Neel, dt=0.05, 200 steps,
    chi_max=256."""
    return Workload("xxz_tebd4_L64", "tebd4", 0.05, 200, 1e-12,
                    [xxz_chain(64, 256, 1.0, 0.5)])


def bh_tdvp2_L32() -> Workload:
    """Two-site TDVP with local Krylov on the Bose-Hubbard chain, L=32, d=5,
    t=1, U=4, unit filling, dt=0.02, 100 steps, chi_max=512, 20 Lanczos
    vectors, tolerance 1e-10, MPO bond dimension 4."""
    return Workload("bh_tdvp2_L32", "tdvp2", 0.02, 100, 1e-12,
                    [bh_chain(32, 4, 512, 1.0, 4.0)], n_krylov=20,
                    krylov_tol=1e-10, mpo_w=4)


def xxz_batch256(n_chains=256, n_steps=50) -> Workload:
    """256 independent XXZ chains, L ~ U{16..64}, chi_max ~ {32,64,128,256},
    Jz_b ~ U(0.5,1.5), random product states, TEBD2, dt=0.05, 50 steps."""
    chains = []
    root = np.random.SeedSequence([MASTER_SEED, 4])
    for c, ss in enumerate(root.spawn(n_chains)):
        r = np.random.Generator(np.random.PCG64(ss))
        L = int(r.integers(16, 65))
        chi = int(r.choice([32, 64, 128, 256]))
        jz = r.uniform(0.5, 1.5, L - 1)
        v = r.normal(size=(L, 2)) + 1j * r.normal(size=(L, 2))
        v /= np.linalg.norm(v, axis=1, keepdims=True)
        chains.append(xxz_chain(L, chi, 1.0, 0.5, None, jz, "random_product", v))
    return Workload("xxz_batch256", "tebd2", 0.05, n_steps, 1e-12, chains)


def xxz_grad_couplings(L: int) -> np.ndarray:
    """Per-bond couplings J_b ~ U(0.8, 1.2) for the differentiated workload."""
    ss = np.random.SeedSequence(MASTER_SEED + 5).spawn(1)[0]
    r = np.random.Generator(np.random.PCG64(ss))
    return r.uniform(0.8, 1.2, L - 1)


def xxz_grad_L32(L=32, chi_max=128, n_steps=40) -> Workload:
    """Differentiated TEBD2 on XXZ, L=32, chi_max=128, J_b ~ U(0.8,1.2),
    Jxy=1, Jz=0.5, Neel, dt=0.05, 40 steps."""
    return Workload("xxz_grad_L32", "tebd2", 0.05, n_steps, 1e-12,
                    [xxz_chain(L, chi_max, 1.0, 0.5, xxz_grad_couplings(L))])


ALL = {
    "tfim_tebd2_L16": tfim_tebd2_L16,
    "xxz_tebd4_L64": xxz_tebd4_L64,
    "bh_tdvp2_L32": bh_tdvp2_L32,
    "xxz_batch256": xxz_batch256,
    "xxz_grad_L32": xxz_grad_L32,
}


def random_complex(shape, key, scale=1.0) -> np.ndarray:
    """Seeded complex Gaussian array, for kernel-level parity inputs."""
    r = _rng(*key)
    return scale * (r.normal(size=shape) + 1j * r.normal(size=shape))


def random_oc_tensors(L, d, chi, key):
    """Seeded random chain in mixed-canonical form at the full bond dimension
    chi_b = min(d^b, d^(L-b), chi): site 0 holds the (normalised) centre,
    sites 1..L-1 are right-canonical (orthonormal rows of [chi_i][d chi_{i+1}],
    from the QR factor of a Gaussian matrix).  For timing whole steps at a bond
    dimension a short evolution does not reach.  Returns (chis, site tensors
    [chi_i][d][chi_{i+1}])."""
    chis = [min(d ** b, d ** (L - b), chi) for b in range(L + 1)]
    out = []
    for i in range(L):
        a, c = chis[i], chis[i + 1]
        q, _ = np.linalg.qr(random_complex((d * c, a), tuple(key) + (i,)))
        out.append(np.ascontiguousarray(q.conj().T).reshape(a, d, c))
    return chis, out


def random_real(shape, key, lo=0.0, hi=1.0) -> np.ndarray:
    r = _rng(*key)
    return r.uniform(lo, hi, size=shape)
