"""Python face of libmps: device buffers in torch tensors, calls through ctypes.

Only argument marshalling happens here; every step of the update runs in the
HIP kernels of libmps.so.  PyTorch supplies device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import ChainDesc, check, lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Handle:
    """An mps_handle on one device (owns the library workspace)."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise RuntimeError("libmps needs a HIP device")
        self.device = device
        h = C.c_void_p()
        code = lib().mps_create(C.byref(h), device)
        if code != 0:
            raise _lib.MPSError(code, "mps_create failed")
        self.h = h

    def close(self):
        if self.h:
            lib().mps_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, code):
        return check(self.h, code)

    def set_option(self, option: int, value: float):
        self.check(lib().mps_set_option(self.h, option, float(value)))

    def reserve(self, nbytes: int):
        self.check(lib().mps_reserve(self.h, C.c_size_t(nbytes)))

    KERNELS = {"theta": 0, "jac_round": 1, "select": 2, "wb_right": 3, "gemm": 4, "prep": 5, "gates": 6}

    def kernel_stats(self, kernel: str, reset=False):
        """(total_ms, launches, useful_flops) of a kernel class (timing on via set_option(3, 1))."""
        ms, n, w = C.c_double(0), C.c_int64(0), C.c_uint64(0)
        self.check(lib().mps_kernel_stats(self.h, _stream(), self.KERNELS[kernel], C.byref(ms), C.byref(n),
                                          C.byref(w), 1 if reset else 0))
        return float(ms.value), int(n.value), int(w.value)

    def device_status(self):
        w = C.c_uint32(0)
        code = lib().mps_device_status(self.h, _stream(), C.byref(w))
        return code, int(w.value)

    # ---- entry points -------------------------------------------------------
    def gates(self, hmat: torch.Tensor, tau: torch.Tensor, want64=True, want128=True):
        """G = exp(-i tau h) for a batch of Hermitian matrices (complex128)."""
        n, dd, _ = hmat.shape
        G64 = torch.empty((n, dd, dd), dtype=torch.complex64, device=hmat.device) if want64 else None
        G128 = torch.empty((n, dd, dd), dtype=torch.complex128, device=hmat.device) if want128 else None
        self.check(lib().mps_gates(self.h, _stream(), n, dd, _ptr(hmat.contiguous()), _ptr(tau.contiguous()),
                                   _ptr(G64), _ptr(G128)))
        return G64, G128

    def truncate(self, theta: torch.Tensor, chi_max: int, eps: float):
        """Truncated SVD of a complex128 matrix: U, S, Vh (first k valid), k, disc, norm2."""
        theta = theta.contiguous()
        m, n = theta.shape
        dev = theta.device
        U = torch.zeros((m, chi_max), dtype=torch.complex128, device=dev)
        S = torch.zeros(chi_max, dtype=torch.float64, device=dev)
        Vh = torch.zeros((chi_max, n), dtype=torch.complex128, device=dev)
        k = torch.zeros(1, dtype=torch.int32, device=dev)
        disc = torch.zeros(1, dtype=torch.float64, device=dev)
        nrm = torch.zeros(1, dtype=torch.float64, device=dev)
        self.check(lib().mps_truncate(self.h, _stream(), _ptr(theta), m, n, chi_max, float(eps), _ptr(U), _ptr(S),
                                      _ptr(Vh), _ptr(k), _ptr(disc), _ptr(nrm)))
        kk = int(k.item())
        return U[:, :kk], S[:kk], Vh[:kk], kk, float(disc.item()), float(nrm.item())


@dataclass
class Chain:
    """Device storage of one Hastings-form chain (layout of mps_chain_desc).

    dtype "c64": B complex64, contractions on FP32 MFMA; "c128": B complex128,
    contractions on FP64 MFMA.  Schmidt values, SVD and observables are FP64.
    """
    L: int
    d: int
    chi_max: int
    B: torch.Tensor        # complex64 or complex128 [L][chi_max][d][chi_max]
    lam: torch.Tensor      # float64 [L+1][chi_max]
    chi: torch.Tensor      # int32 [L+1]
    hbond: torch.Tensor    # complex128 [L-1][d*d][d*d]
    disc: torch.Tensor     # float64 [L-1]

    @property
    def dtype_code(self):
        return _lib.MPS_C128 if self.B.dtype == torch.complex128 else _lib.MPS_C64

    @staticmethod
    def product(vectors: np.ndarray, chi_max: int, hbond: np.ndarray, device="cuda", dtype="c128") -> "Chain":
        L, d = vectors.shape
        tdt = torch.complex128 if dtype == "c128" else torch.complex64
        B = torch.zeros((L, chi_max, d, chi_max), dtype=tdt)
        for i in range(L):
            v = vectors[i] / np.linalg.norm(vectors[i])
            B[i, 0, :, 0] = torch.from_numpy(v.astype(np.complex128)).to(tdt)
        lam = torch.zeros((L + 1, chi_max), dtype=torch.float64)
        lam[:, 0] = 1.0
        chi = torch.ones(L + 1, dtype=torch.int32)
        return Chain(L, d, chi_max, B.to(device), lam.to(device), chi.to(device),
                     torch.from_numpy(np.ascontiguousarray(hbond)).to(device),
                     torch.zeros(L - 1, dtype=torch.float64, device=device))

    def desc(self) -> ChainDesc:
        return ChainDesc(self.L, self.d, self.chi_max, self.dtype_code, self.B.data_ptr(), self.lam.data_ptr(),
                         self.chi.data_ptr(), self.hbond.data_ptr(), self.disc.data_ptr())

    def to_host(self):
        """(B list [chi_l][d][chi_r] complex128, lam list, chi) on the host."""
        chi = self.chi.cpu().numpy()
        Bh = self.B.cpu().numpy()
        lh = self.lam.cpu().numpy()
        B = [Bh[i, :chi[i], :, :chi[i + 1]].astype(np.complex128) for i in range(self.L)]
        lam = [lh[j, :chi[j]].copy() for j in range(self.L + 1)]
        return B, lam, chi


def tebd_step(h: Handle, chains: Sequence[Chain], order: int, dt: float, n_steps: int, eps: float,
              flags: int = 0):
    arr = (ChainDesc * len(chains))(*[c.desc() for c in chains])
    h.check(lib().mps_tebd_step(h.h, _stream(), arr, len(chains), order, float(dt), n_steps, float(eps), flags))


def observe(h: Handle, chain: Chain, op1=None, op2=None, per_bond=False, entropy=False):
    dev = chain.B.device
    site = torch.zeros(chain.L, dtype=torch.float64, device=dev) if op1 is not None else None
    bond = torch.zeros(chain.L - 1, dtype=torch.float64, device=dev) if op2 is not None else None
    ent = torch.zeros(chain.L - 1, dtype=torch.float64, device=dev) if entropy else None
    o1 = torch.as_tensor(op1, dtype=torch.complex128).to(dev).contiguous() if op1 is not None else None
    o2 = torch.as_tensor(op2, dtype=torch.complex128).to(dev).contiguous() if op2 is not None else None
    d = chain.desc()
    h.check(lib().mps_observe(h.h, _stream(), C.byref(d), _ptr(o1), _ptr(site), _ptr(o2), 1 if per_bond else 0,
                              _ptr(bond), _ptr(ent)))
    return site, bond, ent
