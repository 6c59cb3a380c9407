"""Python face of libmps: device buffers in torch tensors, calls through ctypes.

Only argument marshalling happens here; every step of the update runs in the
HIP kernels of libmps.so.  PyTorch supplies device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import ChainDesc, OCChainDesc, check, lib


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_device_matrix(theta):
    """The truncation kernels read theta as complex128 [m][n] in device memory."""
    if not isinstance(theta, torch.Tensor) or theta.dtype != torch.complex128 or theta.dim() != 2:
        raise ValueError("theta must be a complex128 matrix [m][n]")
    if theta.device.type != "cuda":
        raise ValueError(f"theta must be in device memory, not on {theta.device}")


def workspace_size(op: int, dtype: str = "c128", n_chains: int = 1, L: int = 2, d: int = 2, chi_max: int = 1,
                   w: int = 0, n_krylov: int = 0) -> int:
    """mps_workspace_size: device workspace bytes a call of `op` (MPS_OP_*) needs (host only)."""
    code = _lib.MPS_C128 if dtype == "c128" else _lib.MPS_C64
    return int(lib().mps_workspace_size(op, code, n_chains, L, d, chi_max, w, n_krylov))


class Handle:
    """An mps_handle on one device.  With `workspace` (a uint8 device tensor,
    kept alive by the handle) the library works in that memory and never
    allocates after creation (mps_create_ws); otherwise it owns a growable
    workspace."""

    def __init__(self, device: int = 0, workspace: Optional[torch.Tensor] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("libmps needs a HIP device")
        self.device = device
        self.workspace = workspace
        h = C.c_void_p()
        if workspace is not None:
            if workspace.device.type != "cuda" or not workspace.is_contiguous() or workspace.data_ptr() % 256:
                raise ValueError("workspace must be a contiguous, 256-byte aligned device tensor")
            code = lib().mps_create_ws(C.byref(h), device, C.c_void_p(workspace.data_ptr()),
                                       workspace.numel() * workspace.element_size())
        else:
            code = lib().mps_create(C.byref(h), device)
        if code != 0:
            raise _lib.MPSError(code, "mps_create failed")
        self.h = h

    def workspace_needed(self) -> int:
        n = C.c_size_t(0)
        self.check(lib().mps_workspace_needed(self.h, C.byref(n)))
        return int(n.value)

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

    KERNELS = {"theta": 0, "jac_round": 1, "select": 2, "wb_right": 3, "gemm": 4, "prep": 5, "gates": 6,
               "krylov": 7, "warm": 8}

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

    def truncate(self, theta: torch.Tensor, chi_max: int, eps: float, noalloc: bool = False):
        """Truncated SVD of a complex128 matrix: U, S, Vh (first k valid), k, disc, norm2.
        noalloc: through mps_truncate_noalloc (m, n <= 512, no allocation in the library)."""
        _check_device_matrix(theta)
        theta = theta.contiguous()
        m, n = theta.shape
        dev = theta.device
        U = torch.zeros((m, chi_max), dtype=torch.complex128, device=dev)
        S = torch.zeros(chi_max, dtype=torch.float64, device=dev)
        Vh = torch.zeros((chi_max, n), dtype=torch.complex128, device=dev)
        k = torch.zeros(1, dtype=torch.int32, device=dev)
        disc = torch.zeros(1, dtype=torch.float64, device=dev)
        nrm = torch.zeros(1, dtype=torch.float64, device=dev)
        fn = lib().mps_truncate_noalloc if noalloc else lib().mps_truncate
        self.check(fn(self.h, _stream(), _ptr(theta), m, n, chi_max, float(eps), _ptr(U), _ptr(S),
                      _ptr(Vh), _ptr(k), _ptr(disc), _ptr(nrm)))
        kk = int(k.item())
        return U[:, :kk], S[:kk], Vh[:kk], kk, float(disc.item()), float(nrm.item())

    def truncate_ex(self, theta: torch.Tensor, chi_max: int, eps: float, renormalize: bool = False):
        """mps_truncate_ex: truncated SVD of a complex64 or complex128 matrix (the
        SVD in FP64 either way); U, S, Vh (first k valid), k, disc, norm2, with S
        renormalised on request."""
        if (not isinstance(theta, torch.Tensor) or theta.dim() != 2
                or theta.dtype not in (torch.complex64, torch.complex128) or theta.device.type != "cuda"):
            raise ValueError("theta must be a complex64 or complex128 device matrix [m][n]")
        theta = theta.contiguous()
        m, n = theta.shape
        dev, dt = theta.device, theta.dtype
        U = torch.zeros((m, chi_max), dtype=dt, device=dev)
        S = torch.zeros(chi_max, dtype=torch.float64, device=dev)
        Vh = torch.zeros((chi_max, n), dtype=dt, device=dev)
        k = torch.zeros(1, dtype=torch.int32, device=dev)
        disc = torch.zeros(1, dtype=torch.float64, device=dev)
        nrm = torch.zeros(1, dtype=torch.float64, device=dev)
        code = _lib.MPS_C128 if dt == torch.complex128 else _lib.MPS_C64
        self.check(lib().mps_truncate_ex(self.h, _stream(), code, _ptr(theta), m, n, chi_max, float(eps),
                                         1 if renormalize else 0, _ptr(U), _ptr(S), _ptr(Vh), _ptr(k), _ptr(disc),
                                         _ptr(nrm)))
        kk = int(k.item())
        return U[:, :kk], S[:kk], Vh[:kk], kk, float(disc.item()), float(nrm.item())

    def truncate_u1(self, theta: torch.Tensor, row_q, col_q, chi_max: int, eps: float):
        """U(1)-symmetric truncated SVD: theta block diagonal in the row and
        column charges (int sequences, host).  U, S, Vh, q (first k valid), k,
        disc, norm2."""
        _check_device_matrix(theta)
        theta = theta.contiguous()
        m, n = theta.shape
        rq = np.ascontiguousarray(np.asarray(row_q, dtype=np.int32))
        cq = np.ascontiguousarray(np.asarray(col_q, dtype=np.int32))
        if rq.shape != (m,) or cq.shape != (n,):
            raise ValueError("row_q and col_q must have m and n entries")
        dev = theta.device
        U = torch.zeros((m, chi_max), dtype=torch.complex128, device=dev)
        S = torch.zeros(chi_max, dtype=torch.float64, device=dev)
        Vh = torch.zeros((chi_max, n), dtype=torch.complex128, device=dev)
        q = torch.zeros(chi_max, dtype=torch.int32, device=dev)
        k = torch.zeros(1, dtype=torch.int32, device=dev)
        disc = torch.zeros(1, dtype=torch.float64, device=dev)
        nrm = torch.zeros(1, dtype=torch.float64, device=dev)
        self.check(lib().mps_truncate_u1(self.h, _stream(), _ptr(theta), m, n, rq.ctypes.data, cq.ctypes.data,
                                         chi_max, float(eps), _ptr(U), _ptr(S), _ptr(Vh), _ptr(q), _ptr(k),
                                         _ptr(disc), _ptr(nrm)))
        kk = int(k.item())
        return U[:, :kk], S[:kk], Vh[:kk], q[:kk], kk, float(disc.item()), float(nrm.item())


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


def tebd_ckpt_bytes(chains: Sequence[Chain], n_steps: int) -> int:
    """mps_tebd_ckpt_bytes: bytes of the checkpoint arena of tebd_step_ex."""
    arr = (ChainDesc * len(chains))(*[c.desc() for c in chains])
    return int(lib().mps_tebd_ckpt_bytes(arr, len(chains), n_steps))


def tebd_step_ex(h: Handle, chains: Sequence[Chain], order: int, dt: float, n_steps: int, eps: float,
                 flags: int = 0, ckpt: Optional[torch.Tensor] = None, disc_log: Optional[torch.Tensor] = None,
                 obs_op: Optional[torch.Tensor] = None, obs_log: Optional[torch.Tensor] = None):
    """mps_tebd_step_ex: tebd_step with an optional checkpoint arena (uint8 device
    tensor, with flags | MPS_FLAG_CHECKPOINT), an optional float64 device log
    [n_steps][n_layers][n_chains][L_max-1] of every update's discarded weight,
    and, with obs_op (complex128 [d][d] on the device) and obs_log (float64
    [n_steps][n_chains][L_max] on the device), <obs_op at every site> after
    every step (MPS_FLAG_OBSERVE is set for them)."""
    if (obs_op is None) != (obs_log is None):
        raise ValueError("obs_op and obs_log go together")
    if obs_op is not None:
        d = chains[0].d
        l_max = max(c.L for c in chains)
        _c128(obs_op, "obs_op", (d, d))
        _f64(obs_log, "obs_log", (n_steps, len(chains), l_max))
        flags |= _lib.MPS_FLAG_OBSERVE
    if disc_log is not None:
        l_max = max(c.L for c in chains)
        n_layers = {2: 3, 4: 15, 0: 2 * (l_max - 1)}.get(order, 0)
        if (disc_log.dtype != torch.float64 or not disc_log.is_contiguous() or disc_log.device.type != "cuda"
                or disc_log.numel() < n_steps * n_layers * len(chains) * (l_max - 1)):
            raise ValueError("disc_log must be a contiguous float64 device tensor of "
                             "n_steps * n_layers * n_chains * (L_max - 1) entries")
    if ckpt is not None and (ckpt.device.type != "cuda" or not ckpt.is_contiguous()):
        raise ValueError("ckpt must be a contiguous device tensor")
    arr = (ChainDesc * len(chains))(*[c.desc() for c in chains])
    nbytes = ckpt.numel() * ckpt.element_size() if ckpt is not None else 0
    h.check(lib().mps_tebd_step_ex(h.h, _stream(), arr, len(chains), order, float(dt), n_steps, float(eps), flags,
                                   _ptr(ckpt), nbytes, _ptr(disc_log), _ptr(obs_op), _ptr(obs_log)))


def tebd_step_vjp(h: Handle, chains: Sequence[Chain], h0: Sequence[torch.Tensor], ckpt: torch.Tensor,
                  dB: Sequence[torch.Tensor], dlam: Sequence[torch.Tensor], eta: float = 1e-12) -> torch.Tensor:
    """mps_tebd_step_vjp: dL/dJ [n_chains, L_max-1] for state cotangents dB
    (the dtype and layout of each chain's B) and dlam (float64, of lam) of a
    TEBD2 or TEBD4 run recorded by tebd_step_ex with MPS_FLAG_CHECKPOINT."""
    n = len(chains)
    if not (len(h0) == len(dB) == len(dlam) == n):
        raise ValueError("one h0, dB and dlam per chain")
    for c, hh, b, l in zip(chains, h0, dB, dlam):
        if b.shape != c.B.shape or b.dtype != c.B.dtype or not b.is_contiguous() or b.device != c.B.device:
            raise ValueError("dB must have the dtype, layout and device of the chain's B")
        if l.shape != c.lam.shape or l.dtype != torch.float64 or not l.is_contiguous():
            raise ValueError("dlam must be float64 in the layout of the chain's lam")
        if hh.dtype != torch.complex128 or not hh.is_contiguous():
            raise ValueError("h0 must be contiguous complex128")
    l_max = max(c.L for c in chains)
    dJ = torch.zeros((n, l_max - 1), dtype=torch.float64, device=chains[0].B.device)
    arr = (ChainDesc * n)(*[c.desc() for c in chains])
    P = C.c_void_p * n
    h.check(lib().mps_tebd_step_vjp(h.h, _stream(), arr, n, P(*[hh.data_ptr() for hh in h0]), _ptr(ckpt),
                                    ckpt.numel() * ckpt.element_size(), P(*[b.data_ptr() for b in dB]),
                                    P(*[l.data_ptr() for l in dlam]), _ptr(dJ), float(eta)))
    return dJ


def _c128(x, name, shape):
    if (not isinstance(x, torch.Tensor) or x.dtype != torch.complex128 or x.device.type != "cuda"
            or not x.is_contiguous() or tuple(x.shape) != tuple(shape)):
        raise ValueError(f"{name} must be a contiguous complex128 device tensor of shape {tuple(shape)}")


def _f64(x, name, shape):
    if (not isinstance(x, torch.Tensor) or x.dtype != torch.float64 or x.device.type != "cuda"
            or not x.is_contiguous() or tuple(x.shape) != tuple(shape)):
        raise ValueError(f"{name} must be a contiguous float64 device tensor of shape {tuple(shape)}")


def theta_gate_vjp(h: Handle, Bl: torch.Tensor, Br: torch.Tensor, lam_l: torch.Tensor, G: torch.Tensor,
                   theta_bar: torch.Tensor):
    """mps_theta_gate_vjp: (dBl, dBr, dlam_l, dG) for theta' = lam_l G (Bl Br)
    with cotangent theta_bar [chl*d][d*chr].  Bl [chl][d][chm], Br [chm][d][chr],
    G [d*d][d*d], all complex128 on the device; lam_l float64 [chl]."""
    if Bl.dim() != 3 or Br.dim() != 3:
        raise ValueError("Bl and Br are [chi][d][chi]")
    chl, d, chm = Bl.shape
    chr_ = Br.shape[2]
    _c128(Bl, "Bl", (chl, d, chm))
    _c128(Br, "Br", (chm, d, chr_))
    _f64(lam_l, "lam_l", (chl,))
    _c128(G, "G", (d * d, d * d))
    _c128(theta_bar, "theta_bar", (chl * d, d * chr_))
    dBl, dBr, dG = torch.empty_like(Bl), torch.empty_like(Br), torch.empty_like(G)
    dl = torch.empty_like(lam_l)
    h.check(lib().mps_theta_gate_vjp(h.h, _stream(), _ptr(Bl), _ptr(Br), _ptr(lam_l), _ptr(G), _ptr(theta_bar),
                                     chl, d, chm, chr_, _ptr(dBl), _ptr(dBr), _ptr(dl), _ptr(dG)))
    return dBl, dBr, dl, dG


def truncate_vjp(h: Handle, theta: torch.Tensor, S: torch.Tensor, Vh: torch.Tensor, U_bar=None, S_bar=None,
                 Vh_bar=None, eta: float = 0.0) -> torch.Tensor:
    """mps_truncate_vjp: dL/dtheta for the kept factors (U, S, Vh) of a
    truncated SVD of theta [m][n] with k = len(S) kept values; the cotangents
    U_bar [m][k], S_bar [k], Vh_bar [k][n] may each be None (zero)."""
    _check_device_matrix(theta)
    m, n = theta.shape
    k = int(S.shape[0])
    _f64(S, "S", (k,))
    _c128(Vh, "Vh", (k, n))
    if U_bar is not None:
        _c128(U_bar, "U_bar", (m, k))
    if S_bar is not None:
        _f64(S_bar, "S_bar", (k,))
    if Vh_bar is not None:
        _c128(Vh_bar, "Vh_bar", (k, n))
    theta = theta.contiguous()
    out = torch.empty_like(theta)
    h.check(lib().mps_truncate_vjp(h.h, _stream(), _ptr(theta), m, n, k, _ptr(S), _ptr(Vh), _ptr(U_bar), k,
                                   _ptr(S_bar), _ptr(Vh_bar), float(eta), _ptr(out)))
    return out


@dataclass
class Charges:
    """Bond charges of a symmetric chain (layout of mps_u1_chain):
    qbond[b][a] is the charge of sites 0..b-1 in Schmidt state a of bond b,
    qsite[s] the charge of local basis state s; modulus 0 for U(1), n >= 2
    for Z_n (charges modulo n)."""
    qbond: torch.Tensor    # int32 [L+1][chi_max]
    qsite: tuple
    modulus: int = 0

    @staticmethod
    def product(vectors: np.ndarray, qsite, chi_max: int, device="cuda", modulus: int = 0) -> "Charges":
        """Charges of a product of basis states (q_0 = 0, q_{b+1} = q_b + qsite[s_b], modulo n for Z_n)."""
        L, d = vectors.shape
        if len(qsite) != d:
            raise ValueError("qsite needs one charge per local basis state")
        q = torch.zeros((L + 1, chi_max), dtype=torch.int32)
        acc = 0
        for i in range(L):
            nz = np.flatnonzero(np.abs(vectors[i]) > 0)
            if len(nz) != 1:
                raise ValueError("a charge-carrying product state needs a basis state on every site")
            acc += int(qsite[nz[0]])
            if modulus:
                acc %= modulus
            q[i + 1, 0] = acc
        return Charges(q.to(device), tuple(int(x) for x in qsite), int(modulus))

    def desc(self) -> _lib.U1ChainDesc:
        qs = list(self.qsite) + [0] * (5 - len(self.qsite))
        return _lib.U1ChainDesc(self.qbond.data_ptr(), (C.c_int32 * 5)(*qs), self.modulus, (C.c_int32 * 2)())


def _check_charges(chain, q: "Charges"):
    """The bond charges a kernel reads and writes with the chain's chi_max
    stride: a contiguous int32 [L+1][chi_max] tensor on the chain's device,
    at most five site charges."""
    if not isinstance(q, Charges):
        raise ValueError("charges must be Charges")
    t = q.qbond
    if not isinstance(t, torch.Tensor) or t.dtype != torch.int32 or tuple(t.shape) != (chain.L + 1, chain.chi_max):
        raise ValueError(f"qbond must be an int32 tensor [L+1][chi_max] = [{chain.L + 1}][{chain.chi_max}]")
    if not t.is_contiguous():
        raise ValueError("qbond must be contiguous")
    dev = chain.B.device if hasattr(chain, "B") else chain.M.device
    if t.device != dev:
        raise ValueError(f"qbond is on {t.device}, the chain on {dev}")
    if len(q.qsite) > 5 or len(q.qsite) != chain.d:
        raise ValueError("qsite needs one charge per local basis state (d <= 5)")


def _check_charge_list(chains, charges):
    if len(charges) != len(chains):
        raise ValueError("one Charges per chain")
    for c, q in zip(chains, charges):
        _check_charges(c, q)


def tebd_step_u1(h: Handle, chains: Sequence[Chain], charges: Sequence[Charges], order: int, dt: float,
                 n_steps: int, eps: float, flags: int = 0):
    """tebd_step on charge-carrying chains: every update truncated on the
    charge blocks of its bond; charges[i].qbond follows the chain."""
    _check_charge_list(chains, charges)
    arr = (ChainDesc * len(chains))(*[c.desc() for c in chains])
    qa = (_lib.U1ChainDesc * len(chains))(*[q.desc() for q in charges])
    h.check(lib().mps_tebd_step_u1(h.h, _stream(), arr, qa, len(chains), order, float(dt), n_steps, float(eps),
                                   flags))


def ktebd_step(h: Handle, chains: Sequence[Chain], dt: float, n_steps: int, eps: float, n_max: int = 20,
               tol: float = 1e-10, flags: int = 0, n_used=None):
    """Krylov TEBD steps (the sweep with the local Lanczos exponential of every
    bond term).  n_used: optional int32 device tensor [n_chains][2 (L_max-1)]
    receiving the Krylov vectors used by each update of the last step."""
    arr = (ChainDesc * len(chains))(*[c.desc() for c in chains])
    if n_used is not None:
        l_max = max(c.L for c in chains)
        if n_used.dtype != torch.int32 or n_used.numel() < len(chains) * 2 * (l_max - 1) or not n_used.is_contiguous():
            raise ValueError("n_used must be a contiguous int32 tensor of n_chains * 2 (L_max - 1) entries")
    h.check(lib().mps_ktebd_step(h.h, _stream(), arr, len(chains), float(dt), n_steps, float(eps), int(n_max),
                                 float(tol), flags, _ptr(n_used)))


def ktebd_step_u1(h: Handle, chains: Sequence[Chain], charges: Sequence[Charges], dt: float, n_steps: int,
                  eps: float, n_max: int = 20, tol: float = 1e-10, flags: int = 0):
    """ktebd_step on charge-carrying chains (every cut on the charge blocks of its bond)."""
    _check_charge_list(chains, charges)
    arr = (ChainDesc * len(chains))(*[c.desc() for c in chains])
    qa = (_lib.U1ChainDesc * len(chains))(*[q.desc() for q in charges])
    h.check(lib().mps_ktebd_step_u1(h.h, _stream(), arr, qa, len(chains), float(dt), n_steps, float(eps),
                                    int(n_max), float(tol), flags, None))


def cfme_nodes(scheme: int):
    """Nodes c_j of a commutator-free Magnus scheme (2 or 4)."""
    nodes = (C.c_double * 2)()
    n = C.c_int32(0)
    if lib().mps_cfme_nodes(int(scheme), nodes, C.byref(n)) != _lib.MPS_OK:
        raise ValueError(f"unknown commutator-free Magnus scheme {scheme}")
    return np.array(nodes[:n.value])


def tebd_td_step(h: Handle, chains: Sequence[Chain], order: int, dt: float, n_steps: int, eps: float,
                 f_nodes, scheme: int = 2, flags: int = 0, charges: Optional[Sequence["Charges"]] = None):
    """Time-dependent steps; every chain's hbond holds its term split
    [n_terms][L-1][d*d][d*d] and f_nodes[n][j][k] = f_k(t_n + c_j dt).
    charges: one Charges per chain for charge-carrying chains."""
    f = np.ascontiguousarray(f_nodes, dtype=np.float64)
    if f.ndim != 3 or f.shape[0] != n_steps:
        raise ValueError("f_nodes must be [n_steps][n_nodes][n_terms]")
    n_terms = f.shape[2]
    total = 0
    for c in chains:
        dd = c.d * c.d
        if c.hbond.numel() != n_terms * (c.L - 1) * dd * dd:
            raise ValueError("chain hbond must hold n_terms bond-term sets")
        total += (c.L - 1) * dd * dd
    hwork = torch.empty(total, dtype=torch.complex128, device=chains[0].B.device)
    arr = (ChainDesc * len(chains))(*[c.desc() for c in chains])
    if charges is not None:
        _check_charge_list(chains, charges)
        qa = (_lib.U1ChainDesc * len(chains))(*[q.desc() for q in charges])
        h.check(lib().mps_tebd_td_step_u1(h.h, _stream(), arr, qa, len(chains), order, float(dt), n_steps,
                                          float(eps), flags, n_terms, int(scheme), f.ctypes.data_as(C.c_void_p),
                                          _ptr(hwork)))
        return
    h.check(lib().mps_tebd_td_step(h.h, _stream(), arr, len(chains), order, float(dt), n_steps, float(eps), flags,
                                   n_terms, int(scheme), f.ctypes.data_as(C.c_void_p), _ptr(hwork)))


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


def tebd_grad(h: Handle, chain: Chain, h0, dt: float, n_steps: int, eps: float, op1, site: int, op2,
              eta: float = 1e-12):
    """Loss <op1 at site> + sum_b <op2 on bond b> after n_steps TEBD2 steps, and
    its gradient with respect to the per-bond couplings J_b, where the chain's
    bond Hamiltonians are h_b = J_b * h0[b].  The chain is advanced to the final
    state.  Returns (loss, dJ) as device tensors (float64, [] and [L-1])."""
    dev = chain.B.device
    nbytes = lib().mps_tebd_grad_arena_bytes(chain.L, chain.d, chain.chi_max, n_steps)
    if nbytes == 0:
        raise _lib.MPSError(_lib.MPS_ERR_INVALID, "bad shape for the gradient arena")
    arena = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    h0t = torch.as_tensor(h0, dtype=torch.complex128).to(dev).contiguous()
    o1 = torch.as_tensor(op1, dtype=torch.complex128).to(dev).contiguous()
    o2 = torch.as_tensor(op2, dtype=torch.complex128).to(dev).contiguous()
    loss = torch.zeros((), dtype=torch.float64, device=dev)
    dJ = torch.zeros(chain.L - 1, dtype=torch.float64, device=dev)
    d = chain.desc()
    h.check(lib().mps_tebd_grad(h.h, _stream(), C.byref(d), _ptr(h0t), float(dt), n_steps, float(eps), float(eta),
                                _ptr(o1), site, _ptr(o2), _ptr(arena), nbytes, _ptr(loss), _ptr(dJ)))
    return loss, dJ


def tebd_vjp(h: Handle, chain: Chain, h0, dt: float, n_steps: int, eps: float, op1, op2, w_site, w_bond,
             eta: float = 1e-12):
    """Final observables (<op1 at i>, i < L; <op2 on b>, b < L-1) of n_steps TEBD2
    steps from the chain's state, and their vector-Jacobian product with the
    cotangent (w_site, w_bond) with respect to J_b (h_b = J_b h0[b]).  Returns
    (obs [2L-1], dJ [L-1]) as device float64 tensors."""
    dev = chain.B.device
    L = chain.L
    nbytes = lib().mps_tebd_grad_arena_bytes(L, chain.d, chain.chi_max, n_steps)
    if nbytes == 0:
        raise _lib.MPSError(_lib.MPS_ERR_INVALID, "bad shape for the gradient arena")
    arena = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    h0t = torch.as_tensor(h0, dtype=torch.complex128).to(dev).contiguous()
    o1 = torch.as_tensor(op1, dtype=torch.complex128).to(dev).contiguous()
    o2 = torch.as_tensor(op2, dtype=torch.complex128).to(dev).contiguous()
    ws = np.ascontiguousarray(np.asarray(w_site, dtype=np.float64).reshape(L))
    wb = np.ascontiguousarray(np.asarray(w_bond, dtype=np.float64).reshape(L - 1))
    obs = torch.zeros(2 * L - 1, dtype=torch.float64, device=dev)
    dJ = torch.zeros(L - 1, dtype=torch.float64, device=dev)
    d = chain.desc()
    h.check(lib().mps_tebd_vjp(h.h, _stream(), C.byref(d), _ptr(h0t), float(dt), n_steps, float(eps), float(eta),
                               _ptr(o1), ws.ctypes.data_as(C.c_void_p), _ptr(o2), wb.ctypes.data_as(C.c_void_p),
                               _ptr(arena), nbytes, _ptr(obs), _ptr(dJ)))
    return obs, dJ


class TebdObservables(torch.autograd.Function):
    """Final observables of a TEBD2 run as a differentiable function of the
    per-bond couplings J (h_b = J_b h0[b]), from a product state:

        obs = TebdObservables.apply(J, h, vectors, chi_max, h0, dt, n_steps, eps, op1, op2, eta)

    obs[:L] = <op1 at site i>, obs[L:] = <op2 on bond b> (float64, on the GPU).
    The forward runs mps_tebd_step (order 2) and mps_observe; the backward runs
    mps_tebd_vjp with the incoming gradient as the cotangent (it re-runs the
    forward with a checkpoint per step).  dtype "c128" or "c64" (FP32 MFMA
    contractions in the forward and its re-runs; the reverse pass in FP64)."""

    @staticmethod
    def forward(ctx, J, h, vectors, chi_max, h0, dt, n_steps, eps, op1, op2, eta=1e-12, dtype="c128"):
        hb = J.detach().to(torch.complex128)[:, None, None] * torch.as_tensor(h0, dtype=torch.complex128).to(J.device)
        chain = Chain.product(vectors, chi_max, hb.cpu().numpy(), device=J.device, dtype=dtype)
        tebd_step(h, [chain], 2, dt, n_steps, eps)
        site, bond, _ = observe(h, chain, op1, op2)
        ctx.args = (h, vectors, chi_max, h0, dt, n_steps, eps, op1, op2, eta, dtype)
        ctx.save_for_backward(J.detach())
        return torch.cat([site, bond])

    @staticmethod
    def backward(ctx, g):
        (J,) = ctx.saved_tensors
        h, vectors, chi_max, h0, dt, n_steps, eps, op1, op2, eta, dtype = ctx.args
        L = J.numel() + 1
        hb = J.to(torch.complex128)[:, None, None] * torch.as_tensor(h0, dtype=torch.complex128).to(J.device)
        chain = Chain.product(vectors, chi_max, hb.cpu().numpy(), device=J.device, dtype=dtype)
        w = g.detach().double().cpu().numpy()
        _, dJ = tebd_vjp(h, chain, h0, dt, n_steps, eps, op1, op2, w[:L], w[L:], eta)
        return (dJ.to(J.dtype),) + (None,) * 11


class TebdStep(torch.autograd.Function):
    """Final Hastings-form states of a batched TEBD2 (order 2) or TEBD4
    (order 4) run as a differentiable function of the per-bond couplings
    J [n_chains, L_max-1] (chain c has h_b = J[c, b] h0[c][b]), from product
    states:

        outs = TebdStep.apply(J, h, vectors, chi_max, h0, dt, n_steps, eps, eta, order)

    vectors[c] and h0[c] are chain c's initial site vectors and unit bond
    terms (complex128 [L_c-1][d^2][d^2]).  outs = (B_0, lam_0, chi_0, B_1,
    ...) in the capacity layout of Chain; chi_c is not differentiable.  The
    forward runs mps_tebd_step_ex with MPS_FLAG_CHECKPOINT, the backward
    mps_tebd_step_vjp on that checkpoint with the incoming cotangents of the
    B and lam (zero where None).  dtype "c128" or "c64": the chains' B (FP32
    MFMA contractions for c64; the reverse pass in FP64 on the checkpointed
    states widened exactly)."""

    @staticmethod
    def forward(ctx, J, h, vectors, chi_max, h0, dt, n_steps, eps, eta=1e-12, order=2, dtype="c128"):
        n = len(vectors)
        if order not in (2, 4):
            raise ValueError("order must be 2 (TEBD2) or 4 (TEBD4)")
        if J.dim() != 2 or J.shape[0] != n:
            raise ValueError("J must be [n_chains, L_max-1]")
        dev = J.device
        h0d = [torch.as_tensor(np.ascontiguousarray(x), dtype=torch.complex128).to(dev).contiguous() for x in h0]
        chains = []
        for c in range(n):
            L = len(vectors[c])
            if h0d[c].shape[0] != L - 1 or J.shape[1] < L - 1:
                raise ValueError("h0[c] needs L_c-1 bond terms and J at least L_c-1 columns")
            hb = J.detach()[c, :L - 1].to(torch.complex128)[:, None, None] * h0d[c]
            chains.append(Chain.product(vectors[c], chi_max, hb.cpu().numpy(), device=dev, dtype=dtype))
        ck = torch.zeros(tebd_ckpt_bytes(chains, n_steps), dtype=torch.uint8, device=dev)
        tebd_step_ex(h, chains, order, dt, n_steps, eps, flags=_lib.MPS_FLAG_CHECKPOINT, ckpt=ck)
        ctx.state = (h, chains, h0d, ck, eta, J.shape[1])
        outs = []
        for ch in chains:
            outs += [ch.B.clone(), ch.lam.clone(), ch.chi.clone()]
        ctx.mark_non_differentiable(*outs[2::3])
        return tuple(outs)

    @staticmethod
    def backward(ctx, *grads):
        h, chains, h0d, ck, eta, width = ctx.state
        dB = [g.contiguous() if g is not None else torch.zeros_like(ch.B) for g, ch in zip(grads[0::3], chains)]
        dl = [g.contiguous() if g is not None else torch.zeros_like(ch.lam) for g, ch in zip(grads[1::3], chains)]
        dJ = tebd_step_vjp(h, chains, h0d, ck, dB, dl, eta)
        out = torch.zeros((len(chains), width), dtype=torch.float64, device=dJ.device)
        out[:, :dJ.shape[1]] = dJ
        return (out,) + (None,) * 10


def autotune_gemm(h: Handle, kind: int, dtype: str, M: int, N: int, K: int, batch: int = 1, apply: bool = True):
    """mps_autotune_gemm: time the six MFMA tile shapes of the strided (kind 0)
    or batched write-back (kind 1) GEMM at M x N x K and, with apply, make the
    fastest the tile of that shape bucket.  Returns {"times_ms", "best",
    "tiles"} with tiles[i] = (tile_m, tile_n) of candidate i."""
    cap = C.c_int32(8)
    times = (C.c_double * 8)()
    best = C.c_int32(-1)
    code = _lib.MPS_C128 if dtype == "c128" else _lib.MPS_C64
    h.check(lib().mps_autotune_gemm(h.h, _stream(), kind, code, batch, M, N, K, 1 if apply else 0, times,
                                    C.byref(cap), C.byref(best)))
    tiles = []
    for i in range(cap.value):
        tm, tn = C.c_int32(0), C.c_int32(0)
        check(h.h, lib().mps_gemm_candidate(i, C.byref(tm), C.byref(tn)))
        tiles.append((tm.value, tn.value))
    return {"times_ms": [times[i] for i in range(cap.value)], "best": best.value, "tiles": tiles}


def gemm_tile(kind: int, dtype: str, M: int, N: int, index: Optional[int] = None) -> int:
    """The tile candidate of the (kind, dtype, M x N) bucket; with index, set it first."""
    code = _lib.MPS_C128 if dtype == "c128" else _lib.MPS_C64
    if index is not None:
        check(None, lib().mps_set_gemm_tile(kind, code, M, N, index))
    out = C.c_int32(-1)
    check(None, lib().mps_gemm_tile_choice(kind, code, M, N, C.byref(out)))
    return out.value


def autotune(h: Handle, n_mats: int, m: int, n: int, apply: bool = True, cache: str = None):
    """Time the Jacobi launch configurations on a seeded synthetic batch of
    n_mats m x n matrices (mps_autotune_jacobi) and, with apply, leave the
    fastest in the handle.  With a JSON cache path, a bucket measured before on
    the same device model is applied from the cache without timing.
    Returns {"threads", "split_below", "method", "times_ms", "cached"}."""
    import json
    import os
    key = f"{torch.cuda.get_device_name(h.device) if torch.cuda.is_available() else 'cpu'}|{n_mats}|{m}|{n}"
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
    if key in table:
        r = dict(table[key])
        if apply:
            h.set_option(5, r["threads"])
            h.set_option(6, r["split_below"])
            h.set_option(7, r["method"])
        r["cached"] = True
        return r
    cap = C.c_int32(12)
    times = (C.c_double * 12)()
    best = C.c_int32(-1)
    h.check(lib().mps_autotune_jacobi(h.h, _stream(), n_mats, m, n, 1 if apply else 0, times, C.byref(cap),
                                      C.byref(best)))
    t, sb, me = C.c_int32(0), C.c_int32(0), C.c_int32(0)
    check(h.h, lib().mps_autotune_candidate(m, best.value, C.byref(t), C.byref(sb), C.byref(me)))
    r = {"threads": t.value, "split_below": sb.value, "method": me.value,
         "times_ms": [round(times[i], 4) for i in range(cap.value)]}
    if cache:
        table[key] = r
        with open(cache, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
    r["cached"] = False
    return r


def _code(t):
    return _lib.MPS_C128 if t.dtype == torch.complex128 else _lib.MPS_C64


def heff_apply(h: Handle, Lenv, W1, W2, Renv, x):
    """y = H_eff x; shapes Lenv [chl,wl,chl], W1 [wl,wm,d1,d1], W2 [wm,wr,d2,d2] or None,
    Renv [chr,wr,chr], x [chl,d1,d2,chr] (or [chl,d1,chr])."""
    y = torch.empty_like(x)
    chl, wl = Lenv.shape[0], Lenv.shape[1]
    d1, wm = W1.shape[2], W1.shape[1]
    if W2 is not None:
        d2, wr = W2.shape[2], W2.shape[1]
    else:
        d2, wr = 0, 0
    chr_ = Renv.shape[0]
    h.check(lib().mps_heff_apply(h.h, _stream(), _code(x), _ptr(Lenv), _ptr(W1), _ptr(W2), _ptr(Renv), _ptr(x),
                                 _ptr(y), chl, d1, d2, chr_, wl, wm, wr))
    return y


def krylov_expm(h: Handle, Lenv, W1, W2, Renv, x, tau, n_max=20, tol=1e-10):
    """x <- exp(-i tau H_eff) x in place; returns (n_used, err_est)."""
    chl, wl = Lenv.shape[0], Lenv.shape[1]
    d1, wm = W1.shape[2], W1.shape[1]
    d2, wr = (W2.shape[2], W2.shape[1]) if W2 is not None else (0, 0)
    nu = torch.zeros(1, dtype=torch.int32, device=x.device)
    err = torch.zeros(1, dtype=torch.float64, device=x.device)
    tau = complex(tau)
    h.check(lib().mps_krylov_expm(h.h, _stream(), _code(x), _ptr(Lenv), _ptr(W1), _ptr(W2), _ptr(Renv), _ptr(x),
                                  chl, d1, d2, Renv.shape[0], wl, wm, wr, tau.real, tau.imag, n_max, tol,
                                  _ptr(nu), _ptr(err)))
    return int(nu.item()), float(err.item())


def env_update(h: Handle, side: str, env_in, W, A):
    """Left (side='left': A [chi,d,chi2]) or right (side='right': A [chi2,d,chi]) environment update."""
    if side == "left":
        chi_in, d, chi_out = A.shape
        w_in, w_out = W.shape[0], W.shape[1]
    else:
        chi_out, d, chi_in = A.shape
        w_out, w_in = W.shape[0], W.shape[1]
    out = torch.empty((chi_out, w_out, chi_out), dtype=A.dtype, device=A.device)
    h.check(lib().mps_env_update(h.h, _stream(), _code(A), 0 if side == "left" else 1, _ptr(env_in.contiguous()),
                                 _ptr(W.contiguous()), _ptr(A.contiguous()), _ptr(out), chi_in, d, chi_out, w_in,
                                 w_out))
    return out


@dataclass
class OCChain:
    """Mixed-canonical chain for two-site TDVP (layout of mps_oc_chain)."""
    L: int
    d: int
    chi_max: int
    w: int
    M: torch.Tensor      # [L][chi_max*d*chi_max] (compact [chi_i][d][chi_{i+1}] at the start of each block)
    chi: torch.Tensor    # int32 [L+1]
    W: torch.Tensor      # [L][w][w][d][d]
    disc: torch.Tensor   # float64 [L-1]

    @staticmethod
    def product(vectors: np.ndarray, chi_max: int, W: np.ndarray, device="cuda", dtype="c128") -> "OCChain":
        L, d = vectors.shape
        tdt = torch.complex128 if dtype == "c128" else torch.complex64
        M = torch.zeros((L, chi_max * d * chi_max), dtype=tdt)
        for i in range(L):
            v = vectors[i] / np.linalg.norm(vectors[i])
            M[i, :d] = torch.from_numpy(v.astype(np.complex128)).to(tdt)
        return OCChain(L, d, chi_max, W.shape[1], M.to(device), torch.ones(L + 1, dtype=torch.int32, device=device),
                       torch.from_numpy(np.ascontiguousarray(W)).to(tdt).to(device),
                       torch.zeros(L - 1, dtype=torch.float64, device=device))

    def desc(self) -> OCChainDesc:
        return OCChainDesc(self.L, self.d, self.chi_max, _code(self.M), self.w, 0, self.M.data_ptr(),
                           self.chi.data_ptr(), self.W.data_ptr())

    def tensors(self):
        chi = self.chi.cpu().numpy()
        Mh = self.M.cpu().numpy()
        return [Mh[i, :chi[i] * self.d * chi[i + 1]].reshape(chi[i], self.d, chi[i + 1]).astype(np.complex128)
                for i in range(self.L)]

    def to_vector(self):
        Ms = self.tensors()
        v = Ms[0].reshape(-1, Ms[0].shape[2])
        for T in Ms[1:]:
            v = (v @ T.reshape(T.shape[0], -1)).reshape(-1, T.shape[2])
        return v.reshape(-1)


def tdvp2_step(h: Handle, chain: OCChain, dt: float, n_steps: int, eps: float, n_max=20, tol=1e-10,
               charges: Optional["Charges"] = None):
    """Two-site TDVP steps; charges: the chain's Charges for a charge-carrying
    chain (every split on the charge blocks of its bond)."""
    kmax = torch.zeros(1, dtype=torch.int32, device=chain.M.device)
    d = chain.desc()
    if charges is not None:
        _check_charges(chain, charges)
        q = charges.desc()
        h.check(lib().mps_tdvp2_step_u1(h.h, _stream(), C.byref(d), C.byref(q), float(dt), n_steps, float(eps),
                                        n_max, float(tol), _ptr(chain.disc), _ptr(kmax)))
    else:
        h.check(lib().mps_tdvp2_step(h.h, _stream(), C.byref(d), float(dt), n_steps, float(eps), n_max, float(tol),
                                     _ptr(chain.disc), _ptr(kmax)))
    return int(kmax.item())
