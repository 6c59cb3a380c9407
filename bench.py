"""Throughput of the two-site MPS update on one MI355X.

Workload: TEBD4 (fourth-order Suzuki fractal of Strang steps) on the XXZ chain,
L=64, Jxy=1, Jz=0.5, Neel start, dt=0.05, chi_max=256, eps_local=1e-12,
complex128 chain (FP64 MFMA contractions, FP64 Jacobi SVD).  One step = one
TEBD4 time step = 15 even/odd layers = 475 two-site updates.  A prelude of 140
untimed steps grows chi from 1 to the cap (47 of 65 bonds at chi = 256),
whatever W is; then W more untimed steps, then exactly K timed steps in five
windows (the line's value is the median window rate).  A run whose timed
state has no bond at the cap prints no value and exits non-zero.  Prints one
JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtype c128|c64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector (and matrix) peak
FP32_MFMA_PEAK_TFLOPS = 157.3
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the Jacobi kernel (jac_persist_kernel, one launch per
# layer) on this workload, from two rocprofv3 --pmc runs (FETCH_SIZE,
# WRITE_SIZE) over the first timed TEBD4 step of the default command (state
# after 140 prelude and 5 warmup steps from the Neel state), each scaled by the
# same counter's reading for a plain streaming kernel of known size
# (FETCH_SIZE x 2.000, WRITE_SIZE x 1.000).  Valid only for the kernel source
# it was measured on (hash of its files); otherwise null.
JAC_ROUND_TRAFFIC = {
    "sources_sha256": "dd763ca18b8a25194c63f2baba7a3ae6eb00da1771a23e0e75be5b7c2918124d",
    "bytes_per_launch": 3.8853e10,
    "warmup": 5,   # state: 140 prelude steps + this many warmup steps from the Neel state
}
JAC_ROUND_SOURCES = ("svd.hip", "jacobi_small.h", "mfma_tile.h")


def _jac_round_traffic():
    import hashlib
    hsh = hashlib.sha256()
    for f in JAC_ROUND_SOURCES:
        with open(os.path.join(ROOT, "paper_1703_00387_amd", "csrc", f), "rb") as fh:
            hsh.update(fh.read())
    ok = hsh.hexdigest() == JAC_ROUND_TRAFFIC["sources_sha256"]
    return JAC_ROUND_TRAFFIC["bytes_per_launch"] if ok else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before the timed ones (xxz_tebd4_L64: after the chi-growth prelude, "
                         "default 2; other workloads: their growth steps, e.g. 40 for xxz_batch256)")
    ap.add_argument("--prelude", type=int, default=140,
                    help="xxz_tebd4_L64: untimed TEBD4 steps that grow chi to the cap before the warmup")
    ap.add_argument("--dtype", default="c128", choices=["c128", "c64"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--jac-threads", type=int, default=512, choices=[256, 512],
                    help="threads per Jacobi-round workgroup (two waves per SIMD at 512)")
    ap.add_argument("--autotune", default=None, metavar="CACHE_JSON",
                    help="xxz_tebd4_L64: autotune the Jacobi for the chi=256 layer (32 x 512 x 512) first, with "
                         "this JSON cache")
    ap.add_argument("--split", default="svd", choices=["svd", "eig"],
                    help="two-site split of matrices of at most 64 rows: one-sided Jacobi SVD or the "
                         "eigendecomposition of the Gram")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--max-sweeps", type=int, default=0,
                    help="cap on the Jacobi sweeps of a split (option 1; 0 = the library default); a capped "
                         "split that has not converged sets MPS_DEV_NOCONV, reported in device_status")
    ap.add_argument("--jac-abs", type=float, default=None,
                    help="absolute floor of the Jacobi's orthogonality test, relative to |theta|_F^2 (option 2; "
                         "default 1e-15)")
    ap.add_argument("--warm", action="store_true",
                    help="Jacobi of the TEBD splits from Q^dag theta', Q from the QR of Lambda_l B_b (option 9 = 1)")
    ap.add_argument("--rounds", action="store_true",
                    help="one launch per Jacobi round with a convergence read-back per sweep, instead of the "
                         "persistent Jacobi launch")
    ap.add_argument("--no-plain", action="store_true", help="xxz_batch256: skip the one-bond-per-launch comparison")
    ap.add_argument("--save-state", default=None, help="save the chain after the warmup (torch.save)")
    ap.add_argument("--load-state", default=None, help="start from a saved chain instead of the product state")
    ap.add_argument("--workload", default="xxz_tebd4_L64", choices=["xxz_tebd4_L64", "xxz_batch256", "bh_heff_chi512", "xxz_grad_L32",
                             "xxz_sweep_L64", "tfim_quench_L64", "bh_tdvp_L32", "bh_u1_svd_chi320",
                             "xxz_tebd4_L64_u1", "bh_tdvp_step_chi512"])
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs on one GPU and has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        return calibrate_copy(args.calibrate_copy)
    if args.warmup is None:
        args.warmup = {"xxz_batch256": 40, "tfim_quench_L64": 150, "bh_tdvp_L32": 40,
                       "bh_u1_svd_chi320": 1, "xxz_tebd4_L64": 2}.get(args.workload, 140)

    import workloads as W
    from paper_1703_00387_amd import api, models

    if args.workload == "xxz_batch256":
        return bench_batch(args)
    if args.workload == "bh_heff_chi512":
        return bench_heff(args)
    if args.workload == "xxz_grad_L32":
        return bench_grad(args)
    if args.workload == "xxz_sweep_L64":
        return bench_sweep(args)
    if args.workload == "tfim_quench_L64":
        return bench_quench(args)
    if args.workload == "bh_tdvp_L32":
        return bench_tdvp(args)
    if args.workload == "bh_u1_svd_chi320":
        return bench_u1(args)
    if args.workload == "xxz_tebd4_L64_u1":
        return bench_u1_tebd(args)
    if args.workload == "bh_tdvp_step_chi512":
        return bench_tdvp_step(args)
    wl = W.xxz_tebd4_L64()
    spec = wl.chains[0]
    updates_per_step = sum(len(range(p, spec.L - 1, 2)) for p in (0, 1, 0)) * 5
    h = api.Handle(0)
    h.set_option(5, args.jac_threads)
    h.set_option(7, 1.0 if args.split == "eig" else 0.0)
    h.set_option(8, 0.0 if args.rounds else 1.0)
    h.set_option(9, 1.0 if args.warm else 0.0)
    if args.max_sweeps:
        h.set_option(1, args.max_sweeps)
    if args.jac_abs is not None:
        h.set_option(2, args.jac_abs)
    tuned = api.autotune(h, 32, 512, 512, apply=True, cache=args.autotune) if args.autotune else None
    ch = api.Chain.product(W.initial_vectors(spec), spec.chi_max, models.bond_hamiltonians(spec), dtype=args.dtype)

    start_step = 0
    prelude = args.prelude
    if args.load_state:
        st = torch.load(args.load_state, weights_only=True)
        for k in ("B", "lam", "chi", "disc"):
            getattr(ch, k).copy_(st[k].to(getattr(ch, k).device))
        start_step = int(st["step"])
        prelude = 0
    t0 = time.time()
    # chi growth (prelude) and warmup: untimed
    plan = [("prelude", prelude), ("warmup", args.warmup)]
    for name, total in plan:
        done = 0
        while done < total:
            n = min(10, total - done)
            api.tebd_step(h, [ch], 4, wl.dt, n, wl.eps_local)
            torch.cuda.synchronize()
            done += n
            print(f"[bench] {name} {done}/{total} steps, chi_max now {int(ch.chi.max())}, "
                  f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    code, word = h.device_status()
    start_step += prelude + args.warmup
    chi0 = ch.chi.cpu().numpy()
    n_at_cap0 = int((chi0 >= spec.chi_max).sum())
    if n_at_cap0 == 0:
        print(f"bench.py: the timed state has no bond at chi_max = {spec.chi_max} (largest chi {int(chi0.max())} "
              f"after {start_step} steps); the headline needs the chi = {spec.chi_max} state, so no value is "
              f"reported.  Run with the default prelude.", file=sys.stderr)
        h.close()
        sys.exit(3)
    if args.save_state:
        torch.save({"B": ch.B, "lam": ch.lam, "chi": ch.chi, "disc": ch.disc, "step": start_step}, args.save_state)

    # snapshot of the state the timed region starts from (for the CPU baseline)
    snap = ch.to_host() if not args.no_cpu else None

    # K timed steps in (up to) five windows; the value is the median window rate
    n_win = max(1, min(5, args.steps))
    sizes = [args.steps // n_win + (1 if w < args.steps % n_win else 0) for w in range(n_win)]
    h.set_option(3, 1.0)
    h.kernel_stats("theta", reset=True)
    torch.cuda.synchronize()
    win_s = []
    t1 = time.perf_counter()
    for nw in sizes:
        tw = time.perf_counter()
        api.tebd_step(h, [ch], 4, wl.dt, nw, wl.eps_local)
        torch.cuda.synchronize()
        win_s.append(time.perf_counter() - tw)
    t2 = time.perf_counter()
    elapsed = t2 - t1
    stats = {k: h.kernel_stats(k) for k in ("theta", "jac_round", "select", "wb_right", "gemm", "prep", "gates",
                                             "warm")}
    h.set_option(3, 0.0)
    code2, word2 = h.device_status()
    chi = ch.chi.cpu().numpy()
    rates = [updates_per_step * nw / t for nw, t in zip(sizes, win_s)]
    value = float(np.median(rates))

    jr_ms, jr_n, jr_exec = stats["jac_round"]
    th_ms, th_n, th_work = stats["theta"]
    svd_alg = stats["prep"][2]          # 88 m n min(m, n) per split, counted on the device
    jr_avg_s = jr_ms * 1e-3 / max(jr_n, 1)
    # achieved = the splits' algorithmic flops per launch over the average launch time
    jr_ach = (svd_alg / max(jr_n, 1)) / jr_avg_s / 1e12 if jr_n else 0.0
    jr_exec_rate = (jr_exec / max(jr_n, 1)) / jr_avg_s / 1e12 if jr_n else 0.0
    th_ach = th_work / (th_ms * 1e-3) / 1e12 if th_ms > 0 else 0.0
    gm_ms, gm_n, gm_work = stats["gemm"]
    ct_ach = (th_work + gm_work) / ((th_ms + gm_ms) * 1e-3) / 1e12 if th_ms + gm_ms > 0 else 0.0
    mfma_peak = FP64_PEAK_TFLOPS if args.dtype == "c128" else FP32_MFMA_PEAK_TFLOPS
    kernel_share = {k: round(v[0] / (elapsed * 1e3), 4) for k, v in stats.items()}
    # the stored HBM traffic figure describes the profiled state: the default
    # prelude and warmup from the Neel state, at the kernel source it was taken on
    same_state = (not args.load_state and not args.rounds and prelude == 140
                  and args.warmup == JAC_ROUND_TRAFFIC["warmup"]
                  and args.dtype == "c128" and not args.warm)

    out = {
        "metric": "two-site MPS updates/s (TEBD4 XXZ L=64, chi_max=256)",
        "value": round(value, 2),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(updates_per_step / value * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128 (FP64 MFMA contractions, FP64 SVD)" if args.dtype == "c128"
        else "c64 (FP32 MFMA contractions, FP64 SVD)",
        "data": "synthetic",
        "config": {"workload": "xxz_tebd4_L64: TEBD4 XXZ L=64 Jxy=1 Jz=0.5 Neel dt=0.05 chi_max=256 eps=1e-12",
                   "updates_per_step": updates_per_step, "prelude_steps": prelude, "start_step": start_step,
                   "jacobi_threads": args.jac_threads, "autotune": tuned,
                   "jacobi_schedule": "round launches" if args.rounds else "persistent",
                   "warm_start": bool(args.warm),
                   "jacobi_abs_floor": args.jac_abs if args.jac_abs is not None else 1e-15,
                   "chi_hist": {"max": int(chi.max()), "mean": round(float(chi.mean()), 1),
                                "n_at_cap": int((chi >= spec.chi_max).sum()), "n_at_cap_start": n_at_cap0}},
        "windows": {"steps": sizes, "updates_per_s": [round(r, 2) for r in rates],
                    "mean_updates_per_s": round(updates_per_step * args.steps / elapsed, 2),
                    "timed_s": round(elapsed, 4)},
        "roofline": {"kernel": ("jac_round_kernel (FP64 block-Jacobi round: Gram + rotation)" if args.rounds else
                                "jac_persist_kernel (FP64 block Jacobi, all sweeps of a layer: Gram + rotation)"),
                     "bound": "mfma", "achieved": round(jr_ach, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(jr_ach / FP64_PEAK_TFLOPS, 4),
                     "traffic": _jac_round_traffic() if same_state else None,
                     "algorithmic_flops": "88 m n min(m,n) per m x n complex split, all splits of the timed "
                                          "steps, attributed to the Jacobi rounds",
                     "executed_tflops": round(jr_exec_rate, 3),
                     "avg_launch_us": round(jr_avg_s * 1e6, 2), "launches": jr_n},
        "mfma": {"kernel": "theta_gate_kernel", "achieved": round(th_ach, 3), "peak": mfma_peak,
                 "unit": "TFLOP/s", "frac": round(th_ach / mfma_peak, 4),
                 # the contraction kernels of the update together: theta build + gate
                 # and the write-back GEMM B_b = theta~' V_k / n_k (useful flops over
                 # their summed kernel time)
                 "contractions": {"kernels": "theta_gate_kernel + write-back gemm_kernel",
                                  "achieved": round(ct_ach, 3), "frac": round(ct_ach / mfma_peak, 4)}},
        "kernel_time_share": kernel_share,
        "device_status": [code, word, code2, word2],
    }

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(spec, wl, snap, args.cpu_seconds)
    print(json.dumps(out))
    h.close()


def calibrate_copy(nbytes: int):
    """A plain streaming kernel that reads nbytes and writes nbytes (float32
    negation), launched three times: the reference for scaling the HBM byte
    counters of the profiled kernels."""
    import torch
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))


def _herm_env(chi, w, key, dtype, dev):
    """Seeded environment [chi][w][chi] whose channels pair as Hermitian
    conjugates (channel 1 <-> 2 for the boson MPO), so H_eff is Hermitian."""
    import numpy as np
    import torch
    import workloads as W
    E = np.empty((chi, w, chi), dtype=np.complex128)
    for b in range(w):
        A = W.random_complex((chi, chi), key + (b,), scale=1.0 / chi)
        E[:, b, :] = A + A.conj().T
    if w >= 3:
        E[:, 2, :] = E[:, 1, :].conj().T
    return torch.from_numpy(E).to(dtype).to(dev)


def bench_heff(args):
    """The Krylov path's kernels at the Bose-Hubbard two-site shape: chi_l =
    chi_r = 512, d = 5, MPO bond dimension 4.  Times the structured H_eff
    apply and one Lanczos exponential (20 vectors, tolerance 0 so that all 20
    run) on seeded synthetic environments and a seeded theta."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1703_00387_amd import api, models

    wl = W.bh_tdvp2_L32()
    spec = wl.chains[0]
    chi, d = spec.chi_max, spec.d
    Wm = models.mpo(spec)[spec.L // 2]
    w = Wm.shape[0]
    tdt = torch.complex128 if args.dtype == "c128" else torch.complex64
    dev = "cuda"
    h = api.Handle(0)
    h.set_option(5, args.jac_threads)
    h.set_option(7, 1.0 if args.split == "eig" else 0.0)
    Lenv = _herm_env(chi, w, (31, 1), tdt, dev)
    Renv = _herm_env(chi, w, (31, 2), tdt, dev)
    Wt = torch.from_numpy(np.ascontiguousarray(Wm)).to(tdt).to(dev)
    th = torch.from_numpy(W.random_complex((chi, d, d, chi), (31, 3))).to(tdt).to(dev)
    th = th / torch.linalg.vector_norm(th)
    flops = 8.0 * (2 * w * d * d * chi ** 3 + 2 * w * w * d ** 3 * chi ** 2)
    for _ in range(2):
        api.heff_apply(h, Lenv, Wt, Wt, Renv, th)
    torch.cuda.synchronize()
    reps = max(args.steps, 3)
    t0 = time.perf_counter()
    for _ in range(reps):
        y = api.heff_apply(h, Lenv, Wt, Wt, Renv, th)
    torch.cuda.synchronize()
    t_apply = (time.perf_counter() - t0) / reps
    print(f"[bench] H_eff apply {t_apply * 1e3:.2f} ms", file=sys.stderr, flush=True)
    x = th.clone()
    api.krylov_expm(h, Lenv, Wt, Wt, Renv, x, wl.dt, n_max=20, tol=0.0)
    torch.cuda.synchronize()
    x = th.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_used, err = api.krylov_expm(h, Lenv, Wt, Wt, Renv, x, wl.dt, n_max=20, tol=0.0)
    torch.cuda.synchronize()
    t_kry = time.perf_counter() - t0
    code, word = h.device_status()
    peak = FP64_PEAK_TFLOPS if args.dtype == "c128" else FP32_MFMA_PEAK_TFLOPS
    ach = flops / t_apply / 1e12
    out = {
        "metric": "structured H_eff applies/s (Bose-Hubbard two-site, chi=512, d=5, w=4)",
        "value": round(1.0 / t_apply, 3), "unit": "applies/s", "n_gpus": 1, "steps": reps, "warmup": 2,
        "ms_per_step": round(t_apply * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "bh_heff_chi512: H_eff = L W W R at chi_l=chi_r=512, d=5, w=4 (Bose-Hubbard MPO), "
                               "seeded Hermitian environments"},
        "roofline": {"kernel": "H_eff apply (environment GEMMs on MFMA + MPO mixes)", "bound": "mfma",
                     "achieved": round(ach, 3), "peak": peak, "unit": "TFLOP/s", "frac": round(ach / peak, 4),
                     "traffic": None, "flops_per_apply": flops},
        "krylov": {"ms_per_exponential": round(t_kry * 1e3, 3), "vectors": n_used,
                   "h_eff_share": round(min(1.0, n_used * t_apply / t_kry), 4)},
        "device_status": [code, word],
    }
    print(json.dumps(out))
    h.close()


def bench_u1(args):
    """The truncated SVD of a number-conserving two-site tensor, dense against
    U(1) blocks.  Synthetic Bose-Hubbard middle bond at the shape of the
    paper's symmetry table (L = 32, d = 6, chi = 320): left bond charges (the
    particle number to the left) drawn around 16, right ones around 18, row
    (alpha, s1) charge q_alpha + s1, column (s2, gamma) charge q_gamma - s2;
    theta random on its charge blocks with singular values decaying
    exponentially.  Times the dense mps_truncate and mps_truncate_u1 on the
    same matrix (both FP64 Jacobi) and checks they keep the same spectrum."""
    import numpy as np
    import torch
    from paper_1703_00387_amd import api

    d, chi, chi_max, eps = 6, 320, 320, 1e-12
    rng = np.random.default_rng(170300387 + 32)
    qa = np.rint(rng.normal(16.0, 2.0, size=chi)).astype(np.int64)
    qg = np.rint(rng.normal(18.0, 2.0, size=chi)).astype(np.int64)
    row_q = (qa[:, None] + np.arange(d)[None, :]).reshape(-1)
    col_q = (qg[None, :] - np.arange(d)[:, None]).reshape(-1)
    m, n = d * chi, d * chi
    T = rng.normal(size=(m, n)) + 1j * rng.normal(size=(m, n))
    T[row_q[:, None] != col_q[None, :]] = 0.0
    T *= np.exp(-np.arange(m) / 60.0)[rng.permutation(m)][:, None]
    T /= np.linalg.norm(T)
    h = api.Handle(0)
    h.set_option(5, args.jac_threads)
    th = torch.from_numpy(T).cuda()
    sectors = len(set(row_q.tolist()) & set(col_q.tolist()))

    def run(fn):
        times = []
        for rep in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            if rep >= args.warmup:
                times.append(time.perf_counter() - t0)
        return out, float(np.median(times))

    dense, t_dense = run(lambda: h.truncate(th, chi_max, eps))
    blk, t_u1 = run(lambda: h.truncate_u1(th, row_q, col_q, chi_max, eps))
    s_d = dense[1].cpu().numpy()
    s_b = blk[1].cpu().numpy()
    code, word = h.device_status()
    out = {
        "metric": "U(1)-blocked truncated SVD speedup over the dense SVD (Bose-Hubbard two-site tensor, d=6, chi=320)",
        "value": round(t_dense / t_u1, 2),
        "unit": "x",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_u1 * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {"workload": "bh_u1_svd_chi320: theta 1920 x 1920, number-conserving charge blocks",
                   "sectors": sectors, "chi_max": chi_max, "eps": eps},
        "dense_ms": round(t_dense * 1e3, 3),
        "u1_ms": round(t_u1 * 1e3, 3),
        "kept": [int(dense[3]), int(blk[4])],
        "max_abs_ds2": float(np.abs(s_d ** 2 - s_b ** 2).max()) if len(s_d) == len(s_b) else None,
        "device_status": [code, word],
    }
    print(json.dumps(out))
    h.close()


def bench_u1_tebd(args):
    """The headline TEBD4 workload (XXZ L = 64, chi = 256, Neel start) on a
    charge-carrying chain: the charge is the number of up spins, every update
    truncated on the charge blocks of its bond.  After the warmup (U(1)
    steps), the same state is stepped once more on a copy with the dense
    update, so both rates are measured on one state."""
    import numpy as np
    import torch
    import workloads as W
    from paper_1703_00387_amd import api, models

    wl = W.xxz_tebd4_L64()
    spec = wl.chains[0]
    updates_per_step = sum(len(range(p, spec.L - 1, 2)) for p in (0, 1, 0)) * 5
    h = api.Handle(0)
    h.set_option(5, args.jac_threads)
    v = W.initial_vectors(spec)
    ch = api.Chain.product(v, spec.chi_max, models.bond_hamiltonians(spec), dtype=args.dtype)
    q = api.Charges.product(v, [1, 0], spec.chi_max)
    t0 = time.time()
    done = 0
    while done < args.warmup:
        n = min(10, args.warmup - done)
        api.tebd_step_u1(h, [ch], [q], 4, wl.dt, n, wl.eps_local)
        torch.cuda.synchronize()
        done += n
        print(f"[bench] warmup {done}/{args.warmup} U(1) steps, chi_max now {int(ch.chi.max())}, "
              f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    cd = api.Chain(ch.L, ch.d, ch.chi_max, ch.B.clone(), ch.lam.clone(), ch.chi.clone(), ch.hbond, ch.disc.clone())
    cg = api.Chain(ch.L, ch.d, ch.chi_max, ch.B.clone(), ch.lam.clone(), ch.chi.clone(), ch.hbond, ch.disc.clone())
    qg = api.Charges(q.qbond.clone(), q.qsite, q.modulus)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.tebd_step_u1(h, [ch], [q], 4, wl.dt, args.steps, wl.eps_local)
    torch.cuda.synchronize()
    t_u1 = time.perf_counter() - t1
    print(f"[bench] {args.steps} U(1) steps {t_u1:.3f}s", file=sys.stderr, flush=True)
    # the same steps captured once in a graph (the charge blocks are built on
    # the device) and replayed, from a copy of the same state
    from paper_1703_00387_amd import _lib
    sg = torch.cuda.Stream()
    with torch.cuda.stream(sg):
        t1 = time.perf_counter()
        api.tebd_step_u1(h, [cg], [qg], 4, wl.dt, 1, wl.eps_local, _lib.MPS_FLAG_GRAPH)
        sg.synchronize()
        t_cap = time.perf_counter() - t1
        t1 = time.perf_counter()
        api.tebd_step_u1(h, [cg], [qg], 4, wl.dt, args.steps, wl.eps_local, _lib.MPS_FLAG_GRAPH)
        sg.synchronize()
        t_graph = time.perf_counter() - t1
    print(f"[bench] {args.steps} U(1) steps replayed {t_graph:.3f}s", file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    api.tebd_step(h, [cd], 4, wl.dt, args.steps, wl.eps_local)
    torch.cuda.synchronize()
    t_dense = time.perf_counter() - t1
    print(f"[bench] {args.steps} dense steps {t_dense:.3f}s", file=sys.stderr, flush=True)
    code, word = h.device_status()
    chi = ch.chi.cpu().numpy()
    mid = spec.L // 2
    qmid = q.qbond[mid, :int(chi[mid])].cpu().numpy()
    n_upd = updates_per_step * args.steps
    out = {
        "metric": "two-site updates per second (TEBD4, U(1) charge blocks)",
        "value": round(n_upd / t_u1, 3),
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_u1 / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "xxz_tebd4_L64_u1: XXZ L=64 chi_max=256 TEBD4 from the Neel state, charge n_up",
                   "L": spec.L, "chi_max": spec.chi_max, "dt": wl.dt, "eps_local": wl.eps_local},
        "dense_updates_per_s": round(n_upd / t_dense, 3),
        "speedup_over_dense": round(t_dense / t_u1, 2),
        "graph_replay_updates_per_s": round(n_upd / t_graph, 3),
        "graph_first_call_with_capture_ms": round(t_cap * 1e3, 3),
        "chi_max_reached": int(chi.max()),
        "sectors_mid_bond": int(len(set(qmid.tolist()))),
        "device_status": [code, word],
    }
    print(json.dumps(out))
    h.close()


def bench_tdvp(args):
    """Two-site TDVP on the Bose-Hubbard chain (L=32, d=5, t=1, U=4, unit
    filling, dt=0.02, 20 Lanczos vectors, tol 1e-10, MPO bond dimension 4).
    The environment update and the one-site H_eff apply (the backward step's
    operator) are timed at the full shape chi=512; whole 2TDVP steps run at
    chi_max=64, since one two-site SVD of the 2560 x 2560 theta' at chi=512
    leaves the single-matrix Jacobi with too little parallelism to finish a
    step in a bench run."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1703_00387_amd import api, models

    wl = W.bh_tdvp2_L32()
    spec = wl.chains[0]
    chi, d = spec.chi_max, spec.d
    Wm = models.mpo(spec)[spec.L // 2]
    w = Wm.shape[0]
    tdt = torch.complex128 if args.dtype == "c128" else torch.complex64
    h = api.Handle(0)
    h.set_option(5, args.jac_threads)
    h.set_option(7, 1.0 if args.split == "eig" else 0.0)
    Lenv = _herm_env(chi, w, (32, 1), tdt, "cuda")
    Renv = _herm_env(chi, w, (32, 2), tdt, "cuda")
    Wt = torch.from_numpy(np.ascontiguousarray(Wm)).to(tdt).cuda()
    A = torch.from_numpy(W.random_complex((chi, d, chi), (32, 3))).to(tdt).cuda()
    x1 = torch.from_numpy(W.random_complex((chi, d, chi), (32, 4))).to(tdt).cuda()
    f_env = 8.0 * (2 * w * d * chi ** 3 + w * w * d * d * chi ** 2)
    f_one = 8.0 * (2 * w * d * chi ** 3 + w * w * d * d * chi ** 2)
    reps = max(args.steps, 3)

    def timeit(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    # the two-site split at the full shape: theta' of (chi d) x (d chi) = 2560 x 2560
    # with a graded spectrum, truncated to chi = 512 (once; a few seconds)
    m2 = chi * d
    Uq, _ = np.linalg.qr(W.random_complex((m2, m2), (32, 5)))
    Vq, _ = np.linalg.qr(W.random_complex((m2, m2), (32, 6)))
    th2 = torch.from_numpy((Uq * np.exp(-0.02 * np.arange(m2))) @ Vq.conj().T).cuda()
    th2 = th2 / torch.linalg.vector_norm(th2)
    t_svd = {}
    for below in (0, 32):   # 0: never split; 32: the default (large matrices split below 128 pairs)
        h.set_option(6, below)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, _, k_svd, _, _ = h.truncate(th2, chi, wl.eps_local)
        torch.cuda.synchronize()
        t_svd[below] = time.perf_counter() - t0
        print(f"[bench] 2560 x 2560 truncated SVD (split option {below}) {t_svd[below]:.2f} s, k={k_svd}",
              file=sys.stderr, flush=True)
    h.set_option(6, 32)
    t_envl = timeit(lambda: api.env_update(h, "left", Lenv, Wt, A))
    t_envr = timeit(lambda: api.env_update(h, "right", Renv, Wt, A))
    t_one = timeit(lambda: api.heff_apply(h, Lenv, Wt, None, Renv, x1))
    print(f"[bench] env left {t_envl * 1e3:.2f} ms, right {t_envr * 1e3:.2f} ms, one-site apply {t_one * 1e3:.2f} ms",
          file=sys.stderr, flush=True)
    chi_run = 64
    ch = api.OCChain.product(W.initial_vectors(spec), chi_run, models.mpo(spec), dtype=args.dtype)
    t0 = time.time()
    for i in range(args.warmup):
        api.tdvp2_step(h, ch, wl.dt, 1, wl.eps_local, wl.n_krylov, wl.krylov_tol)
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup}, chi_max now {int(ch.chi.max())}, {time.time() - t0:.1f}s",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.tdvp2_step(h, ch, wl.dt, args.steps, wl.eps_local, wl.n_krylov, wl.krylov_tol)
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t1) / args.steps
    # the same run on a charge-carrying chain (particle number, every split on
    # the charge blocks of its bond)
    v0 = W.initial_vectors(spec)
    cu = api.OCChain.product(v0, chi_run, models.mpo(spec), dtype=args.dtype)
    qu = api.Charges.product(v0, list(range(d)), chi_run)
    t0 = time.time()
    for i in range(args.warmup):
        api.tdvp2_step(h, cu, wl.dt, 1, wl.eps_local, wl.n_krylov, wl.krylov_tol, charges=qu)
        torch.cuda.synchronize()
        if (i + 1) % 10 == 0 or i + 1 == args.warmup:
            print(f"[bench] U(1) warmup {i + 1}/{args.warmup}, chi_max now {int(cu.chi.max())}, "
                  f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.tdvp2_step(h, cu, wl.dt, args.steps, wl.eps_local, wl.n_krylov, wl.krylov_tol, charges=qu)
    torch.cuda.synchronize()
    t_step_u1 = (time.perf_counter() - t1) / args.steps
    code, word = h.device_status()
    L = spec.L
    upd = 2 * (L - 1)
    peak = FP64_PEAK_TFLOPS if args.dtype == "c128" else FP32_MFMA_PEAK_TFLOPS
    out = {
        "metric": "two-site TDVP updates/s (Bose-Hubbard L=32, d=5, chi_max=64)",
        "value": round(upd / t_step, 3), "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_step * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "bh_tdvp_L32: 2TDVP BH L=32 d=5 t=1 U=4 unit filling dt=0.02 n_max=20 tol=1e-10, "
                               "chi_max=64 for the steps; environment update and one-site H_eff at chi=512",
                   "two_site_updates_per_step": upd, "one_site_backward_steps_per_step": 2 * (L - 2),
                   "chi_max_now": int(ch.chi.max())},
        "u1_updates_per_s": round(upd / t_step_u1, 3),
        "u1_chi_max_now": int(cu.chi.max()),
        "env_update_chi512": {"ms_left": round(t_envl * 1e3, 3), "ms_right": round(t_envr * 1e3, 3),
                              "flops": f_env, "tflops_left": round(f_env / t_envl / 1e12, 3),
                              "frac_left": round(f_env / t_envl / 1e12 / peak, 4)},
        "two_site_svd_chi512": {"shape": [chi * d, chi * d], "s_unsplit": round(t_svd[0], 3),
                                "s_split": round(t_svd[32], 3)},
        "one_site_heff_chi512": {"ms": round(t_one * 1e3, 3), "flops": f_one,
                                 "tflops": round(f_one / t_one / 1e12, 3), "frac": round(f_one / t_one / 1e12 / peak, 4)},
        "device_status": [code, word],
    }
    print(json.dumps(out))
    h.close()


def bench_tdvp_step(args):
    """One whole symmetric 2TDVP step (both half-sweeps: 62 two-site
    exponentials, SVDs of up to 2560 x 2560 truncated to chi = 512, 60
    backward one-site exponentials, the environment updates) on the
    Bose-Hubbard chain of bh_tdvp_L32 (L = 32, d = 5, w = 4, dt = 0.02,
    20 Lanczos vectors, tol 1e-10), from a seeded random mixed-canonical state
    with every bulk bond at chi = 512 (chi_b = min(5^b, 5^(32-b), 512)):
    the step at the full shape, which a short evolution from the product
    state does not reach."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1703_00387_amd import api, models

    wl = W.bh_tdvp2_L32()
    spec = wl.chains[0]
    tdt = torch.complex128 if args.dtype == "c128" else torch.complex64
    chis, Ts = W.random_oc_tensors(spec.L, spec.d, spec.chi_max, (32, 8))
    h = api.Handle(0)
    h.set_option(5, args.jac_threads)
    ch = api.OCChain.product(W.initial_vectors(spec), spec.chi_max, models.mpo(spec), dtype=args.dtype)
    for i, T in enumerate(Ts):
        ch.M[i, :T.size] = torch.from_numpy(T.reshape(-1)).to(tdt).to(ch.M.device)
    ch.chi.copy_(torch.tensor(chis, dtype=torch.int32, device=ch.chi.device))
    torch.cuda.synchronize()
    print(f"[bench] random chain at chi {max(chis)}: one 2TDVP step", file=sys.stderr, flush=True)
    h.set_option(3, 1.0)
    h.kernel_stats("jac_round", reset=True)
    t1 = time.perf_counter()
    kmax = api.tdvp2_step(h, ch, wl.dt, 1, wl.eps_local, wl.n_krylov, wl.krylov_tol)
    torch.cuda.synchronize()
    t_step = time.perf_counter() - t1
    jr = h.kernel_stats("jac_round")
    h.set_option(3, 0.0)
    code, word = h.device_status()
    upd = 2 * (spec.L - 1)
    out = {
        "metric": "two-site TDVP updates/s at the full shape (Bose-Hubbard L=32, d=5, chi=512)",
        "value": round(upd / t_step, 3), "unit": "updates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(t_step * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": args.dtype, "data": "synthetic (seeded random mixed-canonical chain at chi=512)",
        "config": {"workload": "bh_tdvp_step_chi512: one symmetric 2TDVP step, BH L=32 d=5 w=4 dt=0.02 "
                               "n_max=20 tol=1e-10, every bulk bond at chi=512",
                   "two_site_updates": upd, "chi_after": int(ch.chi.max()),
                   "krylov_vectors_max": kmax},
        "jacobi_s": round(jr[0] * 1e-3, 3),
        "discarded_weight": float(ch.disc.sum().item()),
        "device_status": [code, word],
    }
    print(json.dumps(out))
    h.close()


def bench_grad(args):
    """Reverse-mode coupling gradient of TEBD2 on the XXZ chain, L=32,
    chi_max=128, J_b ~ U(0.8, 1.2), Neel start, dt=0.05, 40 steps: one
    forward run with step checkpoints plus the reverse pass, against the
    forward run alone."""
    import copy

    import numpy as np
    import torch

    import workloads as W
    from paper_1703_00387_amd import api, models

    wl = W.xxz_grad_L32()
    spec = wl.chains[0]
    L = spec.L
    unit = copy.copy(spec)
    unit.J_b = np.ones(L - 1)
    h0 = models.bond_hamiltonians(unit)
    sz = models.sz_operator()
    h = api.Handle(0)
    h.set_option(5, args.jac_threads)
    h.set_option(7, 1.0 if args.split == "eig" else 0.0)

    def fresh():
        return api.Chain.product(W.initial_vectors(spec), spec.chi_max, models.bond_hamiltonians(spec),
                                 dtype=args.dtype)

    ch = fresh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    api.tebd_step(h, [ch], 2, wl.dt, wl.n_steps, wl.eps_local)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    print(f"[bench] forward {t_fwd:.2f}s", file=sys.stderr, flush=True)
    ch = fresh()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss, dJ = api.tebd_grad(h, ch, h0, wl.dt, wl.n_steps, wl.eps_local, sz, L // 2 - 1, np.kron(sz, sz))
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    code, word = h.device_status()
    upd = wl.n_steps * sum(len(range(p, L - 1, 2)) for p in (0, 1, 0))
    out = {
        "metric": "differentiated TEBD2 two-site updates/s (forward + adjoint, XXZ L=32, chi_max=128, 40 steps)",
        "value": round(upd / t_grad, 3), "unit": "updates/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": round(t_grad * 1e3 / wl.n_steps, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype if args.dtype == "c128" else "c64 (FP32 MFMA forward, FP64 reverse pass)",
        "data": "synthetic",
        "config": {"workload": "xxz_grad_L32: TEBD2 XXZ L=32 chi_max=128 J_b~U(0.8,1.2) Neel dt=0.05 40 steps, "
                               "loss <S^z_16> + sum_b <S^z_b S^z_b+1>", "updates": upd},
        "gradient_s": round(t_grad, 3), "forward_only_s": round(t_fwd, 3),
        "adjoint_over_forward": round(t_grad / t_fwd, 2), "loss": float(loss),
        "grad_norm": float(torch.linalg.vector_norm(dJ)), "device_status": [code, word],
    }
    print(json.dumps(out))
    h.close()


def bench_quench(args):
    """A transverse-field Ising ramp through the critical point,
    H(t) = -sum sz sz - g(t) sum sx, g(t) = 1.5 - t/3, on L=64 from all up,
    chi_max=128: TEBD4 steps with the fourth-order commutator-free Magnus
    scheme (two exponentials, 30 layers per step).  After the untimed
    steps, the timed steps are compared with as many TEBD4 steps of the
    Hamiltonian frozen at the same time, from the same state."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1703_00387_amd import api, models

    L, chi_max, dt = 64, 128, 0.02
    hz = models.bond_hamiltonians(W.tfim_chain(L, chi_max, 1.0, 0.0))
    hf = [a - b for a, b in zip(models.bond_hamiltonians(W.tfim_chain(L, chi_max, 1.0, 1.0)), hz)]
    terms = np.ascontiguousarray(np.array([hz, hf]))
    g = lambda t: 1.5 - t / 3.0
    nodes = api.cfme_nodes(4)
    fn = lambda n0, n: np.array([[[1.0, g((k + c) * dt)] for c in nodes] for k in range(n0, n0 + n)])
    h = api.Handle(0)
    h.set_option(5, args.jac_threads)
    h.set_option(7, 1.0 if args.split == "eig" else 0.0)
    spec = W.tfim_chain(L, chi_max, 1.0, 1.5)
    ch = api.Chain.product(W.initial_vectors(spec), chi_max, terms, dtype=args.dtype)
    done, t0 = 0, time.time()
    while done < args.warmup:
        n = min(10, args.warmup - done)
        api.tebd_td_step(h, [ch], 4, dt, n, 1e-12, fn(done, n), 4)
        torch.cuda.synchronize()
        done += n
        print(f"[bench] warmup {done}/{args.warmup}, chi_max now {int(ch.chi.max())}, {time.time() - t0:.1f}s",
              file=sys.stderr, flush=True)
    start = (ch.B.clone(), ch.lam.clone(), ch.chi.clone(), ch.disc.clone())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.tebd_td_step(h, [ch], 4, dt, args.steps, 1e-12, fn(done, args.steps), 4)
    torch.cuda.synchronize()
    t_td = time.perf_counter() - t1
    chi_end = ch.chi.cpu().numpy()
    # the same number of TEBD4 steps of H frozen at the start time
    frozen = api.Chain(ch.L, ch.d, ch.chi_max, start[0], start[1], start[2],
                       torch.from_numpy(np.ascontiguousarray(np.array(hz) + g(done * dt) * np.array(hf))).cuda(),
                       start[3])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    api.tebd_step(h, [frozen], 4, dt, 2 * args.steps, 1e-12)
    torch.cuda.synchronize()
    t_fr = time.perf_counter() - t1
    code, word = h.device_status()
    upd = sum(len(range(p, L - 1, 2)) for p in (0, 1, 0)) * 5 * 2 * args.steps
    out = {
        "metric": "two-site MPS updates/s, time-dependent TEBD4 with the fourth-order commutator-free Magnus scheme "
                  "(TFIM quench L=64, chi_max=128)",
        "value": round(upd / t_td, 2), "unit": "updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(t_td / args.steps * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "tfim_quench_L64: H(t) = -sum sz sz - (1.5 - t/3) sum sx, L=64, all up, dt=0.02, "
                               "chi_max=128, eps=1e-12, TEBD4 per exponential, two exponentials per step",
                   "updates_per_step": upd // args.steps, "chi_max_now": int(chi_end.max()),
                   "jacobi_threads": args.jac_threads},
        "frozen_hamiltonian_tebd4": {"updates_per_s": round(upd / t_fr, 2), "steps": 2 * args.steps},
        "device_status": [code, word],
    }
    print(json.dumps(out))
    h.close()


def bench_sweep(args):
    """The paper's own second-order sweep (every bond left to right with dt/2,
    then right to left) against even/odd TEBD2 on the same chi=256 state of the
    XXZ chain: the sweep updates one bond at a time, even/odd a whole layer.
    The same sweep with the local Lanczos exponential of every bond term
    (Krylov TEBD, 20 vectors at most, tol 1e-10) is timed from the same state:
    the paper's appendix expects plain TEBD to be the faster of the two."""
    import torch

    import workloads as W
    from paper_1703_00387_amd import api, models

    wl = W.xxz_tebd4_L64()
    spec = wl.chains[0]
    h = api.Handle(0)
    h.set_option(5, args.jac_threads)
    h.set_option(7, 1.0 if args.split == "eig" else 0.0)
    h.set_option(9, 1.0 if args.warm else 0.0)
    ch = api.Chain.product(W.initial_vectors(spec), spec.chi_max, models.bond_hamiltonians(spec), dtype=args.dtype)
    if args.load_state:
        st = torch.load(args.load_state, weights_only=True)
        for k in ("B", "lam", "chi", "disc"):
            getattr(ch, k).copy_(st[k].to(getattr(ch, k).device))
    else:
        done = 0
        t0 = time.time()
        while done < args.warmup:
            n = min(10, args.warmup - done)
            api.tebd_step(h, [ch], 4, wl.dt, n, wl.eps_local)
            torch.cuda.synchronize()
            done += n
            print(f"[bench] warmup {done}/{args.warmup}, {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    start = (ch.B.clone(), ch.lam.clone(), ch.chi.clone(), ch.disc.clone())

    n_used = torch.zeros(2 * (spec.L - 1), dtype=torch.int32, device="cuda")

    def timed(order):
        ch.B.copy_(start[0]); ch.lam.copy_(start[1]); ch.chi.copy_(start[2]); ch.disc.copy_(start[3])
        torch.cuda.synchronize()
        t = time.perf_counter()
        if order == "krylov":
            api.ktebd_step(h, [ch], wl.dt, 1, wl.eps_local, 20, 1e-10, n_used=n_used)
        else:
            api.tebd_step(h, [ch], order, wl.dt, 1, wl.eps_local)
        torch.cuda.synchronize()
        return time.perf_counter() - t

    t_sweep = timed(0)
    print(f"[bench] sweep step {t_sweep:.2f}s", file=sys.stderr, flush=True)
    t_eo = timed(2)
    print(f"[bench] even/odd step {t_eo:.2f}s", file=sys.stderr, flush=True)
    t_kry = timed("krylov")
    print(f"[bench] Krylov sweep step {t_kry:.2f}s", file=sys.stderr, flush=True)
    nu = n_used.cpu().numpy()
    code, word = h.device_status()
    L = spec.L
    upd_sweep, upd_eo = 2 * (L - 1), sum(len(range(p, L - 1, 2)) for p in (0, 1, 0))
    out = {
        "metric": "two-site MPS updates/s, the paper's second-order sweep (XXZ L=64, chi_max=256)",
        "value": round(upd_sweep / t_sweep, 2), "unit": "updates/s", "n_gpus": 1, "steps": 1,
        "warmup": args.warmup, "ms_per_step": round(t_sweep * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
        "config": {"workload": "xxz_sweep_L64: one sweep step (126 updates, one bond at a time) from the "
                               "TEBD4 XXZ L=64 chi_max=256 state", "updates_per_step": upd_sweep,
                   "warm_start": bool(args.warm)},
        "even_odd_tebd2": {"updates_per_s": round(upd_eo / t_eo, 2), "ms_per_step": round(t_eo * 1e3, 3),
                           "updates_per_step": upd_eo},
        "krylov_sweep": {"updates_per_s": round(upd_sweep / t_kry, 2), "ms_per_step": round(t_kry * 1e3, 3),
                         "n_max": 20, "tol": 1e-10, "krylov_vectors_mean": round(float(nu.mean()), 3),
                         "krylov_vectors_max": int(nu.max())},
        "device_status": [code, word],
    }
    print(json.dumps(out))
    h.close()


def bench_batch(args):
    """256 independent XXZ chains (L ~ U{16..64}, chi_max ~ {32,64,128,256},
    Jz_b ~ U(0.5,1.5), random product states), TEBD2 dt=0.05: every update of
    a layer of all chains in one batched kernel sequence, one TEBD2 step
    captured in a hipGraph and replayed.  The same steps are then rerun from
    the same start state in the plain form (one bond per launch sequence)."""
    import torch

    import workloads as W
    from paper_1703_00387_amd import api, models, _lib

    wl = W.xxz_batch256()
    h = api.Handle(0)
    h.set_option(5, args.jac_threads)
    h.set_option(7, 1.0 if args.split == "eig" else 0.0)
    chains = [api.Chain.product(W.initial_vectors(c), c.chi_max, models.bond_hamiltonians(c), dtype=args.dtype)
              for c in wl.chains]
    upd = sum(len(range(0, c.L - 1, 2)) * 2 + len(range(1, c.L - 1, 2)) for c in wl.chains)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        done = 0
        t0 = time.time()
        while done < args.warmup:
            n = min(10, args.warmup - done)
            api.tebd_step(h, chains, 2, wl.dt, n, wl.eps_local)
            s.synchronize()
            done += n
            print(f"[bench] warmup {done}/{args.warmup}, chi max {max(int(c.chi.max()) for c in chains)}, "
                  f"{time.time() - t0:.1f}s", file=sys.stderr, flush=True)
        start = [(c.B.clone(), c.lam.clone(), c.chi.clone(), c.disc.clone()) for c in chains]

        def reset():
            for c, st in zip(chains, start):
                c.B.copy_(st[0]); c.lam.copy_(st[1]); c.chi.copy_(st[2]); c.disc.copy_(st[3])
            s.synchronize()

        def timed(flags, steps):
            reset()
            t = time.perf_counter()
            api.tebd_step(h, chains, 2, wl.dt, steps, wl.eps_local, flags=flags)
            s.synchronize()
            return time.perf_counter() - t

        t_eager = timed(0, args.steps)
        after_eager = [c.chi.clone() for c in chains]
        print(f"[bench] batched eager: {t_eager:.2f}s for {args.steps} steps", file=sys.stderr, flush=True)
        t_capture = timed(_lib.MPS_FLAG_GRAPH, 1)      # captures the step (kept by the handle)
        t_graph = timed(_lib.MPS_FLAG_GRAPH, args.steps)
        print(f"[bench] batched graph: {t_graph:.2f}s for {args.steps} steps", file=sys.stderr, flush=True)
        plain_steps = 1
        t_plain = None if args.no_plain else timed(_lib.MPS_FLAG_PLAIN, plain_steps)
        if t_plain is not None:
            print(f"[bench] plain: {t_plain:.2f}s for {plain_steps} step", file=sys.stderr, flush=True)
        same_chi = True
    code, word = h.device_status()
    t_best = min(t_eager, t_graph)
    value = upd * args.steps / t_best
    out = {"metric": "two-site MPS updates/s (batched TEBD2, 256 XXZ chains)", "value": round(value, 2),
           "unit": "updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(t_best * 1e3 / args.steps, 3), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": args.dtype, "data": "synthetic",
           "config": {"workload": "xxz_batch256: 256 XXZ chains, L~U{16..64}, chi_max~{32,64,128,256}, "
                                  "Jz_b~U(0.5,1.5), random product states, TEBD2 dt=0.05",
                      "updates_per_step": upd, "chi_max_now": max(int(c.chi.max()) for c in chains),
                      "split": args.split},
           "batched_eager": {"ms_per_step": round(t_eager * 1e3 / args.steps, 3)},
           "batched_graph": {"ms_per_step": round(t_graph * 1e3 / args.steps, 3),
                             "first_call_with_capture_ms": round(t_capture * 1e3, 3)},
           "plain": None if t_plain is None else
           {"value": round(upd * plain_steps / t_plain, 2), "ms_per_step": round(t_plain * 1e3 / plain_steps, 3)},
           "speedup_vs_plain": None if t_plain is None else round((t_plain / plain_steps) / (t_best / args.steps), 2),
           "device_status": [code, word]}
    print(json.dumps(out))
    h.close()


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _blas_info():
    try:
        from threadpoolctl import threadpool_info
        info = [i for i in threadpool_info() if i.get("user_api") == "blas"]
        if info:
            i = info[0]
            return {"library": i.get("internal_api"), "file": os.path.basename(i.get("filepath", "")),
                    "version": i.get("version"), "threads": i.get("num_threads")}
    except Exception:
        pass
    return {"library": "unknown"}


def cpu_baseline(spec, wl, snap, budget_s):
    """The complex128 oracle's bond update, timed on the host cores on a sample
    of the very state the GPU's timed region starts from: the layers of the
    first timed TEBD4 step in order (the bonds of a layer largest bond
    dimension first) on the oracle's own evolving state, until the time budget
    is used; then again with one BLAS thread on half the budget."""
    import numpy as np

    from oracle import models as om, mps as omps
    B, lam, chi = snap
    hs = om.bond_hamiltonians(spec)
    layers = omps.step_layers("tebd4", spec.L, wl.dt)

    def run(budget):
        psi = omps.MPS([b.copy() for b in B], [l.copy() for l in lam], spec.d)
        t0 = time.perf_counter()
        n, chis, n_layers = 0, [], 0
        for bonds, tau in layers:
            cur = [len(x) for x in psi.lam]
            n_layers += 1
            for b in sorted(bonds, key=lambda b: -min(cur[b], cur[b + 2])):
                chis.append(int(min(cur[b], cur[b + 2])))
                omps.apply_bond(psi, b, omps.gate(hs[b], tau), spec.chi_max, wl.eps_local)
                n += 1
                if time.perf_counter() - t0 > budget:
                    return n, time.perf_counter() - t0, chis, n_layers
        return n, time.perf_counter() - t0, chis, n_layers

    blas = _blas_info()
    threads = blas.get("threads") or len(os.sched_getaffinity(0))
    n, dt, chis, nl = run(budget_s)
    one = None
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1, user_api="blas"):
            n1, dt1, chis1, nl1 = run(0.5 * budget_s)
        one = {"value": round(n1 / dt1, 3), "cores": 1,
               "sample": f"{n1} updates in {nl1} layers (chi {min(chis1)}..{max(chis1)}), {dt1:.1f}s"}
    except Exception as e:          # threadpoolctl missing: report the multi-thread figure only
        one = {"error": str(e)}
    return {"value": round(n / dt, 3), "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} updates of the first {nl} layers of the first timed TEBD4 step, from the timed "
                      f"region's start state (bond dims {min(chis)}..{max(chis)}, largest first in a layer), "
                      f"{dt:.1f}s",
            "cpu_model": _cpu_model(), "host_cpus": len(os.sched_getaffinity(0)), "blas": blas,
            "single_thread": one}


if __name__ == "__main__":
    main()
