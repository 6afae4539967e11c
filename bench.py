"""Throughput of the Synch-EM iteration on one MI355X.

Default workload: windowed Synch-EM on N=100000 observations of D=512 steerable coefficients
(K=32 angular x Q=16 radial), L=360 rotations, a window of W=49 offsets (+-3 sigma of an 8 degree
post-synchronisation error), learned histogram prior with gamma=100.  One step is one EM
iteration over all N observations (E-step correlations, prior-weighted posterior, fused M-step
accumulation, FP64 finalize).  The headline runs the factored E-step in FP32: the correlations
through the per-frequency sums c_jk = sum_q conj(v_jkq) a_kq, an exact rewrite of the contraction
against the W rotated templates, with FP32 arithmetic on FP32 observations.  The same run times
the contraction itself as a correlation GEMM (bf16 split precision: observations and template
each bf16 hi+lo, three products, FP32 accumulation; and fp16), the factored E-step on bf16 hi+lo
and fp16 observations, the refined-resolution window, the plain full-search FP32 EM (all 360
rotations, uniform prior; correlation GEMM and factored), Synchronize and Match, and the FP64 CPU
oracle on the host cores.

Prints one JSON line.  --gpus N with N > 1 is refused: the path runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "EM iter/s and obs·rotations/s, windowed BF16 vs full FP32, at rel err ≤1e-3"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    with open(os.path.join(ROOT, "paper_2105_07372_amd", "csrc", "em_kernels.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def pmc_traffic(variant: str, launches_bytes: float):
    """HBM bytes per launch from the committed rocprofv3 counter summary of this kernel variant,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
        e = d.get(variant)
        if not e or e.get("kernel_source_sha") != kernel_source_hash():
            return None
        return float(e["hbm_bytes_per_launch"])
    except Exception:
        return None


def time_em(em, steps: int, warmup: int, state0):
    import torch
    em.step(warmup)
    em.set_state(*state0)
    em.pass_time(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    em.step(steps, sync=False)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms, n = em.pass_time(reset=True)
    return dt, (ms / n if n else float("nan")), n


def cpu_baseline(V, a0, rb, s2, w, lo, W, budget_s: float):
    """The FP64 oracle, as it stands, on the host cores: whole EM iterations over all N rows
    until about budget_s seconds have been spent (at least one)."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()
                       if p.get("user_api") == "blas"] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    offs = oracle.offsets(lo, W)
    a, rho = a0.copy(), rb.copy()
    t0 = time.perf_counter()
    its, first = 0, None
    while True:
        it = oracle.em_iteration(V, a, rho, s2, w.kbar, w.L, offs, rho_bar=rb, gamma=w.gamma)
        first = it if first is None else first
        a, rho = it["a"], it["rho"]
        its += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": its / dt, "unit": "iter/s", "cores": int(threads), "kind": "oracle",
            "obs_rot_per_s": its / dt * w.N * W,
            "sample": f"{its} full EM iterations of the same workload (N={w.N}, W={W}) from a_0; "
                      f"FP64 numpy, BLAS threads={threads}"}, first


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    # untimed EM iterations before each timed run: a few milliseconds of work bring the GPU
    # from idle to its sustained clocks (5 warm-up steps left the first timed run ~10% slow)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="fp32",
                    choices=["fp32", "bf16x3", "fp16", "bf16", "fp64"])
    ap.add_argument("--correlation", action="store_true",
                    help="run the headline with the correlation GEMM against the rotated "
                         "templates instead of the factored E-step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-baseline", action="store_true", help="skip the full-search FP32 run")
    ap.add_argument("--no-sync", action="store_true", help="skip the Synchronize-and-Match timing")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (calibrates the HBM "
                         "byte counters of a profiler run) and exit")
    args = ap.parse_args()
    if args.precision == "fp64":
        args.correlation = True          # the factored pass runs on the matrix-core precisions
    if args.gpus != 1:
        print(f"bench.py: the path runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU form would split the observations and all-reduce the FP64 "
              "M-step partials once per iteration)", file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as wl
    from paper_2105_07372_amd import EM, learn_prior

    dev = torch.device("cuda:0")
    if args.copy_probe:
        n = args.copy_probe * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4,
                          "launches": 3}))
        return
    w = wl.WORKLOADS["c3"]
    lo, W = w.window
    log(f"bench: generating workload {w.name} N={w.N} D={w.D} L={w.L} W={W}")
    a_true = wl.image(w, 0)
    V = wl.observations(w, 0, a=a_true)
    s2 = wl.noise_variance(a_true, w.snr)
    obs = torch.from_numpy(V.astype(np.complex64)).to(dev)
    err = torch.from_numpy(wl.prior_error_draws(w, 0)).to(dev)
    rb, _, nin = learn_prior(err, w.L, lo, W)
    a0 = V.astype(np.complex64).astype(np.complex128).mean(axis=0)

    # --- headline: windowed, learned prior, gamma = 100
    em = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, window=(lo, W), prior=rb, gamma=w.gamma,
            precision=args.precision, timing=True, factored=not args.correlation)
    info = em.info()
    log(f"bench: windowed {args.precision} {info}")
    dt, pass_ms, nlaunch = time_em(em, args.steps, args.warmup, (a0, rb, 0))
    iters_s = args.steps / dt
    em.set_state(a0, rb, 0)
    wq, amq, _ = em.posterior(0, 2000)
    wq, amq = wq.cpu().numpy().astype(np.float64), amq.cpu().numpy()
    em.step(1)
    a_gpu1, rho_gpu1, _ = em.state()
    ll_gpu0 = em.stats()[-1, 1]
    em.close()
    log(f"bench: windowed {iters_s:.1f} it/s, pass {pass_ms * 1e3:.1f} us")

    variants = {}
    # the correlation GEMM against the W rotated templates (the contraction as stated), and the
    # factored E-step (per-frequency sums, an exact rewrite of it) in the other precisions
    runs = [(f"windowed_correlation_{p}", dict(precision=p)) for p in ("bf16x3", "fp16")
            if not (args.correlation and p == args.precision)]
    runs += [(f"windowed_factored_{p}", dict(precision=p, factored=True))
             for p in ("fp32", "bf16x3", "fp16") if args.correlation or p != args.precision]
    # the refined-resolution window (Section III-C): as many angles as the window, sampled at
    # half-degree steps over the central +-12 degrees, prior shaped like the rotation law there
    ang = (np.arange(W) - W // 2) * np.pi / w.L
    rb_ang = np.exp(-0.5 * (np.degrees(ang) / w.rot_std_deg) ** 2)
    rb_ang /= rb_ang.sum()
    runs += [("windowed_refined_bf16x3", dict(precision="bf16x3", angles=ang, prior=rb_ang))]
    for name, kw in runs:
        kw = dict(kw)
        pr = kw.pop("prior", rb)
        if "angles" not in kw:
            kw["window"] = (lo, W)
        e2 = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, prior=pr, gamma=w.gamma, timing=True, **kw)
        d2, p2, _ = time_em(e2, args.steps, args.warmup, (a0, pr, 0))
        variants[name] = {"iter_per_s": args.steps / d2, "pass_us": p2 * 1e3,
                          "kernel": e2.info()["kernel"],
                          "hbm_frac": float(w.N) * e2.info()["bytes_per_row"] / (p2 * 1e-3) / 1e9
                          / HBM_PEAK_GBS}
        e2.close()
        log(f"bench: {name} {variants[name]['iter_per_s']:.1f} it/s")

    baseline = None
    if not args.no_baseline:
        w2 = wl.WORKLOADS["c2"]
        ef = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, precision="fp32", timing=True,
                a0=wl.random_init(w2, 0))
        nsteps, nwarm = max(5, args.steps // 5), max(2, args.warmup // 10)
        df, pf, _ = time_em(ef, nsteps, nwarm, (wl.random_init(w2, 0), np.full(w.L, 1.0 / w.L), 0))
        baseline = {"workload": "plain full-search EM, FP32 MFMA, same N, D, all L=360 "
                                "rotations, uniform prior",
                    "iter_per_s": nsteps / df, "obs_rot_per_s": nsteps / df * w.N * w.L,
                    "pass_us": pf * 1e3, "kernel": ef.info()["kernel"]}
        ef.close()
        log(f"bench: full search fp32 {baseline['iter_per_s']:.1f} it/s")
        ef = EM(obs, K=w.K, Q=w.Q, L=w.L, sigma2=s2, precision="fp32", timing=True,
                a0=wl.random_init(w2, 0), factored=True)
        df, pf, _ = time_em(ef, nsteps, nwarm, (wl.random_init(w2, 0), np.full(w.L, 1.0 / w.L), 0))
        variants["full_search_factored_fp32"] = {"iter_per_s": nsteps / df, "pass_us": pf * 1e3,
                                                 "kernel": ef.info()["kernel"]}
        ef.close()

    # Synchronize and Match (the step before the path) on the same observations: P = 1024,
    # L = 360, 50 power iterations; each stage's wall time (each call synchronises) and the
    # matrix-core rate of the two contractions
    if not args.no_sync:
        from paper_2105_07372_amd import nearest, ppm, relative_rotations, sync_match
        P_s, it_s = 1024, 50
        sync_match(obs, w.K, w.Q, w.L, P_s, it_s)                     # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rel_s, _, _ = relative_rotations(obs, w.K, w.Q, w.L, P_s)
        t1 = time.perf_counter()
        ppm(rel_s, w.L, it_s)
        t2 = time.perf_counter()
        nearest(obs, w.K, w.Q, P_s)
        t3 = time.perf_counter()
        sync_match(obs, w.K, w.Q, w.L, P_s, it_s)
        t4 = time.perf_counter()
        Lp, K2 = (w.L + 15) // 16 * 16, (2 * w.K + 3) // 4 * 4
        f_rel = 2.0 * P_s * P_s * K2 * Lp                            # MFMA flops of the L-grid step
        f_nn = 2.0 * w.N * P_s * 2 * w.D                             # MFMA flops of the distances
        variants["sync_match"] = {
            "workload": f"Synchronize and Match N={w.N} D={w.D} L={w.L} P={P_s}, {it_s} power "
                        "iterations, FP32 matrix cores (power method FP64)",
            "total_ms": (t4 - t3) * 1e3, "relative_rotations_ms": (t1 - t0) * 1e3,
            "ppm_ms": (t2 - t1) * 1e3, "nearest_ms": (t3 - t2) * 1e3,
            "relative_rotations_tflops": f_rel / (t1 - t0) / 1e12,
            "nearest_tflops": f_nn / (t3 - t2) / 1e12, "fp32_mfma_peak_tflops": 157.3}
        log(f"bench: sync_match {variants['sync_match']['total_ms']:.1f} ms")

    cpu = None
    acc = None
    if not args.no_cpu:
        log("bench: CPU oracle leg")
        import oracle
        cpu, first = cpu_baseline(V, a0, rb, s2, w, lo, W, args.cpu_budget)
        wo, _, _ = oracle.estep(V[:2000], a0, rb, s2, w.kbar, w.L, oracle.offsets(lo, W))
        ao, mo = oracle.argmax_margin(wo)
        sure = mo > 1e-3
        acc = {"a_rel": float(np.linalg.norm(a_gpu1 - first["a"]) / np.linalg.norm(first["a"])),
               "rho_maxabs": float(np.abs(rho_gpu1 - first["rho"]).max()),
               "ll_rel": float(abs(ll_gpu0 - first["ll"]) / abs(first["ll"])),
               "posterior_maxabs_2000_rows": float(np.abs(wq - wo).max()),
               "posterior_frob_rel_2000_rows": float(np.linalg.norm(wq - wo) / np.linalg.norm(wo)),
               "argmax_mismatch_margin_gt_1e-3": int(np.sum(amq[sure] != ao[sure]))}

    bytes_per_launch = float(w.N) * info["bytes_per_row"]
    achieved = bytes_per_launch / (pass_ms * 1e-3) / 1e9
    traffic = pmc_traffic(info["kernel"], bytes_per_launch)
    out = {
        "metric": METRIC,
        "value": iters_s,
        "unit": "iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # the arithmetic: the factored E-step computes in FP32 whatever the observations' storage
        # the arithmetic: the factored E-step forms c_jk in FP32 whatever the storage, and its
        # matrix-core products in bf16 hi + lo for bf16x3 storage, else in FP32
        "dtype": ({"bf16x3": "bf16", "fp16": "fp16", "fp32": "fp32", "fp64": "fp64",
                   "bf16": "bf16"}[args.precision] if args.correlation
                  else ("bf16" if args.precision == "bf16x3" else "fp32")),
        "data": "synthetic",
        "config": {"workload": f"windowed Synch-EM N={w.N} D={w.D} (K={w.K},Q={w.Q}) L={w.L} "
                               f"W={W} gamma={w.gamma} learned prior, {args.precision}"
                               + (", correlation GEMM" if args.correlation else ", factored E-step"),
                   "N": w.N, "D": w.D, "L": w.L, "W": W, "precision": args.precision,
                   "e_step": "correlation GEMM" if args.correlation else "factored"},
        "obs_rot_per_s": iters_s * w.N * W,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "kernel": info["kernel"],
                     "pass_us": pass_ms * 1e3, "launches": nlaunch,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "baseline_full_fp32": baseline,
        "speedup_vs_full_fp32": (iters_s / baseline["iter_per_s"]) if baseline else None,
        "variants": variants,
        "accuracy_vs_oracle": acc,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
