#!/usr/bin/env python3
"""Benchmark of the time-step-targeting DMRG hot path on one MI355X.

One step = one time-step-targeting call on the headline superblock (two-leg Hubbard ladder
2x16, U = 8, m = 1000 states per block, synthetic sector-structured blocks): a Krylov basis of
kdim = 15 Lanczos vectors started from phi (15 products H_sb.psi in FP64 MFMA, full FP64
reorthogonalisation), the device tridiagonal exponential at t = 0, tau/3, 2tau/3, tau
(tau = 0.05), and the combination into the four target vectors.  Inputs are resident in HBM
before the timed region.

value = algorithmic H_sb.psi flops of the step (kdim x F, F from the library's block plan)
        divided by the measured step time, in TFLOP/s.
Also printed: Krylov steps/s, the product-only rate, the roofline of the dominant kernel
(measured live with HIP events on the launch stream) and the FP64 CPU oracle on a bounded
sample of the same workload.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

PEAK_FP64_TFLOPS = 78.6          # MI355X dense FP64 MFMA
PEAK_FP32_TFLOPS = 157.3         # dense FP32 MFMA
PEAK_BF16_TFLOPS = 2500.0        # dense BF16 MFMA (no sparsity)
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of the block-product kernels, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of
# this bench on this workload with the families fixed (--gemm 12), scaled by the readings of a
# plain 512 MiB copy (summary and commands in profiles/).  Valid only for the kernel source they
# were taken on: reported as null once the source differs.
MEASURED_TRAFFIC = {
    "workload": "ladder16_m1000",
    "source": "paper_1103_5391_amd/csrc/gemm.hip",
    "source_sha256": "cc6bbb26839b41a745bf391d466692f0e26921b51a912326ef45acc1a9f6c644",
    "bytes": {"stage2<PF64, 1, 4>": 85.52e6 + 5.20e6, "stage1<PF64, 2>": 30.24e6 + 43.54e6},
    "profile": "profiles/stage2_fp64_ladder16_m1000_kernel_stats.txt",
}


def kernel_name(stage: int, variant: int) -> str:
    """Name of the FP64 kernel that runs a stage under a dmrg_gemm variant (as profilers show it,
    without the namespace)."""
    if variant & 16:
        return "stage1x" if stage == 1 else "stage2x"
    if stage == 1:
        if variant & 1:
            return "stage1_lds<PF64>"
        return "stage1<PF64, 2>" if variant & 4 else "stage1<PF64, 4>"
    if variant & 2:
        return "stage2_lds<PF64>"
    return "stage2<PF64, 1, 4>" if variant & 8 else "stage2<PF64, 2, 4>"


def measured_traffic(workload: str, kernel: str):
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), MEASURED_TRAFFIC["source"])
    try:
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return None
    if sha != MEASURED_TRAFFIC["source_sha256"] or workload != MEASURED_TRAFFIC["workload"]:
        return None
    return MEASURED_TRAFFIC["bytes"].get(kernel)


def _cpu_threads() -> int:
    try:
        from threadpoolctl import threadpool_info
        n = [int(p.get("num_threads", 0)) for p in threadpool_info() if p.get("user_api") == "blas"]
        if n:
            return max(n)
    except Exception:
        pass
    return os.cpu_count() or 1


def cpu_baseline(pb, phi, kdim, tau, F, budget_s=12.0, dens=None):
    """The FP64 oracle (unchanged) timed on the host: whole time-step-targeting steps, repeated
    until about budget_s seconds of work have been timed (at least one; per-step times, median
    reported), then the oracle product alone on one BLAS thread for about budget_s / 3, and the
    oracle density matrix + truncation on dens = (vectors, weights, keep) if given."""
    import numpy as np
    from oracle import krylov as K
    from oracle import matvec as M
    apply_h = lambda v: M.matvec_sector(pb, v)
    t0 = time.perf_counter()
    times = []
    while True:
        t1 = time.perf_counter()
        K.tst_targets(apply_h, phi, tau, kdim)
        times.append(time.perf_counter() - t1)
        el = time.perf_counter() - t0
        if el >= budget_s or el / len(times) * (len(times) + 1) > 2.5 * budget_s:
            break
    per = float(np.median(times))
    out = {"value": kdim * F / per / 1e12, "unit": "TFLOP/s", "cores": _cpu_threads(),
           "os_cpu_count": os.cpu_count(), "kind": "oracle", "steps_per_s": 1.0 / per,
           "sample": f"{len(times)} full time-step-targeting step(s) of the same workload "
                     f"(kdim={kdim}, oracle FP64 NumPy/SciPy), median of the step times, "
                     f"{el:.1f} s timed"}
    try:
        from threadpoolctl import threadpool_limits
        with threadpool_limits(limits=1, user_api="blas"):
            apply_h(phi)
            t0 = time.perf_counter()
            mv = []
            while time.perf_counter() - t0 < budget_s / 3 or not mv:
                t1 = time.perf_counter()
                apply_h(phi)
                mv.append(time.perf_counter() - t1)
        pm = float(np.median(mv))
        out["single_thread"] = {"matvec_tflops": F / pm / 1e12, "matvec_s": pm,
                                "sample": f"{len(mv)} oracle products (median) on 1 BLAS thread"}
    except ImportError:
        pass
    if dens is not None:
        from oracle import density as D
        vecs, wts, keep = dens
        dt = []
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < budget_s / 6 or not dt:
            t1 = time.perf_counter()
            D.truncate(pb, vecs, wts, keep)
            dt.append(time.perf_counter() - t1)
        out["density_truncate"] = {"ms_per_call": round(1e3 * float(np.median(dt)), 3),
                                   "sample": f"{len(dt)} oracle calls (median), same 5 vectors"}
    return out


def batch_section(L, I, torch, steps, warmup, count=64):
    """Configuration of 64 independent chain superblocks (m 100..1000): the batched call (one
    launch per pass for all problems, Lanczos iterations as one HIP graph) against the
    per-problem launch loop, both on the same handles and inputs."""
    import numpy as np
    kdim, tau = 15, 0.1
    pbs = I.batch_workloads(count)
    stream = torch.cuda.current_stream()
    hs = [L.dmrg_create(pb, stream) for pb in pbs]
    F = sum(h.flops() for h in hs)
    pds = [torch.from_numpy(I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + 900 + i))).to("cuda")
           for i, h in enumerate(hs)]
    tds = [torch.empty(8 * h.n, dtype=torch.float64, device="cuda") for h in hs]
    b = L.Batch(hs)
    btune = b.autotune(reps=3)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    def loop():
        for h, p, t in zip(hs, pds, tds):
            h.tst_targets(p, tau, kdim, t, info=False)

    ms_loop = timed(loop)
    out = {"problems": count, "kdim": kdim, "tau": tau, "n_total": int(sum(h.n for h in hs)),
           "autotune_ms": {k: round(float(v), 4) for k, v in btune.items()},
           "flops_per_step": F * kdim, "per_problem_loop_ms": round(ms_loop, 4)}
    for graph in (False, True):
        b.set_graph(graph)
        ms = timed(lambda: b.batch_tst_targets(pds, tau, kdim, tds, info=False))
        key = "batched_graph" if graph else "batched_eager"
        out[key + "_ms"] = round(ms, 4)
        out[key + "_speedup_vs_loop"] = round(ms_loop / ms, 3)
    out["batched_graph_tflops"] = round(F * kdim / (out["batched_graph_ms"] * 1e-3) / 1e12, 4)
    out["per_problem_loop_tflops"] = round(F * kdim / (ms_loop * 1e-3) / 1e12, 4)

    # 4-RHS (per-target) mode: each problem's four targets as four chains advanced by tau, all
    # 256 chains in common launches, against the loop of per-problem 4-chain calls
    cx = [t[2 * h.n * k:2 * h.n * (k + 1)] for h, t in zip(hs, tds) for k in range(4)]
    cy = [torch.empty_like(x) for x in cx]

    def chain_loop():
        for i, h in enumerate(hs):
            h.tst_chains(cx[4 * i:4 * i + 4], tau, kdim, cy[4 * i:4 * i + 4], info=False)

    for h in hs:
        h.set_gemm(h.autotune(reps=3)["variant"])
    ms_cloop = timed(chain_loop)
    b.set_graph(True)
    ms_c = timed(lambda: b.batch_tst_chains(cx, tau, kdim, cy, info=False))
    out["rhs4"] = {"chains": 4 * count, "flops_per_step": 4 * F * kdim,
                   "per_problem_loop_ms": round(ms_cloop, 4), "batched_graph_ms": round(ms_c, 4),
                   "batched_speedup_vs_loop": round(ms_cloop / ms_c, 3),
                   "batched_tflops": round(4 * F * kdim / (ms_c * 1e-3) / 1e12, 4)}
    b.destroy()
    for h in hs:
        h.destroy()
    return out


def _oracle_steps(fn, budget_s):
    """Median seconds of fn() over repeats for about budget_s seconds (at least one)."""
    import numpy as np
    times = []
    t0 = time.perf_counter()
    while True:
        t1 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - t1)
        el = time.perf_counter() - t0
        if el >= budget_s or el / len(times) * (len(times) + 1) > 2.5 * budget_s:
            break
    return float(np.median(times)), len(times), el


def configs_section(L, I, torch, steps, warmup, cpu_budget, run_cpu):
    """The smaller configurations, each on its own handle:
      chain8_exact   Hubbard chain L = 8, U = 4, exact blocks: one product, then 10 Krylov steps
                     (kdim 12, tau 0.1) in FP64; relative error against the oracle's 10 steps
      chain32_m400   chain L = 32, m = 400: time-step-targeting steps (kdim 15) in FP64 and with
                     FP32 block products
      ladder16_m800  ladder 2x16, U = 8, m = 800: the same in FP64 and with BF16x3 products
    and the FP64 oracle on the host for the first two (the same inputs)."""
    import numpy as np
    from oracle import krylov as K
    from oracle import matvec as M
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out, cpu = {}, {}
    # chain L = 8, exact blocks
    name = "chain8_exact"
    w = I.WORKLOADS[name]
    pb = I.make_workload(name)
    h = L.dmrg_create(pb, stream)
    h.set_gemm(h.autotune(reps=5)["variant"])
    F = h.flops()
    x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + w["seed"]))
    xd = torch.from_numpy(x).to("cuda")
    yd = torch.empty_like(xd)
    ms_mv = timed(lambda: h.matvec(xd, yd), 50)
    ms_k = timed(lambda: h.krylov_expm(xd, yd, w["tau"], w["kdim"], w["nsteps"], info=False), 5)
    apply_h = lambda v: M.matvec_sector(pb, v)
    y_ref, _ = K.krylov_expm(apply_h, x, w["tau"], w["kdim"], w["nsteps"])
    err = float(np.linalg.norm(yd.cpu().numpy() - y_ref) / np.linalg.norm(y_ref))
    out[name] = {"n_complex": h.n, "flops_per_matvec": F, "matvec_ms": round(ms_mv, 5),
                 "krylov_ms_per_step": round(ms_k / w["nsteps"], 5),
                 "krylov_steps_per_s": round(1000.0 * w["nsteps"] / ms_k, 2),
                 "kdim": w["kdim"], "tau": w["tau"], "nsteps": w["nsteps"],
                 "rel_err_vs_oracle": err}
    if run_cpu:
        per, cnt, el = _oracle_steps(lambda: K.krylov_expm(apply_h, x, w["tau"], w["kdim"], 1),
                                     cpu_budget / 4)
        cpu[name] = {"ms_per_krylov_step": round(per * 1e3, 4), "steps_per_s": round(1.0 / per, 2),
                     "tflops": w["kdim"] * F / per / 1e12,
                     "gpu_speedup": round(per * 1e3 / (ms_k / w["nsteps"]), 2),
                     "sample": f"{cnt} oracle Krylov steps (kdim {w['kdim']}), median, {el:.1f} s"}
    h.destroy()
    print(f"[bench] {name}: {out[name]}", file=sys.stderr, flush=True)

    # synthetic superblocks with a mixed arithmetic beside FP64
    for name, prec, label in [("chain32_m400", L.DMRG_FP32, "fp32"),
                              ("ladder16_m800", L.DMRG_BF16X3, "bf16x3")]:
        w = I.WORKLOADS[name]
        pb = I.make_workload(name)
        h = L.dmrg_create(pb, stream)
        F = h.flops()
        x = I.random_psi(h.n, np.random.default_rng(I.SEED_BASE + w["seed"] + 1000))
        xd = torch.from_numpy(x).to("cuda")
        td = torch.empty(8 * h.n, dtype=torch.float64, device="cuda")
        yd = torch.empty_like(xd)
        res = {"n_complex": h.n, "flops_per_matvec": F, "kdim": w["kdim"], "tau": w["tau"]}
        ref = None
        for pr, lab in [(L.DMRG_FP64, "fp64"), (prec, label)]:
            h.set_precision(pr)
            h.set_gemm(h.autotune(reps=5)["variant"])
            ms = timed(lambda: h.tst_targets(xd, w["tau"], w["kdim"], td, info=False), steps)
            pm = h.profile_matvec(xd, yd, reps=10)
            ms_mv = pm["ms_stage1"] + pm["ms_stage2"]
            r = {"ms_per_step": round(ms, 5), "krylov_steps_per_s": round(1000.0 / ms, 2),
                 "matvec_ms": round(ms_mv, 5), "matvec_tflops": round(F / (ms_mv * 1e-3) / 1e12, 4),
                 "step_tflops": round(w["kdim"] * F / (ms * 1e-3) / 1e12, 4)}
            if ref is None:
                ref = td.clone()
            else:
                n2 = 2 * h.n
                r["tst_rel_err_vs_fp64"] = max(
                    float(torch.linalg.vector_norm(td[n2 * i:n2 * (i + 1)] - ref[n2 * i:n2 * (i + 1)])
                          / torch.linalg.vector_norm(ref[n2 * i:n2 * (i + 1)])) for i in range(4))
                r["norm_drift"] = max(abs(float(torch.linalg.vector_norm(td[n2 * i:n2 * (i + 1)])) - 1.0)
                                      for i in range(4))
                r["speedup_vs_fp64"] = round(res["fp64"]["ms_per_step"] / ms, 3)
            res[lab] = r
        out[name] = res
        if run_cpu and name == "chain32_m400":
            apply_h = lambda v, pb=pb: M.matvec_sector(pb, v)
            per, cnt, el = _oracle_steps(lambda: K.tst_targets(apply_h, x, w["tau"], w["kdim"]),
                                         cpu_budget / 2)
            cpu[name] = {"ms_per_step": round(per * 1e3, 3), "steps_per_s": round(1.0 / per, 3),
                         "tflops": w["kdim"] * F / per / 1e12,
                         "gpu_fp64_speedup": round(per * 1e3 / res["fp64"]["ms_per_step"], 2),
                         "sample": f"{cnt} oracle time-step-targeting steps (kdim {w['kdim']}), "
                                   f"median, {el:.1f} s"}
        h.destroy()
        print(f"[bench] {name}: {out[name]}", file=sys.stderr, flush=True)
    return out, cpu


def drift_section(L, I, torch, name="ladder32_m2000", steps=50):
    """Config-5 drift: the ladder 2x32 at m = 2000 evolved by `steps` Krylov steps (kdim 20,
    tau 0.05) in every arithmetic from the holon-doublon-like start psi = (c+_{s1 up} P_S) (x)
    c_{s2 dn} psi0 (psi0 a seeded normalised complex vector of the half-filled sector; psi,
    normalised, lies in (N_up + 1, N_dn - 1) = (33, 31)), prepared by the library's local
    operators; per step the norm and the energy Re <psi|H|psi> (FP64 products).  Reports the
    largest drift from step 0 and the largest deviation from the FP64 run."""
    import numpy as np
    w = I.WORKLOADS[name]
    pb0 = I.make_workload(name)
    s1, s2 = pb0.Sblk.sites[-1], pb0.Eblk.sites[0]
    ops_s, ops_e = I.site_ops(pb0.Sblk, s1), I.site_ops(pb0.Eblk, s2)
    psrc, iS, iE = I.with_ops(pb0, [ops_s["cdag_0"]], [ops_e["c_1"]])
    tgt = (pb0.target[0] + 1, pb0.target[1] - 1)
    pb = I.with_ops(pb0, [ops_s["cdag_0"]], [ops_e["c_1"]], target=tgt)[0]
    hs = L.dmrg_create(psrc)
    he = L.dmrg_create(pb)                    # FP64 energies
    hp = L.dmrg_create(pb)
    n = hp.n
    x0 = torch.from_numpy(I.random_psi(hs.n, np.random.default_rng(I.SEED_BASE + w["seed"] + 1000))).cuda()
    psi0 = torch.empty(2 * n, dtype=torch.float64, device="cuda")
    hs.apply_local(hp, [(1.0, iS[0], 0, iE[0], 0, 1)], x0, psi0)
    psi0 /= torch.linalg.vector_norm(psi0)
    hs.destroy()
    hv = torch.empty_like(psi0)

    def energy(v):
        he.matvec(v, hv)
        return float(torch.dot(v, hv))        # Re <v|H v> for the real/imaginary split layout

    out, ref_states, ref_e = {}, [], []
    for prec, label in [(L.DMRG_FP64, "fp64"), (L.DMRG_FP32, "fp32"), (L.DMRG_BF16X3, "bf16x3"),
                        (L.DMRG_BF16X6, "bf16x6")]:
        hp.set_precision(prec)
        hp.autotune(reps=3)
        psi = psi0.clone()
        e0 = energy(psi)
        dn = de = dev_psi = dev_e = 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            hp.krylov_expm(psi, psi, w["tau"], w["kdim"], 1, info=False)
            nrm = float(torch.linalg.vector_norm(psi))
            e = energy(psi)
            dn = max(dn, abs(nrm - 1.0))
            de = max(de, abs(e - e0) / abs(e0))
            if prec == L.DMRG_FP64:
                ref_states.append(psi.clone())
                ref_e.append(e)
            else:
                dev_psi = max(dev_psi, float(torch.linalg.vector_norm(psi - ref_states[s])))
                dev_e = max(dev_e, abs(e - ref_e[s]) / abs(e0))
        torch.cuda.synchronize()
        out[label] = {"max_norm_drift": dn, "max_rel_energy_drift": de,
                      "max_state_dev_vs_fp64": dev_psi, "max_rel_energy_dev_vs_fp64": dev_e,
                      "ms_per_step_incl_energy": round((time.perf_counter() - t0) * 1e3 / steps, 3)}
        print(f"[bench] drift {label}: {out[label]}", file=sys.stderr, flush=True)
    hp.destroy()
    he.destroy()
    res = {"workload": name, "steps": steps, "kdim": w["kdim"], "tau": w["tau"], "energy0": e0,
           "initial_state": "(c+_{s1 up} P_S) x c_{s2 dn} psi0, normalised",
           "sector": list(tgt), "n_complex": n, "per_arithmetic": out}
    return res, (pb, psi0.cpu().numpy(), out["fp64"]["ms_per_step_incl_energy"])


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ladder16_m1000")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="FP64 only (no mixed-arithmetic runs)")
    ap.add_argument("--no-drift", action="store_true", help="skip the 50-step m = 2000 drift run")
    ap.add_argument("--no-rhs4", action="store_true", help="skip the 4-RHS (per-target) mode run")
    ap.add_argument("--no-gs", action="store_true", help="skip the ground-state run")
    ap.add_argument("--no-density", action="store_true",
                    help="skip the density-matrix + truncation run (and the transformation)")
    ap.add_argument("--no-wft", action="store_true", help="skip the wave-function transformation")
    ap.add_argument("--no-local", action="store_true", help="skip the local-operator run")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the smaller configurations (chain L = 8, chain m = 400, ladder m = 800)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="copy a buffer of MIB MiB once before the run: a plain copy kernel of "
                         "known traffic that hardware-counter runs use as the byte scale")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--gemm", type=int, default=-1, metavar="VARIANT",
                    help="kernel families of the FP64 block products (dmrg_set_gemm bits) instead "
                         "of the autotuner's choice, e.g. for hardware-counter runs that must "
                         "see one family")
    ap.add_argument("--tune-cache", default=None, metavar="PATH",
                    help="JSON tuning cache of the headline workload's autotuner: a stored choice "
                         "is applied without timing, a miss is timed and stored")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1103_5391_amd import inputs as I
    from paper_1103_5391_amd import lib as L

    w = I.WORKLOADS[args.workload]
    kdim, tau = w["kdim"], w["tau"]
    print(f"[bench] building workload {args.workload}", file=sys.stderr, flush=True)
    pb = I.make_workload(args.workload)
    torch.cuda.init()
    stream = torch.cuda.current_stream()
    if args.copy_calibration > 0:
        nel = args.copy_calibration * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    h = L.dmrg_create(pb, stream)
    # the library's autotuner picks the kernel family of each block-product stage (unless fixed)
    tune64 = h.autotune(reps=10, cache=args.tune_cache)
    if args.gemm >= 0:
        h.set_gemm(args.gemm)
        tune64["variant"] = args.gemm
    F = h.flops()
    n = h.n
    phi = I.random_psi(n, np.random.default_rng(I.SEED_BASE + w["seed"] + 1000))
    pd = torch.from_numpy(phi).to("cuda")
    td = torch.empty(8 * n, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    print(f"[bench] n={n} F={F:.4g} kdim={kdim}; warmup {args.warmup}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        h.tst_targets(pd, tau, kdim, td, info=False)
    torch.cuda.synchronize()

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        h.tst_targets(pd, tau, kdim, td, info=False)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_step = e0.elapsed_time(e1) / args.steps
    print(f"[bench] {args.steps} steps: {ms_step:.4f} ms/step (wall {wall:.3f} s)", file=sys.stderr,
          flush=True)
    # sanity: unitary evolution keeps the norm of every target
    tn = [float(torch.linalg.vector_norm(td[2 * n * i:2 * n * (i + 1)])) for i in range(4)]
    assert all(abs(x - 1.0) < 1e-9 for x in tn), tn

    # 4-RHS (per-target) mode on the same workload: the four targets as four chains advanced
    # by tau in common launches
    rhs4 = None
    cx = [] if args.no_rhs4 else [td[2 * n * k:2 * n * (k + 1)].clone() for k in range(4)]
    if not args.no_rhs4:
        cy = [torch.empty_like(x) for x in cx]
        for _ in range(args.warmup):
            h.tst_chains(cx, tau, kdim, cy, info=False)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            h.tst_chains(cx, tau, kdim, cy, info=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_rhs4 = e0.elapsed_time(e1) / args.steps
        rhs4 = {"ms_per_step": round(ms_rhs4, 5), "chains": 4,
                "tflops": round(4 * kdim * F / (ms_rhs4 * 1e-3) / 1e12, 4),
                "chain_steps_per_s": round(4000.0 / ms_rhs4, 3),
                "per_chain_speedup_vs_single": round(4 * ms_step / ms_rhs4, 3)}
        print(f"[bench] 4-RHS mode: {rhs4}", file=sys.stderr, flush=True)

    # ground state of the same superblock by restarted Lanczos (kdim 64, to a relative residual
    # of 1e-6 or 60 bases; the synthetic spectrum is dense at the bottom, and a restart from one
    # Ritz vector needs a basis this large to converge in a few bases from a random start)
    gs = None
    if not args.no_gs:
        gkdim = 64
        gd = pd.clone()
        yg = torch.empty_like(gd)
        h.ground_state(gd, yg, gkdim, 1, 0.0, info=False)   # warm-up (tables sized for the kdim)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e_gs, used, ginfo = h.ground_state(gd, yg, gkdim, 60, 1e-6)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        gs = {"kdim": gkdim, "tol": 1e-6, "energy": e_gs, "bases": used,
              "converged": bool(ginfo["converged"]),
              "residual_est": ginfo["err_est"], "ms_total": round(el * 1e3, 3),
              "ms_per_basis": round(el * 1e3 / used, 4),
              "tflops": round(gkdim * used * F / el / 1e12, 4)}
        print(f"[bench] ground state: {gs}", file=sys.stderr, flush=True)

    # density matrix of the five targets (ground state or the start vector, and the four time
    # vectors) with the time-step-targeting weights, and its truncation to m states
    dens, dens_host = None, None
    if not args.no_density:
        gsv = yg if gs is not None else pd
        dv = [gsv] + [td[2 * n * k:2 * n * (k + 1)] for k in range(4)]
        wts = [float(x) for x in h.tst_targets(pd, tau, kdim, td, info=False)[0]]
        keep = int(w.get("m") or 1000)
        rows = [int(r) for r in h.psi_layout()["rows"]]
        evd = torch.empty(sum(rows), dtype=torch.float64, device="cuda")
        vcd = torch.empty(sum(2 * r * r for r in rows), dtype=torch.float64, device="cuda")
        h.density_truncate(dv, wts, keep, evd, vcd)
        torch.cuda.synchronize()
        reps = 5
        e0.record(stream)
        for _ in range(reps):
            kept, terr = h.density_truncate(dv, wts, keep, evd, vcd)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_d = e0.elapsed_time(e1) / reps
        dens = {"ms_per_call": round(ms_d, 4), "vectors": 5, "keep": keep,
                "sectors": len(rows), "largest_sector": max(rows), "states": sum(rows),
                "kept_states": int(sum(kept)), "trunc_err": terr,
                "input_bytes": 5 * 2 * n * 8}
        dens_host = ([x.cpu().numpy() for x in dv], wts, keep)
        print(f"[bench] density + truncation: {dens}", file=sys.stderr, flush=True)

    # wave-function transformation of the five targets for a move of the centre one site to
    # the right, with the kept states just computed (synthetic stored basis of the environment)
    wft = None
    if dens is not None and not args.no_wft:
        mv = I.wft_move(pb, [int(k) for k in kept], seed=w["seed"])
        Wd = [torch.from_numpy(np.concatenate([x.real.T.reshape(-1), x.imag.T.reshape(-1)])).to("cuda")
              for x in mv.W]
        wf = h.wft_create(mv, Wd)
        ys = [torch.empty(2 * wf.n_new, dtype=torch.float64, device="cuda") for _ in dv]
        fl = wf.apply(vcd, dv, ys)
        torch.cuda.synchronize()
        reps = 10
        e0.record(stream)
        for _ in range(reps):
            wf.apply(vcd, dv, ys)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_w = e0.elapsed_time(e1) / reps
        wft = {"ms_per_call": round(ms_w, 4), "vectors": len(dv), "n_new": wf.n_new,
               "flops": fl, "tflops": round(fl / (ms_w * 1e-3) / 1e12, 4),
               "mfma_peak_frac": round(fl / (ms_w * 1e-3) / 1e12 / PEAK_FP64_TFLOPS, 4),
               "norms": [round(float(torch.linalg.vector_norm(y)), 12) for y in ys]}
        wf.destroy()
        print(f"[bench] wave-function transformation: {wft}", file=sys.stderr, flush=True)

    # local operators at the central sites: the doublon factor c+_up n_dn on the first
    # environment site and the holon factor c_dn (1 - n_up) on the last system site applied to
    # the step's last target (into the (N_up + 1, N_dn - 1) sector), and the densities of both
    # central sites measured on the four targets
    local = None
    if not args.no_local:
        s1, s2 = pb.Sblk.sites[-1], pb.Eblk.sites[0]
        ops_s = I.site_ops(pb.Sblk, s1)
        ops_e = I.site_ops(pb.Eblk, s2)
        pbx, iS, iE = I.with_ops(pb, [ops_s["holon_1"], ops_s["n"]], [ops_e["doublon_0"], ops_e["n"]])
        tgt = (pb.target[0] + 1, pb.target[1] - 1)
        pdx = I.with_ops(pb, [ops_s["holon_1"], ops_s["n"]], [ops_e["doublon_0"], ops_e["n"]], target=tgt)[0]
        hx, hd = L.dmrg_create(pbx, stream), L.dmrg_create(pdx, stream)
        xl = td[6 * n:8 * n].contiguous()
        yl = torch.empty(2 * hd.n, dtype=torch.float64, device="cuda")
        hd_terms = [(1.0, iS[0], 0, iE[0], 0, 1)]
        dens_terms = [(1.0, iS[1], 0, -1, 0, 0), (1.0, -1, 0, iE[1], 0, 0)]
        hx.apply_local(hd, hd_terms, xl, yl)
        hx.expect_local(dens_terms, xl)
        torch.cuda.synchronize()
        reps = 20
        e0.record(stream)
        for _ in range(reps):
            hx.apply_local(hd, hd_terms, xl, yl)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_apply = e0.elapsed_time(e1) / reps
        t0 = time.perf_counter()
        vals = [hx.expect_local(dens_terms, td[2 * n * k:2 * n * (k + 1)]).real for k in range(4)]
        ms_expect = (time.perf_counter() - t0) * 1e3 / 4
        local = {"apply_ms": round(ms_apply, 4), "expect_ms_host_clock": round(ms_expect, 4),
                 "holon_doublon_norm": round(float(torch.linalg.vector_norm(yl)), 12),
                 "central_density_per_target": [round(v, 10) for v in vals],
                 "sites": [int(s1), int(s2)], "target_sector": list(tgt)}
        hx.destroy()
        hd.destroy()
        print(f"[bench] local operators: {local}", file=sys.stderr, flush=True)

    # product-only rate and the dominant kernel (HIP events around each launch)
    yd = torch.empty_like(pd)
    prof = h.profile_matvec(pd, yd, reps=20)
    ms_mv = prof["ms_stage1"] + prof["ms_stage2"]
    dom = 1 if prof["ms_stage1"] >= prof["ms_stage2"] else 2
    ms_dom, fl_dom = prof[f"ms_stage{dom}"], prof[f"flops_stage{dom}"]
    achieved = fl_dom / (ms_dom * 1e-3) / 1e12

    # mixed arithmetic of the block products (Lanczos, reorthogonalisation, exponential and
    # combination stay FP64): same step, error against the FP64 targets of this run
    ref = td.clone()
    ref_mv = torch.empty_like(pd)
    h.matvec(pd, ref_mv)
    mixed = {}
    arithmetics = [] if args.no_mixed else [(L.DMRG_FP32, "fp32"), (L.DMRG_BF16X3, "bf16x3"),
                                            (L.DMRG_BF16X6, "bf16x6")]
    for prec, label in arithmetics:
        h.set_precision(prec)
        tune = h.autotune(reps=10)
        for _ in range(args.warmup):
            h.tst_targets(pd, tau, kdim, td, info=False)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            h.tst_targets(pd, tau, kdim, td, info=False)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_p = e0.elapsed_time(e1) / args.steps
        mv = torch.empty_like(pd)
        h.matvec(pd, mv)
        pm = h.profile_matvec(pd, yd, reps=10)
        torch.cuda.synchronize()
        tst_err = max(float(torch.linalg.vector_norm(td[2 * n * i:2 * n * (i + 1)] - ref[2 * n * i:2 * n * (i + 1)]))
                      / float(torch.linalg.vector_norm(ref[2 * n * i:2 * n * (i + 1)])) for i in range(4))
        drift = max(abs(float(torch.linalg.vector_norm(td[2 * n * i:2 * n * (i + 1)])) - 1.0) for i in range(4))
        ms_mv_p = pm["ms_stage1"] + pm["ms_stage2"]
        tf_p = F / (ms_mv_p * 1e-3) / 1e12
        # split arithmetics issue pieces x F MFMA work (3 or 6 products per value product)
        issued = {"fp32": 1, "bf16x3": 3, "bf16x6": 6}[label]
        peak = PEAK_FP32_TFLOPS if label == "fp32" else PEAK_BF16_TFLOPS
        mixed[label] = {
            "ms_per_step": round(ms_p, 5),
            "matvec_tflops": round(tf_p, 4),
            "mfma_peak_frac": round(tf_p / peak, 5),
            "issued_mfma_frac": round(issued * tf_p / peak, 5),
            "krylov_steps_per_s": round(1000.0 / ms_p, 3),
            "speedup_vs_fp64": round(ms_step / ms_p, 3),
            "matvec_ms": round(pm["ms_stage1"] + pm["ms_stage2"], 5),
            "matvec_speedup_vs_fp64": round(ms_mv / (pm["ms_stage1"] + pm["ms_stage2"]), 3),
            "matvec_rel_err_vs_fp64": float(torch.linalg.vector_norm(mv - ref_mv) / torch.linalg.vector_norm(ref_mv)),
            "tst_rel_err_vs_fp64": tst_err,
            "norm_drift": drift,
            "gemm_variant": int(tune["variant"]),
        }
        print(f"[bench] {label}: {ms_p:.4f} ms/step, {mixed[label]}", file=sys.stderr, flush=True)
    h.set_precision(L.DMRG_FP64)
    h.set_gemm(tune64["variant"])

    batched = None
    if not args.no_batch:
        print("[bench] batched configuration (64 superblocks)", file=sys.stderr, flush=True)
        batched = batch_section(L, I, torch, max(3, args.steps // 5), 1)
        print(f"[bench] batched: {batched}", file=sys.stderr, flush=True)

    configs, cpu_configs = None, {}
    if not args.no_configs:
        print("[bench] smaller configurations", file=sys.stderr, flush=True)
        configs, cpu_configs = configs_section(L, I, torch, max(5, args.steps // 3), args.warmup,
                                               args.cpu_budget, not args.no_cpu_baseline)

    drift, drift_host = None, None
    if not args.no_drift:
        print("[bench] drift (ladder 2x32, m = 2000, 50 steps)", file=sys.stderr, flush=True)
        drift, drift_host = drift_section(L, I, torch)

    value = kdim * F / (ms_step * 1e-3) / 1e12
    out = {
        "metric": "H·ψ TFLOP/s + Krylov steps/s (ladder, m=1000) vs FP64 plain; % MFMA peak",
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "lattice": w["lattice"], "L": w["L"],
                   "m": w.get("m"), "U": w["U"], "kdim": kdim, "tau": tau, "n_complex": n,
                   "flops_per_matvec": F, "precision": "fp64", "step": "time-step targeting: "
                   "Krylov basis + tridiagonal exp at 4 times + combination",
                   "gemm_variant": int(tune64["variant"]),
                   "autotune_ms": {k: round(float(v), 5) for k, v in tune64.items()
                                   if k not in ("variant", "cached")},
                   "autotune_cached": bool(tune64.get("cached", False))},
        "krylov_steps_per_s": round(1000.0 / ms_step, 3),
        "matvec_tflops": round(F / (ms_mv * 1e-3) / 1e12, 4),
        "matvec_ms": round(ms_mv, 5),
        "mfma_peak_frac_step": round(value / PEAK_FP64_TFLOPS, 4),
        "rhs4_mode": rhs4,
        "ground_state": gs,
        "density_truncate": dens,
        "wave_function_transformation": wft,
        "local_operators": local,
        "mixed_precision": mixed,
        "batched_64": batched,
        "configs": configs,
        "drift_m2000": drift,
        "roofline": {"bound": "mfma", "kernel": kernel_name(dom, int(tune64["variant"])),
                     "achieved": round(achieved, 4), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP64_TFLOPS, 4),
                     "traffic": measured_traffic(args.workload, kernel_name(dom, int(tune64["variant"]))),
                     "traffic_unit": "bytes per launch",
                     "algorithmic_flop_per_launch": fl_dom,
                     "ms_per_launch": round(ms_dom, 5)},
    }
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pb, phi, kdim, tau, F, args.cpu_budget, dens_host)
        if drift_host is not None:
            # one oracle Krylov step of the m = 2000 ladder from the drift run's start vector
            from oracle import krylov as K
            from oracle import matvec as M
            pb5, psi5, gpu_ms = drift_host
            w5 = I.WORKLOADS["ladder32_m2000"]
            t1 = time.perf_counter()
            K.krylov_expm(lambda v: M.matvec_sector(pb5, v), psi5, w5["tau"], w5["kdim"], 1)
            per = time.perf_counter() - t1
            cpu_configs["ladder32_m2000"] = {
                "ms_per_krylov_step": round(per * 1e3, 1), "steps_per_s": round(1.0 / per, 4),
                "gpu_fp64_speedup_incl_energy": round(per * 1e3 / gpu_ms, 1),
                "sample": f"1 oracle Krylov step (kdim {w5['kdim']}) from the drift run's start vector"}
        out["cpu_baseline"]["configs"] = cpu_configs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
