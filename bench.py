"""Benchmark of the Cholesky-decomposition Sigma(2) quasi-particle path on one GPU.

One step = the whole hot path over one synthetic C60-shaped workload with its
inputs resident in HBM:
  pivoted incomplete Cholesky of the ERI supermatrix to delta = 1e-6 (FP64,
  on-demand s-Gaussian ERI columns)  ->  B^K = C^T L^K C blocks  ->  Newton
  quasi-particle solves (Delta = 1e-5) for the 20 orbitals HOMO-9 ... LUMO+9.
The headline precision runs the transform and contraction in split-bf16
(3-term, FP32 accumulation); FP32 and FP64 are measured beside it, and the
quasi-particle error of each against the FP64 path is reported in meV.

Prints ONE JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HARTREE_EV = 27.211396
HBM_PEAK_GBS = 8000.0
PEAKS_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
FP64_MFMA_TFLOPS = 78.6   # dense FP64 matrix peak
METRIC = "quasi-particle solves/s + contraction TFLOP/s, FP32/BF16x3 vs FP64 at ≤1 meV"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=2)
    p.add_argument("--prec", default="bf16x3", choices=["fp64", "fp32", "bf16x3"])
    p.add_argument("--workload", default="c60", choices=["c60", "large"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-overlap", action="store_true",
                   help="decomposition, then transform (instead of the transform beside the decomposition)")
    p.add_argument("--cpu-targets", type=int, default=4, help="targets in the oracle Newton sample")
    p.add_argument("--quick", action="store_true",
                   help="timed steps and roofline only (no precision, MP2, sweep, aCD or Dyson reports)")
    p.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                   help="only run an elementwise device copy of MIB MiB three times (scales HBM counters)")
    return p.parse_args()


def copy_probe(mib: int):
    """y = 2 x over MIB MiB of float64: reads and writes MIB MiB per launch, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of the other kernels to bytes."""
    import torch
    n = mib * (1 << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 2.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": n * 8, "copy_probe_bytes_written": n * 8, "launches": 3}))


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def committed_traffic(workload: str) -> dict:
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, per
    kernel, if it was taken on this workload and the Cholesky source is unchanged since; else {}."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "cd_kernels_c60_traffic.json")
    src = os.path.join(ROOT, "paper_0912_1459_amd", "csrc", "cd.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except OSError:
        return {}
    if rec.get("cd_hip_sha256") != sha or rec.get("workload_key") != workload:
        return {}
    return {k: v["hbm_bytes_per_launch"] for k, v in rec.get("kernels", {}).items()}


def cpu_baseline(w, delta: float, conv: float, ntarget: int) -> dict:
    """The oracle as it stands on the host cores: CD + transform in full, Newton on a sample."""
    from oracle import eri_cd as E, mo, selfenergy as SE
    cores = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    r = E.pivoted_cd(delta, centres=w.centres, alpha=w.alpha)
    t1 = time.perf_counter()
    sel = w.targets[:ntarget]
    Bsel, Bvo = mo.transform_blocks(r.L, w.C, w.nocc, sel)
    t2 = time.perf_counter()
    SE.solve_targets(Bsel, Bvo, w.eps, w.nocc, sel, conv=conv)
    t3 = time.perf_counter()
    nsel = len(w.targets)
    # transform cost grows with the selected block only mildly: scale the Newton part only
    est = (t1 - t0) + (t2 - t1) + (t3 - t2) * nsel / ntarget
    return {"value": nsel / est, "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": (f"full oracle CD (M={r.M}) and transform, Newton on {ntarget} of {nsel} "
                       f"targets scaled to {nsel}; t_cd={t1 - t0:.2f}s t_transform={t2 - t1:.2f}s "
                       f"t_newton={t3 - t2:.2f}s")}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU sharding "
              "of this path is a design note, not part of this build.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    import torch
    import paper_0912_1459_amd.core as C
    from paper_0912_1459_amd import inputs as I

    dev = "cuda:0"
    torch.cuda.set_device(0)
    w = I.make(args.workload)
    delta = w.delta
    conv = 1e-5
    centres = torch.tensor(w.centres, device=dev)
    alpha = torch.tensor(w.alpha, device=dev)
    Cm = torch.tensor(w.C, device=dev)
    eps = torch.tensor(w.eps, device=dev)
    stream = torch.cuda.current_stream()
    ctx = C.Context(0, stream)
    if args.workload == "large":
        # C = S^-1/2 Q with lambda_min(S) ~ 2e-7: rounding inside an FP32 or split-bf16
        # transform would be amplified ~1/lambda_min, so the transform runs in FP64 and only
        # the blocks are rounded for the contraction
        ctx.set_transform_fp64(True)
    nsel = len(w.targets)
    max_vec = (12 if args.workload == "c60" else 6) * w.nbf     # enough for both workloads at their delta

    def step(prec):
        if args.no_overlap:
            cd = C.cholesky(delta, centres=centres, alpha=alpha, max_vec=max_vec, grow=True, ctx=ctx)
            B = C.transform(cd.Lbuf, cd.nvec, Cm, w.nocc, w.targets, prec, ctx=ctx)
        else:
            # the transform of the vectors made so far runs beside the decomposition
            cd, B = C.cholesky_transform(delta, centres=centres, alpha=alpha, C=Cm, nocc=w.nocc, sel=w.targets,
                                         prec=prec, max_vec=max_vec, ctx=ctx)
        qp = C.qp_solve(B, eps, conv=conv, mode="residues", ctx=ctx)
        return cd, B, qp

    progress(f"{args.workload}: {w.npairs} pairs, warm-up")
    for _ in range(args.warmup):
        step(args.prec)
    torch.cuda.synchronize()
    progress("timed steps")

    # timed region: K whole-path steps, no per-kernel events
    ctx.reset_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        cd, B, qp = step(args.prec)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    st_run = ctx.stats()
    ms_per_step = gpu_ms / args.steps
    value = nsel * args.steps / (gpu_ms / 1e3)

    # the same K steps again with HIP events around every Cholesky step-kernel and pass
    # launch (on the library's stream): per-launch durations for the roofline
    progress(f"{ms_per_step:.1f} ms per step; kernel-timing pass")
    ctx.reset_stats()
    ctx.set_kernel_timing(True)
    for _ in range(args.steps):
        step(args.prec)
    torch.cuda.synchronize()
    st = ctx.stats()
    ctx.set_kernel_timing(False)

    M = cd.nvec
    npairs = w.npairs
    n_step = st["n_cd_step_launch"]
    n_pass = st["n_cd_pass_launch"]
    t_step = st["t_cd_kernel_ms"] / 1e3
    t_pass = st["t_cd_pass_ms"] / 1e3
    cd_kernels = {
        "step": {"launches_per_cd": n_step / args.steps, "total_ms_per_cd": round(t_step * 1e3 / args.steps, 3),
                 "avg_us": round(t_step / max(n_step, 1) * 1e6, 3),
                 "algorithmic_gbs": round(st["bytes_cd_step"] / t_step / 1e9, 1) if t_step > 0 else None},
        "pass": {"launches_per_cd": n_pass / args.steps, "total_ms_per_cd": round(t_pass * 1e3 / args.steps, 3),
                 "avg_us": round(t_pass / max(n_pass, 1) * 1e6, 3),
                 "gbs": round(st["bytes_cd_pass"] / t_pass / 1e9, 1) if t_pass > 0 else None,
                 "tflops_fp64": round(st["flops_cd_pass"] / t_pass / 1e12, 2) if t_pass > 0 else None},
        "misses_per_cd": st["n_cd_miss"] / args.steps,
        "speculative": {"blocks_per_cd": st["n_cd_spec_block"] / args.steps,
                        "steps_per_cd": st["n_cd_spec"] / args.steps,
                        "ms_per_cd": round(st["t_cd_spec_ms"] / args.steps, 3),
                        "state_reads_per_cd": st["n_cd_state_read"] / args.steps},
    }
    traffic = committed_traffic(args.workload)
    if t_pass >= t_step:
        # 2 flops per vector, pair row and candidate: 16 flops per byte of L, above the FP64
        # MFMA ridge (78.6 TF / 8 TB/s)
        per_launch = st["flops_cd_pass"] / max(n_pass, 1)
        avg = t_pass / max(n_pass, 1)
        roofline = {"kernel": "cd_pass_kernel", "bound": "mfma", "achieved": round(per_launch / avg / 1e12, 2),
                    "peak": FP64_MFMA_TFLOPS, "unit": "TFLOP/s",
                    "frac": round(per_launch / avg / 1e12 / FP64_MFMA_TFLOPS, 4),
                    "traffic": traffic.get("cd_pass_kernel"), "launches": n_pass / args.steps,
                    "avg_launch_us": round(avg * 1e6, 3), "units": "2 x pairs x vectors x 64 flops per launch"}
    else:
        per_launch = st["bytes_cd_step"] / max(n_step, 1)
        avg = t_step / max(n_step, 1)
        roofline = {"kernel": "cd_step_kernel", "bound": "hbm", "achieved": round(per_launch / avg / 1e9, 1),
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(per_launch / avg / 1e9 / HBM_PEAK_GBS, 4),
                    "traffic": traffic.get("cd_step_kernel"), "launches": n_step / args.steps,
                    "avg_launch_us": round(avg * 1e6, 3),
                    "units": "pairs x (8 B per vector subtracted + 34..66 B) per launch"}

    if args.quick:
        print(json.dumps({"metric": METRIC, "value": round(value, 2), "unit": "solves/s", "n_gpus": 1,
                          "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
                          "higher_is_better": True, "roofline": roofline,
                          "cd": {"ms": round(st_run["t_cd_ms"] / args.steps, 3), "steps": M,
                                 "kernels": cd_kernels, "transform_overlapped": not args.no_overlap},
                          "phases_ms": {k: round(st_run[k] / args.steps, 3) for k in
                                        ("t_cd_ms", "t_transform_ms", "t_contract_ms", "t_epilogue_ms",
                                         "t_newton_ms")}}))
        return

    progress("precision report")
    # per-precision contraction throughput and accuracy against the FP64 GPU path
    ref_cd, ref_B, ref_qp = step("fp64")
    prec_report = {}
    for prec in ("fp64", "fp32", "bf16x3"):
        B = C.transform(ref_cd.Lbuf, ref_cd.nvec, Cm, w.nocc, w.targets, prec, ctx=ctx)
        om = w.trial_energies()
        C.sigma2(B, eps, om, ctx=ctx)            # warm
        ctx.reset_stats()
        reps = 3
        for _ in range(reps):
            C.sigma2(B, eps, om, ctx=ctx)
        s1 = ctx.stats()
        t_con = s1["t_contract_ms"] / reps
        flops = s1["flops_contract"] / reps
        ctx.reset_stats()
        torch.cuda.synchronize()
        tq0 = time.perf_counter()
        qp_p = C.qp_solve(B, eps, conv=conv, mode="residues", ctx=ctx)
        torch.cuda.synchronize()
        tq = time.perf_counter() - tq0
        err_mev = float(np.abs(qp_p.omega - ref_qp.omega).max() * HARTREE_EV * 1e3)
        tf = flops / (t_con / 1e3) / 1e12
        hw = tf * (3 if prec == "bf16x3" else 1)
        prec_report[prec] = {
            "contract_ms": round(t_con, 4), "contract_tflops": round(tf, 2),
            "mfma_frac": round(hw / PEAKS_TFLOPS[prec], 4),
            "solves_per_s_from_B": round(nsel / tq, 1),
            "max_err_meV_vs_fp64": round(err_mev, 6),
            "newton_iters_max": int(qp_p.iters.max()),
        }
    progress("backward pass")
    # backward pass: adjoint of the solve (FP64 and FP32 blocks) and of the transform, for the
    # cotangent of the sum of all quasi-particle energies
    backward = {}
    for prec in ("fp64", "fp32"):
        B = C.transform(ref_cd.Lbuf, ref_cd.nvec, Cm, w.nocc, w.targets, prec, ctx=ctx)
        qp_p = C.qp_solve(B, eps, conv=1e-10, mode="residues", ctx=ctx)
        ob = np.ones(nsel)
        C.qp_adjoint(B, eps, qp_p.omega, ob, ctx=ctx)                     # warm
        torch.cuda.synchronize()
        tb0 = time.perf_counter()
        gs, gv, ge = C.qp_adjoint(B, eps, qp_p.omega, ob, ctx=ctx)
        torch.cuda.synchronize()
        tb1 = time.perf_counter()
        C.transform_adjoint(ref_cd.Lbuf, ref_cd.nvec, Cm, w.nocc, w.targets, gs, gv, B.ldk, ctx=ctx)
        torch.cuda.synchronize()
        tb2 = time.perf_counter()
        backward[prec] = {"qp_adjoint_ms": round((tb1 - tb0) * 1e3, 3),
                          "transform_adjoint_ms": round((tb2 - tb1) * 1e3, 3)}
        del B, gs, gv, ge

    progress("MP2")
    # MP2 correlation energy, Eq. (MP2), from the same Bvo block in each precision
    mp2_report = {}
    e_ref = None
    for prec in ("fp64", "fp32", "bf16x3"):
        B = C.transform(ref_cd.Lbuf, ref_cd.nvec, Cm, w.nocc, w.targets, prec, ctx=ctx)
        C.mp2_energy(B, eps, ctx=ctx)            # warm
        ctx.reset_stats()
        e = C.mp2_energy(B, eps, ctx=ctx)
        s2 = ctx.stats()
        if prec == "fp64":
            e_ref = e
        tf = s2["flops_mp2"] / (s2["t_mp2_ms"] / 1e3) / 1e12
        mp2_report[prec] = {"energy_Eh": e, "ms": round(s2["t_mp2_ms"], 3), "tflops": round(tf, 2),
                            "mfma_frac": round(tf * (3 if prec == "bf16x3" else 1) / PEAKS_TFLOPS[prec], 4),
                            "rel_err_vs_fp64": abs(e - e_ref) / abs(e_ref)}
    for prec in ("fp32", "bf16x3"):
        prec_report[prec]["contract_speedup_vs_fp64"] = round(
            prec_report["fp64"]["contract_ms"] / prec_report[prec]["contract_ms"], 2)

    # the paper's spectral-window experiment in synthetic form (untimed): window orbitals,
    # CD-4 ... CD-8 against CD-10, FP64, Newton Delta = 1e-5
    from paper_0912_1459_amd import sweep as SW
    sweep = SW.report(w, prec="fp64", conv=conv) if args.workload == "c60" else None

    # atomic CD (one-centre products per atom, then the inner projection onto them) against
    # the full CD at the same delta: decomposition time and quasi-particle shift (FP64)
    acd_report = None
    if args.workload == "c60":
        progress("atomic CD")
        from paper_0912_1459_amd import acd as ACD
        ACD.acd(centres, alpha, delta, ctx=ctx)                     # warm
        torch.cuda.synchronize()
        ta0 = time.perf_counter()
        a = ACD.acd(centres, alpha, delta, ctx=ctx)
        torch.cuda.synchronize()
        ta1 = time.perf_counter()
        C.cholesky(delta, centres=centres, alpha=alpha, max_vec=max_vec, grow=True, ctx=ctx)
        torch.cuda.synchronize()
        ta2 = time.perf_counter()
        Ba = C.transform(a.cd.Lbuf, a.cd.nvec, Cm, w.nocc, w.targets, "fp64", ctx=ctx)
        qa = C.qp_solve(Ba, eps, conv=1e-10, ctx=ctx)
        Bf = C.transform(ref_cd.Lbuf, ref_cd.nvec, Cm, w.nocc, w.targets, "fp64", ctx=ctx)
        qf = C.qp_solve(Bf, eps, conv=1e-10, ctx=ctx)
        acd_report = {"products": int(a.products.size), "per_atom": a.per_atom, "vectors": a.cd.nvec,
                      "full_cd_vectors": ref_cd.nvec, "acd_ms": round((ta1 - ta0) * 1e3, 3),
                      "full_cd_ms": round((ta2 - ta1) * 1e3, 3),
                      "speedup": round((ta2 - ta1) / (ta1 - ta0), 2),
                      "max_qp_shift_meV_vs_full_cd": float(np.abs(qa.omega - qf.omega).max() * HARTREE_EV * 1e3)}
        del Ba, Bf

    # Dyson poles over the targets (non-diagonal self-energy) against the quasi-particle ones
    dyson_report = None
    if nsel <= 31:
        progress("Dyson poles")
        Bd = C.transform(ref_cd.Lbuf, ref_cd.nvec, Cm, w.nocc, w.targets, "fp64", ctx=ctx)
        C.dyson_solve(Bd, eps, conv=conv, ctx=ctx)                  # warm
        ctx.reset_stats()
        dy = C.dyson_solve(Bd, eps, conv=conv, ctx=ctx)
        sd = ctx.stats()
        qd = C.qp_solve(Bd, eps, conv=conv, ctx=ctx)
        dyson_report = {"roots": nsel, "ms": round(sd["t_dyson_ms"], 3), "max_iters": int(dy.iters.max()),
                        "converged": int((dy.status == 0).sum()),
                        "max_shift_meV_vs_quasiparticle": float(np.abs(dy.omega - qd.omega).max() * HARTREE_EV * 1e3),
                        "min_pole_strength": float(dy.pole.min())}
        del Bd

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"f64 CD / {args.prec} contraction",
        "data": "synthetic",
        "config": {"workload": (f"{args.workload}: truncated-icosahedron cage, N={w.nbf} s-Gaussians, "
                                f"{npairs} pairs, delta={delta:g}, nocc={w.nocc}, nvirt={w.nvirt}, "
                                f"{nsel} targets, Newton Delta={conv:g}"),
                   "nvec": M, "prec": args.prec},
        "roofline": roofline,
        "cd": {"ms": round(st_run["t_cd_ms"] / args.steps, 3), "steps": M, "kernels": cd_kernels,
               "transform_overlapped": not args.no_overlap,
               # bytes the plain one-vector-per-step algorithm streams, over the whole decomposition
               "plain_algorithm_equivalent_gbs": round(st_run["bytes_cd"] / (st_run["t_cd_ms"] / 1e3) / 1e9, 1)},
        "phases_ms": {k: round(st_run[k] / args.steps, 3) for k in
                      ("t_cd_ms", "t_transform_ms", "t_contract_ms", "t_epilogue_ms", "t_newton_ms")},
        "precision": prec_report,
        "backward": backward,
        "mp2": mp2_report,
        "sweep": sweep,
        "acd": acd_report,
        "dyson": dyson_report,
        "wall_s": round(wall, 3),
    }
    if not args.no_cpu_baseline and args.workload == "c60":
        out["cpu_baseline"] = cpu_baseline(w, delta, conv, args.cpu_targets)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
