#!/usr/bin/env python3
"""Throughput of the DDM-ELM hot path on one MI355X.

One step = one complete solve (Algorithm 1 of the paper: feature assembly,
batched local least squares, interface Schur complement formation and
solve, back-solve of every local output layer) of the 8x8 Poisson workload:
64 subdomains, 400 tanh neurons each (U[-4,4]), 40x40 interior points and 40
points per edge, manufactured solution sin(pi x) sin(pi y).  Every step uses
its own hidden-layer seed; all inputs are resident in HBM before timing.

Prints one JSON line.  The oracle (FP64 CPU reference) is timed beside it on
the host cores for one solve of the same workload, and its answer is the
parity reference for the GPU result of that instance.
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

MFMA_F64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
HBM_PEAK_GBS = 8000.0
PMC_SUMMARY = os.path.join(ROOT, "profiles", "gram_8x8_fp64_batch8_pmc.txt")


def measured_traffic(gram_code, batch):
    """HBM bytes per Gram launch from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary, if it was taken with this kernel source, kernel choice and batch; else None."""
    import hashlib
    try:
        kv = {}
        for line in open(PMC_SUMMARY):
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        src = os.path.join(ROOT, "paper_2406_15959_amd", "csrc", "kernels.hip")
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if kv.get("kernels_hip_sha256") != sha or int(kv["gram_code"]) != gram_code or int(kv["batch"]) != batch:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch", type=int, default=8, help="problem instances solved together per step")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy_mib > 0:
        import torch
        nbytes = args.calibrate_copy_mib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_dispatch": nbytes, "dispatches": 3}), flush=True)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workload as wl
    from paper_2406_15959_amd import binding as B

    dev = torch.device("cuda:0")
    P = wl.CONFIG_8x8
    cp = B.make_problem(P.x0, P.x1, P.y0, P.y1, P.nsub_x, P.nsub_y, P.neurons, P.q_x, P.q_y,
                        P.m_bdry_edge, P.m_ifc_edge, P.op)
    nb = max(1, args.batch)
    plan = B.Plan(cp, batch=nb)
    s = plan.sizes
    ipts = plan.points(B.POINTS_INTERIOR)
    bpts = plan.points(B.POINTS_BOUNDARY)
    f, g, _ = wl.sample_data(P, ipts, bpts)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(dev)
    df, dg = t(np.stack([f] * nb)), t(np.stack([g] * nb))
    # two batches of instances with distinct hidden-layer seeds, alternated step by step
    seeds = [2000 + i for i in range(2 * nb)]
    inst = []
    for k in range(2):
        Ws, bs = zip(*[wl.hidden_params(P, sd) for sd in seeds[k * nb:(k + 1) * nb]])
        inst.append((t(np.stack(Ws)), t(np.stack(bs))))
    du = torch.zeros(nb * s.n_interface, dtype=torch.float64, device=dev)
    dc = torch.zeros(nb * s.nsub * s.neurons, dtype=torch.float64, device=dev)

    tuned = plan.autotune()
    for i in range(args.warmup):
        W, b = inst[i % len(inst)]
        plan.solve(W, b, df, dg, None, du, dc)
    torch.cuda.synchronize()
    info = plan.solve_info()
    if info.status != 0:
        raise SystemExit(f"warmup solve failed with status {info.status}")

    plan.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        W, b = inst[i % len(inst)]
        plan.solve(W, b, df, dg, None, du, dc)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stage_ms, nsolved = plan.stage_times()
    plan.set_timing(False)
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = args.steps * nb / elapsed

    # Parity of instance 0 against the oracle (and the oracle's own timing).
    W0, b0 = inst[0]
    plan.solve(W0, b0, df, dg, None, du, dc)
    info = plan.solve_info()
    ex, ey = wl.eval_grid(P)
    xy = t(np.stack([ex, ey], 1))
    uh = torch.zeros(len(ex), dtype=torch.float64, device=dev)
    # instance 0 of the batch: its slices of W, b, c are the leading ones
    plan.eval(W0[0].contiguous(), b0[0].contiguous(), dc[:s.nsub * s.neurons].contiguous(), xy, uh)
    torch.cuda.synchronize()
    u_gpu = du[:s.n_interface].cpu().numpy()
    uh_gpu = uh.cpu().numpy()
    parity = {"status": int(info.status),
              "rel_l2_vs_exact_uh": float(np.linalg.norm(uh_gpu - wl.exact_u(P, ex, ey)) /
                                          np.linalg.norm(wl.exact_u(P, ex, ey)))}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import ddm
        from oracle.layout import build_layout
        try:
            from threadpoolctl import threadpool_info
            threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        except Exception:
            threads = len(os.sched_getaffinity(0))
        lay = build_layout(P)
        Wn, bn = wl.hidden_params(P, seeds[0])
        data = ddm.problem_data(P, lay, wl.source_f, wl.boundary_g, wl.coefficient)
        c0 = time.perf_counter()
        sol = ddm.solve(P, Wn, bn, data, lay)
        c1 = time.perf_counter()
        uh_or = ddm.evaluate(P, lay, Wn, bn, sol.c, ex, ey)
        parity["rel_l2_u_gamma_vs_oracle"] = float(np.linalg.norm(u_gpu - sol.u_gamma) / np.linalg.norm(sol.u_gamma))
        parity["rel_l2_uh_vs_oracle"] = float(np.linalg.norm(uh_gpu - uh_or) / np.linalg.norm(uh_or))
        parity["tolerance"] = 1e-8
        parity["ok"] = bool(info.status == 0 and parity["rel_l2_u_gamma_vs_oracle"] <= 1e-8
                            and parity["rel_l2_uh_vs_oracle"] <= 1e-8)
        cpu = {"value": 1.0 / (c1 - c0), "unit": "solves/s", "cores": int(threads), "kind": "oracle",
               "sample": "one full FP64 oracle solve of the same 8x8 workload (hidden-layer seed %d), "
                         "%.1f s" % (seeds[0], c1 - c0)}

    # Roofline of the dominant kernel: the batched FP64 MFMA Gram (SYRK)
    # launch.  Algorithmic work per launch: sum over subdomains of
    # m_s * n * (n + 1) flops (symmetric product, lower triangle).
    m_rows = P.q_x * P.q_y + 4 * P.m_ifc_edge if P.m_ifc_edge == P.m_bdry_edge else s.max_rows
    n = P.neurons
    flops_per_solve = P.nsub * m_rows * 3 * n * (n + 1)
    gram_ms = stage_ms[1] / max(nsolved, 1) / 3.0          # average Gram launch (HIP events)
    achieved = nb * flops_per_solve / 3.0 / (gram_ms * 1e-3) / 1e12 if gram_ms > 0 else 0.0
    kname = ("gemm_strip_kernel<T=%d>" % tuned[0]) if tuned[0] >= 4 else ("gemm_f64_kernel variant %d" % (-1 - tuned[0]))
    roofline = {"bound": "mfma", "kernel": "gram product, " + kname,
                "achieved": achieved, "peak": MFMA_F64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / MFMA_F64_PEAK_TFLOPS, "traffic": measured_traffic(tuned[0], nb),
                "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "avg_launch_ms": gram_ms}
    stages = {name: v / max(nsolved, 1) for name, v in zip(B.STAGE_NAMES, stage_ms)}   # per step
    ok = parity.get("ok", info.status == 0)
    out = {
        "metric": "ELM-DDM solves/sec at fixed rel-L2 vs FP64 oracle: mixed+learned vs plain FP64",
        "value": value if ok else 0.0,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "mode": "plain FP64",
        "config": {"workload": "2D Poisson 8x8 subdomains, 400 tanh neurons each (U[-4,4]), "
                               "40x40 interior points, 40 points per boundary/interface edge; plain FP64",
                   "subdomains": P.nsub, "neurons": n, "interface_unknowns": s.n_interface,
                   "instances_per_step": nb, "autotuned_kernels": tuned},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "stages_ms_per_step": stages,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
