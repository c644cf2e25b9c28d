"""Throughput of the k-point CCGF hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic input: build
b/e vectors, solve every shifted IP and EA system of the batch with the batched
FP64 GMRES (sigma products on MFMA), assemble G = G+ + G-.  The workload is the
Si-like 2x2x2 k-mesh system (4 occupied + 26 virtual spin orbitals per cell,
complex k-blocks, eta = 0.005 Ha): each step covers all 30 orbitals at K = Gamma
and 8 frequencies of the 64-point grid on [-1, 1] Ha, with GMRES stopped at a
relative residual of 1e-8 so that G meets the 1e-6 relative-error target.

Prints ONE JSON line (see README / DESIGN for the fields).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "G(ω) points/sec at 1e-6 rel. error, learned+mixed vs plain FP64; MFMA util"
PEAK_FP64 = 78.6e12  # MI355X dense FP64 matrix peak, FLOP/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="si_k222")
    ap.add_argument("--nw", type=int, default=4, help="frequencies per step (spread over the grid)")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--restart", type=int, default=100)
    ap.add_argument("--maxiter", type=int, default=12000)
    ap.add_argument("--precond-eta", type=float, default=0.2)
    ap.add_argument("--recycle-k", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", choices=["sigma", "copy"], default=None,
                    help="counter-collection runs: 'sigma' applies 3 EA and 3 IP sigma products to the step's "
                         "batch; 'copy' copies a 1 GiB buffer once (HBM-traffic calibration)")
    ap.add_argument("--cpu-sample-s", type=float, default=20.0)
    return ap.parse_args()


def cpu_baseline(sysm, sigma_per_point, budget_s):
    """The oracle timed on the host: sigma products at K = Gamma of the same
    workload, scaled to points/s with the sigma products per point measured on
    the GPU run (the intermediates build is excluded, as cc_gf_init is)."""
    import threading

    from oracle import eom
    from paper_2208_07478_amd import synth

    try:
        import torch
        threads = torch.get_num_threads()
    except Exception:  # pragma: no cover
        threads = os.cpu_count()
    t0 = time.perf_counter()
    E = eom.EOMSystem(sysm)
    build_s = time.perf_counter() - t0
    per = {}
    for part in ("ea", "ip"):
        n = E.size(part)
        x = synth.random_vectors(n, 1, seed=7)[0]
        ts = []
        t_start = time.perf_counter()
        while not ts or (time.perf_counter() - t_start < budget_s / 2 and len(ts) < 5):
            t1 = time.perf_counter()
            E.sigma(part, 0, x)
            ts.append(time.perf_counter() - t1)
        per[part] = (float(np.mean(ts)), len(ts))
    sec_per_point = per["ea"][0] * sigma_per_point["ea"] + per["ip"][0] * sigma_per_point["ip"]
    return {
        "value": 1.0 / sec_per_point,
        "unit": "G(w) points/s",
        "cores": int(os.environ.get("OMP_NUM_THREADS", threads) or threads),
        "kind": "oracle",
        "sample": (f"{per['ea'][1]} EA + {per['ip'][1]} IP oracle sigma products at K=Gamma "
                   f"({per['ea'][0]:.2f} s / {per['ip'][0]:.3f} s each), scaled by the GPU run's "
                   f"{sigma_per_point['ea']:.0f} EA + {sigma_per_point['ip']:.0f} IP sigma products per point; "
                   f"oracle intermediates build {build_s:.0f} s excluded"),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2208_07478_amd import synth
    from paper_2208_07478_amd.ccgf import Context

    torch.cuda.set_device(0)
    if args.probe == "copy":
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")   # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"probe": "copy", "bytes_read": src.numel() * 8, "bytes_written": dst.numel() * 8}))
        return
    sysm = synth.preset_system(args.workload)
    omega, eta = synth.preset_query(args.workload)
    nmo = sysm.nocc + sysm.nvir
    orbs = list(range(nmo))
    t0 = time.perf_counter()
    ctx = Context(sysm, tol=args.tol, restart_m=args.restart, maxiter=args.maxiter, max_batch=nmo * args.nw,
                  timing=True, precond_eta=args.precond_eta, recycle_k=args.recycle_k)
    init_s = time.perf_counter() - t0
    stride = len(omega) // args.nw
    if args.probe == "sigma":
        nb = nmo * args.nw
        for part in ("ea", "ip"):
            X = torch.from_numpy(synth.random_eom_vectors(sysm.kmesh, sysm.nocc, sysm.nvir, part, 0, nb,
                                                          seed=11)).cuda()
            for _ in range(3):
                ctx.sigma(part, 0, X)
        torch.cuda.synchronize()
        ctx.close()
        print(json.dumps({"probe": "sigma", "nvec": nb, "products": 3}))
        return

    def freqs(i):
        # frequencies i, i + stride, ... : every step samples the whole grid
        return omega[(i % stride)::stride][:args.nw]

    def step(i):
        # every step solves the same batch: all orbitals at the frequencies of step 0
        return ctx.solve([0], orbs, freqs(0), eta, allow_noconv=True)

    for i in range(args.warmup):
        print(f"warmup step {i}", file=sys.stderr, flush=True)
        step(i)
    torch.cuda.synchronize()
    tot = {"big_ms": 0.0, "big_launches": 0, "big_flops": 0.0, "n_sigma": 0, "n_iterations": 0,
           "sigma_ms": 0.0, "n_solves": 0, "max_rel_residual": 0.0, "n_unconverged": 0}
    sig_parts = {"ea": 0, "ip": 0}
    t1 = time.perf_counter()
    results = []
    for i in range(args.steps):
        G, Gp, Gm, st = step(args.warmup + i)
        results.append((args.warmup + i, G))
        for k in tot:
            if k == "max_rel_residual":
                tot[k] = max(tot[k], st[k])
            else:
                tot[k] += st[k]
        print(f"step {i}: {st['seconds']:.2f} s, {st['n_iterations']} iterations", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    points = args.steps * nmo * args.nw
    value = points / elapsed

    # per-part sigma counts for the CPU baseline scaling: one more step with one part at a time
    sl = freqs(0)
    for part in ("ea", "ip"):
        _, _, _, stp = ctx.solve([0], orbs, sl, eta, parts=part, allow_noconv=True)
        sig_parts[part] = stp["n_sigma"] / (nmo * args.nw)
    # accuracy of the timed tolerance against a tight solve of the same points (one frequency)
    ctx_t = Context(sysm, tol=1e-11, restart_m=args.restart, maxiter=2 * args.maxiter, max_batch=nmo,
                    precond_eta=args.precond_eta)
    Gt, _, _, stt = ctx_t.solve([0], orbs, sl[:1], eta, allow_noconv=True)
    ctx_t.close()
    Gchk, _, _, _ = ctx.solve([0], orbs, sl[:1], eta, allow_noconv=True)
    rel = float(np.max(np.abs(Gchk - Gt).max(axis=-1) / np.abs(Gt).max(axis=-1)))
    ctx.close()

    avg_ms = tot["big_ms"] / max(tot["big_launches"], 1)
    flops_per_launch = tot["big_flops"] / max(tot["big_launches"], 1)
    achieved = flops_per_launch / (avg_ms * 1e-3) if avg_ms > 0 else 0.0
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "G(w) points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c128",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: Si-like {sysm.kmesh[0]}x{sysm.kmesh[1]}x{sysm.kmesh[2]} k-mesh, "
                         f"{sysm.nocc} occ + {sysm.nvir} vir spin orbitals/cell, K=Gamma, {nmo} orbitals x "
                         f"{args.nw} omega per step (every {stride}th point of the {len(omega)}-point grid on "
                         f"[-1,1] Ha), eta={eta}, plain FP64 GMRES({args.restart}) tol={args.tol}, "
                         f"preconditioner damping {args.precond_eta} Ha, maxiter {args.maxiter}"),
            "points_per_step": nmo * args.nw,
            "precision": "plain_f64",
        },
        "accuracy": {"max_rel_err_vs_tol1e-11": rel, "reference_unconverged": stt["n_unconverged"],
                     "max_rel_residual": tot["max_rel_residual"], "unconverged": tot["n_unconverged"]},
        "solver": {"iterations_per_solve": tot["n_iterations"] / max(tot["n_solves"], 1),
                   "sigma_ms_share": tot["sigma_ms"] / (1e3 * elapsed),
                   "init_s": init_s},
        "roofline": {"bound": "mfma", "kernel": "k_cgemm_f64<0> (EA 1/2 W_abcd r_i^cd)",
                     "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64, "traffic": None,
                     "avg_ms": avg_ms, "flops_per_launch": flops_per_launch},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sysm, sig_parts, args.cpu_sample_s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
