"""Throughput of the k-point CCGF hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic input: build
b/e vectors, solve every shifted IP and EA system of the batch with the batched
GMRES (sigma products on MFMA), assemble G = G+ + G-.  The workload is the
Si-like 2x2x2 k-mesh system (4 occupied + 26 virtual spin orbitals per cell,
complex k-blocks, eta = 0.005 Ha): each step covers all 30 orbitals at K = Gamma
and 8 frequencies spread over the 64-point grid on [-1, 1] Ha (240 points), with
120 right-hand sides in flight per part.

Each solver form (plain FP64; mixed FP32 or BF16-split sigma with FP64
refinement) is timed on the same batch at the same GMRES tolerance, and its G
is compared with a tight plain-FP64 solve of every 4th frequency of the batch
(all orbitals); a point counts at the 1e-6 relative-error target (per orbital:
max over the checked frequencies of |dG| / max |G|).  `value` is the points/s
of the fastest form that meets it.

Prints ONE JSON line.
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "G(ω) points/sec at 1e-6 rel. error, learned+mixed vs plain FP64; MFMA util"
# MI355X dense matrix peaks of each form's MFMA dtype, FLOP/s
PEAK = {"plain_f64": 78.6e12, "mixed_f32": 157.3e12, "mixed_bf16x3": 2.5e15, "learned_mixed_f32": 157.3e12}
# the dominant kernel of each form (EA 1/2 W_abcd r_i^cd over the blocks ka < kb), all N tile
# widths the autotuner may pick (the traffic record covers the same family)
GEMM_NAME = {"plain_f64": "k_cgemm<0, double>", "mixed_f32": "k_cgemm<0, float>",
             "mixed_bf16x3": "k_cgemm_b3<0>", "learned_mixed_f32": "k_cgemm<0, float>"}
PRECISION = {"plain_f64": "f64", "mixed_f32": "f32", "mixed_bf16x3": "bf16x3", "learned_mixed_f32": "f32"}
DTYPE = {"plain_f64": "c128", "mixed_f32": "c64 sigma / c128 Krylov", "mixed_bf16x3": "bf16x3 sigma / c128 Krylov",
         "learned_mixed_f32": "c64 sigma / c128 Krylov, FP32 network"}
TARGET = 1e-6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--workload", default="si_k222")
    ap.add_argument("--nw", type=int, default=8, help="frequencies per step (spread over the grid)")
    ap.add_argument("--batch", type=int, default=120, help="right-hand sides in flight")
    ap.add_argument("--forms", default="plain_f64,mixed_f32,mixed_bf16x3",
                    help="comma list of plain_f64, mixed_f32, mixed_bf16x3, learned_mixed_f32")
    ap.add_argument("--tol", type=float, default=2e-7)
    ap.add_argument("--ref-tol", type=float, default=1e-9)
    ap.add_argument("--check-every", type=int, default=4, help="reference solve on every k-th step frequency")
    ap.add_argument("--restart", type=int, default=200)
    ap.add_argument("--maxiter", type=int, default=12000)
    ap.add_argument("--precond-eta", type=float, default=0.4)
    ap.add_argument("--restart-tail", type=int, default=0,
                    help="restart length once the queue is empty and at most a quarter of the slots iterate")
    ap.add_argument("--seed-m", type=int, default=128,
                    help="shared-Krylov seed steps per orbital before the solves (0: start from zero)")
    ap.add_argument("--no-check", action="store_true", help="skip the reference solve (profiling runs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", choices=["sigma", "copy"], default=None,
                    help="counter-collection runs: 'sigma' applies 6 EA and 6 IP sigma products to a batch of "
                         "--batch vectors (the first ones are the autotuner's trials, the last 3 its choice); "
                         "'copy' copies a 1 GiB buffer once (HBM-traffic calibration)")
    ap.add_argument("--probe-precision", default="f64")
    ap.add_argument("--cpu-sample-s", type=float, default=20.0)
    return ap.parse_args()


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summaries,
    or None when the kernel source changed since the counters were taken."""
    src = os.path.join(ROOT, "paper_2208_07478_amd", "csrc", "sigma.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        for line in open(os.path.join(pdir, name)):
            if line.startswith("<!-- traffic "):
                rec = json.loads(line[len("<!-- traffic "):].rstrip().rstrip("->").strip())
                if rec.get("kernel") == kernel and rec.get("source_sha256") == sha:
                    return rec
    return None


def cpu_baseline(sysm, sigma_per_point, budget_s):
    """The oracle timed on the host: sigma products at K = Gamma of the same
    workload, scaled to points/s with the sigma products per point measured on
    the GPU run (the intermediates build is excluded, as cc_gf_init is)."""
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
                   f"({per['ea'][0]:.2f} s / {per['ip'][0]:.3f} s each), scaled by the headline form's "
                   f"{sigma_per_point['ea']:.0f} EA + {sigma_per_point['ip']:.0f} IP sigma products per point; "
                   f"oracle intermediates build {build_s:.0f} s excluded"),
    }


def col_err(G, Gref):
    """Per orbital: max over frequencies of |G - Gref| / max |Gref|; the worst orbital."""
    den = np.abs(Gref).max(axis=-1)
    den = np.where(den > 0, den, 1.0)
    return float(np.max(np.abs(G - Gref).max(axis=-1) / den))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; --gpus must be 1"}))
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
    nb = nmo * args.nw
    stride = len(omega) // args.nw
    wsel = omega[::stride][:args.nw]
    opts = dict(tol=args.tol, restart_m=args.restart, maxiter=args.maxiter, max_batch=args.batch,
                precond_eta=args.precond_eta, seed_m=args.seed_m, restart_tail=args.restart_tail)
    if args.probe == "sigma":
        ctx = Context(sysm, precision=args.probe_precision, graphs=False, **opts)
        for part in ("ea", "ip"):
            X = torch.from_numpy(synth.random_eom_vectors(sysm.kmesh, sysm.nocc, sysm.nvir, part, 0, args.batch,
                                                          seed=11)).cuda()
            for _ in range(6):
                ctx.sigma(part, 0, X)
        torch.cuda.synchronize()
        ctx.close()
        print(json.dumps({"probe": "sigma", "nvec": args.batch, "products": 6, "precision": args.probe_precision}))
        return

    forms = [f for f in args.forms.split(",") if f]
    res = {}
    for form in forms:
        t0 = time.perf_counter()
        ctx = Context(sysm, timing=True, precision=PRECISION[form], **opts)
        init_s = time.perf_counter() - t0
        learn = None
        if form.startswith("learned"):
            # train on the grid frequencies midway between the step's (not timed; reported)
            wtrain = omega[stride // 2::stride][:args.nw]
            t1 = time.perf_counter()
            learn = ctx.learn(0, orbs, wtrain, eta, allow_noconv=True)
            learn["seconds"] = time.perf_counter() - t1
            print(f"{form} training: {learn['seconds']:.1f} s", file=sys.stderr, flush=True)

        def step():
            # one pass over the batch: IP then EA solves of all orbitals x frequencies, G = G- + G+
            _, _, Gm, sti = ctx.solve([0], orbs, wsel, eta, parts="ip", allow_noconv=True)
            print(f"{form} IP: {sti['seconds']:.1f} s", file=sys.stderr, flush=True)
            _, Gp, _, ste = ctx.solve([0], orbs, wsel, eta, parts="ea", allow_noconv=True)
            print(f"{form} EA: {ste['seconds']:.1f} s", file=sys.stderr, flush=True)
            return Gm + Gp, sti, ste

        for i in range(args.warmup):
            print(f"{form} warmup step {i}", file=sys.stderr, flush=True)
            step()
        torch.cuda.synchronize()
        tot = {"big_ms": 0.0, "big_launches": 0, "big_flops": 0.0, "n_iterations": 0, "sigma_ms": 0.0,
               "n_solves": 0, "max_rel_residual": 0.0, "n_unconverged": 0, "n_steps": 0, "n_reorth": 0,
               "n_guess": 0}
        nsig = {"ip": 0, "ea": 0}
        t1 = time.perf_counter()
        for i in range(args.steps):
            G, sti, ste = step()
            for st in (sti, ste):
                for k in tot:
                    tot[k] = max(tot[k], st[k]) if k == "max_rel_residual" else tot[k] + st[k]
            nsig["ip"] += sti["n_sigma"]
            nsig["ea"] += ste["n_sigma"]
            print(f"{form} step {i}: {sti['seconds'] + ste['seconds']:.2f} s, "
                  f"{sti['n_iterations'] + ste['n_iterations']} iterations", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t1
        ctx.close()
        avg_ms = tot["big_ms"] / max(tot["big_launches"], 1)
        fl = tot["big_flops"] / max(tot["big_launches"], 1)
        ach = fl / (avg_ms * 1e-3) if avg_ms > 0 else 0.0
        res[form] = {
            "points_per_s": args.steps * nb / elapsed,
            "ms_per_step": 1e3 * elapsed / args.steps,
            "G": G,
            "iterations_per_solve": tot["n_iterations"] / max(tot["n_solves"], 1),
            "guesses_used": tot["n_guess"],
            "batched_steps": tot["n_steps"],
            "mean_active": tot["n_iterations"] / max(tot["n_steps"], 1),
            "reorth_fraction": tot["n_reorth"] / max(tot["n_iterations"], 1),
            "sigma_per_point": {p: nsig[p] / (args.steps * nb) for p in nsig},
            "sigma_ms_share": tot["sigma_ms"] / (1e3 * elapsed),
            "max_rel_residual": tot["max_rel_residual"],
            "unconverged": tot["n_unconverged"],
            "init_s": init_s,
            "learn": learn,
            "roofline": {"bound": "mfma", "kernel": GEMM_NAME[form] + " (EA 1/2 W_abcd r_i^cd, blocks ka < kb; "
                                                                     "N tile 32/64/128 by the autotuner)",
                         "achieved": ach / 1e12, "peak": PEAK[form] / 1e12, "unit": "TFLOP/s",
                         "frac": ach / PEAK[form], "avg_ms": avg_ms, "flops_per_launch": fl,
                         "launches": tot["big_launches"]},
        }

    ref = None
    if not args.no_check:
        # tight plain-FP64 solve of every `check_every`-th frequency of the step, all orbitals
        sub = slice(None, None, args.check_every)
        ctx = Context(sysm, **dict(opts, tol=args.ref_tol, maxiter=3 * args.maxiter, seed_m=0))
        _, _, Gm, sti = ctx.solve([0], orbs, wsel[sub], eta, parts="ip", allow_noconv=True)
        print(f"reference IP: {sti['seconds']:.1f} s", file=sys.stderr, flush=True)
        _, Gp, _, ste = ctx.solve([0], orbs, wsel[sub], eta, parts="ea", allow_noconv=True)
        print(f"reference EA: {ste['seconds']:.1f} s", file=sys.stderr, flush=True)
        ctx.close()
        ref = {"G": Gm + Gp, "tol": args.ref_tol, "unconverged": sti["n_unconverged"] + ste["n_unconverged"],
               "points": int(Gm.shape[1] * Gm.shape[2])}
        for form in res:
            res[form]["max_rel_err"] = col_err(res[form]["G"][:, :, sub], ref["G"])

    def meets(f):
        return ref is not None and res[f]["max_rel_err"] <= TARGET and res[f]["unconverged"] == 0

    ok = [f for f in res if meets(f)] or list(res)
    head = max(ok, key=lambda f: res[f]["points_per_s"])
    h = res[head]
    roof = dict(h["roofline"])
    tr = stored_traffic(GEMM_NAME[head])
    roof["traffic"] = tr["bytes_per_launch"] if tr else None
    if tr:
        roof["traffic_note"] = tr.get("note", "")
    forms_out = {}
    for f, r in res.items():
        forms_out[f] = {k: v for k, v in r.items() if k not in ("G",)}
    out = {
        "metric": METRIC,
        "value": h["points_per_s"],
        "unit": "G(w) points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[head],
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: Si-like {sysm.kmesh[0]}x{sysm.kmesh[1]}x{sysm.kmesh[2]} k-mesh, "
                         f"{sysm.nocc} occ + {sysm.nvir} vir spin orbitals/cell, K=Gamma, {nmo} orbitals x "
                         f"{args.nw} omega per step (every {stride}th point of the {len(omega)}-point grid on "
                         f"[-1,1] Ha), eta={eta}, GMRES({args.restart}) tol={args.tol}, {args.batch} right-hand "
                         f"sides in flight, preconditioner damping {args.precond_eta} Ha, maxiter {args.maxiter}"),
            "form": head,
            "points_per_step": nb,
        },
        "accuracy": {"target_rel_err": TARGET, "reference_tol": args.ref_tol,
                     "checked_points": ref["points"] if ref else 0,
                     "reference_unconverged": ref["unconverged"] if ref else None,
                     "max_rel_err": h.get("max_rel_err"), "meets_target": meets(head)},
        "forms": forms_out,
        "speedup_vs_plain_f64": (h["points_per_s"] / res["plain_f64"]["points_per_s"]
                                 if "plain_f64" in res else None),
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sysm, h["sigma_per_point"], args.cpu_sample_s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
