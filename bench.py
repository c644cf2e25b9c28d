"""Throughput of the k-point CCGF hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic input: build
the b / e vectors, solve every shifted IP and EA system of the batch with the
batched GMRES (sigma products on MFMA), assemble G = G+ + G-.  The workload is
the Si-like 3x3x3 k-mesh system (27 k-points, 4 occupied + 26 virtual spin
orbitals per cell, complex k-blocks, eta = 0.005 Ha): step s covers the ten
orbitals p = g, g + 3, ..., g + 27 (g = s mod 3) at K = Gamma at one frequency
of the 256-point grid on [-1, 1] Ha, grid point (37 s + 5) mod 256, so that
successive steps spread over the grid and over the orbitals (10 points per
step; the three groups hold 2, 1 and 1 occupied orbitals).

Forms:
  * the headline form (default ``learned_mixed_bf16x3``): sigma products from
    BF16-split operands (hi + lo, three BF16 MFMA products per real product,
    FP32 accumulation) with FP64 refinement, starting each solve from the guess of a network trained
    (outside the timed region, reported) on plain solves of all orbitals at the
    frequencies of the first --ntrain warmup steps (those solves are the
    warmup's work for those steps), and giving each solve the preconditioner
    damping a second network predicts from probe solves at those frequencies;
  * ``plain_f64`` on the first ``--compare-steps`` timed steps (same
    frequencies, same tolerance), for the speed-up at equal accuracy;
  * the headline context with its network switched off on the same steps (the
    network's own gain);
  * a tight plain-FP64 solve (tol 1e-10) of the same steps, the accuracy
    reference of every form: a point meets the target when |G - G_ref| <=
    1e-6 |G_ref|.

The plain FP64 path behind the reference is pinned to the CPU oracle by the
parity tests (full G on the Si-like 2x2x2 system, sampled sigma blocks on this
3x3x3 system).  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

import numpy as np

T_START = time.perf_counter()
ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "G(ω) points/sec at 1e-6 rel. error, learned+mixed vs plain FP64; MFMA util"
PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16x3": 2.5e15}
HBM_PEAK = 8.0e12
GEMM_NAME = {"f64": "k_cgemm<0, double>", "f32": "k_cgemm<0, float>", "bf16x3": "k_cgemm_b3<0>"}
DTYPE = {"f64": "c128", "f32": "c64 sigma / c128 Krylov", "bf16x3": "bf16x3 sigma / c128 Krylov"}
TARGET = 1e-6


def log(*a):
    print(f"[{time.perf_counter() - T_START:6.1f} s]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="si_k333")
    ap.add_argument("--form", default="learned_mixed_bf16x3",
                    help="headline form: [learned_]mixed_f32, [learned_]mixed_bf16x3 or plain_f64")
    ap.add_argument("--compare-steps", type=int, default=2,
                    help="timed steps also solved by plain FP64, by the headline without its network and "
                         "by the tight reference")
    ap.add_argument("--tol", type=float, default=2e-7)
    ap.add_argument("--ref-tol", type=float, default=1e-10)
    ap.add_argument("--restart", type=int, default=200)
    ap.add_argument("--batch", type=int, default=90, help="right-hand sides in flight per part (fitted to memory)")
    ap.add_argument("--maxiter", type=int, default=20000)
    ap.add_argument("--precond-eta", type=float, default=0.25)
    ap.add_argument("--ntrain", type=int, default=4, help="training frequencies of the networks (the first "
                                                            "warmup steps' frequencies, all orbitals)")
    ap.add_argument("--probe-steps", type=int, default=30, help="GMRES steps of each probe solve of the "
                                                                 "preconditioner network (-1: none)")
    ap.add_argument("--budget-s", type=float, default=430.0,
                    help="wall-clock budget: optional legs are skipped when they would exceed it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", choices=["sigma", "ortho", "copy"], default=None,
                    help="counter-collection runs: 'sigma' applies 6 EA and 6 IP sigma products to a batch of "
                         "--batch vectors; 'ortho' runs one GMRES cycle of --probe-steps steps for ten EA "
                         "right-hand sides (prints the Gram-Schmidt kernels' algorithmic bytes); 'copy' copies "
                         "a 1 GiB buffer once (HBM-traffic calibration)")
    ap.add_argument("--probe-precision", default="f32")
    return ap.parse_args()


def form_precision(form):
    return "f64" if form == "plain_f64" else form.split("_")[-1]


def kernel_source_sha():
    """SHA-256 of the source of the sigma GEMM kernels (k_cgemm, k_cgemm_b3 and their tile
    bodies, from the MFMA arithmetic helpers to the launch helpers)."""
    src = open(os.path.join(ROOT, "paper_2208_07478_amd", "csrc", "sigma.hip")).read()
    a = src.index("// Real arithmetic of one GEMM variant")
    b = src.index("template <int TAG, typename R, int TNT>\nstatic void launch_t(")
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def stored_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summaries,
    or None when the kernel source changed since the counters were taken."""
    sha = kernel_source_sha()
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


def host_info():
    info = {"nproc": os.cpu_count(), "cpu": platform.processor() or "", "ram_gb": None}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["cpu"] = line.split(":", 1)[1].strip()
                break
        for line in open("/proc/meminfo"):
            if line.startswith("MemTotal"):
                info["ram_gb"] = round(int(line.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return info


def cpu_baseline(sysm, sigma_per_point, budget_s):
    """The oracle timed on the host (bounded sample): at K = Gamma, one 2p1h
    output block of sigma_EA and one 2h1p block of sigma_IP for one vector, from
    cold H-bar blocks (the oracle forms every block from the factor on demand;
    its one-body blocks are built beforehand and excluded, as cc_gf_init is),
    extrapolated linearly to the Nk^2 blocks of a product, then to points with
    the headline form's sigma products per point."""
    from oracle import blocks
    from paper_2208_07478_amd import synth

    def threads():
        try:
            from threadpoolctl import threadpool_info
            return max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        except Exception:  # pragma: no cover
            return os.cpu_count()

    def sample(B):
        per = {}
        for part in ("ip", "ea"):
            x = synth.random_eom_vectors(sysm.kmesh, sysm.nocc, sysm.nvir, part, 0, 1, seed=7)[0]
            t = time.perf_counter()
            B.sigma_block(part, 0, x, 0, 0)
            per[part] = time.perf_counter() - t
        return per

    t0 = time.perf_counter()
    B = blocks.BlockSystem(sysm)
    B.fock()
    build_s = time.perf_counter() - t0
    nth = threads()
    per = sample(B)
    nblk = sysm.nk ** 2
    sec_point = nblk * (per["ea"] * sigma_per_point["ea"] + per["ip"] * sigma_per_point["ip"])
    out = {
        "value": 1.0 / sec_point,
        "unit": "G(w) points/s",
        "cores": nth,
        "kind": "oracle",
        "sample": (f"oracle.blocks at K=Gamma: one sigma_EA output block ({per['ea']:.1f} s) and one sigma_IP "
                   f"block ({per['ip']:.2f} s), one vector, cold H-bar blocks, x{nblk} blocks per product, x the "
                   f"headline's {sigma_per_point['ea']:.0f} EA + {sigma_per_point['ip']:.0f} IP products per "
                   f"point; one-body blocks ({build_s:.0f} s) excluded"),
        "host": host_info(),
    }
    # one thread: the IP block again from cold blocks (the EA block would take minutes); the
    # 1-thread figure scales the value by that block's thread speed-up
    left = budget_s - (time.perf_counter() - T_START)
    if left > 20 * per["ip"] + 5:
        B1 = blocks.BlockSystem(sysm)
        B1._F = B._F
        from threadpoolctl import threadpool_limits
        x = synth.random_eom_vectors(sysm.kmesh, sysm.nocc, sysm.nvir, "ip", 0, 1, seed=7)[0]
        with threadpool_limits(1):
            t = time.perf_counter()
            B1.sigma_block("ip", 0, x, 0, 0)
            t1 = time.perf_counter() - t
        out["thread_speedup_ip_block"] = t1 / per["ip"]
        out["value_1thread_est"] = out["value"] / (t1 / per["ip"])
        out["sample_1thread"] = (f"IP block on 1 thread {t1:.2f} s vs {per['ip']:.2f} s on {nth}; value_1thread_est "
                                 f"divides the value by that ratio")
    return out


def pointwise_err(G, Gref):
    return float(np.max(np.abs(G - Gref) / np.maximum(np.abs(Gref), 1e-300)))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the solves of different K, orbitals "
                                   "and frequencies are independent: sharding them over GPUs needs no exchange "
                                   "but the final gather of G); use --gpus 1"}))
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
    grid, eta = synth.preset_query(args.workload)
    nmo = sysm.nocc + sysm.nvir
    orbs = list(range(nmo))
    ng = len(grid)
    nsteps = args.warmup + args.steps
    wstep = [float(grid[(37 * s + 5) % ng]) for s in range(nsteps)]
    ostep = [list(range(s % 3, nmo, 3)) for s in range(nsteps)]
    opts = dict(tol=args.tol, restart_m=args.restart, maxiter=args.maxiter, max_batch=args.batch,
                precond_eta=args.precond_eta)
    log(f"{args.workload}: {sysm.kmesh}, {sysm.nocc}+{sysm.nvir}")
    if args.probe == "ortho":
        # one cycle of L steps for B slots, no second Gram-Schmidt pass: per step j the basis
        # is read twice over its j + 1 vectors (k_dots, k_sub_proj), and these two kernels
        # read w four times (two norms, the dot, the update) and write it once
        L, B = max(args.probe_steps, 1), 10
        ctx = Context(sysm, precision=args.probe_precision, tol=1e-300, restart_m=L, maxiter=L, max_batch=B,
                      precond_eta=args.precond_eta, reorth_ratio=1e-30)
        ctx.solve([0], orbs[:B], [wstep[0]], eta, parts="ea", allow_noconv=True)
        torch.cuda.synchronize()
        ctx.close()
        nk, no, nv = int(np.prod(sysm.kmesh)), sysm.nocc, sysm.nvir
        nb = nv + no * (nk * nk * nv * nv - nk * nv) // 2   # unique EA amplitudes at any K
        eb = 16                                             # basis element bytes (complex double)
        basis = B * nb * eb * L * (L + 1)                   # both passes over the basis, all steps
        wvec = B * nb * 16 * 5 * L
        print(json.dumps({"probe": "ortho", "slots": B, "steps": L, "unique_len": nb, "basis_elem_bytes": eb,
                          "precision": args.probe_precision, "basis_bytes": basis, "w_bytes": wvec,
                          "algorithmic_bytes": basis + wvec}))
        return
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

    def run_steps(ctx, steps, tag):
        """Solve the listed steps; returns (G [len(steps)][10], seconds, totals)."""
        tot = {"big_ms": 0.0, "big_launches": 0, "big_flops": 0.0, "big_bytes": 0.0, "n_iterations": 0,
               "n_solves": 0, "n_unconverged": 0, "n_sigma_ea": 0, "n_sigma_ip": 0, "n_guess": 0, "n_guess_rejected": 0,
               "max_rel_residual": 0.0}
        Gs, secs = [], []
        for s in steps:
            w, ob = wstep[s], ostep[s]
            t = time.perf_counter()
            _, _, Gm, sti = ctx.solve([0], ob, [w], eta, parts="ip", allow_noconv=True)
            _, Gp, _, ste = ctx.solve([0], ob, [w], eta, parts="ea", allow_noconv=True)
            secs.append(time.perf_counter() - t)
            Gs.append((Gm + Gp)[0, :, 0])
            for st in (sti, ste):
                for k in ("big_ms", "big_launches", "big_flops", "big_bytes", "n_iterations", "n_solves",
                          "n_unconverged", "n_guess", "n_guess_rejected"):
                    tot[k] += st[k]
                tot["max_rel_residual"] = max(tot["max_rel_residual"], st["max_rel_residual"])
            tot["n_sigma_ip"] += sti["n_sigma"]
            tot["n_sigma_ea"] += ste["n_sigma"]
            log(f"{tag} w={w:+.4f}: {secs[-1]:.2f} s, {sti['n_iterations'] + ste['n_iterations']} iterations")
        return np.array(Gs), secs, tot

    form = args.form
    prec = form_precision(form)
    learned = form.startswith("learned")
    res = {}
    # ---------------------------------------------------------------- headline
    t0 = time.perf_counter()
    ctx = Context(sysm, timing=True, precision=prec, **opts)
    init_s = time.perf_counter() - t0
    log(f"{form}: cc_gf_init {init_s:.1f} s")
    learn = None
    nwarm_plain = 0
    if learned and args.warmup > 0:
        # the network learns from plain solves of all orbitals at the first warmup steps' frequencies
        # (at least one ordinary warmup step follows when there are two or more: the learned
        # path's first solves build their own plans)
        nwarm_plain = max(1, min(args.ntrain, args.warmup - 1 if args.warmup > 1 else 1))
        wtrain = sorted(set(wstep[:nwarm_plain]))
        learn = {"omega_train": wtrain, "seconds": 0.0}
        for part in ("ip", "ea"):  # (one part per call: each prints when it is done)
            t1 = time.perf_counter()
            ls = ctx.learn(0, orbs, wtrain, eta, parts=part, probe=args.probe_steps, allow_noconv=True)
            ls["seconds"] = time.perf_counter() - t1
            learn[part] = ls
            learn["seconds"] += ls["seconds"]
            log(f"{form}: {part} networks trained at {len(wtrain)} frequencies in {ls['seconds']:.1f} s")
    run_steps(ctx, range(nwarm_plain, args.warmup), f"{form} warmup")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    Gh, secs_h, tot = run_steps(ctx, range(args.warmup, nsteps), form)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t1
    ppstep = len(ostep[0])
    npts = sum(len(ostep[s]) for s in range(args.warmup, nsteps))
    avg_ms = tot["big_ms"] / max(tot["big_launches"], 1)
    fl = tot["big_flops"] / max(tot["big_launches"], 1)
    ach = fl / (avg_ms * 1e-3) if avg_ms > 0 else 0.0
    sigma_pp = {"ea": tot["n_sigma_ea"] / npts, "ip": tot["n_sigma_ip"] / npts}
    res[form] = {"points_per_s": npts / elapsed, "ms_per_step": 1e3 * elapsed / args.steps,
                 "iterations_per_solve": tot["n_iterations"] / max(tot["n_solves"], 1),
                 "sigma_per_point": sigma_pp, "unconverged": tot["n_unconverged"],
                 "guesses_used": tot["n_guess"], "guesses_rejected": tot["n_guess_rejected"],
                 "max_rel_residual": tot["max_rel_residual"], "init_s": init_s, "learn": learn}
    ncmp = max(1, min(args.compare_steps, args.steps))
    wcmp = list(range(args.warmup, args.warmup + ncmp))
    cmp_secs = {form: sum(secs_h[:ncmp])}
    cmp_G = {form: Gh[:ncmp]}
    budget = args.budget_s

    def left():
        return budget - (time.perf_counter() - T_START)

    est_step = elapsed / args.steps
    if learned and left() > 2.0 * ncmp * est_step + 150:
        # the same context with its network switched off: what the network gains
        ctx.learn_enable(False)
        G, secs, t_ = run_steps(ctx, wcmp, form.replace("learned_", "") + " (network off)")
        cmp_secs["network_off"] = sum(secs)
        cmp_G["network_off"] = G
        res[form]["network_off"] = {"iterations_per_solve": t_["n_iterations"] / max(t_["n_solves"], 1),
                                    "steps": ncmp}
        ctx.learn_enable(True)
    ctx.close()
    torch.cuda.synchronize()
    # ------------------------------------------------------- plain FP64, reference
    ref = None
    ctx = Context(sysm, precision="f64", **opts)
    if form != "plain_f64":
        G, secs, t_ = run_steps(ctx, wcmp, "plain_f64")
        cmp_secs["plain_f64"] = sum(secs)
        cmp_G["plain_f64"] = G
        res["plain_f64"] = {"points_per_s": ncmp * ppstep / sum(secs), "steps": ncmp,
                            "iterations_per_solve": t_["n_iterations"] / max(t_["n_solves"], 1),
                            "unconverged": t_["n_unconverged"]}
    # the accuracy reference (not optional): the same plain context at a tight tolerance
    ctx.set_options(tol=args.ref_tol)
    G, secs, t_ = run_steps(ctx, wcmp, "reference")
    ref = {"G": G, "tol": args.ref_tol, "unconverged": t_["n_unconverged"], "points": int(G.size)}
    ctx.close()
    torch.cuda.synchronize()
    acc = {"target_rel_err": TARGET, "reference": "plain FP64 GPU solve at tol %g" % args.ref_tol,
           "checked_points": ref["points"] if ref else 0, "steps_checked": ncmp if ref else 0}
    if ref is not None:
        acc["reference_unconverged"] = ref["unconverged"]
        acc["max_rel_err"] = {k: pointwise_err(v, ref["G"]) for k, v in cmp_G.items()}
    meets = ref is not None and acc["max_rel_err"][form] <= TARGET and tot["n_unconverged"] == 0
    acc["meets_target"] = meets
    # the kernel's bound: its algorithmic flops at the matrix peak of its dtype against its
    # algorithmic bytes (W blocks, vector copy and output once) at the HBM peak, per launch
    by = tot["big_bytes"] / max(tot["big_launches"], 1)
    hbm_bound = by / HBM_PEAK > fl / PEAK[prec]
    kname = GEMM_NAME[prec] + " (EA 1/2 W_abcd r_i^cd over the stored blocks ka < kb)"
    if hbm_bound:
        achb = by / (avg_ms * 1e-3) if avg_ms > 0 else 0.0
        roof = {"bound": "hbm", "kernel": kname, "achieved": achb / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                "frac": achb / HBM_PEAK, "flops_achieved_tflops": ach / 1e12}
    else:
        roof = {"bound": "mfma", "kernel": kname, "achieved": ach / 1e12, "peak": PEAK[prec] / 1e12,
                "unit": "TFLOP/s", "frac": ach / PEAK[prec]}
    roof.update({"avg_ms": avg_ms, "flops_per_launch": fl, "bytes_per_launch": by, "launches": tot["big_launches"]})
    tr = stored_traffic(GEMM_NAME[prec])
    roof["traffic"] = tr["bytes_per_launch"] if tr else None
    speed = None
    if "plain_f64" in cmp_secs and form != "plain_f64":
        speed = {"headline_vs_plain_f64": cmp_secs["plain_f64"] / cmp_secs[form], "steps": ncmp,
                 "frequencies": wcmp}
        if "network_off" in cmp_secs:
            speed["headline_vs_network_off"] = cmp_secs["network_off"] / cmp_secs[form]
    out = {
        "metric": METRIC,
        "value": res[form]["points_per_s"] if meets else None,
        "unit": "G(w) points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res[form]["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: Si-like {sysm.kmesh[0]}x{sysm.kmesh[1]}x{sysm.kmesh[2]} k-mesh, "
                         f"{sysm.nocc} occ + {sysm.nvir} vir spin orbitals/cell, K=Gamma; step s: orbitals "
                         f"p = s mod 3 + 3j (10 of {nmo}) x 1 omega (grid point (37 s + 5) mod {ng} of the "
                         f"{ng}-point grid on [-1,1] Ha), IP + EA, eta={eta}, GMRES({args.restart}) tol={args.tol}, "
                         f"up to {args.batch} right-hand sides in flight, preconditioner damping "
                         f"{args.precond_eta} Ha"),
            "form": form,
            "points_per_step": ppstep,
        },
        "measured_value": res[form]["points_per_s"],
        "accuracy": acc,
        "forms": res,
        "speedup": speed,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(sysm, sigma_pp, budget)
    out["wall_s"] = time.perf_counter() - T_START
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
