"""Mixed precision on the GPU: FP32 sigma products (the Krylov steps' operator)
against the FP64 oracle, and Green's functions from the mixed solver (FP32
Arnoldi, FP64 true residual and refinement every cycle) against dense
inversion at FP64 accuracy."""
import numpy as np
import pytest

from paper_2208_07478_amd import synth
from oracle import eom, solve

pytestmark = pytest.mark.gpu

CASES = [
    dict(kmesh=(2, 1, 1), nocc=2, nvir=5, seed=12),
    dict(kmesh=(3, 1, 1), nocc=3, nvir=9, seed=13),
    dict(kmesh=(2, 2, 1), nocc=2, nvir=7, seed=14),
    # an even number of virtuals: the BF16-split products stage two k at a time
    dict(kmesh=(3, 1, 1), nocc=2, nvir=6, seed=15),
]


def _system(case):
    return synth.make_system(t1_std=0.05, t2_std=0.05, eri_std=0.1, **case)


U32, UB = 2.0 ** -24, 2.0 ** -8  # unit roundoff of FP32 and of BF16


def error_coefficient(prec, kterms):
    """A-priori bound c of |error| <= c sum_k |A_k| |B_k| for one complex product
    sum_k A_k B_k over kterms terms, to first order in the unit roundoffs.
    FP32: operands rounded to FP32 (u each), Gauss' sums Ar + Ai and Br + Bi rounded (u),
    FP32 accumulation of kterms products (kterms u); the real part P1 - P2 carries at most
    (kterms + 3) u S and the imaginary part P3 - P1 - P2 three times that, with
    S = sum |A||B| (|Ar||Br| + |Ai||Bi| <= |A||B|, (|Ar| + |Ai|)(|Br| + |Bi|) <= 2 |A||B|).
    BF16 split: x = hi + lo + d with |lo| <= UB |x| and |d| <= UB^2 |x| (plus the FP32
    rounding of x on the way, u); hi*hi + hi*lo + lo*hi drops at most 3 UB^2 |a||b| per
    real product, and FP32 accumulates 3 kterms products; real and imaginary parts each
    sum two real products bounded by S."""
    if prec == "f32":
        return 4.0 * (kterms + 3) * U32
    return 2.0 * (3.0 * UB * UB + (3.0 * kterms + 2.0) * U32)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("ci", range(len(CASES)))
@pytest.mark.parametrize("part", ["ip", "ea"])
def test_mixed_sigma_error_within_a_priori_bound(ci, part, prec):
    """Each reduced-precision product agrees with the FP64 oracle elementwise within
    c * sum |W| |r| over the terms it takes in reduced precision (the oracle's
    reduced_terms_abs; c from error_coefficient with the longest contraction, nv^2 nk
    terms), plus FP64 rounding of the rest: a wrong MFMA lane layout or a stale copy is
    O(1).  The error must also be well above FP64 rounding (the reduced path really ran)."""
    import torch
    from paper_2208_07478_amd.ccgf import Context
    s = _system(CASES[ci])
    print("case", CASES[ci], part, flush=True)
    E = eom.EOMSystem(s)
    kterms = max(s.nvir * s.nvir, s.nocc * s.nvir, s.nocc * s.nocc) * E.nk
    c = error_coefficient(prec, kterms)
    ctx = Context(s, max_batch=32, precision=prec)
    try:
        for K in range(E.nk):
            X = synth.random_eom_vectors(s.kmesh, s.nocc, s.nvir, part, K, 19, seed=300 + K)
            ref = np.array([E.sigma(part, K, x) for x in X])
            bnd = np.array([E.reduced_terms_abs(part, K, x) for x in X])
            Y = ctx.sigma(part, K, torch.from_numpy(X).cuda()).cpu().numpy()
            err = np.abs(Y - ref)
            slack = 1e-12 * np.abs(ref).max(axis=1, keepdims=True)
            ratio = (err / (c * bnd + slack)).max()
            rel = (np.linalg.norm(Y - ref, axis=1) / np.linalg.norm(ref, axis=1)).max()
            print(part, K, "c", c, "max err / bound", ratio, "max rel err", rel, flush=True)
            assert ratio <= 1.0
            assert rel > 1e-9  # really reduced precision, not the FP64 path
    finally:
        ctx.close()
        torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("ci", range(len(CASES)))
def test_mixed_solver_reaches_fp64_accuracy(ci, prec):
    """FP32 Krylov steps with FP64 refinement reach tol 1e-10 on the FP64
    operator: G+ and G- match dense inversion like the plain FP64 solver."""
    import torch
    from paper_2208_07478_amd.ccgf import Context
    s = _system(CASES[ci])
    print("case", CASES[ci], prec, flush=True)
    E = eom.EOMSystem(s)
    ctx = Context(s, max_batch=32, maxiter=12000, restart_m=60, tol=1e-10, precision=prec)
    try:
        w = np.linspace(-1.0, 1.0, 5)
        eta = 0.02
        nmo = s.nocc + s.nvir
        ks = list(range(E.nk))
        G, Gp, Gm, st = ctx.solve(ks, list(range(nmo)), w, eta)
        assert st["n_unconverged"] == 0
        assert st["max_rel_residual"] <= 1e-10
        cache = {}
        for a, K in enumerate(ks):
            for p in range(nmo):
                gp, gm = solve.dense_gf(E, K, p, w, eta, M_cache=cache)
                scale = max(np.abs(gm).max(), np.abs(gp).max(), 1.0)
                assert np.abs(Gm[a, p] - gm).max() <= 1e-8 * scale
                assert np.abs(Gp[a, p] - gp).max() <= 1e-8 * scale
    finally:
        ctx.close()
        torch.cuda.synchronize()


def _peaks(w, A):
    """Local maxima of A above 5% of its maximum, refined by a 3-point parabola."""
    out = []
    thr = 0.05 * A.max()
    for i in range(1, len(w) - 1):
        if A[i] > A[i - 1] and A[i] >= A[i + 1] and A[i] > thr:
            den = A[i - 1] - 2 * A[i] + A[i + 1]
            off = 0.5 * (A[i - 1] - A[i + 1]) / den if den != 0 else 0.0
            out.append(w[i] + off * (w[1] - w[0]))
    return np.array(out)


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_mixed_forms_keep_spectral_peaks_within_1meV(prec):
    """A(w) = -(1/pi)[Im G+ - Im G-] on a fine grid: the mixed forms reproduce
    plain FP64's peaks (count and positions to 1 meV) and G to 1e-6 relative,
    at the bench's GMRES tolerance."""
    import torch
    from paper_2208_07478_amd.ccgf import Context
    s = _system(CASES[0])
    w = np.linspace(-1.2, 2.0, 321)
    eta = 0.01
    nmo = s.nocc + s.nvir
    ks = list(range(int(np.prod(s.kmesh))))
    res = {}
    for p in ("f64", prec):
        ctx = Context(s, max_batch=64, maxiter=12000, restart_m=60, tol=2e-7, precision=p)
        try:
            res[p] = ctx.solve(ks, list(range(nmo)), w, eta)
        finally:
            ctx.close()
            torch.cuda.synchronize()
    G0, Gp0, Gm0, _ = res["f64"]
    G1, Gp1, Gm1, _ = res[prec]
    mev = 1e-3 / 27.211386
    for a in range(len(ks)):
        for p in range(nmo):
            A0 = -(Gp0[a, p].imag - Gm0[a, p].imag) / np.pi
            A1 = -(Gp1[a, p].imag - Gm1[a, p].imag) / np.pi
            assert np.abs(G1[a, p] - G0[a, p]).max() <= 1e-6 * np.abs(G0[a, p]).max()
            p0, p1 = _peaks(w, A0), _peaks(w, A1)
            assert len(p0) == len(p1) and len(p0) > 0, (a, p)
            assert np.abs(p0 - p1).max() <= mev, (a, p, np.abs(p0 - p1).max())


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
@pytest.mark.parametrize("part", ["ip", "ea"])
def test_reduced_sigma_every_tile_width_matches_oracle(part, prec):
    """The first reduced-precision products of a new shape are the autotuner's trials
    (64-, 32- and, in FP32, 128-wide N tiles), the next ones its choice, then a captured
    graph: each of them is checked against the a-priori bound, on a batch whose N spans
    several 128-wide tiles with a ragged tail."""
    import torch
    from paper_2208_07478_amd.ccgf import Context
    case = dict(kmesh=(2, 1, 1), nocc=3, nvir=9, seed=17)
    s = _system(case)
    E = eom.EOMSystem(s)
    c = error_coefficient(prec, s.nvir * s.nvir * E.nk)
    ctx = Context(s, max_batch=64, precision=prec)
    try:
        X = synth.random_eom_vectors(s.kmesh, s.nocc, s.nvir, part, 1, 53, seed=77)
        ref = np.array([E.sigma(part, 1, x) for x in X])
        bnd = np.array([E.reduced_terms_abs(part, 1, x) for x in X])
        slack = 1e-12 * np.abs(ref).max(axis=1, keepdims=True)
        Xd = torch.from_numpy(X).cuda()
        for call in range(6):
            Y = ctx.sigma(part, 1, Xd).cpu().numpy()
            ratio = (np.abs(Y - ref) / (c * bnd + slack)).max()
            print(part, prec, "call", call, "max err / bound", ratio, flush=True)
            assert ratio <= 1.0
    finally:
        ctx.close()
        torch.cuda.synchronize()
