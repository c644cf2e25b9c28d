"""Model-order reduction on the GPU (cc_gf_mor) against the oracle's reduced
model: same expansion frequencies, same Galerkin model, same grid."""
import numpy as np
import pytest

from paper_2208_07478_amd import synth
from oracle import eom, mor, solve

pytestmark = pytest.mark.gpu


def _system(case):
    return synth.make_system(t1_std=0.05, t2_std=0.05, eri_std=0.1, **case)


def test_mor_matches_oracle_reduced_model():
    """Six expansion points per part (IP on [-1.5, 0], EA on [0, 1.5]) and a
    41-point grid: G+ and G- from the reduced model agree with the oracle's
    model built from exact solutions, and reproduce the full solves at the
    expansion points."""
    import torch
    from paper_2208_07478_amd.ccgf import Context
    case = dict(kmesh=(2, 1, 1), nocc=2, nvir=5, seed=12)
    s = _system(case)
    print("case", case, flush=True)
    E = eom.EOMSystem(s)
    ctx = Context(s, max_batch=32, maxiter=4000, tol=1e-12)
    try:
        eta = 0.05
        w_ip = np.linspace(-1.5, 0.0, 6)
        w_ea = np.linspace(0.0, 1.5, 6)
        grid = np.linspace(-1.5, 1.5, 41)
        nmo = s.nocc + s.nvir
        orbs = list(range(nmo))
        ks = list(range(E.nk))
        G, Gp, Gm, st = ctx.mor(ks, orbs, w_ip, w_ea, grid, eta)
        assert st["n_unconverged"] == 0
        assert st["n_solves"] == len(ks) * nmo * (len(w_ip) + len(w_ea))
        _, Gpe, _, _ = ctx.solve(ks, orbs, w_ea, eta, parts="ea")
        _, _, Gme, _ = ctx.solve(ks, orbs, w_ip, eta, parts="ip")
        for a, K in enumerate(ks):
            for p in orbs:
                ref_m = mor.mor_gf(E, "ip", K, p, w_ip, grid, eta)
                ref_p = mor.mor_gf(E, "ea", K, p, w_ea, grid, eta)
                scale = max(np.abs(ref_m).max(), np.abs(ref_p).max(), 1e-300)
                err = max(np.abs(Gm[a, p] - ref_m).max(), np.abs(Gp[a, p] - ref_p).max()) / scale
                print(K, p, "mor rel err", err, flush=True)
                assert err <= 1e-7, (K, p)
                np.testing.assert_allclose(G[a, p], Gm[a, p] + Gp[a, p], rtol=0, atol=1e-14 * scale)
                # Galerkin: exact at the expansion points up to the solve tolerance
                gi = np.array([np.argmin(np.abs(grid - x)) for x in w_ip])
                ge = np.array([np.argmin(np.abs(grid - x)) for x in w_ea])
                assert np.allclose(grid[gi], w_ip) and np.allclose(grid[ge], w_ea)
                assert np.abs(Gm[a, p, gi] - Gme[a, p]).max() <= 1e-8 * scale
                assert np.abs(Gp[a, p, ge] - Gpe[a, p]).max() <= 1e-8 * scale
    finally:
        ctx.close()
        torch.cuda.synchronize()


def test_mor_with_spanning_basis_equals_full_gf():
    """More expansion points than the space has dimensions: the dependent
    solutions are dropped, the basis spans everything and the reduced model
    is the full G at every frequency (dense inversion), up to the directions
    whose share of the solutions falls under the 1e-10 drop threshold."""
    import torch
    from paper_2208_07478_amd.ccgf import Context
    case = dict(kmesh=(1, 1, 1), nocc=2, nvir=3, seed=31, real=True, naux=8)
    s = _system(case)
    print("case", case, flush=True)
    E = eom.EOMSystem(s)
    assert len(E.unique_index("ip", 0)[0]) < 12 and len(E.unique_index("ea", 0)[0]) < 12
    ctx = Context(s, max_batch=32, maxiter=4000, tol=1e-13)
    try:
        eta = 0.1
        wexp = np.linspace(-2.0, 2.0, 12)
        grid = np.linspace(-3.0, 3.0, 25)
        nmo = s.nocc + s.nvir
        G, Gp, Gm, st = ctx.mor([0], list(range(nmo)), wexp, wexp, grid, eta)
        for p in range(nmo):
            gp, gm = solve.dense_gf(E, 0, p, grid, eta)
            scale = max(np.abs(gp).max(), np.abs(gm).max(), 1e-300)
            err = max(np.abs(Gp[0, p] - gp).max(), np.abs(Gm[0, p] - gm).max()) / scale
            print(p, "rel err vs full", err, flush=True)
            assert err <= 1e-8
    finally:
        ctx.close()
        torch.cuda.synchronize()


def test_mor_rejects_bad_expansion_sets():
    import torch
    from paper_2208_07478_amd import ccgf
    from paper_2208_07478_amd.ccgf import Context
    s = _system(dict(kmesh=(1, 1, 1), nocc=2, nvir=3, seed=31, real=True, naux=8))
    ctx = Context(s)
    try:
        with pytest.raises(ccgf.CCGFError) as ei:
            ctx.mor([0], [0], [], [0.1], [0.0], 0.1)
        assert ei.value.code == ccgf.EINVAL
        with pytest.raises(ccgf.CCGFError):
            ctx.mor([0], [0], np.linspace(-1, 0, ccgf.MOR_MAX + 1), [0.1], [0.0], 0.1)
        G, Gp, Gm, st = ctx.mor([0], [0], None, [0.1, 0.5], [0.0, 0.3], 0.1, parts="ea")
        assert np.all(Gm == 0) and np.all(G == Gp)
    finally:
        ctx.close()
        torch.cuda.synchronize()
