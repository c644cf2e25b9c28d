"""The learned initial guess on the GPU: the training kernels' loss and
gradients against the float64 oracle, and what the trained network changes in
the solves (same G to the solver tolerance, fewer iterations)."""
import numpy as np
import pytest

from oracle import eom, mlp, solve
from paper_2208_07478_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("din,h,dout,N", [(10, 256, 6, 50), (36, 256, 32, 333), (3, 17, 2, 5)])
def test_network_gradient_matches_oracle(din, h, dout, N):
    """FP32 forward/backward on MFMA against float64 back-propagation on the
    same (FP32-representable) parameters and data."""
    from paper_2208_07478_amd.ccgf import mlp_grad
    rng = np.random.default_rng(din * 1000 + N)
    theta = mlp.init(din, h, dout, rng) + 0.05 * rng.standard_normal(mlp.n_params(din, h, dout))
    theta = theta.astype(np.float32).astype(np.float64)
    X = rng.standard_normal((N, din)).astype(np.float32).astype(np.float64)
    T = rng.standard_normal((N, dout)).astype(np.float32).astype(np.float64)
    print("case", din, h, dout, N, flush=True)
    L_ref, g_ref = mlp.grad(theta, X, T, din, h, dout)
    L, g = mlp_grad(din, h, dout, theta, X, T)
    print("loss", L, L_ref, "max grad err", np.abs(g - g_ref).max(), "max grad", np.abs(g_ref).max(), flush=True)
    assert abs(L - L_ref) <= 1e-5 * abs(L_ref)
    assert np.abs(g - g_ref).max() <= 1e-4 * np.abs(g_ref).max()
    for k, (a, b) in enumerate(zip(mlp.unpack(g, din, h, dout), mlp.unpack(g_ref, din, h, dout))):
        assert np.abs(a - b).max() <= 1e-4 * max(np.abs(b).max(), 1e-12), k


def test_learned_guess_keeps_g_and_reports_its_gain():
    """Train on every other frequency of a grid, solve the rest from zero, from
    the nearest training solution and from the network's guess: G agrees with
    dense inversion every time, and the iteration counts are reported."""
    import torch
    from paper_2208_07478_amd.ccgf import Context
    case = dict(kmesh=(2, 1, 1), nocc=2, nvir=5, seed=12)
    s = synth.make_system(t1_std=0.05, t2_std=0.05, eri_std=0.1, **case)
    print("case", case, flush=True)
    E = eom.EOMSystem(s)
    eta = 0.02
    grid = np.linspace(-1.0, 1.0, 25)
    wtrain, wtest = grid[0::2], grid[1::2]
    nmo = s.nocc + s.nvir
    orbs = list(range(nmo))
    ctx = Context(s, tol=1e-10, restart_m=40, maxiter=6000, max_batch=64)
    try:
        runs = {}
        ctx.learn_enable(False)
        runs["zero"] = ctx.solve([0], orbs, wtest, eta)
        ctx.learn_enable(True)
        ctx.learn(0, orbs, wtrain, eta, guess="nearest", accept=1.0)
        runs["nearest"] = ctx.solve([0], orbs, wtest, eta)
        ls = ctx.learn(0, orbs, wtrain, eta, epochs=300, seed=3, accept=1.0)
        print("learn", ls, flush=True)
        assert ls["loss_final"] < ls["loss_initial"]
        runs["network"] = ctx.solve([0], orbs, wtest, eta)
        ctx.learn(0, orbs, wtrain, eta, epochs=300, seed=3)  # default acceptance 0.1
        runs["network_accept0.1"] = ctx.solve([0], orbs, wtest, eta)
        for k, (G, Gp, Gm, st) in runs.items():
            print(k, "iterations", st["n_iterations"], "guesses", st["n_guess"], "rejected", st["n_guess_rejected"],
                  flush=True)
            assert st["n_unconverged"] == 0
        assert runs["zero"][3]["n_guess"] == 0 and runs["network"][3]["n_guess"] > 0
        # with the default acceptance the guesses do not cost iterations overall
        assert runs["network_accept0.1"][3]["n_iterations"] <= 1.05 * runs["zero"][3]["n_iterations"]
        cache = {}
        for p in orbs:
            gp, gm = solve.dense_gf(E, 0, p, wtest, eta, M_cache=cache)
            sc = max(np.abs(gp).max(), np.abs(gm).max())
            for k, (G, Gp, Gm, st) in runs.items():
                assert np.abs(Gp[0, p] - gp).max() <= 1e-8 * sc, k
                assert np.abs(Gm[0, p] - gm).max() <= 1e-8 * sc, k
    finally:
        ctx.close()
        torch.cuda.synchronize()
