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


def _check_g(E, orbs, wtest, eta, runs):
    cache = {}
    for p in orbs:
        gp, gm = solve.dense_gf(E, 0, p, wtest, eta, M_cache=cache)
        sc = max(np.abs(gp).max(), np.abs(gm).max())
        for k, (G, Gp, Gm, st) in runs.items():
            assert st["n_unconverged"] == 0, k
            assert np.abs(Gp[0, p] - gp).max() <= 1e-8 * sc, k
            assert np.abs(Gm[0, p] - gm).max() <= 1e-8 * sc, k


def test_learned_guess_gain_in_a_smooth_window():
    """A case where the network should help: frequencies in the gap between the
    removal and addition spectra, where the solutions change smoothly with w.
    Trained on every other point of the window, the network's guesses for the
    points between need fewer GMRES steps than starting from zero and than
    starting from the nearest training solution; G is unchanged (dense inversion)."""
    import torch
    from paper_2208_07478_amd.ccgf import Context
    case = dict(kmesh=(2, 1, 1), nocc=2, nvir=5, seed=12)
    s = synth.make_system(t1_std=0.05, t2_std=0.05, eri_std=0.1, **case)
    print("case", case, flush=True)
    E = eom.EOMSystem(s)
    eta = 0.005
    window = np.linspace(-0.28, 0.18, 17)
    wtrain, wtest = window[0::2], window[1::2]
    orbs = list(range(s.nocc + s.nvir))
    ctx = Context(s, tol=1e-10, restart_m=60, maxiter=20000, max_batch=128, precond_eta=0.4)
    try:
        runs = {}
        ctx.learn_enable(False)
        runs["zero"] = ctx.solve([0], orbs, wtest, eta)
        ctx.learn(0, orbs, wtrain, eta, guess="nearest", accept=1.0, probe=-1)
        runs["nearest"] = ctx.solve([0], orbs, wtest, eta)
        ls = ctx.learn(0, orbs, wtrain, eta, epochs=300, seed=3, probe=-1)
        print("learn", ls, flush=True)
        assert ls["loss_final"] < ls["loss_initial"]
        runs["network"] = ctx.solve([0], orbs, wtest, eta)
        its = {k: r[3]["n_iterations"] for k, r in runs.items()}
        print("iterations", its, "guesses used", runs["network"][3]["n_guess"], flush=True)
        assert runs["network"][3]["n_guess"] > 0
        assert its["network"] < 0.9 * its["zero"]
        assert its["network"] < its["nearest"]
        _check_g(E, orbs, wtest, eta, runs)
    finally:
        ctx.close()
        torch.cuda.synchronize()


def test_learned_preconditioner_gain_and_fallback():
    """The preconditioner network (damping of the diagonal preconditioner per
    solve, learned from probe solves) on a 2x2x1 system across the whole window
    [-1, 1] Ha at eta = 5 mHa: fewer GMRES steps than the fixed damping, with G
    unchanged (the damping changes only the iteration count; the FP64 residual
    judges every solve)."""
    import torch
    from paper_2208_07478_amd.ccgf import Context
    case = dict(kmesh=(2, 2, 1), nocc=4, nvir=12, seed=5)
    s = synth.make_system(t1_std=0.01, t2_std=0.01, eri_std=0.05, **case)
    print("case", case, flush=True)
    eta = 0.005
    grid = np.linspace(-1.0, 1.0, 33)
    wtrain, wtest = grid[0::2], grid[1::2]
    orbs = list(range(s.nocc + s.nvir))
    ctx = Context(s, tol=1e-10, restart_m=60, maxiter=20000, max_batch=128, precond_eta=0.4)
    try:
        runs = {}
        runs["fixed"] = ctx.solve([0], orbs, wtest, eta)
        ls = ctx.learn(0, orbs, wtrain, eta, epochs=300, seed=3)
        print("learn", ls, flush=True)
        assert ls["precond_loss_final"] < ls["precond_loss_initial"]
        ctx.learn_enable(guess=False, precond=True)
        runs["learned"] = ctx.solve([0], orbs, wtest, eta)
        its = {k: r[3]["n_iterations"] for k, r in runs.items()}
        print("iterations", its, flush=True)
        assert its["learned"] < 0.95 * its["fixed"]
        # the damping changes the iteration count only: both runs give the same G to the tolerance
        # (the plain solver's G is pinned against dense inversion by the parity tests)
        for k in ("Gp", "Gm"):
            i = 1 if k == "Gp" else 2
            a, b = runs["learned"][i], runs["fixed"][i]
            assert np.abs(a - b).max() <= 1e-8 * np.abs(b).max(), k
        assert runs["learned"][3]["n_unconverged"] == 0
    finally:
        ctx.close()
        torch.cuda.synchronize()


def test_trained_networks_survive_save_and_load(tmp_path):
    """cc_gf_learn_save / cc_gf_learn_load: a fresh context of the same system that loads
    the file solves exactly like the context that trained (same G bit for bit, same
    iterations); another system shape and a foreign file are refused."""
    import torch
    from paper_2208_07478_amd.ccgf import CCGFError, Context
    case = dict(kmesh=(2, 1, 1), nocc=2, nvir=5, seed=12)
    s = synth.make_system(t1_std=0.05, t2_std=0.05, eri_std=0.1, **case)
    eta = 0.005
    window = np.linspace(-0.28, 0.18, 9)
    orbs = list(range(s.nocc + s.nvir))
    path = tmp_path / "nets.bin"
    opts = dict(tol=1e-10, restart_m=60, maxiter=20000, max_batch=128, precond_eta=0.4)
    a = Context(s, **opts)
    b = Context(s, **opts)
    try:
        with pytest.raises(CCGFError):
            a.learn_save(path)  # nothing trained yet
        a.learn(0, orbs, window[0::2], eta, epochs=200, seed=3, probe=20)
        a.learn_save(path)
        b.learn_load(path)
        ra = a.solve([0], orbs, window[1::2], eta)
        rb = b.solve([0], orbs, window[1::2], eta)
        print("iterations", ra[3]["n_iterations"], rb[3]["n_iterations"], "guesses", ra[3]["n_guess"], flush=True)
        assert ra[3]["n_iterations"] == rb[3]["n_iterations"] and ra[3]["n_guess"] == rb[3]["n_guess"]
        assert np.array_equal(ra[0], rb[0])
    finally:
        a.close()
        b.close()
    s2 = synth.make_system(t1_std=0.05, t2_std=0.05, eri_std=0.1, kmesh=(2, 1, 1), nocc=2, nvir=6, seed=12)
    c = Context(s2, **opts)
    try:
        with pytest.raises(CCGFError, match="another system shape"):
            c.learn_load(path)
        junk = tmp_path / "junk.bin"
        junk.write_bytes(b"not a network file")
        with pytest.raises(CCGFError):
            c.learn_load(junk)
    finally:
        c.close()
        torch.cuda.synchronize()
