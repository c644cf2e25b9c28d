"""Dense ERI blocks as the integral input (the alternative to the factor for small
systems): the H-bar built from them gives the oracle's sigma products and the same G
as the context built from the factor they come from."""
import numpy as np
import pytest

from oracle import eom
from paper_2208_07478_amd import synth

from test_abi_cpu import dense_eri

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", [dict(kmesh=(2, 1, 1), nocc=2, nvir=5, seed=31),
                                  dict(kmesh=(3, 1, 1), nocc=2, nvir=4, seed=32)])
def test_sigma_and_g_from_eri_blocks(case):
    import torch
    from paper_2208_07478_amd.ccgf import Context
    s = synth.make_system(t1_std=0.05, t2_std=0.05, eri_std=0.1, **case)
    print("case", case, flush=True)
    E = eom.EOMSystem(s)
    D = dense_eri(s)
    cf = Context(s, tol=1e-12, restart_m=60, maxiter=4000, max_batch=32)
    cb = Context(s, tol=1e-12, restart_m=60, maxiter=4000, max_batch=32, eri_blocks=D)
    try:
        for part in ("ip", "ea"):
            for K in range(E.nk):
                X = synth.random_eom_vectors(s.kmesh, s.nocc, s.nvir, part, K, 7, seed=40 + K)
                ref = np.array([E.sigma(part, K, x) for x in X])
                Xd = torch.from_numpy(X).cuda()
                Yb = cb.sigma(part, K, Xd).cpu().numpy()
                Yf = cf.sigma(part, K, Xd).cpu().numpy()
                sc = np.abs(ref).max()
                print(part, K, "blocks vs oracle", np.abs(Yb - ref).max() / sc, "vs factor",
                      np.abs(Yb - Yf).max() / sc, flush=True)
                assert np.abs(Yb - ref).max() <= 1e-12 * sc
                assert np.abs(Yb - Yf).max() <= 1e-12 * sc
        w = np.linspace(-0.6, 0.6, 5)
        orbs = list(range(s.nocc + s.nvir))
        Gb = cb.solve([0, 1], orbs, w, 0.01)[0]
        Gf = cf.solve([0, 1], orbs, w, 0.01)[0]
        print("G max diff", np.abs(Gb - Gf).max() / np.abs(Gf).max(), flush=True)
        assert np.abs(Gb - Gf).max() <= 1e-9 * np.abs(Gf).max()
    finally:
        cf.close()
        cb.close()
        torch.cuda.synchronize()
