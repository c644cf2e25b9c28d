"""Parity of the sigma products on the Si-like 3x3x3 workload (4 + 26 spin
orbitals per cell, 27 k-points): a 120-vector batch at K = Gamma and at
K = (1,1,1), IP and EA, through the C ABI, against the whole 1h / 1p part and
three whole output blocks of the 2h1p / 2p1h part per (K, part) (a block paired
with itself, one below and one above the diagonal of the momentum pair), as
formed by the per-block CPU oracle in tests/golden/make_golden_k333.py."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "si_k333_sigma_samples.npz")


def load_gen():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden_k333", os.path.join(HERE, "golden",
                                                                                   "make_golden_k333.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


@pytest.fixture(scope="module")
def setup():
    import torch
    from paper_2208_07478_amd import synth
    from paper_2208_07478_amd.ccgf import Context
    gen = load_gen()
    gold = np.load(GOLD)
    s = synth.preset_system(gen.PRESET)
    ctx = Context(s, max_batch=gen.NVEC)
    yield s, gen, gold, ctx
    ctx.close()
    torch.cuda.synchronize()


@pytest.mark.parametrize("K,part", [(0, "ea"), (13, "ea"), (0, "ip"), (13, "ip")])
def test_sigma_blocks_k333(setup, K, part):
    import torch
    from paper_2208_07478_amd import synth
    from oracle import blocks
    s, gen, gold, ctx = setup
    X = synth.random_eom_vectors(s.kmesh, s.nocc, s.nvir, part, K, gen.NVEC, seed=gen.vec_seed(part, K))
    print(f"sigma {part} K={K}: {X.shape[0]} vectors of {X.shape[1]}", flush=True)
    Y = ctx.sigma(part, K, torch.from_numpy(X).cuda()).cpu().numpy()
    del X
    n1 = s.nvir if part == "ea" else s.nocc
    worst = 0.0
    for v in gen.VEC_IDS:
        ref = gold[f"{part}_K{K}_v{v}_r1"]
        scale = np.abs(ref).max()
        err = np.abs(Y[v, :n1] - ref).max() / scale
        worst = max(worst, err)
        assert err <= 1e-12, (part, K, v, "r1", err)
        for (k1, k2) in gen.BLOCKS[(K, part)]:
            ref = gold[f"{part}_K{K}_v{v}_b{k1}_{k2}"].ravel()
            off, ln = blocks.block_offset((s.kmesh, s.nocc, s.nvir), part, k1, k2)
            err = np.abs(Y[v, off:off + ln] - ref).max() / np.abs(ref).max()
            worst = max(worst, err)
            assert err <= 1e-12, (part, K, v, (k1, k2), err)
    print(f"{part} K={K}: worst relative error {worst:.2e}", flush=True)
