"""Grouped sigma products over uneven systems (different k-meshes, orbital counts,
parts, momenta and batch widths) in one launch per GEMM term, through the C ABI:
each system's product against the oracle's (FP64) and against that context's own
cc_gf_sigma (FP64 and FP32: the same arithmetic per element, so equal bit for bit)."""
import numpy as np
import pytest

from paper_2208_07478_amd import synth
from oracle import eom

pytestmark = pytest.mark.gpu

SYSTEMS = [  # (case, part, K, nvec)
    (dict(kmesh=(1, 1, 1), nocc=2, nvir=6, real=True, naux=16, seed=71), "ea", 0, 7),
    (dict(kmesh=(2, 1, 1), nocc=2, nvir=5, seed=72), "ip", 1, 3),
    (dict(kmesh=(3, 1, 1), nocc=3, nvir=4, seed=73), "ea", 2, 5),
    (dict(kmesh=(2, 2, 1), nocc=2, nvir=3, seed=74), "ip", 3, 11),
    (dict(kmesh=(1, 2, 2), nocc=1, nvir=4, seed=75), "ea", 1, 2),
    (dict(kmesh=(3, 1, 1), nocc=2, nvir=7, seed=76), "ip", 0, 17),
]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_grouped_sigma_matches_each_system(prec):
    import torch
    from paper_2208_07478_amd import ccgf
    from paper_2208_07478_amd.ccgf import Context
    items, refs, ctxs = [], [], []
    try:
        for case, part, K, nvec in SYSTEMS:
            s = synth.make_system(t1_std=0.05, t2_std=0.05, eri_std=0.1, **case)
            c = Context(s, precision=prec, max_batch=32)
            ctxs.append(c)
            X = synth.random_eom_vectors(s.kmesh, s.nocc, s.nvir, part, K, nvec, seed=case["seed"])
            items.append((c, part, K, torch.from_numpy(X).cuda()))
            refs.append((s, X))
        print("grouped", prec, [(c["kmesh"], c["nocc"], c["nvir"], p, K, nv) for c, p, K, nv in SYSTEMS], flush=True)
        Y = [y.cpu().numpy() for y in ccgf.sigma_group(items)]
        for (c, part, K, Xd), y, (s, X) in zip(items, Y, refs):
            own = c.sigma(part, K, Xd).cpu().numpy()
            assert np.array_equal(y, own), (s.kmesh, part)
            if prec == "f64":
                E = eom.EOMSystem(s)
                ref = np.array([E.sigma(part, K, x) for x in X])
                err = np.abs(y - ref).max() / np.abs(ref).max()
                print(s.kmesh, part, K, "rel err vs oracle", err, flush=True)
                assert err <= 1e-12
        # a second grouped call with other batch widths reuses the tables
        items2 = [(c, p, K, x[: max(1, x.shape[0] // 2)].contiguous()) for (c, p, K, x) in items]
        Y2 = [y.cpu().numpy() for y in ccgf.sigma_group(items2)]
        for (c, p, K, x), y in zip(items2, Y2):
            assert np.array_equal(y, c.sigma(p, K, x).cpu().numpy())
    finally:
        for c in ctxs:
            c.close()
        torch.cuda.synchronize()


def test_grouped_sigma_rejects_mixed_precision_and_repeats():
    import torch
    from paper_2208_07478_amd import ccgf
    from paper_2208_07478_amd.ccgf import Context
    s = synth.make_system((2, 1, 1), 2, 3, seed=77)
    X = torch.from_numpy(synth.random_eom_vectors(s.kmesh, 2, 3, "ea", 0, 2, seed=1)).cuda()
    with Context(s) as a, Context(s, precision="f32") as b:
        with pytest.raises(ccgf.CCGFError, match="precision"):
            ccgf.sigma_group([(a, "ea", 0, X), (b, "ea", 0, X)])
        with pytest.raises(ccgf.CCGFError, match="twice"):
            ccgf.sigma_group([(a, "ea", 0, X), (a, "ea", 0, X)])
    torch.cuda.synchronize()
