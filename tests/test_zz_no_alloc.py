"""cc_gf_dyson_cas_noalloc (the Dyson step for callers that cannot allocate device
memory) against cc_gf_dyson_cas, through the C ABI: two calls in a row, the first
larger than one chunk of the fixed scratch, the second smaller; both must equal
the allocating entry point's results bit for bit (same kernels, same arithmetic
per point), and the singular case must be reported."""
import numpy as np
import pytest

from paper_2208_07478_amd import synth

pytestmark = pytest.mark.gpu


def inputs(nk, nw, N, M, seed):
    ws = np.linspace(-0.8, 0.9, nw)
    eta = 0.05

    def res(n, k, tag):
        z = synth.random_vectors(n * n, 1, seed=seed + 97 * k + tag)[0].reshape(n, n) * 0.3
        h = 0.5 * (z + z.conj().T)
        return np.array([np.linalg.inv((w + 1j * eta) * np.eye(n) - h) for w in ws])

    Ggw = np.array([res(N, k, 1) for k in range(nk)])
    Gcas = np.array([res(M, k, 2) for k in range(nk)])
    Gcc = np.array([res(M, k, 3) for k in range(nk)])
    V = np.array([synth.random_unitary(N, seed=seed, block=k)[:, :M] for k in range(nk)])
    return Ggw, Gcas, Gcc, V


def test_noalloc_matches_allocating_entry_point():
    import torch
    from paper_2208_07478_amd import ccgf
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    # 2 x 70 points of 64 x 64: more than the 113 points one chunk of the fixed scratch holds
    for (nk, nw, N, M) in ((2, 70, 64, 64), (1, 3, 30, 14)):
        args = [t(a) for a in inputs(nk, nw, N, M, seed=500 + N)]
        print("noalloc call", nk, nw, N, M, flush=True)
        G0, Sf0, S0 = ccgf.dyson_cas(*args, self_energies=True)
        G1, Sf1, S1 = ccgf.dyson_cas(*args, self_energies=True, noalloc=True)
        torch.cuda.synchronize()
        for a, b in ((G0, G1), (Sf0, Sf1), (S0, S1)):
            assert torch.equal(a, b)
        assert float(torch.abs(G1).max()) > 0
    Ggw, Gcas, Gcc, V = inputs(1, 2, 6, 3, seed=9)
    Gcc[0, 0] = 0.0
    with pytest.raises(ccgf.CCGFError, match="singular"):
        ccgf.dyson_cas(t(Ggw), t(Gcas), t(Gcc), t(V), noalloc=True)
