"""O2b (per-block H-bar and sigma for large meshes) against O1/O2 (oracle.eom,
pinned by the Fock-space brute force) on several small meshes: every H-bar
block and every sigma block, IP and EA, several total momenta K."""
import itertools

import numpy as np
import pytest

from paper_2208_07478_amd import synth
from oracle import blocks, eom


@pytest.mark.parametrize("kmesh,no,nv,seed", [((3, 1, 1), 2, 3, 41), ((2, 2, 1), 2, 3, 42), ((1, 1, 1), 3, 4, 43)])
def test_hbar_blocks_match_dense_classes(kmesh, no, nv, seed):
    s = synth.make_system(kmesh, no, nv, seed=seed, t1_std=0.2, t2_std=0.2, eri_std=0.2)
    E = eom.EOMSystem(s)
    B = blocks.BlockSystem(s)
    nk = E.nk
    Fov, Foo, Fvv = B.fock()
    assert np.allclose(Fov, E.Fov.data, atol=1e-13)
    assert np.allclose(Foo, E.Foo.data, atol=1e-13)
    assert np.allclose(Fvv, E.Fvv.data, atol=1e-13)
    for k1, k2, k3 in itertools.product(range(nk), repeat=3):
        for name in ("Wvvvv", "Wovvo", "Wvovv", "Wvvvo", "Woooo", "Wooov", "Wovoo"):
            got = getattr(B, name)(k1, k2, k3)
            ref = getattr(E, name).data[k1, k2, k3]
            assert np.allclose(got, ref, atol=1e-13), (name, k1, k2, k3)


@pytest.mark.parametrize("kmesh,no,nv,seed", [((3, 1, 1), 2, 3, 44), ((2, 2, 1), 2, 2, 45), ((1, 2, 3), 1, 2, 46)])
def test_sigma_blocks_match_dense_sigma(kmesh, no, nv, seed):
    s = synth.make_system(kmesh, no, nv, seed=seed, t1_std=0.2, t2_std=0.2, eri_std=0.2)
    E = eom.EOMSystem(s)
    B = blocks.BlockSystem(s)
    nk = E.nk
    for part in ("ea", "ip"):
        for K in range(nk):
            x = synth.random_eom_vectors(kmesh, no, nv, part, K, 1, seed=seed)[0]
            ref = E.sigma(part, K, x)
            n1 = nv if part == "ea" else no
            for k1, k2 in itertools.product(range(nk), repeat=2):
                r1, blk = B.sigma_block(part, K, x, k1, k2)
                off, ln = blocks.block_offset((kmesh, no, nv), part, k1, k2)
                assert np.allclose(r1, ref[:n1], atol=1e-12), (part, K)
                assert np.allclose(blk.ravel(), ref[off:off + ln], atol=1e-12), (part, K, k1, k2)
