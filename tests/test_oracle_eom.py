"""P1: the einsum EOM-CCSD (O1) equals the Fock-space brute force (O0) for M,
b and e on random complex data; P9: antisymmetry and linearity of sigma."""
import numpy as np
import pytest

from paper_2208_07478_amd import synth
from oracle import eom, fock
from oracle.eom import eri_blocks


def mol_pair(no, nv, seed, zero_t1=False, zero_t2=False):
    s = synth.make_system((1, 1, 1), no, nv, seed=seed, t1_std=0.3, t2_std=0.3, eri_std=0.3,
                          zero_t1=zero_t1, zero_t2=zero_t2)
    E = eom.EOMSystem(s)
    n = no + nv
    v = eri_blocks(E.mesh, s.eri_factor, slice(0, n), slice(0, n), slice(0, n), slice(0, n)).data[0, 0, 0]
    f = np.zeros((n, n), complex)
    f[:no, :no] = E.foo.data[0]
    f[no:, no:] = E.fvv.data[0]
    return E, fock.FockSpace(f, v, s.t1[0], s.t2[0, 0, 0], no)


@pytest.mark.parametrize("no,nv,seed,z1,z2", [
    (2, 3, 5, False, False), (2, 3, 6, True, False), (2, 3, 7, False, True),
    (3, 3, 11, False, False), (2, 5, 12, False, False), (4, 2, 13, False, False),
])
def test_sigma_b_e_match_bruteforce(no, nv, seed, z1, z2):
    E, fs = mol_pair(no, nv, seed, z1, z2)
    for part in ("ip", "ea"):
        M0 = fs.eom_matrix(part)
        M1 = E.dense_matrix(part, 0)
        scale = np.abs(M0).max()
        assert np.abs(M0 - M1).max() <= 1e-12 * scale, part
        for p in range(no + nv):
            b0, b1 = fs.b_vector(part, p), E.pack(part, 0, E.b_vector(part, 0, p))
            e0, e1 = fs.e_vector(part, p), E.pack(part, 0, E.e_vector(part, 0, p))
            assert np.allclose(b0, b1, atol=1e-13), (part, p)
            assert np.allclose(e0, e1, atol=1e-13), (part, p)


def test_sigma_antisymmetric_and_linear():
    s = synth.make_system((2, 1, 1), 2, 3, seed=3, t1_std=0.1, t2_std=0.1, eri_std=0.2)
    E = eom.EOMSystem(s)
    rng = np.random.default_rng(0)
    for part in ("ip", "ea"):
        for K in range(2):
            n = E.size(part)
            u1 = E.unpack(part, K, rng.normal(size=len(E.unique_index(part, K)[0])) + 0j)
            u2 = E.unpack(part, K, rng.normal(size=len(E.unique_index(part, K)[0])) * 1j)
            s1 = E.sigma(part, K, u1)
            s2 = E.sigma(part, K, u2)
            s12 = E.sigma(part, K, 2.0 * u1 - 0.5j * u2)
            assert np.allclose(s12, 2.0 * s1 - 0.5j * s2, atol=1e-12)
            # the output is antisymmetric: unpack(pack(s)) reproduces it
            assert np.allclose(E.unpack(part, K, E.pack(part, K, s1)), s1, atol=1e-13)
