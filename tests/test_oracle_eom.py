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


@pytest.mark.parametrize("no,nv,seed", [(2, 3, 15), (3, 3, 16), (2, 4, 17)])
def test_e_vectors_with_independent_lambda_match_bruteforce(no, nv, seed):
    """General Lambda (not T^dagger): the left vectors e of O1 equal the Fock-space
    brute force <Phi|(1 + Lambda) abar ...| with the same Lambda operator."""
    s = synth.make_system((1, 1, 1), no, nv, seed=seed, t1_std=0.3, t2_std=0.3, eri_std=0.3)
    l1, l2 = synth.make_lambda((1, 1, 1), no, nv, seed=seed + 1, l1_std=0.3, l2_std=0.3)
    assert np.abs(l1 - np.conj(s.t1)).max() > 0.1  # independent of T
    E = eom.EOMSystem(s, l1=l1, l2=l2)
    n = no + nv
    v = eri_blocks(E.mesh, s.eri_factor, slice(0, n), slice(0, n), slice(0, n), slice(0, n)).data[0, 0, 0]
    f = np.zeros((n, n), complex)
    f[:no, :no] = E.foo.data[0]
    f[no:, no:] = E.fvv.data[0]
    fs = fock.FockSpace(f, v, s.t1[0], s.t2[0, 0, 0], no, l1=l1[0], l2=l2[0, 0, 0])
    E0 = eom.EOMSystem(s)
    for part in ("ip", "ea"):
        for p in range(n):
            e0, e1 = fs.e_vector(part, p), E.pack(part, 0, E.e_vector(part, 0, p))
            assert np.allclose(e0, e1, atol=1e-13), (part, p)
            # b does not depend on Lambda; e does
            assert np.allclose(E.b_vector(part, 0, p), E0.b_vector(part, 0, p), atol=0)
        assert max(np.abs(E.e_vector(part, 0, p) - E0.e_vector(part, 0, p)).max() for p in range(n)) > 1e-3


def _zeroed(E, names):
    """A shallow copy of E whose listed H-bar blocks are zero."""
    import copy
    Z = copy.copy(E)
    for nm in names:
        setattr(Z, nm, getattr(E, nm).like())
    return Z


def _abs_copy(E, names):
    import copy
    A = copy.copy(E)
    for nm in names:
        t = getattr(E, nm)
        setattr(A, nm, t.like(np.abs(t.data) + 0j))
    return A


# the H-bar blocks that the reduced-precision products hold, per part
_REDUCED = {"ea": ("Wvvvv", "Wovvo", "Fvv"), "ip": ("Woooo", "Wovvo")}
_ALL = ("Foo", "Fov", "Fvv", "Woooo", "Wvvvv", "Wovvo", "Wooov", "Wovoo", "Wvovv", "Wvvvo", "Woovv")


@pytest.mark.parametrize("part", ["ip", "ea"])
def test_reduced_terms_abs_bounds_and_matches_the_terms(part):
    """reduced_terms_abs is the |operand| |r| sum of exactly the sigma terms that hold the
    reduced-precision blocks: (1) it bounds those terms (sigma minus sigma with the blocks
    zeroed) elementwise; (2) with every block and r replaced by their absolute values it
    equals them where the antisymmetriser adds nothing (the W_abcd / W_mnij term alone),
    and (3) its exchange part splits into a term and its (a, b) / (i, j) image."""
    s = synth.make_system((3, 1, 1), 2, 4, seed=21, t1_std=0.1, t2_std=0.1, eri_std=0.2)
    E = eom.EOMSystem(s)
    rng = np.random.default_rng(4)
    n1 = E.no if part == "ip" else E.nv
    for K in range(E.nk):
        nu = len(E.unique_index(part, K)[0])
        x = E.unpack(part, K, rng.normal(size=nu) + 1j * rng.normal(size=nu))
        B = E.reduced_terms_abs(part, K, x)
        assert np.all(B[:n1] == 0) and np.all(B >= 0)
        d = E.sigma(part, K, x) - _zeroed(E, _REDUCED[part]).sigma(part, K, x)
        assert np.all(np.abs(d[n1:]) <= B[n1:] * (1 + 1e-12) + 1e-15)
        # (2) the pair-pair term alone, all blocks non-negative
        A = _abs_copy(E, _ALL)
        xa = np.abs(x) + 0j
        big, exch = _REDUCED[part][0], _REDUCED[part][1:]
        Ab = _zeroed(A, exch)
        d2 = Ab.sigma(part, K, xa) - _zeroed(Ab, (big,)).sigma(part, K, xa)
        B2 = Ab.reduced_terms_abs(part, K, xa)
        assert np.allclose(d2[n1:].real, B2[n1:], rtol=1e-12, atol=1e-14) and B2[n1:].max() > 0
        # (3) the exchange terms alone: sigma gives X - P(X), the bound X + P(X)
        Ax = _zeroed(A, (big,))
        d3 = (Ax.sigma(part, K, xa) - _zeroed(Ax, exch).sigma(part, K, xa)).real
        B3 = Ax.reduced_terms_abs(part, K, xa)
        X, PX = 0.5 * (B3 + d3), 0.5 * (B3 - d3)
        spec = "iab->iba" if part == "ea" else "ija->jia"
        _, x2 = E.split(part, K, X + 0j)
        px = eom.permute(spec, x2)
        assert np.allclose(px.data.real.ravel(), PX[n1:], rtol=1e-12, atol=1e-14)
        assert np.all(X[n1:] >= -1e-14) and X[n1:].max() > 0
