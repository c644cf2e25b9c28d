"""Pins the k-conserving einsum against dense Bloch-basis einsum with explicit
zero blocks (momentum bookkeeping of Eq. 9)."""
import numpy as np
import pytest

from oracle.ktensor import KMesh, KT, keinsum, permute, to_dense, from_dense

P4 = (1, 1, -1, -1)
P2 = (1, -1)


def rand_kt(mesh, osh, signs, const=0, seed=0):
    rng = np.random.default_rng(seed)
    nk = mesh.nk
    shape = [nk] * (len(osh) - 1) + list(osh)
    data = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    return KT(mesh, data, signs, const)


def dense_vec(x: KT):
    """Dense form of a vector-like KT with a nonzero constant (law sum s k = c)."""
    return to_dense(x)


@pytest.mark.parametrize("km", [(3, 1, 1), (2, 2, 1), (1, 2, 3)])
def test_contractions_match_dense(km):
    mesh = KMesh(km)
    a = rand_kt(mesh, (2, 3, 2, 3), (1, -1, 1, -1), seed=1)   # (i, a, j, b)-like
    b = rand_kt(mesh, (2, 2, 3, 3), P4, seed=2)
    c = keinsum("iajb,ijcd->abcd", a, b, out_signs=P4)
    Da, Db = to_dense(a), to_dense(b)
    Dc = np.einsum("iajb,ijcd->abcd", Da, Db)
    assert np.allclose(to_dense(c), Dc, atol=1e-12)
    # k-diagonal two-index times four-index
    f = rand_kt(mesh, (3, 3), P2, seed=3)
    d = keinsum("ce,ijed->ijcd", f, b, out_signs=P4)
    assert np.allclose(to_dense(d), np.einsum("ce,ijed->ijcd", to_dense(f), Db), atol=1e-12)
    # permutation moving the implied index
    p = permute("ijcd->ijdc", b)
    assert np.allclose(to_dense(p), Db.transpose(0, 1, 3, 2), atol=0)


@pytest.mark.parametrize("km", [(3, 1, 1), (2, 2, 1)])
def test_vector_law_with_constant(km):
    mesh = KMesh(km)
    nk = mesh.nk
    K = nk - 1
    w = rand_kt(mesh, (2, 3, 3, 2), (-1, 1, 1, -1), seed=4)
    r = rand_kt(mesh, (2, 3, 3), (-1, 1, 1), const=K, seed=5)  # EA-like r_i^ab
    s = keinsum("kcdi,kcd->i", w.like(w.data), r, out_signs=(1,), out_const=K)
    # dense: only the momentum-K component of the result may be nonzero
    Dw = to_dense(w)
    Dr = np.zeros((nk * 2, nk * 3, nk * 3), complex)
    for ki in range(nk):
        for ka in range(nk):
            kb = r.implied((ki, ka))
            Dr[ki*2:(ki+1)*2, ka*3:(ka+1)*3, kb*3:(kb+1)*3] = r.data[ki, ka]
    Ds = np.einsum("kcdi,kcd->i", Dw, Dr)
    ref = np.zeros(nk * 2, complex)
    ref[K*2:(K+1)*2] = s.data
    assert np.allclose(Ds, ref, atol=1e-12)


def test_roundtrip_dense():
    mesh = KMesh((2, 2, 1))
    a = rand_kt(mesh, (2, 2, 3, 3), P4, seed=9)
    b = from_dense(mesh, to_dense(a), (2, 2, 3, 3), P4)
    assert np.array_equal(a.data, b.data)
