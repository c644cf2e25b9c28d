"""P7: k-point G (O2) equals the Gamma-point supercell G (O1 on unfolded data),
and the momentum-off-diagonal blocks of U^dagger G^sc U vanish.  A 3-point mesh
is included because at Nk = 2 every k equals -k, which would hide sign errors
in the momentum arithmetic."""
import numpy as np
import pytest

from paper_2208_07478_amd import synth
from oracle import eom, solve, unfold
from oracle.ktensor import KMesh


@pytest.mark.parametrize("km,no,nv", [((2, 1, 1), 2, 3), ((3, 1, 1), 2, 2)])
def test_kpoint_equals_supercell(km, no, nv):
    s = synth.make_system(km, no, nv, seed=7, t1_std=0.1, t2_std=0.1, eri_std=0.2)
    E = eom.EOMSystem(s)
    sc, VL, foo, fvv, U = unfold.unfold(s)
    Esc = eom.EOMSystem(sc, foo=foo[None], fvv=fvv[None], v_full=VL)
    om = np.array([-0.7, 0.1, 0.9])
    eta = 0.05
    Gsc = solve.dense_gf_matrix(Esc, 0, om, eta)
    GB = np.einsum("kP,wPQ,Ql->wkl", U.conj().T, Gsc, U)
    mesh = KMesh(km)
    nmo = no + nv
    scale = np.abs(GB).max()
    for K in range(mesh.nk):
        for p in range(nmo):
            gp, gm = solve.dense_gf(E, K, p, om, eta)
            i = unfold.bloch_index(mesh, no, nv, K, p)
            assert np.abs(gp + gm - GB[:, i, i]).max() <= 1e-12 * scale
    for k1 in range(mesh.nk):
        for k2 in range(mesh.nk):
            if k1 != k2:
                i1 = [unfold.bloch_index(mesh, no, nv, k1, p) for p in range(nmo)]
                i2 = [unfold.bloch_index(mesh, no, nv, k2, p) for p in range(nmo)]
                assert np.abs(GB[:, i1][:, :, i2]).max() <= 1e-12 * scale


@pytest.mark.parametrize("km,no,nv", [((2, 1, 1), 2, 2), ((3, 1, 1), 1, 2)])
def test_kpoint_equals_supercell_with_exact_lambda(km, no, nv):
    """The supporting information's validation with a Lambda that is not T^dagger:
    k-point G with given Lambda amplitudes equals the supercell G with the same
    Lambda unfolded (Lambda transforms like T^dagger: unfold conj(l) as t, conjugate)."""
    s = synth.make_system(km, no, nv, seed=9, t1_std=0.1, t2_std=0.1, eri_std=0.2)
    l1, l2 = synth.make_lambda(km, no, nv, seed=10, l1_std=0.1, l2_std=0.1)
    E = eom.EOMSystem(s, l1=l1, l2=l2)
    sc, VL, foo, fvv, U = unfold.unfold(s)
    lam = synth.System(kmesh=s.kmesh, nocc=no, nvir=nv, eps=s.eps, eri_factor=s.eri_factor,
                       t1=np.conj(l1), t2=np.conj(l2))
    scl = unfold.unfold(lam)[0]
    Esc = eom.EOMSystem(sc, foo=foo[None], fvv=fvv[None], v_full=VL, l1=np.conj(scl.t1), l2=np.conj(scl.t2))
    om = np.array([-0.6, 0.2, 1.1])
    eta = 0.05
    Gsc = solve.dense_gf_matrix(Esc, 0, om, eta)
    GB = np.einsum("kP,wPQ,Ql->wkl", U.conj().T, Gsc, U)
    mesh = KMesh(km)
    scale = np.abs(GB).max()
    E0 = eom.EOMSystem(s)
    moved = 0.0
    for K in range(mesh.nk):
        for p in range(no + nv):
            gp, gm = solve.dense_gf(E, K, p, om, eta)
            i = unfold.bloch_index(mesh, no, nv, K, p)
            assert np.abs(gp + gm - GB[:, i, i]).max() <= 1e-12 * scale
            g0p, g0m = solve.dense_gf(E0, K, p, om, eta)
            moved = max(moved, np.abs(gp + gm - g0p - g0m).max())
    assert moved > 1e-4 * scale  # Lambda changes G
