"""Pins of the solves: closed form at T = V = 0 (P3), the zeroth-moment sum
rule and the 1/w tail (P5), orbital-rotation covariance (P8), GMRES against
dense inversion and SciPy (P2), and the eigen-decomposition form of G."""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_2208_07478_amd import synth
from oracle import eom, solve


def test_closed_form_kpoints():
    s = synth.make_system((2, 2, 1), 2, 3, seed=1, zero_t1=True, zero_t2=True, zero_eri=True)
    E = eom.EOMSystem(s)
    w = np.linspace(-1, 1, 5)
    eta = 0.01
    for K in range(4):
        for p in range(5):
            gp, gm = solve.dense_gf(E, K, p, w, eta)
            ref = 1.0 / (w - s.eps[K, p] + (1j * eta if p >= 2 else -1j * eta))
            assert np.allclose(gp + gm, ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("km", [(2, 1, 1), (3, 1, 1)])
def test_sum_rule_and_tail(km):
    s = synth.make_system(km, 2, 3, seed=2, t1_std=0.2, t2_std=0.2, eri_std=0.2)
    E = eom.EOMSystem(s)
    nmo = 5
    for K in range(E.nk):
        S = np.zeros((nmo, nmo), complex)
        for p, q in itertools.product(range(nmo), repeat=2):
            S[p, q] = (E.pack("ea", K, E.e_vector("ea", K, p)) @ E.pack("ea", K, E.b_vector("ea", K, q))
                       + E.pack("ip", K, E.e_vector("ip", K, q)) @ E.pack("ip", K, E.b_vector("ip", K, p)))
        assert np.allclose(S, np.eye(nmo), atol=1e-13)
    w = np.array([1e4, -1e4])
    gp, gm = solve.dense_gf(E, 0, 3, w, 0.01)
    assert np.allclose(w * (gp + gm), 1.0, atol=1e-3)


def _rotate(s, seed):
    """Per-k unitary rotations of the occupied and virtual orbitals."""
    nk, no, nv = s.eri_factor.shape[0], s.nocc, s.nvir
    U = np.zeros((nk, no + nv, no + nv), complex)
    for k in range(nk):
        U[k, :no, :no] = synth.random_unitary(no, seed=seed, block=2 * k)
        U[k, no:, no:] = synth.random_unitary(nv, seed=seed, block=2 * k + 1)
    A = np.einsum("aPp,abLpr,bRr->abLPR", U, s.eri_factor, U.conj())
    foo = np.einsum("kIi,ki,kJi->kIJ", U[:, :no, :no], s.eps[:, :no], U[:, :no, :no].conj())
    fvv = np.einsum("kAa,ka,kBa->kAB", U[:, no:, no:], s.eps[:, no:], U[:, no:, no:].conj())
    t1 = np.einsum("kIi,kia,kAa->kIA", U[:, :no, :no].conj(), s.t1, U[:, no:, no:])
    Uo, Uv = U[:, :no, :no], U[:, no:, no:]
    nkk = nk
    t2 = np.zeros_like(s.t2)
    from oracle.ktensor import KMesh
    mesh = KMesh(s.kmesh)
    for ki, kj, ka in itertools.product(range(nkk), repeat=3):
        kb = mesh.lin([(1, ki), (1, kj), (-1, ka)])
        t2[ki, kj, ka] = np.einsum("Ii,Jj,ijab,Aa,Bb->IJAB", Uo[ki].conj(), Uo[kj].conj(), s.t2[ki, kj, ka],
                                   Uv[ka], Uv[kb])
    r = synth.System(kmesh=s.kmesh, nocc=no, nvir=nv, eps=s.eps, eri_factor=A, t1=t1, t2=t2)
    return r, foo, fvv, U


def test_orbital_rotation_covariance():
    s = synth.make_system((2, 1, 1), 2, 3, seed=4, t1_std=0.2, t2_std=0.2, eri_std=0.2)
    r, foo, fvv, U = _rotate(s, 99)
    E = eom.EOMSystem(s)
    Er = eom.EOMSystem(r, foo=foo, fvv=fvv)
    w = np.array([-0.3, 0.5])
    for K in range(2):
        G = solve.dense_gf_matrix(E, K, w, 0.05)
        Gr = solve.dense_gf_matrix(Er, K, w, 0.05)
        back = np.einsum("Pp,wPQ,Qq->wpq", U[K].conj(), Gr, U[K])
        assert np.allclose(back, G, atol=1e-12)
        assert np.allclose(np.trace(Gr, axis1=1, axis2=2), np.trace(G, axis1=1, axis2=2), atol=1e-12)


def test_gmres_matches_dense_and_scipy():
    s = synth.make_system((2, 1, 1), 2, 4, seed=5, t1_std=0.1, t2_std=0.1, eri_std=0.1)
    E = eom.EOMSystem(s)
    w = np.array([-0.8, 0.05, 0.7])
    eta = 0.02
    for K, p in [(0, 1), (1, 4)]:
        gp, gm = solve.dense_gf(E, K, p, w, eta)
        gp2, gm2, its = solve.gmres_gf(E, K, p, w, eta, tol=1e-13)
        assert np.allclose(gp2, gp, rtol=1e-10, atol=1e-12 * np.abs(gp).max())
        assert np.allclose(gm2, gm, rtol=1e-10, atol=1e-12 * np.abs(gm).max())
    # SciPy's solvers (the paper uses GCROT(m,k)) on one system
    part, K, p, om = "ea", 0, 3, 0.05
    sM, sE = solve.shift_sign(part)
    b = E.pack(part, K, E.b_vector(part, K, p))
    mv = solve.shifted_operator(E, part, K, om, eta)
    op = spla.LinearOperator((b.size, b.size), matvec=mv, dtype=complex)
    xs, info = spla.gcrotmk(op, b, rtol=1e-13, maxiter=2000)
    x, it, res = solve.gmres(mv, b, tol=1e-13)
    assert info == 0 and np.linalg.norm(xs - x) <= 1e-9 * np.linalg.norm(x)


def test_eigen_decomposition_form():
    """G = sum_n (e . R_n)(L_n . b) / (w - s E_n + ...) with the biorthogonal eigenbasis."""
    s = synth.make_system((1, 1, 1), 2, 4, seed=6, t1_std=0.1, t2_std=0.1, eri_std=0.2)
    E = eom.EOMSystem(s)
    w = np.array([-0.4, 0.3])
    eta = 0.02
    for part in ("ip", "ea"):
        M = E.dense_matrix(part, 0)
        ev, R = np.linalg.eig(M)
        L = np.linalg.inv(R)
        sM, sE = solve.shift_sign(part)
        for p in range(6):
            b = E.pack(part, 0, E.b_vector(part, 0, p))
            e = E.pack(part, 0, E.e_vector(part, 0, p))
            g = np.array([np.sum((e @ R) * (L @ b) / (om + 1j * sE * eta + sM * ev)) for om in w])
            x = solve.dense_solutions(E, part, 0, p, w, eta)
            assert np.allclose(g, x @ e, atol=1e-12)


def test_dos_closed_form_and_matrix_diagonal():
    """DOS of the non-interacting system is a sum of Lorentzians (closed form);
    the diagonal of the full matrix is the per-orbital G, and at T = V = 0 the
    off-diagonal elements vanish."""
    s = synth.make_system((2, 1, 1), 2, 3, seed=3, zero_t1=True, zero_t2=True, zero_eri=True)
    E = eom.EOMSystem(s)
    w = np.linspace(-1.2, 2.1, 7)
    eta = 0.03
    for K in range(2):
        G = solve.dense_gf_matrix(E, K, w, eta)
        Gp, Gm = solve.dense_gf_matrix(E, K, w, eta, parts=True)
        assert np.allclose(Gp + Gm, G, rtol=0, atol=1e-15)
        off = G - np.einsum("wpp->wp", G)[:, :, None] * np.eye(5)
        assert np.abs(off).max() == 0.0
        ref = sum(eta / np.pi / ((w - s.eps[K, p]) ** 2 + eta ** 2) for p in range(5))
        assert np.allclose(solve.spectral_trace(Gp, Gm), ref, rtol=1e-13, atol=0)
    s = synth.make_system((3, 1, 1), 2, 3, seed=4, t1_std=0.1, t2_std=0.1, eri_std=0.2)
    E = eom.EOMSystem(s)
    G = solve.dense_gf_matrix(E, 1, w, eta)
    for p in range(5):
        gp, gm = solve.dense_gf(E, 1, p, w, eta)
        assert np.allclose(G[:, p, p], gp + gm, rtol=1e-12, atol=1e-14)
