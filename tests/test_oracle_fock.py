"""Pins of the Fock-space brute force (O0) against closed forms and textbook
results: T = V = 0 poles, Hermiticity at T = 0, the zeroth-moment sum rule and
FCI ionisation energies of a two-electron system."""
import itertools

import numpy as np
import pytest

from oracle import fock


def rand_inputs(no, nv, seed, tamp=0.2, vamp=0.2, zero_t=False, zero_v=False):
    rng = np.random.default_rng(seed)
    n = no + nv
    eps = np.concatenate([np.sort(rng.uniform(-1, -0.3, no)), np.sort(rng.uniform(0.2, 2, nv))])
    f = np.diag(eps).astype(complex)
    g = (rng.normal(size=(n, n, n, n)) + 1j * rng.normal(size=(n, n, n, n))) * vamp
    g = g + g.transpose(2, 3, 0, 1).conj()          # Hermitian <pq|rs> = <rs|pq>*
    g = g + g.transpose(1, 0, 3, 2)                 # particle exchange
    v = g - g.transpose(0, 1, 3, 2)
    if zero_v:
        v[:] = 0
    t1 = (rng.normal(size=(no, nv)) + 1j * rng.normal(size=(no, nv))) * tamp
    t2 = (rng.normal(size=(no, no, nv, nv)) + 1j * rng.normal(size=(no, no, nv, nv))) * tamp
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    if zero_t:
        t1[:] = 0
        t2[:] = 0
    return eps, f, v, t1, t2


def test_closed_form_free_particles():
    """T = 0 and V = 0: G_pp = 1/(w - eps_p - i eta) (occupied), 1/(w - eps_p + i eta) (virtual)."""
    eps, f, v, t1, t2 = rand_inputs(2, 3, 1, zero_t=True, zero_v=True)
    fs = fock.FockSpace(f, v, t1, t2, 2)
    w = np.array([-0.9, -0.2, 0.4, 1.3])
    eta = 0.03
    for p in range(5):
        ref = 1.0 / (w - eps[p] + (1j * eta if p >= 2 else -1j * eta))
        assert np.allclose(fock.greens_function(fs, p, w, eta), ref, rtol=1e-13, atol=0)


def test_hermitian_at_t0():
    eps, f, v, t1, t2 = rand_inputs(2, 3, 2, zero_t=True)
    fs = fock.FockSpace(f, v, t1, t2, 2)
    for part in ("ip", "ea"):
        M = fs.eom_matrix(part)
        assert np.allclose(M, M.conj().T, atol=1e-13)


@pytest.mark.parametrize("no,nv,seed", [(2, 3, 3), (3, 3, 4)])
def test_zeroth_moment_sum_rule(no, nv, seed):
    """e+_p . b+_q + e-_q . b-_p = delta_pq for any T (Lambda = T^dagger)."""
    eps, f, v, t1, t2 = rand_inputs(no, nv, seed)
    fs = fock.FockSpace(f, v, t1, t2, no)
    n = no + nv
    S = np.zeros((n, n), complex)
    for p, q in itertools.product(range(n), repeat=2):
        S[p, q] = fs.e_vector("ea", p) @ fs.b_vector("ea", q) + fs.e_vector("ip", q) @ fs.b_vector("ip", p)
    assert np.allclose(S, np.eye(n), atol=1e-12)


def _fci_t_amplitudes(fs, no, nv):
    """Exact two-electron ground state written as exp(T) Phi (intermediate normalisation)."""
    n = no + nv
    nel = [s for s in range(1 << n) if bin(s).count("1") == no]
    Hn = fs.H[nel][:, nel].toarray()
    E, C = np.linalg.eigh(Hn)
    psi = np.zeros(1 << n, complex)
    psi[nel] = C[:, 0]
    psi /= np.vdot(fs.phi, psi)
    t1 = np.zeros((no, nv), complex)
    for i in range(no):
        for a in range(nv):
            st = fs.ad[no + a] @ fs.a[i] @ fs.phi
            t1[i, a] = np.vdot(st, psi)
    t2 = np.zeros((no, no, nv, nv), complex)
    for i, j in itertools.combinations(range(no), 2):
        for a, b in itertools.combinations(range(nv), 2):
            st = fs.ad[no + a] @ fs.ad[no + b] @ fs.a[j] @ fs.a[i] @ fs.phi
            c = np.vdot(st, psi) - (t1[i, a] * t1[j, b] - t1[i, b] * t1[j, a])
            t2[i, j, a, b] = c
            t2[j, i, a, b] = -c
            t2[i, j, b, a] = -c
            t2[j, i, b, a] = c
    return E[0], t1, t2


def test_fci_ionisation_energies_two_electrons():
    """Two electrons: CCSD is exact and the EOM-IP space is the whole N-1 space,
    so the IP poles equal FCI removal energies E_N - E_{N-1}."""
    no, nv = 2, 4
    eps, f, v, t1, t2 = rand_inputs(no, nv, 7, zero_t=True, vamp=0.05)
    fs0 = fock.FockSpace(f, v, t1, t2, no)
    E0, t1, t2 = _fci_t_amplitudes(fs0, no, nv)
    fs = fock.FockSpace(f, v, t1, t2, no)
    # CC residuals vanish: exp(-T) H exp(T) Phi has no singles/doubles component
    w = fs._exp(fs.T, fs.H @ fs._exp(fs.T, fs.phi), -1.0)
    ecc = np.vdot(fs.phi, w)
    assert abs(ecc - E0) < 1e-10
    resid = w - ecc * fs.phi
    assert np.linalg.norm(resid) < 1e-10
    Em1 = np.linalg.eigvalsh(fs.hamiltonian_sector(no - 1))
    M = fs.eom_matrix("ip")
    ev = np.sort(np.linalg.eigvals(M).real)
    ref = np.sort(Em1 - E0)
    assert np.allclose(ev, ref, atol=1e-10)
