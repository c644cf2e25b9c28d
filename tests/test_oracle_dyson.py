"""Pins of the active-space self-energy correction and Dyson's equation
(oracle.dyson, Eqs. 12-14) by closed forms."""
import numpy as np

from paper_2208_07478_amd import synth
from oracle import dyson


def herm(n, seed, scale=0.3):
    z = synth.random_vectors(n * n, 1, seed=seed)[0].reshape(n, n) * scale
    return 0.5 * (z + z.conj().T)


def resolvent(w, h, eta):
    n = h.shape[-1]
    return np.linalg.inv((w + 1j * eta) * np.eye(n) - h)


def test_cc_equal_to_low_level_in_the_active_space_gives_back_g_gw():
    N, M, eta = 7, 3, 0.05
    h = herm(N, 1)
    V = synth.random_unitary(N, seed=2)[:, :M]
    for w in (-0.4, 0.1, 0.9):
        Ggw = resolvent(w, h, eta)[None, None]
        Gcas = np.conj(V.T) @ Ggw[0, 0] @ V
        G, Sf, S = dyson.cc_gw(Ggw, Gcas[None, None], Gcas[None, None], V[None])
        assert np.abs(S).max() < 1e-12
        assert np.allclose(G, Ggw, rtol=0, atol=1e-12)


def test_complete_active_space_gives_the_rotated_cc_green_function():
    N, eta = 6, 0.04
    h, hc = herm(N, 3), herm(N, 4)
    V = synth.random_unitary(N, seed=5)
    for w in (-0.7, 0.3):
        Ggw = resolvent(w, h, eta)
        Gcc = resolvent(w, hc, eta)
        G, _, _ = dyson.cc_gw(Ggw[None, None], (np.conj(V.T) @ Ggw @ V)[None, None], Gcc[None, None], V[None])
        assert np.allclose(G[0, 0], V @ Gcc @ np.conj(V.T), rtol=0, atol=1e-11 * np.abs(Gcc).max())


def test_static_self_energies_give_the_corrected_resolvent():
    """G_GW = (w - h)^-1, G_GW,CAS = (w - V^H h V)^-1, G_CC,CAS = (w - hc)^-1 make
    Sigma_CAS = hc - V^H h V static, and G_CC+GW the resolvent of h + V Sigma V^H."""
    N, M, eta = 8, 3, 0.05
    h, hc = herm(N, 6), herm(M, 7)
    V = synth.random_unitary(N, seed=8)[:, :M]
    hcas = np.conj(V.T) @ h @ V
    heff = h + V @ (hc - hcas) @ np.conj(V.T)
    ws = np.array([-0.5, -0.1, 0.4])
    Ggw = np.array([resolvent(w, h, eta) for w in ws])[None]
    Gcas = np.array([resolvent(w, hcas, eta) for w in ws])[None]
    Gcc = np.array([resolvent(w, hc, eta) for w in ws])[None]
    G, Sf, S = dyson.cc_gw(Ggw, Gcas, Gcc, V[None])
    for i, w in enumerate(ws):
        assert np.allclose(S[0, i], hc - hcas, rtol=0, atol=1e-11)
        assert np.allclose(G[0, i], resolvent(w, heff, eta), rtol=0, atol=1e-10)
