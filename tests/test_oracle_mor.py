"""Pins of the MOR oracle (O4): the reduced model reproduces the full solve at
the expansion frequencies, and equals it everywhere when the expansion
solutions span the whole EOM space."""
import numpy as np

from paper_2208_07478_amd import synth
from oracle import eom, mor, solve


def test_interpolates_at_expansion_points():
    s = synth.make_system((2, 1, 1), 2, 4, seed=31, t1_std=0.05, t2_std=0.05, eri_std=0.1)
    E = eom.EOMSystem(s)
    eta = 0.02
    for part, wexp in (("ip", np.linspace(-1.0, 0.0, 4)), ("ea", np.linspace(0.0, 1.0, 4))):
        for K, p in ((0, 1), (1, 4)):
            g_full = solve.dense_gf(E, K, p, wexp, eta)
            full = g_full[0] if part == "ea" else g_full[1]
            g_mor = mor.mor_gf(E, part, K, p, wexp, wexp, eta)
            assert np.allclose(g_mor, full, rtol=1e-10, atol=1e-12 * np.abs(full).max())


def test_full_span_reproduces_every_frequency():
    # Gamma, 2 occupied + 3 virtual: the IP space has 2 + 3 = 5 unique coefficients
    s = synth.make_system((1, 1, 1), 2, 3, seed=32, real=True, naux=10)
    E = eom.EOMSystem(s)
    eta = 0.03
    n = len(E.unique_index("ip", 0)[0])
    wexp = np.linspace(-1.2, 0.4, n + 2)
    w = np.linspace(-1.5, 1.5, 31)
    for p in range(5):
        full = solve.dense_gf(E, 0, p, w, eta)[1]
        g_mor = mor.mor_gf(E, "ip", 0, p, wexp, w, eta)
        assert np.allclose(g_mor, full, rtol=1e-9, atol=1e-11 * max(np.abs(full).max(), 1e-300))


def test_basis_is_orthonormal_and_drops_dependent_columns():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(20, 3)) + 1j * rng.normal(size=(20, 3))
    X = np.concatenate([X, X[:, :1] * 2.0 - X[:, 1:2]], axis=1)   # dependent column
    S = mor.orthonormal_basis(X)
    assert S.shape == (20, 3)
    assert np.allclose(S.conj().T @ S, np.eye(3), atol=1e-14)
