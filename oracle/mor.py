"""O4: model-order-reduction frequency interpolation (test infrastructure).

The paper's MOR paragraph: the full shifted systems of Eq. 6 are solved only at
a few expansion frequencies; their solutions span a subspace; Hbar is projected
onto it, giving a model of dimension N_MOR x N_MOR that is then solved at every
frequency of the grid.  Reading taken (one-sided Galerkin, per momentum K,
orbital p and part):

  S      = orthonormal basis of {x(w_1), ..., x(w_N)} (Gram-Schmidt, two
           passes, unique-pair inner product; columns whose norm falls below
           1e-10 of the largest are dropped),
  Ht     = S^H M S,   bt = S^H b,   et = e S   (e . x bilinear as in Eq. 7),
  G(w)   = et (w + s_M Ht + i s_eta eta)^-1 bt.

Parity pins (tests/test_oracle_mor.py): at every expansion point the model
reproduces the full solve (Galerkin property, exact when x(w_j) lies in the
span); when S spans the whole space the model equals the full G at every
frequency.
"""
from __future__ import annotations

import numpy as np

from .solve import dense_solutions, shift_sign


def orthonormal_basis(X: np.ndarray, drop: float = 1e-10) -> np.ndarray:
    """Columns of X (n x N) -> orthonormal S (n x r), Gram-Schmidt in two passes."""
    cols = []
    norms = [np.linalg.norm(X[:, j]) for j in range(X.shape[1])]
    big = max(norms) if norms else 0.0
    for j in range(X.shape[1]):
        w = X[:, j].astype(np.complex128).copy()
        for _ in range(2):
            for s in cols:
                w = w - np.vdot(s, w) * s
        nw = np.linalg.norm(w)
        if nw > drop * big:
            cols.append(w / nw)
    return np.array(cols).T if cols else np.zeros((X.shape[0], 0), complex)


def mor_model(E, part, K, p, w_exp, eta, solutions=None):
    """(Ht, bt, et) of the reduced model of orbital p (unique-coefficient basis)."""
    if solutions is None:
        solutions = dense_solutions(E, part, K, p, w_exp, eta)
    S = orthonormal_basis(np.asarray(solutions).T)
    M = E.dense_matrix(part, K)
    b = E.pack(part, K, E.b_vector(part, K, p))
    e = E.pack(part, K, E.e_vector(part, K, p))
    Ht = S.conj().T @ M @ S
    bt = S.conj().T @ b
    et = e @ S
    return Ht, bt, et


def mor_gf(E, part, K, p, w_exp, omegas, eta, solutions=None):
    """G+ (EA) or G- (IP) of orbital p on the frequency grid from the reduced model."""
    Ht, bt, et = mor_model(E, part, K, p, w_exp, eta, solutions)
    sM, sE = shift_sign(part)
    r = Ht.shape[0]
    I = np.eye(r)
    return np.array([et @ np.linalg.solve((w + 1j * sE * eta) * I + sM * Ht, bt) for w in np.atleast_1d(omegas)])
