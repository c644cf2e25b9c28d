"""Shifted linear solves of Eq. 6 and G = e . x of Eq. 7 (test infrastructure).

For orbital p at momentum K:
  G-_pp(K, w) = e-_p . [(w + M_IP(K) - i eta)^-1 b-_p]
  G+_pp(K, w) = e+_p . [(w - M_EA(K) + i eta)^-1 b+_p]
(Eqs. 6, 7 and 9 read literally, with the time-ordered signs of Eq. 1.)

The plain definition is a direct solve.  ``dense_*`` inverts the explicitly
built matrix (unique-coefficient basis); ``gmres`` is the oracle's own
restarted GMRES for sizes where the dense matrix is too large.  The paper uses
SciPy's GCROT(m,k); any converged Krylov solver reaches the same x within its
tolerance, which the tests check against the dense result and against SciPy.

Parity: dense solves pinned by the closed form at T = V = 0, the zeroth-moment
sum rule and the eigen-decomposition form of G; GMRES pinned against dense
inversion and scipy.sparse.linalg (tests/test_oracle_solve.py).
"""
from __future__ import annotations

import numpy as np


def shift_sign(part):
    """(s_M, s_eta): IP uses w + M - i eta, EA uses w - M + i eta."""
    return (1.0, -1.0) if part == "ip" else (-1.0, 1.0)


def dense_solutions(E, part, K, p, omegas, eta):
    """Solutions x(w) in the unique basis for the right-hand side of orbital p."""
    M = E.dense_matrix(part, K)
    b = E.pack(part, K, E.b_vector(part, K, p))
    sM, sE = shift_sign(part)
    n = M.shape[0]
    I = np.eye(n)
    return np.array([np.linalg.solve((w + 1j * sE * eta) * I + sM * M, b) for w in np.atleast_1d(omegas)])


def dense_gf(E, K, p, omegas, eta, M_cache=None):
    """(G+, G-) for orbital p at momentum K by dense inversion."""
    out = {}
    for part in ("ea", "ip"):
        if M_cache is not None and (part, K) in M_cache:
            M = M_cache[(part, K)]
        else:
            M = E.dense_matrix(part, K)
            if M_cache is not None:
                M_cache[(part, K)] = M
        b = E.pack(part, K, E.b_vector(part, K, p))
        e = E.pack(part, K, E.e_vector(part, K, p))
        sM, sE = shift_sign(part)
        I = np.eye(M.shape[0])
        out[part] = np.array([e @ np.linalg.solve((w + 1j * sE * eta) * I + sM * M, b)
                              for w in np.atleast_1d(omegas)])
    return out["ea"], out["ip"]


def dense_gf_matrix(E, K, omegas, eta, parts=False):
    """Full G_pq(K, w) over all orbitals (needed for the supercell transform).
    G+_pq = e+_p . Y_q,  G-_pq = e-_q . X_p.  With parts=True returns (G+, G-)."""
    nmo = E.no + E.nv
    res = np.zeros((len(np.atleast_1d(omegas)), nmo, nmo), dtype=np.complex128)
    by_part = {"ea": np.zeros_like(res), "ip": np.zeros_like(res)}
    for part in ("ea", "ip"):
        M = E.dense_matrix(part, K)
        sM, sE = shift_sign(part)
        I = np.eye(M.shape[0])
        B = np.array([E.pack(part, K, E.b_vector(part, K, p)) for p in range(nmo)]).T
        Ev = np.array([E.pack(part, K, E.e_vector(part, K, p)) for p in range(nmo)])
        for iw, w in enumerate(np.atleast_1d(omegas)):
            X = np.linalg.solve((w + 1j * sE * eta) * I + sM * M, B)   # column q: solution for b_q
            P = Ev @ X                                                  # P[r, q] = e_r . x_q
            if part == "ea":
                by_part["ea"][iw] = P       # G+_pq = e+_p . Y_q
            else:
                by_part["ip"][iw] = P.T     # G-_pq = e-_q . X_p
            res[iw] += by_part[part][iw]
    if parts:
        return by_part["ea"], by_part["ip"]
    return res


def spectral_trace(Gplus, Gminus):
    """Density of states: trace of A(K, w) = -(1/pi) Im G(K, w) (the equation after
    Eq. 9), for G [..., norb, norb], with each part on the retarded side: Eq. 6 puts
    the removal part G- on the time-ordered side (w + M - i eta, poles above the real
    axis), whose retarded counterpart flips the sign of its imaginary part, so
    A = -(1/pi) (Im G+ - Im G-).  Pinned by the closed form at T = V = 0 (a sum of
    Lorentzians of weight one per orbital)."""
    tr = lambda G: np.trace(G, axis1=-2, axis2=-1)
    return -(np.imag(tr(Gplus)) - np.imag(tr(Gminus))) / np.pi


def gmres(matvec, b, *, dinv=None, x0=None, tol=1e-12, restart=30, maxiter=3000):
    """Restarted GMRES(m) with right preconditioning x = D^-1 u and modified
    Gram-Schmidt Arnoldi.  Stops when ||b - A x|| <= tol ||b|| (true residual
    checked at every restart).  Returns (x, iterations, relative residual)."""
    n = b.shape[0]
    x = np.zeros(n, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    dinv = np.ones(n) if dinv is None else dinv
    bnorm = np.linalg.norm(b)
    if bnorm == 0:
        return x, 0, 0.0
    it = 0
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    while it < maxiter:
        if beta <= tol * bnorm:
            break
        V = np.zeros((restart + 1, n), dtype=np.complex128)
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        cs = np.zeros(restart, dtype=np.complex128)
        sn = np.zeros(restart, dtype=np.complex128)
        g = np.zeros(restart + 1, dtype=np.complex128)
        g[0] = beta
        V[0] = r / beta
        k_used = 0
        for j in range(restart):
            w = matvec(dinv * V[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            # complex Givens rotations G = [[c, s], [-conj(s), c]] with real c
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            a, h = H[j, j], H[j + 1, j]
            rho = np.sqrt(abs(a) ** 2 + abs(h) ** 2)
            if abs(a) == 0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / rho
                sn[j] = (a / abs(a)) * np.conj(h) / rho
            H[j, j] = cs[j] * a + sn[j] * h
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k_used = j + 1
            if abs(g[j + 1]) <= tol * bnorm or it >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:k_used, :k_used]), g[:k_used])
        x = x + dinv * (V[:k_used].T @ y)
        r = b - matvec(x)
        beta = np.linalg.norm(r)
    return x, it, beta / bnorm


def shifted_operator(E, part, K, w, eta, unique=True):
    """A(w) x for the unique-basis vector x (or full storage with unique=False)."""
    sM, sE = shift_sign(part)
    shift = w + 1j * sE * eta
    if unique:
        def mv(u):
            return shift * u + sM * E.pack(part, K, E.sigma(part, K, E.unpack(part, K, u)))
    else:
        def mv(x):
            return shift * x + sM * E.sigma(part, K, x)
    return mv


def gmres_gf(E, K, p, omegas, eta, tol=1e-12, restart=30, maxiter=3000):
    """(G+, G-, iterations) with the oracle's GMRES in the unique basis."""
    out, its = {}, {}
    for part in ("ea", "ip"):
        sM, sE = shift_sign(part)
        b = E.pack(part, K, E.b_vector(part, K, p))
        e = E.pack(part, K, E.e_vector(part, K, p))
        d = E.pack(part, K, E.diag(part, K))
        vals, itl = [], []
        for w in np.atleast_1d(omegas):
            dinv = 1.0 / (w + 1j * sE * eta + sM * d)
            x, it, res = gmres(shifted_operator(E, part, K, w, eta), b, dinv=dinv, tol=tol,
                               restart=restart, maxiter=maxiter)
            vals.append(e @ x)
            itl.append(it)
        out[part] = np.array(vals)
        its[part] = itl
    return out["ea"], out["ip"], its
