"""O0: Fock-space brute force of the CC Green's function (test infrastructure).

Everything is built from second-quantised operators in a Jordan-Wigner
representation on n spin orbitals (occupied first), so no diagram algebra is
involved:

* H = sum h_pq a+_p a_q + 1/4 sum <pq||rs> a+_p a+_q a_s a_r with
  h = f - sum_i <pi||qi>, so that the Fock matrix with respect to the
  reference determinant Phi is f (Eqs. 1-2; the constant shift is irrelevant
  because only commutators and differences enter).
* T = sum t_i^a a+_a a_i + 1/4 sum t_ij^ab a+_a a+_b a_j a_i (CCSD, Eq. 2),
  Lambda = T^dagger (the approximation stated after Eq. 10).
* Hbar = exp(-T) H exp(T), abar_p = exp(-T) a_p exp(T) (Eq. 5).
* EOM-IP space {a_i Phi, a+_a a_j a_i Phi (i<j)} and EOM-EA space
  {a+_a Phi, a+_a a+_b a_i Phi (a<b)} (Eq. 8).  The EOM matrix is the
  connected commutator M[mu, nu] = <mu| [Hbar, R_nu] |Phi>; because every R_nu
  commutes with T this equals <mu| exp(-T) [H, R_nu] exp(T) |Phi>.
* Right-hand sides b_IP(p) = abar_p Phi, b_EA(q) = abar+_q Phi and left
  vectors e_IP(q)[mu] = <Phi|(1+Lambda) abar+_q |mu>,
  e_EA(p)[mu] = <Phi|(1+Lambda) abar_p |mu> (Eqs. 6-7).

Vectors here use the unique-coefficient basis (i<j, a<b) in the order
[singles, then (i<j, a) / (i, a<b) in lexicographic order].

Parity: pinned by closed forms (T = V = 0), the exact zeroth-moment sum rule,
Hermiticity at T = 0 and the FCI ionisation energies of a two-electron system
(tests/test_oracle_fock.py).
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp


def annihilators(n: int):
    """Jordan-Wigner a_p on 2^n states; bit p of the state index = occupation of p."""
    dim = 1 << n
    ops = []
    idx = np.arange(dim)
    for p in range(n):
        occ = (idx >> p) & 1
        src = idx[occ == 1]
        dst = src ^ (1 << p)
        # sign (-1)^(number of occupied orbitals with index < p)
        below = np.array([bin(s & ((1 << p) - 1)).count("1") for s in src])
        sgn = np.where(below % 2 == 0, 1.0, -1.0)
        ops.append(sp.csr_matrix((sgn.astype(np.complex128), (dst, src)), shape=(dim, dim)))
    return ops


class FockSpace:
    """Operators of one molecular problem (nocc occupied + nvir virtual spin orbitals)."""

    def __init__(self, f, v, t1, t2, nocc, l1=None, l2=None):
        n = f.shape[0]
        self.n, self.no, self.nv = n, nocc, n - nocc
        a = annihilators(n)
        ad = [x.conj().T.tocsr() for x in a]
        self.a, self.ad = a, ad
        no = nocc
        # one-body part with the mean-field shift removed so that Fock = f
        h = f - np.einsum("piqi->pq", v[:, :no, :, :no])
        H = sp.csr_matrix((1 << n, 1 << n), dtype=np.complex128)
        for p in range(n):
            for q in range(n):
                if h[p, q] != 0:
                    H = H + h[p, q] * (ad[p] @ a[q])
        pair = {}
        for r in range(n):
            for s in range(n):
                if r != s:
                    pair[(r, s)] = (a[s] @ a[r]).tocsr()  # a_s a_r
        for r in range(n):
            for s in range(n):
                if r == s:
                    continue
                S = sp.csr_matrix((1 << n, 1 << n), dtype=np.complex128)
                for p in range(n):
                    for q in range(n):
                        if p != q and v[p, q, r, s] != 0:
                            S = S + v[p, q, r, s] * pair[(p, q)].conj().T  # (a_q a_p)^+ = a+_p a+_q
                H = H + 0.25 * (S @ pair[(r, s)])
        self.H = H.tocsr()
        # cluster operator and Lambda
        T = sp.csr_matrix((1 << n, 1 << n), dtype=np.complex128)
        for i in range(no):
            for A in range(self.nv):
                if t1[i, A] != 0:
                    T = T + t1[i, A] * (ad[no + A] @ a[i])
        for i in range(no):
            for j in range(no):
                for A in range(self.nv):
                    for B in range(self.nv):
                        c = t2[i, j, A, B]
                        if c != 0:
                            T = T + 0.25 * c * (ad[no + A] @ ad[no + B] @ a[j] @ a[i])
        self.T = T.tocsr()
        if l1 is None and l2 is None:
            self.L = self.T.conj().T.tocsr()   # Lambda = T^dagger
        else:
            L = sp.csr_matrix((1 << n, 1 << n), dtype=np.complex128)
            for i in range(no):
                for A in range(self.nv):
                    L = L + l1[i, A] * (ad[i] @ a[no + A])
            for i in range(no):
                for j in range(no):
                    for A in range(self.nv):
                        for B in range(self.nv):
                            L = L + 0.25 * l2[i, j, A, B] * (ad[i] @ ad[j] @ a[no + B] @ a[no + A])
            self.L = L.tocsr()
        phi = np.zeros(1 << n, dtype=np.complex128)
        phi[(1 << no) - 1] = 1.0
        self.phi = phi
        self.ip_ops = self._ip_basis()
        self.ea_ops = self._ea_basis()

    # exp(c*T) v by the terminating series (T is nilpotent)
    def _exp(self, X, v, c=1.0):
        out = v.copy()
        term = v.copy()
        for k in range(1, 2 * self.n + 2):
            term = (c / k) * (X @ term)
            if not np.any(term):
                break
            out = out + term
        return out

    def _ip_basis(self):
        no, nv = self.no, self.nv
        ops = [self.a[i] for i in range(no)]
        for i, j in itertools.combinations(range(no), 2):
            for A in range(nv):
                ops.append(self.ad[no + A] @ self.a[j] @ self.a[i])
        return ops

    def _ea_basis(self):
        no, nv = self.no, self.nv
        ops = [self.ad[no + A] for A in range(nv)]
        for i in range(no):
            for A, B in itertools.combinations(range(nv), 2):
                ops.append(self.ad[no + A] @ self.ad[no + B] @ self.a[i])
        return ops

    def _states(self, ops):
        return np.array([op @ self.phi for op in ops])

    def _project(self, ops, vec, check=True):
        S = self._states(ops)
        c = S.conj() @ vec
        if check:
            resid = vec - S.T @ c
            assert np.linalg.norm(resid) <= 1e-10 * max(1.0, np.linalg.norm(vec)), \
                "vector leaves the EOM space"
        return c

    def eom_matrix(self, part: str) -> np.ndarray:
        ops = self.ip_ops if part == "ip" else self.ea_ops
        u = self._exp(self.T, self.phi)
        Hu = self.H @ u
        S = self._states(ops)
        cols = []
        for R in ops:
            w = self.H @ (R @ u) - R @ Hu
            z = self._exp(self.T, w, -1.0)
            cols.append(S.conj() @ z)
        return np.array(cols).T

    def b_vector(self, part: str, p: int) -> np.ndarray:
        """IP: abar_p Phi;  EA: abar+_p Phi, in the unique basis."""
        op = self.a[p] if part == "ip" else self.ad[p]
        ops = self.ip_ops if part == "ip" else self.ea_ops
        w = self._exp(self.T, op @ self._exp(self.T, self.phi), -1.0)
        return self._project(ops, w)

    def e_vector(self, part: str, q: int) -> np.ndarray:
        """IP: <Phi|(1+L) abar+_q |mu>;  EA: <Phi|(1+L) abar_q |mu>."""
        ops = self.ip_ops if part == "ip" else self.ea_ops
        # ket psi with <psi| = <Phi|(1+L) exp(-T) X exp(T),  X = a+_q (IP) or a_q (EA)
        Xd = self.a[q] if part == "ip" else self.ad[q]
        Ld = self.L.conj().T.tocsr()
        Td = self.T.conj().T.tocsr()
        psi = self.phi + Ld @ self.phi
        psi = self._exp(Td, psi, -1.0)
        psi = Xd @ psi
        psi = self._exp(Td, psi, 1.0)
        S = self._states(ops)
        return psi.conj() @ S.T

    def hamiltonian_sector(self, nelec: int) -> np.ndarray:
        """Dense H restricted to determinants with nelec electrons (for FCI checks)."""
        idx = [s for s in range(1 << self.n) if bin(s).count("1") == nelec]
        return self.H[idx][:, idx].toarray()


def greens_function(fs: FockSpace, p: int, omega, eta):
    """Diagonal G_pp(omega) = G+ + G- from dense solves of the O0 matrices."""
    Mip = fs.eom_matrix("ip")
    Mea = fs.eom_matrix("ea")
    bi, ei = fs.b_vector("ip", p), fs.e_vector("ip", p)
    be, ee = fs.b_vector("ea", p), fs.e_vector("ea", p)
    out = []
    Iip = np.eye(Mip.shape[0])
    Iea = np.eye(Mea.shape[0])
    for w in np.atleast_1d(omega):
        gm = ei @ np.linalg.solve((w - 1j * eta) * Iip + Mip, bi)
        gp = ee @ np.linalg.solve((w + 1j * eta) * Iea - Mea, be)
        out.append(gp + gm)
    return np.array(out)


def n_ip(no, nv):
    return no + math.comb(no, 2) * nv


def n_ea(no, nv):
    return nv + no * math.comb(nv, 2)
