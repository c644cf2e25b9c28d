"""O2b: sigma products at large k-meshes from H-bar blocks formed one at a time
(test infrastructure).

At a 3x3x3 mesh the dense classes of ``oracle.eom`` do not fit in host memory
(the vvvv class alone is Nk^3 Nv^4 complex numbers, 144 GB for the Si-like
system).  This module evaluates the same similarity-transformed Hamiltonian
blocks and the same EOM-IP/EA-CCSD sigma terms as ``oracle.eom`` (standard
spin-orbital CCSD H-bar, Lambda = T^dagger; Eqs. 6-9 and the cost paragraph of
the paper), but per momentum block and only for the blocks one requested output
block of sigma needs, forming every bare integral block from the momentum-
blocked factor on demand:

    <p k1, q k2 || r k3, s k4> = sum_L A[k1,k3,L,p,r] A[k2,k4,L,q,s]
                               - sum_L A[k1,k4,L,p,s] A[k2,k3,L,q,r],
    k4 = k1 + k2 - k3.

Each H-bar block below writes out the terms of ``EOMSystem._build`` with the
internal momentum sums made explicit; each sigma block writes out the terms of
``EOMSystem.sigma_ea`` / ``sigma_ip`` for one output block.  Nothing is blocked,
fused or reordered beyond selecting which output block to form.

Parity: every H-bar block and every sigma block is pinned against
``oracle.eom`` (itself pinned against the Fock-space brute force) on several
small meshes (tests/test_oracle_blocks.py).
"""
from __future__ import annotations

import functools
import itertools

import numpy as np

from .ktensor import KMesh


class BlockSystem:
    """H-bar and sigma blocks of one synthetic system (``synth.System``)."""

    def __init__(self, sys, cache_blocks: int = 4096):
        self.mesh = KMesh(sys.kmesh)
        self.nk = self.mesh.nk
        self.no, self.nv = sys.nocc, sys.nvir
        self.A = np.asarray(sys.eri_factor, dtype=np.complex128)
        self.t1 = np.asarray(sys.t1, dtype=np.complex128)
        self.t2 = np.asarray(sys.t2, dtype=np.complex128)
        no, nv = self.no, self.nv
        nk = self.nk
        if sys.foo is not None:
            self.foo = np.asarray(sys.foo, dtype=np.complex128)
        else:
            self.foo = np.array([np.diag(sys.eps[k, :no]) for k in range(nk)]).astype(np.complex128)
        if sys.fvv is not None:
            self.fvv = np.asarray(sys.fvv, dtype=np.complex128)
        else:
            self.fvv = np.array([np.diag(sys.eps[k, no:]) for k in range(nk)]).astype(np.complex128)
        self.sl = {"o": slice(0, no), "v": slice(no, no + nv)}
        # bounded caches of the blocks formed so far
        self.v = functools.lru_cache(maxsize=cache_blocks)(self._v)
        for name in ("tau", "Wvvvv", "Wovvo", "Wvovv", "Wvvvo", "Woooo", "Wooov", "Wovoo", "Zovvo"):
            setattr(self, name, functools.lru_cache(maxsize=cache_blocks)(getattr(self, "_" + name)))
        self._F = None

    # ------------------------------------------------------------ momenta
    def k4(self, k1, k2, k3):
        """k1 + k2 - k3 on the mesh."""
        return self.mesh.lin([(1, k1), (1, k2), (-1, k3)])

    # ------------------------------------------------- bare integral blocks
    def _v(self, cls, k1, k2, k3):
        """Antisymmetrised <p k1, q k2 || r k3, s k4> for the orbital classes
        ``cls`` (four letters o / v), from the factor."""
        A = self.A
        s1, s2, s3, s4 = (self.sl[ch] for ch in cls)
        k4 = self.k4(k1, k2, k3)
        d = np.einsum("Lpr,Lqs->pqrs", A[k1, k3][:, s1, s3], A[k2, k4][:, s2, s4], optimize=True)
        x = np.einsum("Lps,Lqr->pqrs", A[k1, k4][:, s1, s4], A[k2, k3][:, s2, s3], optimize=True)
        return d - x

    def T2(self, ki, kj, ka):
        return self.t2[ki, kj, ka]

    def _tau(self, ki, kj, ka):
        """tau_ij^ab = t_ij^ab + t_i^a t_j^b - t_i^b t_j^a (block ki, kj, ka)."""
        kb = self.k4(ki, kj, ka)
        t = self.t2[ki, kj, ka].copy()
        if ka == ki:
            t += np.einsum("ia,jb->ijab", self.t1[ki], self.t1[kj])
        if kb == ki:
            t -= np.einsum("ib,ja->ijab", self.t1[ki], self.t1[kj])
        return t

    # --------------------------------------------------- one-body blocks
    def fock(self):
        """(Fov, Foo, Fvv), each [nk][..][..] (k-diagonal)."""
        if self._F is not None:
            return self._F
        nk, no, nv = self.nk, self.no, self.nv
        t1 = self.t1
        Fov = np.zeros((nk, no, nv), complex)
        Foo = self.foo.copy()
        Fvv = self.fvv.copy()
        for k in range(nk):
            for kn in range(nk):
                Fov[k] += np.einsum("nf,mnef->me", t1[kn], self.v("oovv", k, kn, k))
                Foo[k] += np.einsum("ne,mnie->mi", t1[kn], self.v("ooov", k, kn, k))
                Fvv[k] += np.einsum("mf,amef->ae", t1[kn], self.v("vovv", k, kn, k))
                for ke in range(nk):
                    Foo[k] += 0.5 * np.einsum("inef,mnef->mi", self.tau(k, kn, ke), self.v("oovv", k, kn, ke))
                for km in range(nk):
                    # tau_mn^af (km, kn, k) with <mn||ef> (km, kn, k)
                    Fvv[k] -= 0.5 * np.einsum("mnaf,mnef->ae", self.tau(km, kn, k), self.v("oovv", km, kn, k))
        self._F = (Fov, Foo, Fvv)
        return self._F

    # --------------------------------------------------- two-body blocks
    def _Wvvvv(self, ka, kb, ke):
        """W_abef, block (ka, kb, ke)."""
        t1 = self.t1
        W = self.v("vvvv", ka, kb, ke).copy()
        W -= np.einsum("mb,amef->abef", t1[kb], self.v("vovv", ka, kb, ke))
        W += np.einsum("ma,bmef->abef", t1[ka], self.v("vovv", kb, ka, ke))
        for km in range(self.nk):
            kn = self.k4(ka, kb, km)
            W += 0.5 * np.einsum("mnab,mnef->abef", self.tau(km, kn, ka), self.v("oovv", km, kn, ke))
        return W

    def _Wovvo(self, km, kb, ke):
        """W_mbej, block (km, kb, ke); kj = km + kb - ke."""
        t1, nk = self.t1, self.nk
        kj = self.k4(km, kb, ke)
        W = self.v("ovvo", km, kb, ke).copy()
        W += np.einsum("jf,mbef->mbej", t1[kj], self.v("ovvv", km, kb, ke))
        W -= np.einsum("nb,mnej->mbej", t1[kb], self.v("oovo", km, kb, ke))
        for kn in range(nk):
            kf = self.k4(km, kn, ke)
            W -= np.einsum("jnfb,mnef->mbej", self.T2(kj, kn, kf), self.v("oovv", km, kn, ke))
        y = np.einsum("jf,mnef->mnej", t1[kj], self.v("oovv", km, kb, ke))
        W -= np.einsum("nb,mnej->mbej", t1[kb], y)
        return W

    def _Wvovv(self, ka, km, ke):
        """W_amef, block (ka, km, ke)."""
        return self.v("vovv", ka, km, ke) - np.einsum("na,nmef->amef", self.t1[ka], self.v("oovv", ka, km, ke))

    def _Zovvo(self, km, kb, ke):
        """z_mbej = <mb||ej> - t_nj^bf <mn||ef>, block (km, kb, ke); kj = km + kb - ke."""
        kj = self.k4(km, kb, ke)
        z = self.v("ovvo", km, kb, ke).copy()
        for kn in range(self.nk):
            kf = self.k4(km, kn, ke)
            z -= np.einsum("njbf,mnef->mbej", self.T2(kn, kj, kb), self.v("oovv", km, kn, ke))
            assert self.k4(kn, kj, kb) == kf
        return z

    def _Wvvvo(self, ka, kb, ke):
        """W_abei, block (ka, kb, ke); ki = ka + kb - ke."""
        t1, nk = self.t1, self.nk
        Fov = self.fock()[0]
        ki = self.k4(ka, kb, ke)
        W = self.v("vvvo", ka, kb, ke).copy()
        W -= np.einsum("me,miab->abei", Fov[ke], self.T2(ke, ki, ka))
        W += np.einsum("if,abef->abei", t1[ki], self.Wvvvv(ka, kb, ke))
        for km in range(nk):
            kn = self.k4(ke, ki, km)
            W += 0.5 * np.einsum("mnei,mnab->abei", self.v("oovo", km, kn, ke), self.tau(km, kn, ka))
            W -= np.einsum("mbef,miaf->abei", self.v("ovvv", km, kb, ke), self.T2(km, ki, ka))
            W += np.einsum("maef,mibf->abei", self.v("ovvv", km, ka, ke), self.T2(km, ki, kb))
        W -= np.einsum("ma,mbei->abei", t1[ka], self.Zovvo(ka, kb, ke))
        W += np.einsum("mb,maei->abei", t1[kb], self.Zovvo(kb, ka, ke))
        return W

    def _Woooo(self, km, kn, ki):
        """W_mnij, block (km, kn, ki); kj = km + kn - ki."""
        t1 = self.t1
        kj = self.k4(km, kn, ki)
        W = self.v("oooo", km, kn, ki).copy()
        W += np.einsum("je,mnie->mnij", t1[kj], self.v("ooov", km, kn, ki))
        W -= np.einsum("ie,mnje->mnij", t1[ki], self.v("ooov", km, kn, kj))
        for ke in range(self.nk):
            W += 0.5 * np.einsum("ijef,mnef->mnij", self.tau(ki, kj, ke), self.v("oovv", km, kn, ke))
        return W

    def _Wooov(self, km, kn, ki):
        """W_mnie, block (km, kn, ki)."""
        return self.v("ooov", km, kn, ki) + np.einsum("if,mnfe->mnie", self.t1[ki], self.v("oovv", km, kn, ki))

    def _Wovoo(self, km, kb, ki):
        """W_mbij, block (km, kb, ki); kj = km + kb - ki."""
        t1, nk = self.t1, self.nk
        Fov = self.fock()[0]
        kj = self.k4(km, kb, ki)
        W = self.v("ovoo", km, kb, ki).copy()
        W -= np.einsum("me,ijbe->mbij", Fov[km], self.T2(ki, kj, kb))
        W -= np.einsum("nb,mnij->mbij", t1[kb], self.Woooo(km, kb, ki))
        for ke in range(nk):
            W += 0.5 * np.einsum("mbef,ijef->mbij", self.v("ovvv", km, kb, ke), self.tau(ki, kj, ke))
        for kn in range(nk):
            W += np.einsum("mnie,jnbe->mbij", self.v("ooov", km, kn, ki), self.T2(kj, kn, kb))
            W -= np.einsum("mnje,inbe->mbij", self.v("ooov", km, kn, kj), self.T2(ki, kn, kb))
        W += np.einsum("ie,mbej->mbij", t1[ki], self.Zovvo(km, kb, ki))
        W -= np.einsum("je,mbei->mbij", t1[kj], self.Zovvo(km, kb, kj))
        return W

    # ------------------------------------------------------------ vectors
    def ea_split(self, x):
        nk, no, nv = self.nk, self.no, self.nv
        return x[:nv], x[nv:].reshape(nk, nk, no, nv, nv)

    def ip_split(self, x):
        nk, no, nv = self.nk, self.no, self.nv
        return x[:no], x[no:].reshape(nk, nk, no, no, nv)

    # -------------------------------------------------------------- sigma
    def sigma_ea_r1(self, K, x):
        """The 1p part of M_EA(K) x (rows a, k_a = K)."""
        Fov, Foo, Fvv = self.fock()
        nk = self.nk
        r1, r2 = self.ea_split(x)
        s = Fvv[K] @ r1
        for kl in range(nk):
            s += np.einsum("ld,lad->a", Fov[kl], r2[kl, K])
            for kc in range(nk):
                s += 0.5 * np.einsum("alcd,lcd->a", self.Wvovv(K, kl, kc), r2[kl, kc])
        return s

    def sigma_ea_block(self, K, x, ki, ka):
        """Block (ki, ka) of the 2p1h part of M_EA(K) x: s[i, a, b], kb = K + ki - ka."""
        Fov, Foo, Fvv = self.fock()
        nk = self.nk
        r1, r2 = self.ea_split(x)
        kb = self.k4(K, ki, ka)
        s = np.einsum("abei,e->iab", self.Wvvvo(ka, kb, K), r1)
        s += np.einsum("bd,iad->iab", Fvv[kb], r2[ki, ka])
        s -= np.einsum("ad,ibd->iab", Fvv[ka], r2[ki, kb])
        s -= np.einsum("li,lab->iab", Foo[ki], r2[ki, ka])
        for kc in range(nk):
            s += 0.5 * np.einsum("abcd,icd->iab", self.Wvvvv(ka, kb, kc), r2[ki, kc])
        for kl in range(nk):
            kd = self.k4(K, kl, ka)      # r2[kl][ka](l, a, d)
            s += np.einsum("lbdi,lad->iab", self.Wovvo(kl, kb, kd), r2[kl, ka])
            kd2 = self.k4(K, kl, kb)     # r2[kl][kb](l, b, d)
            s -= np.einsum("ladi,lbd->iab", self.Wovvo(kl, ka, kd2), r2[kl, kb])
        Y = np.zeros(self.no, complex)   # Y_k, k at momentum K
        for kl in range(nk):
            for kc in range(nk):
                Y += np.einsum("klcd,lcd->k", self.v("oovv", K, kl, kc), r2[kl, kc])
        s -= 0.5 * np.einsum("k,kiab->iab", Y, self.T2(K, ki, ka))
        return s

    def sigma_ip_r1(self, K, x):
        """The 1h part of M_IP(K) x (rows i, k_i = K)."""
        Fov, Foo, Fvv = self.fock()
        nk = self.nk
        r1, r2 = self.ip_split(x)
        s = -(Foo[K].T @ r1)
        for km in range(nk):
            s += np.einsum("me,ime->i", Fov[km], r2[K, km])
            for kn in range(nk):
                s -= 0.5 * np.einsum("mnie,mne->i", self.Wooov(km, kn, K), r2[km, kn])
        return s

    def sigma_ip_block(self, K, x, ki, kj):
        """Block (ki, kj) of the 2h1p part of M_IP(K) x: s[i, j, a], ka = ki + kj - K."""
        Fov, Foo, Fvv = self.fock()
        nk = self.nk
        r1, r2 = self.ip_split(x)
        ka = self.k4(ki, kj, K)
        s = -np.einsum("maij,m->ija", self.Wovoo(K, ka, ki), r1)
        s += np.einsum("ae,ije->ija", Fvv[ka], r2[ki, kj])
        s -= np.einsum("mi,mja->ija", Foo[ki], r2[ki, kj])
        s += np.einsum("mj,mia->ija", Foo[kj], r2[kj, ki])
        for km in range(nk):
            kn = self.k4(ki, kj, km)
            s += 0.5 * np.einsum("mnij,mna->ija", self.Woooo(km, kn, ki), r2[km, kn])
            ke = self.k4(km, kj, K)      # r2[km][kj](m, j, e)
            s += np.einsum("maei,mje->ija", self.Wovvo(km, ka, ke), r2[km, kj])
            ke2 = self.k4(km, ki, K)     # r2[km][ki](m, i, e)
            s -= np.einsum("maej,mie->ija", self.Wovvo(km, ka, ke2), r2[km, ki])
        X = np.zeros(self.nv, complex)   # X_e, e at momentum K
        for km in range(nk):
            for kn in range(nk):
                X += np.einsum("mnef,mnf->e", self.v("oovv", km, kn, K), r2[km, kn])
        s += 0.5 * np.einsum("e,ijae->ija", X, self.T2(ki, kj, ka))
        return s

    def sigma_block(self, part, K, x, k1, k2):
        """(r1 part, block (k1, k2) of the r2 part) of M(K) x."""
        if part == "ea":
            return self.sigma_ea_r1(K, x), self.sigma_ea_block(K, x, k1, k2)
        return self.sigma_ip_r1(K, x), self.sigma_ip_block(K, x, k1, k2)


def block_offset(sys_shape, part, k1, k2):
    """Offset of the r2 block (k1, k2) in the flat EOM vector and its length."""
    kmesh, no, nv = sys_shape
    nk = int(np.prod(kmesh))
    if part == "ea":
        b2 = no * nv * nv
        return nv + (k1 * nk + k2) * b2, b2
    b2 = no * no * nv
    return no + (k1 * nk + k2) * b2, b2


def all_blocks(nk):
    return list(itertools.product(range(nk), repeat=2))
