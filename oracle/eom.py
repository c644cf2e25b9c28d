"""O1/O2: k-point EOM-IP/EA-CCSD sigma products, b and e vectors (test infrastructure).

Spin-orbital EOM-CCSD in the Bloch basis.  The paper gives the linear systems
(Eq. 6), the EOM ansatz (Eq. 8), the k-point CCGF (Eq. 9), Lambda = T^dagger
(the approximation after Eq. 10) and the cost of the EA/IP products; it does
not print the similarity-transformed Hamiltonian.  The blocks used here are the
standard spin-orbital CCSD Hbar elements (one-body F, two-body W, plus the
three-body W_oovv * T2 terms); every prefactor and sign is pinned against the
Fock-space brute force of ``oracle.fock`` (tests/test_oracle_eom.py), not
taken on trust.

Reading of the paper used throughout:
* spin orbitals, nocc/nvir counted per cell;
* Fock matrix block diagonal per k with f_ov = 0;
* M is the connected commutator <mu|[Hbar, R]|Phi>;
* IP solves (omega + M - i eta) x = b, EA solves (omega - M + i eta) y = b
  (Eq. 6 read literally); G = e . x is bilinear (no conjugation of e).

Vector layouts (full antisymmetric storage, both orders of a pair present):
* IP, momentum K: r1[i] (k_i = K); r2[ki, kj, i, j, a] with ka = ki + kj - K.
* EA, momentum K: r1[a] (k_a = K); r2[ki, ka, i, a, b] with kb = K + ki - ka.
The flat form is [r1, r2.ravel()].  The unique-coefficient norm is
|r1|^2 + 1/2 |r2|^2.

A one-point mesh is the molecular case; a supercell is run through the same
code at one k-point (``oracle.unfold``).
"""
from __future__ import annotations

import itertools

import numpy as np

from .ktensor import KMesh, KT, keinsum, permute

P4 = (1, 1, -1, -1)
P2 = (1, -1)


def eri_blocks(mesh: KMesh, A: np.ndarray, s1: slice, s2: slice, s3: slice, s4: slice) -> KT:
    """Antisymmetrised <p k1 q k2 || r k3 s k4> = <pq|rs> - <pq|sr> for one
    orbital class, from the factor <pq|rs> = sum_L A[k1,k3,L,p,r] A[k2,k4,L,q,s]."""
    nk = mesh.nk
    shp = [s.stop - s.start for s in (s1, s2, s3, s4)]
    data = np.zeros([nk, nk, nk] + shp, dtype=np.complex128)
    for k1, k2, k3 in itertools.product(range(nk), repeat=3):
        k4 = mesh.lin([(1, k1), (1, k2), (-1, k3)])
        d = np.einsum("Lpr,Lqs->pqrs", A[k1, k3][:, s1, s3], A[k2, k4][:, s2, s4], optimize=True)
        x = np.einsum("Lps,Lqr->pqrs", A[k1, k4][:, s1, s4], A[k2, k3][:, s2, s3], optimize=True)
        data[k1, k2, k3] = d - x
    return KT(mesh, data, P4, 0)


class EOMSystem:
    """Hbar blocks of one synthetic system (a ``synth.System`` or equivalent)."""

    CLASSES = ("oooo", "ooov", "oovo", "oovv", "ovoo", "ovvo", "ovvv", "vovv", "vvvo", "vvvv")

    def __init__(self, sys, foo=None, fvv=None, l1=None, l2=None, v_full=None):
        """``sys`` carries kmesh, nocc, nvir, eps, eri_factor, t1, t2.  For a
        single k-point ``v_full`` (antisymmetrised <pq||rs>, all orbitals) may
        replace the factor, as needed for a supercell."""
        mesh = KMesh(sys.kmesh)
        self.mesh = mesh
        nk = mesh.nk
        no, nv = sys.nocc, sys.nvir
        self.no, self.nv, self.nk = no, nv, nk
        o, v = slice(0, no), slice(no, no + nv)
        sl = {"o": o, "v": v}
        if v_full is None:
            self.v = {c: eri_blocks(mesh, sys.eri_factor, *[sl[ch] for ch in c]) for c in self.CLASSES}
        else:
            assert nk == 1
            self.v = {c: KT(mesh, np.asarray(v_full)[tuple(sl[ch] for ch in c)][None, None, None].copy(), P4, 0)
                      for c in self.CLASSES}
        if foo is None:
            foo = np.array([np.diag(sys.eps[k, :no]) for k in range(nk)]).astype(np.complex128)
        if fvv is None:
            fvv = np.array([np.diag(sys.eps[k, no:]) for k in range(nk)]).astype(np.complex128)
        self.foo = KT(mesh, np.asarray(foo, dtype=np.complex128), P2)
        self.fvv = KT(mesh, np.asarray(fvv, dtype=np.complex128), P2)
        self.t1 = KT(mesh, np.asarray(sys.t1, dtype=np.complex128), P2)
        self.t2 = KT(mesh, np.asarray(sys.t2, dtype=np.complex128), P4)
        # Lambda = T^dagger unless given: lambda_a^i = conj(t_i^a), lambda_ab^ij = conj(t_ij^ab)
        self.l1 = self.t1.like(np.conj(self.t1.data)) if l1 is None else KT(mesh, l1, P2)
        self.l2 = self.t2.like(np.conj(self.t2.data)) if l2 is None else KT(mesh, l2, P4)
        self._build()

    # ------------------------------------------------------------------ Hbar
    def _build(self):
        v, t1, t2 = self.v, self.t1, self.t2
        ke = keinsum
        tt = ke("ia,jb->ijab", t1, t1, out_signs=P4)
        tau = t2 + tt - permute("ijab->ijba", tt)
        self.tau = tau

        Fov = ke("nf,mnef->me", t1, v["oovv"], out_signs=P2)
        Foo = self.foo.copy()
        ke("ne,mnie->mi", t1, v["ooov"], out_signs=P2, out=Foo)
        ke("inef,mnef->mi", tau, v["oovv"], out_signs=P2, out=Foo, alpha=0.5)
        Fvv = self.fvv.copy()
        ke("mf,amef->ae", t1, v["vovv"], out_signs=P2, out=Fvv)
        ke("mnaf,mnef->ae", tau, v["oovv"], out_signs=P2, out=Fvv, alpha=-0.5)

        Woooo = v["oooo"].copy()
        x = ke("je,mnie->mnij", t1, v["ooov"], out_signs=P4)
        Woooo = Woooo + x - permute("mnij->mnji", x)
        ke("ijef,mnef->mnij", tau, v["oovv"], out_signs=P4, out=Woooo, alpha=0.5)

        Wvvvv = v["vvvv"].copy()
        x = ke("mb,amef->abef", t1, v["vovv"], out_signs=P4)
        Wvvvv = Wvvvv - x + permute("abef->baef", x)
        ke("mnab,mnef->abef", tau, v["oovv"], out_signs=P4, out=Wvvvv, alpha=0.5)

        Wovvo = v["ovvo"].copy()
        ke("jf,mbef->mbej", t1, v["ovvv"], out_signs=P4, out=Wovvo)
        ke("nb,mnej->mbej", t1, v["oovo"], out_signs=P4, out=Wovvo, alpha=-1.0)
        ke("jnfb,mnef->mbej", t2, v["oovv"], out_signs=P4, out=Wovvo, alpha=-1.0)
        y = ke("jf,mnef->mnej", t1, v["oovv"], out_signs=P4)
        ke("nb,mnej->mbej", t1, y, out_signs=P4, out=Wovvo, alpha=-1.0)

        Wooov = v["ooov"].copy()
        ke("if,mnfe->mnie", t1, v["oovv"], out_signs=P4, out=Wooov)

        Wvovv = v["vovv"].copy()
        ke("na,nmef->amef", t1, v["oovv"], out_signs=P4, out=Wvovv, alpha=-1.0)

        # W_mbij
        Wovoo = v["ovoo"].copy()
        ke("me,ijbe->mbij", Fov, t2, out_signs=P4, out=Wovoo, alpha=-1.0)
        ke("nb,mnij->mbij", t1, Woooo, out_signs=P4, out=Wovoo, alpha=-1.0)
        ke("mbef,ijef->mbij", v["ovvv"], tau, out_signs=P4, out=Wovoo, alpha=0.5)
        x = ke("mnie,jnbe->mbij", v["ooov"], t2, out_signs=P4)
        Wovoo = Wovoo + x - permute("mbij->mbji", x)
        z = v["ovvo"].copy()
        ke("njbf,mnef->mbej", t2, v["oovv"], out_signs=P4, out=z, alpha=-1.0)
        x = ke("ie,mbej->mbij", t1, z, out_signs=P4)
        Wovoo = Wovoo + x - permute("mbij->mbji", x)

        # W_abei
        Wvvvo = v["vvvo"].copy()
        ke("me,miab->abei", Fov, t2, out_signs=P4, out=Wvvvo, alpha=-1.0)
        ke("if,abef->abei", t1, Wvvvv, out_signs=P4, out=Wvvvo)
        ke("mnei,mnab->abei", v["oovo"], tau, out_signs=P4, out=Wvvvo, alpha=0.5)
        x = ke("mbef,miaf->abei", v["ovvv"], t2, out_signs=P4)
        Wvvvo = Wvvvo - x + permute("abei->baei", x)
        z = v["ovvo"].copy()
        ke("nibf,mnef->mbei", t2, v["oovv"], out_signs=P4, out=z, alpha=-1.0)
        x = ke("ma,mbei->abei", t1, z, out_signs=P4)
        Wvvvo = Wvvvo - x + permute("abei->baei", x)

        self.Fov, self.Foo, self.Fvv = Fov, Foo, Fvv
        self.Woooo, self.Wvvvv, self.Wovvo = Woooo, Wvvvv, Wovvo
        self.Wooov, self.Wvovv, self.Wovoo, self.Wvvvo = Wooov, Wvovv, Wovoo, Wvvvo
        self.Woovv = v["oovv"]

    # -------------------------------------------------------------- vectors
    def ip_shapes(self):
        return (self.no,), (self.nk, self.nk, self.no, self.no, self.nv)

    def ea_shapes(self):
        return (self.nv,), (self.nk, self.nk, self.no, self.nv, self.nv)

    def vec_kt(self, part, K, r1=None, r2=None):
        s1, s2 = self.ip_shapes() if part == "ip" else self.ea_shapes()
        r1 = np.zeros(s1, complex) if r1 is None else np.asarray(r1, complex).reshape(s1)
        r2 = np.zeros(s2, complex) if r2 is None else np.asarray(r2, complex).reshape(s2)
        sg2 = (1, 1, -1) if part == "ip" else (-1, 1, 1)
        return KT(self.mesh, r1, (1,), K), KT(self.mesh, r2, sg2, K)

    def size(self, part):
        s1, s2 = self.ip_shapes() if part == "ip" else self.ea_shapes()
        return int(np.prod(s1) + np.prod(s2))

    def split(self, part, K, x):
        s1, s2 = self.ip_shapes() if part == "ip" else self.ea_shapes()
        n1 = int(np.prod(s1))
        return self.vec_kt(part, K, x[:n1], x[n1:])

    @staticmethod
    def join(r1: KT, r2: KT):
        return np.concatenate([r1.data.ravel(), r2.data.ravel()])

    # --------------------------------------------------------------- sigma
    def sigma_ip(self, K, x):
        r1, r2 = self.split("ip", K, x)
        ke = keinsum
        S1 = (1,)
        S2 = (1, 1, -1)
        s1 = ke("mi,m->i", self.Foo, r1, out_signs=S1, out_const=K, alpha=-1.0)
        ke("me,ime->i", self.Fov, r2, out_signs=S1, out_const=K, out=s1)
        ke("mnie,mne->i", self.Wooov, r2, out_signs=S1, out_const=K, out=s1, alpha=-0.5)

        s2 = ke("maij,m->ija", self.Wovoo, r1, out_signs=S2, out_const=K, alpha=-1.0)
        ke("ae,ije->ija", self.Fvv, r2, out_signs=S2, out_const=K, out=s2)
        x1 = ke("mi,mja->ija", self.Foo, r2, out_signs=S2, out_const=K)
        s2 = s2 - x1 + permute("ija->jia", x1)
        ke("mnij,mna->ija", self.Woooo, r2, out_signs=S2, out_const=K, out=s2, alpha=0.5)
        x2 = ke("maei,mje->ija", self.Wovvo, r2, out_signs=S2, out_const=K)
        s2 = s2 + x2 - permute("ija->jia", x2)
        X = ke("mnef,mnf->e", self.Woovv, r2, out_signs=S1, out_const=K)
        ke("e,ijae->ija", X, self.t2, out_signs=S2, out_const=K, out=s2, alpha=0.5)
        return self.join(s1, s2)

    def sigma_ea(self, K, x):
        r1, r2 = self.split("ea", K, x)
        ke = keinsum
        S1 = (1,)
        S2 = (-1, 1, 1)
        s1 = ke("ac,c->a", self.Fvv, r1, out_signs=S1, out_const=K)
        ke("ld,lad->a", self.Fov, r2, out_signs=S1, out_const=K, out=s1)
        ke("alcd,lcd->a", self.Wvovv, r2, out_signs=S1, out_const=K, out=s1, alpha=0.5)

        s2 = ke("abej,e->jab", self.Wvvvo, r1, out_signs=S2, out_const=K)
        x1 = ke("bd,iad->iab", self.Fvv, r2, out_signs=S2, out_const=K)
        s2 = s2 + x1 - permute("iab->iba", x1)
        ke("li,lab->iab", self.Foo, r2, out_signs=S2, out_const=K, out=s2, alpha=-1.0)
        ke("abcd,icd->iab", self.Wvvvv, r2, out_signs=S2, out_const=K, out=s2, alpha=0.5)
        x2 = ke("lbdi,lad->iab", self.Wovvo, r2, out_signs=S2, out_const=K)
        s2 = s2 + x2 - permute("iab->iba", x2)
        Y = ke("klcd,lcd->k", self.Woovv, r2, out_signs=S1, out_const=K)
        ke("k,kiab->iab", Y, self.t2, out_signs=S2, out_const=K, out=s2, alpha=-0.5)
        return self.join(s1, s2)

    def sigma(self, part, K, x):
        return self.sigma_ip(K, x) if part == "ip" else self.sigma_ea(K, x)

    def reduced_terms_abs(self, part, K, x):
        """Elementwise sum of |operand| |r| over the sigma terms that the mixed forms take
        as reduced-precision products, as a real full vector (zero on the one-quasiparticle
        part, which stays in FP64): EA 1/2 W_abcd r_i^cd and (W_lbdi r_l^ad + F_bd r_i^ad)
        taken before the (a, b) antisymmetriser, so that both of its images count; IP
        1/2 W_mnij r_mn^a and W_maei r_mj^e likewise over (i, j).  The rounding error of a
        product sum_k A_k B_k is at most a small multiple of sum_k |A_k| |B_k|, so a
        multiple of this vector bounds those products' error elementwise a priori."""
        r1, r2 = self.split(part, K, x)
        ab = lambda t: t.like(np.abs(t.data))
        ke = keinsum
        if part == "ea":
            S2 = (-1, 1, 1)
            b = ke("abcd,icd->iab", ab(self.Wvvvv), ab(r2), out_signs=S2, out_const=K, alpha=0.5)
            x2 = ke("lbdi,lad->iab", ab(self.Wovvo), ab(r2), out_signs=S2, out_const=K)
            ke("bd,iad->iab", ab(self.Fvv), ab(r2), out_signs=S2, out_const=K, out=x2)
            b = b + x2 + permute("iab->iba", x2)
        else:
            S2 = (1, 1, -1)
            b = ke("mnij,mna->ija", ab(self.Woooo), ab(r2), out_signs=S2, out_const=K, alpha=0.5)
            x2 = ke("maei,mje->ija", ab(self.Wovvo), ab(r2), out_signs=S2, out_const=K)
            b = b + x2 + permute("ija->jia", x2)
        return np.concatenate([np.zeros(r1.data.size), b.data.real.ravel()])

    # ---------------------------------------------------------- diagonal
    def diag(self, part, K):
        """Diagonal of M from the one-body blocks (the preconditioner D)."""
        m = self.mesh
        foo = np.array([np.diag(self.Foo.data[k]) for k in range(self.nk)])
        fvv = np.array([np.diag(self.Fvv.data[k]) for k in range(self.nk)])
        if part == "ip":
            d1 = -foo[K]
            d2 = np.zeros(self.ip_shapes()[1], complex)
            for ki, kj in itertools.product(range(self.nk), repeat=2):
                ka = m.lin([(1, ki), (1, kj), (-1, K)])
                d2[ki, kj] = (fvv[ka][None, None, :] - foo[ki][:, None, None] - foo[kj][None, :, None])
        else:
            d1 = fvv[K].copy()
            d2 = np.zeros(self.ea_shapes()[1], complex)
            for ki, ka in itertools.product(range(self.nk), repeat=2):
                kb = m.lin([(1, K), (1, ki), (-1, ka)])
                d2[ki, ka] = (fvv[ka][None, :, None] + fvv[kb][None, None, :] - foo[ki][:, None, None])
        return np.concatenate([d1.ravel(), d2.ravel()])

    # ------------------------------------------------ b and e vectors (C6)
    def _kslice(self, x: KT, pos: int, orb: int, kval: int) -> KT:
        """Fix index ``pos`` of a block tensor at (orbital, momentum)."""
        m = self.mesh
        nk = self.nk
        r = x.rank
        signs = tuple(s for i, s in enumerate(x.signs) if i != pos)
        const = m.lin([(1, x.const), (-x.signs[pos], kval)])
        shp = [nk] * (r - 2) + [d for i, d in enumerate(x.orb_shape) if i != pos]
        out = KT(m, np.zeros(shp, complex), signs, const)
        for ks in itertools.product(range(nk), repeat=r - 1):
            full = list(ks) + [x.implied(ks)]
            if full[pos] != kval:
                continue
            rest = [k for i, k in enumerate(full) if i != pos]
            idx = [slice(None)] * r
            idx[pos] = orb
            out.data[tuple(rest[: r - 2])] = x.block(ks)[tuple(idx)]
        return out

    def b_vector(self, part, K, p):
        no = self.no
        t1, t2 = self.t1, self.t2
        if part == "ip":
            r1, r2 = self.vec_kt("ip", K)
            if p < no:
                r1.data[p] = 1.0
            else:
                c = p - no
                r1.data[:] = t1.data[K][:, c]
                tc = self._kslice(t2, 3, c, K)          # (k,l,a), kk+kl-ka = K
                r2.data[:] = -tc.data
        else:
            r1, r2 = self.vec_kt("ea", K)
            if p >= no:
                r1.data[p - no] = 1.0
            else:
                k0 = p
                r1.data[:] = -t1.data[K][k0, :]
                tk = self._kslice(t2, 0, k0, K)         # (l,a,b), kl-ka-kb = -K
                r2.data[:] = -tk.data
        return self.join(r1, r2)

    def e_vector(self, part, K, q):
        no = self.no
        t1, l1, l2 = self.t1, self.l1, self.l2
        ke = keinsum
        if part == "ip":
            e1, e2 = self.vec_kt("ip", K)
            if q >= no:
                b = q - no
                e1.data[:] = l1.data[K][:, b]
                lb = self._kslice(l2, 2, b, K)          # (i,j,a): ki+kj-ka = K
                e2.data[:] = lb.data
            else:
                k0 = q
                e1.data[k0] += 1.0
                e1.data[:] -= l1.data[K] @ t1.data[K][k0, :]
                tk = self._kslice(self.t2, 0, k0, K)     # t_{k0 l}^{cd}: (l,c,d)
                ke("lcd,ilcd->i", tk, l2, out_signs=(1,), out_const=K, out=e1, alpha=-0.5)
                m = self.mesh
                for ki, kj in itertools.product(range(self.nk), repeat=2):
                    ka = m.lin([(1, ki), (1, kj), (-1, K)])
                    if ki == K:
                        e2.data[ki, kj][k0, :, :] += l1.data[kj]        # lambda_a^j
                    if kj == K:
                        e2.data[ki, kj][:, k0, :] -= l1.data[ki]        # lambda_a^i
                # - sum_c t_{k0}^c lambda_{ca}^{ij}, c at momentum K
                for c in range(self.nv):
                    lc = self._kslice(l2, 2, c, K)
                    e2.data[:] -= t1.data[K][k0, c] * lc.data
            return self.join(e1, e2)
        else:
            e1, e2 = self.vec_kt("ea", K)
            if q < no:
                i0 = q
                e1.data[:] = -l1.data[K][i0, :]
                li = self._kslice(l2, 1, i0, K)          # lambda_ab^{j i0}: (j,a,b)
                e2.data[:] = li.data
            else:
                c0 = q - no
                e1.data[c0] += 1.0
                e1.data[:] -= t1.data[K][:, c0] @ l1.data[K]
                tc = self._kslice(self.t2, 3, c0, K)     # t_kl^{d c0}: (k,l,d)
                ke("kld,klda->a", tc, l2, out_signs=(1,), out_const=K, out=e1, alpha=-0.5)
                m = self.mesh
                for ki, ka in itertools.product(range(self.nk), repeat=2):
                    kb = m.lin([(1, K), (1, ki), (-1, ka)])
                    if ka == K:
                        e2.data[ki, ka][:, c0, :] += l1.data[ki]        # lambda_b^i
                    if kb == K:
                        e2.data[ki, ka][:, :, c0] -= l1.data[ki]        # lambda_a^i
                for j in range(no):
                    lj = self._kslice(l2, 1, j, K)                       # lambda_ab^{i j}
                    e2.data[:] += t1.data[K][j, c0] * lj.data
            return self.join(e1, e2)

    # ------------------------------------------------ unique-coefficient maps
    def unique_index(self, part, K):
        """Flat full-storage positions of the unique coefficients (i<j or a<b by
        combined (k, p) index) in the brute-force ordering, plus the positions of
        their antisymmetric partners."""
        no, nv, nk = self.no, self.nv, self.nk
        m = self.mesh
        s1, s2 = self.ip_shapes() if part == "ip" else self.ea_shapes()
        n1 = int(np.prod(s1))
        idx2 = np.arange(int(np.prod(s2))).reshape(s2) + n1
        pos, partner = list(range(n1)), list(range(n1))
        if part == "ip":
            for I, J in itertools.combinations(range(nk * no), 2):
                ki, i = divmod(I, no)
                kj, j = divmod(J, no)
                for a in range(nv):
                    pos.append(idx2[ki, kj, i, j, a])
                    partner.append(idx2[kj, ki, j, i, a])
        else:
            for ki in range(nk):
                for i in range(no):
                    for A, B in itertools.combinations(range(nk * nv), 2):
                        ka, a = divmod(A, nv)
                        kb, b = divmod(B, nv)
                        if m.lin([(1, K), (1, ki), (-1, ka)]) != kb:
                            continue
                        pos.append(idx2[ki, ka, i, a, b])
                        partner.append(idx2[ki, kb, i, b, a])
        return np.array(pos), np.array(partner), n1

    def pack(self, part, K, x):
        pos, _, _ = self.unique_index(part, K)
        return x[pos]

    def unpack(self, part, K, u):
        pos, partner, n1 = self.unique_index(part, K)
        x = np.zeros(self.size(part), complex)
        x[pos] = u
        x[partner[n1:]] = -u[n1:]
        return x

    def dense_matrix(self, part, K):
        """M in the unique basis, column by column from sigma."""
        pos, partner, n1 = self.unique_index(part, K)
        n = len(pos)
        M = np.zeros((n, n), complex)
        for c in range(n):
            u = np.zeros(n, complex)
            u[c] = 1.0
            M[:, c] = self.pack(part, K, self.sigma(part, K, self.unpack(part, K, u)))
        return M
