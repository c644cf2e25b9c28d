"""O3: Bloch k-blocks -> Gamma-point supercell (test infrastructure).

The k-point CCGF is checked against a supercell (molecular) calculation in the
paper's Supporting Information (Sec. I, diamond on a 3x1x1 mesh).  With
Lambda = T^dagger on both sides the two must agree to rounding, which pins all
momentum bookkeeping of Eq. 9.

Bloch orbital psi_{k p} = sum_R U[(R,p),(k,p)] phi_{R p} with
U = exp(i k.R) / sqrt(Nk), applied separately to the occupied and the virtual
orbitals (supercell ordering: all occupied (R, i) R-major, then all virtual).
Integrals transform with U on bra (creation) indices and conj(U) on ket
(annihilation) indices; G^Bloch = U^dagger G^supercell U.

Parity: pinned by the Nk = 2 and Nk = 3 supercell identities and by the
vanishing of the momentum-off-diagonal blocks of U^dagger G U
(tests/test_oracle_unfold.py).
"""
from __future__ import annotations

import itertools
import types

import numpy as np

from .ktensor import KMesh


def bloch_unitary(mesh: KMesh, norb: int) -> np.ndarray:
    """U[(R, p), (k, p)] = exp(2 pi i n_k . r_R / m) / sqrt(Nk)."""
    nk = mesh.nk
    m = np.array(mesh.m, dtype=float)
    U = np.zeros((nk * norb, nk * norb), dtype=np.complex128)
    for R in range(nk):
        for k in range(nk):
            ph = np.exp(2j * np.pi * np.sum(mesh.pts[k] * mesh.pts[R] / m)) / np.sqrt(nk)
            for p in range(norb):
                U[R * norb + p, k * norb + p] = ph
    return U


def unfold(sys):
    """Return (supercell system at one k-point, v_full, foo, fvv, Uo, Uv)."""
    mesh = KMesh(sys.kmesh)
    nk = mesh.nk
    no, nv = sys.nocc, sys.nvir
    nmo = no + nv
    # dense Bloch-basis antisymmetrised integrals over all (k, p)
    A = sys.eri_factor
    NO, NV = nk * no, nk * nv
    N = NO + NV

    def gidx(k, p):  # supercell-style ordering of Bloch orbitals: occ block then vir block
        return k * no + p if p < no else NO + k * nv + (p - no)

    VB = np.zeros((N, N, N, N), dtype=np.complex128)
    for k1, k2, k3 in itertools.product(range(nk), repeat=3):
        k4 = mesh.lin([(1, k1), (1, k2), (-1, k3)])
        d = np.einsum("Lpr,Lqs->pqrs", A[k1, k3], A[k2, k4])
        x = np.einsum("Lps,Lqr->pqrs", A[k1, k4], A[k2, k3])
        blk = d - x
        i1 = [gidx(k1, p) for p in range(nmo)]
        i2 = [gidx(k2, p) for p in range(nmo)]
        i3 = [gidx(k3, p) for p in range(nmo)]
        i4 = [gidx(k4, p) for p in range(nmo)]
        VB[np.ix_(i1, i2, i3, i4)] = blk
    FB = np.zeros((N, N), dtype=np.complex128)
    for k in range(nk):
        ii = [gidx(k, p) for p in range(nmo)]
        if getattr(sys, "foo", None) is not None:
            FB[np.ix_(ii[:no], ii[:no])] = sys.foo[k]
            FB[np.ix_(ii[no:], ii[no:])] = sys.fvv[k]
        else:
            FB[np.ix_(ii, ii)] = np.diag(sys.eps[k])
    T1B = np.zeros((NO, NV), dtype=np.complex128)
    for k in range(nk):
        T1B[k * no:(k + 1) * no, k * nv:(k + 1) * nv] = sys.t1[k]
    T2B = np.zeros((NO, NO, NV, NV), dtype=np.complex128)
    for ki, kj, ka in itertools.product(range(nk), repeat=3):
        kb = mesh.lin([(1, ki), (1, kj), (-1, ka)])
        T2B[ki * no:(ki + 1) * no, kj * no:(kj + 1) * no,
            ka * nv:(ka + 1) * nv, kb * nv:(kb + 1) * nv] = sys.t2[ki, kj, ka]
    Uo = bloch_unitary(mesh, no)
    Uv = bloch_unitary(mesh, nv)
    U = np.zeros((N, N), dtype=np.complex128)
    U[:NO, :NO] = Uo
    U[NO:, NO:] = Uv
    Uc = U.conj()
    VL = np.einsum("Pp,Qq,pqrs,Rr,Ss->PQRS", U, U, VB, Uc, Uc, optimize=True)
    FL = U @ FB @ U.conj().T
    T1L = np.einsum("Ii,ia,Aa->IA", Uo.conj(), T1B, Uv, optimize=True)
    T2L = np.einsum("Ii,Jj,ijab,Aa,Bb->IJAB", Uo.conj(), Uo.conj(), T2B, Uv, Uv, optimize=True)
    sc = types.SimpleNamespace(kmesh=(1, 1, 1), nocc=NO, nvir=NV, eps=None, eri_factor=None,
                               t1=T1L[None], t2=T2L[None, None, None])
    return sc, VL, FL[:NO, :NO], FL[NO:, NO:], U


def bloch_index(mesh: KMesh, no: int, nv: int, k: int, p: int) -> int:
    """Position of Bloch orbital (k, p) in the supercell-ordered basis."""
    nk = mesh.nk
    return k * no + p if p < no else nk * no + k * nv + (p - no)
