"""Seeded synthetic inputs shaped like the periodic CCGF workloads.

Everything here is input generation only: orbital energies, a momentum-blocked
low-rank two-electron factor and antisymmetric cluster amplitudes, each drawn
from a seeded, block-addressable stream so that any k-block can be regenerated
on its own.  Nothing in this module evaluates the Green's-function method; the
CPU oracle and the HIP path both take their inputs from here and from nowhere
else.

Conventions of the produced arrays (spin orbitals, occupied first):

* ``kmesh`` is a Gamma-centred integer mesh (m1, m2, m3); a k-point is the
  integer triple n with k = n / m, flattened as n1*m2*m3 + n2*m3 + n3.
* ``eps[k, p]``: real orbital energies, sorted within occupied and virtual.
* ``eri_factor[k1, k3, L, p, r]``: complex factor A with
  A[k3, k1, L, r, p] = conj(A[k1, k3, L, p, r]).  The physicists' integral of
  four Bloch spin orbitals is <p k1, q k2 | r k3, s k4> = sum_L
  A[k1, k3, L, p, r] * A[k2, k4, L, q, s] for k4 = k1 + k2 - k3 (and zero
  otherwise); this is Hermitian, symmetric under particle exchange and positive
  semidefinite, and real with 8-fold symmetry when nk = 1 and the factor is
  real.
* ``t1[k, i, a]``: singles (k_i = k_a = k).
* ``t2[ki, kj, ka, i, j, a, b]`` with kb = ki + kj - ka, antisymmetric in
  (i,ki)<->(j,kj) and in (a,ka)<->(b,kb).

Two-body k-blocks carry the usual 1/Nk normalisation of Bloch-basis integrals
(``knorm="1/Nk"``): the requested standard deviation is divided by Nk.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

BASE_SEED = 220807478

# tensor ids for the block-addressable streams
TID_EPS = 1
TID_ERI = 2
TID_T1 = 3
TID_T2 = 4
TID_VEC = 5
TID_ROT = 6
TID_MISC = 7
TID_LAM1 = 8
TID_LAM2 = 9


def _rng(seed: int, tid: int, *block: int) -> np.random.Generator:
    """Independent Philox stream keyed by (seed, tensor id, block index)."""
    ss = np.random.SeedSequence([int(seed) & 0xFFFFFFFF, int(tid)] + [int(b) for b in block])
    return np.random.Generator(np.random.Philox(ss))


def _cnormal(rng: np.random.Generator, shape, std: float, real: bool) -> np.ndarray:
    """Complex Gaussian with E|z|^2 = std^2 (Re, Im ~ N(0, std^2/2)); real if asked."""
    if real:
        return rng.normal(0.0, std, size=shape).astype(np.complex128)
    s = std / np.sqrt(2.0)
    return rng.normal(0.0, s, size=shape) + 1j * rng.normal(0.0, s, size=shape)


def kmesh_points(kmesh: Sequence[int]) -> np.ndarray:
    """Integer triples of the mesh in flattened order, shape [nk, 3]."""
    m1, m2, m3 = kmesh
    return np.array([(a, b, c) for a in range(m1) for b in range(m2) for c in range(m3)], dtype=np.int64)


def _kflat(n: np.ndarray, kmesh: Sequence[int]) -> int:
    m1, m2, m3 = kmesh
    return int((n[0] % m1) * m2 * m3 + (n[1] % m2) * m3 + (n[2] % m3))


def _ksum_table(kmesh: Sequence[int]) -> np.ndarray:
    """tab[k1, k2, k3] = flat index of k1 + k2 - k3 (mod the mesh)."""
    pts = kmesh_points(kmesh)
    nk = len(pts)
    tab = np.zeros((nk, nk, nk), dtype=np.int64)
    for a in range(nk):
        for b in range(nk):
            for c in range(nk):
                tab[a, b, c] = _kflat(pts[a] + pts[b] - pts[c], kmesh)
    return tab


@dataclasses.dataclass
class System:
    """One synthetic periodic system (all two-body data as k-blocks)."""

    kmesh: tuple
    nocc: int
    nvir: int
    eps: np.ndarray
    eri_factor: np.ndarray
    t1: np.ndarray
    t2: np.ndarray
    foo: Optional[np.ndarray] = None
    fvv: Optional[np.ndarray] = None
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def nk(self) -> int:
        return int(np.prod(self.kmesh))

    @property
    def nmo(self) -> int:
        return self.nocc + self.nvir

    @property
    def naux(self) -> int:
        return int(self.eri_factor.shape[2])


def make_system(kmesh=(1, 1, 1), nocc=2, nvir=6, *, seed=BASE_SEED, naux=None,
                eri_std=0.05, t1_std=0.01, t2_std=0.02, knorm="1/Nk",
                eps_occ=(-1.0, -0.3), eps_vir=(0.2, 2.0), real=False,
                zero_t1=False, zero_t2=False, zero_eri=False) -> System:
    """Build a seeded synthetic system.

    ``real=True`` (only meaningful for nk = 1) draws a real symmetric factor and
    real amplitudes, which gives real ERIs with 8-fold symmetry.
    """
    kmesh = tuple(int(x) for x in kmesh)
    nk = int(np.prod(kmesh))
    nmo = nocc + nvir
    if naux is None:
        naux = 2 * nmo
    if real and nk != 1:
        raise ValueError("real data only for a single k-point")
    scale = (1.0 / nk) if knorm == "1/Nk" else 1.0

    # orbital energies, sorted within the occupied and the virtual block
    eps = np.zeros((nk, nmo))
    for k in range(nk):
        r = _rng(seed, TID_EPS, k)
        eo = np.sort(r.uniform(eps_occ[0], eps_occ[1], size=nocc))
        ev = np.sort(r.uniform(eps_vir[0], eps_vir[1], size=nvir))
        eps[k, :nocc] = eo
        eps[k, nocc:] = ev

    # low-rank factor A[k1, k3, L, p, r], Hermitian under (k1,p) <-> (k3,r)
    target = eri_std * scale
    s = np.sqrt(target / np.sqrt(naux))
    A = np.zeros((nk, nk, naux, nmo, nmo), dtype=np.complex128)
    for k1 in range(nk):
        for k3 in range(k1, nk):
            r = _rng(seed, TID_ERI, k1, k3)
            Z = _cnormal(r, (naux, nmo, nmo), s, real)
            if k1 == k3:
                Z = (Z + np.conj(Z.transpose(0, 2, 1))) / np.sqrt(2.0)
                A[k1, k1] = Z
            else:
                A[k1, k3] = Z
                A[k3, k1] = np.conj(Z.transpose(0, 2, 1))
    if zero_eri:
        A[:] = 0

    t1 = np.zeros((nk, nocc, nvir), dtype=np.complex128)
    if not zero_t1:
        for k in range(nk):
            t1[k] = _cnormal(_rng(seed, TID_T1, k), (nocc, nvir), t1_std, real)

    if zero_t2:
        t2 = np.zeros((nk, nk, nk, nocc, nocc, nvir, nvir), dtype=np.complex128)
    else:
        t2 = _doubles(kmesh, nocc, nvir, seed, TID_T2, t2_std * scale, real)
    meta = dict(seed=seed, eri_std=eri_std, t1_std=t1_std, t2_std=t2_std, knorm=knorm,
                naux=naux, real=real)
    return System(kmesh=kmesh, nocc=nocc, nvir=nvir, eps=eps, eri_factor=A, t1=t1, t2=t2,
                  meta=meta)


def _doubles(kmesh, nocc, nvir, seed, tid, std, real):
    """Seeded doubles amplitudes [ki][kj][ka][i][j][a][b] (kb = ki + kj - ka),
    antisymmetric under (i,ki)<->(j,kj) and (a,ka)<->(b,kb)."""
    nk = int(np.prod(kmesh))
    out = np.zeros((nk, nk, nk, nocc, nocc, nvir, nvir), dtype=np.complex128)
    tab = _ksum_table(kmesh)
    raw = {}

    def blk(ki, kj, ka):
        key = (ki, kj, ka)
        if key not in raw:
            raw[key] = _cnormal(_rng(seed, tid, ki, kj, ka), (nocc, nocc, nvir, nvir), std, real)
        return raw[key]

    for ki in range(nk):
        for kj in range(nk):
            for ka in range(nk):
                kb = tab[ki, kj, ka]
                x = (blk(ki, kj, ka)
                     - blk(kj, ki, ka).transpose(1, 0, 2, 3)
                     - blk(ki, kj, kb).transpose(0, 1, 3, 2)
                     + blk(kj, ki, kb).transpose(1, 0, 3, 2))
                out[ki, kj, ka] = 0.5 * x
    return out


def make_lambda(kmesh, nocc, nvir, *, seed=BASE_SEED, l1_std=0.01, l2_std=0.02, knorm="1/Nk", real=False):
    """Seeded Lambda amplitudes (l1[k][i][a], l2 like t2), independent of T: a
    stand-in for solved k-point Lambda equations, which the inputs here do not have."""
    kmesh = tuple(int(x) for x in kmesh)
    nk = int(np.prod(kmesh))
    scale = (1.0 / nk) if knorm == "1/Nk" else 1.0
    l1 = np.zeros((nk, nocc, nvir), dtype=np.complex128)
    for k in range(nk):
        l1[k] = _cnormal(_rng(seed, TID_LAM1, k), (nocc, nvir), l1_std, real)
    l2 = _doubles(kmesh, nocc, nvir, seed, TID_LAM2, l2_std * scale, real)
    return l1, l2


def random_vectors(n: int, nvec: int, *, seed=BASE_SEED, tid=TID_VEC, std=1.0) -> np.ndarray:
    """nvec complex Gaussian vectors of length n (no structure imposed)."""
    return _cnormal(_rng(seed, tid, n, nvec), (nvec, n), std, False)


def random_unitary(n: int, *, seed=BASE_SEED, block=0) -> np.ndarray:
    """Haar-like random unitary from the QR of a complex Gaussian matrix."""
    z = _cnormal(_rng(seed, TID_ROT, n, block), (n, n), 1.0, False)
    q, r = np.linalg.qr(z)
    d = np.diag(r)
    return q * (d / np.abs(d))


# ----------------------------------------------------------------------------
# Workload presets.  Shapes and distributions follow the Si-like and ZnO-like
# workloads (2x2x2 / 3x3x3 meshes, 4+26 and 9+40 spin orbitals per cell); the
# real crystals' integrals are not available, so these seeded stand-ins are
# used throughout.
# ----------------------------------------------------------------------------

PRESETS = {
    # Gamma only, 2 occupied + 6 virtual spin orbitals, real 8-fold ERIs
    "gamma_2o6v": dict(kmesh=(1, 1, 1), nocc=2, nvir=6, eri_std=0.05, t1_std=0.01,
                       t2_std=0.02, naux=16, real=True, eta=0.01,
                       omega=(-1.0, 1.0, 16), cfg=0),
    # Si-like 2x2x2 mesh, 4 + 26 spin orbitals per cell
    "si_k222": dict(kmesh=(2, 2, 2), nocc=4, nvir=26, eri_std=0.05, t1_std=0.01,
                    t2_std=0.01, eta=0.005, omega=(-1.0, 1.0, 64), cfg=1),
    # Si-like 3x3x3 mesh
    "si_k333": dict(kmesh=(3, 3, 3), nocc=4, nvir=26, eri_std=0.05, t1_std=0.01,
                    t2_std=0.01, eta=0.005, omega=(-1.0, 1.0, 256), cfg=2),
    # ZnO-like 3x3x3 mesh, 9 + 40 spin orbitals per cell, narrow deep band
    "zno_k333": dict(kmesh=(3, 3, 3), nocc=9, nvir=40, eri_std=0.03, t1_std=0.01,
                     t2_std=0.01, eta=0.005, omega=(-1.5, 1.5, 1000), eps_occ=(-0.8, -0.6),
                     cfg=4),
}


def preset_system(name: str, **overrides) -> System:
    p = dict(PRESETS[name])
    cfg = p.pop("cfg")
    p.pop("eta")
    p.pop("omega")
    p.update(overrides)
    p.setdefault("seed", BASE_SEED + 100 * cfg)
    return make_system(**p)


def preset_query(name: str):
    """(omega grid, eta) of a preset."""
    p = PRESETS[name]
    lo, hi, n = p["omega"]
    return np.linspace(lo, hi, n), p["eta"]


def eom_vector_shapes(kmesh, nocc, nvir, part):
    """(n1, r2 shape) of an EOM vector in full antisymmetric storage:
    IP [r1[i], r2[ki][kj][i][j][a]] and EA [r1[a], r2[ki][ka][i][a][b]]."""
    nk = int(np.prod(kmesh))
    if part == "ip":
        return nocc, (nk, nk, nocc, nocc, nvir)
    return nvir, (nk, nk, nocc, nvir, nvir)


def random_eom_vectors(kmesh, nocc, nvir, part, K, nvec, *, seed=BASE_SEED):
    """nvec seeded random vectors of total momentum K, antisymmetric in the pair
    indices (IP: (i,ki)<->(j,kj); EA: (a,ka)<->(b,kb) with kb = K + ki - ka),
    flat in the layout of ``eom_vector_shapes``.  Input construction only."""
    n1, shp = eom_vector_shapes(kmesh, nocc, nvir, part)
    nk = shp[0]
    tab = _ksum_table(kmesh)
    rng = _rng(seed, TID_VEC, K, nvec, 1 if part == "ea" else 0)
    out = np.zeros((nvec, n1 + int(np.prod(shp))), dtype=np.complex128)
    for v in range(nvec):
        r1 = _cnormal(rng, (n1,), 1.0, False)
        x = _cnormal(rng, shp, 1.0, False)
        y = np.zeros_like(x)
        for k1 in range(nk):
            for k2 in range(nk):
                if part == "ip":   # partner block [kj][ki](j,i,a)
                    y[k1, k2] = (x[k1, k2] - x[k2, k1].transpose(1, 0, 2)) / np.sqrt(2.0)
                else:              # partner block [ki][kb](i,b,a), kb = K + ki - ka
                    kb = tab[K, k1, k2]
                    y[k1, k2] = (x[k1, k2] - x[k1, kb].transpose(0, 2, 1)) / np.sqrt(2.0)
        out[v, :n1] = r1
        out[v, n1:] = y.ravel()
    return out
