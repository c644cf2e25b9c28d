"""Momentum-blocked tensors and a k-conserving einsum (test infrastructure).

In the Bloch basis every orbital index p carries a crystal momentum k_p and a
tensor element is nonzero only if the momenta of its indices satisfy a linear
conservation law (Eq. 9 and the momentum-conserving k-blocks of the periodic
formulation).  A ``KT`` stores only the allowed blocks:

    sum_x  s_x * k_x  =  c          (s_x = +1 / -1, c a k-point)

with the first (rank - 1) momenta as leading array axes and the last one
implied by the law.  Two-electron integrals and doubles use (+,+,-,-) with
c = 0; one-body quantities and singles are k-diagonal (+,-); an EOM vector of
total momentum K uses c = K.

``keinsum`` evaluates an einsum over such tensors by enumerating every
momentum assignment allowed by all operands' laws and contracting the dense
orbital blocks with numpy.  A single-k mesh reduces it to plain einsum, which
is the molecular (supercell) case.

Parity: the enumeration is pinned against dense Bloch-basis einsum with
explicit zero blocks (tests/test_oracle_ktensor.py).
"""
from __future__ import annotations

import itertools
from typing import Dict, Sequence, Tuple

import numpy as np


class KMesh:
    """Gamma-centred integer mesh with modular momentum arithmetic."""

    def __init__(self, kmesh: Sequence[int]):
        self.m = tuple(int(x) for x in kmesh)
        m1, m2, m3 = self.m
        self.pts = np.array([(a, b, c) for a in range(m1) for b in range(m2) for c in range(m3)])
        self.nk = len(self.pts)
        nk = self.nk
        self.add = np.zeros((nk, nk), dtype=np.int64)
        self.neg = np.zeros(nk, dtype=np.int64)
        for i in range(nk):
            self.neg[i] = self.flat(-self.pts[i])
            for j in range(nk):
                self.add[i, j] = self.flat(self.pts[i] + self.pts[j])

    def flat(self, n) -> int:
        m1, m2, m3 = self.m
        return int((n[0] % m1) * m2 * m3 + (n[1] % m2) * m3 + (n[2] % m3))

    def lin(self, terms) -> int:
        """sum of s*k over (s, k) pairs, s = +-1."""
        acc = 0
        for s, k in terms:
            acc = self.add[acc, k if s > 0 else self.neg[k]]
        return int(acc)


class KT:
    """Block tensor: data[k_0, ..., k_{r-2}, orbital axes...]; last k implied."""

    def __init__(self, mesh: KMesh, data: np.ndarray, signs: Tuple[int, ...], const: int = 0):
        self.mesh = mesh
        self.signs = tuple(int(s) for s in signs)
        self.const = int(const)
        self.rank = len(self.signs)
        self.data = data
        assert data.ndim == 2 * self.rank - 1, (data.shape, signs)

    @property
    def orb_shape(self):
        return self.data.shape[self.rank - 1:]

    def implied(self, ks) -> int:
        """Momentum of the last index given the leading ones."""
        m = self.mesh
        rest = m.lin([(-s, k) for s, k in zip(self.signs[:-1], ks)] + [(1, self.const)])
        return int(rest if self.signs[-1] > 0 else m.neg[rest])

    def block(self, ks):
        return self.data[tuple(ks[: self.rank - 1])]

    def like(self, data=None):
        return KT(self.mesh, np.zeros_like(self.data) if data is None else data, self.signs, self.const)

    def __add__(self, o):
        self._check(o)
        return self.like(self.data + o.data)

    def __sub__(self, o):
        self._check(o)
        return self.like(self.data - o.data)

    def __neg__(self):
        return self.like(-self.data)

    def __mul__(self, c):
        return self.like(self.data * c)

    __rmul__ = __mul__

    def _check(self, o):
        assert self.signs == o.signs and self.const == o.const and self.data.shape == o.data.shape

    def copy(self):
        return self.like(self.data.copy())


def _plan(letters, laws):
    """Order letters into free ones and ones fixed by a law; returns a list of
    (letter, law-or-None).  A law is (list of (sign, letter)), const)."""
    placed = set()
    order = []
    pending = list(letters)
    while pending:
        progress = True
        while progress:
            progress = False
            for terms, const in laws:
                unplaced = [l for _, l in terms if l not in placed]
                if len(set(unplaced)) == 1:
                    l = unplaced[0]
                    order.append((l, (terms, const)))
                    placed.add(l)
                    pending.remove(l)
                    progress = True
        if pending:
            l = pending[0]
            order.append((l, None))
            placed.add(l)
            pending.remove(l)
    return order


def keinsum(spec: str, *ops: KT, out_signs, out_const: int = 0, fixed: Dict[str, int] = None,
            out: KT = None, alpha=1.0) -> KT:
    """k-conserving einsum.  ``spec`` is a plain einsum string over orbital
    letters; each letter also carries a momentum.  ``fixed`` pins momenta of
    chosen letters (to compute selected output blocks only)."""
    ins, outl = spec.replace(" ", "").split("->")
    ins = ins.split(",")
    assert len(ins) == len(ops)
    mesh = ops[0].mesh
    letters = []
    for s in ins + [outl]:
        for ch in s:
            if ch not in letters:
                letters.append(ch)
    laws = []
    for s, op in zip(ins, ops):
        assert len(s) == op.rank
        laws.append(([(sg, ch) for sg, ch in zip(op.signs, s)], op.const))
    fixed = dict(fixed or {})
    plan = _plan([l for l in letters if l not in fixed], [
        ([(sg, ch) for sg, ch in terms], c) for terms, c in laws
    ] if not fixed else _reduce_laws(laws, fixed, mesh))
    out_rank = len(outl)
    if out is None:
        oshape = [mesh.nk] * (out_rank - 1)
        dims = {}
        for s, op in zip(ins, ops):
            for ch, d in zip(s, op.orb_shape):
                dims[ch] = d
        oshape += [dims[ch] for ch in outl]
        out = KT(mesh, np.zeros(oshape, dtype=np.complex128), out_signs, out_const)
    free = [l for l, law in plan if law is None]
    path_cache = {}
    for vals in itertools.product(range(mesh.nk), repeat=len(free)):
        kv = dict(fixed)
        it = iter(vals)
        for l, law in plan:
            if law is None:
                kv[l] = next(it)
            else:
                terms, c = law
                # s_l k_l = c - sum_{others} s k
                acc = [(1, c)] + [(-sg, kv[ch]) for sg, ch in terms if ch != l]
                sl = sum(sg for sg, ch in terms if ch == l)
                r = mesh.lin(acc)
                kv[l] = r if sl > 0 else int(mesh.neg[r])
        ok = True
        for terms, c in laws:
            if mesh.lin([(sg, kv[ch]) for sg, ch in terms]) != c:
                ok = False
                break
        if not ok:
            continue
        # output law must hold automatically
        assert mesh.lin([(sg, kv[ch]) for sg, ch in zip(out.signs, outl)]) == out.const
        blocks = [op.block([kv[ch] for ch in s]) for s, op in zip(ins, ops)]
        key = tuple(b.shape for b in blocks)
        if key not in path_cache:
            path_cache[key] = np.einsum_path(spec, *blocks, optimize="optimal")[0]
        res = np.einsum(spec, *blocks, optimize=path_cache[key])
        idx = tuple(kv[ch] for ch in outl[:-1])
        out.data[idx] += alpha * res
    return out


def _reduce_laws(laws, fixed, mesh):
    # laws stay the same; fixed letters are treated as already placed by _plan
    red = []
    for terms, c in laws:
        t2 = [(sg, ch) for sg, ch in terms if ch not in fixed]
        c2 = mesh.lin([(1, c)] + [(-sg, fixed[ch]) for sg, ch in terms if ch in fixed])
        if t2:
            red.append((t2, c2))
    return red


def permute(spec: str, x: KT, out_signs=None, out_const=None) -> KT:
    """Index permutation, e.g. permute('pqrs->pqsr', x)."""
    ins, outl = spec.split("->")
    if out_signs is None:
        sg = dict(zip(ins, x.signs))
        out_signs = tuple(sg[ch] for ch in outl)
    return keinsum(spec, x, out_signs=out_signs, out_const=x.const if out_const is None else out_const)


def to_dense(x: KT, offsets: Sequence[Sequence[int]] = None) -> np.ndarray:
    """Dense Bloch-basis array with combined (k, p) indices (k-major)."""
    mesh = x.mesh
    nk = mesh.nk
    osh = x.orb_shape
    D = np.zeros([nk * d for d in osh], dtype=np.complex128)
    for ks in itertools.product(range(nk), repeat=x.rank - 1):
        kl = x.implied(ks)
        kk = list(ks) + [kl]
        sl = tuple(slice(k * d, (k + 1) * d) for k, d in zip(kk, osh))
        D[sl] = x.block(ks)
    return D


def from_dense(mesh: KMesh, D: np.ndarray, osh, signs, const=0) -> KT:
    nk = mesh.nk
    r = len(osh)
    data = np.zeros([nk] * (r - 1) + list(osh), dtype=np.complex128)
    x = KT(mesh, data, signs, const)
    for ks in itertools.product(range(nk), repeat=r - 1):
        kl = x.implied(ks)
        kk = list(ks) + [kl]
        sl = tuple(slice(k * d, (k + 1) * d) for k, d in zip(kk, osh))
        data[ks] = D[sl]
    return x
