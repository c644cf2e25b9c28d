"""ctypes binding of libccgf.so (argument marshalling only).

Every step of the computation runs in the HIP library; this module only
converts numpy arrays / torch tensors into the pointers and sizes that the C
ABI in include/ccgf.h expects.  Importing it without the built library raises,
so nothing can silently fall back to a CPU path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libccgf.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ESTATE, EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
HOST, DEVICE = 0, 1
PART_IP, PART_EA, PART_BOTH = 1, 2, 3
PLAIN_F64, MIXED_F32, MIXED_BF16X3 = 0, 1, 2
PRECISIONS = {"f64": PLAIN_F64, "plain_f64": PLAIN_F64, "f32": MIXED_F32, "mixed_f32": MIXED_F32,
              "bf16x3": MIXED_BF16X3, "mixed_bf16x3": MIXED_BF16X3}

EXPORTS = ("cc_gf_init", "cc_gf_solve", "cc_gf_solve_matrix", "cc_gf_mor", "cc_gf_vector_size", "cc_gf_sigma",
           "cc_gf_sigma_group", "cc_gf_vectors",
           "cc_gf_learn", "cc_gf_learn_enable", "cc_gf_learn_save", "cc_gf_learn_load", "cc_gf_set_options",
           "cc_gf_mlp_grad", "cc_gf_dyson_cas",
           "cc_gf_dyson_cas_noalloc", "cc_gf_dyson_last_error", "cc_gf_free", "cc_gf_last_error")
MOR_MAX = 32


class System(ctypes.Structure):
    _fields_ = [("kmesh", ctypes.c_int * 3), ("nocc", ctypes.c_int), ("nvir", ctypes.c_int),
                ("eps", ctypes.c_void_p), ("foo", ctypes.c_void_p), ("fvv", ctypes.c_void_p),
                ("naux", ctypes.c_int), ("eri_factor", ctypes.c_void_p), ("t1", ctypes.c_void_p),
                ("t2", ctypes.c_void_p), ("mem_space", ctypes.c_int), ("l1", ctypes.c_void_p),
                ("l2", ctypes.c_void_p), ("eri_blocks", ctypes.c_void_p)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("restart_m", ctypes.c_int), ("maxiter", ctypes.c_int),
                ("tol", ctypes.c_double), ("max_batch", ctypes.c_int), ("hip_stream", ctypes.c_void_p),
                ("timing", ctypes.c_int), ("precond_eta", ctypes.c_double), ("recycle_k", ctypes.c_int),
                ("reorth_ratio", ctypes.c_double), ("autotune", ctypes.c_int),
                ("autotune_cache", ctypes.c_char_p), ("restart_tail", ctypes.c_int), ("graphs", ctypes.c_int),
                ("seed_m", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("n_solves", ctypes.c_longlong), ("n_iterations", ctypes.c_longlong),
                ("n_sigma", ctypes.c_longlong), ("max_iterations", ctypes.c_int),
                ("n_unconverged", ctypes.c_int), ("max_rel_residual", ctypes.c_double),
                ("seconds", ctypes.c_double),
                ("big_ms", ctypes.c_double), ("big_launches", ctypes.c_longlong),
                ("big_flops", ctypes.c_double), ("sigma_ms", ctypes.c_double),
                ("sigma_launches", ctypes.c_longlong), ("n_steps", ctypes.c_longlong),
                ("n_reorth", ctypes.c_longlong), ("n_guess", ctypes.c_longlong),
                ("n_guess_rejected", ctypes.c_longlong), ("big_bytes", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LearnOptions(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_double),
                ("seed", ctypes.c_ulonglong), ("hidden", ctypes.c_int), ("guess", ctypes.c_int),
                ("accept", ctypes.c_double), ("probe", ctypes.c_int)]


class LearnStats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_longlong), ("rank", ctypes.c_int), ("loss_initial", ctypes.c_double),
                ("loss_final", ctypes.c_double), ("solve_seconds", ctypes.c_double),
                ("train_seconds", ctypes.c_double), ("solve_iterations", ctypes.c_longlong),
                ("probe_seconds", ctypes.c_double), ("precond_loss_initial", ctypes.c_double),
                ("precond_loss_final", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class CCGFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"ccgf error {code}: {msg}")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2208_07478_amd.build`")
    # torch (device memory and streams) must bring in its HIP runtime first: it loads
    # libamdhip64.so by its unversioned name, so loading the library before torch would
    # leave two HIP runtimes in the process
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, ip, dp = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)
    lib.cc_gf_init.argtypes = [ctypes.POINTER(System), ctypes.POINTER(Options), ctypes.POINTER(vp)]
    lib.cc_gf_init.restype = ctypes.c_int
    lib.cc_gf_solve.argtypes = [vp, ctypes.c_int, ip, ctypes.c_int, ip, ctypes.c_int, dp, ctypes.c_double,
                                ctypes.c_int, vp, vp, vp, ctypes.POINTER(Stats)]
    lib.cc_gf_solve.restype = ctypes.c_int
    lib.cc_gf_solve_matrix.argtypes = [vp, ctypes.c_int, ip, ctypes.c_int, ip, ctypes.c_int, dp, ctypes.c_double,
                                       ctypes.c_int, vp, vp, vp, vp, ctypes.POINTER(Stats)]
    lib.cc_gf_solve_matrix.restype = ctypes.c_int
    lib.cc_gf_mor.argtypes = [vp, ctypes.c_int, ip, ctypes.c_int, ip, ctypes.c_int, dp, ctypes.c_int, dp,
                              ctypes.c_int, dp, ctypes.c_double, ctypes.c_int, vp, vp, vp, ctypes.POINTER(Stats)]
    lib.cc_gf_mor.restype = ctypes.c_int
    lib.cc_gf_vector_size.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong)]
    lib.cc_gf_vector_size.restype = ctypes.c_int
    lib.cc_gf_sigma.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp]
    lib.cc_gf_sigma.restype = ctypes.c_int
    lib.cc_gf_sigma_group.argtypes = [ctypes.c_int, ctypes.POINTER(vp), ip, ip, ip, ctypes.POINTER(vp),
                                      ctypes.POINTER(vp)]
    lib.cc_gf_sigma_group.restype = ctypes.c_int
    lib.cc_gf_vectors.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp]
    lib.cc_gf_vectors.restype = ctypes.c_int
    lib.cc_gf_learn.argtypes = [vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ctypes.c_int, dp, ctypes.c_double,
                                ctypes.POINTER(LearnOptions), ctypes.POINTER(LearnStats)]
    lib.cc_gf_learn.restype = ctypes.c_int
    lib.cc_gf_set_options.argtypes = [vp, ctypes.POINTER(Options)]
    lib.cc_gf_set_options.restype = ctypes.c_int
    lib.cc_gf_learn_enable.argtypes = [vp, ctypes.c_int]
    lib.cc_gf_learn_enable.restype = ctypes.c_int
    for fn in (lib.cc_gf_learn_save, lib.cc_gf_learn_load):
        fn.argtypes = [vp, ctypes.c_char_p]
        fn.restype = ctypes.c_int
    fp = ctypes.POINTER(ctypes.c_float)
    lib.cc_gf_mlp_grad.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, fp, ctypes.c_int, fp, fp, fp,
                                   ctypes.POINTER(ctypes.c_double)]
    lib.cc_gf_mlp_grad.restype = ctypes.c_int
    lib.cc_gf_dyson_cas.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp, vp, vp, vp, vp, vp,
                                    vp, vp]
    lib.cc_gf_dyson_cas.restype = ctypes.c_int
    lib.cc_gf_dyson_cas_noalloc.argtypes = lib.cc_gf_dyson_cas.argtypes
    lib.cc_gf_dyson_cas_noalloc.restype = ctypes.c_int
    lib.cc_gf_dyson_last_error.argtypes = []
    lib.cc_gf_dyson_last_error.restype = ctypes.c_char_p
    lib.cc_gf_free.argtypes = [vp]
    lib.cc_gf_free.restype = None
    lib.cc_gf_last_error.argtypes = [vp]
    lib.cc_gf_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _c128(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


def _part(p):
    if isinstance(p, str):
        return {"ip": PART_IP, "ea": PART_EA, "both": PART_BOTH}[p.lower()]
    return int(p)


class Context:
    """One system on the GPU (wraps cc_gf_init / cc_gf_free)."""

    def __init__(self, system, *, tol=1e-10, restart_m=30, maxiter=2000, max_batch=64, stream=None,
                 timing=False, foo=None, fvv=None, l1=None, l2=None, precond_eta=0.0, recycle_k=0, precision="f64",
                 reorth_ratio=0.0, autotune=True, autotune_cache=None, graphs=True, restart_tail=0,
                 seed_m=0, eri_blocks=None):
        """eri_blocks: dense <pq|rs> blocks [k1][k2][k3][nmo]^4 to use instead of the system's
        ERI factor (small systems)."""
        lib = load()
        import torch  # device memory and streams only
        self._torch = torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        s = system
        self._keep = [np.ascontiguousarray(np.asarray(s.eps, dtype=np.float64)),
                      None if eri_blocks is not None else _c128(s.eri_factor), _c128(s.t1), _c128(s.t2)]
        blocks_a = None if eri_blocks is None else _c128(eri_blocks)
        foo_a = None if foo is None else _c128(foo)
        fvv_a = None if fvv is None else _c128(fvv)
        l1_a = None if l1 is None else _c128(l1)
        l2_a = None if l2 is None else _c128(l2)
        self._keep += [foo_a, fvv_a, l1_a, l2_a, blocks_a]
        cs = System()
        cs.kmesh = (ctypes.c_int * 3)(*[int(x) for x in s.kmesh])
        cs.nocc, cs.nvir = int(s.nocc), int(s.nvir)
        cs.eps = self._keep[0].ctypes.data
        cs.foo = None if foo_a is None else foo_a.ctypes.data
        cs.fvv = None if fvv_a is None else fvv_a.ctypes.data
        cs.naux = 0 if blocks_a is not None else int(self._keep[1].shape[2])
        cs.eri_factor = None if blocks_a is not None else self._keep[1].ctypes.data
        cs.eri_blocks = None if blocks_a is None else blocks_a.ctypes.data
        cs.t1 = self._keep[2].ctypes.data
        cs.t2 = self._keep[3].ctypes.data
        cs.mem_space = HOST
        cs.l1 = None if l1_a is None else l1_a.ctypes.data
        cs.l2 = None if l2_a is None else l2_a.ctypes.data
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self._optargs = dict(tol=tol, restart_m=restart_m, maxiter=maxiter, max_batch=max_batch, timing=timing,
                             precond_eta=precond_eta, recycle_k=recycle_k, reorth_ratio=reorth_ratio,
                             autotune=autotune, graphs=graphs, restart_tail=restart_tail, seed_m=seed_m)
        self._prec = prec
        opt = self._options(stream, autotune_cache=autotune_cache, **self._optargs)
        self._opt = opt
        h = ctypes.c_void_p()
        rc = lib.cc_gf_init(ctypes.byref(cs), ctypes.byref(opt), ctypes.byref(h))
        if rc != OK:
            raise CCGFError(rc, lib.cc_gf_last_error(None).decode())
        self._h = h
        self._keep = None
        self.nk = int(np.prod(s.kmesh))
        self.nocc, self.nvir = int(s.nocc), int(s.nvir)
        self.nmo = self.nocc + self.nvir

    def _options(self, stream, *, tol, restart_m, maxiter, max_batch, timing, precond_eta, recycle_k, reorth_ratio,
                 autotune, graphs, restart_tail, seed_m, autotune_cache=None):
        return Options(self._prec, int(restart_m), int(maxiter), float(tol), int(max_batch),
                       ctypes.c_void_p(stream.cuda_stream), 1 if timing else 0, float(precond_eta),
                       int(recycle_k), float(reorth_ratio), 0 if autotune else -1,
                       None if autotune_cache is None else str(autotune_cache).encode(), int(restart_tail),
                       0 if graphs else -1, int(seed_m))

    def set_options(self, **changes):
        """Change solver options (not the precision) of the live context."""
        unknown = set(changes) - set(self._optargs)
        if unknown:
            raise TypeError(f"unknown options {sorted(unknown)}")
        args = dict(self._optargs, **changes)
        opt = self._options(self.stream, **args)
        self._check(load().cc_gf_set_options(self._h, ctypes.byref(opt)))
        self._optargs, self._opt = args, opt

    def _check(self, rc, allow=()):
        if rc != OK and rc not in allow:
            raise CCGFError(rc, load().cc_gf_last_error(self._h).decode())
        return rc

    def close(self):
        if getattr(self, "_h", None):
            load().cc_gf_free(self._h)
            self._h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def vector_size(self, part) -> int:
        n = ctypes.c_longlong()
        self._check(load().cc_gf_vector_size(self._h, _part(part), ctypes.byref(n)))
        return int(n.value)

    def sigma(self, part, K: int, x):
        """y = M(K) x for a [nvec, n] complex128 CUDA tensor."""
        torch = self._torch
        assert x.is_cuda and x.dtype == torch.complex128 and x.is_contiguous()
        n = self.vector_size(part)
        xx = x.reshape(-1, n)
        y = torch.empty_like(xx)
        self._check(load().cc_gf_sigma(self._h, _part(part), int(K), int(xx.shape[0]), xx.data_ptr(),
                                       y.data_ptr()))
        return y.reshape(x.shape)

    def vectors(self, part, K: int, p: int):
        """(b, e) CUDA tensors of orbital p at momentum K."""
        torch = self._torch
        n = self.vector_size(part)
        b = torch.empty(n, dtype=torch.complex128, device="cuda")
        e = torch.empty(n, dtype=torch.complex128, device="cuda")
        self._check(load().cc_gf_vectors(self._h, _part(part), int(K), int(p), b.data_ptr(), e.data_ptr()))
        return b, e

    def solve(self, kidx: Sequence[int], orbs: Sequence[int], omega, eta: float, parts="both",
              allow_noconv=False):
        """G, G+, G-, stats for the diagonal G_pp(K, w); arrays [nkq][norb][nw]."""
        kidx = np.ascontiguousarray(np.asarray(kidx, dtype=np.int32))
        orbs = np.ascontiguousarray(np.asarray(orbs, dtype=np.int32))
        om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        shape = (len(kidx), len(orbs), len(om))
        G = np.zeros(shape, dtype=np.complex128)
        Gp = np.zeros(shape, dtype=np.complex128)
        Gm = np.zeros(shape, dtype=np.complex128)
        st = Stats()
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = load().cc_gf_solve(self._h, len(kidx), kidx.ctypes.data_as(ip), len(orbs), orbs.ctypes.data_as(ip),
                                len(om), om.ctypes.data_as(dp), float(eta), _part(parts), G.ctypes.data,
                                Gp.ctypes.data, Gm.ctypes.data, ctypes.byref(st))
        self._check(rc, allow=(ENOCONV,) if allow_noconv else ())
        return G, Gp, Gm, st.as_dict()

    def solve_matrix(self, kidx: Sequence[int], orbs: Sequence[int], omega, eta: float, parts="both",
                     allow_noconv=False):
        """G, G+, G- [nkq][nw][norb][norb], DOS [nkq][nw] and stats for the full G_pq(K, w)."""
        kidx = np.ascontiguousarray(np.asarray(kidx, dtype=np.int32))
        orbs = np.ascontiguousarray(np.asarray(orbs, dtype=np.int32))
        om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        shape = (len(kidx), len(om), len(orbs), len(orbs))
        G = np.zeros(shape, dtype=np.complex128)
        Gp = np.zeros(shape, dtype=np.complex128)
        Gm = np.zeros(shape, dtype=np.complex128)
        dos = np.zeros((len(kidx), len(om)), dtype=np.float64)
        st = Stats()
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = load().cc_gf_solve_matrix(self._h, len(kidx), kidx.ctypes.data_as(ip), len(orbs), orbs.ctypes.data_as(ip),
                                       len(om), om.ctypes.data_as(dp), float(eta), _part(parts), G.ctypes.data,
                                       Gp.ctypes.data, Gm.ctypes.data, dos.ctypes.data, ctypes.byref(st))
        self._check(rc, allow=(ENOCONV,) if allow_noconv else ())
        return G, Gp, Gm, dos, st.as_dict()

    def learn(self, K: int, orbs: Sequence[int], omega_train, eta: float, parts="both", epochs=0, batch=0, lr=0.0,
              seed=0, hidden=0, guess="network", accept=0.0, probe=0, allow_noconv=False):
        """Train the initial-guess network of momentum K on plain solves at omega_train."""
        orbs = np.ascontiguousarray(np.asarray(orbs, dtype=np.int32))
        wt = np.ascontiguousarray(np.asarray(omega_train, dtype=np.float64))
        lo = LearnOptions(int(epochs), int(batch), float(lr), int(seed), int(hidden),
                          {"network": 0, "nearest": 1}[guess], float(accept), int(probe))
        ls = LearnStats()
        rc = load().cc_gf_learn(self._h, _part(parts), int(K), len(orbs), orbs.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                len(wt), wt.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), float(eta),
                                ctypes.byref(lo), ctypes.byref(ls))
        self._check(rc, allow=(ENOCONV,) if allow_noconv else ())
        return ls.as_dict()

    def learn_enable(self, on=True, *, guess=None, precond=None):
        """Use the trained networks (on) or none; guess / precond select each one."""
        g = on if guess is None else guess
        p = on if precond is None else precond
        self._check(load().cc_gf_learn_enable(self._h, (1 if g else 0) | (2 if p else 0)))

    def learn_save(self, path):
        """Write the trained networks (every part and K) to path."""
        self._check(load().cc_gf_learn_save(self._h, os.fsencode(path)))

    def learn_load(self, path):
        """Replace this context's networks by those saved at path (same system shape)."""
        self._check(load().cc_gf_learn_load(self._h, os.fsencode(path)))

    def mor(self, kidx: Sequence[int], orbs: Sequence[int], wexp_ip, wexp_ea, omega, eta: float, parts="both",
            allow_noconv=False):
        """Model-order-reduced G, G+, G-, stats on the grid omega from full solves at the
        expansion frequencies wexp_ip (IP) and wexp_ea (EA); arrays [nkq][norb][nw]."""
        kidx = np.ascontiguousarray(np.asarray(kidx, dtype=np.int32))
        orbs = np.ascontiguousarray(np.asarray(orbs, dtype=np.int32))
        om = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        wi = np.ascontiguousarray(np.asarray(wexp_ip if wexp_ip is not None else [], dtype=np.float64))
        wa = np.ascontiguousarray(np.asarray(wexp_ea if wexp_ea is not None else [], dtype=np.float64))
        shape = (len(kidx), len(orbs), len(om))
        G = np.zeros(shape, dtype=np.complex128)
        Gp = np.zeros(shape, dtype=np.complex128)
        Gm = np.zeros(shape, dtype=np.complex128)
        st = Stats()
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        rc = load().cc_gf_mor(self._h, len(kidx), kidx.ctypes.data_as(ip), len(orbs), orbs.ctypes.data_as(ip),
                              len(wi), wi.ctypes.data_as(dp), len(wa), wa.ctypes.data_as(dp),
                              len(om), om.ctypes.data_as(dp), float(eta), _part(parts), G.ctypes.data,
                              Gp.ctypes.data, Gm.ctypes.data, ctypes.byref(st))
        self._check(rc, allow=(ENOCONV,) if allow_noconv else ())
        return G, Gp, Gm, st.as_dict()


def sigma_group(items):
    """Grouped sigma products: items is a list of (Context, part, K, x) with x a CUDA
    complex128 [nvec, n] tensor; returns the list of y tensors."""
    lib = load()
    import torch
    n = len(items)
    vp = ctypes.c_void_p
    ys = [torch.empty_like(x) for (_, _, _, x) in items]
    for (_, _, _, x) in items:
        assert x.is_cuda and x.dtype == torch.complex128 and x.is_contiguous()
    ctxs = (vp * n)(*[c._h.value for (c, _, _, _) in items])
    parts = (ctypes.c_int * n)(*[_part(p) for (_, p, _, _) in items])
    ks = (ctypes.c_int * n)(*[int(k) for (_, _, k, _) in items])
    nv = (ctypes.c_int * n)(*[int(x.shape[0]) for (_, _, _, x) in items])
    xp = (vp * n)(*[x.data_ptr() for (_, _, _, x) in items])
    yp = (vp * n)(*[y.data_ptr() for y in ys])
    rc = lib.cc_gf_sigma_group(n, ctxs, parts, ks, nv, xp, yp)
    if rc != OK:
        raise CCGFError(rc, lib.cc_gf_last_error(items[0][0]._h).decode())
    return ys


def dyson_cas(Ggw, Ggw_cas, Gcc, V, stream=None, self_energies=False, noalloc=False):
    """G_CC+GW [nk][nw][N][N] (and optionally Sigma_full, Sigma_CAS) from CUDA complex128
    tensors Ggw [nk][nw][N][N], Ggw_cas and Gcc [nk][nw][M][M], V [nk][N][M]; noalloc
    calls the entry point that allocates nothing (its fixed per-device scratch).
    The outputs are allocated here by torch, as any caller of the C ABI provides them."""
    lib = load()
    import torch
    for t in (Ggw, Ggw_cas, Gcc, V):
        assert t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()
    nk, nw, N = Ggw.shape[0], Ggw.shape[1], Ggw.shape[2]
    M = V.shape[2]
    assert Ggw.shape == (nk, nw, N, N) and Ggw_cas.shape == (nk, nw, M, M) and Gcc.shape == (nk, nw, M, M)
    assert V.shape == (nk, N, M)
    out = torch.empty_like(Ggw)
    sf = torch.empty_like(Ggw) if self_energies else None
    sc = torch.empty_like(Gcc) if self_energies else None
    if stream is None:
        stream = torch.cuda.current_stream()
    fn = lib.cc_gf_dyson_cas_noalloc if noalloc else lib.cc_gf_dyson_cas
    rc = fn(nk, nw, N, M, Ggw.data_ptr(), Ggw_cas.data_ptr(), Gcc.data_ptr(), V.data_ptr(),
                             out.data_ptr(), sf.data_ptr() if sf is not None else None,
                             sc.data_ptr() if sc is not None else None, ctypes.c_void_p(stream.cuda_stream))
    if rc != OK:
        raise CCGFError(rc, lib.cc_gf_dyson_last_error().decode())
    return (out, sf, sc) if self_energies else out


def mlp_grad(din: int, hidden: int, dout: int, theta, X, T):
    """(loss, gradient) of the initial-guess network on the GPU (FP32)."""
    f32 = lambda a: np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    theta, X, T = f32(theta), f32(X), f32(T)
    g = np.zeros_like(theta)
    L = ctypes.c_double()
    fp = ctypes.POINTER(ctypes.c_float)
    rc = load().cc_gf_mlp_grad(int(din), int(hidden), int(dout), theta.ctypes.data_as(fp), int(X.shape[0]),
                               X.ctypes.data_as(fp), T.ctypes.data_as(fp), g.ctypes.data_as(fp), ctypes.byref(L))
    if rc != OK:
        raise CCGFError(rc, "cc_gf_mlp_grad failed")
    return L.value, g
