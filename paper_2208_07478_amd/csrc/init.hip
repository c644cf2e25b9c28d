// Device construction of the EOM-CCSD Hbar blocks and of the b / e vectors.
//
// All blocks are built once per system in FP64 by element-wise kernels (one
// thread per output element, explicit momentum loops).  The blocks are the
// spin-orbital CCSD similarity-transformed Hamiltonian elements (one-body F,
// two-body W and the W_oovv * T2 three-body pieces) that make up the
// connected EOM-IP/EA-CCSD matrix; Lambda = T^dagger enters the left vectors
// (approximation stated after Eq. 10).  The right-hand sides b and left
// vectors e follow from abar = exp(-T) a exp(T) = a - [T, a] (Eqs. 5-7).
#include "ccgf_internal.h"

namespace {

template <class F>
__global__ void k_foreach(size_t n, F f) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f(i);
}

template <class F>
void foreach_(hipStream_t s, size_t n, F f) {
  if (n == 0) return;
  size_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_foreach<F>, dim3((unsigned)blocks), dim3(256), 0, s, n, f);
}

struct I7 {
  int k1, k2, k3, a, b, c, d;
};
__device__ inline I7 dec(size_t i, int nk, int n1, int n2, int n3, int n4) {
  I7 r;
  r.d = (int)(i % n4); i /= n4;
  r.c = (int)(i % n3); i /= n3;
  r.b = (int)(i % n2); i /= n2;
  r.a = (int)(i % n1); i /= n1;
  r.k3 = (int)(i % nk); i /= nk;
  r.k2 = (int)(i % nk); i /= nk;
  r.k1 = (int)i;
  return r;
}

// Antisymmetrised <p k1, q k2 || r k3, s k4> = <pq|rs> - <pq|sr> (global orbital indices)
// from the factor, or from the dense blocks D when those were given instead.
struct Eri {
  const cplx *A;
  int nk, naux, nmo;
  KTab kt;
  const cplx *D;
  __device__ inline cplx fac(int ka, int kb, int L, int p, int r) const {
    return A[((((size_t)ka * nk + kb) * naux + L) * nmo + p) * nmo + r];
  }
  __device__ inline cplx dense(int k1, int k2, int k3, int p, int q, int r, int s) const {
    return D[((((((size_t)k1 * nk + k2) * nk + k3) * nmo + p) * nmo + q) * nmo + r) * nmo + s];
  }
  __device__ inline cplx operator()(int k1, int k2, int k3, int p, int q, int r, int s) const {
    int k4 = kt.c3(k1, k2, k3);
    if (D) return csub(dense(k1, k2, k3, p, q, r, s), dense(k1, k2, k4, p, q, s, r));
    cplx acc = mkc(0, 0);
    for (int L = 0; L < naux; ++L) {
      cfma(acc, fac(k1, k3, L, p, r), fac(k2, k4, L, q, s));
      cplx x = fac(k1, k4, L, p, s);
      cplx y = fac(k2, k3, L, q, r);
      acc.x -= x.x * y.x - x.y * y.y;
      acc.y -= x.x * y.y + x.y * y.x;
    }
    return acc;
  }
};

// Lambda amplitudes: the given l1 / l2 ([k][i][a] and [ki][kj][ka][i][j][a][b], the layouts of
// t1 / t2), or T^dagger (lambda_a^i = conj(t_i^a), lambda_ab^ij = conj(t_ij^ab)) when none are given
struct Lam {
  T2d t1;
  T4 t2;
  const cplx *l1, *l2;
  __device__ inline cplx one(int k, int i, int a) const {
    return l1 ? l1[((size_t)k * t1.n1 + i) * t1.n2 + a] : cconj(t1(k, i, a));
  }
  __device__ inline cplx two(int ki, int kj, int ka, int i, int j, int a, int b) const {
    return l2 ? l2[t2.at(ki, kj, ka, i, j, a, b)] : cconj(t2(ki, kj, ka, i, j, a, b));
  }
};

}  // namespace

long long vec_len(const ccgf_ctx *c, int part) {
  long long nk = c->nk, no = c->no, nv = c->nv;
  return part == CCGF_PART_IP ? no + nk * nk * no * no * nv : nv + nk * nk * no * nv * nv;
}

static T4 make_t4(ccgf_ctx *c, int n1, int n2, int n3, int n4, bool alloc = true) {
  T4 t{nullptr, c->nk, n1, n2, n3, n4};
  if (alloc) t.p = (cplx *)dev_alloc(c, t.size() * sizeof(cplx));
  return t;
}

int build_hbar(ccgf_ctx *c) {
  const int nk = c->nk, no = c->no, nv = c->nv, nmo = c->nmo;
  hipStream_t s = c->stream;
  KTab kt{nk, c->kc3};
  Eri eri{c->fac, nk, c->naux, nmo, kt, c->eri_dense};

  // ---- bare antisymmetrised integral classes (o = occupied, v = virtual)
  auto cls = [&](const char *spec) {
    int n[4], off[4];
    for (int i = 0; i < 4; ++i) {
      n[i] = spec[i] == 'o' ? no : nv;
      off[i] = spec[i] == 'o' ? 0 : no;
    }
    T4 t = make_t4(c, n[0], n[1], n[2], n[3]);
    if (!t.p) return t;
    int o0 = off[0], o1 = off[1], o2 = off[2], o3 = off[3];
    int n0 = n[0], n1 = n[1], n2 = n[2], n3 = n[3];
    foreach_(s, t.size(), [=] __device__(size_t i) {
      I7 x = dec(i, nk, n0, n1, n2, n3);
      t.p[i] = eri(x.k1, x.k2, x.k3, x.a + o0, x.b + o1, x.c + o2, x.d + o3);
    });
    return t;
  };
  // (the ovvv and vvvo classes are not stored: <mb||ef> = -<bm||ef> is read from the vovv
  // class, and <ab||ei> is formed from the factor where it is needed once)
  T4 Voooo = cls("oooo"), Vooov = cls("ooov"), Voovo = cls("oovo"), Voovv = cls("oovv");
  T4 Vovoo = cls("ovoo"), Vovvo = cls("ovvo"), Vvovv = cls("vovv");
  if (!Voooo.p || !Vooov.p || !Voovo.p || !Voovv.p || !Vovoo.p || !Vovvo.p || !Vvovv.p) return CCGF_ENOMEM;
  struct OVVV {
    T4 vo;
    __device__ inline cplx operator()(int km, int kb, int ke, int m, int b, int e, int f) const {
      cplx x = vo(kb, km, ke, b, m, e, f);
      return mkc(-x.x, -x.y);
    }
  } Vovvv{Vvovv};

  T2d t1{c->t1, no, nv};
  T4 t2{c->t2, nk, no, no, nv, nv};
  T2d foo{c->foo, no, no}, fvv{c->fvv, nv, nv};

  // tau_ij^ab = t_ij^ab + t_i^a t_j^b - t_i^b t_j^a
  T4 tau = make_t4(c, no, no, nv, nv);
  if (!tau.p) return CCGF_ENOMEM;
  foreach_(s, tau.size(), [=] __device__(size_t i) {
    I7 x = dec(i, nk, no, no, nv, nv);
    int ki = x.k1, kj = x.k2, ka = x.k3, kb = kt.c3(ki, kj, ka);
    cplx v = t2.p[i];
    if (ka == ki) v = cadd(v, cmul(t1(ki, x.a, x.c), t1(kj, x.b, x.d)));
    if (kb == ki) v = csub(v, cmul(t1(ki, x.a, x.d), t1(kj, x.b, x.c)));
    tau.p[i] = v;
  });

  // ---- one-body blocks
  c->Fov = (cplx *)dev_alloc(c, sizeof(cplx) * nk * no * nv);
  c->Foo = (cplx *)dev_alloc(c, sizeof(cplx) * nk * no * no);
  c->Fvv = (cplx *)dev_alloc(c, sizeof(cplx) * nk * nv * nv);
  if (!c->Fov || !c->Foo || !c->Fvv) return CCGF_ENOMEM;
  T2d Fov{c->Fov, no, nv}, Foo{c->Foo, no, no}, Fvv{c->Fvv, nv, nv};
  foreach_(s, (size_t)nk * no * nv, [=] __device__(size_t i) {
    int e = i % nv, m = (i / nv) % no, k = (int)(i / ((size_t)nv * no));
    cplx acc = mkc(0, 0);
    for (int kn = 0; kn < nk; ++kn)
      for (int n = 0; n < no; ++n)
        for (int f = 0; f < nv; ++f) cfma(acc, t1(kn, n, f), Voovv(k, kn, k, m, n, e, f));
    Fov.p[i] = acc;
  });
  foreach_(s, (size_t)nk * no * no, [=] __device__(size_t i) {
    int ii = i % no, m = (i / no) % no, k = (int)(i / ((size_t)no * no));
    cplx acc = foo(k, m, ii);
    for (int kn = 0; kn < nk; ++kn)
      for (int n = 0; n < no; ++n)
        for (int e = 0; e < nv; ++e) cfma(acc, t1(kn, n, e), Vooov(k, kn, k, m, n, ii, e));
    cplx h = mkc(0, 0);
    for (int kn = 0; kn < nk; ++kn)
      for (int ke = 0; ke < nk; ++ke)
        for (int n = 0; n < no; ++n)
          for (int e = 0; e < nv; ++e)
            for (int f = 0; f < nv; ++f) cfma(h, tau(k, kn, ke, ii, n, e, f), Voovv(k, kn, ke, m, n, e, f));
    Foo.p[i] = cadd(acc, cscale(h, 0.5));
  });
  foreach_(s, (size_t)nk * nv * nv, [=] __device__(size_t i) {
    int e = i % nv, a = (i / nv) % nv, k = (int)(i / ((size_t)nv * nv));
    cplx acc = fvv(k, a, e);
    for (int km = 0; km < nk; ++km)
      for (int m = 0; m < no; ++m)
        for (int f = 0; f < nv; ++f) cfma(acc, t1(km, m, f), Vvovv(k, km, k, a, m, e, f));
    cplx h = mkc(0, 0);
    for (int km = 0; km < nk; ++km)
      for (int kn = 0; kn < nk; ++kn)
        for (int m = 0; m < no; ++m)
          for (int n = 0; n < no; ++n)
            for (int f = 0; f < nv; ++f) cfma(h, tau(km, kn, k, m, n, a, f), Voovv(km, kn, k, m, n, e, f));
    Fvv.p[i] = csub(acc, cscale(h, 0.5));
  });

  // ---- W_mnij
  T4 Woooo = make_t4(c, no, no, no, no);
  if (!Woooo.p) return CCGF_ENOMEM;
  c->Woooo = Woooo.p;
  foreach_(s, Woooo.size(), [=] __device__(size_t i) {
    I7 x = dec(i, nk, no, no, no, no);
    int km = x.k1, kn = x.k2, ki = x.k3, kj = kt.c3(km, kn, ki);
    int m = x.a, n = x.b, ii = x.c, j = x.d;
    cplx acc = Voooo.p[i];
    for (int e = 0; e < nv; ++e) {
      cfma(acc, t1(kj, j, e), Vooov(km, kn, ki, m, n, ii, e));
      cplx y = cmul(t1(ki, ii, e), Vooov(km, kn, kj, m, n, j, e));
      acc = csub(acc, y);
    }
    cplx h = mkc(0, 0);
    for (int ke = 0; ke < nk; ++ke)
      for (int e = 0; e < nv; ++e)
        for (int f = 0; f < nv; ++f) cfma(h, tau(ki, kj, ke, ii, j, e, f), Voovv(km, kn, ke, m, n, e, f));
    Woooo.p[i] = cadd(acc, cscale(h, 0.5));
  });

  // ---- W_abef (bare vvvv integrals formed on the fly from the factor), stored blocks only
  std::vector<int> wtrip;  // (ka, kb, kc) of each stored block
  c->wblk_h.assign((size_t)nk * nk * nk, -1);
  for (int ka = 0; ka < nk; ++ka)
    for (int kb = ka; kb < nk; ++kb)
      for (int kc = 0; kc < nk; ++kc) {
        const int kd = c->kc3_h[((size_t)ka * nk + kb) * nk + kc];
        if (kc > kd) continue;
        c->wblk_h[((size_t)ka * nk + kb) * nk + kc] = (int)(wtrip.size() / 3);
        wtrip.push_back(ka);
        wtrip.push_back(kb);
        wtrip.push_back(kc);
      }
  c->nwblk = (long long)(wtrip.size() / 3);
  const size_t nv4 = (size_t)nv * nv * nv * nv;
  c->wblk = (int *)dev_alloc(c, sizeof(int) * c->wblk_h.size());
  int *d_trip = (int *)dev_alloc(c, sizeof(int) * wtrip.size());
  c->Wvvvv = (cplx *)dev_alloc(c, sizeof(cplx) * nv4 * (size_t)c->nwblk);
  if (!c->wblk || !d_trip || !c->Wvvvv) return CCGF_ENOMEM;
  hipMemcpyAsync(c->wblk, c->wblk_h.data(), sizeof(int) * c->wblk_h.size(), hipMemcpyHostToDevice, s);
  hipMemcpyAsync(d_trip, wtrip.data(), sizeof(int) * wtrip.size(), hipMemcpyHostToDevice, s);
  cplx *Wpk = c->Wvvvv;
  const WPacked Wvvvv{c->Wvvvv, c->wblk, kt, nv};
  foreach_(s, nv4 * (size_t)c->nwblk, [=] __device__(size_t i) {
    const size_t q = i / nv4, r = i % nv4;
    int ka = d_trip[3 * q], kb = d_trip[3 * q + 1], ke = d_trip[3 * q + 2];
    int f = (int)(r % nv), e = (int)((r / nv) % nv), b = (int)((r / ((size_t)nv * nv)) % nv),
        a = (int)(r / ((size_t)nv * nv * nv));
    cplx acc = eri(ka, kb, ke, no + a, no + b, no + e, no + f);
    for (int m = 0; m < no; ++m) {
      acc = csub(acc, cmul(t1(kb, m, b), Vvovv(ka, kb, ke, a, m, e, f)));
      cfma(acc, t1(ka, m, a), Vvovv(kb, ka, ke, b, m, e, f));
    }
    cplx h = mkc(0, 0);
    for (int km = 0; km < nk; ++km) {
      int kn = kt.c3(ka, kb, km);
      for (int m = 0; m < no; ++m)
        for (int n = 0; n < no; ++n) cfma(h, tau(km, kn, ka, m, n, a, b), Voovv(km, kn, ke, m, n, e, f));
    }
    Wpk[i] = cadd(acc, cscale(h, 0.5));
  });

  // ---- Z_mbej = <mb||ej> - t_nj^bf <mn||ef>  (shared by W_mbej, W_mbij, W_abei)
  T4 Z = make_t4(c, no, nv, nv, no);
  if (!Z.p) return CCGF_ENOMEM;
  foreach_(s, Z.size(), [=] __device__(size_t i) {
    I7 x = dec(i, nk, no, nv, nv, no);
    int km = x.k1, kb = x.k2, ke = x.k3, kj = kt.c3(km, kb, ke);
    cplx acc = Vovvo.p[i];
    for (int kn = 0; kn < nk; ++kn)
      for (int n = 0; n < no; ++n)
        for (int f = 0; f < nv; ++f)
          acc = csub(acc, cmul(t2(kn, kj, kb, n, x.d, x.b, f), Voovv(km, kn, ke, x.a, n, x.c, f)));
    Z.p[i] = acc;
  });

  // ---- W_mbej
  T4 Wovvo = make_t4(c, no, nv, nv, no);
  if (!Wovvo.p) return CCGF_ENOMEM;
  c->Wovvo = Wovvo.p;
  foreach_(s, Wovvo.size(), [=] __device__(size_t i) {
    I7 x = dec(i, nk, no, nv, nv, no);
    int km = x.k1, kb = x.k2, ke = x.k3, kj = kt.c3(km, kb, ke);
    int m = x.a, b = x.b, e = x.c, j = x.d;
    cplx acc = Z.p[i];
    for (int f = 0; f < nv; ++f) cfma(acc, t1(kj, j, f), Vovvv(km, kb, ke, m, b, e, f));
    for (int n = 0; n < no; ++n) {
      acc = csub(acc, cmul(t1(kb, n, b), Voovo(km, kb, ke, m, n, e, j)));
      cplx tn = t1(kb, n, b);
      for (int f = 0; f < nv; ++f)
        acc = csub(acc, cmul(cmul(t1(kj, j, f), tn), Voovv(km, kb, ke, m, n, e, f)));
    }
    Wovvo.p[i] = acc;
  });

  // ---- W_mnie, W_amef
  T4 Wooov = make_t4(c, no, no, no, nv);
  T4 Wvovv = make_t4(c, nv, no, nv, nv);
  if (!Wooov.p || !Wvovv.p) return CCGF_ENOMEM;
  c->Wooov = Wooov.p;
  c->Wvovv = Wvovv.p;
  foreach_(s, Wooov.size(), [=] __device__(size_t i) {
    I7 x = dec(i, nk, no, no, no, nv);
    cplx acc = Vooov.p[i];
    for (int f = 0; f < nv; ++f) cfma(acc, t1(x.k3, x.c, f), Voovv(x.k1, x.k2, x.k3, x.a, x.b, f, x.d));
    Wooov.p[i] = acc;
  });
  foreach_(s, Wvovv.size(), [=] __device__(size_t i) {
    I7 x = dec(i, nk, nv, no, nv, nv);
    cplx acc = Vvovv.p[i];
    for (int n = 0; n < no; ++n)
      acc = csub(acc, cmul(t1(x.k1, n, x.a), Voovv(x.k1, x.k2, x.k3, n, x.b, x.c, x.d)));
    Wvovv.p[i] = acc;
  });

  // ---- W_mbij
  T4 Wovoo = make_t4(c, no, nv, no, no);
  if (!Wovoo.p) return CCGF_ENOMEM;
  c->Wovoo = Wovoo.p;
  foreach_(s, Wovoo.size(), [=] __device__(size_t i) {
    I7 x = dec(i, nk, no, nv, no, no);
    int km = x.k1, kb = x.k2, ki = x.k3, kj = kt.c3(km, kb, ki);
    int m = x.a, b = x.b, ii = x.c, j = x.d;
    cplx acc = Vovoo.p[i];
    for (int e = 0; e < nv; ++e) acc = csub(acc, cmul(Fov(km, m, e), t2(ki, kj, kb, ii, j, b, e)));
    for (int n = 0; n < no; ++n) acc = csub(acc, cmul(t1(kb, n, b), Woooo(km, kb, ki, m, n, ii, j)));
    cplx h = mkc(0, 0);
    for (int ke = 0; ke < nk; ++ke)
      for (int e = 0; e < nv; ++e)
        for (int f = 0; f < nv; ++f) cfma(h, Vovvv(km, kb, ke, m, b, e, f), tau(ki, kj, ke, ii, j, e, f));
    acc = cadd(acc, cscale(h, 0.5));
    for (int kn = 0; kn < nk; ++kn)
      for (int n = 0; n < no; ++n)
        for (int e = 0; e < nv; ++e) {
          cfma(acc, Vooov(km, kn, ki, m, n, ii, e), t2(kj, kn, kb, j, n, b, e));
          acc = csub(acc, cmul(Vooov(km, kn, kj, m, n, j, e), t2(ki, kn, kb, ii, n, b, e)));
        }
    for (int e = 0; e < nv; ++e) {
      cfma(acc, t1(ki, ii, e), Z(km, kb, ki, m, b, e, j));
      acc = csub(acc, cmul(t1(kj, j, e), Z(km, kb, kj, m, b, e, ii)));
    }
    Wovoo.p[i] = acc;
  });

  // ---- W_abei
  T4 Wvvvo = make_t4(c, nv, nv, nv, no);
  if (!Wvvvo.p) return CCGF_ENOMEM;
  c->Wvvvo = Wvvvo.p;
  foreach_(s, Wvvvo.size(), [=] __device__(size_t i) {
    I7 x = dec(i, nk, nv, nv, nv, no);
    int ka = x.k1, kb = x.k2, ke = x.k3, ki = kt.c3(ka, kb, ke);
    int a = x.a, b = x.b, e = x.c, ii = x.d;
    cplx acc = eri(ka, kb, ke, no + a, no + b, no + e, ii);
    for (int m = 0; m < no; ++m) acc = csub(acc, cmul(Fov(ke, m, e), t2(ke, ki, ka, m, ii, a, b)));
    for (int f = 0; f < nv; ++f) cfma(acc, t1(ki, ii, f), Wvvvv(ka, kb, ke, a, b, e, f));
    cplx h = mkc(0, 0);
    for (int km = 0; km < nk; ++km) {
      int kn = kt.c3(ke, ki, km);
      for (int m = 0; m < no; ++m)
        for (int n = 0; n < no; ++n) cfma(h, Voovo(km, kn, ke, m, n, e, ii), tau(km, kn, ka, m, n, a, b));
    }
    acc = cadd(acc, cscale(h, 0.5));
    for (int km = 0; km < nk; ++km)
      for (int m = 0; m < no; ++m)
        for (int f = 0; f < nv; ++f) {
          acc = csub(acc, cmul(Vovvv(km, kb, ke, m, b, e, f), t2(km, ki, ka, m, ii, a, f)));
          cfma(acc, Vovvv(km, ka, ke, m, a, e, f), t2(km, ki, kb, m, ii, b, f));
        }
    for (int m = 0; m < no; ++m) {
      acc = csub(acc, cmul(t1(ka, m, a), Z(ka, kb, ke, m, b, e, ii)));
      cfma(acc, t1(kb, m, b), Z(kb, ka, ke, m, a, e, ii));
    }
    Wvvvo.p[i] = acc;
  });

  // ---- GEMM-ready permutations of W_mbej and W_mnij used by the sigma products
  T4 WvoP = make_t4(c, nv, no, no, nv);  // [kx][ki][km](x, i, m, e) = W_mxei
  T4 WooP = make_t4(c, no, no, no, no);  // [ki][kj][km](i, j, m, n) = W_mnij
  if (!WvoP.p || !WooP.p) return CCGF_ENOMEM;
  c->WvoP = WvoP.p;
  c->WooP = WooP.p;
  foreach_(s, WvoP.size(), [=] __device__(size_t i) {
    I7 x = dec(i, nk, nv, no, no, nv);
    int kx = x.k1, ki = x.k2, km = x.k3, ke = kt.c3(km, kx, ki);
    WvoP.p[i] = Wovvo(km, kx, ke, x.c, x.a, x.d, x.b);
  });
  foreach_(s, WooP.size(), [=] __device__(size_t i) {
    I7 x = dec(i, nk, no, no, no, no);
    int ki = x.k1, kj = x.k2, km = x.k3, kn = kt.c3(ki, kj, km);
    WooP.p[i] = Woooo(km, kn, ki, x.c, x.d, x.a, x.b);
  });
  // EA operand of the same product with the virtual Fock block folded in: the sigma_EA term
  // F_bd r_i^ad has the form of W_lbdi r_l^ad with l = i, so [kb][ki][ki](b, i, i, d) += F_bd(kb)
  T4 WvoPea = make_t4(c, nv, no, no, nv);
  if (!WvoPea.p) return CCGF_ENOMEM;
  c->WvoPea = WvoPea.p;
  const cplx *Fvv_ = c->Fvv;
  foreach_(s, WvoPea.size(), [=] __device__(size_t i) {
    I7 x = dec(i, nk, nv, no, no, nv);
    cplx w = WvoP.p[i];
    if (x.k3 == x.k2 && x.c == x.b) w = cadd(w, Fvv_[((size_t)x.k1 * nv + x.a) * nv + x.d]);
    WvoPea.p[i] = w;
  });

  c->Voovv = Voovv.p;
  if (hip_check(c, hipStreamSynchronize(s), "building Hbar blocks") != CCGF_OK) return CCGF_EDEVICE;
  // release the integral classes that the products do not read
  auto release = [&](cplx *p) {
    for (auto &q : c->allocs)
      if (q == (void *)p) {
        hipFree(q);
        q = nullptr;
      }
  };
  release(Voooo.p); release(Vooov.p); release(Voovo.p); release(Vovoo.p); release(Vovvo.p);
  release(Vvovv.p); release(tau.p); release(Z.p); release((cplx *)d_trip);
  // blocks that only fed the others
  release(c->Woooo); c->Woooo = nullptr;
  release(c->Wovvo); c->Wovvo = nullptr;
  if (c->opt.precision != CCGF_PLAIN_F64) {  // reduced-precision operands of the big products
    // complex-float copies of the GEMM operands (rounded once, here), or for the BF16-split
    // form their split copies (four bf16 planes per element, the same size)
    const bool split = c->opt.precision == CCGF_MIXED_BF16X3;
    auto to32 = [&](const cplx *src, size_t nel) -> float2 * {
      float2 *d = (float2 *)dev_alloc(c, nel * sizeof(float2));
      if (!d) return nullptr;
      if (split)
        foreach_(s, nel, [=] __device__(size_t i) {
          B3E e;
          split_bf(src[i].x, e.rh, e.rl);
          split_bf(src[i].y, e.ih, e.il);
          ((B3E *)d)[i] = e;
        });
      else
        foreach_(s, nel, [=] __device__(size_t i) { d[i] = make_float2((float)src[i].x, (float)src[i].y); });
      return d;
    };
    c->Wvvvv32 = to32(c->Wvvvv, nv4 * (size_t)c->nwblk);
    c->WvoP32 = to32(WvoP.p, WvoP.size());
    c->WooP32 = to32(WooP.p, WooP.size());
    c->WvoPea32 = to32(WvoPea.p, WvoPea.size());
    if (!c->Wvvvv32 || !c->WvoP32 || !c->WooP32 || !c->WvoPea32) return CCGF_ENOMEM;
  }
  return hip_check(c, hipStreamSynchronize(s), "building the FP32 operands");
}

// *out = sum of v over a 256-thread block
__device__ inline void block_store_sum(cplx v, cplx *out) {
  __shared__ double sh[2][256];
  sh[0][threadIdx.x] = v.x;
  sh[1][threadIdx.x] = v.y;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = mkc(sh[0][0], sh[1][0]);
}

// h[i] = sum over kl, kc, l, c, d of t2[K][kl][kc](p, l, c, d) lambda2[K][kl][kc](i, l, c, d),
// one 256-thread block per occupied i (the 1h overlap term of the IP e vector)
__global__ __launch_bounds__(256) void k_t2_overlap(T4 t2, Lam lam, int K, int p, cplx *__restrict__ h) {
  const int ii = blockIdx.x, nk = t2.nk, no = t2.n2, nv = t2.n4;
  const long long tot = (long long)nk * nk * no * nv * nv;
  cplx acc = mkc(0, 0);
  for (long long q = threadIdx.x; q < tot; q += blockDim.x) {
    long long r = q;
    const int d = (int)(r % nv);
    r /= nv;
    const int cc = (int)(r % nv);
    r /= nv;
    const int l = (int)(r % no);
    r /= no;
    const int kc = (int)(r % nk), kl = (int)(r / nk);
    cfma(acc, t2(K, kl, kc, p, l, cc, d), lam.two(K, kl, kc, ii, l, cc, d));
  }
  block_store_sum(acc, h + ii);
}

// h[a] = sum over kk, kl, k, l, d of t2[kk][kl][kd](k, l, d, c0) lambda2[kk][kl][kd](k, l, d, a),
// kd = kk + kl - K, one 256-thread block per virtual a (the 1p overlap term of the EA e vector)
__global__ __launch_bounds__(256) void k_t2_overlap_ea(T4 t2, Lam lam, KTab kt, int K, int c0,
                                                       cplx *__restrict__ h) {
  const int a = blockIdx.x, nk = t2.nk, no = t2.n1, nv = t2.n4;
  const long long tot = (long long)nk * nk * no * no * nv;
  cplx acc = mkc(0, 0);
  for (long long q = threadIdx.x; q < tot; q += blockDim.x) {
    long long r = q;
    const int d = (int)(r % nv);
    r /= nv;
    const int l = (int)(r % no);
    r /= no;
    const int k = (int)(r % no);
    r /= no;
    const int kl = (int)(r % nk), kk = (int)(r / nk);
    const int kd = kt.c3(kk, kl, K);
    cfma(acc, t2(kk, kl, kd, k, l, d, c0), lam.two(kk, kl, kd, k, l, d, a));
  }
  block_store_sum(acc, h + a);
}

// b and e vectors of orbital p at momentum K (either pointer may be null).
int build_vectors(ccgf_ctx *c, int part, int K, int p, cplx *bv, cplx *ev) {
  const int nk = c->nk, no = c->no, nv = c->nv;
  hipStream_t s = c->stream;
  KTab kt{nk, c->kc3};
  T2d t1{c->t1, no, nv};
  T4 t2{c->t2, nk, no, no, nv, nv};
  const Lam lam{t1, t2, c->l1, c->l2};
  const size_t n = (size_t)vec_len(c, part);
  if (part == CCGF_PART_IP) {
    // IP layout: [r1[i]], r2[ki][kj][i][j][a], ka = ki + kj - K
    const size_t n2 = (size_t)no * no * nv;
    if (bv) {
      foreach_(s, n, [=] __device__(size_t x) {
        cplx v = mkc(0, 0);
        if (x < (size_t)no) {
          if (p < no) v = mkc(x == (size_t)p ? 1.0 : 0.0, 0);
          else v = t1(K, (int)x, p - no);
        } else if (p >= no) {
          size_t y = x - no;
          size_t blk = y / n2, r = y % n2;
          int ki = (int)(blk / nk), kj = (int)(blk % nk);
          int a = (int)(r % nv), j = (int)((r / nv) % no), ii = (int)(r / ((size_t)nv * no));
          int ka = kt.c3(ki, kj, K);
          cplx tv = t2(ki, kj, ka, ii, j, a, p - no);
          v = mkc(-tv.x, -tv.y);
        }
        bv[x] = v;
      });
    }
    if (ev) {
      if (!c->e_overlap) c->e_overlap = (cplx *)dev_alloc(c, sizeof(cplx) * (size_t)std::max(no, nv));
      if (!c->e_overlap) return CCGF_ENOMEM;
      cplx *hov = c->e_overlap;
      if (p < no) hipLaunchKernelGGL(k_t2_overlap, dim3(no), dim3(256), 0, s, t2, lam, K, p, hov);
      foreach_(s, n, [=] __device__(size_t x) {
        cplx v = mkc(0, 0);
        if (x < (size_t)no) {
          int ii = (int)x;
          if (p >= no) {
            v = lam.one(K, ii, p - no);
          } else {
            v = mkc(ii == p ? 1.0 : 0.0, 0);
            for (int cc = 0; cc < nv; ++cc) v = csub(v, cmul(t1(K, p, cc), lam.one(K, ii, cc)));
            v = csub(v, cscale(hov[ii], 0.5));
          }
        } else {
          size_t y = x - no;
          size_t blk = y / n2, r = y % n2;
          int ki = (int)(blk / nk), kj = (int)(blk % nk);
          int a = (int)(r % nv), j = (int)((r / nv) % no), ii = (int)(r / ((size_t)nv * no));
          if (p >= no) {
            v = lam.two(ki, kj, K, ii, j, p - no, a);
          } else {
            if (ki == K && ii == p) v = cadd(v, lam.one(kj, j, a));
            if (kj == K && j == p) v = csub(v, lam.one(ki, ii, a));
            for (int cc = 0; cc < nv; ++cc) v = csub(v, cmul(t1(K, p, cc), lam.two(ki, kj, K, ii, j, cc, a)));
          }
        }
        ev[x] = v;
      });
    }
  } else {
    // EA layout: [r1[a]], r2[ki][ka][i][a][b], kb = K + ki - ka
    const size_t n2 = (size_t)no * nv * nv;
    if (bv) {
      foreach_(s, n, [=] __device__(size_t x) {
        cplx v = mkc(0, 0);
        if (x < (size_t)nv) {
          if (p >= no) v = mkc((int)x == p - no ? 1.0 : 0.0, 0);
          else {
            cplx tv = t1(K, p, (int)x);
            v = mkc(-tv.x, -tv.y);
          }
        } else if (p < no) {
          size_t y = x - nv;
          size_t blk = y / n2, r = y % n2;
          int kl = (int)(blk / nk), ka = (int)(blk % nk);
          int b = (int)(r % nv), a = (int)((r / nv) % nv), l = (int)(r / ((size_t)nv * nv));
          cplx tv = t2(K, kl, ka, p, l, a, b);
          v = mkc(-tv.x, -tv.y);
        }
        bv[x] = v;
      });
    }
    if (ev) {
      if (!c->e_overlap) c->e_overlap = (cplx *)dev_alloc(c, sizeof(cplx) * (size_t)std::max(no, nv));
      if (!c->e_overlap) return CCGF_ENOMEM;
      cplx *hov = c->e_overlap;
      if (p >= no) hipLaunchKernelGGL(k_t2_overlap_ea, dim3(nv), dim3(256), 0, s, t2, lam, kt, K, p - no, hov);
      foreach_(s, n, [=] __device__(size_t x) {
        cplx v = mkc(0, 0);
        if (x < (size_t)nv) {
          int a = (int)x;
          if (p < no) {
            cplx q = lam.one(K, p, a);
            v = mkc(-q.x, -q.y);
          } else {
            int c0 = p - no;
            v = mkc(a == c0 ? 1.0 : 0.0, 0);
            for (int j = 0; j < no; ++j) v = csub(v, cmul(t1(K, j, c0), lam.one(K, j, a)));
            v = csub(v, cscale(hov[a], 0.5));
          }
        } else {
          size_t y = x - nv;
          size_t blk = y / n2, r = y % n2;
          int ki = (int)(blk / nk), ka = (int)(blk % nk);
          int b = (int)(r % nv), a = (int)((r / nv) % nv), ii = (int)(r / ((size_t)nv * nv));
          int kb = kt.c3(K, ki, ka);
          if (p < no) {
            v = lam.two(ki, K, ka, ii, p, a, b);
          } else {
            int c0 = p - no;
            if (ka == K && a == c0) v = cadd(v, lam.one(ki, ii, b));
            if (kb == K && b == c0) v = csub(v, lam.one(ki, ii, a));
            for (int j = 0; j < no; ++j) cfma(v, t1(K, j, c0), lam.two(ki, K, ka, ii, j, a, b));
          }
        }
        ev[x] = v;
      });
    }
  }
  return hip_check(c, hipGetLastError(), "building b/e vectors");
}
