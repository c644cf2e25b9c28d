// C ABI of the CCGF library: argument checking, upload, context life cycle and
// the frequency / orbital / momentum loops of cc_gf_solve (Eqs. 6, 7, 9).
#include <chrono>
#include <exception>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ccgf_internal.h"

static thread_local std::string g_init_err = "no error";

int set_err(ccgf_ctx *c, int code, const std::string &msg) {
  if (c) c->err = msg;
  else g_init_err = msg;
  return code;
}

int hip_check(ccgf_ctx *c, hipError_t e, const char *what) {
  if (e == hipSuccess) return CCGF_OK;
  return set_err(c, CCGF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void *dev_alloc(ccgf_ctx *c, size_t bytes) {
  void *p = nullptr;
  if (hipMalloc(&p, bytes < 16 ? 16 : bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  c->allocs.push_back(p);
  return p;
}

static int kflat(const int m[3], int a, int b, int c3) {
  a = ((a % m[0]) + m[0]) % m[0];
  b = ((b % m[1]) + m[1]) % m[1];
  c3 = ((c3 % m[2]) + m[2]) % m[2];
  return (a * m[1] + b) * m[2] + c3;
}

static void free_all(ccgf_ctx *c) {
  for (void *p : c->allocs)
    if (p) hipFree(p);
  c->allocs.clear();
}

// Host-side checks of the symmetry the formulation relies on (host inputs only).
static int validate_host(ccgf_ctx *c, const ccgf_system *s) {
  const int nk = c->nk, no = c->no, nv = c->nv, nmo = c->nmo, naux = c->naux;
  for (const double *t2 : {s->t2, s->l2}) {
    if (!t2) continue;
    const char *name = t2 == s->t2 ? "t2" : "l2";
    double amax = 0, dev = 0;
    auto T2 = [&](int ki, int kj, int ka, int i, int j, int a, int b, int comp) {
      size_t off = ((((((size_t)ki * nk + kj) * nk + ka) * no + i) * no + j) * nv + a) * nv + b;
      return t2[2 * off + comp];
    };
    for (int ki = 0; ki < nk; ++ki)
      for (int kj = 0; kj < nk; ++kj)
        for (int ka = 0; ka < nk; ++ka) {
          int kb = c->kc3_h[((size_t)ki * nk + kj) * nk + ka];
          for (int i = 0; i < no; ++i)
            for (int j = 0; j < no; ++j)
              for (int a = 0; a < nv; ++a)
                for (int b = 0; b < nv; ++b)
                  for (int q = 0; q < 2; ++q) {
                    double x = T2(ki, kj, ka, i, j, a, b, q);
                    amax = std::fmax(amax, std::fabs(x));
                    dev = std::fmax(dev, std::fabs(x + T2(kj, ki, ka, j, i, a, b, q)));
                    dev = std::fmax(dev, std::fabs(x + T2(ki, kj, kb, i, j, b, a, q)));
                  }
        }
    if (dev > 1e-10 * std::fmax(amax, 1e-300) && dev > 0)
      return set_err(c, CCGF_EINVAL, std::string(name) + " is not antisymmetric under i<->j / a<->b (max deviation " +
                                         std::to_string(dev) + ")");
  }
  if (!s->eri_factor) {  // dense blocks: <pq|rs> = conj(<rs|pq>) and <pq|rs> = <qp|sr>
    const double *D = s->eri_blocks;
    auto off = [&](int k1, int k2, int k3, int p, int q, int r, int t) {
      return ((((((size_t)k1 * nk + k2) * nk + k3) * nmo + p) * nmo + q) * nmo + r) * nmo + t;
    };
    double amax = 0, dev = 0;
    for (int k1 = 0; k1 < nk; ++k1)
      for (int k2 = 0; k2 < nk; ++k2)
        for (int k3 = 0; k3 < nk; ++k3) {
          const int k4 = c->kc3_h[((size_t)k1 * nk + k2) * nk + k3];
          for (int p = 0; p < nmo; ++p)
            for (int q = 0; q < nmo; ++q)
              for (int r = 0; r < nmo; ++r)
                for (int t = 0; t < nmo; ++t) {
                  const size_t o = off(k1, k2, k3, p, q, r, t), h = off(k3, k4, k1, r, t, p, q),
                               x = off(k2, k1, k4, q, p, t, r);
                  amax = std::fmax(amax, std::fabs(D[2 * o]) + std::fabs(D[2 * o + 1]));
                  dev = std::fmax(dev, std::fabs(D[2 * o] - D[2 * h]) + std::fabs(D[2 * o + 1] + D[2 * h + 1]));
                  dev = std::fmax(dev, std::fabs(D[2 * o] - D[2 * x]) + std::fabs(D[2 * o + 1] - D[2 * x + 1]));
                }
        }
    if (dev > 1e-10 * std::fmax(amax, 1e-300) && dev > 0)
      return set_err(c, CCGF_EINVAL, "eri_blocks violate <pq|rs> = conj(<rs|pq>) or <pq|rs> = <qp|sr>");
    return CCGF_OK;
  }
  const double *A = s->eri_factor;
  double amax = 0, dev = 0;
  for (int k1 = 0; k1 < nk; ++k1)
    for (int k3 = 0; k3 < nk; ++k3)
      for (int L = 0; L < naux; ++L)
        for (int p = 0; p < nmo; ++p)
          for (int r = 0; r < nmo; ++r) {
            size_t o1 = ((((size_t)k1 * nk + k3) * naux + L) * nmo + p) * nmo + r;
            size_t o2 = ((((size_t)k3 * nk + k1) * naux + L) * nmo + r) * nmo + p;
            amax = std::fmax(amax, std::fabs(A[2 * o1]) + std::fabs(A[2 * o1 + 1]));
            dev = std::fmax(dev, std::fabs(A[2 * o1] - A[2 * o2]) + std::fabs(A[2 * o1 + 1] + A[2 * o2 + 1]));
          }
  if (dev > 1e-10 * std::fmax(amax, 1e-300) && dev > 0)
    return set_err(c, CCGF_EINVAL, "eri_factor violates A[k3][k1][L][r][p] = conj(A[k1][k3][L][p][r])");
  return CCGF_OK;
}

static int cc_gf_init_impl(const ccgf_system *s, const ccgf_options *opt, ccgf_ctx **out) {
  if (!out) return set_err(nullptr, CCGF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!s) return set_err(nullptr, CCGF_EINVAL, "system is NULL");
  for (int d = 0; d < 3; ++d)
    if (s->kmesh[d] < 1) return set_err(nullptr, CCGF_EINVAL, "kmesh entries must be >= 1");
  if (s->nocc < 1 || s->nvir < 1) return set_err(nullptr, CCGF_EINVAL, "nocc and nvir must be >= 1");
  if ((s->eri_factor == nullptr) == (s->eri_blocks == nullptr))
    return set_err(nullptr, CCGF_EINVAL, "give exactly one of eri_factor and eri_blocks");
  if (s->eri_factor && s->naux < 1) return set_err(nullptr, CCGF_EINVAL, "naux must be >= 1");
  if (!s->eps || !s->t1 || !s->t2) return set_err(nullptr, CCGF_EINVAL, "eps, t1 and t2 are required");
  if (s->mem_space != CCGF_HOST && s->mem_space != CCGF_DEVICE)
    return set_err(nullptr, CCGF_EINVAL, "mem_space must be CCGF_HOST or CCGF_DEVICE");
  if ((s->l1 == nullptr) != (s->l2 == nullptr))
    return set_err(nullptr, CCGF_EINVAL, "give both l1 and l2, or neither (Lambda = T^dagger)");
  ccgf_options o{};
  if (opt) o = *opt;
  if (o.precision != CCGF_PLAIN_F64 && o.precision != CCGF_MIXED_F32 && o.precision != CCGF_MIXED_BF16X3)
    return set_err(nullptr, CCGF_EUNSUPPORTED, "precision must be CCGF_PLAIN_F64, CCGF_MIXED_F32 or CCGF_MIXED_BF16X3");
  if (o.restart_m == 0) o.restart_m = 30;
  if (o.maxiter == 0) o.maxiter = 2000;
  if (o.tol == 0) o.tol = 1e-10;
  if (o.max_batch == 0) o.max_batch = 64;
  if (o.restart_m < 1 || o.restart_m > 2000 || o.maxiter < 1 || o.tol < 0 || o.max_batch < 1 ||
      o.recycle_k < 0 || o.recycle_k > 200 || o.precond_eta < 0 || o.reorth_ratio < 0 || o.reorth_ratio > 1 ||
      o.autotune < -1 || o.autotune > 0 || o.graphs < -1 || o.graphs > 0 || o.restart_tail < 0 ||
      o.restart_tail > 2000 || o.seed_m < 0 || o.seed_m > 2000)
    return set_err(nullptr, CCGF_EINVAL, "options out of range");

  ccgf_ctx *c = new ccgf_ctx();
  c->opt = o;
  if (o.autotune_cache) c->tune_path = o.autotune_cache;
  c->opt.autotune_cache = nullptr;  // the path is kept in the context
  tune_load(c);
  c->stream = (hipStream_t)o.hip_stream;
  for (int d = 0; d < 3; ++d) c->m[d] = s->kmesh[d];
  c->nk = s->kmesh[0] * s->kmesh[1] * s->kmesh[2];
  c->no = s->nocc;
  c->nv = s->nvir;
  c->nmo = s->nocc + s->nvir;
  c->naux = s->eri_factor ? s->naux : 0;
  const int nk = c->nk, no = c->no, nv = c->nv, nmo = c->nmo;
  // momentum table k1 + k2 - k3
  c->kc3_h.resize((size_t)nk * nk * nk);
  auto dec = [&](int k, int v[3]) {
    v[2] = k % c->m[2];
    v[1] = (k / c->m[2]) % c->m[1];
    v[0] = k / (c->m[1] * c->m[2]);
  };
  for (int a = 0; a < nk; ++a)
    for (int b = 0; b < nk; ++b)
      for (int d = 0; d < nk; ++d) {
        int va[3], vb[3], vd[3];
        dec(a, va);
        dec(b, vb);
        dec(d, vd);
        c->kc3_h[((size_t)a * nk + b) * nk + d] =
            kflat(c->m, va[0] + vb[0] - vd[0], va[1] + vb[1] - vd[1], va[2] + vb[2] - vd[2]);
      }
  if (s->mem_space == CCGF_HOST) {
    int rc = validate_host(c, s);
    if (rc != CCGF_OK) {
      g_init_err = c->err;
      delete c;
      return rc;
    }
  }
  const hipMemcpyKind kind = s->mem_space == CCGF_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  auto upload = [&](const void *src, size_t bytes) -> cplx * {
    cplx *d = (cplx *)dev_alloc(c, bytes);
    if (!d) return nullptr;
    if (hipMemcpyAsync(d, src, bytes, kind, c->stream) != hipSuccess) return nullptr;
    return d;
  };
  size_t n_t1 = (size_t)nk * no * nv, n_t2 = (size_t)nk * nk * nk * no * no * nv * nv;
  size_t n_fac = (size_t)nk * nk * c->naux * nmo * nmo;
  size_t n_dense = (size_t)nk * nk * nk * nmo * nmo * nmo * nmo;
  c->kc3 = (int *)dev_alloc(c, sizeof(int) * c->kc3_h.size());
  if (c->kc3) hipMemcpy(c->kc3, c->kc3_h.data(), sizeof(int) * c->kc3_h.size(), hipMemcpyHostToDevice);
  c->t1 = upload(s->t1, sizeof(cplx) * n_t1);
  c->t2 = upload(s->t2, sizeof(cplx) * n_t2);
  bool lam_ok = true;
  if (s->l1) {
    c->l1 = upload(s->l1, sizeof(cplx) * n_t1);
    c->l2 = upload(s->l2, sizeof(cplx) * n_t2);
    lam_ok = c->l1 && c->l2;
  }
  if (s->eri_factor) c->fac = upload(s->eri_factor, sizeof(cplx) * n_fac);
  else c->eri_dense = upload(s->eri_blocks, sizeof(cplx) * n_dense);
  // Fock blocks: given, or diag(eps)
  std::vector<cplx> hfoo((size_t)nk * no * no, mkc(0, 0)), hfvv((size_t)nk * nv * nv, mkc(0, 0));
  std::vector<double> heps((size_t)nk * nmo);
  if (s->mem_space == CCGF_HOST) std::memcpy(heps.data(), s->eps, sizeof(double) * heps.size());
  else hipMemcpy(heps.data(), s->eps, sizeof(double) * heps.size(), hipMemcpyDeviceToHost);
  for (int k = 0; k < nk; ++k) {
    for (int i = 0; i < no; ++i) hfoo[((size_t)k * no + i) * no + i] = mkc(heps[(size_t)k * nmo + i], 0);
    for (int a = 0; a < nv; ++a) hfvv[((size_t)k * nv + a) * nv + a] = mkc(heps[(size_t)k * nmo + no + a], 0);
  }
  c->foo = (cplx *)dev_alloc(c, sizeof(cplx) * hfoo.size());
  c->fvv = (cplx *)dev_alloc(c, sizeof(cplx) * hfvv.size());
  if (c->foo && c->fvv) {
    if (s->foo) hipMemcpy(c->foo, s->foo, sizeof(cplx) * hfoo.size(), kind);
    else hipMemcpy(c->foo, hfoo.data(), sizeof(cplx) * hfoo.size(), hipMemcpyHostToDevice);
    if (s->fvv) hipMemcpy(c->fvv, s->fvv, sizeof(cplx) * hfvv.size(), kind);
    else hipMemcpy(c->fvv, hfvv.data(), sizeof(cplx) * hfvv.size(), hipMemcpyHostToDevice);
  }
  if (!c->kc3 || !c->t1 || !c->t2 || (!c->fac && !c->eri_dense) || !c->foo || !c->fvv || !lam_ok) {
    g_init_err = "device allocation or upload failed";
    free_all(c);
    delete c;
    return CCGF_ENOMEM;
  }
  int rc = build_hbar(c);
  if (rc == CCGF_OK) rc = hip_check(c, hipStreamSynchronize(c->stream), "cc_gf_init");
  if (rc != CCGF_OK) {
    g_init_err = c->err.empty() ? "building Hbar failed (out of device memory?)" : c->err;
    free_all(c);
    delete c;
    return rc;
  }
  *out = c;
  return CCGF_OK;
}

extern "C" int cc_gf_vector_size(const ccgf_ctx *c, int part, long long *n) {
  if (!c) return CCGF_ESTATE;
  if (!n || (part != CCGF_PART_IP && part != CCGF_PART_EA)) return CCGF_EINVAL;
  *n = vec_len(c, part);
  return CCGF_OK;
}

static int cc_gf_sigma_impl(ccgf_ctx *c, int part, int K, int nvec, const double *x, double *y) {
  if (!c) return CCGF_ESTATE;
  if (part != CCGF_PART_IP && part != CCGF_PART_EA) return set_err(c, CCGF_EINVAL, "part must be IP or EA");
  if (K < 0 || K >= c->nk) return set_err(c, CCGF_EINVAL, "K out of range");
  if (nvec < 0 || (nvec > 0 && (!x || !y))) return set_err(c, CCGF_EINVAL, "bad vectors");
  if (x == y && nvec > 0) return set_err(c, CCGF_EINVAL, "x and y must not alias");
  int rc = sigma_apply(c, part, K, nvec, (const cplx *)x, (cplx *)y, c->opt.precision);
  if (rc != CCGF_OK) return rc;
  return hip_check(c, hipStreamSynchronize(c->stream), "cc_gf_sigma");
}

static int cc_gf_sigma_group_impl(int nsys, ccgf_ctx *const *ctxs, const int *parts, const int *K, const int *nvec,
                                 const double *const *x, double *const *y) {
  if (nsys < 1 || !ctxs || !ctxs[0]) return CCGF_ESTATE;
  ccgf_ctx *c0 = ctxs[0];
  if (!parts || !K || !nvec || !x || !y) return set_err(c0, CCGF_EINVAL, "NULL array argument");
  if (c0->opt.precision == CCGF_MIXED_BF16X3)
    return set_err(c0, CCGF_EUNSUPPORTED, "grouped products run in FP64 or FP32");
  for (int i = 0; i < nsys; ++i) {
    ccgf_ctx *c = ctxs[i];
    if (!c) return set_err(c0, CCGF_ESTATE, "NULL context");
    if (c->opt.precision != c0->opt.precision) return set_err(c0, CCGF_EINVAL, "systems differ in precision");
    if (parts[i] != CCGF_PART_IP && parts[i] != CCGF_PART_EA) return set_err(c0, CCGF_EINVAL, "part must be IP or EA");
    if (K[i] < 0 || K[i] >= c->nk) return set_err(c0, CCGF_EINVAL, "K out of range");
    if (nvec[i] < 0 || (nvec[i] > 0 && (!x[i] || !y[i]))) return set_err(c0, CCGF_EINVAL, "bad vectors");
    if (nvec[i] > 0 && x[i] == y[i]) return set_err(c0, CCGF_EINVAL, "x and y must not alias");
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == c) return set_err(c0, CCGF_EINVAL, "a context appears twice (its workspace is per product)");
  }
  // every context's own work is done before its workspace is reused on the first stream
  for (int i = 0; i < nsys; ++i)
    if (hip_check(c0, hipStreamSynchronize(ctxs[i]->stream), "cc_gf_sigma_group") != CCGF_OK) return CCGF_EDEVICE;
  int rc = sigma_group(nsys, ctxs, parts, K, nvec, (const cplx *const *)x, (cplx *const *)y);
  if (rc != CCGF_OK) return rc;
  return hip_check(c0, hipStreamSynchronize(c0->stream), "cc_gf_sigma_group");
}

static int cc_gf_vectors_impl(ccgf_ctx *c, int part, int K, int p, double *b, double *e) {
  if (!c) return CCGF_ESTATE;
  if (part != CCGF_PART_IP && part != CCGF_PART_EA) return set_err(c, CCGF_EINVAL, "part must be IP or EA");
  if (K < 0 || K >= c->nk || p < 0 || p >= c->nmo) return set_err(c, CCGF_EINVAL, "K or p out of range");
  int rc = build_vectors(c, part, K, p, (cplx *)b, (cplx *)e);
  if (rc != CCGF_OK) return rc;
  return hip_check(c, hipStreamSynchronize(c->stream), "cc_gf_vectors");
}

// The solves of cc_gf_solve and cc_gf_solve_matrix.  With Gmat (host [nkq][nw][norb][norb]) every
// solution is also dotted with every left vector of the call: G+_pq = e+_p . Y_q, G-_pq = e-_q . X_p.
static int solve_common(ccgf_ctx *c, int nkq, const int *kidx, int norb, const int *orbs, int nw,
                        const double *omega, double eta, int parts, double *G, double *Gp, double *Gm,
                        cplx *Gmat, cplx *Gpmat, cplx *Gmmat, ccgf_stats *st) {
  auto t0 = std::chrono::steady_clock::now();
  if (nkq < 0 || norb < 0 || nw < 0) return set_err(c, CCGF_EINVAL, "negative counts");
  if ((nkq && !kidx) || (norb && !orbs) || (nw && !omega) || !(G || Gmat))
    return set_err(c, CCGF_EINVAL, "NULL array argument");
  if (!(eta > 0)) return set_err(c, CCGF_EINVAL, "eta must be > 0");
  if (parts < 1 || parts > 3) return set_err(c, CCGF_EINVAL, "parts must be CCGF_PART_IP, _EA or _BOTH");
  for (int a = 0; a < nkq; ++a)
    if (kidx[a] < 0 || kidx[a] >= c->nk) return set_err(c, CCGF_EINVAL, "kidx out of range");
  for (int b = 0; b < norb; ++b)
    if (orbs[b] < 0 || orbs[b] >= c->nmo) return set_err(c, CCGF_EINVAL, "orbital index out of range");
  for (int w = 0; w < nw; ++w)
    if (!std::isfinite(omega[w])) return set_err(c, CCGF_EINVAL, "omega must be finite");
  ccgf_stats local{};
  ccgf_stats *S = st ? st : &local;
  std::memset(S, 0, sizeof(*S));
  c->t_big_ms = c->t_big_flops = c->t_big_bytes = c->t_sigma_ms = 0;
  c->t_big_launches = c->t_sigma_launches = 0;
  const size_t ntot = (size_t)nkq * norb * nw;
  std::vector<cplx> Gsum(ntot, mkc(0, 0)), Gplus(ntot, mkc(0, 0)), Gminus(ntot, mkc(0, 0));
  int status = CCGF_OK;
  const int nrhs = norb * nw;
  std::vector<int> rhs_orb(nrhs);
  std::vector<double> rhs_w(nrhs);
  for (int b = 0; b < norb; ++b)
    for (int w = 0; w < nw; ++w) {
      rhs_orb[b * nw + w] = b;
      rhs_w[b * nw + w] = omega[w];
    }
  std::vector<cplx> res(nrhs), cols(Gmat ? (size_t)nrhs * norb : 0);
  const size_t nmat = (size_t)norb * norb;
  if (Gmat) {
    std::fill(Gmat, Gmat + (size_t)nkq * nw * nmat, mkc(0, 0));
    if (Gpmat) std::fill(Gpmat, Gpmat + (size_t)nkq * nw * nmat, mkc(0, 0));
    if (Gmmat) std::fill(Gmmat, Gmmat + (size_t)nkq * nw * nmat, mkc(0, 0));
  }
  for (int part : {CCGF_PART_IP, CCGF_PART_EA}) {
    if (!(parts & part) || nrhs == 0) continue;
    const long long n = vec_len(c, part);
    cplx *Bv = (cplx *)nullptr, *Ev = (cplx *)nullptr;
    if (hipMalloc(&Bv, sizeof(cplx) * (size_t)norb * n) != hipSuccess ||
        hipMalloc(&Ev, sizeof(cplx) * (size_t)norb * n) != hipSuccess) {
      if (Bv) hipFree(Bv);
      (void)hipGetLastError();
      return set_err(c, CCGF_ENOMEM, "no device memory for right-hand sides");
    }
    for (int a = 0; a < nkq && status != CCGF_EDEVICE && status != CCGF_ENOMEM; ++a) {
      const int K = kidx[a];
      for (int b = 0; b < norb; ++b) {
        int rc = build_vectors(c, part, K, orbs[b], Bv + (size_t)b * n, Ev + (size_t)b * n);
        if (rc != CCGF_OK) status = rc;
      }
      if (status != CCGF_OK && status != CCGF_ENOCONV) break;
      Guess gs;
      const Guess *gp = nullptr;
      cplx *chat = nullptr;
      std::vector<double> peta;
      bool have_peta = false;
      for (const LearnModel &M : c->models)
        if (M.part == part && M.K == K) {
          if ((c->learn_on & CCGF_LEARN_GUESS) &&
              learn_guess(c, M, nrhs, rhs_orb.data(), orbs, rhs_w.data(), gs, &chat))
            gp = &gs;
          if (c->learn_on & CCGF_LEARN_PRECOND)
            have_peta = learn_precond(c, M, nrhs, rhs_orb.data(), orbs, rhs_w.data(), peta);
          break;
        }
      cplx *seedQ = nullptr;
      if (!gp && c->opt.seed_m > 0) {
        int rs = seed_krylov(c, part, K, norb, Bv, nrhs, rhs_orb.data(), rhs_w.data(), eta, gs, &seedQ, &chat, S);
        if (rs == CCGF_OK && seedQ) gp = &gs;
        else if (rs == CCGF_EDEVICE) {
          status = rs;
          break;
        }
      }
      int rc = solve_batched(c, part, K, nrhs, rhs_orb.data(), rhs_w.data(), eta, Bv, Ev, res.data(), S, nullptr, gp,
                             Gmat ? cols.data() : nullptr, Gmat ? norb : 0, have_peta ? peta.data() : nullptr);
      if (chat) hipFree(chat);
      if (seedQ) hipFree(seedQ);
      if (rc != CCGF_OK) {
        if (rc == CCGF_ENOCONV) set_err(c, rc, "some shifted systems did not reach tol");
        status = (status == CCGF_OK || rc != CCGF_ENOCONV) ? rc : status;
        if (rc != CCGF_ENOCONV) break;
      }
      for (int r = 0; r < nrhs; ++r) {
        size_t o = ((size_t)a * norb + rhs_orb[r]) * nw + (r % nw);
        Gsum[o] = cadd(Gsum[o], res[r]);
        if (part == CCGF_PART_EA) Gplus[o] = res[r];
        else Gminus[o] = res[r];
      }
      if (Gmat)
        for (int r = 0; r < nrhs; ++r) {
          const int b = rhs_orb[r], w = r % nw;
          cplx *Ga = Gmat + ((size_t)a * nw + w) * nmat;
          cplx *Gpart = part == CCGF_PART_EA ? Gpmat : Gmmat;
          if (Gpart) Gpart += ((size_t)a * nw + w) * nmat;
          for (int q = 0; q < norb; ++q) {
            // EA: column b of G+ (Y of orbital b against e+_q); IP: row b of G- (X of b against e-_q)
            const size_t o = part == CCGF_PART_EA ? (size_t)q * norb + b : (size_t)b * norb + q;
            const cplx v = cols[(size_t)r * norb + q];
            Ga[o] = cadd(Ga[o], v);
            if (Gpart) Gpart[o] = v;
          }
        }
    }
    hipFree(Bv);
    hipFree(Ev);
    if (status != CCGF_OK && status != CCGF_ENOCONV) break;
  }
  if (G) std::memcpy(G, Gsum.data(), sizeof(cplx) * ntot);
  if (Gp) std::memcpy(Gp, Gplus.data(), sizeof(cplx) * ntot);
  if (Gm) std::memcpy(Gm, Gminus.data(), sizeof(cplx) * ntot);
  S->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  timing_harvest(c);
  S->big_ms = c->t_big_ms;
  S->big_launches = c->t_big_launches;
  S->big_flops = c->t_big_flops;
  S->big_bytes = c->t_big_bytes;
  S->sigma_ms = c->t_sigma_ms;
  S->sigma_launches = c->t_sigma_launches;
  return status;
}

static int cc_gf_solve_impl(ccgf_ctx *c, int nkq, const int *kidx, int norb, const int *orbs, int nw,
                           const double *omega, double eta, int parts, double *G, double *Gp, double *Gm,
                           ccgf_stats *st) {
  if (!c) return CCGF_ESTATE;
  if (!G) return set_err(c, CCGF_EINVAL, "NULL array argument");
  return solve_common(c, nkq, kidx, norb, orbs, nw, omega, eta, parts, G, Gp, Gm, nullptr, nullptr, nullptr, st);
}

static int cc_gf_solve_matrix_impl(ccgf_ctx *c, int nkq, const int *kidx, int norb, const int *orbs, int nw,
                                  const double *omega, double eta, int parts, double *G, double *Gp, double *Gm,
                                  double *dos, ccgf_stats *st) {
  if (!c) return CCGF_ESTATE;
  if (!G) return set_err(c, CCGF_EINVAL, "NULL array argument");
  if (nkq < 0 || norb < 0 || nw < 0) return set_err(c, CCGF_EINVAL, "negative counts");
  // the parts are kept for the density of states even when the caller does not want them
  const size_t nm = (size_t)nkq * nw * norb * norb;
  std::vector<cplx> lp(dos && !Gp ? nm : 0), lm(dos && !Gm ? nm : 0);
  cplx *P = Gp ? (cplx *)Gp : (dos ? lp.data() : nullptr);
  cplx *Q = Gm ? (cplx *)Gm : (dos ? lm.data() : nullptr);
  int rc = solve_common(c, nkq, kidx, norb, orbs, nw, omega, eta, parts, nullptr, nullptr, nullptr, (cplx *)G, P, Q,
                        st);
  if (dos && (rc == CCGF_OK || rc == CCGF_ENOCONV)) {
    // A(K, w) = -(1/pi) Im G(K, w) with each part on the retarded side (G- of Eq. 6 is time
    // ordered: its imaginary part changes sign), traced over the requested orbitals
    for (int a = 0; a < nkq; ++a)
      for (int w = 0; w < nw; ++w) {
        double t = 0;
        for (int p = 0; p < norb; ++p) {
          const size_t o = (((size_t)a * nw + w) * norb + p) * norb + p;
          t += P[o].y - Q[o].y;
        }
        dos[(size_t)a * nw + w] = -t / M_PI;
      }
  }
  return rc;
}

static int cc_gf_mor_impl(ccgf_ctx *c, int nkq, const int *kidx, int norb, const int *orbs, int nexp_ip,
                         const double *wexp_ip, int nexp_ea, const double *wexp_ea, int nw, const double *omega,
                         double eta, int parts, double *G, double *Gp, double *Gm, ccgf_stats *st) {
  if (!c) return CCGF_ESTATE;
  auto t0 = std::chrono::steady_clock::now();
  if (nkq < 0 || norb < 0 || nw < 0) return set_err(c, CCGF_EINVAL, "negative counts");
  if ((nkq && !kidx) || (norb && !orbs) || (nw && !omega) || !G)
    return set_err(c, CCGF_EINVAL, "NULL array argument");
  if (!(eta > 0)) return set_err(c, CCGF_EINVAL, "eta must be > 0");
  if (parts < 1 || parts > 3) return set_err(c, CCGF_EINVAL, "parts must be CCGF_PART_IP, _EA or _BOTH");
  for (int part : {CCGF_PART_IP, CCGF_PART_EA}) {
    if (!(parts & part)) continue;
    const int ne = part == CCGF_PART_IP ? nexp_ip : nexp_ea;
    const double *we = part == CCGF_PART_IP ? wexp_ip : wexp_ea;
    if (ne < 1 || ne > CCGF_MOR_MAX) return set_err(c, CCGF_EINVAL, "expansion point count must be in 1..32");
    if (!we) return set_err(c, CCGF_EINVAL, "NULL expansion frequencies");
    for (int j = 0; j < ne; ++j)
      if (!std::isfinite(we[j])) return set_err(c, CCGF_EINVAL, "expansion frequencies must be finite");
  }
  for (int a = 0; a < nkq; ++a)
    if (kidx[a] < 0 || kidx[a] >= c->nk) return set_err(c, CCGF_EINVAL, "kidx out of range");
  for (int b = 0; b < norb; ++b)
    if (orbs[b] < 0 || orbs[b] >= c->nmo) return set_err(c, CCGF_EINVAL, "orbital index out of range");
  for (int w = 0; w < nw; ++w)
    if (!std::isfinite(omega[w])) return set_err(c, CCGF_EINVAL, "omega must be finite");
  ccgf_stats local{};
  ccgf_stats *S = st ? st : &local;
  std::memset(S, 0, sizeof(*S));
  c->t_big_ms = c->t_big_flops = c->t_big_bytes = c->t_sigma_ms = 0;
  c->t_big_launches = c->t_sigma_launches = 0;
  const size_t ntot = (size_t)nkq * norb * nw;
  std::vector<cplx> Gsum(ntot, mkc(0, 0)), Gplus(ntot, mkc(0, 0)), Gminus(ntot, mkc(0, 0));
  std::vector<cplx> res((size_t)norb * nw);
  int status = CCGF_OK;
  for (int part : {CCGF_PART_IP, CCGF_PART_EA}) {
    if (!(parts & part) || norb == 0) continue;
    const int ne = part == CCGF_PART_IP ? nexp_ip : nexp_ea;
    const double *we = part == CCGF_PART_IP ? wexp_ip : wexp_ea;
    for (int a = 0; a < nkq; ++a) {
      int rc = mor_part(c, part, kidx[a], norb, orbs, ne, we, nw, omega, eta, res.data(), S);
      if (rc != CCGF_OK) {
        if (rc == CCGF_ENOCONV) set_err(c, rc, "some expansion-point solves did not reach tol");
        status = (status == CCGF_OK || rc != CCGF_ENOCONV) ? rc : status;
        if (rc != CCGF_ENOCONV) break;
      }
      for (int b = 0; b < norb; ++b)
        for (int w = 0; w < nw; ++w) {
          size_t o = ((size_t)a * norb + b) * nw + w;
          cplx g = res[(size_t)b * nw + w];
          Gsum[o] = cadd(Gsum[o], g);
          if (part == CCGF_PART_EA) Gplus[o] = g;
          else Gminus[o] = g;
        }
    }
    if (status != CCGF_OK && status != CCGF_ENOCONV) break;
  }
  std::memcpy(G, Gsum.data(), sizeof(cplx) * ntot);
  if (Gp) std::memcpy(Gp, Gplus.data(), sizeof(cplx) * ntot);
  if (Gm) std::memcpy(Gm, Gminus.data(), sizeof(cplx) * ntot);
  S->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  timing_harvest(c);
  S->big_ms = c->t_big_ms;
  S->big_launches = c->t_big_launches;
  S->big_flops = c->t_big_flops;
  S->big_bytes = c->t_big_bytes;
  S->sigma_ms = c->t_sigma_ms;
  S->sigma_launches = c->t_sigma_launches;
  return status;
}

static int cc_gf_learn_impl(ccgf_ctx *c, int parts, int K, int norb, const int *orbs, int ntrain, const double *wtr,
                           double eta, const ccgf_learn_options *opt, ccgf_learn_stats *st) {
  if (!c) return CCGF_ESTATE;
  if (parts < 1 || parts > 3) return set_err(c, CCGF_EINVAL, "parts must be CCGF_PART_IP, _EA or _BOTH");
  if (K < 0 || K >= c->nk) return set_err(c, CCGF_EINVAL, "K out of range");
  if (norb < 1 || !orbs) return set_err(c, CCGF_EINVAL, "no orbitals");
  for (int b = 0; b < norb; ++b)
    if (orbs[b] < 0 || orbs[b] >= c->nmo) return set_err(c, CCGF_EINVAL, "orbital index out of range");
  if (ntrain < 1 || ntrain > 32 || !wtr) return set_err(c, CCGF_EINVAL, "ntrain must be in 1..32");
  for (int j = 0; j < ntrain; ++j)
    if (!std::isfinite(wtr[j]) || (j > 0 && !(wtr[j] > wtr[j - 1])))
      return set_err(c, CCGF_EINVAL, "training frequencies must be finite and strictly ascending");
  if (!(eta > 0)) return set_err(c, CCGF_EINVAL, "eta must be > 0");
  ccgf_learn_options lo{};
  if (opt) lo = *opt;
  if (lo.epochs == 0) lo.epochs = 300;
  if (lo.batch == 0) lo.batch = 256;
  if (lo.lr == 0) lo.lr = 1e-3;
  if (lo.hidden == 0) lo.hidden = 256;
  if (lo.accept == 0) lo.accept = 0.1;
  if (lo.probe == 0) lo.probe = 40;
  if (lo.epochs < 0 || lo.batch < 1 || !(lo.lr > 0) || lo.hidden < 1 || lo.hidden > 4096 ||
      (lo.guess != CCGF_GUESS_NETWORK && lo.guess != CCGF_GUESS_NEAREST) || !(lo.accept > 0) || lo.accept > 1 ||
      lo.probe < -1 || lo.probe > 2000)
    return set_err(c, CCGF_EINVAL, "learning options out of range");
  ccgf_learn_stats local{};
  ccgf_learn_stats *S = st ? st : &local;
  std::memset(S, 0, sizeof(*S));
  int status = CCGF_OK;
  c->learn_on = CCGF_LEARN_GUESS | CCGF_LEARN_PRECOND;  // a fresh model is used until disabled
  for (int part : {CCGF_PART_IP, CCGF_PART_EA}) {
    if (!(parts & part)) continue;
    int rc = learn_part(c, part, K, norb, orbs, ntrain, wtr, eta, lo, S);
    if (rc == CCGF_ENOCONV) {
      set_err(c, rc, "some training solves did not reach tol");
      status = rc;
    } else if (rc != CCGF_OK) {
      return rc;
    }
  }
  return status;
}

static int cc_gf_set_options_impl(ccgf_ctx *c, const ccgf_options *opt) {
  if (!c) return CCGF_ESTATE;
  if (!opt) return set_err(c, CCGF_EINVAL, "options are NULL");
  ccgf_options o = *opt;
  if (o.precision != c->opt.precision)
    return set_err(c, CCGF_EUNSUPPORTED, "the precision is fixed when the context is built");
  if (o.restart_m == 0) o.restart_m = 30;
  if (o.maxiter == 0) o.maxiter = 2000;
  if (o.tol == 0) o.tol = 1e-10;
  if (o.max_batch == 0) o.max_batch = 64;
  if (o.restart_m < 1 || o.restart_m > 2000 || o.maxiter < 1 || o.tol < 0 || o.max_batch < 1 ||
      o.recycle_k < 0 || o.recycle_k > 200 || o.precond_eta < 0 || o.reorth_ratio < 0 || o.reorth_ratio > 1 ||
      o.autotune < -1 || o.autotune > 0 || o.graphs < -1 || o.graphs > 0 || o.restart_tail < 0 ||
      o.restart_tail > 2000 || o.seed_m < 0 || o.seed_m > 2000)
    return set_err(c, CCGF_EINVAL, "options out of range");
  if (hip_check(c, hipStreamSynchronize(c->stream), "cc_gf_set_options") != CCGF_OK) return CCGF_EDEVICE;
  if (o.hip_stream != c->opt.hip_stream) c->stream = (hipStream_t)o.hip_stream;
  o.autotune_cache = nullptr;  // the autotune file stays the one given to cc_gf_init
  c->opt = o;
  return CCGF_OK;
}

extern "C" int cc_gf_learn_enable(ccgf_ctx *c, int on) {
  if (!c) return CCGF_ESTATE;
  if (on < 0 || on > (CCGF_LEARN_GUESS | CCGF_LEARN_PRECOND))
    return set_err(c, CCGF_EINVAL, "on must be a mask of CCGF_LEARN_GUESS and CCGF_LEARN_PRECOND");
  c->learn_on = on;
  return CCGF_OK;
}

// ---------------------------------------------------------------- trained networks on disk
static const char kNetMagic[8] = {'C', 'C', 'G', 'F', 'N', 'E', 'T', '1'};
static const int kNetVersion = 1;

static void free_model(LearnModel &M) {
  if (M.Q) hipFree(M.Q);
  if (M.theta) hipFree(M.theta);
  if (M.theta_p) hipFree(M.theta_p);
  M.Q = nullptr;
  M.theta = M.theta_p = nullptr;
}

static int learn_save_impl(ccgf_ctx *c, const char *path) {
  if (!c) return CCGF_ESTATE;
  if (!path) return set_err(c, CCGF_EINVAL, "path is NULL");
  if (c->models.empty()) return set_err(c, CCGF_ESTATE, "no trained networks to save (call cc_gf_learn)");
  if (int rc = hip_check(c, hipStreamSynchronize(c->stream), "learn_save")) return rc;
  FILE *f = std::fopen(path, "wb");
  if (!f) return set_err(c, CCGF_EINVAL, std::string("cannot open ") + path + " for writing");
  bool ok = true;
  auto put = [&](const void *p, size_t b) { ok = ok && (b == 0 || std::fwrite(p, 1, b, f) == b); };
  put(kNetMagic, 8);
  const int hdr[5] = {kNetVersion, c->nk, c->no, c->nv, (int)c->models.size()};
  put(hdr, sizeof hdr);
  for (const LearnModel &M : c->models) {
    const int iv[11] = {M.part, M.K, M.norb, M.ntrain, M.R, M.din, M.dout, M.hidden, M.mode, M.pdin, M.pdout};
    const double dv[4] = {M.accept, M.wscale, M.wstep, M.pbase};
    put(iv, sizeof iv);
    put(dv, sizeof dv);
    put(M.orbs.data(), sizeof(int) * M.norb);
    put(M.occ.data(), sizeof(int) * M.norb);
    put(M.fpp.data(), sizeof(double) * M.norb);
    put(M.wtrain.data(), sizeof(double) * M.ntrain);
    put(M.scale.data(), sizeof(double) * M.norb);
    put(M.C.data(), sizeof(cplx) * M.C.size());
    const long long n = vec_len(c, M.part);
    put(&n, sizeof n);
    std::vector<cplx> hq((size_t)M.R * n);  // one orbital's basis at a time
    for (int b = 0; b < M.norb && ok; ++b) {
      ok = hipMemcpy(hq.data(), M.Q + (size_t)b * hq.size(), sizeof(cplx) * hq.size(), hipMemcpyDeviceToHost) ==
           hipSuccess;
      put(hq.data(), sizeof(cplx) * hq.size());
    }
    const long long np = mlp_nparams(M.din, M.hidden, M.dout);
    const long long npp = M.theta_p ? mlp_nparams(M.pdin, M.hidden, M.pdout) : 0;
    std::vector<float> th((size_t)std::max(np, npp));
    put(&np, sizeof np);
    ok = ok && hipMemcpy(th.data(), M.theta, sizeof(float) * np, hipMemcpyDeviceToHost) == hipSuccess;
    put(th.data(), sizeof(float) * np);
    put(&npp, sizeof npp);
    if (npp) {
      ok = ok && hipMemcpy(th.data(), M.theta_p, sizeof(float) * npp, hipMemcpyDeviceToHost) == hipSuccess;
      put(th.data(), sizeof(float) * npp);
    }
  }
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return set_err(c, CCGF_EINVAL, std::string("writing ") + path + " failed");
  return CCGF_OK;
}

static int learn_load_impl(ccgf_ctx *c, const char *path) {
  if (!c) return CCGF_ESTATE;
  if (!path) return set_err(c, CCGF_EINVAL, "path is NULL");
  FILE *f = std::fopen(path, "rb");
  if (!f) return set_err(c, CCGF_EINVAL, std::string("cannot open ") + path);
  bool ok = true;
  auto get = [&](void *p, size_t b) { ok = ok && (b == 0 || std::fread(p, 1, b, f) == b); };
  std::string why;
  char magic[8];
  int hdr[5] = {0, 0, 0, 0, 0};
  get(magic, 8);
  get(hdr, sizeof hdr);
  if (ok && (std::memcmp(magic, kNetMagic, 8) != 0 || hdr[0] != kNetVersion))
    why = "not a network file of this version";
  else if (ok && (hdr[1] != c->nk || hdr[2] != c->no || hdr[3] != c->nv))
    why = "the networks were trained on another system shape";
  else if (ok && (hdr[4] < 1 || hdr[4] > 2 * c->nk)) why = "bad model count";
  std::vector<LearnModel> models;
  auto fail = [&](const std::string &m) {
    for (LearnModel &M : models) free_model(M);
    std::fclose(f);
    return set_err(c, CCGF_EINVAL, std::string(path) + ": " + m);
  };
  if (!ok) return fail("truncated header");
  if (!why.empty()) return fail(why);
  for (int q = 0; q < hdr[4]; ++q) {
    models.emplace_back();
    LearnModel &M = models.back();
    int iv[11];
    double dv[4];
    get(iv, sizeof iv);
    get(dv, sizeof dv);
    if (!ok) return fail("truncated model header");
    M.part = iv[0], M.K = iv[1], M.norb = iv[2], M.ntrain = iv[3], M.R = iv[4], M.din = iv[5], M.dout = iv[6];
    M.hidden = iv[7], M.mode = iv[8], M.pdin = iv[9], M.pdout = iv[10];
    M.accept = dv[0], M.wscale = dv[1], M.wstep = dv[2], M.pbase = dv[3];
    if ((M.part != CCGF_PART_IP && M.part != CCGF_PART_EA) || M.K < 0 || M.K >= c->nk || M.norb < 1 ||
        M.norb > c->nmo || M.ntrain < 1 || M.ntrain > 32 || M.R < 1 || M.R > 4096 || M.din < 1 || M.dout < 1 ||
        M.hidden < 1 || M.hidden > 4096 || M.pdin < 0 || M.pdout < 0 || M.dout > 4096 || M.din > 4096)
      return fail("model dimensions out of range");
    M.orbs.resize(M.norb);
    M.occ.resize(M.norb);
    M.fpp.resize(M.norb);
    M.wtrain.resize(M.ntrain);
    M.scale.resize(M.norb);
    M.C.resize((size_t)M.norb * M.ntrain * M.R);
    get(M.orbs.data(), sizeof(int) * M.norb);
    get(M.occ.data(), sizeof(int) * M.norb);
    get(M.fpp.data(), sizeof(double) * M.norb);
    get(M.wtrain.data(), sizeof(double) * M.ntrain);
    get(M.scale.data(), sizeof(double) * M.norb);
    get(M.C.data(), sizeof(cplx) * M.C.size());
    long long n = 0;
    get(&n, sizeof n);
    if (!ok) return fail("truncated model");
    if (n != vec_len(c, M.part)) return fail("vector length differs from this system's");
    if ((double)M.R * (double)n * sizeof(cplx) > 64.0 * (double)(1ull << 30))
      return fail("basis staging above 64 GiB per orbital");
    for (int b = 0; b < M.norb; ++b)
      if (M.orbs[b] < 0 || M.orbs[b] >= c->nmo) return fail("orbital index out of range");
    std::vector<cplx> hq((size_t)M.R * n);
    if (hipMalloc(&M.Q, sizeof(cplx) * hq.size() * M.norb) != hipSuccess) {
      (void)hipGetLastError();
      M.Q = nullptr;
      return fail("device allocation of the basis failed");
    }
    for (int b = 0; b < M.norb && ok; ++b) {
      get(hq.data(), sizeof(cplx) * hq.size());
      ok = ok && hipMemcpy(M.Q + (size_t)b * hq.size(), hq.data(), sizeof(cplx) * hq.size(),
                           hipMemcpyHostToDevice) == hipSuccess;
    }
    long long np = 0, npp = 0;
    get(&np, sizeof np);
    if (!ok || np != mlp_nparams(M.din, M.hidden, M.dout)) return fail("bad guess-network parameters");
    std::vector<float> th((size_t)np);
    get(th.data(), sizeof(float) * np);
    if (!ok || hipMalloc(&M.theta, sizeof(float) * np) != hipSuccess ||
        hipMemcpy(M.theta, th.data(), sizeof(float) * np, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      return fail("reading or uploading the guess network failed");
    }
    get(&npp, sizeof npp);
    if (!ok || (npp != 0 && npp != mlp_nparams(M.pdin, M.hidden, M.pdout)))
      return fail("bad preconditioner-network parameters");
    if (npp) {
      th.resize((size_t)npp);
      get(th.data(), sizeof(float) * npp);
      if (!ok || hipMalloc(&M.theta_p, sizeof(float) * npp) != hipSuccess ||
          hipMemcpy(M.theta_p, th.data(), sizeof(float) * npp, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return fail("reading or uploading the preconditioner network failed");
      }
    }
  }
  std::fclose(f);
  if (int rc = hip_check(c, hipStreamSynchronize(c->stream), "learn_load")) {
    for (LearnModel &M : models) free_model(M);
    return rc;
  }
  for (LearnModel &M : c->models) free_model(M);
  c->models = std::move(models);
  c->learn_on = CCGF_LEARN_GUESS | CCGF_LEARN_PRECOND;
  return CCGF_OK;
}

// (no C++ exception crosses the ABI: host allocations that fail report CCGF_ENOMEM)
extern "C" int cc_gf_init(const ccgf_system *s, const ccgf_options *opt, ccgf_ctx **out) {
  try {
    return cc_gf_init_impl(s, opt, out);
  } catch (const std::exception &ex) {
    return set_err(nullptr, CCGF_ENOMEM, std::string("cc_gf_init: ") + ex.what());
  }
}

extern "C" int cc_gf_sigma(ccgf_ctx *c, int part, int K, int nvec, const double *x, double *y) {
  try {
    return cc_gf_sigma_impl(c, part, K, nvec, x, y);
  } catch (const std::exception &ex) {
    return set_err(c, CCGF_ENOMEM, std::string("cc_gf_sigma: ") + ex.what());
  }
}

extern "C" int cc_gf_sigma_group(int nsys, ccgf_ctx *const *ctxs, const int *parts, const int *K, const int *nvec,
                                 const double *const *x, double *const *y) {
  try {
    return cc_gf_sigma_group_impl(nsys, ctxs, parts, K, nvec, x, y);
  } catch (const std::exception &ex) {
    return set_err(nullptr, CCGF_ENOMEM, std::string("cc_gf_sigma_group: ") + ex.what());
  }
}

extern "C" int cc_gf_vectors(ccgf_ctx *c, int part, int K, int p, double *b, double *e) {
  try {
    return cc_gf_vectors_impl(c, part, K, p, b, e);
  } catch (const std::exception &ex) {
    return set_err(c, CCGF_ENOMEM, std::string("cc_gf_vectors: ") + ex.what());
  }
}

extern "C" int cc_gf_solve(ccgf_ctx *c, int nkq, const int *kidx, int norb, const int *orbs, int nw,
                           const double *omega, double eta, int parts, double *G, double *Gp, double *Gm,
                           ccgf_stats *st) {
  try {
    return cc_gf_solve_impl(c, nkq, kidx, norb, orbs, nw, omega, eta, parts, G, Gp, Gm, st);
  } catch (const std::exception &ex) {
    return set_err(c, CCGF_ENOMEM, std::string("cc_gf_solve: ") + ex.what());
  }
}

extern "C" int cc_gf_solve_matrix(ccgf_ctx *c, int nkq, const int *kidx, int norb, const int *orbs, int nw,
                                  const double *omega, double eta, int parts, double *G, double *Gp, double *Gm,
                                  double *dos, ccgf_stats *st) {
  try {
    return cc_gf_solve_matrix_impl(c, nkq, kidx, norb, orbs, nw, omega, eta, parts, G, Gp, Gm, dos, st);
  } catch (const std::exception &ex) {
    return set_err(c, CCGF_ENOMEM, std::string("cc_gf_solve_matrix: ") + ex.what());
  }
}

extern "C" int cc_gf_mor(ccgf_ctx *c, int nkq, const int *kidx, int norb, const int *orbs, int nexp_ip,
                         const double *wexp_ip, int nexp_ea, const double *wexp_ea, int nw, const double *omega,
                         double eta, int parts, double *G, double *Gp, double *Gm, ccgf_stats *st) {
  try {
    return cc_gf_mor_impl(c, nkq, kidx, norb, orbs, nexp_ip, wexp_ip, nexp_ea, wexp_ea, nw, omega, eta, parts, G,
                          Gp, Gm, st);
  } catch (const std::exception &ex) {
    return set_err(c, CCGF_ENOMEM, std::string("cc_gf_mor: ") + ex.what());
  }
}

extern "C" int cc_gf_learn(ccgf_ctx *c, int parts, int K, int norb, const int *orbs, int ntrain, const double *wtr,
                           double eta, const ccgf_learn_options *opt, ccgf_learn_stats *st) {
  try {
    return cc_gf_learn_impl(c, parts, K, norb, orbs, ntrain, wtr, eta, opt, st);
  } catch (const std::exception &ex) {
    return set_err(c, CCGF_ENOMEM, std::string("cc_gf_learn: ") + ex.what());
  }
}

extern "C" int cc_gf_set_options(ccgf_ctx *c, const ccgf_options *opt) {
  try {
    return cc_gf_set_options_impl(c, opt);
  } catch (const std::exception &ex) {
    return set_err(c, CCGF_ENOMEM, std::string("cc_gf_set_options: ") + ex.what());
  }
}

extern "C" int cc_gf_learn_save(ccgf_ctx *c, const char *path) {
  try {
    return learn_save_impl(c, path);
  } catch (const std::exception &ex) {
    return set_err(c, CCGF_ENOMEM, std::string("learn_save: ") + ex.what());
  }
}

extern "C" int cc_gf_learn_load(ccgf_ctx *c, const char *path) {
  try {
    return learn_load_impl(c, path);
  } catch (const std::exception &ex) {
    return set_err(c, CCGF_ENOMEM, std::string("learn_load: ") + ex.what());
  }
}

extern "C" void cc_gf_free(ccgf_ctx *c) {
  if (!c) return;
  hipStreamSynchronize(c->stream);
  for (LearnModel &M : c->models) {
    if (M.Q) hipFree(M.Q);
    if (M.theta) hipFree(M.theta);
    if (M.theta_p) hipFree(M.theta_p);
  }
  c->models.clear();
  timing_release(c);
  tune_save(c);
  for (auto &P : c->plans)
    for (auto &g : P.graphs) hipGraphExecDestroy(g.exec);
  c->plans.clear();
  if (c->cap_stream) hipStreamDestroy(c->cap_stream);
  if (c->side_stream) hipStreamDestroy(c->side_stream);
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  for (int q = 0; q < 2; ++q)
    if (c->tev[q]) hipEventDestroy(c->tev[q]);
  free_all(c);
  delete c;
}

extern "C" const char *cc_gf_last_error(const ccgf_ctx *c) {
  if (!c) return g_init_err.c_str();
  return c->err.empty() ? "no error" : c->err.c_str();
}
