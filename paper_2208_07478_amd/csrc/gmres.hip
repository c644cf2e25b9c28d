// Batched restarted GMRES for the shifted EOM systems of Eq. 6:
//   IP: (w + M_IP - i eta) x = b,   EA: (w - M_EA + i eta) y = b,
// right-preconditioned by the diagonal D = w + s_M diag(M) + s_eta i eta, with
// classical Gram-Schmidt applied twice (CGS2) for the Arnoldi step and complex
// Givens rotations for the Hessenberg least-squares problem, all in FP64.  All
// right-hand sides of one momentum K and part (orbitals x frequencies) advance
// together, so one sigma product per step serves the whole batch.  Inner
// products count each unordered pair once (weight 1/2 on the doubly stored
// 2h1p / 2p1h part), which makes full antisymmetric storage an isometric copy
// of the unique-coefficient space.  G = e . x is bilinear (Eq. 7).
#include "ccgf_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>

#define DOT_ITEMS 8
#define DOT_CHUNK (256 * DOT_ITEMS)

namespace {

__device__ inline double wgt(long long x, int n1) { return x < n1 ? 1.0 : 0.5; }

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// block-wide sum of a complex value; result valid in thread 0
__device__ inline cplx block_sum(cplx v, double *sh) {
  double re = wave_sum(v.x), im = wave_sum(v.y);
  int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) {
    sh[2 * w] = re;
    sh[2 * w + 1] = im;
  }
  __syncthreads();
  cplx r = mkc(0, 0);
  if (threadIdx.x == 0) {
    int nw = blockDim.x >> 6;
    for (int q = 0; q < nw; ++q) {
      r.x += sh[2 * q];
      r.y += sh[2 * q + 1];
    }
  }
  return r;
}

// partial[v][chunk][i] = sum_{x in chunk} wgt(x) * op(U_i[v][x]) * W[v][x],
// U_i[v] = U + uoff[v] + i * su_i (op = conj if conjU), W[v] = W + v * n
__global__ __launch_bounds__(256) void k_dots(const cplx *__restrict__ U, const long long *__restrict__ uoff,
                                              long long su_i, int ni, const cplx *__restrict__ W, long long n,
                                              int n1, int conjU, const int *__restrict__ active,
                                              cplx *__restrict__ partial, int nchunk, int ldp) {
  const int v = blockIdx.y, ch = blockIdx.x;
  if (active && !active[v]) return;
  __shared__ double sh[16];
  const long long base = (long long)ch * DOT_CHUNK;
  cplx wv[DOT_ITEMS];
  long long xs[DOT_ITEMS];
#pragma unroll
  for (int t = 0; t < DOT_ITEMS; ++t) {
    long long x = base + threadIdx.x + 256LL * t;
    xs[t] = x;
    wv[t] = x < n ? cscale(W[(size_t)v * n + x], wgt(x, n1)) : mkc(0, 0);
  }
  const cplx *Ub = U + uoff[v];
  for (int i = 0; i < ni; ++i) {
    const cplx *Ui = Ub + (size_t)i * su_i;
    cplx acc = mkc(0, 0);
#pragma unroll
    for (int t = 0; t < DOT_ITEMS; ++t)
      if (xs[t] < n) {
        if (conjU) cfmac(acc, Ui[xs[t]], wv[t]);
        else cfma(acc, Ui[xs[t]], wv[t]);
      }
    cplx r = block_sum(acc, sh);
    if (threadIdx.x == 0) partial[((size_t)v * nchunk + ch) * ldp + i] = r;
  }
}

// out[v][i] = sum_chunk partial; if H != null also H[v][i][col] += out
__global__ void k_dots_reduce(const cplx *__restrict__ partial, int nchunk, int ldp, int ni,
                              const int *__restrict__ active, cplx *__restrict__ out, int ldo,
                              cplx *__restrict__ H, int ldh, long long shv, int col) {
  const int v = blockIdx.x;
  if (active && !active[v]) return;
  for (int i = threadIdx.x; i < ni; i += blockDim.x) {
    cplx s = mkc(0, 0);
    for (int ch = 0; ch < nchunk; ++ch) s = cadd(s, partial[((size_t)v * nchunk + ch) * ldp + i]);
    out[(size_t)v * ldo + i] = s;
    if (H) {
      cplx *h = H + (size_t)v * shv + (size_t)i * ldh + col;
      *h = cadd(*h, s);
    }
  }
}

// W[v] -= sum_i h[v][i] * V_i[v],  V_i[v] = V + i * svi + v * n
__global__ __launch_bounds__(256) void k_sub_proj(cplx *__restrict__ W, const cplx *__restrict__ V, long long svi,
                                                  long long n, int ni, const cplx *__restrict__ h, int ldh,
                                                  const int *__restrict__ active) {
  const int v = blockIdx.y;
  if (active && !active[v]) return;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  cplx acc = W[(size_t)v * n + x];
  for (int i = 0; i < ni; ++i) acc = csub(acc, cmul(h[(size_t)v * ldh + i], V[(size_t)i * svi + (size_t)v * n + x]));
  W[(size_t)v * n + x] = acc;
}

__global__ void k_diag(int part, int nk, int no, int nv, int K, const int *__restrict__ kc3,
                       const cplx *__restrict__ Foo, const cplx *__restrict__ Fvv, cplx *__restrict__ d,
                       long long n) {
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  auto fo = [&](int k, int i) { return Foo[((size_t)k * no + i) * no + i]; };
  auto fv = [&](int k, int a) { return Fvv[((size_t)k * nv + a) * nv + a]; };
  cplx r;
  if (part == CCGF_PART_IP) {
    if (x < no) {
      cplx f = fo(K, (int)x);
      r = mkc(-f.x, -f.y);
    } else {
      long long y = x - no, b2 = (long long)no * no * nv;
      long long blk = y / b2, w = y % b2;
      int ki = (int)(blk / nk), kj = (int)(blk % nk);
      int a = (int)(w % nv), j = (int)((w / nv) % no), i = (int)(w / ((long long)nv * no));
      int ka = kc3[(ki * nk + kj) * nk + K];
      r = csub(csub(fv(ka, a), fo(ki, i)), fo(kj, j));
    }
  } else {
    if (x < nv) {
      r = fv(K, (int)x);
    } else {
      long long y = x - nv, b2 = (long long)no * nv * nv;
      long long blk = y / b2, w = y % b2;
      int ki = (int)(blk / nk), ka = (int)(blk % nk);
      int b = (int)(w % nv), a = (int)((w / nv) % nv), i = (int)(w / ((long long)nv * nv));
      int kb = kc3[(K * nk + ki) * nk + ka];
      r = csub(cadd(fv(ka, a), fv(kb, b)), fo(ki, i));
    }
  }
  d[x] = r;
}

// z[v] = V_j[v] / (shift_v + sM diag)   (zero for finished right-hand sides)
__global__ void k_precond(cplx *__restrict__ z, const cplx *__restrict__ Vj, const cplx *__restrict__ diag,
                          const cplx *__restrict__ shift, double sM, long long n, const int *__restrict__ active) {
  const int v = blockIdx.y;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  if (active && !active[v]) {
    z[(size_t)v * n + x] = mkc(0, 0);
    return;
  }
  cplx dd = cadd(shift[v], cscale(diag[x], sM));
  cplx u = Vj[(size_t)v * n + x];
  double den = dd.x * dd.x + dd.y * dd.y;
  z[(size_t)v * n + x] = mkc((u.x * dd.x + u.y * dd.y) / den, (u.y * dd.x - u.x * dd.y) / den);
}

// compact gather: z[slot] = X[idx[slot]] / (shift + sM diag)  (sM = 0 and nodiv: plain copy)
__global__ void k_gather_precond(cplx *__restrict__ z, const cplx *__restrict__ X, const cplx *__restrict__ diag,
                                 const cplx *__restrict__ shift, double sM, long long n, const int *__restrict__ idx,
                                 int divide) {
  const int slot = blockIdx.y, v = idx[slot];
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  cplx u = X[(size_t)v * n + x];
  if (divide) {
    cplx dd = cadd(shift[v], cscale(diag[x], sM));
    double den = dd.x * dd.x + dd.y * dd.y;
    u = mkc((u.x * dd.x + u.y * dd.y) / den, (u.y * dd.x - u.x * dd.y) / den);
  }
  z[(size_t)slot * n + x] = u;
}

// w[idx[slot]] = shift z[slot] + sM s[slot]
__global__ void k_scatter_shift(cplx *__restrict__ w, const cplx *__restrict__ z, const cplx *__restrict__ sg,
                                const cplx *__restrict__ shift, double sM, long long n, const int *__restrict__ idx) {
  const int slot = blockIdx.y, v = idx[slot];
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  size_t o = (size_t)slot * n + x;
  w[(size_t)v * n + x] = cadd(cmul(shift[v], z[o]), cscale(sg[o], sM));
}

// out[idx[slot]] = b - (shift x + sM s[slot])
__global__ void k_residual_c(cplx *__restrict__ out, const cplx *__restrict__ b, const cplx *__restrict__ xs,
                             const cplx *__restrict__ sg, const cplx *__restrict__ shift, double sM, long long n,
                             const int *__restrict__ idx) {
  const int slot = blockIdx.y, v = idx[slot];
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  size_t o = (size_t)v * n + e;
  out[o] = csub(b[o], cadd(cmul(shift[v], xs[o]), cscale(sg[(size_t)slot * n + e], sM)));
}

// w = shift z + sM w
__global__ void k_shift(cplx *__restrict__ w, const cplx *__restrict__ z, const cplx *__restrict__ shift, double sM,
                        long long n) {
  const int v = blockIdx.y;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  size_t o = (size_t)v * n + x;
  w[o] = cadd(cmul(shift[v], z[o]), cscale(w[o], sM));
}

// r = b - (shift x + sM s); stored into out
__global__ void k_residual(cplx *__restrict__ out, const cplx *__restrict__ b, const cplx *__restrict__ x,
                           const cplx *__restrict__ s, const cplx *__restrict__ shift, double sM, long long n) {
  const int v = blockIdx.y;
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  size_t o = (size_t)v * n + e;
  out[o] = csub(b[o], cadd(cmul(shift[v], x[o]), cscale(s[o], sM)));
}

// V_{j+1}[v] = w[v] * inv[v]
__global__ void k_scale(cplx *out, const cplx *w, const double *__restrict__ inv, long long n,
                        const int *__restrict__ active) {
  const int v = blockIdx.y;
  if (active && !active[v]) return;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  out[(size_t)v * n + x] = cscale(w[(size_t)v * n + x], inv[v]);
}

// One Givens step per right-hand side (column j of its Hessenberg matrix).
// H[v] is (m+1) x m row-major with leading dimension m.
__global__ void k_givens(int nvec, int m, int j, cplx *__restrict__ H, cplx *__restrict__ cs, cplx *__restrict__ sn,
                         cplx *__restrict__ g, const cplx *__restrict__ nrm2, double *__restrict__ inv,
                         int *__restrict__ active, int *__restrict__ kused, const double *__restrict__ thresh,
                         const int *__restrict__ jlim) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec || !active[v]) return;
  cplx *Hv = H + (size_t)v * (m + 1) * m;
  cplx *c = cs + (size_t)v * m, *s = sn + (size_t)v * m, *gv = g + (size_t)v * (m + 1);
  double hn = sqrt(fmax(nrm2[(size_t)v * (m + 1)].x, 0.0));
  Hv[(size_t)(j + 1) * m + j] = mkc(hn, 0);
  inv[v] = hn > 0 ? 1.0 / hn : 0.0;
  for (int i = 0; i < j; ++i) {
    cplx a = Hv[(size_t)i * m + j], b = Hv[(size_t)(i + 1) * m + j];
    // [c s; -conj(s) c] with real c
    cplx t = cadd(cscale(a, c[i].x), cmul(s[i], b));
    Hv[(size_t)(i + 1) * m + j] = cadd(cscale(cmul(cconj(s[i]), a), -1.0), cscale(b, c[i].x));
    Hv[(size_t)i * m + j] = t;
  }
  cplx a = Hv[(size_t)j * m + j], h = Hv[(size_t)(j + 1) * m + j];
  double aa = sqrt(a.x * a.x + a.y * a.y), hh = sqrt(h.x * h.x + h.y * h.y);
  double rho = sqrt(aa * aa + hh * hh);
  if (aa == 0.0) {
    c[j] = mkc(0, 0);
    s[j] = mkc(1, 0);
  } else {
    c[j] = mkc(aa / rho, 0);
    s[j] = cscale(cmul(cscale(a, 1.0 / aa), cconj(h)), 1.0 / rho);
  }
  Hv[(size_t)j * m + j] = cadd(cscale(a, c[j].x), cmul(s[j], h));
  Hv[(size_t)(j + 1) * m + j] = mkc(0, 0);
  cplx gj = gv[j];
  gv[j + 1] = cscale(cmul(cconj(s[j]), gj), -1.0);
  gv[j] = cscale(gj, c[j].x);
  kused[v] = j + 1;
  double res = sqrt(gv[j + 1].x * gv[j + 1].x + gv[j + 1].y * gv[j + 1].y);
  if (res <= thresh[v] || hn == 0.0 || j + 1 >= jlim[v]) active[v] = 0;
}

// y = R^-1 g (upper triangular, kused[v] columns), in place into ysol
__global__ void k_backsolve(int nvec, int m, const cplx *__restrict__ H, const cplx *__restrict__ g,
                            const int *__restrict__ kused, cplx *__restrict__ ysol, const int *__restrict__ done) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec || done[v]) return;
  const cplx *Hv = H + (size_t)v * (m + 1) * m;
  const cplx *gv = g + (size_t)v * (m + 1);
  cplx *y = ysol + (size_t)v * m;
  int k = kused[v];
  for (int i = k - 1; i >= 0; --i) {
    cplx s = gv[i];
    for (int l = i + 1; l < k; ++l) s = csub(s, cmul(Hv[(size_t)i * m + l], y[l]));
    cplx d = Hv[(size_t)i * m + i];
    double den = d.x * d.x + d.y * d.y;
    y[i] = den > 0 ? mkc((s.x * d.x + s.y * d.y) / den, (s.y * d.x - s.x * d.y) / den) : mkc(0, 0);
  }
}

// x[v] += D^-1 (sum_i y_i V_i[v])
__global__ void k_update_x(cplx *__restrict__ xs, const cplx *__restrict__ V, long long svi, long long n, int m,
                           const cplx *__restrict__ ysol, const int *__restrict__ kused,
                           const cplx *__restrict__ diag, const cplx *__restrict__ shift, double sM,
                           const int *__restrict__ done) {
  const int v = blockIdx.y;
  if (done[v]) return;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  cplx acc = mkc(0, 0);
  int k = kused[v];
  for (int i = 0; i < k; ++i) cfma(acc, ysol[(size_t)v * m + i], V[(size_t)i * svi + (size_t)v * n + x]);
  cplx dd = cadd(shift[v], cscale(diag[x], sM));
  double den = dd.x * dd.x + dd.y * dd.y;
  cplx q = mkc((acc.x * dd.x + acc.y * dd.y) / den, (acc.y * dd.x - acc.x * dd.y) / den);
  xs[(size_t)v * n + x] = cadd(xs[(size_t)v * n + x], q);
}

}  // namespace

struct GmresWork {
  long long n = 0;
  int B = 0, m = 0, nchunk = 0, ldp = 0;
  cplx *V = nullptr, *x = nullptr, *z = nullptr, *w = nullptr, *b = nullptr, *diag = nullptr, *wc = nullptr;
  cplx *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *htmp = nullptr, *partial = nullptr;
  cplx *shift = nullptr, *pshift = nullptr, *ysol = nullptr, *gout = nullptr;
  double *inv = nullptr, *thresh = nullptr;
  int *active = nullptr, *kused = nullptr, *done = nullptr, *jlim = nullptr, *aidx = nullptr;
  long long *uoff = nullptr, *eoff = nullptr;
  std::vector<void *> mine;
  bool failed = false;
};

static void *walloc(ccgf_ctx *c, GmresWork &W, size_t bytes) {
  (void)c;
  void *p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(bytes, 16)) != hipSuccess) {
    (void)hipGetLastError();
    W.failed = true;
    return nullptr;
  }
  W.mine.push_back(p);
  return p;
}
static void wfree(GmresWork &W) {
  for (void *p : W.mine) hipFree(p);
  W.mine.clear();
}

int solve_batched(ccgf_ctx *c, int part, int K, int nrhs, const int *rhs_orb, const double *rhs_omega, double eta,
                  const cplx *Bvecs, const cplx *Evecs, cplx *Gout, ccgf_stats *st) {
  const long long n = vec_len(c, part);
  const int n1 = part == CCGF_PART_IP ? c->no : c->nv;
  const double sM = part == CCGF_PART_IP ? 1.0 : -1.0;
  const double sE = part == CCGF_PART_IP ? -1.0 : 1.0;
  const int m = c->opt.restart_m;
  const int Bmax = std::max(1, std::min(c->opt.max_batch, nrhs));
  hipStream_t s = c->stream;
  GmresWork W;
  W.n = n;
  W.B = Bmax;
  W.m = m;
  W.nchunk = (int)((n + DOT_CHUNK - 1) / DOT_CHUNK);
  W.ldp = m + 1;
  const size_t vb = (size_t)Bmax * n;
  W.V = (cplx *)walloc(c, W, sizeof(cplx) * vb * (m + 1));
  W.x = (cplx *)walloc(c, W, sizeof(cplx) * vb);
  W.z = (cplx *)walloc(c, W, sizeof(cplx) * vb);
  W.w = (cplx *)walloc(c, W, sizeof(cplx) * vb);
  W.wc = (cplx *)walloc(c, W, sizeof(cplx) * vb);
  W.b = (cplx *)walloc(c, W, sizeof(cplx) * vb);
  W.diag = (cplx *)walloc(c, W, sizeof(cplx) * n);
  W.H = (cplx *)walloc(c, W, sizeof(cplx) * Bmax * (m + 1) * m);
  W.cs = (cplx *)walloc(c, W, sizeof(cplx) * Bmax * m);
  W.sn = (cplx *)walloc(c, W, sizeof(cplx) * Bmax * m);
  W.g = (cplx *)walloc(c, W, sizeof(cplx) * Bmax * (m + 1));
  W.htmp = (cplx *)walloc(c, W, sizeof(cplx) * Bmax * (m + 1));
  W.partial = (cplx *)walloc(c, W, sizeof(cplx) * (size_t)Bmax * W.nchunk * W.ldp);
  W.shift = (cplx *)walloc(c, W, sizeof(cplx) * Bmax);
  W.pshift = (cplx *)walloc(c, W, sizeof(cplx) * Bmax);
  W.ysol = (cplx *)walloc(c, W, sizeof(cplx) * Bmax * m);
  W.gout = (cplx *)walloc(c, W, sizeof(cplx) * Bmax);
  W.inv = (double *)walloc(c, W, sizeof(double) * Bmax);
  W.thresh = (double *)walloc(c, W, sizeof(double) * Bmax);
  W.active = (int *)walloc(c, W, sizeof(int) * Bmax);
  W.kused = (int *)walloc(c, W, sizeof(int) * Bmax);
  W.done = (int *)walloc(c, W, sizeof(int) * Bmax);
  W.jlim = (int *)walloc(c, W, sizeof(int) * Bmax);
  W.aidx = (int *)walloc(c, W, sizeof(int) * Bmax);
  W.uoff = (long long *)walloc(c, W, sizeof(long long) * Bmax);
  W.eoff = (long long *)walloc(c, W, sizeof(long long) * Bmax);
  if (W.failed) {
    wfree(W);
    return set_err(c, CCGF_ENOMEM, "GMRES workspace allocation failed (reduce max_batch or restart_m)");
  }
  const unsigned gx = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_diag, dim3(gx), dim3(256), 0, s, part, c->nk, c->no, c->nv, K, c->kc3, c->Foo, c->Fvv,
                     W.diag, n);

  int status = CCGF_OK;
  std::vector<cplx> hshift(Bmax), hpshift(Bmax), hh((size_t)Bmax * (m + 1)), g0((size_t)Bmax * (m + 1));
  const double peta = std::max(eta, c->opt.precond_eta);
  std::vector<double> hbnorm(Bmax), hthr(Bmax), hbeta(Bmax), hinv(Bmax);
  std::vector<int> hconv(Bmax), hkused(Bmax), hact(Bmax), hskip(Bmax), its(Bmax), hjlim(Bmax);
  std::vector<long long> hoff(Bmax), heoff(Bmax);
  std::vector<int> alist;
  alist.reserve(Bmax);
  const double tol = c->opt.tol;
  const int maxit = c->opt.maxiter;
  const size_t svi = (size_t)Bmax * n;
  auto sync = [&](const char *what) -> int {
    if (hipStreamSynchronize(s) != hipSuccess) return hip_check(c, hipGetLastError(), what);
    return hip_check(c, hipGetLastError(), what);
  };
  // weighted squared norms of the B vectors at X into hh[v*(m+1)]
  auto norms = [&](const cplx *X, int B) {
    hipLaunchKernelGGL(k_dots, dim3(W.nchunk, B), dim3(256), 0, s, X, W.uoff, 0LL, 1, X, n, n1, 1,
                       (const int *)nullptr, W.partial, W.nchunk, W.ldp);
    hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(64), 0, s, W.partial, W.nchunk, W.ldp, 1, (const int *)nullptr,
                       W.htmp, m + 1, (cplx *)nullptr, 0, 0LL, 0);
    hipMemcpyAsync(hh.data(), W.htmp, sizeof(cplx) * B * (m + 1), hipMemcpyDeviceToHost, s);
  };

  for (int r0 = 0; r0 < nrhs && status != CCGF_EDEVICE; r0 += Bmax) {
    const int B = std::min(Bmax, nrhs - r0);
    for (int v = 0; v < B; ++v) {
      hshift[v] = mkc(rhs_omega[r0 + v], sE * eta);
      hpshift[v] = mkc(rhs_omega[r0 + v], sE * peta);
      hoff[v] = (long long)v * n;  // each RHS's own vector inside a [B][n] batch
      heoff[v] = (long long)rhs_orb[r0 + v] * n;
      hipMemcpyAsync(W.b + (size_t)v * n, Bvecs + (size_t)rhs_orb[r0 + v] * n, sizeof(cplx) * n,
                     hipMemcpyDeviceToDevice, s);
    }
    hipMemcpyAsync(W.shift, hshift.data(), sizeof(cplx) * B, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(W.pshift, hpshift.data(), sizeof(cplx) * B, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(W.uoff, hoff.data(), sizeof(long long) * B, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(W.eoff, heoff.data(), sizeof(long long) * B, hipMemcpyHostToDevice, s);
    hipMemsetAsync(W.x, 0, sizeof(cplx) * (size_t)B * n, s);
    norms(W.b, B);  // x0 = 0, so r0 = b
    if (int rc = sync("GMRES start")) {
      wfree(W);
      return rc;
    }
    for (int v = 0; v < B; ++v) {
      hbnorm[v] = std::sqrt(std::max(hh[(size_t)v * (m + 1)].x, 0.0));
      hbeta[v] = hbnorm[v];
      hthr[v] = tol * hbnorm[v];
      hconv[v] = hbnorm[v] == 0.0;
      its[v] = 0;
      hinv[v] = hbeta[v] > 0 ? 1.0 / hbeta[v] : 0.0;
    }
    hipMemcpyAsync(W.thresh, hthr.data(), sizeof(double) * B, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(W.inv, hinv.data(), sizeof(double) * B, hipMemcpyHostToDevice, s);
    hipLaunchKernelGGL(k_scale, dim3(gx, B), dim3(256), 0, s, W.V, W.b, W.inv, n, (const int *)nullptr);

    while (true) {  // restart cycles
      int npart = 0;
      for (int v = 0; v < B; ++v) {
        hact[v] = (!hconv[v] && its[v] < maxit) ? 1 : 0;
        hskip[v] = !hact[v];
        hjlim[v] = std::min(m, std::max(0, maxit - its[v]));  // iteration budget of this cycle
        npart += hact[v];
      }
      if (npart == 0) break;
      hipMemcpyAsync(W.jlim, hjlim.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
      hipMemcpyAsync(W.active, hact.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
      hipMemcpyAsync(W.done, hskip.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
      hipMemsetAsync(W.H, 0, sizeof(cplx) * B * (m + 1) * m, s);
      std::fill(g0.begin(), g0.end(), mkc(0, 0));
      for (int v = 0; v < B; ++v) g0[(size_t)v * (m + 1)] = mkc(hbeta[v], 0);
      hipMemcpyAsync(W.g, g0.data(), sizeof(cplx) * B * (m + 1), hipMemcpyHostToDevice, s);
      hipMemsetAsync(W.kused, 0, sizeof(int) * B, s);
      for (int j = 0; j < m; ++j) {
        cplx *Vj = W.V + (size_t)j * svi;
        // only the right-hand sides still iterating enter the sigma product
        alist.clear();
        for (int v = 0; v < B; ++v)
          if (hact[v]) alist.push_back(v);
        const int na = (int)alist.size();
        hipMemcpyAsync(W.aidx, alist.data(), sizeof(int) * na, hipMemcpyHostToDevice, s);
        hipLaunchKernelGGL(k_gather_precond, dim3(gx, na), dim3(256), 0, s, W.z, Vj, W.diag, W.pshift, sM, n, W.aidx, 1);
        int rc = sigma_apply(c, part, K, na, W.z, W.wc);
        if (rc != CCGF_OK) {
          wfree(W);
          return rc;
        }
        if (st) st->n_sigma += na;
        hipLaunchKernelGGL(k_scatter_shift, dim3(gx, na), dim3(256), 0, s, W.w, W.z, W.wc, W.shift, sM, n, W.aidx);
        for (int pass = 0; pass < 2; ++pass) {  // CGS2 against V_0..V_j
          hipLaunchKernelGGL(k_dots, dim3(W.nchunk, B), dim3(256), 0, s, W.V, W.uoff, (long long)svi, j + 1, W.w, n,
                             n1, 1, W.active, W.partial, W.nchunk, W.ldp);
          hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(64), 0, s, W.partial, W.nchunk, W.ldp, j + 1, W.active,
                             W.htmp, m + 1, W.H, m, (long long)(m + 1) * m, j);
          hipLaunchKernelGGL(k_sub_proj, dim3(gx, B), dim3(256), 0, s, W.w, W.V, (long long)svi, n, j + 1, W.htmp,
                             m + 1, W.active);
        }
        hipLaunchKernelGGL(k_dots, dim3(W.nchunk, B), dim3(256), 0, s, W.w, W.uoff, 0LL, 1, W.w, n, n1, 1, W.active,
                           W.partial, W.nchunk, W.ldp);
        hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(64), 0, s, W.partial, W.nchunk, W.ldp, 1, W.active, W.htmp,
                           m + 1, (cplx *)nullptr, 0, 0LL, 0);
        hipLaunchKernelGGL(k_givens, dim3((B + 63) / 64), dim3(64), 0, s, B, m, j, W.H, W.cs, W.sn, W.g, W.htmp,
                           W.inv, W.active, W.kused, W.thresh, W.jlim);
        if (j + 1 < m)
          hipLaunchKernelGGL(k_scale, dim3(gx, B), dim3(256), 0, s, W.V + (size_t)(j + 1) * svi, W.w, W.inv, n,
                             W.active);
        hipMemcpyAsync(hact.data(), W.active, sizeof(int) * B, hipMemcpyDeviceToHost, s);
        if (int rc2 = sync("GMRES iteration")) {
          wfree(W);
          return rc2;
        }
        int any = 0;
        for (int v = 0; v < B; ++v) any |= hact[v];
        if (!any) break;  // every right-hand side has finished this cycle
      }
      hipLaunchKernelGGL(k_backsolve, dim3((B + 63) / 64), dim3(64), 0, s, B, m, W.H, W.g, W.kused, W.ysol, W.done);
      hipLaunchKernelGGL(k_update_x, dim3(gx, B), dim3(256), 0, s, W.x, W.V, (long long)svi, n, m, W.ysol, W.kused,
                         W.diag, W.pshift, sM, W.done);
      hipMemcpyAsync(hkused.data(), W.kused, sizeof(int) * B, hipMemcpyDeviceToHost, s);
      // true residual r = b - A x (right-hand sides of this cycle) into V_0 and its norm
      alist.clear();
      for (int v = 0; v < B; ++v)
        if (!hskip[v]) alist.push_back(v);
      const int np = (int)alist.size();
      hipMemcpyAsync(W.aidx, alist.data(), sizeof(int) * np, hipMemcpyHostToDevice, s);
      hipLaunchKernelGGL(k_gather_precond, dim3(gx, np), dim3(256), 0, s, W.z, W.x, W.diag, W.shift, 0.0, n, W.aidx, 0);
      int rc = sigma_apply(c, part, K, np, W.z, W.wc);
      if (rc != CCGF_OK) {
        wfree(W);
        return rc;
      }
      if (st) st->n_sigma += np;
      hipLaunchKernelGGL(k_residual_c, dim3(gx, np), dim3(256), 0, s, W.V, W.b, W.x, W.wc, W.shift, sM, n, W.aidx);
      norms(W.V, B);
      if (int rc2 = sync("GMRES restart")) {
        wfree(W);
        return rc2;
      }
      for (int v = 0; v < B; ++v) {
        if (hskip[v]) continue;  // finished earlier: keep its residual
        hbeta[v] = std::sqrt(std::max(hh[(size_t)v * (m + 1)].x, 0.0));
        its[v] += hkused[v];
        hconv[v] = hbnorm[v] == 0.0 || hbeta[v] <= tol * hbnorm[v];
        hinv[v] = hbeta[v] > 0 ? 1.0 / hbeta[v] : 0.0;
      }
      hipMemcpyAsync(W.inv, hinv.data(), sizeof(double) * B, hipMemcpyHostToDevice, s);
      hipLaunchKernelGGL(k_scale, dim3(gx, B), dim3(256), 0, s, W.V, W.V, W.inv, n, (const int *)nullptr);
    }
    // G = e . x (bilinear, Eq. 7)
    hipLaunchKernelGGL(k_dots, dim3(W.nchunk, B), dim3(256), 0, s, Evecs, W.eoff, 0LL, 1, W.x, n, n1, 0,
                       (const int *)nullptr, W.partial, W.nchunk, W.ldp);
    hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(64), 0, s, W.partial, W.nchunk, W.ldp, 1, (const int *)nullptr,
                       W.htmp, m + 1, (cplx *)nullptr, 0, 0LL, 0);
    hipMemcpyAsync(hh.data(), W.htmp, sizeof(cplx) * B * (m + 1), hipMemcpyDeviceToHost, s);
    if (int rc2 = sync("G assembly")) {
      wfree(W);
      return rc2;
    }
    for (int v = 0; v < B; ++v) {
      Gout[r0 + v] = hh[(size_t)v * (m + 1)];
      double rel = hbnorm[v] > 0 ? hbeta[v] / hbnorm[v] : 0.0;
      bool ok = hbnorm[v] == 0.0 || rel <= tol;
      if (st) {
        st->n_solves += 1;
        st->n_iterations += its[v];
        st->max_iterations = std::max(st->max_iterations, its[v]);
        st->max_rel_residual = std::max(st->max_rel_residual, rel);
        if (!ok) st->n_unconverged += 1;
      }
      if (!ok) status = CCGF_ENOCONV;
    }
  }
  wfree(W);
  return status;
}
