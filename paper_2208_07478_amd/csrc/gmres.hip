// Batched Krylov solver for the shifted EOM systems of Eq. 6:
//   IP: (w + M_IP - i eta) x = b,   EA: (w - M_EA + i eta) y = b,
// right-preconditioned by the diagonal D = w + s_M diag(M) + s_eta i eta_p.
// The paper solves these with GCROT(m,k); here each outer cycle is an Arnoldi
// process of up to m steps on (I - C C^H) A, followed by the minimal-residual
// correction u and its image c = A u, which join a recycled set of the k most
// recent (u, c) pairs (k = 0 is restarted GMRES(m)).  Classical Gram-Schmidt is
// applied twice (CGS2) against C and the Arnoldi basis, and complex Givens
// rotations solve the Hessenberg least-squares problem, all in FP64.  The
// second Gram-Schmidt pass runs only where the first left less than a set
// fraction of ||w|| (0.1 by default: with the damped diagonal preconditioner
// nearly every step loses more than the classical 1/sqrt(2), and the extra pass
// then doubles the orthogonalisation traffic for little gain in convergence).
// The right-hand sides of one momentum K and part (orbitals x frequencies) share
// a batch of slots that is refilled as solves finish, so one sigma product per
// step serves the whole batch.  Inner products count each unordered pair once
// (weight 1/2 on the doubly stored 2h1p / 2p1h part), which makes full
// antisymmetric storage an isometric copy of the unique-coefficient space; the
// GMRES basis is kept in that unique space (half the vector length), sigma
// works on full storage, and residuals and guesses are projected onto
// antisymmetric vectors.  G = e . x is bilinear (Eq. 7).
#include "ccgf_internal.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <random>

#define DOT_ITEMS 8
#define DOT_CHUNK (256 * DOT_ITEMS)

namespace {

__device__ inline double wgt(long long x, int n1) { return x < n1 ? 1.0 : 0.5; }

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// partial[v][chunk][i] = sum_{x in chunk} wgt(x) * op(U_i[v][x]) * W[v][x],
// U_i[v] = U + uoff[v] + i * su_i (op = conj if conjU), W[v] = W + v * n,
// i < ni0 (+ nlist[v] when a per-slot count is given).  The chunk of W stays in
// registers; the U_i are taken DOT_G at a time with all their loads in flight
// before one block reduction for the group (conj(U) W is formed as conj(U conj(W))
// so that the loop has no branch on conjU).
#define DOT_G 4
__global__ __launch_bounds__(256) void k_dots(const cplx *__restrict__ U, const long long *__restrict__ uoff,
                                              long long su_i, int ni0, const cplx *__restrict__ W, long long n,
                                              int n1, int conjU, const int *__restrict__ active,
                                              cplx *__restrict__ partial, int nchunk, int ldp,
                                              const int *__restrict__ nlist) {
  const int v = blockIdx.y, ch = blockIdx.x;
  if (active && !active[v]) return;
  const int ni = nlist ? nlist[v] + ni0 : ni0;
  __shared__ double sh[2][4][2 * DOT_G];
  const long long base = (long long)ch * DOT_CHUNK + threadIdx.x;
  const bool full = (long long)(ch + 1) * DOT_CHUNK <= n;
  cplx wv[DOT_ITEMS];
  const cplx *Wb = W + (size_t)v * n + base;
  if (full) {
#pragma unroll
    for (int t = 0; t < DOT_ITEMS; ++t) wv[t] = Wb[256 * t];
  } else {
#pragma unroll
    for (int t = 0; t < DOT_ITEMS; ++t) wv[t] = base + 256LL * t < n ? Wb[256 * t] : mkc(0, 0);
  }
#pragma unroll
  for (int t = 0; t < DOT_ITEMS; ++t) {
    const double c = wgt(base + 256LL * t, n1);
    wv[t] = mkc(c * wv[t].x, (conjU ? -c : c) * wv[t].y);
  }
  const cplx *Ub = U + uoff[v];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int par = 0;
  for (int i0 = 0; i0 < ni; i0 += DOT_G, par ^= 1) {
    cplx acc[DOT_G];
#pragma unroll
    for (int g = 0; g < DOT_G; ++g) acc[g] = mkc(0, 0);
    const int ng = min(DOT_G, ni - i0);
    if (full && ng == DOT_G) {
#pragma unroll
      for (int g = 0; g < DOT_G; ++g) {
        const cplx *Ug = Ub + (size_t)(i0 + g) * su_i + base;
        cplx u[DOT_ITEMS];
#pragma unroll
        for (int t = 0; t < DOT_ITEMS; ++t) u[t] = Ug[256 * t];
#pragma unroll
        for (int t = 0; t < DOT_ITEMS; ++t) cfma(acc[g], u[t], wv[t]);
      }
    } else {
      for (int t = 0; t < DOT_ITEMS; ++t) {
        const long long x = base + 256LL * t;
        if (x < n)
          for (int g = 0; g < ng; ++g) cfma(acc[g], Ub[(size_t)(i0 + g) * su_i + x], wv[t]);
      }
    }
#pragma unroll
    for (int g = 0; g < DOT_G; ++g) {
      acc[g].x = wave_sum(acc[g].x);
      acc[g].y = wave_sum(acc[g].y);
    }
    if (lane == 0)
#pragma unroll
      for (int g = 0; g < DOT_G; ++g) {
        sh[par][wave][2 * g] = acc[g].x;
        sh[par][wave][2 * g + 1] = acc[g].y;
      }
    __syncthreads();  // (the next group writes the other half of sh)
    if (threadIdx.x < ng) {
      const int g = threadIdx.x;
      double re = 0, im = 0;
      for (int q = 0; q < 4; ++q) {
        re += sh[par][q][2 * g];
        im += sh[par][q][2 * g + 1];
      }
      partial[((size_t)v * nchunk + ch) * ldp + i0 + g] = mkc(re, conjU ? -im : im);
    }
  }
}

// out[v][i] = sum_chunk partial; if H != null also H[v][i][col] += out (and H2 likewise);
// per-slot counts and columns as in k_dots.  One 256-thread block per slot: 64 columns at a
// time, each summed over the chunks by four thread groups (independent loads in flight), then
// the four group sums added in LDS.
__global__ __launch_bounds__(256) void k_dots_reduce(const cplx *__restrict__ partial, int nchunk, int ldp, int ni0,
                                                     const int *__restrict__ active, cplx *__restrict__ out, int ldo,
                                                     cplx *__restrict__ H, int ldh, long long shv, int col0,
                                                     cplx *__restrict__ H2, const int *__restrict__ nlist,
                                                     const int *__restrict__ colv) {
  const int v = blockIdx.x;
  if (active && !active[v]) return;
  const int ni = nlist ? nlist[v] + ni0 : ni0;
  const int col = colv ? colv[v] : col0;
  const int il = threadIdx.x & 63, grp = threadIdx.x >> 6;
  __shared__ double red[2][4][64];
  for (int i0 = 0; i0 < ni; i0 += 64) {
    const int i = i0 + il;
    cplx acc = mkc(0, 0);
    if (i < ni)
      for (int ch = grp; ch < nchunk; ch += 4) acc = cadd(acc, partial[((size_t)v * nchunk + ch) * ldp + i]);
    red[0][grp][il] = acc.x;
    red[1][grp][il] = acc.y;
    __syncthreads();
    if (grp == 0 && i < ni) {
      const cplx s = mkc(red[0][0][il] + red[0][1][il] + red[0][2][il] + red[0][3][il],
                         red[1][0][il] + red[1][1][il] + red[1][2][il] + red[1][3][il]);
      out[(size_t)v * ldo + i] = s;
      if (H) {
        cplx *h = H + (size_t)v * shv + (size_t)i * ldh + col;
        *h = cadd(*h, s);
      }
      if (H2) {
        cplx *h = H2 + (size_t)v * shv + (size_t)i * ldh + col;
        *h = cadd(*h, s);
      }
    }
    __syncthreads();
  }
}

// W[v] -= sum_i h[v][i] * V_i[v],  V_i[v] = V + i * svi + v * n
__global__ __launch_bounds__(256) void k_sub_proj(cplx *__restrict__ W, const cplx *__restrict__ V, long long svi,
                                                  long long n, int ni0, const cplx *__restrict__ h, int ldh,
                                                  const int *__restrict__ active, const int *__restrict__ nlist) {
  const int v = blockIdx.y;
  if (active && !active[v]) return;
  const int ni = nlist ? nlist[v] + ni0 : ni0;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const cplx *Vx = V + (size_t)v * n + x;
  const cplx *hv = h + (size_t)v * ldh;
  cplx acc = W[(size_t)v * n + x];
  int i = 0;
  for (; i + 8 <= ni; i += 8) {  // eight loads in flight per thread
    cplx u[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) u[q] = Vx[(size_t)(i + q) * svi];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc = csub(acc, cmul(hv[i + q], u[q]));
  }
  for (; i < ni; ++i) acc = csub(acc, cmul(hv[i], Vx[(size_t)i * svi]));
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

// compact gather: z[slot] = X[idx[slot]] / (shift + sM diag)  (sM = 0 and nodiv: plain copy);
// with jv the source is column jv[v] of a basis with stride svi.  Source vectors have
// length nx; with unp they hold the unique elements only and element x of the full
// vector is sign * X[|unp[x]| - 1] (unp[x] = 0: a structural zero).
__global__ void k_gather_precond(cplx *__restrict__ z, const cplx *__restrict__ X, const cplx *__restrict__ diag,
                                 const cplx *__restrict__ shift, double sM, long long n, const int *__restrict__ idx,
                                 int divide, const int *__restrict__ jv, long long svi, const int *__restrict__ unp,
                                 long long nx) {
  const int slot = blockIdx.y, v = idx[slot];
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const size_t base = (jv ? (size_t)jv[v] * svi : 0) + (size_t)v * nx;
  cplx u;
  if (unp) {
    const int q = unp[x];
    u = q == 0 ? mkc(0, 0) : X[base + (size_t)(abs(q) - 1)];
    if (q < 0) u = mkc(-u.x, -u.y);
  } else {
    u = X[base + x];
  }
  if (divide) {
    cplx dd = cadd(shift[v], cscale(diag[x], sM));
    double den = dd.x * dd.x + dd.y * dd.y;
    u = mkc((u.x * dd.x + u.y * dd.y) / den, (u.y * dd.x - u.x * dd.y) / den);
  }
  z[(size_t)slot * n + x] = u;
}

// w[idx[slot]] = shift z[slot] + sM s[slot], for the nout elements pk[p] of the
// full vectors (length nz) when pk is given (the unique elements), else all of them
__global__ void k_scatter_shift(cplx *__restrict__ w, const cplx *__restrict__ z, const cplx *__restrict__ sg,
                                const cplx *__restrict__ shift, double sM, long long nout,
                                const int *__restrict__ idx, const long long *__restrict__ pk, long long nz) {
  const int slot = blockIdx.y, v = idx[slot];
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nout) return;
  size_t o = (size_t)slot * nz + (pk ? pk[p] : p);
  w[(size_t)v * nout + p] = cadd(cmul(shift[v], z[o]), cscale(sg[o], sM));
}

// Project the listed full vectors onto the antisymmetric amplitudes: each pair of
// copies becomes (a, -a) with a = (r[pk] - r[pkm]) / 2, structural zeros become 0
// (rounding in a product leaves the two copies unequal by a few ulps; the Krylov
// basis holds one copy, so the residual it can reduce is this projection).
__global__ void k_antisym(cplx *__restrict__ r, long long n, const long long *__restrict__ pk,
                          const long long *__restrict__ pkm, long long np, const long long *__restrict__ zl,
                          long long nz, const int *__restrict__ idx) {
  const int v = idx[blockIdx.y];
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  cplx *rv = r + (size_t)v * n;
  if (t < np) {
    const long long m = pkm[t];
    if (m >= 0) {
      const cplx a = rv[pk[t]], b = rv[m];
      const cplx h = mkc(0.5 * (a.x - b.x), 0.5 * (a.y - b.y));
      rv[pk[t]] = h;
      rv[m] = mkc(-h.x, -h.y);
    }
  } else if (t < np + nz) {
    rv[zl[t - np]] = mkc(0, 0);
  }
}

// out[v][p] = w[v][pk[p]] * inv[v] (pk = NULL: p itself); out has length nout, w length nw
__global__ void k_scale_pack(cplx *__restrict__ out, const cplx *__restrict__ w, const double *__restrict__ inv,
                             long long nout, const long long *__restrict__ pk, long long nw,
                             const int *__restrict__ active) {
  const int v = blockIdx.y;
  if (active && !active[v]) return;
  long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nout) return;
  out[(size_t)v * nout + p] = cscale(w[(size_t)v * nw + (pk ? pk[p] : p)], inv[v]);
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

// V_{j+1}[v] = w[v] * inv[v]
__global__ void k_scale(cplx *out, const cplx *w, const double *__restrict__ inv, long long n,
                        const int *__restrict__ active) {
  const int v = blockIdx.y;
  if (active && !active[v]) return;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  out[(size_t)v * n + x] = cscale(w[(size_t)v * n + x], inv[v]);
}

// out[idx[slot]] = w[idx[slot]] * inv[idx[slot]]
// out column jv[v] + 1 (stride svi) of slot idx[...] = w * inv
__global__ void k_scale_idx(cplx *__restrict__ out, const cplx *__restrict__ w, const double *__restrict__ inv,
                            long long n, const int *__restrict__ idx, const int *__restrict__ jv, long long svi) {
  const int v = idx[blockIdx.y];
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  out[(size_t)(jv[v] + 1) * svi + (size_t)v * n + x] = cscale(w[(size_t)v * n + x], inv[v]);
}

// Start an Arnoldi cycle in the flagged slots: zero H, H0 and the recycled-space
// coefficients, g = (||r||, 0, ...), no columns used yet.
__global__ void k_cycle_start(int m, int kslots, const int *__restrict__ start, const double *__restrict__ rn,
                              cplx *__restrict__ H, cplx *__restrict__ H0, cplx *__restrict__ Bm,
                              cplx *__restrict__ g, int *__restrict__ kused) {
  const int v = blockIdx.x;
  if (!start[v]) return;
  const size_t hs = (size_t)(m + 1) * m;
  for (size_t i = threadIdx.x; i < hs; i += blockDim.x) {
    H[(size_t)v * hs + i] = mkc(0, 0);
    H0[(size_t)v * hs + i] = mkc(0, 0);
  }
  for (size_t i = threadIdx.x; i < (size_t)kslots * m; i += blockDim.x) Bm[(size_t)v * kslots * m + i] = mkc(0, 0);
  for (int i = threadIdx.x; i <= m; i += blockDim.x) g[(size_t)v * (m + 1) + i] = mkc(i == 0 ? rn[v] : 0.0, 0);
  if (threadIdx.x == 0) kused[v] = 0;
}

// One Givens step per right-hand side (column jv[v] of its Hessenberg matrix).
// H[v] is (m+1) x m row-major with leading dimension m.
__global__ void k_givens(int nvec, int m, const int *__restrict__ jv, cplx *__restrict__ H, cplx *__restrict__ cs,
                         cplx *__restrict__ sn, cplx *__restrict__ g, const cplx *__restrict__ nrm2, int ldn,
                         double *__restrict__ inv, int *__restrict__ active, int *__restrict__ kused,
                         const double *__restrict__ thresh, const int *__restrict__ jlim, cplx *__restrict__ H0) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec || !active[v]) return;
  const int j = jv[v];
  cplx *Hv = H + (size_t)v * (m + 1) * m;
  cplx *c = cs + (size_t)v * m, *s = sn + (size_t)v * m, *gv = g + (size_t)v * (m + 1);
  double hn = sqrt(fmax(nrm2[(size_t)v * ldn].x, 0.0));
  Hv[(size_t)(j + 1) * m + j] = mkc(hn, 0);
  H0[(size_t)v * (m + 1) * m + (size_t)(j + 1) * m + j] = mkc(hn, 0);
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

// y = R^-1 g (upper triangular, kused[v] columns) into ysol; one block per slot,
// column-oriented back substitution (the updates of each column run in parallel)
__global__ void k_backsolve(int nvec, int m, const cplx *__restrict__ H, const cplx *__restrict__ g,
                            const int *__restrict__ kused, cplx *__restrict__ ysol, const int *__restrict__ done) {
  const int v = blockIdx.x;
  if (v >= nvec || done[v]) return;
  const cplx *Hv = H + (size_t)v * (m + 1) * m;
  cplx *y = ysol + (size_t)v * m;
  const int k = kused[v];
  for (int i = threadIdx.x; i < k; i += blockDim.x) y[i] = g[(size_t)v * (m + 1) + i];
  __syncthreads();
  for (int l = k - 1; l >= 0; --l) {
    cplx d = Hv[(size_t)l * m + l];
    double den = d.x * d.x + d.y * d.y;
    cplx s = y[l];
    cplx yl = den > 0 ? mkc((s.x * d.x + s.y * d.y) / den, (s.y * d.x - s.x * d.y) / den) : mkc(0, 0);
    __syncthreads();  // every thread has read y[l]
    if (threadIdx.x == 0) y[l] = yl;
    for (int i = threadIdx.x; i < l; i += blockDim.x) y[i] = csub(y[i], cmul(Hv[(size_t)i * m + l], yl));
    __syncthreads();
  }
}

// X[v] += sum_i h[v][i] * U_i[v]  (masked)
__global__ __launch_bounds__(256) void k_add_proj(cplx *__restrict__ X, const cplx *__restrict__ U, long long svi,
                                                  long long n, int ni, const cplx *__restrict__ h, int ldh,
                                                  const int *__restrict__ active) {
  const int v = blockIdx.y;
  if (!active[v]) return;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  cplx acc = X[(size_t)v * n + x];
  for (int i = 0; i < ni; ++i) cfma(acc, h[(size_t)v * ldh + i], U[(size_t)i * svi + (size_t)v * n + x]);
  X[(size_t)v * n + x] = acc;
}

// w0n[v] = ||w||^2 before projection (read from the reduced dots)
__global__ void k_take_norm(int nvec, const cplx *__restrict__ nrm2, int ld, double *__restrict__ w0n,
                            const int *__restrict__ active) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec || !active[v]) return;
  w0n[v] = nrm2[(size_t)v * ld].x;
}

// second Gram-Schmidt pass only where one pass left less than ratio2 of ||w||^2
__global__ void k_need_reorth(int nvec, const cplx *__restrict__ nrm2, int ld, const double *__restrict__ w0n,
                              const int *__restrict__ active, int *__restrict__ need, double ratio2) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec) return;
  need[v] = active[v] && nrm2[(size_t)v * ld].x < ratio2 * w0n[v];
}

// t = Bm y (recycled-space coefficients, kc entries) and d = H0 y (kused + 1 entries);
// one block per slot, one thread per output entry
__global__ void k_gcrot_small(int nvec, int m, int kc, const cplx *__restrict__ Bm, const cplx *__restrict__ H0,
                              const cplx *__restrict__ ysol, const int *__restrict__ kused, cplx *__restrict__ t,
                              cplx *__restrict__ d, const int *__restrict__ skip, int ldt) {
  const int v = blockIdx.x;
  if (v >= nvec || skip[v]) return;
  const int k = kused[v];
  const cplx *y = ysol + (size_t)v * m;
  for (int l = threadIdx.x; l < kc; l += blockDim.x) {
    cplx acc = mkc(0, 0);
    for (int i = 0; i < k; ++i) cfma(acc, Bm[(size_t)v * ldt * m + (size_t)l * m + i], y[i]);
    t[(size_t)v * ldt + l] = acc;
  }
  for (int r = threadIdx.x; r <= k; r += blockDim.x) {
    cplx acc = mkc(0, 0);
    for (int i = 0; i < k; ++i) cfma(acc, H0[(size_t)v * (m + 1) * m + (size_t)r * m + i], y[i]);
    d[(size_t)v * (m + 1) + r] = acc;
  }
}

// u = D^-1 V y - U t,  c = V d;  x += u, r -= c;  u, c stored into the recycle slot.
// The basis columns have length nvb and stride svv; with unp they hold the unique
// elements only (element e of the full vector is sign * V[|unp[e]| - 1], 0: zero).
__global__ __launch_bounds__(256) void k_gcrot_combine(
    long long n, int m, long long svi, const cplx *__restrict__ V, const cplx *__restrict__ ysol,
    const cplx *__restrict__ d, const int *__restrict__ kused, int kc, const cplx *Ub,
    const cplx *__restrict__ t, int ldt, const cplx *__restrict__ diag, const cplx *__restrict__ pshift, double sM,
    cplx *uout, cplx *__restrict__ cout, cplx *__restrict__ xs, cplx *__restrict__ rs,
    const int *__restrict__ skip, const int *__restrict__ unp, long long nvb, long long svv) {
  const int v = blockIdx.y;
  if (skip[v]) return;
  long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int k = kused[v];
  const int q = unp ? unp[e] : (int)e + 1;
  cplx vy = mkc(0, 0), cc = mkc(0, 0);
  if (q != 0) {
    const cplx *Ve = V + (size_t)v * nvb + (size_t)(abs(q) - 1);
    for (int i = 0; i < k; ++i) {
      cplx vi = Ve[(size_t)i * svv];
      cfma(vy, ysol[(size_t)v * m + i], vi);
      cfma(cc, d[(size_t)v * (m + 1) + i], vi);
    }
    cfma(cc, d[(size_t)v * (m + 1) + k], Ve[(size_t)k * svv]);
    if (q < 0) {
      vy = mkc(-vy.x, -vy.y);
      cc = mkc(-cc.x, -cc.y);
    }
  }
  cplx dd = cadd(pshift[v], cscale(diag[e], sM));
  double den = dd.x * dd.x + dd.y * dd.y;
  cplx u = mkc((vy.x * dd.x + vy.y * dd.y) / den, (vy.y * dd.x - vy.x * dd.y) / den);
  for (int l = 0; l < kc; ++l) u = csub(u, cmul(t[(size_t)v * ldt + l], Ub[(size_t)l * svi + (size_t)v * n + e]));
  const size_t o = (size_t)v * n + e;
  uout[o] = u;  // may overwrite the oldest recycled u of this element, already read above
  cout[o] = cc;
  xs[o] = cadd(xs[o], u);
  rs[o] = csub(rs[o], cc);
}

// inv[v] = 1 / sqrt(nrm2[v]) for the right-hand sides that took part
__global__ void k_inv_sqrt(int nvec, const cplx *__restrict__ nrm2, int ld, double *__restrict__ inv,
                           const int *__restrict__ skip) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvec || skip[v]) return;
  double q = sqrt(fmax(nrm2[(size_t)v * ld].x, 0.0));
  inv[v] = q > 0 ? 1.0 / q : 0.0;
}

// u, c *= inv (participating right-hand sides)
__global__ void k_scale2(cplx *__restrict__ a, cplx *__restrict__ b, const double *__restrict__ inv, long long n,
                         const int *__restrict__ skip) {
  const int v = blockIdx.y;
  if (skip[v]) return;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  size_t o = (size_t)v * n + x;
  a[o] = cscale(a[o], inv[v]);
  b[o] = cscale(b[o], inv[v]);
}

// dst[v] = src[soff[v]] (strided gather / scatter of whole vectors)
__global__ void k_copy_vecs(cplx *__restrict__ dst, const long long *__restrict__ doff, const cplx *__restrict__ src,
                            const long long *__restrict__ soff, long long n) {
  const int v = blockIdx.y;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  dst[doff[v] + x] = src[soff[v] + x];
}

// X[idx[y]] = sum_i Q[qoff[y] + i qs] * ch[coff[y] + i]  (guess x0 = Q c_hat)
__global__ void k_expand(cplx *__restrict__ X, const cplx *__restrict__ Q, const long long *__restrict__ qoff,
                         const cplx *__restrict__ ch, const long long *__restrict__ coff, int R, long long n,
                         const int *__restrict__ idx, long long qs) {
  const int y = blockIdx.y, v = idx[y];
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  cplx acc = mkc(0, 0);
  for (int i = 0; i < R; ++i) cfma(acc, ch[coff[y] + i], Q[qoff[y] + (long long)i * qs + x]);
  X[(size_t)v * n + x] = acc;
}

// W[v] -= sum_i h[v][i] * U_i[v],  U_i[v] = U + uoff[v] + i * n
__global__ __launch_bounds__(256) void k_sub_proj_off(cplx *__restrict__ W, const cplx *__restrict__ U,
                                                      const long long *__restrict__ uoff, long long n, int ni,
                                                      const cplx *__restrict__ h, int ldh) {
  const int v = blockIdx.y;
  long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= n) return;
  const cplx *Ub = U + uoff[v];
  cplx acc = W[(size_t)v * n + x];
  for (int i = 0; i < ni; ++i) acc = csub(acc, cmul(h[(size_t)v * ldh + i], Ub[(size_t)i * n + x]));
  W[(size_t)v * n + x] = acc;
}

// Reduced model of Eq. 6 for one orbital per thread row: solve
// (w + s_M Ht + i s_eta eta) y = bt by Gaussian elimination with partial pivoting, G = et . y
template <int MAXR>
__global__ void k_mor_eval(int norb, int r, int nw, const double *__restrict__ omega, double eta_s, double sM,
                           const cplx *__restrict__ Ht, const cplx *__restrict__ bt, const cplx *__restrict__ et,
                           cplx *__restrict__ G) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= norb * nw) return;
  const int b = t / nw, w = t % nw;
  cplx A[MAXR * MAXR], y[MAXR];
  const cplx sh = mkc(omega[w], eta_s);
  for (int j = 0; j < r; ++j) {
    for (int k = 0; k < r; ++k) {
      cplx h = cscale(Ht[((size_t)b * r + j) * r + k], sM);
      A[j * MAXR + k] = j == k ? cadd(h, sh) : h;
    }
    y[j] = bt[(size_t)b * r + j];
  }
  for (int col = 0; col < r; ++col) {
    int piv = col;
    double best = -1;
    for (int j = col; j < r; ++j) {
      cplx q = A[j * MAXR + col];
      double m = q.x * q.x + q.y * q.y;
      if (m > best) best = m, piv = j;
    }
    if (piv != col) {
      for (int k = 0; k < r; ++k) {
        cplx tmp = A[col * MAXR + k];
        A[col * MAXR + k] = A[piv * MAXR + k];
        A[piv * MAXR + k] = tmp;
      }
      cplx tmp = y[col];
      y[col] = y[piv];
      y[piv] = tmp;
    }
    cplx d = A[col * MAXR + col];
    double den = d.x * d.x + d.y * d.y;
    if (den == 0) continue;
    cplx inv = mkc(d.x / den, -d.y / den);
    for (int j = col + 1; j < r; ++j) {
      cplx f = cmul(A[j * MAXR + col], inv);
      for (int k = col; k < r; ++k) A[j * MAXR + k] = csub(A[j * MAXR + k], cmul(f, A[col * MAXR + k]));
      y[j] = csub(y[j], cmul(f, y[col]));
    }
  }
  for (int j = r - 1; j >= 0; --j) {
    cplx acc = y[j];
    for (int k = j + 1; k < r; ++k) acc = csub(acc, cmul(A[j * MAXR + k], y[k]));
    cplx d = A[j * MAXR + j];
    double den = d.x * d.x + d.y * d.y;
    y[j] = den > 0 ? mkc((acc.x * d.x + acc.y * d.y) / den, (acc.y * d.x - acc.x * d.y) / den) : mkc(0, 0);
  }
  cplx g = mkc(0, 0);
  for (int j = 0; j < r; ++j) cfma(g, et[(size_t)b * r + j], y[j]);
  G[t] = g;
}

}  // namespace

struct GmresWork {
  std::vector<void *> mine;
  bool failed = false;
};

static void *walloc(GmresWork &W, size_t bytes) {
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

// Unique elements of the EOM vectors of (part, K): the 2h1p / 2p1h amplitudes are
// stored twice (r[ki][ka](i,a,b) = -r[ki][kb](i,b,a) for EA, r[ki][kj](i,j,a) =
// -r[kj][ki](j,i,a) for IP; zero on the diagonal of a block paired with itself).
// pk[p] = full index of unique element p (the 1h / 1p part, then the canonical
// copies in storage order); unp[x] = +-(p + 1) for the element x of a full vector
// that equals +-unique p, 0 for a structural zero.  The unit weight of every
// unique element reproduces the unique-pair inner product of the full vectors.
// pkm[p] is the full index of the other copy (-1 for the 1h / 1p part); zl lists the
// structural zeros.
static void build_pack(const ccgf_ctx *c, int part, int K, long long n, std::vector<long long> &pk,
                       std::vector<int> &unp, std::vector<long long> &pkm, std::vector<long long> &zl) {
  const int nk = c->nk, no = c->no, nv = c->nv;
  auto c3 = [&](int a, int b, int d) { return c->kc3_h[((size_t)a * nk + b) * nk + d]; };
  unp.assign((size_t)n, 0);
  pk.clear();
  pkm.clear();
  zl.clear();
  const int n1 = part == CCGF_PART_IP ? no : nv;
  for (int x = 0; x < n1; ++x) {
    pk.push_back(x);
    pkm.push_back(-1);
    unp[x] = (int)pk.size();
  }
  if (part == CCGF_PART_EA) {
    const long long b2 = (long long)no * nv * nv;
    for (int ki = 0; ki < nk; ++ki)
      for (int ka = 0; ka < nk; ++ka) {
        const int kb = c3(K, ki, ka);
        if (ka > kb) continue;
        const long long off = nv + (ki * nk + ka) * b2, offm = nv + (ki * nk + kb) * b2;
        for (int i = 0; i < no; ++i)
          for (int a = 0; a < nv; ++a)
            for (int b = 0; b < nv; ++b) {
              if (ka == kb && a == b) zl.push_back(off + ((long long)i * nv + a) * nv + b);
              if (ka == kb && a >= b) continue;
              pk.push_back(off + ((long long)i * nv + a) * nv + b);
              pkm.push_back(offm + ((long long)i * nv + b) * nv + a);
              unp[off + ((long long)i * nv + a) * nv + b] = (int)pk.size();
              unp[offm + ((long long)i * nv + b) * nv + a] = -(int)pk.size();
            }
      }
  } else {
    const long long b2 = (long long)no * no * nv;
    for (int ki = 0; ki < nk; ++ki)
      for (int kj = ki; kj < nk; ++kj) {
        const long long off = no + (ki * nk + kj) * b2, offm = no + (kj * nk + ki) * b2;
        for (int i = 0; i < no; ++i)
          for (int j = 0; j < no; ++j) {
            if (ki == kj && i == j)
              for (int a = 0; a < nv; ++a) zl.push_back(off + ((long long)i * no + j) * nv + a);
            if (ki == kj && i >= j) continue;
            for (int a = 0; a < nv; ++a) {
              pk.push_back(off + ((long long)i * no + j) * nv + a);
              pkm.push_back(offm + ((long long)j * no + i) * nv + a);
              unp[off + ((long long)i * no + j) * nv + a] = (int)pk.size();
              unp[offm + ((long long)j * no + i) * nv + a] = -(int)pk.size();
            }
          }
      }
  }
}

int solve_batched(ccgf_ctx *c, int part, int K, int nrhs, const int *rhs_orb, const double *rhs_omega, double eta,
                  const cplx *Bvecs, const cplx *Evecs, cplx *Gout, ccgf_stats *st, cplx *Xout, const Guess *guess,
                  cplx *Gcols, int ncols, const double *rhs_peta, double *rhs_res) {
  const long long n = vec_len(c, part);
  const int n1 = part == CCGF_PART_IP ? c->no : c->nv;
  const double sM = part == CCGF_PART_IP ? 1.0 : -1.0;
  const double sE = part == CCGF_PART_IP ? -1.0 : 1.0;
  const int kr = c->opt.recycle_k;          // recycled pairs (0: GMRES(m))
  const int kslots = std::max(kr, 1);
  int Bmax = std::max(1, std::min(c->opt.max_batch, nrhs));
  // GMRES keeps its Krylov basis (and w) as unique elements only, which halves the
  // orthogonalisation traffic; GCROT keeps full vectors (its recycled pairs are full)
  const bool packed = kr == 0;
  std::vector<long long> hpk, hpkm, hzl;
  std::vector<int> hunp;
  if (packed) build_pack(c, part, K, n, hpk, hunp, hpkm, hzl);
  const long long nb = packed ? (long long)hpk.size() : n;  // basis vector length
  {
    // fit the batch to the free device memory: per slot the basis of restart_m + 1 vectors,
    // eight full-length work vectors and the sigma product's workspace (1.5 vectors)
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
      const double per_slot = 16.0 * ((double)nb * (c->opt.restart_m + 1) + (double)n * (7.5 + 2 * kslots));
      const double budget = 0.92 * (double)fr - 16.0 * 4.0 * (double)n - 64.0 * (1 << 20);
      const int fit = budget > 0 ? (int)std::min<double>(budget / per_slot, 1 << 20) : 0;
      if (fit < 1)
        return set_err(c, CCGF_ENOMEM, "not enough device memory for one right-hand side's Krylov basis "
                                       "(reduce restart_m)");
      Bmax = std::min(Bmax, fit);
    }
  }
  // cycle lengths: restart_m, and restart_tail for cycles that start once the queue is
  // empty and at most a quarter of the slots are still busy (few slots: long cycles are
  // cheap to orthogonalise and help the slowest solves most); m sizes the workspace
  const int m_run = c->opt.restart_m;
  int m = m_run;
  if (kr == 0 && c->opt.restart_tail > m_run) {
    size_t fr = 0, tot = 0;
    const size_t per_col = sizeof(cplx) * (size_t)Bmax * n;
    int fit = m_run;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess && per_col > 0) {
      const double cols = 0.7 * (double)fr / (double)per_col - 8.0;  // basis columns that fit
      if (cols > m_run) fit = (int)std::min<double>(c->opt.restart_tail, cols);
    }
    m = std::max(m_run, std::min(c->opt.restart_tail, fit));
  }
  const int m_tail = m;
  const int nchunk = (int)((n + DOT_CHUNK - 1) / DOT_CHUNK);
  const int n1b = packed ? (int)nb : n1;                     // unit weights when packed
  const int nchb = (int)((nb + DOT_CHUNK - 1) / DOT_CHUNK);
  const int ldp = std::max(m, kslots) + 1;
  hipStream_t s = c->stream;
  GmresWork W;
  const size_t vb = (size_t)Bmax * n;
  const size_t svi = vb;
  const size_t svb = (size_t)Bmax * nb;  // basis column stride
  cplx *V = (cplx *)walloc(W, sizeof(cplx) * svb * (m + 1));
  long long *pkd = packed ? (long long *)walloc(W, sizeof(long long) * std::max<size_t>(1, hpk.size())) : nullptr;
  int *unpd = packed ? (int *)walloc(W, sizeof(int) * (size_t)n) : nullptr;
  long long *pkmd = packed ? (long long *)walloc(W, sizeof(long long) * std::max<size_t>(1, hpkm.size())) : nullptr;
  long long *zld = packed ? (long long *)walloc(W, sizeof(long long) * std::max<size_t>(1, hzl.size())) : nullptr;
  long long *uoffb = (long long *)walloc(W, sizeof(long long) * Bmax);
  cplx *Ub = (cplx *)walloc(W, sizeof(cplx) * vb * kslots);
  cplx *Cb = (cplx *)walloc(W, sizeof(cplx) * vb * kslots);
  cplx *X = (cplx *)walloc(W, sizeof(cplx) * vb);
  cplx *R = (cplx *)walloc(W, sizeof(cplx) * vb);
  cplx *Z = (cplx *)walloc(W, sizeof(cplx) * vb);
  cplx *Wv = (cplx *)walloc(W, sizeof(cplx) * vb);
  cplx *Wc = (cplx *)walloc(W, sizeof(cplx) * vb);
  cplx *Bv = (cplx *)walloc(W, sizeof(cplx) * vb);
  cplx *diag = (cplx *)walloc(W, sizeof(cplx) * n);
  cplx *H = (cplx *)walloc(W, sizeof(cplx) * Bmax * (m + 1) * m);
  cplx *H0 = (cplx *)walloc(W, sizeof(cplx) * Bmax * (m + 1) * m);
  cplx *Bm = (cplx *)walloc(W, sizeof(cplx) * Bmax * kslots * m);
  cplx *cs = (cplx *)walloc(W, sizeof(cplx) * Bmax * m);
  cplx *sn = (cplx *)walloc(W, sizeof(cplx) * Bmax * m);
  cplx *g = (cplx *)walloc(W, sizeof(cplx) * Bmax * (m + 1));
  cplx *htmp = (cplx *)walloc(W, sizeof(cplx) * Bmax * ldp);
  cplx *partial = (cplx *)walloc(W, sizeof(cplx) * (size_t)Bmax * nchunk * ldp);
  cplx *shift = (cplx *)walloc(W, sizeof(cplx) * Bmax);
  cplx *pshift = (cplx *)walloc(W, sizeof(cplx) * Bmax);
  cplx *ysol = (cplx *)walloc(W, sizeof(cplx) * Bmax * m);
  cplx *tv = (cplx *)walloc(W, sizeof(cplx) * Bmax * kslots);
  cplx *dv = (cplx *)walloc(W, sizeof(cplx) * Bmax * (m + 1));
  double *inv = (double *)walloc(W, sizeof(double) * Bmax);
  double *thresh = (double *)walloc(W, sizeof(double) * Bmax);
  int *active = (int *)walloc(W, sizeof(int) * Bmax);
  int *kused = (int *)walloc(W, sizeof(int) * Bmax);
  int *skip = (int *)walloc(W, sizeof(int) * Bmax);
  int *jlim = (int *)walloc(W, sizeof(int) * Bmax);
  int *aidx = (int *)walloc(W, sizeof(int) * Bmax);
  int *need = (int *)walloc(W, sizeof(int) * Bmax);
  int *fmask = (int *)walloc(W, sizeof(int) * Bmax);
  int *jvd = (int *)walloc(W, sizeof(int) * Bmax);
  long long *goff = (long long *)walloc(W, sizeof(long long) * 2 * Bmax);
  double *w0n = (double *)walloc(W, sizeof(double) * Bmax);
  long long *uoff = (long long *)walloc(W, sizeof(long long) * Bmax);
  long long *eoff = (long long *)walloc(W, sizeof(long long) * Bmax);
  // whole columns: e_r . x for every left vector r of the call (Eqs. 7 and 9 off the diagonal)
  const bool cols = Gcols != nullptr && ncols > 0;
  cplx *partE = cols ? (cplx *)walloc(W, sizeof(cplx) * (size_t)Bmax * nchunk * ncols) : nullptr;
  cplx *outE = cols ? (cplx *)walloc(W, sizeof(cplx) * (size_t)Bmax * ncols) : nullptr;
  long long *zoff = cols ? (long long *)walloc(W, sizeof(long long) * Bmax) : nullptr;
  if (W.failed) {
    wfree(W);
    return set_err(c, CCGF_ENOMEM, "solver workspace allocation failed (reduce max_batch, restart_m or recycle_k)");
  }
  const unsigned gx = (unsigned)((n + 255) / 256), gxb = (unsigned)((nb + 255) / 256);
  hipLaunchKernelGGL(k_diag, dim3(gx), dim3(256), 0, s, part, c->nk, c->no, c->nv, K, c->kc3, c->Foo, c->Fvv, diag,
                     n);
  if (packed) {
    hipMemcpyAsync(pkd, hpk.data(), sizeof(long long) * hpk.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(unpd, hunp.data(), sizeof(int) * (size_t)n, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(pkmd, hpkm.data(), sizeof(long long) * hpkm.size(), hipMemcpyHostToDevice, s);
    if (!hzl.empty()) hipMemcpyAsync(zld, hzl.data(), sizeof(long long) * hzl.size(), hipMemcpyHostToDevice, s);
  }

  int status = CCGF_OK;
  const double peta = std::max(eta, c->opt.precond_eta);
  const double rr = c->opt.reorth_ratio > 0 ? c->opt.reorth_ratio : 0.1;
  const double ratio2 = rr * rr;
  std::vector<cplx> hshift(Bmax), hpshift(Bmax), hh((size_t)Bmax * ldp);
  std::vector<double> hbnorm(Bmax), hthr(Bmax), hrn(Bmax), hinv(Bmax);
  std::vector<int> hconv(Bmax), hkused(Bmax), hact(Bmax), hskip(Bmax), its(Bmax), hjlim(Bmax), hneed(Bmax);
  std::vector<long long> hoff(Bmax), hoffb(Bmax), heoff(Bmax);
  std::vector<int> alist;
  alist.reserve(Bmax);
  const double tol = c->opt.tol;
  const int maxit = c->opt.maxiter;
  auto sync = [&](const char *what) -> int {
    if (hipStreamSynchronize(s) != hipSuccess) return hip_check(c, hipGetLastError(), what);
    return hip_check(c, hipGetLastError(), what);
  };
  // weighted squared norms of the B vectors at Xp into hh[v * ldp]
  auto norms = [&](const cplx *Xp, int B) {
    hipLaunchKernelGGL(k_dots, dim3(nchunk, B), dim3(256), 0, s, Xp, uoff, 0LL, 1, Xp, n, n1, 1,
                       (const int *)nullptr, partial, nchunk, ldp, (const int *)nullptr);
    hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchunk, ldp, 1, (const int *)nullptr, htmp,
                       ldp, (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)nullptr);
  };
  // true residual b - A x of the listed right-hand sides into R and its norm into hh
  auto true_residual = [&](int B) -> int {
    const int np = (int)alist.size();
    if (np == 0) return CCGF_OK;
    hipMemcpyAsync(aidx, alist.data(), sizeof(int) * np, hipMemcpyHostToDevice, s);
    hipLaunchKernelGGL(k_gather_precond, dim3(gx, np), dim3(256), 0, s, Z, X, diag, shift, 0.0, n, aidx, 0,
                       (const int *)nullptr, 0LL, (const int *)nullptr, n);
    int rc = sigma_apply(c, part, K, np, Z, Wc);
    if (rc != CCGF_OK) return rc;
    if (st) st->n_sigma += np;
    hipLaunchKernelGGL(k_residual_c, dim3(gx, np), dim3(256), 0, s, R, Bv, X, Wc, shift, sM, n, aidx);
    if (packed) {
      const long long tot = nb + (long long)hzl.size();
      hipLaunchKernelGGL(k_antisym, dim3((unsigned)((tot + 255) / 256), np), dim3(256), 0, s, R, n,
                         (const long long *)pkd, (const long long *)pkmd, nb, (const long long *)zld,
                         (long long)hzl.size(), aidx);
    }
    norms(R, B);
    hipMemcpyAsync(hh.data(), htmp, sizeof(cplx) * B * ldp, hipMemcpyDeviceToHost, s);
    return sync("true residual");
  };

  // Slots of the batch hold right-hand sides; a slot whose right-hand side has
  // converged (or spent maxiter) is retired at the next cycle boundary (G = e.x,
  // statistics) and refilled with the next pending right-hand side, so the batch
  // stays full while any remain.  With recycling (GCROT) the recycled space
  // belongs to the whole batch, which is therefore refilled only when empty.
  const int B = Bmax;
  const bool refill_each = kr == 0;
  std::vector<int> rhs_of(B, -1);
  int next = 0;
  for (int v = 0; v < B; ++v) {
    hoff[v] = (long long)v * n;  // each slot's own vector inside a [B][n] batch
    hoffb[v] = (long long)v * nb;
    heoff[v] = 0;
    hconv[v] = 1;
    its[v] = 0;
    hbnorm[v] = hrn[v] = 0;
  }
  hipMemcpyAsync(uoff, hoff.data(), sizeof(long long) * B, hipMemcpyHostToDevice, s);
  hipMemcpyAsync(uoffb, hoffb.data(), sizeof(long long) * B, hipMemcpyHostToDevice, s);
  if (cols) hipMemsetAsync(zoff, 0, sizeof(long long) * B, s);
  // G = e . x (bilinear, Eq. 7), statistics and solutions of the listed slots; frees them
  auto retire = [&](const std::vector<int> &fin) -> int {
    alist.clear();
    for (int v : fin)
      if (!hconv[v] && hbnorm[v] > 0) alist.push_back(v);
    if (!alist.empty()) {  // final true residual of right-hand sides that spent their budget
      std::vector<int> cand = alist;
      if (int rc = true_residual(B)) return rc;
      for (int v : cand) hrn[v] = std::sqrt(std::max(hh[(size_t)v * ldp].x, 0.0));
    }
    std::vector<int> msk(B, 0);
    for (int v : fin) msk[v] = 1;
    hipMemcpyAsync(fmask, msk.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
    hipLaunchKernelGGL(k_dots, dim3(nchunk, B), dim3(256), 0, s, Evecs, eoff, 0LL, 1, X, n, n1, 0,
                       (const int *)fmask, partial, nchunk, ldp, (const int *)nullptr);
    hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchunk, ldp, 1, (const int *)fmask, htmp,
                       ldp, (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)nullptr);
    hipMemcpyAsync(hh.data(), htmp, sizeof(cplx) * B * ldp, hipMemcpyDeviceToHost, s);
    std::vector<cplx> hcol;
    if (cols) {  // every left vector of the call against the finished solutions
      hipLaunchKernelGGL(k_dots, dim3(nchunk, B), dim3(256), 0, s, Evecs, zoff, (long long)n, ncols, X, n, n1, 0,
                         (const int *)fmask, partE, nchunk, ncols, (const int *)nullptr);
      hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partE, nchunk, ncols, ncols, (const int *)fmask,
                         outE, ncols, (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr,
                         (const int *)nullptr);
      hcol.resize((size_t)B * ncols);
      hipMemcpyAsync(hcol.data(), outE, sizeof(cplx) * hcol.size(), hipMemcpyDeviceToHost, s);
    }
    if (Xout)  // solutions, for the reduced model
      for (int v : fin)
        hipMemcpyAsync(Xout + (size_t)rhs_of[v] * n, X + (size_t)v * n, sizeof(cplx) * n, hipMemcpyDeviceToDevice, s);
    if (int rc2 = sync("G assembly")) return rc2;
    for (int v : fin) {
      Gout[rhs_of[v]] = hh[(size_t)v * ldp];
      if (cols)
        for (int r = 0; r < ncols; ++r) Gcols[(size_t)rhs_of[v] * ncols + r] = hcol[(size_t)v * ncols + r];
      double rel = hbnorm[v] > 0 ? hrn[v] / hbnorm[v] : 0.0;
      bool ok = hbnorm[v] == 0.0 || rel <= tol;
      if (rhs_res) rhs_res[rhs_of[v]] = rel;
      if (st) {
        st->n_solves += 1;
        st->n_iterations += its[v];
        st->max_iterations = std::max(st->max_iterations, its[v]);
        st->max_rel_residual = std::max(st->max_rel_residual, rel);
        if (!ok) st->n_unconverged += 1;
      }
      if (!ok) status = CCGF_ENOCONV;
      rhs_of[v] = -1;
    }
    return CCGF_OK;
  };
  // start the listed (just assigned) slots from x0 = 0, r0 = b
  auto load = [&](const std::vector<int> &fresh) -> int {
    std::vector<int> msk(B, 0);
    for (int v : fresh) {
      const int r = rhs_of[v];
      msk[v] = 1;
      hshift[v] = mkc(rhs_omega[r], sE * eta);
      hpshift[v] = mkc(rhs_omega[r], sE * (rhs_peta && rhs_peta[r] >= 0 ? std::max(eta, rhs_peta[r]) : peta));
      heoff[v] = (long long)rhs_orb[r] * n;
      hipMemcpyAsync(Bv + (size_t)v * n, Bvecs + (size_t)rhs_orb[r] * n, sizeof(cplx) * n, hipMemcpyDeviceToDevice,
                     s);
      hipMemsetAsync(X + (size_t)v * n, 0, sizeof(cplx) * n, s);
      hipMemcpyAsync(R + (size_t)v * n, Bvecs + (size_t)rhs_orb[r] * n, sizeof(cplx) * n, hipMemcpyDeviceToDevice,
                     s);
    }
    hipMemcpyAsync(shift, hshift.data(), sizeof(cplx) * B, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(pshift, hpshift.data(), sizeof(cplx) * B, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(eoff, heoff.data(), sizeof(long long) * B, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(fmask, msk.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
    hipLaunchKernelGGL(k_dots, dim3(nchunk, B), dim3(256), 0, s, Bv, uoff, 0LL, 1, Bv, n, n1, 1, (const int *)fmask,
                       partial, nchunk, ldp, (const int *)nullptr);
    hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchunk, ldp, 1, (const int *)fmask, htmp,
                       ldp, (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)nullptr);
    hipMemcpyAsync(hh.data(), htmp, sizeof(cplx) * B * ldp, hipMemcpyDeviceToHost, s);
    if (int rc = sync("solver start")) return rc;
    for (int v : fresh) {
      hbnorm[v] = std::sqrt(std::max(hh[(size_t)v * ldp].x, 0.0));
      hrn[v] = hbnorm[v];
      hthr[v] = tol * hbnorm[v];
      hconv[v] = hbnorm[v] == 0.0;
      its[v] = 0;
    }
    hipMemcpyAsync(thresh, hthr.data(), sizeof(double) * B, hipMemcpyHostToDevice, s);
    if (guess) {  // start from the network's guess where its residual is below ||b||
      std::vector<int> gl;
      std::vector<long long> go(2 * B);
      for (int v : fresh) {
        const int q = guess->qidx[rhs_of[v]];
        if (q < 0 || hbnorm[v] == 0.0) continue;
        go[gl.size()] = (long long)q * (guess->qs_q ? guess->qs_q : guess->R * n);
        go[B + gl.size()] = (long long)rhs_of[v] * guess->R;
        gl.push_back(v);
      }
      if (!gl.empty()) {
        const int ng = (int)gl.size();
        hipMemcpyAsync(goff, go.data(), sizeof(long long) * 2 * B, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(aidx, gl.data(), sizeof(int) * ng, hipMemcpyHostToDevice, s);
        hipLaunchKernelGGL(k_expand, dim3(gx, ng), dim3(256), 0, s, X, guess->Q, goff, guess->chat, goff + B,
                           guess->R, n, aidx, guess->qs_i ? guess->qs_i : n);
        if (packed) {  // keep x exactly antisymmetric: sigma is evaluated only on such vectors
          const long long tot = nb + (long long)hzl.size();
          hipLaunchKernelGGL(k_antisym, dim3((unsigned)((tot + 255) / 256), ng), dim3(256), 0, s, X, n,
                             (const long long *)pkd, (const long long *)pkmd, nb, (const long long *)zld,
                             (long long)hzl.size(), aidx);
        }
        alist = gl;
        if (int rc = true_residual(B)) return rc;
        for (int v : gl) {
          const double rn = std::sqrt(std::max(hh[(size_t)v * ldp].x, 0.0));
          if (rn < guess->accept * hbnorm[v]) {
            hrn[v] = rn;
            hconv[v] = rn <= hthr[v];
            if (st) st->n_guess += 1;
          } else {  // discard: x0 = 0, r0 = b
            hipMemsetAsync(X + (size_t)v * n, 0, sizeof(cplx) * n, s);
            hipMemcpyAsync(R + (size_t)v * n, Bv + (size_t)v * n, sizeof(cplx) * n, hipMemcpyDeviceToDevice, s);
            if (st) st->n_guess_rejected += 1;
          }
        }
      }
    }
    return CCGF_OK;
  };

  // Each slot runs its own restart cycles: one Arnoldi step per loop pass for
  // every slot inside a cycle (per-slot column hj), the cycle end (correction,
  // residual, convergence) as soon as the slot's Givens step stops it, then a
  // new cycle, or retirement and refill.  With recycling the cycles of the
  // whole batch are kept in step instead (the recycled pairs are shared).
  std::vector<int> hj(B, 0), incyc(B, 0), smask(B, 0);
  int cyc = 0;  // synchronised cycles (recycling)
  while (true) {
    {  // retire finished slots, refill free ones
      std::vector<int> fin, fresh;
      bool busy = false;
      for (int v = 0; v < B; ++v)
        if (rhs_of[v] >= 0) {
          if (!incyc[v] && (hconv[v] || its[v] >= maxit)) fin.push_back(v);
          else busy = true;
        }
      if (!refill_each && busy) fin.clear();
      if (!fin.empty())
        if (int rc = retire(fin)) {
          wfree(W);
          return rc;
        }
      bool empty = true;
      for (int v = 0; v < B; ++v) empty = empty && rhs_of[v] < 0;
      if (refill_each || empty)
        for (int v = 0; v < B && next < nrhs; ++v)
          if (rhs_of[v] < 0) {
            rhs_of[v] = next++;
            fresh.push_back(v);
          }
      if (!fresh.empty()) {
        if (int rc = load(fresh)) {
          wfree(W);
          return rc;
        }
        if (!refill_each) cyc = 0;
      }
    }
    {  // start cycles
      bool anyin = false;
      int busy = 0;
      for (int v = 0; v < B; ++v) {
        anyin = anyin || incyc[v];
        busy += rhs_of[v] >= 0 && !hconv[v] && its[v] < maxit;
      }
      const int mcyc = (refill_each && next >= nrhs && 4 * busy <= B) ? m_tail : m_run;
      int nstart = 0, occupied = 0;
      for (int v = 0; v < B; ++v) {
        occupied += rhs_of[v] >= 0;
        smask[v] = rhs_of[v] >= 0 && !incyc[v] && !hconv[v] && its[v] < maxit && (refill_each || !anyin);
        if (smask[v]) {
          ++nstart;
          incyc[v] = 1;
          hj[v] = 0;
          hjlim[v] = std::min(mcyc, std::max(0, maxit - its[v]));  // iteration budget of this cycle
          hinv[v] = hrn[v] > 0 ? 1.0 / hrn[v] : 0.0;
        }
      }
      if (nstart > 0) {  // (host arrays stay untouched until the step's synchronisation)
        hipMemcpyAsync(fmask, smask.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(jlim, hjlim.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(inv, hinv.data(), sizeof(double) * B, hipMemcpyHostToDevice, s);
        hipMemcpyAsync(w0n, hrn.data(), sizeof(double) * B, hipMemcpyHostToDevice, s);
        hipLaunchKernelGGL(k_scale_pack, dim3(gxb, B), dim3(256), 0, s, V, R, inv, nb, (const long long *)pkd, n,
                           fmask);  // V_0 = r / ||r||
        hipLaunchKernelGGL(k_cycle_start, dim3(B), dim3(256), 0, s, m, kslots, fmask, w0n, H, H0, Bm, g, kused);
      }
      bool anyc = false;
      for (int v = 0; v < B; ++v) anyc = anyc || incyc[v];
      if (!anyc) {
        if (occupied == 0 && next >= nrhs) break;
        continue;  // occupied slots are all finished: retire them first
      }
    }
    const int kc = refill_each ? 0 : std::min(cyc, kr);  // recycled pairs in use
    const int rslot = kr > 0 ? cyc % kr : 0;
    // one Arnoldi step for every slot inside a cycle
    alist.clear();
    for (int v = 0; v < B; ++v) {
      hact[v] = incyc[v];
      if (hact[v]) alist.push_back(v);
    }
    const int na = (int)alist.size();
    hipMemcpyAsync(active, hact.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(jvd, hj.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
    hipMemcpyAsync(aidx, alist.data(), sizeof(int) * na, hipMemcpyHostToDevice, s);
    hipLaunchKernelGGL(k_gather_precond, dim3(gx, na), dim3(256), 0, s, Z, V, diag, pshift, sM, n, aidx, 1, jvd,
                       (long long)svb, (const int *)unpd, nb);
    int rc = sigma_apply(c, part, K, na, Z, Wc, c->opt.precision);
    if (rc != CCGF_OK) {
      wfree(W);
      return rc;
    }
    if (st) st->n_sigma += na;
    hipLaunchKernelGGL(k_scatter_shift, dim3(gxb, na), dim3(256), 0, s, Wv, Z, Wc, shift, sM, nb, aidx,
                       (const long long *)pkd, n);
    // ||w||^2 before projection (for the reorthogonalisation test)
    hipLaunchKernelGGL(k_dots, dim3(nchb, B), dim3(256), 0, s, Wv, uoffb, 0LL, 1, Wv, nb, n1b, 1, active, partial,
                       nchb, ldp, (const int *)nullptr);
    hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchb, ldp, 1, active, htmp, ldp,
                       (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)nullptr);
    hipLaunchKernelGGL(k_take_norm, dim3((B + 63) / 64), dim3(64), 0, s, B, htmp, ldp, w0n, active);
    // classical Gram-Schmidt against the recycled C and V_0..V_j, a second pass where the first
    // removed most of w
    for (int pass = 0; pass < 2; ++pass) {
      const int *mask = pass == 0 ? active : need;
      if (kc > 0) {  // (GCROT: full vectors, nb = n)
        hipLaunchKernelGGL(k_dots, dim3(nchunk, B), dim3(256), 0, s, Cb, uoff, (long long)svi, kc, Wv, n, n1, 1,
                           mask, partial, nchunk, ldp, (const int *)nullptr);
        hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchunk, ldp, kc, mask, htmp, ldp, Bm, m,
                           (long long)kslots * m, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)jvd);
        hipLaunchKernelGGL(k_sub_proj, dim3(gx, B), dim3(256), 0, s, Wv, Cb, (long long)svi, n, kc, htmp, ldp, mask,
                           (const int *)nullptr);
      }
      hipLaunchKernelGGL(k_dots, dim3(nchb, B), dim3(256), 0, s, V, uoffb, (long long)svb, 1, Wv, nb, n1b, 1, mask,
                         partial, nchb, ldp, (const int *)jvd);
      hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchb, ldp, 1, mask, htmp, ldp, H, m,
                         (long long)(m + 1) * m, 0, H0, (const int *)jvd, (const int *)jvd);
      hipLaunchKernelGGL(k_sub_proj, dim3(gxb, B), dim3(256), 0, s, Wv, V, (long long)svb, nb, 1, htmp, ldp, mask,
                         (const int *)jvd);
      hipLaunchKernelGGL(k_dots, dim3(nchb, B), dim3(256), 0, s, Wv, uoffb, 0LL, 1, Wv, nb, n1b, 1, mask, partial,
                         nchb, ldp, (const int *)nullptr);
      hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchb, ldp, 1, mask, htmp, ldp,
                         (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)nullptr);
      if (pass == 0)
        hipLaunchKernelGGL(k_need_reorth, dim3((B + 63) / 64), dim3(64), 0, s, B, htmp, ldp, w0n, active, need,
                           ratio2);
    }
    hipLaunchKernelGGL(k_givens, dim3((B + 63) / 64), dim3(64), 0, s, B, m, jvd, H, cs, sn, g, htmp, ldp, inv, active,
                       kused, thresh, jlim, H0);
    // V_{j+1} = w / h_{j+1,j} (also for j + 1 = m: the image c = V H y uses it).  k_givens
    // clears `active` of right-hand sides that finish here, so use this step's list aidx.
    hipLaunchKernelGGL(k_scale_idx, dim3(gxb, na), dim3(256), 0, s, V, Wv, inv, nb, aidx, jvd, (long long)svb);
    hipMemcpyAsync(hact.data(), active, sizeof(int) * B, hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(hneed.data(), need, sizeof(int) * B, hipMemcpyDeviceToHost, s);
    if (int rc2 = sync("solver iteration")) {
      wfree(W);
      return rc2;
    }
    if (st) {
      st->n_steps += 1;
      for (int v = 0; v < B; ++v) st->n_reorth += hneed[v];
    }
    // slots whose cycle ended in this step (all of them together when recycling)
    std::vector<int> ended;
    bool still = false;
    for (int v : alist) {
      hj[v] += 1;
      if (!hact[v]) ended.push_back(v);
      else still = true;
    }
    if (!refill_each && still) ended.clear();
    if (ended.empty()) continue;
    for (int v = 0; v < B; ++v) hskip[v] = 1;
    for (int v : ended) hskip[v] = 0;
    hipMemcpyAsync(skip, hskip.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
    // minimal-residual correction of the cycle and its image under A
    hipLaunchKernelGGL(k_backsolve, dim3(B), dim3(256), 0, s, B, m, H, g, kused, ysol, skip);
    hipLaunchKernelGGL(k_gcrot_small, dim3(B), dim3(256), 0, s, B, m, kc, Bm, H0, ysol, kused, tv, dv, skip, kslots);
    cplx *us = Ub + (size_t)rslot * svi, *cs_ = Cb + (size_t)rslot * svi;
    hipLaunchKernelGGL(k_gcrot_combine, dim3(gx, B), dim3(256), 0, s, n, m, (long long)svi, V, ysol, dv, kused, kc, Ub,
                       tv, kslots, diag, pshift, sM, us, cs_, X, R, skip, (const int *)unpd, nb, (long long)svb);
    if (kr > 0) {  // normalise the new pair so that c has unit norm
      norms(cs_, B);
      hipLaunchKernelGGL(k_inv_sqrt, dim3((B + 63) / 64), dim3(64), 0, s, B, htmp, ldp, inv, skip);
      hipLaunchKernelGGL(k_scale2, dim3(gx, B), dim3(256), 0, s, us, cs_, inv, n, skip);
    }
    norms(R, B);
    hipMemcpyAsync(hh.data(), htmp, sizeof(cplx) * B * ldp, hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(hkused.data(), kused, sizeof(int) * B, hipMemcpyDeviceToHost, s);
    if (int rc2 = sync("solver cycle")) {
      wfree(W);
      return rc2;
    }
    alist.clear();
    for (int v : ended) {
      incyc[v] = 0;
      hrn[v] = std::sqrt(std::max(hh[(size_t)v * ldp].x, 0.0));
      its[v] += hkused[v];
      hconv[v] = hrn[v] <= tol * hbnorm[v];
      // mixed precision: every cycle restarts from the FP64 true residual (iterative refinement)
      if (hconv[v] || c->opt.precision != CCGF_PLAIN_F64) alist.push_back(v);
    }
    // confirm convergence with the true residual (the recursive one can drift)
    if (!alist.empty()) {
      std::vector<int> cand = alist;
      if (int rc3 = true_residual(B)) {
        wfree(W);
        return rc3;
      }
      std::vector<int> redo(B, 0);
      int nredo = 0;
      for (int v : cand) {
        hrn[v] = std::sqrt(std::max(hh[(size_t)v * ldp].x, 0.0));
        hconv[v] = hrn[v] <= tol * hbnorm[v];
        if (!hconv[v]) redo[v] = 1, ++nredo;
      }
      const int kcn = refill_each ? 0 : std::min(cyc + 1, kr);
      if (nredo && kcn > 0) {
        // restore r _|_ C for the restarted residuals: x += U (C^H r), r -= C (C^H r)
        hipMemcpyAsync(active, redo.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
        hipLaunchKernelGGL(k_dots, dim3(nchunk, B), dim3(256), 0, s, Cb, uoff, (long long)svi, kcn, R, n, n1, 1,
                           active, partial, nchunk, ldp, (const int *)nullptr);
        hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchunk, ldp, kcn, active, htmp, ldp,
                           (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)nullptr);
        hipLaunchKernelGGL(k_add_proj, dim3(gx, B), dim3(256), 0, s, X, Ub, (long long)svi, n, kcn, htmp, ldp, active);
        hipLaunchKernelGGL(k_sub_proj, dim3(gx, B), dim3(256), 0, s, R, Cb, (long long)svi, n, kcn, htmp, ldp, active,
                           (const int *)nullptr);
        norms(R, B);
        hipMemcpyAsync(hh.data(), htmp, sizeof(cplx) * B * ldp, hipMemcpyDeviceToHost, s);
        if (int rc2 = sync("residual projection")) {
          wfree(W);
          return rc2;
        }
        for (int v = 0; v < B; ++v)
          if (redo[v]) hrn[v] = std::sqrt(std::max(hh[(size_t)v * ldp].x, 0.0));
      }
    }
    if (!refill_each) ++cyc;
  }
  wfree(W);
  return status;
}

// ------------------------------------------------------------------ shared Krylov seed
// The Krylov space of sigma from b is also that of every shifted operator
// shift I -/+ sigma, so one Arnoldi run per orbital serves all its frequencies:
// with sigma Q_m = Q_{m+1} H (H of size (m+1) x m), (shift I + sM sigma) Q_m =
// Q_{m+1} (shift I + sM H), and the GMRES iterate of each (orbital, w) over that
// space is x0 = Q_m y with y minimising || beta e_1 - (shift I + sM H) y ||.

// H[v][j + 1][j] = ||w_v|| after orthogonalisation (row-major, ldh = m) and the
// scale 1 / ||w_v|| of the next basis vector; a right-hand side whose remainder is
// negligible next to ||sigma v_j|| (the norm of H's column) has reached an
// invariant space: its basis stops at j + 1 columns
__global__ void k_seed_norm(int B, const cplx *__restrict__ htmp, int ldp, cplx *__restrict__ H, int m, int j,
                            double *__restrict__ inv, int *__restrict__ act, int *__restrict__ mlen) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= B || !act[v]) return;
  cplx *Hv = H + (size_t)v * (m + 1) * m;
  const double h = sqrt(fmax(htmp[(size_t)v * ldp].x, 0.0));
  double col2 = h * h;
  for (int i = 0; i <= j; ++i) col2 += Hv[(size_t)i * m + j].x * Hv[(size_t)i * m + j].x + Hv[(size_t)i * m + j].y * Hv[(size_t)i * m + j].y;
  Hv[(size_t)(j + 1) * m + j] = mkc(h, 0);
  if (!(h > 1e-13 * sqrt(col2))) {
    mlen[v] = j + 1;
    act[v] = 0;
    inv[v] = 0.0;
  } else {
    inv[v] = 1.0 / h;
  }
}

// Per right-hand side r (one thread each): Givens QR of (shift_r I + sM H[orb_r])
// restricted to the orbital's mlen columns, then y by back substitution into
// chat[r][0 .. m) (zero beyond mlen, and all zero if the triangle is singular).
// R (upper triangle, column j at Rw + j m), the rotations and g are per-r scratch.
__global__ void k_seed_ls(int nrhs, int m, const cplx *__restrict__ H, const int *__restrict__ mlen,
                          const int *__restrict__ orb, const cplx *__restrict__ shift, double sM,
                          const double *__restrict__ beta, cplx *__restrict__ Rw, cplx *__restrict__ cs,
                          cplx *__restrict__ sn, cplx *__restrict__ gv, cplx *__restrict__ chat) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  const int q = orb[r];
  const int me = q >= 0 ? mlen[q] : 0;
  cplx *y = chat + (size_t)r * m;
  for (int i = 0; i < m; ++i) y[i] = mkc(0, 0);
  if (me == 0) return;
  const cplx *Hq = H + (size_t)q * (m + 1) * m;
  cplx *Rr = Rw + (size_t)r * m * m, *c = cs + (size_t)r * m, *sv = sn + (size_t)r * m, *g = gv + (size_t)r * (m + 1);
  const cplx sh = shift[r];
  g[0] = mkc(beta[q], 0);
  for (int j = 0; j < me; ++j) {
    cplx *col = Rr + (size_t)j * m;
    for (int i = 0; i <= j; ++i) col[i] = cscale(Hq[(size_t)i * m + j], sM);
    col[j] = cadd(col[j], sh);
    cplx sub = cscale(Hq[(size_t)(j + 1) * m + j], sM);
    for (int i = 0; i < j; ++i) {  // earlier rotations on rows (i, i + 1)
      const cplx a0 = col[i], a1 = col[i + 1];
      col[i] = cadd(cmul(cconj(c[i]), a0), cmul(cconj(sv[i]), a1));
      col[i + 1] = csub(cmul(c[i], a1), cmul(sv[i], a0));
    }
    const double rr = hypot(hypot(col[j].x, col[j].y), hypot(sub.x, sub.y));
    if (rr == 0.0) return;  // singular: no guess
    c[j] = cscale(col[j], 1.0 / rr);
    sv[j] = cscale(sub, 1.0 / rr);
    col[j] = mkc(rr, 0);
    const cplx gj = g[j];
    g[j] = cmul(cconj(c[j]), gj);
    g[j + 1] = cscale(cmul(sv[j], gj), -1.0);
  }
  for (int i = me - 1; i >= 0; --i) {
    cplx acc = g[i];
    for (int k = i + 1; k < me; ++k) acc = csub(acc, cmul(Rr[(size_t)k * m + i], y[k]));
    y[i] = cscale(acc, 1.0 / Rr[(size_t)i * m + i].x);  // the diagonal of R is real, > 0
  }
}

int seed_krylov(ccgf_ctx *c, int part, int K, int norb, const cplx *Bvecs, int nrhs, const int *rhs_orb,
                const double *rhs_omega, double eta, Guess &gs, cplx **Qout, cplx **chat_out, ccgf_stats *st) {
  *Qout = nullptr;
  *chat_out = nullptr;
  int m = c->opt.seed_m;
  if (m <= 0 || norb <= 0 || nrhs <= 0) return CCGF_OK;
  const long long n = vec_len(c, part);
  {
    // the seed bases may take at most a third of the free device memory (the solves
    // that use them need the rest); fewer steps where they would not fit, none below 8
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) {
      const double per_col = 16.0 * (double)norb * (double)n;
      const int fit = (int)std::min<double>(fr / 3.0 / per_col - 1.0, 4096.0);
      if (fit < 8) return CCGF_OK;
      m = std::min(m, fit);
    }
  }
  const int n1 = part == CCGF_PART_IP ? c->no : c->nv;
  const double sM = part == CCGF_PART_IP ? 1.0 : -1.0;
  const double sE = part == CCGF_PART_IP ? -1.0 : 1.0;
  const int B = norb;
  const int nchunk = (int)((n + DOT_CHUNK - 1) / DOT_CHUNK);
  const int ldp = m + 2;
  const size_t vb = (size_t)B * n;
  hipStream_t s = c->stream;
  GmresWork W;
  cplx *Q = nullptr, *chat = nullptr;
  if (hipMalloc(&Q, sizeof(cplx) * vb * (m + 1)) != hipSuccess ||
      hipMalloc(&chat, sizeof(cplx) * (size_t)nrhs * m) != hipSuccess) {
    (void)hipGetLastError();
    if (Q) hipFree(Q);
    return CCGF_ENOMEM;
  }
  cplx *Z = (cplx *)walloc(W, sizeof(cplx) * vb);
  cplx *Wv = (cplx *)walloc(W, sizeof(cplx) * vb);
  cplx *H = (cplx *)walloc(W, sizeof(cplx) * B * (size_t)(m + 1) * m);
  cplx *htmp = (cplx *)walloc(W, sizeof(cplx) * B * ldp);
  cplx *partial = (cplx *)walloc(W, sizeof(cplx) * (size_t)B * nchunk * ldp);
  double *inv = (double *)walloc(W, sizeof(double) * B);
  double *beta = (double *)walloc(W, sizeof(double) * B);
  int *act = (int *)walloc(W, sizeof(int) * B);
  int *mlen = (int *)walloc(W, sizeof(int) * B);
  int *orb = (int *)walloc(W, sizeof(int) * nrhs);
  long long *uoff = (long long *)walloc(W, sizeof(long long) * B);
  cplx *shift = (cplx *)walloc(W, sizeof(cplx) * nrhs);
  cplx *Rw = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * m * m);
  cplx *cs = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * m);
  cplx *sn = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * m);
  cplx *gv = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * (m + 1));
  auto fail = [&](int rc) {
    wfree(W);
    hipFree(Q);
    hipFree(chat);
    return rc;
  };
  if (W.failed) return fail(CCGF_ENOMEM);
  const unsigned gx = (unsigned)((n + 255) / 256);
  std::vector<long long> hoff(B);
  for (int v = 0; v < B; ++v) hoff[v] = (long long)v * n;
  hipMemcpyAsync(uoff, hoff.data(), sizeof(long long) * B, hipMemcpyHostToDevice, s);
  hipMemsetAsync(Q, 0, sizeof(cplx) * vb * (m + 1), s);
  hipMemsetAsync(H, 0, sizeof(cplx) * B * (size_t)(m + 1) * m, s);
  // beta_q = ||b_q||, v_0 = b_q / beta_q
  hipLaunchKernelGGL(k_dots, dim3(nchunk, B), dim3(256), 0, s, Bvecs, uoff, 0LL, 1, Bvecs, n, n1, 1,
                     (const int *)nullptr, partial, nchunk, ldp, (const int *)nullptr);
  hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchunk, ldp, 1, (const int *)nullptr, htmp, ldp,
                     (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)nullptr);
  std::vector<cplx> hh((size_t)B * ldp);
  hipMemcpyAsync(hh.data(), htmp, sizeof(cplx) * B * ldp, hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(hip_check(c, hipGetLastError(), "seed start"));
  std::vector<double> hb(B), hinv(B);
  std::vector<int> hact(B), hml(B);
  for (int v = 0; v < B; ++v) {
    hb[v] = std::sqrt(std::max(hh[(size_t)v * ldp].x, 0.0));
    hact[v] = hb[v] > 0.0;
    hml[v] = hact[v] ? m : 0;
    hinv[v] = hact[v] ? 1.0 / hb[v] : 0.0;
  }
  hipMemcpyAsync(beta, hb.data(), sizeof(double) * B, hipMemcpyHostToDevice, s);
  hipMemcpyAsync(inv, hinv.data(), sizeof(double) * B, hipMemcpyHostToDevice, s);
  hipMemcpyAsync(act, hact.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
  hipMemcpyAsync(mlen, hml.data(), sizeof(int) * B, hipMemcpyHostToDevice, s);
  hipLaunchKernelGGL(k_scale, dim3(gx, B), dim3(256), 0, s, Q, Bvecs, inv, n, (const int *)act);
  for (int j = 0; j < m; ++j) {
    // sigma of column j through fixed operands (one captured launch sequence serves every step)
    hipMemcpyAsync(Z, Q + (size_t)j * vb, sizeof(cplx) * vb, hipMemcpyDeviceToDevice, s);
    if (int rc = sigma_apply(c, part, K, B, Z, Wv, c->opt.precision)) return fail(rc);
    if (st) st->n_sigma += B;
    for (int pass = 0; pass < 2; ++pass) {  // classical Gram-Schmidt, twice
      hipLaunchKernelGGL(k_dots, dim3(nchunk, B), dim3(256), 0, s, Q, uoff, (long long)vb, j + 1, Wv, n, n1, 1,
                         (const int *)act, partial, nchunk, ldp, (const int *)nullptr);
      hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchunk, ldp, j + 1, (const int *)act, htmp,
                         ldp, H, m, (long long)(m + 1) * m, j, (cplx *)nullptr, (const int *)nullptr,
                         (const int *)nullptr);
      hipLaunchKernelGGL(k_sub_proj, dim3(gx, B), dim3(256), 0, s, Wv, Q, (long long)vb, n, j + 1, htmp, ldp,
                         (const int *)act, (const int *)nullptr);
    }
    hipLaunchKernelGGL(k_dots, dim3(nchunk, B), dim3(256), 0, s, Wv, uoff, 0LL, 1, Wv, n, n1, 1, (const int *)act,
                       partial, nchunk, ldp, (const int *)nullptr);
    hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchunk, ldp, 1, (const int *)act, htmp, ldp,
                       (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)nullptr);
    hipLaunchKernelGGL(k_seed_norm, dim3((B + 63) / 64), dim3(64), 0, s, B, htmp, ldp, H, m, j, inv, act, mlen);
    hipLaunchKernelGGL(k_scale, dim3(gx, B), dim3(256), 0, s, Q + (size_t)(j + 1) * vb, Wv, inv, n,
                       (const int *)act);
  }
  std::vector<cplx> hsh(nrhs);
  for (int r = 0; r < nrhs; ++r) hsh[r] = mkc(rhs_omega[r], sE * eta);
  hipMemcpyAsync(shift, hsh.data(), sizeof(cplx) * nrhs, hipMemcpyHostToDevice, s);
  hipMemcpyAsync(orb, rhs_orb, sizeof(int) * nrhs, hipMemcpyHostToDevice, s);
  hipLaunchKernelGGL(k_seed_ls, dim3((nrhs + 63) / 64), dim3(64), 0, s, nrhs, m, H, mlen, orb, shift, sM, beta, Rw, cs,
                     sn, gv, chat);
  if (hipStreamSynchronize(s) != hipSuccess) return fail(hip_check(c, hipGetLastError(), "seed"));
  if (int rc = hip_check(c, hipGetLastError(), "seed")) return fail(rc);
  wfree(W);
  gs.Q = Q;
  gs.chat = chat;
  gs.R = m;
  // a seed is kept wherever it leaves less residual than x0 = 0
  gs.accept = 1.0;
  gs.qs_i = (long long)vb;
  gs.qs_q = n;
  gs.qidx.assign(rhs_orb, rhs_orb + nrhs);
  for (int &q : gs.qidx)
    if (q < 0 || q >= B || !hact[q]) q = -1;
  *Qout = Q;
  *chat_out = chat;
  return CCGF_OK;
}

// Orthonormal basis of every group of ncol columns of S ([ngroup][ncol][n]), in
// place: Gram-Schmidt applied twice in the unique-pair inner product; a column
// whose remainder falls below 1e-10 of its group's largest column is set to zero.
static int group_basis(ccgf_ctx *c, long long n, int n1, int ngroup, int ncol, cplx *S) {
  const int nrhs = ngroup * ncol;
  const int nchunk = (int)((n + DOT_CHUNK - 1) / DOT_CHUNK);
  const int ldp = ncol + 1;
  hipStream_t s = c->stream;
  GmresWork W;
  cplx *Wt = (cplx *)walloc(W, sizeof(cplx) * (size_t)ngroup * n);
  cplx *partial = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * nchunk * ldp);
  cplx *out = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * ldp);
  double *inv = (double *)walloc(W, sizeof(double) * ngroup);
  long long *off_a = (long long *)walloc(W, sizeof(long long) * nrhs);
  long long *off_b = (long long *)walloc(W, sizeof(long long) * ngroup);
  long long *off_c = (long long *)walloc(W, sizeof(long long) * ngroup);
  if (W.failed) {
    wfree(W);
    return set_err(c, CCGF_ENOMEM, "basis workspace allocation failed");
  }
  const unsigned gx = (unsigned)((n + 255) / 256);
  std::vector<long long> ha(nrhs), hb(ngroup), hc(ngroup);
  std::vector<cplx> hh((size_t)nrhs * ldp);
  auto dots = [&](const cplx *U, const long long *uoff, long long su, int ni, const cplx *Wp, int B) {
    hipLaunchKernelGGL(k_dots, dim3(nchunk, B), dim3(256), 0, s, U, uoff, su, ni, Wp, n, n1, 1, (const int *)nullptr,
                       partial, nchunk, ldp, (const int *)nullptr);
    hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchunk, ldp, ni, (const int *)nullptr, out,
                       ldp, (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)nullptr);
  };
  for (int v = 0; v < nrhs; ++v) ha[v] = (long long)v * n;
  hipMemcpyAsync(off_a, ha.data(), sizeof(long long) * nrhs, hipMemcpyHostToDevice, s);
  dots(S, off_a, 0, 1, S, nrhs);
  hipMemcpyAsync(hh.data(), out, sizeof(cplx) * nrhs * ldp, hipMemcpyDeviceToHost, s);
  if (int rc = hip_check(c, hipStreamSynchronize(s), "basis norms")) {
    wfree(W);
    return rc;
  }
  std::vector<double> big(ngroup, 0.0);
  for (int b = 0; b < ngroup; ++b)
    for (int j = 0; j < ncol; ++j)
      big[b] = std::max(big[b], std::sqrt(std::max(hh[(size_t)(b * ncol + j) * ldp].x, 0.0)));
  for (int b = 0; b < ngroup; ++b) hb[b] = (long long)b * n, hc[b] = (long long)b * ncol * n;
  hipMemcpyAsync(off_b, hb.data(), sizeof(long long) * ngroup, hipMemcpyHostToDevice, s);
  hipMemcpyAsync(off_c, hc.data(), sizeof(long long) * ngroup, hipMemcpyHostToDevice, s);
  std::vector<double> hinv(ngroup);
  for (int j = 0; j < ncol; ++j) {  // column j of every group against columns 0..j-1
    for (int b = 0; b < ngroup; ++b) ha[b] = (long long)(b * ncol + j) * n;
    hipMemcpyAsync(off_a, ha.data(), sizeof(long long) * ngroup, hipMemcpyHostToDevice, s);
    hipLaunchKernelGGL(k_copy_vecs, dim3(gx, ngroup), dim3(256), 0, s, Wt, off_b, S, off_a, n);
    for (int pass = 0; pass < 2 && j > 0; ++pass) {
      dots(S, off_c, n, j, Wt, ngroup);
      hipLaunchKernelGGL(k_sub_proj_off, dim3(gx, ngroup), dim3(256), 0, s, Wt, S, off_c, n, j, out, ldp);
    }
    dots(Wt, off_b, 0, 1, Wt, ngroup);
    hipMemcpyAsync(hh.data(), out, sizeof(cplx) * ngroup * ldp, hipMemcpyDeviceToHost, s);
    if (int rc = hip_check(c, hipStreamSynchronize(s), "basis")) {
      wfree(W);
      return rc;
    }
    for (int b = 0; b < ngroup; ++b) {
      double nb = std::sqrt(std::max(hh[(size_t)b * ldp].x, 0.0));
      hinv[b] = (nb > 1e-10 * big[b] && nb > 0) ? 1.0 / nb : 0.0;  // dependent column -> zero
    }
    hipMemcpyAsync(inv, hinv.data(), sizeof(double) * ngroup, hipMemcpyHostToDevice, s);
    hipLaunchKernelGGL(k_scale, dim3(gx, ngroup), dim3(256), 0, s, Wt, Wt, inv, n, (const int *)nullptr);
    hipLaunchKernelGGL(k_copy_vecs, dim3(gx, ngroup), dim3(256), 0, s, S, off_a, Wt, off_b, n);
  }
  int rc = hip_check(c, hipStreamSynchronize(s), "basis");
  wfree(W);
  return rc;
}

// Model-order reduction (MOR paragraph): full solves at the expansion
// frequencies, an orthonormal basis S of their solutions per orbital (CGS
// twice, columns below 1e-10 of the largest zeroed), the Galerkin model
// Ht = S^H M S, bt = S^H b, et = e S, and its solution on the whole grid.
int mor_part(ccgf_ctx *c, int part, int K, int norb, const int *orbs, int nexp, const double *wexp, int nw,
             const double *omega, double eta, cplx *Gout, ccgf_stats *st) {
  const long long n = vec_len(c, part);
  const int n1 = part == CCGF_PART_IP ? c->no : c->nv;
  const double sM = part == CCGF_PART_IP ? 1.0 : -1.0;
  const double sE = part == CCGF_PART_IP ? -1.0 : 1.0;
  const int nrhs = norb * nexp;
  const int nchunk = (int)((n + DOT_CHUNK - 1) / DOT_CHUNK);
  const int ldp = nexp + 1;
  hipStream_t s = c->stream;
  GmresWork W;
  cplx *Bv = (cplx *)walloc(W, sizeof(cplx) * (size_t)norb * n);
  cplx *Ev = (cplx *)walloc(W, sizeof(cplx) * (size_t)norb * n);
  cplx *S = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * n);
  cplx *MS = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * n);
  cplx *partial = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * nchunk * ldp);
  cplx *out = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * ldp);
  cplx *Ht = (cplx *)walloc(W, sizeof(cplx) * (size_t)norb * nexp * nexp);
  cplx *bt = (cplx *)walloc(W, sizeof(cplx) * (size_t)norb * nexp);
  cplx *et = (cplx *)walloc(W, sizeof(cplx) * (size_t)norb * nexp);
  cplx *Gd = (cplx *)walloc(W, sizeof(cplx) * (size_t)norb * nw);
  double *dom = (double *)walloc(W, sizeof(double) * nw);
  long long *off_a = (long long *)walloc(W, sizeof(long long) * nrhs);
  long long *off_c = (long long *)walloc(W, sizeof(long long) * nrhs);
  if (W.failed) {
    wfree(W);
    return set_err(c, CCGF_ENOMEM, "MOR workspace allocation failed");
  }
  // full solves at the expansion frequencies (right-hand side index = b * nexp + j)
  for (int b = 0; b < norb; ++b) {
    int rc = build_vectors(c, part, K, orbs[b], Bv + (size_t)b * n, Ev + (size_t)b * n);
    if (rc != CCGF_OK) {
      wfree(W);
      return rc;
    }
  }
  std::vector<int> rorb(nrhs);
  std::vector<double> rw(nrhs);
  for (int b = 0; b < norb; ++b)
    for (int j = 0; j < nexp; ++j) rorb[b * nexp + j] = b, rw[b * nexp + j] = wexp[j];
  std::vector<cplx> gexp(nrhs);
  int status = solve_batched(c, part, K, nrhs, rorb.data(), rw.data(), eta, Bv, Ev, gexp.data(), st, S);
  if (status != CCGF_OK && status != CCGF_ENOCONV) {
    wfree(W);
    return status;
  }
  std::vector<long long> ha(nrhs), hc(nrhs);
  std::vector<cplx> hh((size_t)nrhs * ldp);
  auto upload = [&](long long *d, const std::vector<long long> &h, int cnt) {
    hipMemcpyAsync(d, h.data(), sizeof(long long) * cnt, hipMemcpyHostToDevice, s);
  };
  auto dots = [&](const cplx *U, const long long *uoff, long long su, int ni, const cplx *Wp, int B, int conjU) {
    hipLaunchKernelGGL(k_dots, dim3(nchunk, B), dim3(256), 0, s, U, uoff, su, ni, Wp, n, n1, conjU,
                       (const int *)nullptr, partial, nchunk, ldp, (const int *)nullptr);
    hipLaunchKernelGGL(k_dots_reduce, dim3(B), dim3(256), 0, s, partial, nchunk, ldp, ni, (const int *)nullptr, out,
                       ldp, (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)nullptr);
  };
  if (int rc = group_basis(c, n, n1, norb, nexp, S)) {
    wfree(W);
    return rc;
  }
  for (int b = 0; b < norb; ++b) hc[b] = (long long)b * nexp * n;
  upload(off_c, hc, norb);
  // M S, then Ht[b][j][k] = <s_bj, (M S)_bk>, bt = <s_bj, b_b>, et = e_b . s_bj
  int rc = sigma_apply(c, part, K, nrhs, S, MS, 0);
  if (rc != CCGF_OK) {
    wfree(W);
    return rc;
  }
  if (st) st->n_sigma += nrhs;
  for (int v = 0; v < nrhs; ++v) ha[v] = (long long)(v / nexp) * nexp * n;
  upload(off_a, ha, nrhs);
  dots(S, off_a, n, nexp, MS, nrhs, 1);  // out[(b,k)][j]
  std::vector<cplx> hHt((size_t)norb * nexp * nexp), hbt((size_t)norb * nexp), het((size_t)norb * nexp);
  hipMemcpyAsync(hh.data(), out, sizeof(cplx) * nrhs * ldp, hipMemcpyDeviceToHost, s);
  if (int rc2 = hip_check(c, hipStreamSynchronize(s), "MOR projection")) {
    wfree(W);
    return rc2;
  }
  for (int b = 0; b < norb; ++b)
    for (int k = 0; k < nexp; ++k)
      for (int j = 0; j < nexp; ++j) hHt[((size_t)b * nexp + j) * nexp + k] = hh[(size_t)(b * nexp + k) * ldp + j];
  dots(S, off_c, n, nexp, Bv, norb, 1);
  hipMemcpyAsync(hh.data(), out, sizeof(cplx) * norb * ldp, hipMemcpyDeviceToHost, s);
  if (int rc2 = hip_check(c, hipStreamSynchronize(s), "MOR projection")) {
    wfree(W);
    return rc2;
  }
  for (int b = 0; b < norb; ++b)
    for (int j = 0; j < nexp; ++j) hbt[(size_t)b * nexp + j] = hh[(size_t)b * ldp + j];
  dots(S, off_c, n, nexp, Ev, norb, 0);
  hipMemcpyAsync(hh.data(), out, sizeof(cplx) * norb * ldp, hipMemcpyDeviceToHost, s);
  if (int rc2 = hip_check(c, hipStreamSynchronize(s), "MOR projection")) {
    wfree(W);
    return rc2;
  }
  for (int b = 0; b < norb; ++b)
    for (int j = 0; j < nexp; ++j) het[(size_t)b * nexp + j] = hh[(size_t)b * ldp + j];
  hipMemcpyAsync(Ht, hHt.data(), sizeof(cplx) * hHt.size(), hipMemcpyHostToDevice, s);
  hipMemcpyAsync(bt, hbt.data(), sizeof(cplx) * hbt.size(), hipMemcpyHostToDevice, s);
  hipMemcpyAsync(et, het.data(), sizeof(cplx) * het.size(), hipMemcpyHostToDevice, s);
  hipMemcpyAsync(dom, omega, sizeof(double) * nw, hipMemcpyHostToDevice, s);
  const int nt = norb * nw;
  if (nexp <= 16)
    hipLaunchKernelGGL(k_mor_eval<16>, dim3((nt + 63) / 64), dim3(64), 0, s, norb, nexp, nw, dom, sE * eta, sM, Ht,
                       bt, et, Gd);
  else
    hipLaunchKernelGGL(k_mor_eval<32>, dim3((nt + 63) / 64), dim3(64), 0, s, norb, nexp, nw, dom, sE * eta, sM, Ht,
                       bt, et, Gd);
  hipMemcpyAsync(Gout, Gd, sizeof(cplx) * nt, hipMemcpyDeviceToHost, s);
  if (int rc2 = hip_check(c, hipStreamSynchronize(s), "MOR evaluation")) {
    wfree(W);
    return rc2;
  }
  wfree(W);
  return status;
}

// Training of the initial-guess network of one (part, K): plain solves at the
// training frequencies, per-orbital reduced basis and coordinates of their
// solutions, pairs (w_j, w_ref, c_ref) -> c_j, Adam on the GPU.
int learn_part(ccgf_ctx *c, int part, int K, int norb, const int *orbs, int ntrain, const double *wtr, double eta,
               const ccgf_learn_options &lo, ccgf_learn_stats *ls) {
  const long long n = vec_len(c, part);
  const int n1 = part == CCGF_PART_IP ? c->no : c->nv;
  const int nrhs = norb * ntrain, R = ntrain;
  const int nchunk = (int)((n + DOT_CHUNK - 1) / DOT_CHUNK);
  const int ldp = R + 1;
  hipStream_t s = c->stream;
  auto t0 = std::chrono::steady_clock::now();
  LearnModel M;
  M.part = part;
  M.K = K;
  M.norb = norb;
  M.ntrain = ntrain;
  M.R = R;
  M.hidden = lo.hidden;
  M.mode = lo.guess;
  M.accept = lo.accept;
  M.din = 4 + 2 * R;
  M.dout = 2 * R;
  if (hipMalloc(&M.Q, sizeof(cplx) * (size_t)nrhs * n) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(c, CCGF_ENOMEM, "no device memory for the learned basis");
  }
  auto fail = [&](int rc) {
    if (M.Q) hipFree(M.Q);
    if (M.theta) hipFree(M.theta);
    if (M.theta_p) hipFree(M.theta_p);
    return rc;
  };
  GmresWork W;
  cplx *Bv = (cplx *)walloc(W, sizeof(cplx) * (size_t)norb * n);
  cplx *Ev = (cplx *)walloc(W, sizeof(cplx) * (size_t)norb * n);
  cplx *X = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * n);
  cplx *partial = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * nchunk * ldp);
  cplx *out = (cplx *)walloc(W, sizeof(cplx) * (size_t)nrhs * ldp);
  long long *off_a = (long long *)walloc(W, sizeof(long long) * nrhs);
  if (W.failed) {
    wfree(W);
    return fail(set_err(c, CCGF_ENOMEM, "learning workspace allocation failed"));
  }
  for (int b = 0; b < norb; ++b)
    if (int rc = build_vectors(c, part, K, orbs[b], Bv + (size_t)b * n, Ev + (size_t)b * n)) {
      wfree(W);
      return fail(rc);
    }
  std::vector<int> rorb(nrhs);
  std::vector<double> rw(nrhs);
  for (int b = 0; b < norb; ++b)
    for (int j = 0; j < ntrain; ++j) rorb[b * ntrain + j] = b, rw[b * ntrain + j] = wtr[j];
  std::vector<cplx> gtr(nrhs);
  ccgf_stats st{};
  int status = solve_batched(c, part, K, nrhs, rorb.data(), rw.data(), eta, Bv, Ev, gtr.data(), &st, X);
  if (status != CCGF_OK && status != CCGF_ENOCONV) {
    wfree(W);
    return fail(status);
  }
  auto t1 = std::chrono::steady_clock::now();
  hipMemcpyAsync(M.Q, X, sizeof(cplx) * (size_t)nrhs * n, hipMemcpyDeviceToDevice, s);
  if (int rc = group_basis(c, n, n1, norb, R, M.Q)) {
    wfree(W);
    return fail(rc);
  }
  // C[b][j][i] = <q_{b,i}, x_{b,j}>
  std::vector<long long> ha(nrhs);
  for (int v = 0; v < nrhs; ++v) ha[v] = (long long)(v / ntrain) * ntrain * n;
  hipMemcpyAsync(off_a, ha.data(), sizeof(long long) * nrhs, hipMemcpyHostToDevice, s);
  hipLaunchKernelGGL(k_dots, dim3(nchunk, nrhs), dim3(256), 0, s, M.Q, off_a, n, R, X, n, n1, 1, (const int *)nullptr,
                     partial, nchunk, ldp, (const int *)nullptr);
  hipLaunchKernelGGL(k_dots_reduce, dim3(nrhs), dim3(256), 0, s, partial, nchunk, ldp, R, (const int *)nullptr, out, ldp,
                     (cplx *)nullptr, 0, 0LL, 0, (cplx *)nullptr, (const int *)nullptr, (const int *)nullptr);
  std::vector<cplx> hh((size_t)nrhs * ldp);
  hipMemcpyAsync(hh.data(), out, sizeof(cplx) * nrhs * ldp, hipMemcpyDeviceToHost, s);
  // diagonal Fock elements of the orbitals at K (features)
  std::vector<cplx> fd(norb);
  for (int b = 0; b < norb; ++b) {
    const int p = orbs[b];
    const cplx *src = p < c->no ? c->Foo + ((size_t)K * c->no + p) * c->no + p
                                : c->Fvv + ((size_t)K * c->nv + (p - c->no)) * c->nv + (p - c->no);
    hipMemcpyAsync(&fd[b], src, sizeof(cplx), hipMemcpyDeviceToHost, s);
  }
  if (int rc = hip_check(c, hipStreamSynchronize(s), "learning coordinates")) {
    wfree(W);
    return fail(rc);
  }
  wfree(W);
  M.orbs.assign(orbs, orbs + norb);
  M.wtrain.assign(wtr, wtr + ntrain);
  M.C.resize((size_t)nrhs * R);
  M.scale.assign(norb, 1.0);
  M.occ.resize(norb);
  M.fpp.resize(norb);
  for (int b = 0; b < norb; ++b) {
    M.occ[b] = orbs[b] < c->no;
    M.fpp[b] = fd[b].x;
    double big = 0;
    for (int j = 0; j < ntrain; ++j) {
      double nn = 0;
      for (int i = 0; i < R; ++i) {
        cplx v = hh[(size_t)(b * ntrain + j) * ldp + i];
        M.C[((size_t)b * ntrain + j) * R + i] = v;
        nn += v.x * v.x + v.y * v.y;
      }
      big = std::max(big, std::sqrt(nn));
    }
    M.scale[b] = big > 0 ? 1.0 / big : 1.0;
  }
  double wmax = 0;
  for (int j = 0; j < ntrain; ++j) wmax = std::max(wmax, std::fabs(wtr[j]));
  M.wscale = wmax > 0 ? wmax : 1.0;
  M.wstep = ntrain > 1 ? (wtr[ntrain - 1] - wtr[0]) / (ntrain - 1) : 1.0;
  if (!(M.wstep > 0)) M.wstep = 1.0;
  // training pairs
  std::vector<float> F, T;
  long long P = 0;
  for (int b = 0; b < norb; ++b)
    for (int j = 0; j < ntrain; ++j)
      for (int jr = std::max(0, j - 2); jr <= std::min(ntrain - 1, j + 2); ++jr) {
        F.resize((size_t)(P + 1) * M.din);
        T.resize((size_t)(P + 1) * M.dout);
        learn_features(M, b, wtr[j], jr, &F[(size_t)P * M.din]);
        for (int i = 0; i < R; ++i) {  // target: the move of the coordinates from the reference solution
          cplx v = M.C[((size_t)b * ntrain + j) * R + i], r0 = M.C[((size_t)b * ntrain + jr) * R + i];
          T[(size_t)P * M.dout + i] = (float)((v.x - r0.x) * M.scale[b]);
          T[(size_t)P * M.dout + R + i] = (float)((v.y - r0.y) * M.scale[b]);
        }
        ++P;
      }
  double L0 = 0, L1 = 0;
  // the untrained network (zero output layer) proposes the reference solution itself
  if (int rc = mlp_train(c, M.din, M.hidden, M.dout, P, F, T, lo.epochs, lo.batch, lo.lr, lo.seed, true, &M.theta,
                         &L0, &L1))
    return fail(rc);
  // preconditioner network: probe solves of every training (p, w) with each candidate damping
  double probe_s = 0, PL0 = 0, PL1 = 0;
  if (lo.probe >= 0) {
    auto tp = std::chrono::steady_clock::now();
    const int nc = CCGF_PRECOND_CANDIDATES;
    M.pbase = std::max(eta, c->opt.precond_eta);
    const int npr = nrhs * nc;
    std::vector<int> porb(npr);
    std::vector<double> pw(npr), pe(npr), pres(npr, 1.0);
    for (int r = 0; r < nrhs; ++r)
      for (int q = 0; q < nc; ++q) {
        porb[r * nc + q] = rorb[r];
        pw[r * nc + q] = rw[r];
        pe[r * nc + q] = kPrecondCand[q] * M.pbase;
      }
    GmresWork W2;
    cplx *Bp = (cplx *)walloc(W2, sizeof(cplx) * (size_t)norb * n);
    cplx *Ep = (cplx *)walloc(W2, sizeof(cplx) * (size_t)norb * n);
    if (W2.failed) {
      wfree(W2);
      return fail(set_err(c, CCGF_ENOMEM, "no device memory for the probe solves"));
    }
    for (int b = 0; b < norb; ++b)
      if (int rc = build_vectors(c, part, K, orbs[b], Bp + (size_t)b * n, Ep + (size_t)b * n)) {
        wfree(W2);
        return fail(rc);
      }
    const ccgf_options keep = c->opt;
    c->opt.maxiter = lo.probe;
    c->opt.tol = 0.0;          // run every probe for its full step count
    c->opt.restart_m = std::max(keep.restart_m, lo.probe);
    std::vector<cplx> gdump(npr);
    ccgf_stats pst{};
    int prc = solve_batched(c, part, K, npr, porb.data(), pw.data(), eta, Bp, Ep, gdump.data(), &pst, nullptr,
                            nullptr, nullptr, 0, pe.data(), pres.data());
    c->opt = keep;
    wfree(W2);
    if (prc != CCGF_OK && prc != CCGF_ENOCONV) return fail(prc);
    M.pdin = 4;
    M.pdout = nc;
    std::vector<float> PF((size_t)nrhs * M.pdin), PT((size_t)nrhs * nc);
    for (int r = 0; r < nrhs; ++r) {
      precond_features(M, rorb[r], rw[r], &PF[(size_t)r * M.pdin]);
      for (int q = 0; q < nc; ++q) PT[(size_t)r * nc + q] = (float)std::log10(std::max(pres[r * nc + q], 1e-16));
    }
    if (int rc = mlp_train(c, M.pdin, M.hidden, M.pdout, nrhs, PF, PT, lo.epochs, lo.batch, lo.lr, lo.seed + 1,
                           false, &M.theta_p, &PL0, &PL1))
      return fail(rc);
    probe_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - tp).count();
  }
  auto t2 = std::chrono::steady_clock::now();
  if (ls) {
    ls->pairs += P;
    ls->rank = R;
    ls->loss_initial += L0;
    ls->loss_final += L1;
    ls->probe_seconds += probe_s;
    ls->precond_loss_initial += PL0;
    ls->precond_loss_final += PL1;
    ls->solve_seconds += std::chrono::duration<double>(t1 - t0).count();
    ls->train_seconds += std::chrono::duration<double>(t2 - t1).count();
    ls->solve_iterations += st.n_iterations;
  }
  for (auto it = c->models.begin(); it != c->models.end(); ++it)
    if (it->part == part && it->K == K) {
      if (it->Q) hipFree(it->Q);
      if (it->theta) hipFree(it->theta);
      if (it->theta_p) hipFree(it->theta_p);
      c->models.erase(it);
      break;
    }
  c->models.push_back(M);
  return status;
}
