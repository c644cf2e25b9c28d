// Active-space self-energy correction and Dyson's equation (Eqs. 12-14):
//   Sigma_CAS(k, w)  = G_GW,CAS^-1(k, w) - G_CC,CAS^-1(k, w)            (M x M)
//   Sigma_full(k, w) = V(k) Sigma_CAS(k, w) V(k)^H                       (N x N)
//   G_CC+GW(k, w)    = [G_GW,full^-1(k, w) - Sigma_full(k, w)]^-1        (N x N)
// for every (k, w) of a batch.  The matrices are small (N, M <= 64): each batched
// step runs one work-group per matrix.  Inversions are Gauss-Jordan eliminations
// with partial pivoting on the augmented matrix [A | I] held in a scratch buffer;
// the products are one thread per output element.  The work is split into chunks
// of (k, w) points that fit the scratch buffer, so a fixed-size buffer serves any
// batch.
#include "ccgf_internal.h"

#include <algorithm>
#include <mutex>

namespace {

constexpr int DYSON_NMAX = 64;

// In place on the augmented matrices W[b] (n x 2n, row-major, left half A, right half
// I on entry): Gauss-Jordan with partial pivoting; on exit the right half is A^-1.
// bad[b * bstride] is set when a pivot vanishes (singular A).
__global__ __launch_bounds__(256) void k_gj_inverse(cplx *__restrict__ Wall, int n, int *__restrict__ bad,
                                                    int bstride) {
  const int b = blockIdx.x, tid = threadIdx.x, n2 = 2 * n;
  cplx *W = Wall + (size_t)b * n * n2;
  __shared__ double sv[256];
  __shared__ int si[256];
  __shared__ cplx fac[DYSON_NMAX];
  __shared__ cplx prow[2 * DYSON_NMAX];
  for (int col = 0; col < n; ++col) {
    // pivot: the largest |W[r][col]|, r >= col
    double best = -1.0;
    int arg = col;
    for (int r = col + tid; r < n; r += blockDim.x) {
      const cplx x = W[(size_t)r * n2 + col];
      const double m = x.x * x.x + x.y * x.y;
      if (m > best) best = m, arg = r;
    }
    sv[tid] = best;
    si[tid] = arg;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
      if (tid < o && (sv[tid + o] > sv[tid] || (sv[tid + o] == sv[tid] && si[tid + o] < si[tid]))) {
        sv[tid] = sv[tid + o];
        si[tid] = si[tid + o];
      }
      __syncthreads();
    }
    const int p = si[0];
    const double pm = sv[0];
    __syncthreads();
    if (!(pm > 0.0)) {
      if (tid == 0) bad[(size_t)b * bstride] = 1;
      return;  // the whole block leaves together (pm is shared)
    }
    // swap rows p and col, then scale the pivot row by 1 / pivot (kept in LDS)
    const cplx piv = W[(size_t)p * n2 + col];
    const double den = piv.x * piv.x + piv.y * piv.y;
    const cplx ip = mkc(piv.x / den, -piv.y / den);
    for (int j = tid; j < n2; j += blockDim.x) {
      const cplx a = W[(size_t)p * n2 + j], c0 = W[(size_t)col * n2 + j];
      prow[j] = cmul(a, ip);
      if (p != col) W[(size_t)p * n2 + j] = c0;
    }
    __syncthreads();
    for (int r = tid; r < n; r += blockDim.x) fac[r] = r == col ? mkc(0, 0) : W[(size_t)r * n2 + col];
    __syncthreads();
    for (int j = tid; j < n2; j += blockDim.x) W[(size_t)col * n2 + j] = prow[j];
    // eliminate column col from every other row
    for (int e = tid; e < n * n2; e += blockDim.x) {
      const int r = e / n2, j = e % n2;
      if (r == col) continue;
      W[(size_t)r * n2 + j] = csub(W[(size_t)r * n2 + j], cmul(fac[r], prow[j]));
    }
    __syncthreads();
  }
}

// W[b] = [A[b] | I] for A[b] = src + b * sa (n x n, leading dimension n)
__global__ void k_augment(cplx *__restrict__ W, const cplx *__restrict__ A, long long sa, int n) {
  const int b = blockIdx.x, n2 = 2 * n;
  for (int e = threadIdx.x; e < n * n2; e += blockDim.x) {
    const int r = e / n2, j = e % n2;
    W[(size_t)b * n * n2 + e] = j < n ? A[(size_t)b * sa + (size_t)r * n + j] : mkc(j - n == r ? 1.0 : 0.0, 0);
  }
}

// C[b] = alpha * (right half of W1[b]) + beta * (right half of W2[b])  (n x n)
__global__ void k_combine(cplx *__restrict__ C, long long sc, const cplx *__restrict__ W1, double alpha,
                          const cplx *__restrict__ W2, double beta, int n) {
  const int b = blockIdx.x, n2 = 2 * n;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int r = e / n, j = e % n;
    cplx v = cscale(W1[(size_t)b * n * n2 + (size_t)r * n2 + n + j], alpha);
    if (W2) v = cadd(v, cscale(W2[(size_t)b * n * n2 + (size_t)r * n2 + n + j], beta));
    C[(size_t)b * sc + e] = v;
  }
}

// S[b] = V[k(b)] X[b] V[k(b)]^H: (N x M)(M x M)(M x N); k(b) = (b0 + b) / nw
__global__ void k_backtransform(cplx *__restrict__ S, const cplx *__restrict__ X, const cplx *__restrict__ V,
                                int N, int M, int b0, int nw, cplx *__restrict__ T) {
  const int b = blockIdx.x;
  const cplx *Vk = V + (size_t)((b0 + b) / nw) * N * M;
  const cplx *Xb = X + (size_t)b * M * M;
  cplx *Tb = T + (size_t)b * N * M;
  for (int e = threadIdx.x; e < N * M; e += blockDim.x) {  // T = V X
    const int r = e / M, j = e % M;
    cplx acc = mkc(0, 0);
    for (int q = 0; q < M; ++q) cfma(acc, Vk[(size_t)r * M + q], Xb[(size_t)q * M + j]);
    Tb[e] = acc;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < N * N; e += blockDim.x) {  // S = T V^H
    const int r = e / N, j = e % N;
    cplx acc = mkc(0, 0);
    for (int q = 0; q < M; ++q) cfma(acc, Tb[(size_t)r * M + q], cconj(Vk[(size_t)j * M + q]));
    S[(size_t)b * N * N + e] = acc;
  }
}

// W[b] = [right half of W[b] - Sf[b] | I]   (n = N): G_GW^-1 - Sigma_full, augmented
__global__ void k_dyson_rhs(cplx *__restrict__ W, const cplx *__restrict__ Sf, int n) {
  const int b = blockIdx.x, n2 = 2 * n;
  cplx *Wb = W + (size_t)b * n * n2;
  // read the inverse first (row r of the right half), then overwrite: each thread owns whole rows
  for (int r = threadIdx.x; r < n; r += blockDim.x)
    for (int j = 0; j < n; ++j) {
      const cplx v = csub(Wb[(size_t)r * n2 + n + j], Sf[(size_t)b * n * n + (size_t)r * n + j]);
      Wb[(size_t)r * n2 + j] = v;
      Wb[(size_t)r * n2 + n + j] = mkc(r == j ? 1.0 : 0.0, 0);
    }
}

}  // namespace

static long long dyson_scratch_per_point(int N, int M) {
  // two M x 2M augmented matrices, one N x 2N, the N x N back-transformed self-energy,
  // the N x M intermediate and the M x M self-energy
  return 2LL * M * 2 * M + (long long)N * 2 * N + (long long)N * N + (long long)N * M + (long long)M * M;
}

// bad: one flag per (k, w) point (bstride 1) or a single flag (bstride 0)
static int dyson_cas_run(hipStream_t s, int nk, int nw, int N, int M, const cplx *Ggw, const cplx *Ggw_cas,
                         const cplx *Gcc, const cplx *V, cplx *Gout, cplx *Sfull, cplx *Scas, cplx *scratch,
                         long long scratch_elems, int *bad, int bstride) {
  const long long per = dyson_scratch_per_point(N, M);
  const int npts = nk * nw;
  const int chunk = (int)std::min<long long>(npts, scratch_elems / per);
  if (chunk < 1) return CCGF_ENOMEM;
  for (int b0 = 0; b0 < npts; b0 += chunk) {
    const int nb = std::min(chunk, npts - b0);
    cplx *WA = scratch;                                // [nb][M][2M]  G_GW,CAS
    cplx *WB = WA + (size_t)nb * M * 2 * M;            // [nb][M][2M]  G_CC,CAS
    cplx *WG = WB + (size_t)nb * M * 2 * M;            // [nb][N][2N]  G_GW,full
    cplx *SF = WG + (size_t)nb * N * 2 * N;            // [nb][N][N]   Sigma_full
    cplx *TT = SF + (size_t)nb * N * N;                // [nb][N][M]
    cplx *SC = TT + (size_t)nb * N * M;                // [nb][M][M]   Sigma_CAS
    const size_t MM = (size_t)M * M, NN = (size_t)N * N;
    hipLaunchKernelGGL(k_augment, dim3(nb), dim3(256), 0, s, WA, Ggw_cas + (size_t)b0 * MM, (long long)MM, M);
    hipLaunchKernelGGL(k_augment, dim3(nb), dim3(256), 0, s, WB, Gcc + (size_t)b0 * MM, (long long)MM, M);
    hipLaunchKernelGGL(k_augment, dim3(nb), dim3(256), 0, s, WG, Ggw + (size_t)b0 * NN, (long long)NN, N);
    hipLaunchKernelGGL(k_gj_inverse, dim3(nb), dim3(256), 0, s, WA, M, bad + (size_t)b0 * bstride, bstride);
    hipLaunchKernelGGL(k_gj_inverse, dim3(nb), dim3(256), 0, s, WB, M, bad + (size_t)b0 * bstride, bstride);
    hipLaunchKernelGGL(k_gj_inverse, dim3(nb), dim3(256), 0, s, WG, N, bad + (size_t)b0 * bstride, bstride);
    // Sigma_CAS = G_GW,CAS^-1 - G_CC,CAS^-1
    hipLaunchKernelGGL(k_combine, dim3(nb), dim3(256), 0, s, SC, (long long)MM, WA, 1.0, WB, -1.0, M);
    if (Scas)
      hipMemcpyAsync(Scas + (size_t)b0 * MM, SC, sizeof(cplx) * nb * MM, hipMemcpyDeviceToDevice, s);
    hipLaunchKernelGGL(k_backtransform, dim3(nb), dim3(256), 0, s, SF, SC, V, N, M, b0, nw, TT);
    if (Sfull)
      hipMemcpyAsync(Sfull + (size_t)b0 * NN, SF, sizeof(cplx) * nb * NN, hipMemcpyDeviceToDevice, s);
    // G = (G_GW^-1 - Sigma_full)^-1
    hipLaunchKernelGGL(k_dyson_rhs, dim3(nb), dim3(256), 0, s, WG, SF, N);
    hipLaunchKernelGGL(k_gj_inverse, dim3(nb), dim3(256), 0, s, WG, N, bad + (size_t)b0 * bstride, bstride);
    hipLaunchKernelGGL(k_combine, dim3(nb), dim3(256), 0, s, Gout + (size_t)b0 * NN, (long long)NN, WG, 1.0,
                       (const cplx *)nullptr, 0.0, N);
  }
  return hipGetLastError() == hipSuccess ? CCGF_OK : CCGF_EDEVICE;
}

static thread_local std::string g_dyson_err = "no error";

static int dyson_check(int nk, int nw, int N, int M, const double *Ggw, const double *Ggw_cas, const double *Gcc,
                       const double *V, const double *Gout) {
  if (nk < 1 || nw < 0 || N < 1 || M < 1 || M > N || N > DYSON_NMAX) {
    g_dyson_err = "sizes must satisfy nk >= 1, nw >= 0, 1 <= M <= N <= 64";
    return CCGF_EINVAL;
  }
  if (nw > 0 && (!Ggw || !Ggw_cas || !Gcc || !V || !Gout)) {
    g_dyson_err = "NULL matrix argument";
    return CCGF_EINVAL;
  }
  return CCGF_OK;
}

static int dyson_finish(hipStream_t s, int rc, int *dbad, int npts) {
  if (rc != CCGF_OK) {
    g_dyson_err = rc == CCGF_ENOMEM ? "scratch too small for one (k, w) point" : "kernel launch failed";
    return rc;
  }
  std::vector<int> hb(npts);
  hipMemcpyAsync(hb.data(), dbad, sizeof(int) * npts, hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) {
    g_dyson_err = std::string("cc_gf_dyson_cas: ") + hipGetErrorString(hipGetLastError());
    return CCGF_EDEVICE;
  }
  for (int b = 0; b < npts; ++b)
    if (hb[b]) {
      g_dyson_err = "a matrix to invert is singular at (k, w) point " + std::to_string(b);
      return CCGF_EINVAL;
    }
  return CCGF_OK;
}

extern "C" int cc_gf_dyson_cas(int nk, int nw, int N, int M, const double *Ggw, const double *Ggw_cas,
                               const double *Gcc, const double *V, double *Gout, double *Sfull_opt,
                               double *Scas_opt, void *hip_stream) {
  if (int rc = dyson_check(nk, nw, N, M, Ggw, Ggw_cas, Gcc, V, Gout)) return rc;
  if (nw == 0) return CCGF_OK;
  hipStream_t s = (hipStream_t)hip_stream;
  const int npts = nk * nw;
  const long long per = dyson_scratch_per_point(N, M);
  cplx *scratch = nullptr;
  int *dbad = nullptr;
  if (hipMalloc(&scratch, sizeof(cplx) * (size_t)per * npts) != hipSuccess ||
      hipMalloc(&dbad, sizeof(int) * npts) != hipSuccess) {
    (void)hipGetLastError();
    if (scratch) hipFree(scratch);
    g_dyson_err = "device allocation of the scratch failed";
    return CCGF_ENOMEM;
  }
  hipMemsetAsync(dbad, 0, sizeof(int) * npts, s);
  int rc = dyson_cas_run(s, nk, nw, N, M, (const cplx *)Ggw, (const cplx *)Ggw_cas, (const cplx *)Gcc,
                         (const cplx *)V, (cplx *)Gout, (cplx *)Sfull_opt, (cplx *)Scas_opt, scratch,
                         per * npts, dbad, 1);
  rc = dyson_finish(s, rc, dbad, npts);
  hipStreamSynchronize(s);
  hipFree(scratch);
  hipFree(dbad);
  return rc;
}

extern "C" const char *cc_gf_dyson_last_error(void) { return g_dyson_err.c_str(); }

// ------------------------------------------------------------------ without allocation
// Scratch of cc_gf_dyson_cas_noalloc: one fixed array per device (64 MiB), alive until
// the process ends.  The first 256 bytes hold the singular-matrix flag, the rest the
// matrices of one chunk of (k, w) points.  Host code reaches it only through the address
// hipGetSymbolAddress returns on each device.
#define DYSON_SCRATCH_ELEMS (1LL << 22)
#define DYSON_SCRATCH_HEAD 16
static __device__ __align__(256) cplx scratch[DYSON_SCRATCH_HEAD + DYSON_SCRATCH_ELEMS];

namespace {
__global__ void k_clear_flag(int *f) { *f = 0; }

std::mutex g_scratch_mu;
cplx *g_scratch_ptr[256] = {};  // per device ordinal
}  // namespace

// The device address of `scratch` on the current device (looked up once per device).
static int dyson_scratch(cplx **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 256) {
    (void)hipGetLastError();
    g_dyson_err = "no current HIP device";
    return CCGF_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      g_dyson_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return CCGF_EDEVICE;
    }
    g_scratch_ptr[dev] = (cplx *)p;
  }
  *out = g_scratch_ptr[dev];
  return CCGF_OK;
}

extern "C" int cc_gf_dyson_cas_noalloc(int nk, int nw, int N, int M, const double *Ggw, const double *Ggw_cas,
                                       const double *Gcc, const double *V, double *Gout, double *Sfull_opt,
                                       double *Scas_opt, void *hip_stream) {
  if (int rc = dyson_check(nk, nw, N, M, Ggw, Ggw_cas, Gcc, V, Gout)) return rc;
  if (dyson_scratch_per_point(N, M) > DYSON_SCRATCH_ELEMS) {
    g_dyson_err = "one (k, w) point needs more than the fixed scratch of cc_gf_dyson_cas_noalloc";
    return CCGF_EINVAL;
  }
  if (nw == 0) return CCGF_OK;
  cplx *base = nullptr;
  if (int rc = dyson_scratch(&base)) return rc;
  hipStream_t s = (hipStream_t)hip_stream;
  int *flag = (int *)base;
  hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, s, flag);
  int rc = dyson_cas_run(s, nk, nw, N, M, (const cplx *)Ggw, (const cplx *)Ggw_cas, (const cplx *)Gcc,
                         (const cplx *)V, (cplx *)Gout, (cplx *)Sfull_opt, (cplx *)Scas_opt,
                         base + DYSON_SCRATCH_HEAD, DYSON_SCRATCH_ELEMS, flag, 0);
  if (rc != CCGF_OK) {
    g_dyson_err = "kernel launch failed";
    return rc;
  }
  int hflag = 0;
  hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (hipStreamSynchronize(s) != hipSuccess) {
    g_dyson_err = std::string("cc_gf_dyson_cas_noalloc: ") + hipGetErrorString(hipGetLastError());
    return CCGF_EDEVICE;
  }
  if (hflag) {
    g_dyson_err = "a matrix to invert is singular";
    return CCGF_EINVAL;
  }
  return CCGF_OK;
}
