// The learned initial-guess network: a three-layer perceptron (two tanh hidden
// layers, linear output) trained by least squares with Adam, in FP32 on MFMA.
// Parameters are one flat vector W1, b1, W2, b2, W3, b3 (weights row-major
// [out][in]).  Forward:  a1 = tanh(X W1^T + b1), a2 = tanh(a1 W2^T + b2),
// Y = a2 W3^T + b3;  loss L = |Y - T|^2 / (2N);  backward by the chain rule.
#include "ccgf_internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

typedef float v4f __attribute__((ext_vector_type(4)));

namespace {

// C(m,n) = alpha sum_k A(m,k) B(k,n) + beta C(m,n) with strided operands,
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn], C row-major ldc.
// One wave per 16x16 output tile on the FP32 16x16x4 MFMA (lane l feeds
// A(l%16, k0 + l/16) and B(k0 + l/16, l%16); item v of lane l is C(4(l/16)+v, l%16)).
__global__ __launch_bounds__(256) void k_sgemm(int M, int N, int K, float alpha, const float *__restrict__ A,
                                               long long sam, long long sak, const float *__restrict__ B,
                                               long long sbk, long long sbn, float beta, float *__restrict__ C,
                                               int ldc) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tilesN = (N + 15) / 16;
  const int tile = blockIdx.x * 4 + wave;
  const int tm = tile / tilesN, tn = tile % tilesN;
  if (tm * 16 >= M) return;  // whole waves leave together
  const int r = lane & 15, kk = lane >> 4;
  const int am = tm * 16 + r, bn = tn * 16 + r;
  v4f acc = {0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += 4) {
    const int k = k0 + kk;
    float a = (am < M && k < K) ? A[am * sam + k * sak] : 0.0f;
    float b = (bn < N && k < K) ? B[k * sbk + bn * sbn] : 0.0f;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int m = tm * 16 + 4 * kk + v, n = tn * 16 + r;
    if (m < M && n < N) {
      float val = alpha * acc[v];
      if (beta != 0.0f) val += beta * C[(size_t)m * ldc + n];
      C[(size_t)m * ldc + n] = val;
    }
  }
}

// Y[n][j] = act(Y[n][j] + b[j]) (act = tanh when tanh_ != 0)
__global__ void k_bias_act(int N, int D, float *__restrict__ Y, const float *__restrict__ b, int tanh_) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)N * D) return;
  float z = Y[t] + b[t % D];
  Y[t] = tanh_ ? tanhf(z) : z;
}

// dY = (Y - T) / N and per-block partial sums of (Y - T)^2
__global__ void k_loss_grad(long long cnt, int N, const float *__restrict__ Y, const float *__restrict__ T,
                            float *__restrict__ dY, double *__restrict__ part) {
  __shared__ double sh[256];
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double e2 = 0;
  if (t < cnt) {
    float d = Y[t] - T[t];
    dY[t] = d / (float)N;
    e2 = (double)d * d;
  }
  sh[threadIdx.x] = e2;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// dZ = dA * (1 - A^2) (back through tanh), in place on dA
__global__ void k_tanh_back(long long cnt, float *__restrict__ dA, const float *__restrict__ A) {
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < cnt) dA[t] *= 1.0f - A[t] * A[t];
}

// db[j] = sum_n dZ[n][j]
__global__ void k_colsum(int N, int D, const float *__restrict__ dZ, float *__restrict__ db) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= D) return;
  float s = 0;
  for (int n = 0; n < N; ++n) s += dZ[(size_t)n * D + j];
  db[j] = s;
}

// Adam (Kingma & Ba, Algorithm 1) with bias correction; t counts from 1
__global__ void k_adam(long long cnt, float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m,
                       float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  float mi = b1 * m[i] + (1 - b1) * g[i];
  float vi = b2 * v[i] + (1 - b2) * g[i] * g[i];
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

void sgemm(hipStream_t s, int M, int N, int K, float alpha, const float *A, long long sam, long long sak,
           const float *B, long long sbk, long long sbn, float beta, float *C, int ldc) {
  const int tiles = ((M + 15) / 16) * ((N + 15) / 16);
  hipLaunchKernelGGL(k_sgemm, dim3((tiles + 3) / 4), dim3(256), 0, s, M, N, K, alpha, A, sam, sak, B, sbk, sbn, beta,
                     C, ldc);
}

unsigned blocks(long long cnt) { return (unsigned)((cnt + 255) / 256); }

}  // namespace

long long mlp_nparams(int din, int h, int dout) {
  return (long long)h * din + h + (long long)h * h + h + (long long)dout * h + dout;
}

bool mlp_alloc(MlpWork &w, int din, int h, int dout, int nmax) {
  auto al = [&](size_t n) -> float * {
    void *p = nullptr;
    if (hipMalloc(&p, sizeof(float) * (n < 4 ? 4 : n)) != hipSuccess) {
      (void)hipGetLastError();
      w.failed = true;
      return nullptr;
    }
    w.ptrs.push_back(p);
    return (float *)p;
  };
  w.din = din;
  w.h = h;
  w.dout = dout;
  w.nmax = nmax;
  const long long np = mlp_nparams(din, h, dout);
  w.grad = al(np);
  w.a1 = al((size_t)nmax * h);
  w.a2 = al((size_t)nmax * h);
  w.y = al((size_t)nmax * dout);
  w.dy = al((size_t)nmax * dout);
  w.d2 = al((size_t)nmax * h);
  w.d1 = al((size_t)nmax * h);
  void *p = nullptr;
  if (hipMalloc(&p, sizeof(double) * (size_t)(blocks((long long)nmax * dout) + 1)) != hipSuccess) {
    (void)hipGetLastError();
    w.failed = true;
  } else {
    w.ptrs.push_back(p);
    w.lpart = (double *)p;
  }
  return !w.failed;
}

void mlp_free(MlpWork &w) {
  for (void *p : w.ptrs)
    if (p) hipFree(p);
  w.ptrs.clear();
}

// Y = network(X) for N rows (into w.y); X, theta on the device
void mlp_forward(hipStream_t s, MlpWork &w, const float *theta, int N, const float *X) {
  const int din = w.din, h = w.h, dout = w.dout;
  const float *W1 = theta, *b1 = W1 + (size_t)h * din, *W2 = b1 + h, *b2 = W2 + (size_t)h * h, *W3 = b2 + h,
              *b3 = W3 + (size_t)dout * h;
  sgemm(s, N, h, din, 1.0f, X, din, 1, W1, 1, din, 0.0f, w.a1, h);
  hipLaunchKernelGGL(k_bias_act, dim3(blocks((long long)N * h)), dim3(256), 0, s, N, h, w.a1, b1, 1);
  sgemm(s, N, h, h, 1.0f, w.a1, h, 1, W2, 1, h, 0.0f, w.a2, h);
  hipLaunchKernelGGL(k_bias_act, dim3(blocks((long long)N * h)), dim3(256), 0, s, N, h, w.a2, b2, 1);
  sgemm(s, N, dout, h, 1.0f, w.a2, h, 1, W3, 1, h, 0.0f, w.y, dout);
  hipLaunchKernelGGL(k_bias_act, dim3(blocks((long long)N * dout)), dim3(256), 0, s, N, dout, w.y, b3, 0);
}

// forward + backward: gradient into w.grad; returns the number of loss partials in w.lpart
int mlp_backward(hipStream_t s, MlpWork &w, const float *theta, int N, const float *X, const float *T) {
  const int din = w.din, h = w.h, dout = w.dout;
  mlp_forward(s, w, theta, N, X);
  const float *W2 = theta + (size_t)h * din + h, *W3 = W2 + (size_t)h * h + h;
  float *gW1 = w.grad, *gb1 = gW1 + (size_t)h * din, *gW2 = gb1 + h, *gb2 = gW2 + (size_t)h * h, *gW3 = gb2 + h,
        *gb3 = gW3 + (size_t)dout * h;
  const long long cnt = (long long)N * dout;
  hipLaunchKernelGGL(k_loss_grad, dim3(blocks(cnt)), dim3(256), 0, s, cnt, N, w.y, T, w.dy, w.lpart);
  // output layer: gW3 = dY^T a2, gb3 = sum dY, d2 = dY W3
  sgemm(s, dout, h, N, 1.0f, w.dy, 1, dout, w.a2, h, 1, 0.0f, gW3, h);
  hipLaunchKernelGGL(k_colsum, dim3((dout + 255) / 256), dim3(256), 0, s, N, dout, w.dy, gb3);
  sgemm(s, N, h, dout, 1.0f, w.dy, dout, 1, W3, h, 1, 0.0f, w.d2, h);
  hipLaunchKernelGGL(k_tanh_back, dim3(blocks((long long)N * h)), dim3(256), 0, s, (long long)N * h, w.d2, w.a2);
  // second layer
  sgemm(s, h, h, N, 1.0f, w.d2, 1, h, w.a1, h, 1, 0.0f, gW2, h);
  hipLaunchKernelGGL(k_colsum, dim3((h + 255) / 256), dim3(256), 0, s, N, h, w.d2, gb2);
  sgemm(s, N, h, h, 1.0f, w.d2, h, 1, W2, h, 1, 0.0f, w.d1, h);
  hipLaunchKernelGGL(k_tanh_back, dim3(blocks((long long)N * h)), dim3(256), 0, s, (long long)N * h, w.d1, w.a1);
  // first layer
  sgemm(s, h, din, N, 1.0f, w.d1, 1, h, X, din, 1, 0.0f, gW1, din);
  hipLaunchKernelGGL(k_colsum, dim3((h + 255) / 256), dim3(256), 0, s, N, h, w.d1, gb1);
  return (int)blocks(cnt);
}

void mlp_adam(hipStream_t s, long long np, float *theta, const float *g, float *m, float *v, int t, float lr) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, (float)t), c2 = 1.0f - std::pow(b2, (float)t);
  hipLaunchKernelGGL(k_adam, dim3(blocks(np)), dim3(256), 0, s, np, theta, g, m, v, lr, b1, b2, 1e-8f, c1, c2);
}

// ------------------------------------------------------------------ C ABI (no context)
extern "C" int cc_gf_mlp_grad(int din, int hidden, int dout, const float *theta, int N, const float *X,
                              const float *T, float *grad, double *loss) {
  if (din < 1 || hidden < 1 || dout < 1 || N < 1 || din > 4096 || hidden > 4096 || dout > 4096)
    return CCGF_EINVAL;
  if (!theta || !X || !T || !grad) return CCGF_EINVAL;
  const long long np = mlp_nparams(din, hidden, dout);
  MlpWork w;
  float *dth = nullptr, *dX = nullptr, *dT = nullptr;
  int rc = CCGF_OK;
  if (!mlp_alloc(w, din, hidden, dout, N) || hipMalloc(&dth, sizeof(float) * np) != hipSuccess ||
      hipMalloc(&dX, sizeof(float) * (size_t)N * din) != hipSuccess ||
      hipMalloc(&dT, sizeof(float) * (size_t)N * dout) != hipSuccess) {
    (void)hipGetLastError();
    rc = CCGF_ENOMEM;
  }
  if (rc == CCGF_OK) {
    hipStream_t s = nullptr;
    hipMemcpy(dth, theta, sizeof(float) * np, hipMemcpyHostToDevice);
    hipMemcpy(dX, X, sizeof(float) * (size_t)N * din, hipMemcpyHostToDevice);
    hipMemcpy(dT, T, sizeof(float) * (size_t)N * dout, hipMemcpyHostToDevice);
    const int nb = mlp_backward(s, w, dth, N, dX, dT);
    std::vector<double> lp(nb);
    hipMemcpy(grad, w.grad, sizeof(float) * np, hipMemcpyDeviceToHost);
    hipMemcpy(lp.data(), w.lpart, sizeof(double) * nb, hipMemcpyDeviceToHost);
    if (hipDeviceSynchronize() != hipSuccess || hipGetLastError() != hipSuccess) rc = CCGF_EDEVICE;
    double L = 0;
    for (double x : lp) L += x;
    if (loss) *loss = 0.5 * L / N;
  }
  if (dth) hipFree(dth);
  if (dX) hipFree(dX);
  if (dT) hipFree(dT);
  mlp_free(w);
  return rc;
}

// ------------------------------------------------------------------ features and guesses
// Network input of orbital b of a model at frequency w, from the training
// solution jr ("previous solution"): w, its offset from w_jr in training steps,
// the orbital's Fock diagonal, its occupation, and the scaled reduced coordinates.
void learn_features(const LearnModel &M, int b, double w, int jr, float *f) {
  f[0] = (float)(w / M.wscale);
  f[1] = (float)((w - M.wtrain[jr]) / M.wstep);
  f[2] = (float)(M.fpp[b] / M.wscale);
  f[3] = M.occ[b] ? 1.0f : -1.0f;
  for (int i = 0; i < M.R; ++i) {
    cplx v = M.C[((size_t)b * M.ntrain + jr) * M.R + i];
    f[4 + i] = (float)(v.x * M.scale[b]);
    f[4 + M.R + i] = (float)(v.y * M.scale[b]);
  }
}

bool learn_guess(ccgf_ctx *c, const LearnModel &M, int nrhs, const int *rhs_orb, const int *orbs,
                 const double *rhs_omega, Guess &g, cplx **chat_dev) {
  *chat_dev = nullptr;
  g.qidx.assign(nrhs, -1);
  std::vector<int> rows, refs;
  std::vector<float> F;
  for (int r = 0; r < nrhs; ++r) {
    const int p = orbs[rhs_orb[r]];
    int bm = -1;
    for (int b = 0; b < M.norb; ++b)
      if (M.orbs[b] == p) bm = b;
    if (bm < 0) continue;
    int jr = 0;
    for (int j = 1; j < M.ntrain; ++j)
      if (std::fabs(M.wtrain[j] - rhs_omega[r]) < std::fabs(M.wtrain[jr] - rhs_omega[r])) jr = j;
    F.resize((rows.size() + 1) * M.din);
    learn_features(M, bm, rhs_omega[r], jr, &F[rows.size() * M.din]);
    g.qidx[r] = bm;
    rows.push_back(r);
    refs.push_back(jr);
  }
  if (rows.empty()) return false;
  const int N = (int)rows.size();
  hipStream_t s = c->stream;
  MlpWork w;
  float *dF = nullptr;
  cplx *dch = nullptr;
  bool ok = mlp_alloc(w, M.din, M.hidden, M.dout, N) && hipMalloc(&dF, sizeof(float) * F.size()) == hipSuccess &&
            hipMalloc(&dch, sizeof(cplx) * (size_t)nrhs * M.R) == hipSuccess;
  std::vector<float> Y((size_t)N * M.dout, 0.0f);
  if (ok && M.mode == CCGF_GUESS_NETWORK) {
    hipMemcpyAsync(dF, F.data(), sizeof(float) * F.size(), hipMemcpyHostToDevice, s);
    mlp_forward(s, w, M.theta, N, dF);
    hipMemcpyAsync(Y.data(), w.y, sizeof(float) * Y.size(), hipMemcpyDeviceToHost, s);
    ok = hipStreamSynchronize(s) == hipSuccess;
  }
  std::vector<cplx> ch((size_t)nrhs * M.R, mkc(0, 0));
  if (ok) {
    // c_hat = c_ref + network output (the output alone is the move from the reference)
    for (int k = 0; k < N; ++k) {
      const int r = rows[k], bm = g.qidx[r], jr = refs[k];
      for (int i = 0; i < M.R; ++i) {
        cplx c0 = M.C[((size_t)bm * M.ntrain + jr) * M.R + i];
        ch[(size_t)r * M.R + i] = mkc(c0.x + Y[(size_t)k * M.dout + i] / M.scale[bm],
                                      c0.y + Y[(size_t)k * M.dout + M.R + i] / M.scale[bm]);
      }
    }
    hipMemcpyAsync(dch, ch.data(), sizeof(cplx) * ch.size(), hipMemcpyHostToDevice, s);
    ok = hipStreamSynchronize(s) == hipSuccess;
  }
  if (dF) hipFree(dF);
  mlp_free(w);
  if (!ok) {
    (void)hipGetLastError();
    if (dch) hipFree(dch);
    g.qidx.assign(nrhs, -1);
    return false;  // no guess: the solves start from zero
  }
  g.Q = M.Q;
  g.chat = dch;
  g.R = M.R;
  g.accept = M.accept;
  *chat_dev = dch;
  return true;
}

// ------------------------------------------------------------------ training
int mlp_train(ccgf_ctx *c, int din, int hidden, int dout, long long P, const std::vector<float> &F,
              const std::vector<float> &T, int epochs, int batch, double lr, unsigned long long seed, bool zero_out,
              float **theta, double *L0, double *L1) {
  *theta = nullptr;
  hipStream_t s = c->stream;
  // parameters: uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and zero biases; with zero_out the
  // output layer starts at zero (the untrained network outputs 0)
  const long long np = mlp_nparams(din, hidden, dout);
  std::vector<float> th(np, 0.0f);
  std::mt19937_64 rng(seed);
  {
    long long o = 0;
    const int fin[3] = {din, hidden, hidden}, fout[3] = {hidden, hidden, dout};
    for (int l = 0; l < (zero_out ? 2 : 3); ++l) {
      std::uniform_real_distribution<float> U(-1.0f / std::sqrt((float)fin[l]), 1.0f / std::sqrt((float)fin[l]));
      for (long long q = 0; q < (long long)fout[l] * fin[l]; ++q) th[o + q] = U(rng);
      o += (long long)fout[l] * fin[l] + fout[l];
    }
  }
  const int bs = (int)std::min<long long>(P, batch);
  MlpWork w;
  float *dth = nullptr, *dF = nullptr, *dT = nullptr, *mm = nullptr, *vv = nullptr;
  bool ok = mlp_alloc(w, din, hidden, dout, (int)P) && hipMalloc(&dth, sizeof(float) * np) == hipSuccess &&
            hipMalloc(&dF, sizeof(float) * F.size()) == hipSuccess &&
            hipMalloc(&dT, sizeof(float) * T.size()) == hipSuccess && hipMalloc(&mm, sizeof(float) * np) == hipSuccess &&
            hipMalloc(&vv, sizeof(float) * np) == hipSuccess;
  auto cleanup = [&](bool keep_theta) {
    mlp_free(w);
    if (dF) hipFree(dF);
    if (dT) hipFree(dT);
    if (mm) hipFree(mm);
    if (vv) hipFree(vv);
    if (!keep_theta && dth) hipFree(dth);
  };
  if (!ok) {
    (void)hipGetLastError();
    cleanup(false);
    return set_err(c, CCGF_ENOMEM, "no device memory for the network");
  }
  hipMemcpyAsync(dth, th.data(), sizeof(float) * np, hipMemcpyHostToDevice, s);
  hipMemsetAsync(mm, 0, sizeof(float) * np, s);
  hipMemsetAsync(vv, 0, sizeof(float) * np, s);
  auto full_loss = [&](double &L) -> int {
    hipMemcpyAsync(dF, F.data(), sizeof(float) * F.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dT, T.data(), sizeof(float) * T.size(), hipMemcpyHostToDevice, s);
    const int nb = mlp_backward(s, w, dth, (int)P, dF, dT);
    std::vector<double> lp(nb);
    hipMemcpyAsync(lp.data(), w.lpart, sizeof(double) * nb, hipMemcpyDeviceToHost, s);
    int rc = hip_check(c, hipStreamSynchronize(s), "network loss");
    L = 0;
    for (double x : lp) L += x;
    L *= 0.5 / (double)P;
    return rc;
  };
  if (int rc = full_loss(*L0)) {
    cleanup(false);
    return rc;
  }
  std::vector<long long> perm(P);
  std::vector<float> Fs(F.size()), Ts(T.size());
  int t = 0;
  for (int e = 0; e < epochs; ++e) {
    for (long long q = 0; q < P; ++q) perm[q] = q;
    std::shuffle(perm.begin(), perm.end(), rng);
    for (long long q = 0; q < P; ++q) {
      std::copy(&F[(size_t)perm[q] * din], &F[(size_t)perm[q] * din] + din, &Fs[(size_t)q * din]);
      std::copy(&T[(size_t)perm[q] * dout], &T[(size_t)perm[q] * dout] + dout, &Ts[(size_t)q * dout]);
    }
    hipMemcpyAsync(dF, Fs.data(), sizeof(float) * Fs.size(), hipMemcpyHostToDevice, s);
    hipMemcpyAsync(dT, Ts.data(), sizeof(float) * Ts.size(), hipMemcpyHostToDevice, s);
    for (long long q0 = 0; q0 + bs <= P; q0 += bs) {
      mlp_backward(s, w, dth, bs, dF + (size_t)q0 * din, dT + (size_t)q0 * dout);
      mlp_adam(s, np, dth, w.grad, mm, vv, ++t, (float)lr);
    }
    if (int rc = hip_check(c, hipStreamSynchronize(s), "network training")) {  // host arrays reused next epoch
      cleanup(false);
      return rc;
    }
  }
  if (int rc = full_loss(*L1)) {
    cleanup(false);
    return rc;
  }
  cleanup(true);
  *theta = dth;
  return CCGF_OK;
}

// ------------------------------------------------------------------ preconditioner network
const double kPrecondCand[CCGF_PRECOND_CANDIDATES] = {0.25, 0.5, 1.0, 1.5, 2.5};

void precond_features(const LearnModel &M, int b, double w, float *f) {
  f[0] = (float)(w / M.wscale);
  f[1] = (float)(M.fpp[b] / M.wscale);
  f[2] = M.occ[b] ? 1.0f : -1.0f;
  f[3] = (float)((w - M.fpp[b]) / M.wscale);
}

bool learn_precond(ccgf_ctx *c, const LearnModel &M, int nrhs, const int *rhs_orb, const int *orbs,
                   const double *rhs_omega, std::vector<double> &peta) {
  if (!M.theta_p || nrhs <= 0) return false;
  std::vector<int> rows;
  std::vector<float> F;
  for (int r = 0; r < nrhs; ++r) {
    const int p = orbs[rhs_orb[r]];
    int bm = -1;
    for (int b = 0; b < M.norb; ++b)
      if (M.orbs[b] == p) bm = b;
    if (bm < 0) continue;
    F.resize((rows.size() + 1) * M.pdin);
    precond_features(M, bm, rhs_omega[r], &F[rows.size() * M.pdin]);
    rows.push_back(r);
  }
  if (rows.empty()) return false;
  const int N = (int)rows.size();
  hipStream_t s = c->stream;
  MlpWork w;
  float *dF = nullptr;
  bool ok = mlp_alloc(w, M.pdin, M.hidden, M.pdout, N) && hipMalloc(&dF, sizeof(float) * F.size()) == hipSuccess;
  std::vector<float> Y((size_t)N * M.pdout, 0.0f);
  if (ok) {
    hipMemcpyAsync(dF, F.data(), sizeof(float) * F.size(), hipMemcpyHostToDevice, s);
    mlp_forward(s, w, M.theta_p, N, dF);
    hipMemcpyAsync(Y.data(), w.y, sizeof(float) * Y.size(), hipMemcpyDeviceToHost, s);
    ok = hipStreamSynchronize(s) == hipSuccess;
  }
  if (dF) hipFree(dF);
  mlp_free(w);
  if (!ok) {
    (void)hipGetLastError();
    return false;
  }
  // -1: the context's own damping (orbitals the network was not trained on)
  peta.assign(nrhs, -1.0);
  for (int k = 0; k < N; ++k) {
    int best = 0;
    for (int q = 1; q < M.pdout; ++q)
      if (Y[(size_t)k * M.pdout + q] < Y[(size_t)k * M.pdout + best]) best = q;
    peta[rows[k]] = kPrecondCand[best] * M.pbase;
  }
  return true;
}
