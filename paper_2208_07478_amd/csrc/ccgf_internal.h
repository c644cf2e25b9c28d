// Internal declarations of the MI355X CCGF library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ccgf.h"

typedef double2 cplx;  // {x = re, y = im}

__host__ __device__ inline cplx mkc(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline cplx cadd(cplx a, cplx b) { return mkc(a.x + b.x, a.y + b.y); }
__host__ __device__ inline cplx csub(cplx a, cplx b) { return mkc(a.x - b.x, a.y - b.y); }
__host__ __device__ inline cplx cmul(cplx a, cplx b) {
  return mkc(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline cplx cconj(cplx a) { return mkc(a.x, -a.y); }
__host__ __device__ inline cplx cscale(cplx a, double s) { return mkc(a.x * s, a.y * s); }
// acc += a * b
__host__ __device__ inline void cfma(cplx &acc, cplx a, cplx b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
}
// acc += conj(a) * b
__host__ __device__ inline void cfmac(cplx &acc, cplx a, cplx b) {
  acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
}

// Momentum arithmetic on the Gamma-centred mesh, as a table: kc3[(k1*nk+k2)*nk+k3] = k1+k2-k3.
struct KTab {
  int nk;
  const int *kc3;  // device
  __device__ inline int c3(int k1, int k2, int k3) const { return kc3[(k1 * nk + k2) * nk + k3]; }
};

// Dense 4-index momentum-blocked tensor [k1][k2][k3][n1][n2][n3][n4] (k4 implied).
struct T4 {
  cplx *p;
  int nk, n1, n2, n3, n4;
  __host__ __device__ inline size_t blk(int k1, int k2, int k3) const {
    return (((size_t)k1 * nk + k2) * nk + k3) * ((size_t)n1 * n2 * n3 * n4);
  }
  __host__ __device__ inline size_t at(int k1, int k2, int k3, int a, int b, int c, int d) const {
    return blk(k1, k2, k3) + (((size_t)a * n2 + b) * n3 + c) * n4 + d;
  }
  __device__ inline cplx operator()(int k1, int k2, int k3, int a, int b, int c, int d) const {
    return p[at(k1, k2, k3, a, b, c, d)];
  }
  size_t size() const { return (size_t)nk * nk * nk * n1 * n2 * n3 * n4; }
};

// k-diagonal 2-index tensor [k][n1][n2].
struct T2d {
  cplx *p;
  int n1, n2;
  __device__ inline cplx operator()(int k, int a, int b) const {
    return p[((size_t)k * n1 + a) * n2 + b];
  }
};

// One launch of the segmented complex GEMM: for every task t and every tile,
//   C_t[m][n] = alpha * sum_{s in segs(t)} sum_k A_s[m][k] B_s[k][n]  (+ C_t if accumulate)
// Index maps are two-level: for an index x with split L, offset = (x / L) * s0 + (x % L) * s1.
struct IdxMap {
  int L;
  long long s0, s1;
};
struct GemmTask {
  long long c_off;
  int seg_begin, nseg;
};
struct GemmSeg {
  long long a_off, b_off;
};
struct GemmShape {
  int M, N, K;
  IdxMap am, ak;  // A[m][k]
  IdxMap bk, bn;  // B[k][n]
  IdxMap cm, cn;  // C[m][n]
  double alpha_re, alpha_im;
  int accumulate;
};

struct GemmPlan {
  GemmShape shape;
  int ntask;
  GemmTask *d_tasks;
  GemmSeg *d_segs;
  std::vector<GemmTask> tasks;
  std::vector<GemmSeg> segs;
};

struct SigmaPlan {  // per (part, K, batch layout)
  int part, K, nvec;
  long long n;
  GemmPlan g_big;   // EA: W_vvvv term; IP: W_oooo term (writes sigma2)
  GemmPlan g_ovvo;  // W_ovvo term into the scratch vector
  GemmPlan g_r1;    // EA: W_abei r^e; IP: -W_maij r_m  (accumulates into sigma2)
  GemmPlan g_red1;  // split-K partial sums of the 1p / 1h rows of sigma (EA W_alcd, IP W_mnie)
  GemmPlan g_red2;  // split-K partial sums of the three-body intermediate (<kl||cd> r / <mn||ef> r)
  bool ready = false;
};

struct ccgf_ctx {
  int m[3];
  int nk, no, nv, nmo, naux;
  hipStream_t stream = nullptr;
  ccgf_options opt;
  std::string err;
  std::vector<int> kc3_h;
  int *kc3 = nullptr;
  // inputs
  cplx *t1 = nullptr, *t2 = nullptr, *fac = nullptr, *foo = nullptr, *fvv = nullptr;
  // Hbar blocks (complex double)
  cplx *Foo = nullptr, *Fvv = nullptr, *Fov = nullptr;
  cplx *Woooo = nullptr, *Wooov = nullptr, *Wovoo = nullptr, *Wovvo = nullptr;
  cplx *Wvovv = nullptr, *Wvvvo = nullptr, *Wvvvv = nullptr, *Voovv = nullptr;
  cplx *WvoP = nullptr;   // W_ovvo permuted to [kx][ki][km](x, i, m, e)
  cplx *WooP = nullptr;   // W_oooo permuted to [ki][kj][km](i, j, m, n)
  // complex-float copies of the GEMM operands for the mixed-precision products
  float2 *Wvvvv32 = nullptr, *WvoP32 = nullptr, *WooP32 = nullptr;
  std::vector<void *> allocs;
  // sigma workspace
  cplx *sig_tmp = nullptr;  // scratch vector batch for the W_ovvo term
  size_t sig_tmp_elems = 0;
  cplx *sig_r1aux = nullptr;  // per-RHS 3-body contraction (nvec x max(no, nv))
  size_t sig_r1aux_elems = 0;
  cplx *sig_part = nullptr;  // split-range partial sums of the 1h / 1p rows
  size_t sig_part_elems = 0;
  std::vector<SigmaPlan> plans;
  // event timing of the sigma products (options.timing)
  // sigma timing (options.timing): events of recent products, read once they have completed
  struct TimedSigma {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};  // sigma start, sigma end, big GEMM start, end
    int big = 0;           // count the big GEMM (EA products)
    double flops = 0;      // its algorithmic flops
    bool pending = false;
  };
  std::vector<TimedSigma> tring;
  int tnext = 0;
  double t_big_ms = 0, t_big_flops = 0, t_sigma_ms = 0;
  long long t_big_launches = 0, t_sigma_launches = 0;
};

// helpers implemented in api.cpp
int set_err(ccgf_ctx *c, int code, const std::string &msg);
int hip_check(ccgf_ctx *c, hipError_t e, const char *what);
void *dev_alloc(ccgf_ctx *c, size_t bytes);

// init.hip
int build_hbar(ccgf_ctx *c);
int build_vectors(ccgf_ctx *c, int part, int K, int p, cplx *b, cplx *e);
long long vec_len(const ccgf_ctx *c, int part);

// sigma.hip
int sigma_apply(ccgf_ctx *c, int part, int K, int nvec, const cplx *x, cplx *y, int prec = 0);
// Accumulate the timings of the recorded sigma products (waits for any still running).
void timing_harvest(ccgf_ctx *c);
void timing_release(ccgf_ctx *c);
void gemm_launch(int tag, const GemmPlan &plan, const void *A, const cplx *B, cplx *C, hipStream_t s, int prec);
void plan_upload(ccgf_ctx *c, GemmPlan &p);

// gmres.hip
int solve_batched(ccgf_ctx *c, int part, int K, int nrhs, const int *rhs_orb_slot, const double *rhs_omega,
                  double eta, const cplx *Bvecs, const cplx *Evecs, cplx *Gout, ccgf_stats *st,
                  cplx *Xout = nullptr);
int mor_part(ccgf_ctx *c, int part, int K, int norb, const int *orbs, int nexp, const double *wexp, int nw,
             const double *omega, double eta, cplx *Gout, ccgf_stats *st);
