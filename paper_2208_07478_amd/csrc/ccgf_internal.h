// Internal declarations of the MI355X CCGF library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <map>
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

// One complex element split for the BF16 products: x = hi + lo to about 2^-16 relative,
// hi = bf16(x), lo = bf16(x - hi), for the real and the imaginary part (8 bytes, the size
// of a complex float, so that the split operands take the complex float copies' place)
struct B3E {
  __bf16 rh, rl, ih, il;
};
static_assert(sizeof(B3E) == 8, "split element layout");
__device__ inline void split_bf(double x, __bf16 &h, __bf16 &l) {
  h = (__bf16)(float)x;
  l = (__bf16)(float)(x - (double)(float)h);
}
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

// Read access to the stored W_abcd blocks (see ccgf_ctx::wblk_h): any block (ka, kb, kc)
// is +-(a stored block) with the pair indices swapped where the momenta were.
struct WPacked {
  const cplx *p;
  const int *tab;  // device wblk
  KTab kt;
  int nv;
  __device__ inline cplx operator()(int ka, int kb, int kc, int a, int b, int c, int d) const {
    double sg = 1.0;
    if (ka > kb) {
      int t = ka; ka = kb; kb = t;
      t = a; a = b; b = t;
      sg = -sg;
    }
    const int kd = kt.c3(ka, kb, kc);
    if (kc > kd) {
      kc = kd;
      int t = c; c = d; d = t;
      sg = -sg;
    }
    const size_t q = (size_t)tab[(ka * kt.nk + kb) * kt.nk + kc];
    const size_t nv2 = (size_t)nv * nv;
    return cscale(p[q * nv2 * nv2 + ((size_t)a * nv + b) * nv2 + (size_t)c * nv + d], sg);
  }
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
  double w = 1.0;  // weight of this segment's products (exact: 1 or 1/2)
};
struct GemmShape {
  int M, N, K;
  IdxMap am, ak;  // A[m][k]
  IdxMap bk, bn;  // B[k][n]
  IdxMap cm, cn;  // C[m][n]
  double alpha_re, alpha_im;
  int accumulate;
  // optional index tables (device): row m stands for mtab[m] in am and cm, k for ktab[k]
  // in ak and bk (the strict upper triangle of an antisymmetric index pair)
  const int *mtab = nullptr, *ktab = nullptr;
};

struct GemmPlan {
  GemmShape shape;
  int m_ext = 0, k_ext = 0;     // index ranges reached through mtab / ktab (0: M / K)
  int tn[3] = {0, 0, 0};        // N tile width picked by the autotuner per precision (0: not yet)
  int trials[3] = {0, 0, 0};    // timed trial launches so far
  float tms[3][3] = {};         // their times (64-wide, 32-wide, 128-wide)
  bool pairs = false;           // k pairs (2k, 2k + 1) adjacent and 16-byte aligned in A and B
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
  GemmPlan g_bigt;  // EA: W_vvvv term of blocks ka = kb, segments kc = kd (both pairs a<b, c<d)
  GemmPlan g_bigd;  // EA: W_vvvv term of blocks ka = kb, segments kc < kd (pairs a<b)
  int *d_tri = nullptr;  // pair table p -> a * nv + b, a < b
  GemmPlan g_ovvo;  // W_ovvo term into the scratch vector
  GemmPlan g_r1;    // EA: W_abei r^e; IP: -W_maij r_m  (accumulates into sigma2)
  GemmPlan g_red1;  // split-K partial sums of the 1p / 1h rows of sigma (EA W_alcd, IP W_mnie)
  GemmPlan g_red2;  // split-K partial sums of the three-body intermediate (<kl||cd> r / <mn||ef> r)
  // EA: output blocks of the W_abcd product left to antisymmetry, sigma[ki][ka](i,a,b) =
  // -sigma[ki][kb](i,b,a): offsets of the destination and source blocks in a vector (equal
  // offsets: the rows a >= b of a block ka = kb)
  int nfill = 0;
  long long *d_fill = nullptr;  // [2][nfill]
  std::vector<long long> fill_h;  // host copy, checked against the vector size
  struct Captured {
    const void *x, *y;
    int prec;
    hipGraphExec_t exec;
  };
  std::vector<Captured> graphs;  // captured launch sequences, most recent last
  bool ready = false;
};

// Device buffers of the learned-guess network for up to nmax rows.
struct MlpWork {
  int din = 0, h = 0, dout = 0, nmax = 0;
  float *grad = nullptr, *a1 = nullptr, *a2 = nullptr, *y = nullptr, *dy = nullptr, *d1 = nullptr, *d2 = nullptr;
  double *lpart = nullptr;
  std::vector<void *> ptrs;
  bool failed = false;
};
long long mlp_nparams(int din, int h, int dout);
bool mlp_alloc(MlpWork &w, int din, int h, int dout, int nmax);
void mlp_free(MlpWork &w);
void mlp_forward(hipStream_t s, MlpWork &w, const float *theta, int N, const float *X);
int mlp_backward(hipStream_t s, MlpWork &w, const float *theta, int N, const float *X, const float *T);
void mlp_adam(hipStream_t s, long long np, float *theta, const float *g, float *m, float *v, int t, float lr);

// A trained initial-guess network for one (part, K): the per-orbital reduced
// basis of the training solutions, their reduced coordinates (the network's
// "previous solution" inputs) and the FP32 parameters.
struct LearnModel {
  int part = 0, K = 0, norb = 0, ntrain = 0, R = 0, din = 0, dout = 0, hidden = 0;
  int mode = 0;                 // CCGF_GUESS_*
  double accept = 0.1;          // residual ratio below which a guess is used
  std::vector<int> orbs;        // orbital ids
  std::vector<int> occ;         // 1 for occupied orbitals
  std::vector<double> fpp;      // diagonal Fock element of each orbital at K (real part)
  std::vector<double> wtrain;   // training frequencies
  std::vector<double> scale;    // per orbital: 1 / largest |c|
  std::vector<cplx> C;          // [norb][ntrain][R] reduced coordinates of the training solutions
  double wscale = 1, wstep = 1;
  cplx *Q = nullptr;            // device [norb][R][n] orthonormal basis (zero columns allowed)
  float *theta = nullptr;       // device parameters
  // preconditioner network: features -> log10 residual after the probe steps per candidate damping
  int pdin = 0, pdout = 0;
  double pbase = 0;             // damping unit: max(eta, precond_eta) at training
  float *theta_p = nullptr;     // device parameters (null: none trained)
};
// Features of the preconditioner network for orbital b at frequency w.
void precond_features(const LearnModel &M, int b, double w, float *f);
extern const double kPrecondCand[CCGF_PRECOND_CANDIDATES];
// Per-right-hand-side damping chosen by the preconditioner network (false: none).
bool learn_precond(ccgf_ctx *c, const LearnModel &M, int nrhs, const int *rhs_orb, const int *orbs,
                   const double *rhs_omega, std::vector<double> &peta);
// Train a three-layer perceptron on (F [P][din], T [P][dout]) with Adam; *theta (device) receives
// the parameters (allocated here); L0 / L1 the loss before and after.
int mlp_train(ccgf_ctx *c, int din, int hidden, int dout, long long P, const std::vector<float> &F,
              const std::vector<float> &T, int epochs, int batch, double lr, unsigned long long seed, bool zero_out,
              float **theta, double *L0, double *L1);
// Initial guesses for solve_batched: x0 of right-hand side r = Q[qidx[r]] chat[r]
struct Guess {
  const cplx *Q = nullptr;      // [nq][R][n]
  const cplx *chat = nullptr;   // device [nrhs][R]
  std::vector<int> qidx;        // per right-hand side, -1 for none
  int R = 0;
  double accept = 1.0;          // keep x0 only if ||b - A x0|| < accept ||b||
  long long qs_i = 0, qs_q = 0; // strides of Q between columns and between q (0: n and R n)
};
void learn_features(const LearnModel &M, int b, double w, int jr, float *f);

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
  cplx *l1 = nullptr, *l2 = nullptr;  // Lambda amplitudes when given (NULL: Lambda = T^dagger)
  // Hbar blocks (complex double)
  cplx *Foo = nullptr, *Fvv = nullptr, *Fov = nullptr;
  // W_abcd is antisymmetric under (a,ka)<->(b,kb) and (c,kc)<->(d,kd): only the blocks
  // (ka, kb, kc) with ka <= kb and kc <= kd = ka + kb - kc are stored, each whole
  // (nv^4 elements), in the order of their flat triple; wblk_h[(ka*nk+kb)*nk+kc] is the
  // stored block's ordinal, -1 for the blocks that antisymmetry gives
  std::vector<int> wblk_h;
  int *wblk = nullptr;  // device copy of wblk_h
  long long nwblk = 0;
  cplx *Woooo = nullptr, *Wooov = nullptr, *Wovoo = nullptr, *Wovvo = nullptr;
  cplx *Wvovv = nullptr, *Wvvvo = nullptr, *Wvvvv = nullptr, *Voovv = nullptr;
  cplx *eri_dense = nullptr;  // dense <pq|rs> blocks [k1][k2][k3][p][q][r][s] when given instead of the factor
  cplx *WvoP = nullptr;   // W_ovvo permuted to [kx][ki][km](x, i, m, e)
  cplx *WvoPea = nullptr; // the same with F_vv added on the blocks km = ki, m = i (EA operand)
  cplx *WooP = nullptr;   // W_oooo permuted to [ki][kj][km](i, j, m, n)
  // complex-float copies of the GEMM operands for the mixed-precision products (B3E split
  // copies, the same size, for the BF16-split form)
  float2 *Wvvvv32 = nullptr, *WvoP32 = nullptr, *WooP32 = nullptr, *WvoPea32 = nullptr;
  std::vector<void *> allocs;
  // sigma workspace
  cplx *sig_tmp = nullptr;  // scratch vector batch for the W_ovvo term
  size_t sig_tmp_elems = 0;
  cplx *sig_r1aux = nullptr;  // per-RHS 3-body contraction (nvec x max(no, nv))
  size_t sig_r1aux_elems = 0;
  cplx *e_overlap = nullptr;  // [max(no, nv)] scratch of the e vectors (t2 overlap term)
  float2 *sig_x32 = nullptr;  // complex float (or B3E split) copy of the vectors (reduced-precision GEMMs)
  size_t sig_x32_elems = 0;
  cplx *sig_part = nullptr;  // split-range partial sums of the 1h / 1p rows
  size_t sig_part_elems = 0;
  std::vector<SigmaPlan> plans;
  std::vector<LearnModel> models;  // trained initial-guess networks
  // GEMM tile autotuning: chosen N tile width per GEMM shape, and events for the trials
  std::map<std::string, int> tuned;
  hipEvent_t tev[2] = {nullptr, nullptr};
  hipStream_t cap_stream = nullptr;  // private stream on which sigma launch sequences are captured
  // second stream of a sigma product: the terms that do not write the W_abcd / W_mnij output
  // run there beside that product (fork and join by events; default priority)
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // tables of the grouped launches over several systems (sigma_group)
  void *grp_buf = nullptr;
  size_t grp_bytes = 0;
  std::string tune_path;
  int learn_on = 3;                 // use them in cc_gf_solve (CCGF_LEARN_* mask)
  // event timing of the sigma products (options.timing)
  // sigma timing (options.timing): events of recent products, read once they have completed
  struct TimedSigma {
    hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};  // sigma start, sigma end, big GEMM start, end
    int big = 0;           // count the big GEMM (EA products)
    double flops = 0;      // its algorithmic flops
    double bytes = 0;      // and HBM bytes
    bool pending = false;
  };
  std::vector<TimedSigma> tring;
  int tnext = 0;
  double t_big_ms = 0, t_big_flops = 0, t_big_bytes = 0, t_sigma_ms = 0;
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
// sigma products of several systems, one launch per GEMM term over all of them (ctxs[0]'s stream)
int sigma_group(int nsys, ccgf_ctx *const *ctxs, const int *parts, const int *Ks, const int *nvecs,
                const cplx *const *xs, cplx *const *ys);
// Accumulate the timings of the recorded sigma products (waits for any still running).
void timing_harvest(ccgf_ctx *c);
void timing_release(ccgf_ctx *c);
// Read / write the autotuner's choices (one "key tn" line per GEMM shape).
void tune_load(ccgf_ctx *c);
void tune_save(const ccgf_ctx *c);
// B: complex double vectors for prec 0, their complex float copy for prec 1 and 2
void gemm_launch(int tag, const GemmPlan &plan, const void *A, const void *B, cplx *C, hipStream_t s, int prec,
                 int tn);
void plan_upload(ccgf_ctx *c, GemmPlan &p);

// gmres.hip
// Shared Krylov seed of the solves of one (part, K): Arnoldi of sigma from every orbital's b,
// then the GMRES minimiser of each right-hand side's own shift over it (Guess with Q = the
// bases, owned by *Q; chat owned by *chat).  On CCGF_ENOMEM nothing is seeded and both stay NULL.
int seed_krylov(ccgf_ctx *c, int part, int K, int norb, const cplx *Bvecs, int nrhs, const int *rhs_orb,
                const double *rhs_omega, double eta, Guess &g, cplx **Q, cplx **chat, ccgf_stats *st);
int solve_batched(ccgf_ctx *c, int part, int K, int nrhs, const int *rhs_orb_slot, const double *rhs_omega,
                  double eta, const cplx *Bvecs, const cplx *Evecs, cplx *Gout, ccgf_stats *st,
                  cplx *Xout = nullptr, const Guess *guess = nullptr, cplx *Gcols = nullptr, int ncols = 0,
                  const double *rhs_peta = nullptr, double *rhs_res = nullptr);
int learn_part(ccgf_ctx *c, int part, int K, int norb, const int *orbs, int ntrain, const double *wtrain, double eta,
               const ccgf_learn_options &lo, ccgf_learn_stats *ls);
// Device reduced coordinates (chat, [nrhs][R]) of the network's guesses for the listed
// right-hand sides (call orbital index rhs_orb into orbs); fills g.qidx; returns false
// when no guess applies.
bool learn_guess(ccgf_ctx *c, const LearnModel &M, int nrhs, const int *rhs_orb, const int *orbs,
                 const double *rhs_omega, Guess &g, cplx **chat_dev);
int mor_part(ccgf_ctx *c, int part, int K, int norb, const int *orbs, int nexp, const double *wexp, int nw,
             const double *omega, double eta, cplx *Gout, ccgf_stats *st);
