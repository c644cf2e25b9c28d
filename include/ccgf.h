/*
 * ccgf.h -- C ABI of the MI355X periodic coupled-cluster Green's function library.
 *
 * The library computes the diagonal k-point CCGF (Eq. 9 of Laughon, Yu & Zhu,
 * "Periodic Coupled-Cluster Green's Function for Photoemission Spectra of
 * Realistic Solids"):
 *
 *   G_pp(K, w) = G+_pp + G-_pp,
 *   G-_pp = e-_p . [(w + (Hbar - E) - i eta)^-1 b-_p]          (IP, Eq. 6b/7b)
 *   G+_pp = e+_p . [(w - (Hbar - E) + i eta)^-1 b+_p]          (EA, Eq. 6a/7a)
 *
 * with b-_p = abar_p|Phi>, b+_p = abar+_p|Phi>, e-_p = <Phi|(1+Lambda) abar+_p,
 * e+_p = <Phi|(1+Lambda) abar_p restricted to the EOM-CCSD spaces of Eq. 8
 * (1h + 2h1p for IP, 1p + 2p1h for EA), Lambda = T^dagger (the approximation
 * stated after Eq. 10) unless the caller gives Lambda amplitudes, and Hbar - E
 * the EOM-CCSD matrix, i.e. the connected
 * commutator <mu|[Hbar, R_nu]|Phi>.  The products are bilinear (e is not
 * conjugated).  Every shifted system is solved by a batched, diagonally
 * right-preconditioned restarted GMRES on the GPU whose matrix-vector product
 * is the k-blocked EOM-IP/EA-CCSD sigma product; its cost is the one quoted in
 * the paper's scaling paragraph (EA O(Nk^3 No Nv^4), IP O(Nk^3 No^3 Nv^2) per
 * k-point, frequency and orbital).
 *
 * Conventions (all functions):
 *  - Spin orbitals, occupied first: p in [0, nocc) occupied, [nocc, nmo) virtual.
 *  - Complex numbers are interleaved {re, im} doubles.
 *  - k-points: Gamma-centred integer mesh kmesh = (m1, m2, m3); point n = (n1,n2,n3)
 *    has flat index n1*m2*m3 + n2*m3 + n3 and momentum arithmetic is modulo the mesh.
 *  - Two-electron integrals are given by a momentum-blocked factor A with
 *    <p k1, q k2 | r k3, s k4> = sum_L A[k1][k3][L][p][r] * A[k2][k4][L][q][s]
 *    for k4 = k1 + k2 - k3 (zero otherwise) and A[k3][k1][L][r][p] = conj(A[k1][k3][L][p][r]).
 *  - Amplitudes: t1[k][i][a] (k_i = k_a = k); t2[ki][kj][ka][i][j][a][b] with
 *    kb = ki + kj - ka, antisymmetric under (i,ki)<->(j,kj) and (a,ka)<->(b,kb).
 *  - EOM vectors of total momentum K use full antisymmetric storage:
 *      IP: [r1[i] (k_i = K), r2[ki][kj][i][j][a] (ka = ki + kj - K)]
 *      EA: [r1[a] (k_a = K), r2[ki][ka][i][a][b] (kb = K + ki - ka)]
 *    so nIP = nocc + nk^2 nocc^2 nvir and nEA = nvir + nk^2 nocc nvir^2 complex
 *    entries; norms count each unordered pair once (|r1|^2 + |r2|^2 / 2).
 *
 * Errors: every call returns a status code; no C++ exception crosses the ABI.
 * cc_gf_last_error() gives a message for the last non-OK status of a context
 * (or, with a NULL context, of the last failed cc_gf_init in this thread).
 * A context is not thread-safe; calls on one context must not overlap.
 */
#ifndef CCGF_H
#define CCGF_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ccgf_ctx ccgf_ctx;

enum {
  CCGF_OK = 0,
  CCGF_EINVAL = -1,       /* bad argument, shape or symmetry */
  CCGF_ENOMEM = -2,       /* device (or host working) allocation failed; no C++ exception leaves the library */
  CCGF_EDEVICE = -3,      /* HIP runtime error */
  CCGF_ENOCONV = -4,      /* some solve missed the tolerance; G still written */
  CCGF_ESTATE = -5,       /* call out of order (e.g. NULL context) */
  CCGF_EUNSUPPORTED = -6  /* option not supported by the library */
};

enum { CCGF_HOST = 0, CCGF_DEVICE = 1 };
enum { CCGF_PART_IP = 1, CCGF_PART_EA = 2, CCGF_PART_BOTH = 3 };
/* Arithmetic of the sigma products inside the Krylov steps.  The residuals that
 * decide convergence, the Arnoldi orthogonalisation, the Hessenberg least squares
 * and the solution updates are FP64 in every mode; in the mixed modes the FP64
 * true residual restarts every cycle, so the restarted solve is an iterative
 * refinement and still reaches tol.  CCGF_MIXED_F32: the big products from
 * complex-float operands on FP32 MFMA.  CCGF_MIXED_BF16X3: from operands split
 * into bf16 hi + lo (x = hi + lo to about 2^-16), three BF16 MFMA products per
 * real product (hi hi + hi lo + lo hi) with FP32 accumulation; both operand copies
 * take 8 bytes per complex element. */
enum { CCGF_PLAIN_F64 = 0, CCGF_MIXED_F32 = 1, CCGF_MIXED_BF16X3 = 2 };

/* One periodic system.  All pointers are borrowed for the duration of
 * cc_gf_init only (the library copies what it needs to the device); they are
 * host pointers when mem_space == CCGF_HOST and device pointers when
 * mem_space == CCGF_DEVICE. */
typedef struct {
  int kmesh[3];              /* Gamma-centred mesh, each >= 1 */
  int nocc, nvir;            /* spin orbitals per cell, both >= 1 */
  const double *eps;         /* real [nk][nmo]: Fock diagonal (f_ov = 0) */
  const double *foo;         /* optional complex [nk][nocc][nocc]; NULL -> diag(eps) */
  const double *fvv;         /* optional complex [nk][nvir][nvir]; NULL -> diag(eps) */
  int naux;                  /* factor rank per k-pair, >= 1 (with eri_factor) */
  const double *eri_factor;  /* complex [nk][nk][naux][nmo][nmo] (see header comment); or NULL and
                                eri_blocks given */
  const double *t1;          /* complex [nk][nocc][nvir] */
  const double *t2;          /* complex [nk][nk][nk][nocc][nocc][nvir][nvir] */
  int mem_space;             /* CCGF_HOST or CCGF_DEVICE */
  /* Lambda (de-excitation) amplitudes of the left state (1 + Lambda) of Eq. 5, in the
   * layouts of t1 and t2 (l1[k][i][a] = lambda_a^i, l2[ki][kj][ka][i][j][a][b] =
   * lambda_ab^ij, antisymmetric like t2).  NULL (both): Lambda = T^dagger, the
   * approximation stated after Eq. 10.  Either both or neither; they enter only the
   * left vectors e of Eq. 7. */
  const double *l1;
  const double *l2;
  /* Alternative to eri_factor for small systems: the physicists' integrals as dense
   * momentum blocks, complex [k1][k2][k3][nmo][nmo][nmo][nmo] = <p k1, q k2 | r k3, s k4>
   * with k4 = k1 + k2 - k3, in the factor's normalisation.  Exactly one of eri_factor
   * and eri_blocks is given.  Checked when given in host memory (CCGF_EINVAL):
   * <pq|rs> = conj(<rs|pq>) and <pq|rs> = <qp|sr> to 1e-10 of the largest element. */
  const double *eri_blocks;
} ccgf_system;

typedef struct {
  int precision;    /* CCGF_PLAIN_F64; CCGF_MIXED_F32: the Krylov steps' sigma products take the
                       W_abcd, W_lbdi (EA) and W_mnij, W_maei (IP) GEMMs in complex float on FP32
                       MFMA; CCGF_MIXED_BF16X3: the same GEMMs as three BF16 products per real
                       product (hi*hi + hi*lo + lo*hi, FP32 accumulation) on BF16 MFMA.  Both
                       mixed forms keep residuals, orthogonalisation, the Hessenberg least
                       squares and a refinement from the FP64 true residual every cycle in
                       FP64, and need half the size of those blocks again in memory. */
  int restart_m;    /* Krylov vectors per cycle, 1..2000; 0 -> 30 */
  int maxiter;      /* total GMRES iterations per solve; 0 -> 2000 */
  double tol;       /* relative residual ||b - A x|| / ||b|| in the unique-pair norm; 0 -> 1e-10 */
  int max_batch;    /* right-hand sides solved together (frequencies x orbitals); 0 -> 64 */
  void *hip_stream; /* hipStream_t to run on; NULL -> the default stream */
  int timing;       /* nonzero: time the sigma kernels with HIP events (adds a wait per product) */
  double precond_eta; /* damping of the diagonal preconditioner D = w -/+ diag(M) +/- i max(eta, precond_eta);
                         0 -> eta.  Changes only the iteration count, not the solution. */
  int recycle_k;      /* GCROT(m,k): correction pairs (u, A u) kept across cycles, 0..200;
                         0 -> restarted GMRES(m). */
  double reorth_ratio; /* second Gram-Schmidt pass for a right-hand side when one pass leaves
                          less than this fraction of ||w|| (Daniel-Gragg-Kaufman-Stewart test,
                          whose classical value is 1/sqrt(2)); 0 -> 0.1; 1 -> always two passes;
                          range [0, 1]. */
  int autotune;          /* 0: pick each sigma GEMM's N tile width (64 or 32) by timing both on
                            the first two launches of every new shape; -1: always 64 */
  const char *autotune_cache; /* NULL, or a text file of earlier choices, read by cc_gf_init
                            and rewritten by cc_gf_free */
  int restart_tail;      /* restart length for cycles that start once every right-hand side of a
                            call is in flight and at most a quarter of the batch is still
                            iterating (the slowest solves); 0 -> restart_m; up to 2000, reduced
                            to fit 70% of the free device memory (GMRES only, not GCROT) */
  int graphs;            /* 0: once a sigma plan's GEMM widths are tuned, capture its launch
                            sequence (per operand pair and precision, up to 8) into a HIP graph
                            and replay it; -1: launch eagerly.  Timed runs launch eagerly. */
  int seed_m;            /* 0: every solve starts from x0 = 0.  > 0 (up to 2000): before the
                            solves of a (part, K), seed_m Arnoldi steps of sigma itself from
                            each orbital's b (all orbitals of the call batched together); the
                            Krylov space of sigma from b is that of every shifted operator
                            (w -/+ i eta) -/+ sigma, so each (orbital, w) takes the GMRES
                            minimiser over it as its starting guess where that leaves less
                            residual than x0 = 0 (elsewhere x0 = 0).  Needs (seed_m + 1) x
                            norb vectors of device memory; without it the solves start from 0.
                            Ignored while a trained guess network is enabled. */
} ccgf_options;

typedef struct {
  long long n_solves;        /* shifted systems solved */
  long long n_iterations;    /* GMRES iterations summed over solves */
  long long n_sigma;         /* sigma products applied (one per RHS per product) */
  int max_iterations;        /* largest iteration count of a single solve */
  int n_unconverged;         /* solves that missed tol */
  double max_rel_residual;   /* largest final true relative residual */
  double seconds;            /* wall time of the call */
  /* filled only when options.timing is set (HIP events on the context stream): */
  double big_ms;             /* time in the dominant sigma GEMM (EA: W_abcd term; IP: W_mnij term) */
  long long big_launches;    /* launches of that GEMM */
  double big_flops;          /* its algorithmic flops (8 per complex multiply-add) */
  double sigma_ms;           /* time in whole sigma products */
  long long sigma_launches;  /* sigma products (each over a batch of vectors) */
  long long n_steps;         /* batched Arnoldi steps (one sigma product over the active batch each) */
  long long n_reorth;        /* right-hand-side steps that needed the second Gram-Schmidt pass */
  long long n_guess;         /* solves started from a guess (trained network or Krylov seed) */
  long long n_guess_rejected; /* guesses discarded, started from 0 instead: ||b - A x0|| was not
                                 below accept ||b|| (network) or ||b|| (Krylov seed) */
  double big_bytes;          /* (timing) algorithmic HBM bytes of the big_launches: the W blocks each
                                reads, once, the vectors' operand copy once, the output written once */
} ccgf_stats;

/* Validates the system (shapes, t2 and l2 antisymmetry, factor Hermiticity, each to
 * 1e-10 relative), uploads it on the given stream and builds the
 * similarity-transformed Hamiltonian blocks on the device in FP64.
 * Returns CCGF_EINVAL for invalid input, CCGF_ENOMEM if the device is full.
 * On success *out owns all device memory until cc_gf_free. */
int cc_gf_init(const ccgf_system *sys, const ccgf_options *opt, ccgf_ctx **out);

/* Diagonal G_pp(K, w) for every (kidx[a], orbs[b], omega[c]) -- Eqs. 6, 7, 9.
 *  kidx:  nkq host ints in [0, nk);  orbs: norb host ints in [0, nmo);
 *  omega: nw host doubles (Hartree);  eta > 0 (Hartree);  parts: CCGF_PART_*.
 *  G, Gplus_opt, Gminus_opt: host complex [nkq][norb][nw], caller-allocated
 *  (the optional ones may be NULL).  G receives G+ + G- of the requested parts.
 *  st_opt may be NULL.  Returns CCGF_ENOCONV if any solve missed tol (G is
 *  still written).  tol applies to the residual of the equations on the
 *  unique 2h1p / 2p1h amplitudes (the full-storage residual projected onto
 *  antisymmetric vectors).  Device memory per call: the GMRES basis of
 *  (restart_m + 1) x min(max_batch, norb * nw) vectors of unique amplitudes
 *  (about half the full vector length; full length with recycle_k > 0), a few
 *  full-length vectors per slot, and the seed basis when seed_m > 0. */
int cc_gf_solve(ccgf_ctx *ctx, int nkq, const int *kidx, int norb, const int *orbs,
                int nw, const double *omega, double eta, int parts,
                double *G, double *Gplus_opt, double *Gminus_opt, ccgf_stats *st_opt);

/* Whole matrices G_pq(K, w) over the requested orbitals (Eqs. 7 and 9 with p != q)
 * and the density of states, the trace of the spectral function A(K, w) = -(1/pi) Im G(K, w)
 * (the equation after Eq. 9) taken with each part on the retarded side:
 * A = -(1/pi) (Im G+ - Im G-), since the removal part of Eq. 6 (w + M - i eta) is time
 * ordered (at T = V = 0 this is one unit-weight Lorentzian per orbital).  The
 * right-hand sides and solves are those of cc_gf_solve
 * (one solve per orbital, frequency and part); each solution is dotted with the left
 * vectors of every requested orbital:  G+_pq = e+_p . Y_q(w),  G-_pq = e-_q . X_p(w).
 *  G, Gplus_opt, Gminus_opt: host complex [nkq][nw][norb][norb] with element [a][w][i][j] =
 *  G_{orbs[i], orbs[j]}(kidx[a], omega[w]) (the optional ones may be NULL; G receives
 *  G+ + G- of the requested parts).  dos_opt: host real [nkq][nw], the trace of A over the
 *  requested orbitals, or NULL.  Other arguments, errors and device memory as in
 *  cc_gf_solve, plus (norb x norb) complex per right-hand side in flight. */
int cc_gf_solve_matrix(ccgf_ctx *ctx, int nkq, const int *kidx, int norb, const int *orbs,
                       int nw, const double *omega, double eta, int parts,
                       double *G, double *Gplus_opt, double *Gminus_opt, double *dos_opt,
                       ccgf_stats *st_opt);

/* Learned initial guess (a network trained on the solver's own solutions).
 * Not part of the paper's method: a companion to it that changes only where
 * GMRES starts, never what it converges to. */
typedef struct {
  int epochs;              /* passes over the training pairs; 0 -> 300 */
  int batch;               /* pairs per Adam step; 0 -> 256 */
  double lr;               /* Adam step size; 0 -> 1e-3 */
  unsigned long long seed; /* parameter initialisation and shuffling */
  int hidden;              /* width of the two tanh hidden layers; 0 -> 256 */
  int guess;               /* CCGF_GUESS_NETWORK (0): x0 from the network;
                              CCGF_GUESS_NEAREST: x0 = the training solution at the
                              nearest training frequency (no network; for comparison) */
  double accept;           /* a guess is used only if ||b - A x0|| < accept * ||b||, in (0, 1];
                              0 -> 0.1 (a guess that leaves most of b tends to slow GMRES:
                              its residual is rich in the near-resonant directions) */
  int probe;               /* learned preconditioner: GMRES steps of each probe solve (below);
                              0 -> 40; -1: no preconditioner network */
} ccgf_learn_options;
enum { CCGF_GUESS_NETWORK = 0, CCGF_GUESS_NEAREST = 1 };

typedef struct {
  long long pairs;          /* training pairs */
  int rank;                 /* reduced-basis size per orbital (training frequencies) */
  double loss_initial;      /* mean squared error / 2 over all pairs before and after training */
  double loss_final;
  double solve_seconds;     /* plain solves that produced the training solutions */
  double train_seconds;     /* network training on the GPU */
  long long solve_iterations;
  double probe_seconds;     /* probe solves of the preconditioner network */
  double precond_loss_initial; /* its mean squared error / 2 before and after training */
  double precond_loss_final;
} ccgf_learn_stats;

/* Candidate dampings of the learned preconditioner, in units of the largest of eta and
 * the context's precond_eta: D = w -/+ diag(M) +/- i eta_p with eta_p one of these. */
#define CCGF_PRECOND_CANDIDATES 5

/* Train the initial-guess network of momentum K and the given parts
 * (CCGF_PART_*), and the preconditioner network.  The plain solver (the context's options) solves the shifted
 * systems of Eq. 6 for every (orbs[b], omega_train[j]); per orbital, the
 * solutions are orthonormalised (Gram-Schmidt twice, dependent columns zeroed)
 * into a basis Q_p of rank ntrain, and c_j = Q_p^H x_j are their reduced
 * coordinates.  A three-layer perceptron (two tanh hidden layers, FP32,
 * trained by Adam on the GPU; zero output layer at the start) learns the move
 *   (w, (w - w_ref)/step, Fock diagonal of p, occupied flag, c_ref) -> c(w) - c_ref
 * from the pairs (j, j_ref) with |j - j_ref| <= 2.  Afterwards cc_gf_solve
 * starts each (K, p, w) solve of a trained orbital from x0 = Q_p c_hat,
 * c_hat = c_ref + network output, with c_ref taken at the training frequency
 * nearest to w; a guess whose residual is not below accept * ||b|| is
 * discarded and the solve starts from zero.
 * Preconditioner network (unless opt->probe = -1): every training (p, w) is
 * solved again from zero for opt->probe GMRES steps with each candidate damping
 * eta_p of the diagonal preconditioner (0.25, 0.5, 1, 1.5, 2.5 times the context's
 * damping), all in one batch, and a second perceptron of the same form learns
 *   (w, Fock diagonal of p, occupied flag, w - Fock diagonal) -> log10 of each
 * candidate's relative residual after those steps.  cc_gf_solve then gives each
 * (K, p, w) solve the damping the network predicts to leave the smallest residual:
 * a per-right-hand-side diagonal correction of D, judged like any preconditioner
 * by the FP64 true residual (it changes the iteration count, never the solution).
 * The model replaces any earlier one of the same (part, K).  ntrain in 1..32,
 * sorted ascending, finite.  opt and st may be NULL.  Device memory: ntrain * norb
 * vectors per part are kept for the basis. */
int cc_gf_learn(ccgf_ctx *ctx, int parts, int K, int norb, const int *orbs, int ntrain,
                const double *omega_train, double eta, const ccgf_learn_options *opt_opt,
                ccgf_learn_stats *st_opt);

/* Replace the solver options of a context (tolerance, restart length, batch width,
 * stream, preconditioner damping, seed length, timing, ...) without rebuilding its
 * Hamiltonian blocks.  The precision must equal the one the context was built with
 * (CCGF_EUNSUPPORTED otherwise: its operand copies are made by cc_gf_init); the
 * autotune file stays the one given to cc_gf_init.  Zero fields take the defaults of
 * cc_gf_init; out-of-range values give CCGF_EINVAL and leave the context unchanged.
 * Waits for the context's stream before switching. */
int cc_gf_set_options(ccgf_ctx *ctx, const ccgf_options *opt);

/* Which trained networks cc_gf_solve uses: a mask of CCGF_LEARN_GUESS (initial
 * guesses) and CCGF_LEARN_PRECOND (per-solve preconditioner damping); 0 ignores
 * both.  Every cc_gf_learn call sets both again. */
enum { CCGF_LEARN_GUESS = 1, CCGF_LEARN_PRECOND = 2 };
int cc_gf_learn_enable(ccgf_ctx *ctx, int on);

/* Persist the networks trained by cc_gf_learn (all parts and momenta) to a file at
 * path, and read them back into a context of the same system shape (k-mesh, nocc,
 * nvir: CCGF_EINVAL otherwise).  The file holds, per (part, K), the two networks'
 * parameters, their feature scales, the training frequencies and orbitals, and the
 * guess network's reduced basis Q (norb x rank vectors of the part's length, so it can
 * be gigabytes at large meshes).  Loading replaces every model of the context and
 * enables both networks (cc_gf_learn_enable).  Save: CCGF_ESTATE when nothing is
 * trained; I/O failures give CCGF_EINVAL with the reason in cc_gf_last_error.  The
 * format is this library's own (a magic tag and version first); host memory for one
 * model's basis is used as staging. */
int cc_gf_learn_save(ccgf_ctx *ctx, const char *path);
int cc_gf_learn_load(ccgf_ctx *ctx, const char *path);

/* Least-squares loss and its gradient for the network above, for checking the
 * training kernels: theta, X [N][din], T [N][dout], grad [nparams] are HOST
 * FP32 arrays (parameter order W1 [hidden][din], b1, W2 [hidden][hidden], b2,
 * W3 [dout][hidden], b3); *loss_opt = |Y - T|^2 / (2N).  Runs on the current
 * device; allocates and frees its own device buffers.  Dimensions 1..4096. */
int cc_gf_mlp_grad(int din, int hidden, int dout, const float *theta, int N, const float *X,
                   const float *T, float *grad, double *loss_opt);

/* Largest number of expansion frequencies per part accepted by cc_gf_mor. */
#define CCGF_MOR_MAX 32

/* Model-order-reduced G_pp(K, w) (MOR paragraph of the results; Eqs. 6, 7, 9):
 * for every (kidx[a], orbs[b]) and part, the shifted systems of Eq. 6 are
 * solved in full (same solver and tol as cc_gf_solve) only at the expansion
 * frequencies wexp_ip[0..nexp_ip) (IP) and wexp_ea[0..nexp_ea) (EA); their
 * solutions are orthonormalised (Gram-Schmidt twice, unique-pair inner
 * product, columns below 1e-10 of the largest solution norm dropped) into S;
 * the model Ht = S^H M S, bt = S^H b, et = e S is then solved on every omega
 * (one-sided Galerkin projection; exact at the expansion points up to the
 * solve tolerance).  Counts: nexp_* in 1..CCGF_MOR_MAX for each requested
 * part (the other part's pointer may be NULL).  Other arguments, layouts and
 * ownership as in cc_gf_solve.  Returns CCGF_ENOCONV if an expansion solve
 * missed tol (G is still written). */
int cc_gf_mor(ccgf_ctx *ctx, int nkq, const int *kidx, int norb, const int *orbs,
              int nexp_ip, const double *wexp_ip, int nexp_ea, const double *wexp_ea,
              int nw, const double *omega, double eta, int parts,
              double *G, double *Gplus_opt, double *Gminus_opt, ccgf_stats *st_opt);

/* Length (complex entries) of an EOM vector of the given part (CCGF_PART_IP or
 * CCGF_PART_EA) in the full antisymmetric storage described above. */
int cc_gf_vector_size(const ccgf_ctx *ctx, int part, long long *n);

/* sigma = M(K) r for nvec vectors: the EOM-IP or EOM-EA matrix (connected
 * commutator of Hbar, the hot product inside every solve of Eq. 6), in the
 * arithmetic of the context's Krylov steps (options.precision).
 * x, y: DEVICE complex [nvec][n] (n from cc_gf_vector_size), not aliased;
 * x must be antisymmetric in its pair indices.  Runs on the context stream
 * and returns after the product is complete. */
int cc_gf_sigma(ccgf_ctx *ctx, int part, int K, int nvec, const double *x, double *y);

/* The sigma products of several systems at once (uneven k-meshes, orbital counts and
 * parts): y_i = M_i(K[i]) x_i for i < nsys, as cc_gf_sigma on each context (same
 * arithmetic per element), with every GEMM term of the products (W_abcd, W_mnij, W_ovvo,
 * the couplings and the 1h / 1p reductions) issued as ONE launch whose tasks cover all
 * the systems, each task with its own shape and operands; small systems then share the
 * chip instead of each under-filling it.  ctxs: distinct contexts of the same precision
 * (CCGF_PLAIN_F64 or CCGF_MIXED_F32; CCGF_EUNSUPPORTED for the BF16 split) on one device;
 * parts[i] CCGF_PART_IP or CCGF_PART_EA; x[i], y[i]: DEVICE complex [nvec[i]][n_i], not
 * aliased, x antisymmetric in its pair indices.  Runs on ctxs[0]'s stream after waiting
 * for every context's stream; returns after the products are complete.  Errors go to
 * ctxs[0] (cc_gf_last_error). */
int cc_gf_sigma_group(int nsys, ccgf_ctx *const *ctxs, const int *parts, const int *K, const int *nvec,
                      const double *const *x, double *const *y);

/* Right-hand side b (abar_p|Phi> for IP, abar+_p|Phi> for EA) and left vector
 * e (<Phi|(1+Lambda) abar+_p for IP, <Phi|(1+Lambda) abar_p for EA) of orbital
 * p at momentum K (Eqs. 6-7).  b, e: DEVICE complex [n]; either may be NULL. */
int cc_gf_vectors(ccgf_ctx *ctx, int part, int K, int p, double *b, double *e);

/* Active-space self-energy correction and Dyson's equation (Eqs. 12-14):
 *   Sigma_CAS  = G_GW,CAS^-1 - G_CC,CAS^-1                    (M x M)
 *   Sigma_full = V Sigma_CAS V^H                               (N x N)
 *   G_CC+GW    = [G_GW,full^-1 - Sigma_full]^-1                (N x N)
 * at every (k, w) of a batch; needs no context.  All arrays are DEVICE complex:
 *   Ggw     [nk][nw][N][N]  G_GW,full, the low-level Green's function in the full orbital basis;
 *   Ggw_cas [nk][nw][M][M]  G_GW,CAS, the low-level Green's function of the active space (for
 *                           instance V^H G_GW,full V, or a low-level calculation within the space);
 *   Gcc     [nk][nw][M][M]  G_CC,CAS, the CCGF of the active space (cc_gf_solve_matrix of the
 *                           active-space system, G+ + G-);
 *   V       [nk][N][M]      active natural orbitals in the full basis (columns);
 *   Gout    [nk][nw][N][N]  receives G_CC+GW; Sfull_opt [nk][nw][N][N] and Scas_opt
 *                           [nk][nw][M][M] receive the self-energies when not NULL.
 * Row-major matrices.  Sizes: nk >= 1, nw >= 0, 1 <= M <= N <= 64.  Runs on hip_stream (NULL:
 * the default stream) and returns after the results are complete.  Returns CCGF_EINVAL for
 * bad sizes or when a matrix to invert is singular (Gauss-Jordan with partial pivoting in
 * FP64 finds a zero pivot), CCGF_ENOMEM when the scratch buffer (about 16 (4 M^2 + 3 N^2 +
 * N M + M^2) bytes per (k, w) point) cannot be allocated.  Messages: cc_gf_dyson_last_error. */
int cc_gf_dyson_cas(int nk, int nw, int N, int M, const double *Ggw, const double *Ggw_cas,
                    const double *Gcc, const double *V, double *Gout, double *Sfull_opt,
                    double *Scas_opt, void *hip_stream);

/* cc_gf_dyson_cas for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): same arguments, results
 * and errors, but it calls no allocating routine.  Its scratch is one fixed 64 MiB array per
 * device, held until the process ends; batches larger than it holds are processed in chunks
 * of (k, w) points, and a (k, w) point that alone needs more (impossible for N <= 64) gives
 * CCGF_EINVAL.  Every call on a device shares that device's array: calls that overlap on one
 * device (other host threads, other streams) race and must not be issued.  It reports a
 * singular matrix without saying at which point, and returns after the results are complete. */
int cc_gf_dyson_cas_noalloc(int nk, int nw, int N, int M, const double *Ggw, const double *Ggw_cas,
                            const double *Gcc, const double *V, double *Gout, double *Sfull_opt,
                            double *Scas_opt, void *hip_stream);

/* Message for the last failed cc_gf_dyson_cas(_noalloc) call of this thread (never NULL). */
const char *cc_gf_dyson_last_error(void);

/* Releases all device memory of the context (NULL is ignored). */
void cc_gf_free(ccgf_ctx *ctx);

/* Message for the last non-OK status (never NULL). */
const char *cc_gf_last_error(const ccgf_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* CCGF_H */
