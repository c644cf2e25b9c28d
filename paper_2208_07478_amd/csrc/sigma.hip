// k-point EOM-IP/EA-CCSD sigma products on gfx950.
//
// The dominant terms (EA: 1/2 W_abcd r_i^cd, cost O(Nk^3 No Nv^4); IP: the
// W_mbej and W_mnij terms, O(Nk^3 No^3 Nv^2); the paper's scaling paragraph)
// are block-dense complex contractions over momentum-conserving k-blocks.  They
// run as one segmented complex GEMM per term: a task is one output k-block for
// all right-hand sides at once (N = pair index x RHS), its segments are the
// summed momentum blocks, and the complex product is three real FP64 MFMA
// 16x16x4 products per step (Gauss' three-multiplication form).  The 1p/1h ->
// 2p1h/2h1p couplings are small-K GEMMs of the same kind.  The one-body F terms,
// the antisymmetriser and the three-body T2 piece are element-wise (one thread
// per element, looping over the right-hand sides); the 1p/1h rows are
// reductions split over blocks.
#include "ccgf_internal.h"

#include <algorithm>
#include <type_traits>
#include <cstdio>
#include <cstdlib>
#include <cstring>

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

#define TM 64
#define TK 16

__device__ inline long long imap(const IdxMap &m, int x) {
  if (x < m.L) return (long long)x * m.s1;  // one-level maps never divide
  return (long long)(x / m.L) * m.s0 + (long long)(x % m.L) * m.s1;
}

// Real arithmetic of one GEMM variant: FP64 (A complex double) or FP32 (A complex
// float, vectors read from their complex float copy, FP32 accumulation).  ROW gives the
// output row of MFMA item v in lane group g (l / 16), measured per instruction:
// the FP64 16x16x4 spreads a lane's four items over rows g, g+4, g+8, g+12, the
// FP32 16x16x4 gives them four consecutive rows 4g .. 4g+3.
template <typename R>
struct Mf;
template <>
struct Mf<double> {
  typedef v4d V4;
  typedef double2 AE;
  __device__ static inline V4 mm(double a, double b, V4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int g, int v) { return g + 4 * v; }
};
template <>
struct Mf<float> {
  typedef v4f V4;
  typedef float2 AE;
  __device__ static inline V4 mm(float a, float b, V4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static inline int row(int g, int v) { return 4 * g + v; }
};

// C[m][n] = alpha * sum_seg sum_k A[m][k] B[k][n] (+ C), complex, on MFMA.
// TAG only separates the uses in kernel traces (0: EA W_abcd, 1: EA W_lbdi,
// 2: IP W_mnij, 3: IP W_maei, 4: EA W_abei r^e, 5: IP W_maij r_m, 6: EA 1p-row
// reductions W_alcd r, <kl||cd> r, 7: IP 1h-row reductions W_mnie r, <mn||ef> r,
// 8 and 9: EA W_abcd on the blocks ka = kb, pairs kc = kd and kc < kd).
// TNT is the tile width in N (64; 16, 32 or 48 for narrow batches, the smallest
// that holds N so that little of the MFMA work is padding; 128 in FP32 to read W
// fewer times); the four waves of a block own 32x32 (TNT = 64), 16 x TNT
// (TNT <= 48) or 32x64 (TNT = 128) output sub-tiles.
// One output tile (tm, tn) of one task: the body shared by the launch over one shape
// (k_cgemm) and the launch over the tasks of several systems (k_cgemm_group).
template <int TAG, typename R, int TNT>
__device__ __forceinline__ void cgemm_tile(const GemmShape &sh, const GemmTask &task,
                                           const GemmSeg *__restrict__ segs,
                                           const typename Mf<R>::AE *__restrict__ A,
                                           const typename Mf<R>::AE *__restrict__ B, cplx *__restrict__ C, int tm,
                                           int tn) {
  typedef typename Mf<R>::V4 V4;
  typedef typename Mf<R>::AE AE;
  // k-slab: 32 for the FP32 W_abcd products (half the barriers per k), else 16
  constexpr int KS = (sizeof(R) == 4 && (TAG == 0 || TAG == 8 || TAG == 9)) ? 2 * TK : TK;
  constexpr int RPP = 256 / KS;            // rows staged per pass of the block
  constexpr int AJ = TM / RPP;             // A rows staged per thread
  constexpr int NBJ = TNT / RPP;           // B rows staged per thread
  // narrow tiles (16, 32, 48 columns): the four waves split the 64 rows, each holding every
  // column; 64 and 128 columns: 2 x 2 waves of 32 rows
  constexpr bool NARROW = TNT <= 48;
  constexpr int AM = NARROW ? 1 : 2;                 // MFMA row tiles per wave
  constexpr int BN = NARROW ? TNT / 16 : TNT / 32;   // MFMA column tiles per wave
  __shared__ R Ar[TM][KS + 1], Ai[TM][KS + 1], Br[TNT][KS + 1], Bi[TNT][KS + 1];
  const int tid = threadIdx.x;

  // each thread stages column kt of rows rt + RPP j of both tiles
  const int kt = tid & (KS - 1), rt = tid / KS;
  long long aoff[AJ], boff[NBJ];
  bool aok[AJ], bok[NBJ];
#pragma unroll
  for (int j = 0; j < AJ; ++j) {
    int m = tm * TM + rt + RPP * j;
    aok[j] = m < sh.M;
    aoff[j] = aok[j] ? imap(sh.am, sh.mtab ? sh.mtab[m] : m) : 0;
  }
#pragma unroll
  for (int j = 0; j < NBJ; ++j) {
    int n = tn * TNT + rt + RPP * j;
    bok[j] = n < sh.N;
    boff[j] = bok[j] ? imap(sh.bn, n) : 0;
  }
  const int ksteps = (sh.K + KS - 1) / KS;
  const int nsteps = task.nseg * ksteps;

  // Gauss' three-product form: P1 = Ar Br, P2 = Ai Bi, P3 = (Ar + Ai)(Br + Bi);
  // C = (P1 - P2) + i (P3 - P1 - P2)
  V4 P1[AM][BN], P2[AM][BN], P3[AM][BN];
#pragma unroll
  for (int a = 0; a < AM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b) {
      P1[a][b] = (V4){0, 0, 0, 0};
      P2[a][b] = (V4){0, 0, 0, 0};
      P3[a][b] = (V4){0, 0, 0, 0};
    }

  AE ra[AJ], rb[NBJ];
  auto load = [&](int step) {
    int s = step / ksteps;
    int k = (step - s * ksteps) * KS + kt;
    GemmSeg sg = segs[task.seg_begin + s];
    const bool kok = k < sh.K;
    if (kok && sh.ktab) k = sh.ktab[k];
    const AE *Ap = A + sg.a_off + (kok ? imap(sh.ak, k) : 0);
    const AE *Bp = B + sg.b_off + (kok ? imap(sh.bk, k) : 0);
    const R w = (R)sg.w;  // 1 or 1/2: exact in either precision
    // unconditional loads (an element outside the operand reads the operand's first one
    // instead and is zeroed after the load): no branch around each load
#pragma unroll
    for (int j = 0; j < AJ; ++j) {
      const bool ok = aok[j] && kok;
      const AE a = *(ok ? Ap + aoff[j] : A);
      ra[j] = ok ? a : AE{0, 0};
    }
#pragma unroll
    for (int j = 0; j < NBJ; ++j) {
      const bool ok = bok[j] && kok;
      const AE b = *(ok ? Bp + boff[j] : B);
      rb[j] = ok ? AE{b.x * w, b.y * w} : AE{0, 0};
    }
  };

  const int wave = tid >> 6, lane = tid & 63;
  // rows [rbase, rbase + 16 AM) and columns [cbase, cbase + 16 BN) of the tile belong to this wave
  const int rbase = NARROW ? wave * 16 : (wave >> 1) * 32;
  const int cbase = NARROW ? 0 : (wave & 1) * (TNT / 2);
  const int lr = lane & 15, lk = lane >> 4;

  if (nsteps > 0) load(0);
  for (int step = 0; step < nsteps; ++step) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < AJ; ++j) {
      Ar[rt + RPP * j][kt] = (R)ra[j].x;
      Ai[rt + RPP * j][kt] = (R)ra[j].y;
    }
#pragma unroll
    for (int j = 0; j < NBJ; ++j) {
      Br[rt + RPP * j][kt] = (R)rb[j].x;
      Bi[rt + RPP * j][kt] = (R)rb[j].y;
    }
    __syncthreads();
    if (step + 1 < nsteps) load(step + 1);
#pragma unroll
    for (int kk = 0; kk < KS; kk += 4) {
      R a_r[AM], a_i[AM], a_s[AM], b_r[BN], b_i[BN], b_s[BN];
#pragma unroll
      for (int q = 0; q < AM; ++q) {
        a_r[q] = Ar[rbase + q * 16 + lr][kk + lk];
        a_i[q] = Ai[rbase + q * 16 + lr][kk + lk];
        a_s[q] = a_r[q] + a_i[q];
      }
#pragma unroll
      for (int q = 0; q < BN; ++q) {
        b_r[q] = Br[cbase + q * 16 + lr][kk + lk];
        b_i[q] = Bi[cbase + q * 16 + lr][kk + lk];
        b_s[q] = b_r[q] + b_i[q];
      }
#pragma unroll
      for (int a = 0; a < AM; ++a)
#pragma unroll
        for (int b = 0; b < BN; ++b) {
          P1[a][b] = Mf<R>::mm(a_r[a], b_r[b], P1[a][b]);
          P2[a][b] = Mf<R>::mm(a_i[a], b_i[b], P2[a][b]);
          P3[a][b] = Mf<R>::mm(a_s[a], b_s[b], P3[a][b]);
        }
    }
  }

#pragma unroll
  for (int a = 0; a < AM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int row = rbase + a * 16 + Mf<R>::row(lk, v);
        int col = cbase + b * 16 + lr;
        int m = tm * TM + row, n = tn * TNT + col;
        if (m < sh.M && n < sh.N) {
          long long off = task.c_off + imap(sh.cm, sh.mtab ? sh.mtab[m] : m) + imap(sh.cn, n);
          double p1 = P1[a][b][v], p2 = P2[a][b][v];
          double re = p1 - p2, im = (double)P3[a][b][v] - p1 - p2;
          cplx val = mkc(sh.alpha_re * re - sh.alpha_im * im, sh.alpha_re * im + sh.alpha_im * re);
          if (sh.accumulate) val = cadd(val, C[off]);
          C[off] = val;
        }
      }
}

// XCD-aware block order: the hardware hands block b to XCD b % 8, so XCD x runs blocks
// x, x + 8, ...; give it the consecutive logical tiles [x q + min(x, r), ...) (q = total / 8,
// r = total % 8: the first r XCDs take one more).  Tiles of one task that read the same
// operand panel (its N tiles, its M tiles) then share an XCD and its L2.
__device__ inline int xcd_block(int total) {
  const int bid = blockIdx.x, x = bid & 7, j = bid >> 3;
  const int q = total >> 3, r = total & 7;
  return x * q + min(x, r) + j;
}

template <int TAG, typename R, int TNT>
__global__ __launch_bounds__(256, TNT <= 48 ? 4 : 2) void k_cgemm(GemmShape sh, const GemmTask *__restrict__ tasks,
                                                                  const GemmSeg *__restrict__ segs,
                                                                  const typename Mf<R>::AE *__restrict__ A,
                                                                  const typename Mf<R>::AE *__restrict__ B,
                                                                  cplx *__restrict__ C, int tilesM, int tilesN,
                                                                  int total) {
  const int bid = xcd_block(total);
  const int per_task = tilesM * tilesN;
  const int t = bid / per_task, r = bid % per_task;
  cgemm_tile<TAG, R, TNT>(sh, tasks[t], segs, A, B, C, r / tilesN, r % tilesN);
}

// One launch over the tasks of several systems (uneven shapes): task g covers the blocks
// [tile0, tile0 + tilesM * tilesN) and carries its shape and operand bases.
struct GroupTask {
  const void *A, *B;
  cplx *C;
  GemmTask task;
  int shape, tile0, tilesM, tilesN;
};

template <int TAG, typename R, int TNT>
__global__ __launch_bounds__(256, TNT <= 48 ? 4 : 2) void k_cgemm_group(const GemmShape *__restrict__ shapes,
                                                                        const GroupTask *__restrict__ gt, int ntask,
                                                                        const GemmSeg *__restrict__ segs, int total) {
  const int bid = xcd_block(total);
  int lo = 0, hi = ntask - 1;  // the last task whose first block is <= bid
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (gt[mid].tile0 <= bid) lo = mid;
    else hi = mid - 1;
  }
  const GroupTask g = gt[lo];
  const int r = bid - g.tile0;
  cgemm_tile<TAG, R, TNT>(shapes[g.shape], g.task, segs, (const typename Mf<R>::AE *)g.A,
                          (const typename Mf<R>::AE *)g.B, g.C, r / g.tilesN, r % g.tilesN);
}

// BF16-split variant of the same product for the mixed form.  Both operands are
// stored pre-split, four bf16 planes per complex element (re hi, re lo, im hi, im lo
// with hi = bf16(x) and lo = bf16(x - hi), so x = hi + lo to about 2^-16 relative):
// W once when the context is built, the vectors once per product (k_to_b3).  Each
// real product is taken as hi*hi + hi*lo + lo*hi on the 16x16x32 BF16 MFMA with FP32
// accumulation, and the complex product from its four real products (the two cross
// terms share an accumulator): twelve MFMAs per 16x16x32 step, no conversions in the
// inner loop.  Lane l feeds row (or column) l%16 and k = 8(l/16) .. +7; item v of
// lane l is row 4(l/16)+v.  Tiles and staging follow cgemm_tile, with k-slabs of 32.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
// the two bf16 values packed in a 32-bit word (low half first), each times w; exact for
// w = 1/2 on normal values (the bf16 bits sit in the top half of an FP32 word)
__device__ inline unsigned scale_bf2(unsigned x, float w) {
  const float lo = __uint_as_float(x << 16) * w, hi = __uint_as_float(x & 0xffff0000u) * w;
  return (__float_as_uint(lo) >> 16) | (__float_as_uint(hi) & 0xffff0000u);
}
__device__ inline __bf16 bf_lo(unsigned x) { return __builtin_bit_cast(__bf16, (unsigned short)(x & 0xffffu)); }
__device__ inline __bf16 bf_hi(unsigned x) { return __builtin_bit_cast(__bf16, (unsigned short)(x >> 16)); }

// PAIR: each thread stages the k pair (2 kt, 2 kt + 1) of its rows with one 16-byte load
// and writes each plane's two values with one 4-byte LDS store (for operands whose k pairs
// are adjacent and 16-byte aligned, GemmPlan::pairs); else one element and four 2-byte stores.
template <int TAG, int TNT, bool PAIR>
__device__ __forceinline__ void cgemm_b3_tile(const GemmShape &sh, const GemmTask &task,
                                              const GemmSeg *__restrict__ segs, const B3E *__restrict__ A,
                                              const B3E *__restrict__ B, cplx *__restrict__ C, int tm, int tn) {
  constexpr int KS = 32, LD = KS + 8;  // k-slab; LDS row stride in bf16 (rows stay 16-byte aligned)
  constexpr int KP = PAIR ? 2 : 1;     // k per thread
  constexpr int RPP = 256 * KP / KS;   // rows staged per pass of the block
  constexpr int AJ = TM / RPP;         // A rows staged per thread
  constexpr int NBJ = TNT / RPP;       // B rows staged per thread
  static_assert(NBJ >= 1, "tile narrower than a staging pass");
  constexpr bool NARROW = TNT <= 48;
  constexpr int AM = NARROW ? 1 : 2;                // MFMA row tiles per wave
  constexpr int BN = NARROW ? TNT / 16 : TNT / 32;  // MFMA column tiles per wave
  __shared__ __attribute__((aligned(16))) __bf16 As[4][TM][LD];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[4][TNT][LD];
  const int tid = threadIdx.x;
  const int kt = tid & (KS / KP - 1), rt = tid / (KS / KP);
  long long aoff[AJ], boff[NBJ];
  bool aok[AJ], bok[NBJ];
#pragma unroll
  for (int j = 0; j < AJ; ++j) {
    int m = tm * TM + rt + RPP * j;
    aok[j] = m < sh.M;
    aoff[j] = aok[j] ? imap(sh.am, sh.mtab ? sh.mtab[m] : m) : 0;
  }
#pragma unroll
  for (int j = 0; j < NBJ; ++j) {
    int n = tn * TNT + rt + RPP * j;
    bok[j] = n < sh.N;
    boff[j] = bok[j] ? imap(sh.bn, n) : 0;
  }
  const int ksteps = (sh.K + KS - 1) / KS;
  const int nsteps = task.nseg * ksteps;
  v4f Prr[AM][BN], Pii[AM][BN], Px[AM][BN];
#pragma unroll
  for (int a = 0; a < AM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b) {
      Prr[a][b] = (v4f){0, 0, 0, 0};
      Pii[a][b] = (v4f){0, 0, 0, 0};
      Px[a][b] = (v4f){0, 0, 0, 0};
    }
  // staged values: KP elements (KP x 8 bytes) per row and thread
  typedef typename std::conditional<PAIR, uint4, uint2>::type SV;
  SV ra[AJ], rb[NBJ];
  auto load = [&](int step) {
    int s = step / ksteps;
    int k = (step - s * ksteps) * KS + KP * kt;
    GemmSeg sg = segs[task.seg_begin + s];
    const bool kok = k < sh.K;  // (with PAIR, K is even: k + 1 < K too)
    if (kok && sh.ktab) k = sh.ktab[k];
    const B3E *Ap = A + sg.a_off + (kok ? imap(sh.ak, k) : 0);
    const B3E *Bp = B + sg.b_off + (kok ? imap(sh.bk, k) : 0);
    // unconditional loads (an element outside the operand reads the operand's first one
    // instead and is zeroed after the load): no branch around each load
    const SV z{};
#pragma unroll
    for (int j = 0; j < AJ; ++j) {
      const bool ok = aok[j] && kok;
      const SV v = *(const SV *)(ok ? Ap + aoff[j] : A);
      ra[j] = ok ? v : z;
    }
#pragma unroll
    for (int j = 0; j < NBJ; ++j) {
      const bool ok = bok[j] && kok;
      const SV v = *(const SV *)(ok ? Bp + boff[j] : B);
      rb[j] = ok ? v : z;
    }
    if (sg.w != 1.0) {  // 1/2 (self-paired segments): exact on each bf16 value
      const float w = (float)sg.w;
#pragma unroll
      for (int j = 0; j < NBJ; ++j) {
        rb[j].x = scale_bf2(rb[j].x, w);
        rb[j].y = scale_bf2(rb[j].y, w);
        if constexpr (PAIR) {
          rb[j].z = scale_bf2(rb[j].z, w);
          rb[j].w = scale_bf2(rb[j].w, w);
        }
      }
    }
  };
  // one thread's staged values into the four planes of rows r (element e of the pair: word
  // 2 e holds (re hi, re lo), word 2 e + 1 (im hi, im lo), low half first)
  auto stage = [&](auto &P, int r, const SV &v) {
    if constexpr (PAIR) {
      const unsigned w0 = v.x, w1 = v.y, w2 = v.z, w3 = v.w;
      *(unsigned *)&P[0][r][2 * kt] = (w0 & 0xffffu) | (w2 << 16);
      *(unsigned *)&P[1][r][2 * kt] = (w0 >> 16) | (w2 & 0xffff0000u);
      *(unsigned *)&P[2][r][2 * kt] = (w1 & 0xffffu) | (w3 << 16);
      *(unsigned *)&P[3][r][2 * kt] = (w1 >> 16) | (w3 & 0xffff0000u);
    } else {
      P[0][r][kt] = bf_lo(v.x);
      P[1][r][kt] = bf_hi(v.x);
      P[2][r][kt] = bf_lo(v.y);
      P[3][r][kt] = bf_hi(v.y);
    }
  };
  const int wave = tid >> 6, lane = tid & 63;
  const int rbase = NARROW ? wave * 16 : (wave >> 1) * 32;
  const int cbase = NARROW ? 0 : (wave & 1) * (TNT / 2);
  const int lr = lane & 15, lk = lane >> 4;
  if (nsteps > 0) load(0);
  for (int step = 0; step < nsteps; ++step) {
    __syncthreads();
#pragma unroll
    for (int j = 0; j < AJ; ++j) stage(As, rt + RPP * j, ra[j]);
#pragma unroll
    for (int j = 0; j < NBJ; ++j) stage(Bs, rt + RPP * j, rb[j]);
    __syncthreads();
    if (step + 1 < nsteps) load(step + 1);
    v8bf fa[AM][4];
#pragma unroll
    for (int q = 0; q < AM; ++q)
#pragma unroll
      for (int p = 0; p < 4; ++p) fa[q][p] = *(const v8bf *)&As[p][rbase + q * 16 + lr][8 * lk];
#pragma unroll
    for (int b = 0; b < BN; ++b) {
      v8bf fb[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) fb[p] = *(const v8bf *)&Bs[p][cbase + b * 16 + lr][8 * lk];
#pragma unroll
      for (int a = 0; a < AM; ++a) {
        // planes: 0 re hi, 1 re lo, 2 im hi, 3 im lo
        Prr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[0], Prr[a][b], 0, 0, 0);
        Prr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[1], Prr[a][b], 0, 0, 0);
        Prr[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][1], fb[0], Prr[a][b], 0, 0, 0);
        Pii[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][2], fb[2], Pii[a][b], 0, 0, 0);
        Pii[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][2], fb[3], Pii[a][b], 0, 0, 0);
        Pii[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][3], fb[2], Pii[a][b], 0, 0, 0);
        Px[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[2], Px[a][b], 0, 0, 0);
        Px[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][0], fb[3], Px[a][b], 0, 0, 0);
        Px[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][1], fb[2], Px[a][b], 0, 0, 0);
        Px[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][2], fb[0], Px[a][b], 0, 0, 0);
        Px[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][2], fb[1], Px[a][b], 0, 0, 0);
        Px[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[a][3], fb[0], Px[a][b], 0, 0, 0);
      }
    }
  }
#pragma unroll
  for (int a = 0; a < AM; ++a)
#pragma unroll
    for (int b = 0; b < BN; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int row = rbase + a * 16 + 4 * lk + v;
        int col = cbase + b * 16 + lr;
        int m = tm * TM + row, n = tn * TNT + col;
        if (m < sh.M && n < sh.N) {
          long long off = task.c_off + imap(sh.cm, sh.mtab ? sh.mtab[m] : m) + imap(sh.cn, n);
          const double re = (double)Prr[a][b][v] - (double)Pii[a][b][v], im = Px[a][b][v];
          cplx val = mkc(sh.alpha_re * re - sh.alpha_im * im, sh.alpha_re * im + sh.alpha_im * re);
          if (sh.accumulate) val = cadd(val, C[off]);
          C[off] = val;
        }
      }
}

template <int TAG, int TNT, bool PAIR>
__global__ __launch_bounds__(256, 2) void k_cgemm_b3(GemmShape sh, const GemmTask *__restrict__ tasks,
                                                     const GemmSeg *__restrict__ segs, const B3E *__restrict__ A,
                                                     const B3E *__restrict__ B, cplx *__restrict__ C, int tilesM,
                                                     int tilesN, int total) {
  const int bid = xcd_block(total);
  const int per_task = tilesM * tilesN;
  const int t = bid / per_task, r = bid % per_task;
  cgemm_b3_tile<TAG, TNT, PAIR>(sh, tasks[t], segs, A, B, C, r / tilesN, r % tilesN);
}

template <int TAG, int TNT>
static void launch_b3t(const GemmPlan &plan, const void *A, const void *B, cplx *C, hipStream_t s) {
  const GemmShape &sh = plan.shape;
  const int tilesM = (sh.M + TM - 1) / TM, tilesN = (sh.N + TNT - 1) / TNT;
  const long long total = (long long)plan.ntask * tilesM * tilesN;
  if (plan.pairs)
    hipLaunchKernelGGL((k_cgemm_b3<TAG, TNT, true>), dim3((unsigned)total), dim3(256), 0, s, sh, plan.d_tasks,
                       plan.d_segs, (const B3E *)A, (const B3E *)B, C, tilesM, tilesN, (int)total);
  else
    hipLaunchKernelGGL((k_cgemm_b3<TAG, TNT, false>), dim3((unsigned)total), dim3(256), 0, s, sh, plan.d_tasks,
                       plan.d_segs, (const B3E *)A, (const B3E *)B, C, tilesM, tilesN, (int)total);
}
template <int TAG>
static void launch_b3(const GemmPlan &plan, const void *A, const void *B, cplx *C, hipStream_t s, int tn) {
  if (tn == 16) launch_b3t<TAG, 16>(plan, A, B, C, s);
  else if (tn == 32) launch_b3t<TAG, 32>(plan, A, B, C, s);
  else if (tn == 48) launch_b3t<TAG, 48>(plan, A, B, C, s);
  else launch_b3t<TAG, 64>(plan, A, B, C, s);  // (no 128-wide tile: it would spill)
}

template <int TAG, typename R, int TNT>
static void launch_t(const GemmPlan &plan, const void *A, const void *B, cplx *C, hipStream_t s) {
  const GemmShape &sh = plan.shape;
  const int tilesM = (sh.M + TM - 1) / TM, tilesN = (sh.N + TNT - 1) / TNT;
  const long long total = (long long)plan.ntask * tilesM * tilesN;
  hipLaunchKernelGGL((k_cgemm<TAG, R, TNT>), dim3((unsigned)total), dim3(256), 0, s, sh, plan.d_tasks, plan.d_segs,
                     (const typename Mf<R>::AE *)A, (const typename Mf<R>::AE *)B, C, tilesM, tilesN, (int)total);
}

template <int TAG, typename R>
static void launch_w(const GemmPlan &plan, const void *A, const void *B, cplx *C, hipStream_t s, int tn) {
  if (tn == 32) launch_t<TAG, R, 32>(plan, A, B, C, s);
  else if (tn == 128 && sizeof(R) == 4) launch_t<TAG, float, 128>(plan, A, B, C, s);
  else launch_t<TAG, R, 64>(plan, A, B, C, s);
}
// the big products also have 16- and 48-wide tiles (narrow batches)
template <int TAG, typename R>
static void launch_wn(const GemmPlan &plan, const void *A, const void *B, cplx *C, hipStream_t s, int tn) {
  if (tn == 16) launch_t<TAG, R, 16>(plan, A, B, C, s);
  else if (tn == 48) launch_t<TAG, R, 48>(plan, A, B, C, s);
  else launch_w<TAG, R>(plan, A, B, C, s, tn);
}

// prec 0: FP64 operands (A and B complex double); prec 1: FP32 (A complex float,
// B the vectors' complex float copy); prec 2: BF16-split products from the split
// operands (A and the vectors' split copy, four bf16 planes per element).  Tags 4 to 7 run in FP64 only.
// tn: N tile width (16, 32, 48, 64 or 128), chosen per plan in tuned_launch.
void gemm_launch(int tag, const GemmPlan &plan, const void *A, const void *B, cplx *C, hipStream_t s, int prec,
                 int tn) {
  const GemmShape &sh = plan.shape;
  if (plan.ntask == 0 || sh.M == 0 || sh.N == 0) return;
#define CASE(T)                                                                              \
  case T:                                                                                    \
    if (prec == 2) launch_b3<T>(plan, A, B, C, s, tn);                                       \
    else if (prec) launch_wn<T, float>(plan, A, B, C, s, tn);                                \
    else launch_wn<T, double>(plan, A, B, C, s, tn);                                         \
    break;
  switch (tag) {
    CASE(0) CASE(1) CASE(2) CASE(3) CASE(8) CASE(9)
    case 4:
      launch_wn<4, double>(plan, A, B, C, s, tn);
      break;
    case 6:
      launch_wn<6, double>(plan, A, B, C, s, tn);
      break;
    case 7:
      launch_wn<7, double>(plan, A, B, C, s, tn);
      break;
    default:
      launch_wn<5, double>(plan, A, B, C, s, tn);
  }
#undef CASE
}

// algorithmic flops of one launch (8 per complex multiply-add)
static double plan_flops(const GemmPlan &p) {
  return 8.0 * p.shape.M * (double)p.shape.N * p.shape.K * (double)p.segs.size();
}
// algorithmic HBM bytes of one launch: every segment's A block once (complex double, or
// 8 bytes per element in the reduced-precision forms), the vectors' operand copy once
// (nx elements) and every task's output block written once (complex double)
static double plan_bytes(const GemmPlan &p, double nx, int prec) {
  const double ea = prec ? 8.0 : 16.0;
  return ea * ((double)p.segs.size() * p.shape.M * p.shape.K + nx) + 16.0 * (double)p.ntask * p.shape.M * p.shape.N;
}

// k pairs (2k, 2k + 1) adjacent under an index map with even offsets for even k
static bool map_pairs(const IdxMap &m, int ext) {
  if (m.s1 != 1) return false;
  return m.L >= ext || (m.L % 2 == 0 && m.s0 % 2 == 0);
}
// every offset of an index map even
static bool offs_even(const IdxMap &m, int ext) { return m.s1 % 2 == 0 && (m.L >= ext || m.s0 % 2 == 0); }

void plan_upload(ccgf_ctx *c, GemmPlan &p) {
  {  // can the BF16-split GEMM stage this plan's operands two k at a time (16-byte aligned pairs)?
    const GemmShape &sh = p.shape;
    bool ok = !sh.ktab && !sh.mtab && sh.K % 2 == 0 && map_pairs(sh.ak, sh.K) && map_pairs(sh.bk, sh.K) &&
              offs_even(sh.am, sh.M) && offs_even(sh.bn, sh.N);
    for (const GemmSeg &g : p.segs) ok = ok && g.a_off % 2 == 0 && g.b_off % 2 == 0;
    p.pairs = ok;
  }
  p.ntask = (int)p.tasks.size();
  p.d_tasks = (GemmTask *)dev_alloc(c, sizeof(GemmTask) * std::max<size_t>(1, p.tasks.size()));
  p.d_segs = (GemmSeg *)dev_alloc(c, sizeof(GemmSeg) * std::max<size_t>(1, p.segs.size()));
  if (!p.d_tasks || !p.d_segs) return;
  hipMemcpy(p.d_tasks, p.tasks.data(), sizeof(GemmTask) * p.tasks.size(), hipMemcpyHostToDevice);
  hipMemcpy(p.d_segs, p.segs.data(), sizeof(GemmSeg) * p.segs.size(), hipMemcpyHostToDevice);
}

static IdxMap one(long long s) { return IdxMap{1 << 30, 0, s}; }
static IdxMap two(int L, long long s0, long long s1) { return IdxMap{L, s0, s1}; }

static int host_c3(const ccgf_ctx *c, int a, int b, int d) { return c->kc3_h[((size_t)a * c->nk + b) * c->nk + d]; }

static void build_plans(ccgf_ctx *c, SigmaPlan &P) {
  const int nk = c->nk, no = c->no, nv = c->nv, K = P.K, nvec = P.nvec;
  const long long n = P.n;
  if (P.part == CCGF_PART_EA) {
    const long long b2 = (long long)no * nv * nv;
    // 1/2 W_abcd r_i^cd:  C(ab ; i,v) over segments kc
    GemmPlan &g = P.g_big;
    g.shape.M = nv * nv;
    g.shape.N = no * nvec;
    g.shape.K = nv * nv;
    g.shape.am = one((long long)nv * nv);
    g.shape.ak = one(1);
    g.shape.bk = one(1);
    g.shape.bn = two(no, n, (long long)nv * nv);
    g.shape.cm = one(1);
    g.shape.cn = two(no, n, (long long)nv * nv);
    g.shape.alpha_re = 1.0;
    g.shape.alpha_im = 0;
    g.shape.accumulate = 0;
    // W and r are antisymmetric in (c,kc) <-> (d,kd), so segments kc and kd = ka + kb - kc
    // contribute alike: one of each pair at weight 1 (a self-paired segment at 1/2).  The
    // output blocks (ki, ka) and (ki, kb) are negative transposes of each other: only
    // ka <= kb is computed, the other block is filled afterwards.  A block ka = kb is itself
    // antisymmetric in (a, b): its rows a < b are computed (g_bigt, g_bigd) and the rest filled,
    // and its self-paired segments kc = kd (there is always kc = ka) run over c < d only.
    // W blocks (ka <= kb, kc <= kd) are the stored ones
    const long long nv4 = (long long)nv * nv * nv * nv;
    auto wblk = [&](int ka, int kb, int kc) -> long long {
      return (long long)c->wblk_h[((size_t)ka * nk + kb) * nk + kc] * nv4;
    };
    std::vector<long long> fill;
    GemmPlan &gt = P.g_bigt, &gd = P.g_bigd;
    const int np = nv * (nv - 1) / 2;
    gt.shape = g.shape;
    gt.shape.M = np;
    gt.shape.K = np;
    gt.m_ext = gt.k_ext = nv * nv;
    gd.shape = g.shape;
    gd.shape.M = np;
    gd.shape.accumulate = 1;  // after g_bigt, which writes every block ka = kb
    gd.m_ext = nv * nv;
    for (int ki = 0; ki < nk; ++ki)
      for (int ka = 0; ka < nk; ++ka) {
        int kb = host_c3(c, K, ki, ka);
        const long long cblk = nv + (ki * nk + ka) * b2;
        if (ka > kb) {
          fill.push_back(cblk);
          fill.push_back(nv + (ki * nk + kb) * b2);
          continue;
        }
        if (ka == kb) {
          fill.push_back(cblk);
          fill.push_back(cblk);
          GemmTask tt{cblk, (int)gt.segs.size(), 0}, td{cblk, (int)gd.segs.size(), 0};
          for (int kc = 0; kc < nk; ++kc) {
            const int kd = host_c3(c, ka, kb, kc);
            if (kc > kd) continue;
            GemmSeg sg{wblk(ka, kb, kc), nv + (ki * nk + kc) * b2, 1.0};
            if (kc == kd) gt.segs.push_back(sg), ++tt.nseg;
            else gd.segs.push_back(sg), ++td.nseg;
          }
          gt.tasks.push_back(tt);
          if (td.nseg) gd.tasks.push_back(td);
          continue;
        }
        GemmTask t{cblk, (int)g.segs.size(), 0};
        for (int kc = 0; kc < nk; ++kc) {
          const int kd = host_c3(c, ka, kb, kc);
          if (kc > kd) continue;
          g.segs.push_back(GemmSeg{wblk(ka, kb, kc), nv + (ki * nk + kc) * b2, kc == kd ? 0.5 : 1.0});
          ++t.nseg;
        }
        g.tasks.push_back(t);
      }
    // heaviest tasks first: the last blocks of the grid then finish together
    std::stable_sort(g.tasks.begin(), g.tasks.end(),
                     [](const GemmTask &x, const GemmTask &y) { return x.nseg > y.nseg; });
    if (np > 0) {
      std::vector<int> tri;
      for (int a = 0; a < nv; ++a)
        for (int b = a + 1; b < nv; ++b) tri.push_back(a * nv + b);
      P.d_tri = (int *)dev_alloc(c, sizeof(int) * tri.size());
      if (P.d_tri) hipMemcpy(P.d_tri, tri.data(), sizeof(int) * tri.size(), hipMemcpyHostToDevice);
      gt.shape.mtab = gt.shape.ktab = gd.shape.mtab = P.d_tri;
    } else {
      gt.tasks.clear();
      gd.tasks.clear();
    }
    P.nfill = (int)fill.size() / 2;
    if (P.nfill > 0) {
      std::vector<long long> &h = P.fill_h;
      h.resize(2 * P.nfill);
      for (int q = 0; q < P.nfill; ++q) h[q] = fill[2 * q], h[P.nfill + q] = fill[2 * q + 1];
      P.d_fill = (long long *)dev_alloc(c, sizeof(long long) * h.size());
      if (P.d_fill) hipMemcpy(P.d_fill, h.data(), sizeof(long long) * h.size(), hipMemcpyHostToDevice);
    }
    // P(ab) (W_lbdi r_l^ad + F_bd r_i^ad) without the antisymmetriser: X(b,i ; a,v) over segments kl
    // (the operand is W_ovvo with F_vv folded into its blocks kl = ki, l = i)
    GemmPlan &h = P.g_ovvo;
    h.shape.M = nv * no;
    h.shape.N = nv * nvec;
    h.shape.K = no * nv;
    h.shape.am = one((long long)no * nv);
    h.shape.ak = one(1);
    h.shape.bk = two(nv, (long long)nv * nv, 1);
    h.shape.bn = two(nv, n, nv);
    h.shape.cm = two(no, 1, (long long)nv * nv);
    h.shape.cn = two(nv, n, nv);
    h.shape.alpha_re = 1;
    h.shape.alpha_im = 0;
    h.shape.accumulate = 0;
    T4 Wp{nullptr, nk, nv, no, no, nv};
    for (int ki = 0; ki < nk; ++ki)
      for (int ka = 0; ka < nk; ++ka) {
        int kb = host_c3(c, K, ki, ka);
        GemmTask t{nv + (ki * nk + ka) * b2, (int)h.segs.size(), nk};
        for (int kl = 0; kl < nk; ++kl)
          h.segs.push_back(GemmSeg{(long long)Wp.blk(kb, ki, kl), nv + (kl * nk + ka) * b2});
        h.tasks.push_back(t);
      }
  } else {
    const long long b2 = (long long)no * no * nv;
    // 1/2 W_mnij r_mn^a:  C(ij ; a,v) over segments km
    GemmPlan &g = P.g_big;
    g.shape.M = no * no;
    g.shape.N = nv * nvec;
    g.shape.K = no * no;
    g.shape.am = one((long long)no * no);
    g.shape.ak = one(1);
    g.shape.bk = one(nv);
    g.shape.bn = two(nv, n, 1);
    g.shape.cm = one(nv);
    g.shape.cn = two(nv, n, 1);
    g.shape.alpha_re = 0.5;
    g.shape.alpha_im = 0;
    g.shape.accumulate = 0;
    T4 W{nullptr, nk, no, no, no, no};
    for (int ki = 0; ki < nk; ++ki)
      for (int kj = 0; kj < nk; ++kj) {
        GemmTask t{no + (ki * nk + kj) * b2, (int)g.segs.size(), nk};
        for (int km = 0; km < nk; ++km) {
          int kn = host_c3(c, ki, kj, km);
          g.segs.push_back(GemmSeg{(long long)W.blk(ki, kj, km), no + (km * nk + kn) * b2});
        }
        g.tasks.push_back(t);
      }
    // P(ij) W_maei r_mj^e (without the antisymmetriser): X(a,i ; j,v) over segments km
    GemmPlan &h = P.g_ovvo;
    h.shape.M = nv * no;
    h.shape.N = no * nvec;
    h.shape.K = no * nv;
    h.shape.am = one((long long)no * nv);
    h.shape.ak = one(1);
    h.shape.bk = two(nv, (long long)no * nv, 1);
    h.shape.bn = two(no, n, nv);
    h.shape.cm = two(no, 1, (long long)no * nv);
    h.shape.cn = two(no, n, nv);
    h.shape.alpha_re = 1;
    h.shape.alpha_im = 0;
    h.shape.accumulate = 0;
    T4 Wp{nullptr, nk, nv, no, no, nv};
    for (int ki = 0; ki < nk; ++ki)
      for (int kj = 0; kj < nk; ++kj) {
        int ka = host_c3(c, ki, kj, K);
        GemmTask t{no + (ki * nk + kj) * b2, (int)h.segs.size(), nk};
        for (int km = 0; km < nk; ++km)
          h.segs.push_back(GemmSeg{(long long)Wp.blk(ka, ki, km), no + (km * nk + kj) * b2});
        h.tasks.push_back(t);
      }
  }
  // coupling of the one-quasiparticle part into the three-quasiparticle part
  GemmPlan &q = P.g_r1;
  if (P.part == CCGF_PART_EA) {
    // sigma2[ki][ka](i,a,b) += sum_e W_abei r^e : C(ab,i ; v) = sum_e A(ab,i ; e) r1(e ; v)
    const long long b2 = (long long)no * nv * nv;
    q.shape.M = nv * nv * no;
    q.shape.N = nvec;
    q.shape.K = nv;
    q.shape.am = two(no, (long long)nv * no, 1);
    q.shape.ak = one(no);
    q.shape.bk = one(1);
    q.shape.bn = one(n);
    q.shape.cm = two(no, 1, (long long)nv * nv);
    q.shape.cn = one(n);
    q.shape.alpha_re = 1;
    q.shape.alpha_im = 0;
    q.shape.accumulate = 1;
    T4 Wt{nullptr, nk, nv, nv, nv, no};
    for (int ki = 0; ki < nk; ++ki)
      for (int ka = 0; ka < nk; ++ka) {
        int kb = host_c3(c, K, ki, ka);
        q.tasks.push_back(GemmTask{nv + (ki * nk + ka) * b2, (int)q.segs.size(), 1});
        q.segs.push_back(GemmSeg{(long long)Wt.blk(ka, kb, K), 0});
      }
  } else {
    // sigma2[ki][kj](i,j,a) -= sum_m W_maij r_m : C(ij,a ; v) = -sum_m A(ij,a ; m) r1(m ; v)
    const long long b2 = (long long)no * no * nv;
    q.shape.M = no * no * nv;
    q.shape.N = nvec;
    q.shape.K = no;
    q.shape.am = two(nv, 1, (long long)no * no);
    q.shape.ak = one((long long)nv * no * no);
    q.shape.bk = one(1);
    q.shape.bn = one(n);
    q.shape.cm = one(1);
    q.shape.cn = one(n);
    q.shape.alpha_re = -1;
    q.shape.alpha_im = 0;
    q.shape.accumulate = 1;
    T4 Wt{nullptr, nk, no, nv, no, no};
    for (int ki = 0; ki < nk; ++ki)
      for (int kj = 0; kj < nk; ++kj) {
        int ka = host_c3(c, ki, kj, K);
        q.tasks.push_back(GemmTask{no + (ki * nk + kj) * b2, (int)q.segs.size(), 1});
        q.segs.push_back(GemmSeg{(long long)Wt.blk(K, ka, ki), 0});
      }
  }
  // 1p / 1h rows of sigma and the three-body intermediate: long contractions over
  // the whole r2 vector, split over its momentum blocks and the first occupied
  // index (one task each, enough blocks to fill the chip) into partial sums
  // part[z][row][v] that k_r1_finish adds up.
  {
    const int nrow = no + nv;
    GemmPlan &u = P.g_red1, &w = P.g_red2;
    if (P.part == CCGF_PART_EA) {
      const long long b2 = (long long)no * nv * nv, kl2 = (long long)nv * nv;
      // rows a: 1/2 W_alcd r_l^cd, A = Wvovv[K][kl][kc](a,l,c,d), chunk l
      u.shape.M = nv;
      u.shape.K = (int)kl2;
      u.shape.am = one(b2);
      u.shape.ak = one(1);
      u.shape.alpha_re = 0.5;
      // rows k: <kl||cd> r_l^cd, A = Voovv[K][kl][kc](k,l,c,d), chunk l
      w.shape.M = no;
      w.shape.K = (int)kl2;
      w.shape.am = one(b2);
      w.shape.ak = one(1);
      w.shape.alpha_re = 1;
      T4 Wa{nullptr, nk, nv, no, nv, nv}, Va{nullptr, nk, no, no, nv, nv};
      for (int kl = 0; kl < nk; ++kl)
        for (int kc = 0; kc < nk; ++kc)
          for (int l = 0; l < no; ++l) {
            const long long z = ((long long)kl * nk + kc) * no + l, boff = nv + (kl * nk + kc) * b2 + l * kl2;
            u.tasks.push_back(GemmTask{z * nrow * nvec, (int)u.segs.size(), 1});
            u.segs.push_back(GemmSeg{(long long)Wa.blk(K, kl, kc) + l * kl2, boff});
            w.tasks.push_back(GemmTask{(z * nrow + nv) * nvec, (int)w.segs.size(), 1});
            w.segs.push_back(GemmSeg{(long long)Va.blk(K, kl, kc) + l * kl2, boff});
          }
    } else {
      const long long b2 = (long long)no * no * nv, km2 = (long long)no * nv;
      // rows i: -1/2 W_mnie r_mn^e, A = Wooov[km][kn][K](m,n,i,e), chunk m
      u.shape.M = no;
      u.shape.K = (int)km2;
      u.shape.am = one(nv);
      u.shape.ak = two(nv, (long long)no * nv, 1);
      u.shape.alpha_re = -0.5;
      // rows e: <mn||ef> r_mn^f, A = Voovv[km][kn][K](m,n,e,f), chunk m
      w.shape.M = nv;
      w.shape.K = (int)km2;
      w.shape.am = one(nv);
      w.shape.ak = two(nv, (long long)nv * nv, 1);
      w.shape.alpha_re = 1;
      T4 Wa{nullptr, nk, no, no, no, nv}, Va{nullptr, nk, no, no, nv, nv};
      for (int km = 0; km < nk; ++km)
        for (int kn = 0; kn < nk; ++kn)
          for (int mm = 0; mm < no; ++mm) {
            const long long z = ((long long)km * nk + kn) * no + mm, boff = no + (km * nk + kn) * b2 + mm * km2;
            u.tasks.push_back(GemmTask{z * nrow * nvec, (int)u.segs.size(), 1});
            u.segs.push_back(GemmSeg{(long long)Wa.blk(km, kn, K) + mm * (long long)no * no * nv, boff});
            w.tasks.push_back(GemmTask{(z * nrow + no) * nvec, (int)w.segs.size(), 1});
            w.segs.push_back(GemmSeg{(long long)Va.blk(km, kn, K) + mm * (long long)no * nv * nv, boff});
          }
    }
    for (GemmPlan *g : {&u, &w}) {
      g->shape.N = nvec;
      g->shape.bk = one(1);
      g->shape.bn = one(n);
      g->shape.cm = one(nvec);
      g->shape.cn = one(1);
      g->shape.alpha_im = 0;
      g->shape.accumulate = 0;
    }
  }
  plan_upload(c, P.g_big);
  plan_upload(c, P.g_bigt);
  plan_upload(c, P.g_bigd);
  plan_upload(c, P.g_ovvo);
  plan_upload(c, P.g_r1);
  plan_upload(c, P.g_red1);
  plan_upload(c, P.g_red2);
  P.ready = true;
}

// Largest offset an index map reaches for x in [0, len).
static long long map_max(const IdxMap &m, int len) {
  if (len <= 0) return 0;
  long long hi = (long long)((len - 1) / m.L) * m.s0;
  long long lo = (long long)std::min(len - 1, m.L - 1) * m.s1;
  return hi + lo;
}

// Host-side proof that every access of a plan stays inside its buffers.
static bool plan_in_bounds(const GemmPlan &p, size_t a_elems, size_t b_elems, size_t c_elems) {
  const GemmShape &s = p.shape;
  const int me = s.mtab ? p.m_ext : s.M, ke = s.ktab ? p.k_ext : s.K;  // tables hold indices below the ext
  long long am = map_max(s.am, me) + map_max(s.ak, ke);
  long long bm = map_max(s.bk, ke) + map_max(s.bn, s.N);
  long long cm = map_max(s.cm, me) + map_max(s.cn, s.N);
  for (const GemmTask &t : p.tasks) {
    if (t.c_off < 0 || (size_t)(t.c_off + cm) >= c_elems) return false;
    if (t.seg_begin < 0 || (size_t)(t.seg_begin + t.nseg) > p.segs.size()) return false;
  }
  for (const GemmSeg &g : p.segs) {
    if (g.a_off < 0 || (size_t)(g.a_off + am) >= a_elems) return false;
    if (g.b_off < 0 || (size_t)(g.b_off + bm) >= b_elems) return false;
  }
  return true;
}

// ------------------------------------------------------------------ reductions
__device__ inline double wsum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// One wave per (row, vector): add the split-K partial sums of the reduction GEMMs
// and, for the rows of sigma1, the Fock terms; rows >= n1 are the three-body
// intermediate, written to aux.
//   EA, row a:  F_ac r^c + F_ld r_l^ad            (r2 block [kl][K], kd = kl)
//   IP, row i: -F_mi r_m + F_me r_im^e            (r2 block [K][km], ke = km)
__global__ __launch_bounds__(256) void k_r1_finish(int ea, int nk, int no, int nv, int K, int nrow, int n1,
                                                   int nvec, int nz, long long n, const cplx *__restrict__ part,
                                                   const cplx *__restrict__ x, cplx *__restrict__ y,
                                                   cplx *__restrict__ aux, int ldaux, const cplx *__restrict__ Foo,
                                                   const cplx *__restrict__ Fvv, const cplx *__restrict__ Fov) {
  const int t = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (t >= nrow * nvec) return;  // whole waves leave together
  const int row = t / nvec, v = t % nvec;
  cplx acc = mkc(0, 0);
  for (int zz = lane; zz < nz; zz += 64) acc = cadd(acc, part[((size_t)zz * nrow + row) * nvec + v]);
  if (row < n1) {
    const cplx *xv = x + (size_t)v * n;
    const int nf = nk * no * nv;
    if (ea) {
      const int a = row;
      const long long b2 = (long long)no * nv * nv;
      for (int c3 = lane; c3 < nv; c3 += 64) cfma(acc, Fvv[((size_t)K * nv + a) * nv + c3], xv[c3]);
      for (int w = lane; w < nf; w += 64) {
        const int kl = w / (no * nv), l = (w / nv) % no, d = w % nv;
        cfma(acc, Fov[((size_t)kl * no + l) * nv + d], xv[nv + (kl * nk + K) * b2 + ((size_t)l * nv + a) * nv + d]);
      }
    } else {
      const int i = row;
      const long long b2 = (long long)no * no * nv;
      for (int m = lane; m < no; m += 64) acc = csub(acc, cmul(Foo[((size_t)K * no + m) * no + i], xv[m]));
      for (int w = lane; w < nf; w += 64) {
        const int km = w / (no * nv), m = (w / nv) % no, e = w % nv;
        cfma(acc, Fov[((size_t)km * no + m) * nv + e], xv[no + (K * nk + km) * b2 + ((size_t)i * no + m) * nv + e]);
      }
    }
  }
  const double re = wsum(acc.x), im = wsum(acc.y);
  if (lane == 0) {
    if (row < n1) y[(size_t)v * n + row] = mkc(re, im);
    else aux[(size_t)v * ldaux + (row - n1)] = mkc(re, im);
  }
}

// EA blocks of the W_abcd product left to antisymmetry: y[dst](i,a,b) = -y[src](i,b,a);
// for dst = src only the rows a >= b are written (a = b: zero)
__global__ void k_vvvv_fill(cplx *__restrict__ y, long long n, int nvec, int nv, long long b2,
                            const long long *__restrict__ dst, const long long *__restrict__ src, int nfill) {
  const int f = blockIdx.y;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= b2) return;
  const int b = (int)(e % nv), a = (int)((e / nv) % nv), i = (int)(e / ((long long)nv * nv));
  const long long t = ((long long)i * nv + b) * nv + a;
  const bool self = dst[f] == src[f];  // a block ka = kb: rows a < b are computed, a = b vanish
  if (self && a < b) return;
  for (int v = blockIdx.z; v < nvec; v += gridDim.z) {
    cplx x = a == b && self ? mkc(0, 0) : y[(size_t)v * n + src[f] + t];
    y[(size_t)v * n + dst[f] + e] = mkc(-x.x, -x.y);
  }
}

// element-wise EA 2p1h terms: one thread per sigma2 element, vectors over grid y
__global__ __launch_bounds__(256) void k_ea_local(int nk, int no, int nv, int K, int nvec, long long n,
                                                  const int *__restrict__ kc3, const cplx *__restrict__ x,
                                                  cplx *__restrict__ y, const cplx *__restrict__ X,
                                                  const cplx *__restrict__ aux, const cplx *__restrict__ Foo,
                                                  const cplx *__restrict__ Fvv, const cplx *__restrict__ t2) {
  const long long b2 = (long long)no * nv * nv;
  const long long n2 = (long long)nk * nk * b2;
  const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= n2) return;
  const long long blk = z / b2, w = z % b2;
  const int ki = (int)(blk / nk), ka = (int)(blk % nk);
  const int b = (int)(w % nv), a = (int)((w / nv) % nv), i = (int)(w / ((long long)nv * nv));
  const int kb = kc3[(K * nk + ki) * nk + ka];
  const size_t oab = (size_t)(ki * nk + ka) * b2, oba = (size_t)(ki * nk + kb) * b2;
  const cplx *T = t2 + (((size_t)K * nk + ki) * nk + ka) * (size_t)(no * no * nv * nv);
  const int ldaux = no > nv ? no : nv;
  for (int v = blockIdx.y; v < nvec; v += gridDim.y) {
    const cplx *r2 = x + (size_t)v * n + nv;
    cplx acc = y[(size_t)v * n + nv + z];
    // - F_li r_l^ab
    for (int l = 0; l < no; ++l)
      acc = csub(acc, cmul(Foo[((size_t)ki * no + l) * no + i], r2[oab + ((size_t)l * nv + a) * nv + b]));
    // P(ab) (W_lbdi r_l^ad + F_bd r_i^ad) from the GEMM scratch (F folded into its operand)
    const cplx *Xv = X + (size_t)v * n + nv;
    acc = cadd(acc, Xv[oab + ((size_t)i * nv + a) * nv + b]);
    acc = csub(acc, Xv[oba + ((size_t)i * nv + b) * nv + a]);
    // three-body: - 1/2 sum_k Y_k t_ki^ab, t2 block [K][ki][ka]
    cplx h = mkc(0, 0);
    for (int k = 0; k < no; ++k) cfma(h, aux[(size_t)v * ldaux + k], T[(((size_t)k * no + i) * nv + a) * nv + b]);
    acc = csub(acc, cscale(h, 0.5));
    y[(size_t)v * n + nv + z] = acc;
  }
}

// ------------------------------------------------------------------ IP
// element-wise IP 2h1p terms: one thread per sigma2 element, vectors over grid y
__global__ __launch_bounds__(256) void k_ip_local(int nk, int no, int nv, int K, int nvec, long long n,
                                                  const int *__restrict__ kc3, const cplx *__restrict__ x,
                                                  cplx *__restrict__ y, const cplx *__restrict__ X,
                                                  const cplx *__restrict__ aux, const cplx *__restrict__ Foo,
                                                  const cplx *__restrict__ Fvv, const cplx *__restrict__ t2) {
  const long long b2 = (long long)no * no * nv;
  const long long n2 = (long long)nk * nk * b2;
  const long long z = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (z >= n2) return;
  const long long blk = z / b2, w = z % b2;
  const int ki = (int)(blk / nk), kj = (int)(blk % nk);
  const int a = (int)(w % nv), j = (int)((w / nv) % no), i = (int)(w / ((long long)nv * no));
  const int ka = kc3[(ki * nk + kj) * nk + K];
  const size_t oij = (size_t)(ki * nk + kj) * b2, oji = (size_t)(kj * nk + ki) * b2;
  const cplx *Fa = Fvv + ((size_t)ka * nv + a) * nv;
  const cplx *T = t2 + (((size_t)ki * nk + kj) * nk + ka) * (size_t)(no * no * nv * nv) +
                  (((size_t)i * no + j) * nv + a) * nv;
  const int ldaux = no > nv ? no : nv;
  for (int v = blockIdx.y; v < nvec; v += gridDim.y) {
    const cplx *r2 = x + (size_t)v * n + no;
    cplx acc = y[(size_t)v * n + no + z];
    // F_ae r_ij^e
    const cplx *rij = r2 + oij + ((size_t)i * no + j) * nv;
    for (int e = 0; e < nv; ++e) cfma(acc, Fa[e], rij[e]);
    // - P(ij) F_mi r_mj^a
    for (int m = 0; m < no; ++m) {
      acc = csub(acc, cmul(Foo[((size_t)ki * no + m) * no + i], r2[oij + ((size_t)m * no + j) * nv + a]));
      cfma(acc, Foo[((size_t)kj * no + m) * no + j], r2[oji + ((size_t)m * no + i) * nv + a]);
    }
    // P(ij) W_maei r_mj^e from the GEMM scratch
    const cplx *Xv = X + (size_t)v * n + no;
    acc = cadd(acc, Xv[oij + ((size_t)i * no + j) * nv + a]);
    acc = csub(acc, Xv[oji + ((size_t)j * no + i) * nv + a]);
    // three-body: + 1/2 sum_e Xe_e t_ij^ae, t2 block [ki][kj][ka] (ke = K)
    cplx h = mkc(0, 0);
    for (int e = 0; e < nv; ++e) cfma(h, aux[(size_t)v * ldaux + e], T[e]);
    acc = cadd(acc, cscale(h, 0.5));
    y[(size_t)v * n + no + z] = acc;
  }
}

// Launch a plan with the N tile width the autotuner picked for its shape.  Products of
// narrow batches (N <= 48) take the narrowest tile that holds N without trials.  Otherwise the first two launches of an unseen shape are timed trials of the 64- and 32-wide
// variants (each does the real work); the 32-wide one is kept only if it is at
// least 5% faster.  Choices are cached per shape in the context (and in the
// autotune file when one is configured).
static int tuned_launch(ccgf_ctx *c, int tag, GemmPlan &p, const void *A, const void *B, cplx *C, hipStream_t s,
                        int prec) {
  if (p.tn[prec] == 0 && c->opt.autotune < 0) p.tn[prec] = 64;
  // narrow batches (N <= 48): the narrowest tile that holds N, where the MFMA work is least
  // padding (the A operand is streamed once either way); for the couplings and split-K rows
  // N is the number of vectors itself
  if (p.tn[prec] == 0 && p.shape.N <= 48) p.tn[prec] = 16 * ((p.shape.N + 15) / 16);
  if (p.tn[prec] == 0) {
    char key[160];
    std::snprintf(key, sizeof key, "t%d p%d M%d N%d K%d s%zu n%d", tag, prec, p.shape.M, p.shape.N, p.shape.K,
                  p.segs.size(), p.ntask);
    auto it = c->tuned.find(key);
    if (it != c->tuned.end()) {
      p.tn[prec] = it->second;
    } else {
      if (!c->tev[0])
        for (int q = 0; q < 2; ++q)
          if (hipEventCreate(&c->tev[q]) != hipSuccess) return hip_check(c, hipGetLastError(), "autotune events");
      int &tr = p.trials[prec];
      static const int cands[3] = {64, 32, 128};  // 128 only for the FP32 GEMMs
      const int ncand = prec == 1 ? 3 : 2;
      const int cand = cands[tr];
      hipEventRecord(c->tev[0], s);
      gemm_launch(tag, p, A, B, C, s, prec, cand);
      hipEventRecord(c->tev[1], s);
      if (hipEventSynchronize(c->tev[1]) == hipSuccess) hipEventElapsedTime(&p.tms[prec][tr], c->tev[0], c->tev[1]);
      if (++tr == ncand) {  // a narrower or wider tile only where it is 5% faster than 64
        int best = 0;
        for (int q = 1; q < ncand; ++q)
          if (p.tms[prec][q] < 0.95f * p.tms[prec][best]) best = q;
        p.tn[prec] = cands[best];
        c->tuned[key] = p.tn[prec];
      }
      return CCGF_OK;
    }
  }
  gemm_launch(tag, p, A, B, C, s, prec, p.tn[prec]);
  return CCGF_OK;
}

void tune_load(ccgf_ctx *c) {
  if (c->tune_path.empty()) return;
  FILE *f = std::fopen(c->tune_path.c_str(), "r");
  if (!f) return;
  char line[256];
  while (std::fgets(line, sizeof line, f)) {
    char *sp = std::strrchr(line, ' ');
    if (!sp) continue;
    int tn = std::atoi(sp + 1);
    if (tn != 32 && tn != 64 && tn != 128) continue;
    c->tuned[std::string(line, sp - line)] = tn;
  }
  std::fclose(f);
}

void tune_save(const ccgf_ctx *c) {
  if (c->tune_path.empty() || c->tuned.empty()) return;
  FILE *f = std::fopen(c->tune_path.c_str(), "w");
  if (!f) return;
  for (const auto &kv : c->tuned) std::fprintf(f, "%s %d\n", kv.first.c_str(), kv.second);
  std::fclose(f);
}

__global__ void k_to_f32(const cplx *__restrict__ x, float2 *__restrict__ y, size_t tot) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < tot) y[i] = float2{(float)x[i].x, (float)x[i].y};
}

// the split copy of the vectors for the BF16-split products
__global__ void k_to_b3(const cplx *__restrict__ x, B3E *__restrict__ y, size_t tot) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= tot) return;
  B3E e;
  split_bf(x[i].x, e.rh, e.rl);
  split_bf(x[i].y, e.ih, e.il);
  y[i] = e;
}

// The launches of one sigma product on stream s (event records only when ts is set).
static int sigma_enqueue(ccgf_ctx *c, SigmaPlan *P, int part, int K, int nvec, const cplx *x, cplx *y, int prec,
                         hipStream_t s, ccgf_ctx::TimedSigma *ts) {
  const int nk = c->nk, no = c->no, nv = c->nv;
  const long long n = P->n;
  const unsigned gy = (unsigned)std::min(nvec, 65535);
  // the reduced-precision GEMMs read the vectors through one complex float copy
  const void *xb = x;
  if (prec) {
    const size_t tot = (size_t)nvec * n;
    if (prec == 2)  // (the split copy has the complex float copy's size: four bf16 per element)
      hipLaunchKernelGGL(k_to_b3, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x, (B3E *)c->sig_x32, tot);
    else
      hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, x, c->sig_x32, tot);
    xb = c->sig_x32;
  }
  // fork: the side stream takes the terms that write other buffers than the big product's
  // blocks (the diagonal W_abcd blocks, the W_ovvo scratch, the split-K partial sums), so that
  // their small, HBM-bound launches overlap the big one; join before the terms that read them
  hipStream_t s2 = c->side_stream;
  hipEventRecord(c->ev_fork, s);
  hipStreamWaitEvent(s2, c->ev_fork, 0);
  if (part == CCGF_PART_EA) {
    if (prec && !c->Wvvvv32) return set_err(c, CCGF_ESTATE, "mixed-precision operands were not built");
    const void *Wbig = prec ? (const void *)c->Wvvvv32 : (const void *)c->Wvvvv;
    const void *Wovvo = prec ? (const void *)c->WvoPea32 : (const void *)c->WvoPea;
    int rc = CCGF_OK;
    if (!rc && P->g_bigt.ntask) rc = tuned_launch(c, 8, P->g_bigt, Wbig, xb, y, s2, prec);
    if (!rc && P->g_bigd.ntask) rc = tuned_launch(c, 9, P->g_bigd, Wbig, xb, y, s2, prec);
    if (!rc) rc = tuned_launch(c, 1, P->g_ovvo, Wovvo, xb, c->sig_tmp, s2, prec);
    if (!rc) rc = tuned_launch(c, 6, P->g_red1, c->Wvovv, x, c->sig_part, s2, 0);
    if (!rc) rc = tuned_launch(c, 6, P->g_red2, c->Voovv, x, c->sig_part, s2, 0);
    hipEventRecord(c->ev_join, s2);
    if (ts) hipEventRecord(ts->e[2], s);
    if (!rc) rc = tuned_launch(c, 0, P->g_big, Wbig, xb, y, s, prec);
    if (ts) hipEventRecord(ts->e[3], s);
    hipStreamWaitEvent(s, c->ev_join, 0);
    if (P->nfill > 0) {
      const long long b2 = (long long)no * nv * nv;
      hipLaunchKernelGGL(k_vvvv_fill, dim3((unsigned)((b2 + 255) / 256), P->nfill, std::min(nvec, 64)), dim3(256), 0,
                         s, y, n, nvec, nv, b2, P->d_fill, P->d_fill + P->nfill, P->nfill);
    }
    if (!rc) rc = tuned_launch(c, 4, P->g_r1, c->Wvvvo, x, y, s, 0);
    if (rc) return rc;
    hipLaunchKernelGGL(k_r1_finish, dim3((unsigned)(((nv + no) * nvec + 3) / 4)), dim3(256), 0, s, 1, nk, no, nv, K,
                       nv + no, nv, nvec, nk * nk * no, n, c->sig_part, x, y, c->sig_r1aux, std::max(no, nv), c->Foo,
                       c->Fvv, c->Fov);
    long long tot = (long long)nk * nk * no * nv * nv;
    hipLaunchKernelGGL(k_ea_local, dim3((unsigned)((tot + 255) / 256), gy), dim3(256), 0, s, nk, no, nv, K, nvec, n,
                       c->kc3, x, y, c->sig_tmp, c->sig_r1aux, c->Foo, c->Fvv, c->t2);
  } else {
    if (prec && !c->WooP32) return set_err(c, CCGF_ESTATE, "mixed-precision operands were not built");
    const void *Wbig = prec ? (const void *)c->WooP32 : (const void *)c->WooP;
    const void *Wovvo = prec ? (const void *)c->WvoP32 : (const void *)c->WvoP;
    int rc = tuned_launch(c, 3, P->g_ovvo, Wovvo, xb, c->sig_tmp, s2, prec);
    if (!rc) rc = tuned_launch(c, 7, P->g_red1, c->Wooov, x, c->sig_part, s2, 0);
    if (!rc) rc = tuned_launch(c, 7, P->g_red2, c->Voovv, x, c->sig_part, s2, 0);
    hipEventRecord(c->ev_join, s2);
    if (ts) hipEventRecord(ts->e[2], s);
    if (!rc) rc = tuned_launch(c, 2, P->g_big, Wbig, xb, y, s, prec);
    if (ts) hipEventRecord(ts->e[3], s);
    hipStreamWaitEvent(s, c->ev_join, 0);
    if (!rc) rc = tuned_launch(c, 5, P->g_r1, c->Wovoo, x, y, s, 0);
    if (rc) return rc;
    hipLaunchKernelGGL(k_r1_finish, dim3((unsigned)(((nv + no) * nvec + 3) / 4)), dim3(256), 0, s, 0, nk, no, nv, K,
                       no + nv, no, nvec, nk * nk * no, n, c->sig_part, x, y, c->sig_r1aux, std::max(no, nv), c->Foo,
                       c->Fvv, c->Fov);
    long long tot = (long long)nk * nk * no * no * nv;
    hipLaunchKernelGGL(k_ip_local, dim3((unsigned)((tot + 255) / 256), gy), dim3(256), 0, s, nk, no, nv, K, nvec, n,
                       c->kc3, x, y, c->sig_tmp, c->sig_r1aux, c->Foo, c->Fvv, c->t2);
  }
  return CCGF_OK;
}

// Captured graphs hold the workspace addresses: drop them all before a workspace moves.
static void drop_graphs(ccgf_ctx *c) {
  hipStreamSynchronize(c->stream);
  for (auto &P : c->plans) {
    for (auto &g : P.graphs) hipGraphExecDestroy(g.exec);
    P.graphs.clear();
  }
}

// The plan of (part, K, nvec) and the workspace of a product of nvec vectors.
static int sigma_prepare(ccgf_ctx *c, int part, int K, int nvec, int prec, SigmaPlan **Pout) {
  const long long n = vec_len(c, part);
  // workspace
  size_t need = (size_t)nvec * n;
  if (c->sig_tmp_elems < need) {
    drop_graphs(c);
    if (c->sig_tmp) {
      for (auto &q : c->allocs)
        if (q == c->sig_tmp) q = nullptr;
      hipFree(c->sig_tmp);
    }
    c->sig_tmp = (cplx *)dev_alloc(c, need * sizeof(cplx));
    c->sig_tmp_elems = c->sig_tmp ? need : 0;
    if (!c->sig_tmp) return CCGF_ENOMEM;
  }
  const int ldaux = std::max(c->no, c->nv);
  size_t need_aux = (size_t)nvec * ldaux;
  if (prec && c->sig_x32_elems < need) {
    drop_graphs(c);
    if (c->sig_x32) {
      for (auto &q : c->allocs)
        if (q == c->sig_x32) q = nullptr;
      hipFree(c->sig_x32);
    }
    c->sig_x32 = (float2 *)dev_alloc(c, need * sizeof(float2));
    c->sig_x32_elems = c->sig_x32 ? need : 0;
    if (!c->sig_x32) return CCGF_ENOMEM;
  }
  if (c->sig_r1aux_elems < need_aux) {
    drop_graphs(c);
    if (c->sig_r1aux) {
      for (auto &q : c->allocs)
        if (q == c->sig_r1aux) q = nullptr;
      hipFree(c->sig_r1aux);
    }
    c->sig_r1aux = (cplx *)dev_alloc(c, need_aux * sizeof(cplx));
    c->sig_r1aux_elems = c->sig_r1aux ? need_aux : 0;
    if (!c->sig_r1aux) return CCGF_ENOMEM;
  }
  {
    const size_t need_part = (size_t)c->nk * c->nk * c->no * (size_t)(c->no + c->nv) * nvec;
    if (c->sig_part_elems < need_part) {
      drop_graphs(c);
      if (c->sig_part) {
        for (auto &q : c->allocs)
          if (q == c->sig_part) q = nullptr;
        hipFree(c->sig_part);
      }
      c->sig_part = (cplx *)dev_alloc(c, need_part * sizeof(cplx));
      c->sig_part_elems = c->sig_part ? need_part : 0;
      if (!c->sig_part) return CCGF_ENOMEM;
    }
  }
  if (!c->side_stream) {
    if (hipStreamCreateWithFlags(&c->side_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess)
      return hip_check(c, hipGetLastError(), "sigma side stream");
  }
  SigmaPlan *P = nullptr;
  for (auto &q : c->plans)
    if (q.part == part && q.K == K && q.nvec == nvec) P = &q;
  if (!P) {
    c->plans.emplace_back();
    P = &c->plans.back();
    P->part = part;
    P->K = K;
    P->nvec = nvec;
    P->n = n;
    build_plans(c, *P);
    if (!P->g_big.d_tasks || !P->g_bigt.d_tasks || !P->g_bigd.d_tasks || !P->g_ovvo.d_tasks || !P->g_r1.d_tasks ||
        !P->g_red1.d_tasks || !P->g_red2.d_tasks || (P->nfill > 0 && !P->d_fill) ||
        (P->g_bigt.ntask > 0 && !P->d_tri))
      return CCGF_ENOMEM;
    const size_t nk3 = (size_t)c->nk * c->nk * c->nk;
    const size_t vb = (size_t)nvec * n;
    const size_t pe = c->sig_part_elems;
    const size_t oovv = nk3 * c->no * c->no * c->nv * c->nv;
    bool ok;
    if (part == CCGF_PART_EA)
      ok = plan_in_bounds(P->g_big, (size_t)c->nwblk * c->nv * c->nv * c->nv * c->nv, vb, vb) &&
           plan_in_bounds(P->g_bigt, (size_t)c->nwblk * c->nv * c->nv * c->nv * c->nv, vb, vb) &&
           plan_in_bounds(P->g_bigd, (size_t)c->nwblk * c->nv * c->nv * c->nv * c->nv, vb, vb) &&
           plan_in_bounds(P->g_ovvo, nk3 * c->nv * c->no * c->no * c->nv, vb, vb) &&
           plan_in_bounds(P->g_r1, nk3 * c->nv * c->nv * c->nv * c->no, vb, vb) &&
           plan_in_bounds(P->g_red1, nk3 * c->nv * c->no * c->nv * c->nv, vb, pe) &&
           plan_in_bounds(P->g_red2, oovv, vb, pe);
    else
      ok = plan_in_bounds(P->g_big, nk3 * c->no * c->no * c->no * c->no, vb, vb) &&
           plan_in_bounds(P->g_ovvo, nk3 * c->nv * c->no * c->no * c->nv, vb, vb) &&
           plan_in_bounds(P->g_r1, nk3 * c->no * c->nv * c->no * c->no, vb, vb) &&
           plan_in_bounds(P->g_red1, nk3 * c->no * c->no * c->no * c->nv, vb, pe) &&
           plan_in_bounds(P->g_red2, oovv, vb, pe);
    for (long long f : P->fill_h)  // blocks of sigma2 (no x nv x nv) inside one vector
      ok = ok && f >= c->nv && f + (long long)c->no * c->nv * c->nv <= P->n;
    if (!ok) {
      c->plans.pop_back();
      return set_err(c, CCGF_EINVAL, "internal: sigma GEMM plan exceeds its buffers");
    }
  }
  *Pout = P;
  return CCGF_OK;
}

int sigma_apply(ccgf_ctx *c, int part, int K, int nvec, const cplx *x, cplx *y, int prec) {
  if (nvec <= 0) return CCGF_OK;
  SigmaPlan *P = nullptr;
  if (int rc = sigma_prepare(c, part, K, nvec, prec, &P)) return rc;
  hipStream_t s = c->stream;
  const bool timing = c->opt.timing != 0;
  ccgf_ctx::TimedSigma *ts = nullptr;
  if (timing) {
    if (c->tring.empty()) {
      c->tring.resize(64);
      for (auto &r : c->tring)
        for (int q = 0; q < 4; ++q)
          if (hipEventCreate(&r.e[q]) != hipSuccess) return hip_check(c, hipGetLastError(), "timing events");
    }
    // earlier products have completed by now wherever the solver or the caller
    // synchronised the stream; the wait below only bites for back-to-back calls
    timing_harvest(c);
    ts = &c->tring[c->tnext];
    c->tnext = (c->tnext + 1) % (int)c->tring.size();
    // the W_abcd statistics count the products in the context's own precision only (a
    // mixed form's FP64 true residuals go to the sigma totals alone)
    ts->big = part == CCGF_PART_EA && prec == c->opt.precision;
    ts->flops = ts->big ? plan_flops(P->g_big) : 0.0;
    ts->bytes = ts->big ? plan_bytes(P->g_big, (double)nvec * P->n, prec) : 0.0;
    hipEventRecord(ts->e[0], s);
  }
  // (the coupling and reduction GEMMs always run in FP64)
  const int pb = prec == 2 ? 2 : prec;
  const bool tuned = P->g_big.tn[pb] && P->g_ovvo.tn[pb] && P->g_r1.tn[0] && P->g_red1.tn[0] && P->g_red2.tn[0];
  if (!timing && c->opt.graphs == 0 && tuned) {
    // replay (or capture once) the launch sequence of this plan, operands and precision
    SigmaPlan::Captured *g = nullptr;
    for (auto &q : P->graphs)
      if (q.x == (const void *)x && q.y == (const void *)y && q.prec == prec) g = &q;
    if (!g) {
      if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess)
        return hip_check(c, hipGetLastError(), "capture stream");
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      if (hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return hip_check(c, hipGetLastError(), "sigma capture");
      int rc = sigma_enqueue(c, P, part, K, nvec, x, y, prec, c->cap_stream, nullptr);
      hipError_t e = hipStreamEndCapture(c->cap_stream, &graph);
      if (rc) {
        if (graph) hipGraphDestroy(graph);
        return rc;
      }
      if (e != hipSuccess || hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        if (graph) hipGraphDestroy(graph);
        return hip_check(c, hipGetLastError(), "sigma graph");
      }
      hipGraphDestroy(graph);
      if (P->graphs.size() >= 8) {  // keep the most recent operand pairs
        hipGraphExecDestroy(P->graphs.front().exec);
        P->graphs.erase(P->graphs.begin());
      }
      P->graphs.push_back({x, y, prec, exec});
      g = &P->graphs.back();
    }
    if (hipGraphLaunch(g->exec, s) != hipSuccess) return hip_check(c, hipGetLastError(), "sigma graph launch");
    return hip_check(c, hipGetLastError(), "sigma launch");
  }
  if (int rc = sigma_enqueue(c, P, part, K, nvec, x, y, prec, s, ts)) return rc;
  if (timing) {
    hipEventRecord(ts->e[1], s);
    ts->pending = true;
  }
  return hip_check(c, hipGetLastError(), "sigma launch");
}

void timing_harvest(ccgf_ctx *c) {
  for (auto &r : c->tring) {
    if (!r.pending) continue;
    float a = 0, b = 0;
    if (hipEventSynchronize(r.e[1]) == hipSuccess) {
      hipEventElapsedTime(&b, r.e[0], r.e[1]);
      c->t_sigma_ms += b;
      c->t_sigma_launches += 1;
      if (r.big) {
        hipEventElapsedTime(&a, r.e[2], r.e[3]);
        c->t_big_ms += a;
        c->t_big_launches += 1;
        c->t_big_flops += r.flops;
        c->t_big_bytes += r.bytes;
      }
    }
    r.pending = false;
  }
}

void timing_release(ccgf_ctx *c) {
  for (auto &r : c->tring)
    for (int q = 0; q < 4; ++q)
      if (r.e[q]) hipEventDestroy(r.e[q]);
  c->tring.clear();
}

// ------------------------------------------------------------------ several systems at once
// sigma products of several systems (uneven Nk, No, Nv; IP or EA each) in one sequence: every
// GEMM term is one launch over the tasks of all systems that have it, each task with its own
// shape and operands (k_cgemm_group); the element-wise terms run per system.  The products
// are those of sigma_apply term by term (the same tile arithmetic per output element).
namespace {
struct GroupLaunch {
  int tag, tn, prec;
  size_t shape0, task0, seg0;  // offsets of this launch's tables in the device buffer
  int ntask, total;
};

template <int TAG, typename R>
void launch_group_t(const GroupLaunch &L, const GemmShape *dsh, const GroupTask *dtk, const GemmSeg *dsg,
                    hipStream_t s) {
  const GemmShape *sh = dsh + L.shape0;
  const GroupTask *tk = dtk + L.task0;
  const GemmSeg *sg = dsg + L.seg0;
  if (L.tn == 16)
    hipLaunchKernelGGL((k_cgemm_group<TAG, R, 16>), dim3(L.total), dim3(256), 0, s, sh, tk, L.ntask, sg, L.total);
  else if (L.tn == 32)
    hipLaunchKernelGGL((k_cgemm_group<TAG, R, 32>), dim3(L.total), dim3(256), 0, s, sh, tk, L.ntask, sg, L.total);
  else
    hipLaunchKernelGGL((k_cgemm_group<TAG, R, 64>), dim3(L.total), dim3(256), 0, s, sh, tk, L.ntask, sg, L.total);
}

void launch_group(const GroupLaunch &L, const GemmShape *dsh, const GroupTask *dtk, const GemmSeg *dsg,
                  hipStream_t s) {
#define GCASE(T)                                                                   \
  case T:                                                                          \
    if (L.prec) launch_group_t<T, float>(L, dsh, dtk, dsg, s);                     \
    else launch_group_t<T, double>(L, dsh, dtk, dsg, s);                           \
    break;
  switch (L.tag) {
    GCASE(0) GCASE(1) GCASE(2) GCASE(3) GCASE(8) GCASE(9)
    case 4: launch_group_t<4, double>(L, dsh, dtk, dsg, s); break;
    case 5: launch_group_t<5, double>(L, dsh, dtk, dsg, s); break;
    case 6: launch_group_t<6, double>(L, dsh, dtk, dsg, s); break;
    default: launch_group_t<7, double>(L, dsh, dtk, dsg, s);
  }
#undef GCASE
}
}  // namespace

int sigma_group(int nsys, ccgf_ctx *const *ctxs, const int *parts, const int *Ks, const int *nvecs,
                const cplx *const *xs, cplx *const *ys) {
  ccgf_ctx *c0 = ctxs[0];
  const int prec = c0->opt.precision;
  hipStream_t s = c0->stream;
  std::vector<SigmaPlan *> P(nsys, nullptr);
  for (int i = 0; i < nsys; ++i) {
    if (nvecs[i] <= 0) continue;
    if (int rc = sigma_prepare(ctxs[i], parts[i], Ks[i], nvecs[i], prec, &P[i]))
      return set_err(c0, rc, "system " + std::to_string(i) + ": " + ctxs[i]->err);
  }
  // the operands of each term, per system
  struct Item {
    const GemmPlan *plan;
    const void *A, *B;
    cplx *C;
  };
  auto xb = [&](int i) -> const void * { return prec ? (const void *)ctxs[i]->sig_x32 : (const void *)xs[i]; };
  std::vector<std::pair<int, std::vector<Item>>> terms;  // (tag, items), in launch order
  auto add = [&](int tag, int i, const GemmPlan &g, const void *A, const void *B, cplx *C) {
    if (g.ntask == 0 || g.shape.M == 0 || g.shape.N == 0) return;
    for (auto &t : terms)
      if (t.first == tag) {
        t.second.push_back({&g, A, B, C});
        return;
      }
    terms.push_back({tag, {{&g, A, B, C}}});
  };
  for (int i = 0; i < nsys; ++i) {
    if (!P[i]) continue;
    ccgf_ctx *c = ctxs[i];
    if (parts[i] == CCGF_PART_EA) {
      const void *Wbig = prec ? (const void *)c->Wvvvv32 : (const void *)c->Wvvvv;
      add(0, i, P[i]->g_big, Wbig, xb(i), ys[i]);
    } else {
      add(2, i, P[i]->g_big, prec ? (const void *)c->WooP32 : (const void *)c->WooP, xb(i), ys[i]);
    }
  }
  for (int i = 0; i < nsys; ++i)
    if (P[i] && parts[i] == CCGF_PART_EA) {
      ccgf_ctx *c = ctxs[i];
      const void *Wbig = prec ? (const void *)c->Wvvvv32 : (const void *)c->Wvvvv;
      add(8, i, P[i]->g_bigt, Wbig, xb(i), ys[i]);
    }
  for (int i = 0; i < nsys; ++i)
    if (P[i] && parts[i] == CCGF_PART_EA) {
      ccgf_ctx *c = ctxs[i];
      const void *Wbig = prec ? (const void *)c->Wvvvv32 : (const void *)c->Wvvvv;
      add(9, i, P[i]->g_bigd, Wbig, xb(i), ys[i]);
    }
  for (int i = 0; i < nsys; ++i) {
    if (!P[i]) continue;
    ccgf_ctx *c = ctxs[i];
    if (parts[i] == CCGF_PART_EA) {
      add(1, i, P[i]->g_ovvo, prec ? (const void *)c->WvoPea32 : (const void *)c->WvoPea, xb(i), c->sig_tmp);
      add(6, i, P[i]->g_red1, c->Wvovv, xs[i], c->sig_part);
      add(6, i, P[i]->g_red2, c->Voovv, xs[i], c->sig_part);
    } else {
      add(3, i, P[i]->g_ovvo, prec ? (const void *)c->WvoP32 : (const void *)c->WvoP, xb(i), c->sig_tmp);
      add(7, i, P[i]->g_red1, c->Wooov, xs[i], c->sig_part);
      add(7, i, P[i]->g_red2, c->Voovv, xs[i], c->sig_part);
    }
  }
  const size_t nfirst = terms.size();  // the terms above run before the antisymmetric fill
  for (int i = 0; i < nsys; ++i) {
    if (!P[i]) continue;
    ccgf_ctx *c = ctxs[i];
    if (parts[i] == CCGF_PART_EA) add(4, i, P[i]->g_r1, c->Wvvvo, xs[i], ys[i]);
    else add(5, i, P[i]->g_r1, c->Wovoo, xs[i], ys[i]);
  }
  // tables of every launch, uploaded once
  std::vector<GemmShape> shapes;
  std::vector<GroupTask> tasks;
  std::vector<GemmSeg> segs;
  std::vector<GroupLaunch> launches;
  for (auto &t : terms) {
    const int tag = t.first;
    const bool big = tag <= 3 || tag == 8 || tag == 9;
    int maxN = 0;
    for (const Item &it : t.second) maxN = std::max(maxN, it.plan->shape.N);
    const int tn = maxN <= 16 ? 16 : maxN <= 32 ? 32 : big ? 64 : 32;
    GroupLaunch L{tag, tn, big ? prec : 0, shapes.size(), tasks.size(), segs.size(), 0, 0};
    int tile = 0;
    for (const Item &it : t.second) {
      const GemmPlan &g = *it.plan;
      const int si = (int)(shapes.size() - L.shape0), seg0 = (int)(segs.size() - L.seg0);
      shapes.push_back(g.shape);
      segs.insert(segs.end(), g.segs.begin(), g.segs.end());
      const int tM = (g.shape.M + TM - 1) / TM, tN = (g.shape.N + tn - 1) / tn;
      for (GemmTask k : g.tasks) {
        k.seg_begin += seg0;
        tasks.push_back(GroupTask{it.A, it.B, it.C, k, si, tile, tM, tN});
        tile += tM * tN;
      }
    }
    L.ntask = (int)(tasks.size() - L.task0);
    L.total = tile;
    launches.push_back(L);
  }
  const size_t bytes = shapes.size() * sizeof(GemmShape) + tasks.size() * sizeof(GroupTask) +
                       segs.size() * sizeof(GemmSeg) + 3 * 256;
  if (c0->grp_bytes < bytes) {
    if (c0->grp_buf) {
      hipStreamSynchronize(s);
      for (auto &q : c0->allocs)
        if (q == c0->grp_buf) q = nullptr;
      hipFree(c0->grp_buf);
    }
    c0->grp_buf = dev_alloc(c0, bytes);
    c0->grp_bytes = c0->grp_buf ? bytes : 0;
    if (!c0->grp_buf) return set_err(c0, CCGF_ENOMEM, "no device memory for the grouped launch tables");
  }
  auto align = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char *base = (char *)c0->grp_buf;
  GemmShape *dsh = (GemmShape *)base;
  GroupTask *dtk = (GroupTask *)(base + align(shapes.size() * sizeof(GemmShape)));
  GemmSeg *dsg = (GemmSeg *)((char *)dtk + align(tasks.size() * sizeof(GroupTask)));
  // the previous grouped call has finished (it synchronised before returning)
  if (hipMemcpy(dsh, shapes.data(), shapes.size() * sizeof(GemmShape), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dtk, tasks.data(), tasks.size() * sizeof(GroupTask), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dsg, segs.data(), segs.size() * sizeof(GemmSeg), hipMemcpyHostToDevice) != hipSuccess)
    return hip_check(c0, hipGetLastError(), "grouped launch tables");
  // the reduced-precision products read complex-float copies of the vectors
  for (int i = 0; i < nsys; ++i)
    if (P[i] && prec) {
      const size_t tot = (size_t)nvecs[i] * P[i]->n;
      hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, xs[i], ctxs[i]->sig_x32,
                         tot);
    }
  for (size_t l = 0; l < nfirst; ++l) launch_group(launches[l], dsh, dtk, dsg, s);
  // blocks left to antisymmetry, before the terms that accumulate into them
  for (int i = 0; i < nsys; ++i)
    if (P[i] && parts[i] == CCGF_PART_EA && P[i]->nfill > 0) {
      const int no = ctxs[i]->no, nv = ctxs[i]->nv;
      const long long b2 = (long long)no * nv * nv;
      hipLaunchKernelGGL(k_vvvv_fill, dim3((unsigned)((b2 + 255) / 256), P[i]->nfill, std::min(nvecs[i], 64)),
                         dim3(256), 0, s, ys[i], P[i]->n, nvecs[i], nv, b2, P[i]->d_fill, P[i]->d_fill + P[i]->nfill,
                         P[i]->nfill);
    }
  for (size_t l = nfirst; l < launches.size(); ++l) launch_group(launches[l], dsh, dtk, dsg, s);
  for (int i = 0; i < nsys; ++i) {
    if (!P[i]) continue;
    ccgf_ctx *c = ctxs[i];
    const int nk = c->nk, no = c->no, nv = c->nv, K = Ks[i], nvec = nvecs[i];
    const long long n = P[i]->n;
    const unsigned gy = (unsigned)std::min(nvec, 65535);
    if (parts[i] == CCGF_PART_EA) {
      hipLaunchKernelGGL(k_r1_finish, dim3((unsigned)(((nv + no) * nvec + 3) / 4)), dim3(256), 0, s, 1, nk, no, nv, K,
                         nv + no, nv, nvec, nk * nk * no, n, c->sig_part, xs[i], ys[i], c->sig_r1aux, std::max(no, nv),
                         c->Foo, c->Fvv, c->Fov);
      const long long tot = (long long)nk * nk * no * nv * nv;
      hipLaunchKernelGGL(k_ea_local, dim3((unsigned)((tot + 255) / 256), gy), dim3(256), 0, s, nk, no, nv, K, nvec, n,
                         c->kc3, xs[i], ys[i], c->sig_tmp, c->sig_r1aux, c->Foo, c->Fvv, c->t2);
    } else {
      hipLaunchKernelGGL(k_r1_finish, dim3((unsigned)(((nv + no) * nvec + 3) / 4)), dim3(256), 0, s, 0, nk, no, nv, K,
                         no + nv, no, nvec, nk * nk * no, n, c->sig_part, xs[i], ys[i], c->sig_r1aux, std::max(no, nv),
                         c->Foo, c->Fvv, c->Fov);
      const long long tot = (long long)nk * nk * no * no * nv;
      hipLaunchKernelGGL(k_ip_local, dim3((unsigned)((tot + 255) / 256), gy), dim3(256), 0, s, nk, no, nv, K, nvec, n,
                         c->kc3, xs[i], ys[i], c->sig_tmp, c->sig_r1aux, c->Foo, c->Fvv, c->t2);
    }
  }
  return hip_check(c0, hipGetLastError(), "grouped sigma launch");
}
