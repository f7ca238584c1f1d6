// Device-side descriptors shared by the kernels and the host runtime.
//
// Layout in HBM (per matrix; all buffers 256-byte aligned, inside the caller's
// workspace).  The iterate is oriented as X = G (m <= n) or X = G^T (m > n),
// so X is s x L with s = min(m, n) <= L = max(m, n) and the Gram matrix is
// s x s (the smaller side).  s and L are padded with zeros to sp, Lp
// (multiples of the block tile, 128 or 256).  Zero rows/columns stay exactly zero under
// X <- aX + (bA + cA^2)X, so every kernel runs on the padded shape with no
// bounds checks; only the input read and the final store see m, n.
//   Xf      sp x Lp  fp32   master iterate (row-major)
//   Xb, Xb1 sp x Lp  bf16   operand copies of X_t (bf16/fp8 paths), used in turn:
//                           step t reads Xb (t even) or Xb1 (t odd) in the Gram
//                           product and in B X, and its update writes the other
//   XT[2]   Lp x sp  fp32   X^T operand for B X on the fp32 path (ping-pong across steps)
//   Af      sp x sp  fp32   A = X X^T (fp32 path only)
//   As      sp x sp  bf16   A in bf16 on the bf16/fp8 paths, read by A^2 and by
//                           the bA term of B (fp32 path: Af itself)
//   Bs      sp x sp  bf16 or fp32   B - beta I, B = bA + cA^2 (beta: see shift_beta)
//   Xq, Aq  sp x Lp, sp x sp  e4m3  operand copies for the FP8 steps (256 tile)
//   part    split-K partial tiles of the Gram-side products
//   red     per-tile partial sums of squares (fp64) and maxima (fp32) of G
//   trp     per-tile partials of tr(A_t) and ||A_t||_F^2 (fp32), for the shift beta_t
//   scal    per-matrix scalars (scale, amax values), cnt: arrival counters
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pe {

constexpr int kTileSmall = 128; // GEMM block tiles: 128 x 128 or 256 x 256
constexpr int kTileLarge = 256;
constexpr int kPrepTile = 64;   // norm/prep tile
constexpr int kPrepGroup = 4;   // tiles per norm-pass item (one partial sum each)
constexpr int kThreads = 256;   // threads per block (4 wave64)
constexpr int kMaxSteps = 64;

enum Prec : int32_t { kF32 = 0, kBF16 = 1, kFP8 = 2 };

// scal[] slots
enum : int32_t {
  kScScale = 0,    // sigma = 1 / (1.01 ||G||_F + 1e-7)
  kScAmaxG = 1,    // max |G| (float bits)
  kScFro = 2,      // ||G||_F as float
  kScBeta = 3,     // shift beta_t = tr(B_t)/s of the current step (update: a + beta)
  kScPowN = 4,     // spectrum-aware init: ||A v|| of the last power step
  kScInitA = 5,    // spectrum-aware init: coefficients (a, b) of the init cubic
  kScInitB = 6,
  kScAmaxX = 8,    // +t : max |X_t| (uint bits of a non-negative float), t = 0..63
  kScAmaxA = 72,   // +t : max |A_t| for step t (0-based)
  kScN = 136
};

struct MatDesc {
  const void* G;
  void* Out;
  int64_t ldg, ldo;
  int32_t m, n, s, L;
  int32_t sp, Lp, trans, g_bf16;
  int32_t out_bf16, nb, nbL, sel;
  float* Xf;
  void* Xb;
  void* Xb1;
  void* XT0;
  void* XT1;
  float* Af;
  void* As;
  void* Bs;
  float* part;
  double* red;      // [n_prep] doubles then [n_prep] floats
  float* scal;      // [kScN]
  uint32_t* cnt;    // [4]
  float* trp;       // [syrk_nt][2] per-tile partials of tr(A) and ||A||_F^2 (Gram epilogue)
  int32_t n_prep, syrk_nt, upd_nt, gram_split;
  int32_t a2_split, bt, g_vec, o_vec;  // bt: block tile edge; g_vec / o_vec: 16-byte
                                       // loads of G / stores of the bf16 output
  // learned l-predictor (null unless the call selects schedules per matrix)
  int32_t* selp;    // schedule class of this matrix
  int32_t* flagp;   // 1: the fallback re-run recomputes this matrix
  float* A2f;       // sp x sp fp32: A^2 of step 1, before the class is known
  float* mom;       // [syrk_nt][4] per-tile partial moments tr(A^k), k = 1..4
  float* feat;      // [16] features (diagnostic copy)
  float* est;       // [2]: estimate of ||X X^T - I||_2, flag
  float* vec;       // power iteration vectors: v [sp], y [sp], w [Lp]
  // FP8 steps on the 256 tile: e4m3 copies of the Gram-side operands
  uint8_t* Xq;      // sp x Lp: e4m3(q X_t), written by the quantisation pass
  uint8_t* Aq;      // sp x sp: e4m3(q A_t)
  // fast rectangular iteration (FP32): sp x sp buffers, see kFb* below
  float* fb[6];
  // Muon step (caller's m x n layout): momentum M (FP32) updated by the norm
  // pass, weights W updated by the last step's epilogue
  float* M;
  void* W;
  int64_t ldm, ldw;
  int32_t w_bf16;
  // 1: X_0 is exactly its bf16 copy (bf16 input, bf16/FP8 compute, no Muon
  // momentum): the norm pass stores no FP32 X_0 and the first update reads Xb
  int32_t x0b;
};

// Roles of MatDesc::fb in the fast rectangular iteration: the segment's R_t
// (ping-pong), D_t = Q_t - (prod a) I (ping-pong), P = R_t B_t, and B_t.
enum : int32_t { kFbR0 = 0, kFbR1 = 1, kFbD0 = 2, kFbP = 3, kFbB = 4, kFbD1 = 5, kFbNone = -1 };

struct KArgs {
  const MatDesc* descs;  // device array of `count` descriptors
  const int32_t* offs;   // per-matrix prefix offsets of this phase's items, count+1
  int32_t count;
  int32_t total;         // items in this launch
  int32_t t;             // 0-based step
  int32_t last;          // 1 on the final step
  int32_t fp8;           // this step's Gram-side products take e4m3 operands
  int32_t fp8_next;      // the next step's Gram product takes e4m3 operands
  int32_t norm_mode;
  int32_t tmax;          // rows of the selectable coefficient table
  float a, b, c;         // coefficients of step t (fixed schedule)
  const float* sel_coef; // [n_sched][tmax][3] or nullptr: per-matrix class schedules
  int32_t raw_a2;        // step-1 A^2 of the learned path: store A^2 and its moments
  int32_t fallback;      // fallback re-run: skip matrices whose flag is 0
  const float* mlp;      // predictor parameters (device) for the selection kernel
  int32_t force_class;   // >= 0: use this class instead of the network's choice
  int32_t fixed_class;
  float tau;             // fallback threshold
  int32_t est_phase;     // power-iteration phase selector
  const int32_t* ord;    // position -> matrix of this phase's item order (nullptr: identity)
  // fast rectangular iteration (gemm_fast_kernel and the update): operand and
  // epilogue buffers (MatDesc::fb roles) and coefficients of
  //   out = cacc * acc + c1 * E1 + c2 * E2 + cdiag * I
  int32_t fast;          // 1: a launch of the fast iteration
  int32_t fp_, fq_, fe1, fe2, fout;
  float cacc, c1, c2, cdiag;
  int32_t fscale;        // cacc is multiplied by sigma^2 (first segment's Gram)
  float mbeta, mlr, mwd; // Muon momentum coefficient, learning rate, weight decay
  int32_t init_step;     // the spectrum-aware init step: (a, b, 0) from scal[kScInitA/B]
  const int32_t* sel_steps;  // [n_sched]: steps T' of each class's schedule (learned path)
  int32_t x0b;           // first update: every matrix of the call reads X_0 from its bf16 copy
};

// Spectral shift of the update.  In real arithmetic
//   X_{t+1} = a X + B X = (a + beta) X + (B - beta I) X
// for any beta.  The product takes bf16 copies of its operands, whose rounding
// errors enter as (B - beta I) dX and dB X; beta = tr(B) / s, the mean
// eigenvalue of B, minimises ||B - beta I||_F and with it the error carried
// by isotropic rounding noise (on inputs whose singular values sit close
// together, B is close to a multiple of I and the unshifted product rounds away
// most of the update).  tr(B) = b tr(A) + c ||A||_F^2 for symmetric A; the Gram
// epilogue leaves per-tile partials of both, and every caller reduces them in
// the same fixed order, so all blocks agree on beta bit for bit.
__device__ __forceinline__ float shift_beta(const MatDesc& d, float b, float c) {
  const int lane = threadIdx.x & 63;
  float tr = 0.0f, fr = 0.0f;
  for (int u = lane; u < d.syrk_nt; u += 64) {
    tr += d.trp[2 * u];
    fr += d.trp[2 * u + 1];
  }
  // butterfly sums: every lane ends with the same bits (addition commutes exactly)
  for (int off = 32; off > 0; off >>= 1) {
    tr += __shfl_xor(tr, off);
    fr += __shfl_xor(fr, off);
  }
  return d.s > 0 ? (b * tr + c * fr) / (float)d.s : 0.0f;
}

constexpr int kClasses = 8;
constexpr int kFeat = 16;
constexpr int kMlpH = 64;
constexpr int kMlpParams = kFeat * kMlpH + kMlpH + kMlpH * kMlpH + kMlpH + kMlpH * kClasses + kClasses;

// Device memory is filled from kernel arguments (copied at launch), so the
// host needs neither pinned staging nor a synchronisation to upload tables.
constexpr int kPutWords = 960;
struct PutChunk {
  uint32_t* dst;
  int32_t nwords;
  int32_t pad;
  uint32_t w[kPutWords];
};

}  // namespace pe
