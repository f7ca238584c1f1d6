// Host runtime of the C ABI in pe.h: argument checks, workspace layout, tile
// tables, launch sequence of the online stage, plans and hipGraph capture.
//
// Launch sequence for T steps (Section 3.5 / the Appendix A.1 listing, with
// the scale folded into step 1):
//   prep                                   ||G||_F, max|G|, X_0 copies
//   for t: gram [+ reduce], a2 [+ reduce], update
// Each launch covers every matrix of the call (grouped, persistent blocks).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pe.h"
#include "pe_device.h"

namespace pe {
hipError_t launch_put(const PutChunk& c, hipStream_t st);
hipError_t launch_finalize(const KArgs& a, hipStream_t st);
hipError_t launch_select(const KArgs& a, hipStream_t st);
hipError_t launch_combine(int prec, const KArgs& a, hipStream_t st);
hipError_t launch_quant(int kind, const KArgs& a, int grid_cap, hipStream_t st);
hipError_t launch_fast(int kind, const KArgs& a, int grid_cap, hipStream_t st);
hipError_t launch_power(int prec, int phase, const KArgs& a, hipStream_t st);
hipError_t launch_est(const KArgs& a, int iters, hipStream_t st, const int32_t* offs_a, int total_a,
                      const int32_t* offs_b, int total_b);
hipError_t launch_mlp_forward(const float* params, const float* feats, int B, float* logits,
                              hipStream_t st);
hipError_t launch_mlp_grad(const float* params, const float* feats, const int32_t* labels, int B,
                           float* part, float* part_loss, float* grad_out, float* loss_out,
                           float* upd_params, float* m, float* v, int step, float lr, hipStream_t st);
hipError_t launch_quantize(const void* x, int x_bf16, uint8_t* q, int64_t n, float scale,
                           hipStream_t st);
hipError_t launch_prep(int prec, const KArgs& a, int grid_cap, hipStream_t st);
void warm_launch_grids();
hipError_t launch_gemm(int prec, int bt, int kind, const KArgs& a, int grid_cap, hipStream_t st);
hipError_t launch_reduce(int prec, int bt, int kind, const KArgs& a, int grid_cap, hipStream_t st);
}  // namespace pe

using namespace pe;

namespace {

thread_local std::string g_last_error;

enum Phase { PH_PREP = 0, PH_GRAM, PH_A2, PH_UPD, PH_RGRAM, PH_RA2, PH_COMBINE, PH_EST_A, PH_EST_B,
             PH_QX, PH_QA, PH_FSYRK, PH_PW, PH_N };

// Schedule classes of the learned path: (l, T'), T' = 0 meaning the call's T;
// class 4 is the caller's schedule for all T steps.  Steps past a class's T'
// leave the matrix as it is (its kernels skip it; the last step copies X).
struct ClassDef { double ell; int steps; };
constexpr ClassDef kClassTable[kClasses] = {{1e-1, 2}, {1e-1, 3}, {3e-2, 3}, {1e-2, 4},
                                            {1e-3, 0}, {3e-3, 4}, {3e-4, 0}, {1e-4, 0}};
constexpr int kFixedClass = 4;
int class_steps(int c, int T) { return kClassTable[c].steps > 0 ? std::min(T, kClassTable[c].steps) : T; }
constexpr int kEstIters = 8;

bool learned_mode(const pe_opts* o) { return o->predictor != nullptr || o->force_class >= 0; }

constexpr int kGemmGridCap = 512;       // 128-tile kernel: 2 resident blocks per CU x 256 CUs
constexpr int kGemmGridCapLarge = 256;  // 256-tile kernel: 1 resident block per CU
constexpr int kPrepGridCap = 2048;
constexpr int kReduceGridCap = 1024;
constexpr int kQuantGridCap = 2048;
// Gram-side items wanted per launch before split-K kicks in.  Split-K buys
// parallelism with FP32 partial tiles written and summed by a second launch;
// measured on a single 4096 x 1024 bf16 matrix (36 Gram tiles of 128), splits
// of 15 / 8 / 4 / 2 / 1 gave 0.83 / 0.68 / 0.58 / 0.55 / 0.58 ms per call, so
// the target stays low: a couple of splits for calls with tens of tiles.
constexpr int kFillTarget = 64;

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }
int64_t round_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

pe_status hip_fail(hipError_t e, const char* where) {
  char buf[256];
  snprintf(buf, sizeof buf, "%s: %s", where, hipGetErrorString(e));
  g_last_error = buf;
  return PE_EHIP;
}

// Launch classes: (precision, block tile).  Every phase launches once per class
// present in a call, over the items of that class's matrices only, so one
// grouped call can mix tiles (per-shape-class choices of the autotuned table)
// and precisions (matrices too small for bf16 rounding to average out run
// FP32 operands inside a bf16 call).
constexpr int kNCls = 4;
inline int cls_of(int prec, int bt) { return (prec == kF32 ? 0 : 2) + (bt == kTileLarge ? 1 : 0); }
inline int cls_prec(int c) { return c < 2 ? kF32 : kBF16; }
inline int cls_bt(int c) { return (c & 1) ? kTileLarge : kTileSmall; }

struct Layout {
  std::vector<MatDesc> descs;           // device pointers filled when ws != nullptr
  std::vector<int32_t> prec, bt;        // per matrix
  // item tables: offs[ph][cls] holds count + 1 prefix offsets in which the
  // matrices of other classes contribute no items (phases that do not depend
  // on the class -- the estimate's matrix-vector products -- keep every
  // matrix in class 0's table)
  std::vector<int32_t> offs[PH_N][kNCls];
  int32_t totals[PH_N][kNCls] = {};
  // Gram items per class ordered by matrix, longest k (Lp) first: per-tile
  // work is proportional to Lp, and persistent blocks take items round-robin,
  // so long tiles first and short ones last balance the CUs
  std::vector<int32_t> ord_gram[kNCls];
  size_t bytes = 0;
  size_t descs_off = 0, offs_off = 0, coef_off = 0;
  size_t sel_off = 0;  // learned plans: kSelWords words per matrix (class, flag, features, estimate)
  bool x0b = false;    // every bf16-path matrix has MatDesc::x0b
};

// per-matrix selection record of a learned plan, contiguous over the matrices
// so pe_plan_selection reads all of them with one copy: words 0-15 class and
// fallback flag, 16-31 the 16 features, 32-47 the estimate
constexpr int kSelWords = 48;

bool valid_matrix(const pe_matrix& m) {
  if (m.m < 0 || m.n < 0) return false;
  if (m.m == 0 || m.n == 0) return true;
  if (!m.G || (!m.X && !m.W)) return false;
  if (m.ldg < m.n || (m.X && m.ldx < m.n)) return false;
  if (m.g_dtype != PE_F32 && m.g_dtype != PE_BF16) return false;
  if (m.X && m.x_dtype != PE_F32 && m.x_dtype != PE_BF16) return false;
  if (m.M && m.ldm < m.n) return false;
  if (m.W && (m.ldw < m.n || (m.w_dtype != PE_F32 && m.w_dtype != PE_BF16))) return false;
  if (m.m > (1 << 20) || m.n > (1 << 20)) return false;
  return true;
}

pe_status check_opts(const pe_opts* o) {
  if (!o) return PE_EINVAL;
  if (o->T < 1 || o->T > kMaxSteps || !o->abc) return PE_EINVAL;
  if (o->compute < PE_COMPUTE_F32 || o->compute > PE_COMPUTE_FP8) return PE_EINVAL;
  if (o->norm_mode != 0 && o->norm_mode != 1) return PE_EINVAL;
  if (o->tile < 0 || o->tile > 2) return PE_EINVAL;
  if (o->compute == PE_COMPUTE_FP8) {
    if (o->fp8_steps < 0 || o->fp8_steps > o->T - 1) return PE_EINVAL;
  }
  for (int i = 0; i < 3 * o->T; ++i)
    if (!std::isfinite(o->abc[i])) return PE_EINVAL;
  if (o->force_class < -1 || o->force_class >= kClasses) return PE_EINVAL;
  if (!std::isfinite(o->fallback_tau)) return PE_EINVAL;
  if (o->split_k < 0 || o->split_k > 64) return PE_EINVAL;
  if (o->fast_restart < 0 || !std::isfinite(o->fast_eps) || o->fast_eps < 0.0f) return PE_EINVAL;
  if (o->fast_restart > 0 &&
      (o->compute != PE_COMPUTE_F32 || learned_mode(o) || o->tile == 2)) return PE_EUNSUPPORTED;
  if (!(o->muon_beta >= 0.0f && o->muon_beta < 1.0f) || !std::isfinite(o->muon_lr) ||
      !std::isfinite(o->muon_wd)) return PE_EINVAL;
  if (o->spectral_init < 0 || o->spectral_init > 1000) return PE_EINVAL;
  if (o->spectral_init > 0 &&
      ((o->compute == PE_COMPUTE_FP8 && o->fp8_steps > 0) || learned_mode(o) || o->fast_restart > 0))
    return PE_EUNSUPPORTED;
  return PE_OK;
}

// Block tile per matrix: 256 x 256 (8 waves, 32x32 MFMA fragments, wave tile
// 128 x 64) halves the LDS and L2 traffic per flop of the 128 x 128 tile, but
// pads s and L to multiples of 256 and yields 4x fewer tiles.  The choice comes
// from the autotuned table, keyed by shape class (precision, s bucket, aspect
// bucket; see shape_class()) and call regime (_x1 / _xN, see tile_for());
// without an entry the 256 tile is taken for s >= 512 when the call's update
// has at least one 256 tile per CU.  FP32 matrices always take the 128 tile.
std::mutex g_tab_mu;
std::map<std::string, int> g_tile_table;

std::string shape_class(int prec, int64_t s, int64_t L) {
  static const int64_t sb[] = {256, 512, 1024, 2048, 4096};
  int i = 0;
  while (i < 5 && s > sb[i]) ++i;
  const double a = (double)L / (double)s;
  const int ab = a <= 1.5 ? 1 : (a <= 4.0 ? 4 : 16);
  char buf[64];
  snprintf(buf, sizeof buf, "%s_s%lld_a%d", prec == kF32 ? "f32" : "bf16",
           (long long)(i < 5 ? sb[i] : 8192), ab);
  return buf;
}

// Precision of one matrix: FP32 on the FP32 path; on the bf16/FP8 paths FP32
// as well when the smaller side is below kTinyS, where a handful of singular
// values leave bf16 rounding errors nothing to average over (relative errors
// up to ~1e-1 at s = 2-8 on Gaussian inputs) and the products cost nothing.
constexpr int64_t kTinyS = 16;
int prec_for(const pe_opts* o, int64_t s) {
  if (o->compute == PE_COMPUTE_F32 || s < kTinyS) return kF32;
  return kBF16;
}

// Call regimes of the autotuned table: "xN" for calls with at least
// kBatchFlops algorithmic FLOP per step (3 s^2 L + s^3 summed over the
// matrices; the autotuner's batches carry ~3e12 per step) or with more than
// kBatchTiles update tiles of 256 (four per CU of the 256-CU part: then the
// 256 tile leaves no CU idle), "x1" below.  A batch of 48 GPT-small matrices
// (2.2e11 FLOP, 1296 tiles) runs 2.76 ms per call on the 256 tile against
// 3.00 on the 128 tile, while a single 2048 x 32768 matrix (1024 tiles)
// keeps the 128 tile (2.13 against 2.35 ms).
constexpr double kBatchFlops = 3e12;
constexpr int64_t kBatchTiles = 1024;

// Block tile of one matrix.  Forced by opts.tile; else the autotuned table's
// entry for the matrix's shape class in the call's regime; else 256 for bf16
// matrices with s >= 512 in calls whose update has at least one 256-tile per
// CU, 128 otherwise.
int tile_for(const pe_opts* o, int prec, int64_t s, int64_t L, bool batch_regime, int64_t upd_tiles256) {
  if (o->tile == 1) return kTileSmall;
  if (o->tile == 2) return kTileLarge;
  if (prec == kF32) return kTileSmall;
  {
    std::lock_guard<std::mutex> lk(g_tab_mu);
    if (!g_tile_table.empty()) {
      auto it = g_tile_table.find(shape_class(prec, s, L) + (batch_regime ? "_xN" : "_x1"));
      if (it != g_tile_table.end()) return it->second == 2 ? kTileLarge : kTileSmall;
    }
  }
  return (s >= 512 && upd_tiles256 >= 256) ? kTileLarge : kTileSmall;
}

// Build the per-matrix descriptors and the item tables.  With ws == nullptr
// only sizes are computed.
pe_status build_layout(int count, const pe_matrix* mats, const pe_opts* o, char* ws, Layout* L) {
  L->descs.clear();
  L->prec.assign(count, kBF16);
  L->bt.assign(count, kTileSmall);
  for (int p = 0; p < PH_N; ++p)
    for (int c = 0; c < kNCls; ++c) L->offs[p][c].assign(1, 0);
  // update tiles of the whole call at the 256 tile (the built-in tile rule)
  int64_t upd256 = 0;
  double call_flops = 0.0;
  for (int i = 0; i < count; ++i) {
    const pe_matrix& m = mats[i];
    if (m.m <= 0 || m.n <= 0) continue;
    const int64_t s = std::min(m.m, m.n), Lx = std::max(m.m, m.n);
    upd256 += round_up(s, kTileLarge) / kTileLarge * (round_up(Lx, kTileLarge) / kTileLarge);
    call_flops += 3.0 * (double)s * s * Lx + (double)s * s * s;
  }
  const bool batch_regime = call_flops >= kBatchFlops || upd256 > kBatchTiles;
  // first pass: precision, tile, shapes and Gram-side tile counts per class
  // (for the split-K choice)
  struct Shape { int64_t s, L, sp, Lp; int nb, nbL, syrk, upd, prep, prec, bt, cls; };
  std::vector<Shape> sh;
  int64_t syrk_total[kNCls] = {};
  for (int i = 0; i < count; ++i) {
    const pe_matrix& m = mats[i];
    Shape q{};
    q.prec = kBF16;
    q.bt = kTileSmall;
    if (m.m > 0 && m.n > 0) {
      q.s = std::min(m.m, m.n);
      q.L = std::max(m.m, m.n);
      q.prec = prec_for(o, q.s);
      q.bt = tile_for(o, q.prec, q.s, q.L, batch_regime, upd256);
      const int bt = q.bt;
      q.sp = round_up(q.s, bt);
      q.Lp = round_up(q.L, bt);
      q.nb = (int)(q.sp / bt);
      q.nbL = (int)(q.Lp / bt);
      q.syrk = q.nb * (q.nb + 1) / 2;
      q.upd = q.nb * q.nbL;
      // items of kPrepGroup tiles (sp and Lp are multiples of 128, so the tile count is a multiple of 4)
      q.prep = (int)((q.sp / kPrepTile) * (q.Lp / kPrepTile) / kPrepGroup);
    }
    q.cls = cls_of(q.prec, q.bt);
    syrk_total[q.cls] += q.syrk;
    L->prec[i] = q.prec;
    L->bt[i] = q.bt;
    sh.push_back(q);
  }
  int want[kNCls];
  for (int c = 0; c < kNCls; ++c)
    want[c] = syrk_total[c] > 0 ? (int)std::min<int64_t>(64, (kFillTarget + syrk_total[c] - 1) / syrk_total[c]) : 1;
  size_t off = 0;
  L->descs_off = off;
  off = align_up(off + sizeof(MatDesc) * (size_t)std::max(count, 1));
  L->offs_off = off;
  off = align_up(off + sizeof(int32_t) * ((size_t)PH_N * kNCls * (count + 1) + (size_t)kNCls * count));
  const bool learned = learned_mode(o);
  L->coef_off = off;
  if (learned) off = align_up(off + sizeof(float) * kClasses * 3 * (size_t)o->T + sizeof(int32_t) * kClasses);
  L->sel_off = off;
  if (learned) off = align_up(off + sizeof(int32_t) * kSelWords * (size_t)std::max(count, 1));
  for (int i = 0; i < count; ++i) {
    const pe_matrix& m = mats[i];
    const Shape& q = sh[i];
    const int prec = q.prec, bt = q.bt;
    const size_t esz = prec == kF32 ? 4 : 2;
    const bool q8 = prec == kBF16 && o->compute == PE_COMPUTE_FP8 && o->fp8_steps > 0 && bt == kTileLarge;
    MatDesc d;
    memset(&d, 0, sizeof d);
    d.G = m.G;
    d.Out = m.X;
    d.ldg = m.ldg;
    d.ldo = m.ldx;
    d.M = m.M;
    d.ldm = m.ldm;
    d.W = m.W;
    d.ldw = m.ldw;
    d.w_bf16 = m.W && m.w_dtype == PE_BF16;
    d.m = (int32_t)m.m;
    d.n = (int32_t)m.n;
    d.s = (int32_t)q.s;
    d.L = (int32_t)q.L;
    d.sp = (int32_t)q.sp;
    d.Lp = (int32_t)q.Lp;
    d.trans = m.m > m.n;
    d.g_bf16 = m.g_dtype == PE_BF16;
    // 16-byte loads of G rows need an aligned base and a leading dimension
    // that keeps every row 16-byte aligned
    {
      const int64_t per16 = d.g_bf16 ? 8 : 4;
      d.g_vec = ((uintptr_t)m.G % 16 == 0) && (m.ldg % per16 == 0);
    }
    // the first update reads X_0 from its bf16 copy when that copy is exact;
    // a first update that is also the last (one step) reads the FP32 master
    d.x0b = prec != kF32 && d.g_bf16 && !m.M && o->T + (o->spectral_init > 0 ? 1 : 0) >= 2;
    d.out_bf16 = m.X && m.x_dtype == PE_BF16;
    d.o_vec = d.out_bf16 && ((uintptr_t)m.X % 16 == 0) && (m.ldx % 8 == 0);
    d.nb = q.nb;
    d.nbL = q.nbL;
    d.bt = bt;
    d.n_prep = q.prep;
    d.syrk_nt = q.syrk;
    d.upd_nt = q.upd;
    // split-K: enough Gram-side items to fill the GPU, at least 4 k-stages per
    // split of the Gram; A^2 (k = s, short) splits only with 16 k-stages per
    // split, since its reduce also runs the combine epilogue (on one 4096 x
    // 1024 bf16 matrix a two-way A^2 split took 12 us plus 22 us of reduce)
    const int bk = prec == kF32 ? 32 : 64;
    const int max_gram = std::max<int64_t>(1, q.Lp / (4 * bk));
    const int max_a2 = std::max<int64_t>(1, q.sp / (16 * bk));
    const int cap = o->split_k > 0 ? o->split_k : 64;
    d.gram_split = q.syrk ? std::min(std::min(want[q.cls], max_gram), cap) : 1;
    d.a2_split = q.syrk ? std::min(std::min(want[q.cls], max_a2), cap) : 1;
    if (q.syrk) {
      auto take = [&](size_t bytes) {
        char* p = ws ? ws + off : nullptr;
        off = align_up(off + bytes);
        return (void*)p;
      };
      const size_t X = (size_t)q.sp * q.Lp, A = (size_t)q.sp * q.sp;
      d.Xf = (float*)take(X * 4);
      if (prec == kF32) {
        d.XT0 = take(X * 4);
        d.XT1 = take(X * 4);
      } else {
        d.Xb = take(X * 2);
        d.Xb1 = take(X * 2);
      }
      // A in FP32 on the fp32 path; the bf16 paths keep only its bf16 copy,
      // which both A^2 and the bA term of the combine read
      // (bf16 paths: an FP32 A only for the spectrum-aware init's power method)
      d.Af = (prec == kF32 || o->spectral_init > 0) ? (float*)take(A * 4) : nullptr;
      d.As = prec == kF32 ? (void*)d.Af : take(A * 2);
      d.Bs = take(A * esz);
      const int split = std::max(d.gram_split, d.a2_split);
      d.part = split > 1 ? (float*)take((size_t)q.syrk * split * bt * bt * 4) : nullptr;
      d.red = (double*)take((size_t)q.prep * 12 + 16);
      d.scal = (float*)take(kScN * 4);
      d.cnt = (uint32_t*)take(64);  // reserved
      d.trp = (float*)take((size_t)q.syrk * 2 * 4);
      // e4m3 operand copies of the FP8 steps (256 tile)
      if (q8) {
        d.Xq = (uint8_t*)take(X);
        d.Aq = (uint8_t*)take(A);
      }
      if (o->fast_restart > 0)
        for (int k = 0; k < 6; ++k) d.fb[k] = (float*)take(A * 4);
      if (o->spectral_init > 0 && !learned) d.vec = (float*)take(((size_t)2 * q.sp + q.Lp) * 4);
      if (learned) {
        int32_t* rec = ws ? (int32_t*)(ws + L->sel_off) + (size_t)i * kSelWords : nullptr;
        d.selp = rec;
        d.flagp = rec ? rec + 1 : nullptr;
        d.feat = rec ? (float*)(rec + 16) : nullptr;
        d.est = rec ? (float*)(rec + 32) : nullptr;
        d.A2f = (float*)take(A * 4);
        d.mom = (float*)take((size_t)q.syrk * 4 * 4);
        d.vec = (float*)take(((size_t)2 * q.sp + q.Lp) * 4);
      }
    }
    L->descs.push_back(d);
    // this matrix's items in its class's tables, none in the others
    auto push = [&](int ph, int n) {
      for (int c = 0; c < kNCls; ++c) L->offs[ph][c].push_back(L->offs[ph][c].back() + (c == q.cls ? n : 0));
    };
    auto push_all = [&](int ph, int n) {
      for (int c = 0; c < kNCls; ++c) L->offs[ph][c].push_back(L->offs[ph][c].back() + (c == 0 ? n : 0));
    };
    push(PH_PREP, q.syrk ? q.prep : 0);
    push(PH_GRAM, q.syrk ? q.syrk * d.gram_split : 0);
    push(PH_A2, q.syrk ? q.syrk * d.a2_split : 0);
    push(PH_UPD, q.syrk ? q.upd : 0);
    // spectrum-aware init: power-method rows, four per item
    push(PH_PW, (q.syrk && o->spectral_init > 0) ? (int)((q.sp + 3) / 4) : 0);
    // fast rectangular iteration: unsplit upper-triangle tiles
    push(PH_FSYRK, (q.syrk && o->fast_restart > 0) ? q.syrk : 0);
    push(PH_RGRAM, (q.syrk && d.gram_split > 1) ? q.syrk : 0);
    push(PH_RA2, (q.syrk && d.a2_split > 1) ? q.syrk : 0);
    push(PH_COMBINE, (q.syrk && learned) ? (int)q.sp : 0);
    // quantisation passes: 16384 elements per item (sizes are multiples of 65536)
    push(PH_QX, (q.syrk && q8) ? (int)((size_t)q.sp * q.Lp / 16384) : 0);
    push(PH_QA, (q.syrk && q8) ? (int)((size_t)q.sp * q.sp / 16384) : 0);
    // power iteration: w = X^T v (length L), then y = X w (length s); a product
    // along the rows of the caller's m x n output takes one wave per row (4 per
    // block), one across its columns 64 columns per block
    {
      const bool t = m.m > m.n;
      const int rows4 = (int)((m.m + 3) / 4), cols64 = (int)((m.n + 63) / 64);
      push_all(PH_EST_A, (q.syrk && learned) ? (t ? rows4 : cols64) : 0);
      push_all(PH_EST_B, (q.syrk && learned) ? (t ? cols64 : rows4) : 0);
    }
  }
  // the first update reads X_0 from its bf16 copy only when every bf16-path
  // matrix of the call can (one kernel per launch, no per-matrix branch)
  {
    bool all = true;
    for (size_t i = 0; i < L->descs.size(); ++i)
      if (L->prec[i] != kF32 && L->descs[i].syrk_nt > 0) all = all && L->descs[i].x0b;
    for (auto& d : L->descs) d.x0b = all ? d.x0b : 0;
    L->x0b = all;
  }
  for (int c = 0; c < kNCls; ++c) {
    // Gram phase in longest-k-first matrix order (stable)
    std::vector<int32_t> ord(count);
    for (int i = 0; i < count; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return sh[x].Lp > sh[y].Lp; });
    std::vector<int32_t> o2(1, 0);
    for (int k = 0; k < count; ++k) {
      const int i = ord[k];
      o2.push_back(o2.back() + (L->offs[PH_GRAM][c][i + 1] - L->offs[PH_GRAM][c][i]));
    }
    L->offs[PH_GRAM][c].swap(o2);
    L->ord_gram[c].swap(ord);
  }
  for (int p = 0; p < PH_N; ++p)
    for (int c = 0; c < kNCls; ++c) L->totals[p][c] = L->offs[p][c].back();
  L->bytes = off;
  return PE_OK;
}

// Items of a phase over all classes (zero: nothing to launch).
int32_t phase_total(const Layout& L, int ph) {
  int32_t t = 0;
  for (int c = 0; c < kNCls; ++c) t += L.totals[ph][c];
  return t;
}

pe_status validate(int count, const pe_matrix* mats, const pe_opts* o) {
  if (count < 0 || (count > 0 && !mats)) return PE_EINVAL;
  if (count > 100000) return PE_EINVAL;
  pe_status st = check_opts(o);
  if (st != PE_OK) return st;
  bool muon = false;
  for (int i = 0; i < count; ++i) {
    if (!valid_matrix(mats[i])) return PE_EINVAL;
    muon = muon || mats[i].M || mats[i].W;
  }
  // the fallback re-run would apply the momentum and the weight step twice,
  // and its estimate reads X
  if (muon && learned_mode(o) && o->fallback_tau > 0.0f) return PE_EUNSUPPORTED;
  return PE_OK;
}

// Copy host words to device memory through kernel arguments (stream-ordered).
pe_status put_words(void* dst, const void* src, size_t bytes, hipStream_t st) {
  const uint32_t* w = (const uint32_t*)src;
  size_t nw = (bytes + 3) / 4;
  uint32_t* d = (uint32_t*)dst;
  while (nw > 0) {
    PutChunk c;
    memset(&c, 0, sizeof c);
    const int n = (int)std::min<size_t>(nw, kPutWords);
    c.dst = d;
    c.nwords = n;
    memcpy(c.w, w, (size_t)n * 4);
    hipError_t e = launch_put(c, st);
    if (e != hipSuccess) return hip_fail(e, "upload");
    d += n;
    w += n;
    nw -= n;
  }
  return PE_OK;
}

}  // namespace

struct pe_plan {
  int count = 0;
  int fp8_steps = 0;   // leading steps whose Gram-side products take e4m3 operands
  int T = 0;
  int norm_mode = 0;
  float muon_beta = 0.0f, muon_lr = 0.0f, muon_wd = 0.0f;
  int spectral_init = 0;    // > 0: power steps of the spectrum-aware init step
  int t0 = 0;               // kernel steps before the schedule (1 with the init step)
  int fast_restart = 0;     // > 0: Algorithm 4 in segments of this many steps
  float fast_eps = 0.0f;
  std::vector<float> abc;
  bool learned = false;
  const float* mlp = nullptr;
  int force_class = -1;
  float tau = 0.0f;
  float* d_coef = nullptr;     // [classes][T][3]
  int32_t* d_steps = nullptr;  // [classes]: T' of each class
  Layout L;
  MatDesc* d_descs = nullptr;
  int32_t* d_offs = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

pe_status upload(pe_plan* p, char* ws, hipStream_t st) {
  p->d_descs = (MatDesc*)(ws + p->L.descs_off);
  p->d_offs = (int32_t*)(ws + p->L.offs_off);
  pe_status s = put_words(p->d_descs, p->L.descs.data(), sizeof(MatDesc) * p->L.descs.size(), st);
  if (s != PE_OK) return s;
  std::vector<int32_t> offs;
  for (int ph = 0; ph < PH_N; ++ph)
    for (int c = 0; c < kNCls; ++c) offs.insert(offs.end(), p->L.offs[ph][c].begin(), p->L.offs[ph][c].end());
  for (int c = 0; c < kNCls; ++c) offs.insert(offs.end(), p->L.ord_gram[c].begin(), p->L.ord_gram[c].end());
  s = put_words(p->d_offs, offs.data(), offs.size() * 4, st);
  if (s != PE_OK || !p->learned) return s;
  // schedule table of the classes (class 4 is the caller's schedule), rows
  // past a class's T' the identity step (1, 0, 0); then the classes' T'
  const size_t nt = (size_t)kClasses * p->T * 3;
  std::vector<uint32_t> tab(nt + kClasses);
  float* ft = (float*)tab.data();
  std::vector<double> abc(3 * (size_t)p->T);
  for (int c = 0; c < kClasses; ++c) {
    const int steps = class_steps(c, p->T);
    if (c != kFixedClass) {
      // the first T' steps of the greedy T-step schedule are its T'-step schedule
      s = pe_coeffs(kClassTable[c].ell, p->T, nullptr, abc.data(), nullptr, nullptr, nullptr);
      if (s != PE_OK) return s;
    }
    for (int t = 0; t < p->T; ++t)
      for (int k = 0; k < 3; ++k) {
        const float v = t >= steps ? (k == 0 ? 1.0f : 0.0f)
                                   : (c == kFixedClass ? p->abc[3 * t + k] : (float)abc[3 * t + k]);
        ft[((size_t)c * p->T + t) * 3 + k] = v;
      }
    ((int32_t*)tab.data())[nt + c] = steps;
  }
  p->d_coef = (float*)(ws + p->L.coef_off);
  p->d_steps = (int32_t*)(p->d_coef + nt);
  return put_words(p->d_coef, tab.data(), tab.size() * 4, st);
}

KArgs base_args(const pe_plan* p) {
  KArgs a;
  memset(&a, 0, sizeof a);
  a.descs = p->d_descs;
  a.count = p->count;
  a.norm_mode = p->norm_mode;
  a.tmax = p->T;
  a.mbeta = p->muon_beta;
  a.mlr = p->muon_lr;
  a.mwd = p->muon_wd;
  if (p->learned) {
    a.sel_coef = p->d_coef;
    a.sel_steps = p->d_steps;
    a.mlp = p->mlp;
    a.force_class = p->force_class;
    a.fixed_class = kFixedClass;
    a.tau = p->tau;
  }
  return a;
}

const int32_t* offs_ptr(const pe_plan* p, int ph, int c) {
  return p->d_offs + ((size_t)ph * kNCls + c) * (p->count + 1);
}

void set_phase(const pe_plan* p, KArgs* a, int ph, int c) {
  a->offs = offs_ptr(p, ph, c);
  a->ord = ph == PH_GRAM ? p->d_offs + (size_t)PH_N * kNCls * (p->count + 1) + (size_t)c * p->count : nullptr;
  a->total = p->L.totals[ph][c];
}

// kernel step t: the init step (t < t0) or schedule step t - t0
void set_step(const pe_plan* p, KArgs* a, int t) {
  a->t = t;
  a->last = t == p->T + p->t0 - 1;
  if (t < p->t0) {
    a->init_step = 1;
    a->a = a->b = a->c = 0.0f;  // (a, b) per matrix from the power bound; c = 0
    return;
  }
  a->a = p->abc[3 * (t - p->t0) + 0];
  a->b = p->abc[3 * (t - p->t0) + 1];
  a->c = p->abc[3 * (t - p->t0) + 2];
}

pe_status enqueue_norm(const pe_plan* p, hipStream_t st, int fallback = 0) {
  KArgs a = base_args(p);
  a.fallback = fallback;
  hipError_t e;
  for (int c = 0; c < kNCls; ++c) {
    if (!p->L.totals[PH_PREP][c]) continue;
    set_phase(p, &a, PH_PREP, c);
    if ((e = launch_prep(cls_prec(c), a, kPrepGridCap, st)) != hipSuccess) return hip_fail(e, "prep launch");
  }
  if ((e = launch_finalize(a, st)) != hipSuccess) return hip_fail(e, "finalize launch");
  return PE_OK;
}

// kind: 0 Gram, 1 A^2 + combine, 2 update; one launch (plus its split-K
// reduction) per class present
pe_status enqueue_gemm(const pe_plan* p, int t, int kind, hipStream_t st, int fallback = 0) {
  static const int ph_main[3] = {PH_GRAM, PH_A2, PH_UPD};
  static const int ph_red[3] = {PH_RGRAM, PH_RA2, -1};
  static const char* names[3] = {"gram launch", "a2 launch", "update launch"};
  for (int c = 0; c < kNCls; ++c) {
    if (!p->L.totals[ph_main[kind]][c]) continue;
    const int bt = cls_bt(c);
    KArgs a = base_args(p);
    set_step(p, &a, t);
    set_phase(p, &a, ph_main[kind], c);
    // e4m3 Gram-side products in the first fp8_steps steps, bf16 matrices only
    const bool q = cls_prec(c) == kBF16;
    a.fp8 = q && t < p->fp8_steps;
    a.fp8_next = q && t + 1 < p->fp8_steps;
    a.fallback = fallback;
    a.x0b = kind == 2 && t == 0 && p->L.x0b;
    // learned path, step 1: A^2 and its moments are kept until the class is chosen
    a.raw_a2 = p->learned && !fallback && t == 0 && kind == 1;
    // Gram-side products of the FP8 steps run the e4m3 kernels; updates stay bf16
    const int prec = (a.fp8 && kind != 2) ? kFP8 : cls_prec(c);
    hipError_t e;
    if (prec == kFP8 && bt == kTileLarge) {
      // the 256 tile reads e4m3 copies: quantise X_t (or A_t) with its scale first
      set_phase(p, &a, kind == 0 ? PH_QX : PH_QA, c);
      if ((e = launch_quant(kind, a, kQuantGridCap, st)) != hipSuccess) return hip_fail(e, "quantisation launch");
      set_phase(p, &a, ph_main[kind], c);
    }
    e = launch_gemm(prec, bt, kind, a, bt == kTileLarge ? kGemmGridCapLarge : kGemmGridCap, st);
    if (e != hipSuccess) return hip_fail(e, names[kind]);
    if (ph_red[kind] >= 0 && p->L.totals[ph_red[kind]][c]) {
      set_phase(p, &a, ph_red[kind], c);
      if ((e = launch_reduce(prec, bt, kind, a, kReduceGridCap, st)) != hipSuccess)
        return hip_fail(e, "split-k reduce");
    }
  }
  return PE_OK;
}

// learned path between step 1's A^2 and its update: choose the class, form B
pe_status enqueue_select(const pe_plan* p, hipStream_t st) {
  KArgs a = base_args(p);
  set_step(p, &a, 0);
  hipError_t e = launch_select(a, st);
  if (e != hipSuccess) return hip_fail(e, "select launch");
  for (int c = 0; c < kNCls; ++c) {
    if (!p->L.totals[PH_COMBINE][c]) continue;
    set_phase(p, &a, PH_COMBINE, c);
    if ((e = launch_combine(cls_prec(c), a, st)) != hipSuccess) return hip_fail(e, "combine launch");
  }
  return PE_OK;
}

// Algorithm 4 in segments of fast_restart steps (FP32 class only): per
// segment the Gram matrix, then per step B_t, D_t and (but for the last step)
// R_{t+1}, and the update X <- q X + D X; see gemm_fast_kernel.
pe_status enqueue_fast(const pe_plan* p, hipStream_t st) {
  pe_status s = enqueue_norm(p, st, 0);
  if (s != PE_OK) return s;
  const int c = cls_of(kF32, kTileSmall);
  hipError_t e;
  // kind 0: Gram of X, 1: symmetric product of two fb buffers
  auto product = [&](int kind, int fp_, int fq_, int fe1, float c1, int fe2, float c2, float cacc,
                     int fout, float cdiag, int fscale, int seg) -> pe_status {
    KArgs a = base_args(p);
    set_phase(p, &a, PH_FSYRK, c);
    a.t = seg;
    a.fast = 1;
    a.fp_ = fp_;
    a.fq_ = fq_;
    a.fe1 = fe1;
    a.fe2 = fe2;
    a.c1 = c1;
    a.c2 = c2;
    a.cacc = cacc;
    a.fout = fout;
    a.cdiag = cdiag;
    a.fscale = fscale;
    if ((e = launch_fast(kind, a, kGemmGridCap, st)) != hipSuccess) return hip_fail(e, "fast product");
    return PE_OK;
  };
  int seg = 0;
  for (int t0 = 0; t0 < p->T; t0 += p->fast_restart, ++seg) {
    const int k = std::min(p->fast_restart, p->T - t0);
    int r = kFbR0, dcur = kFbD0;
    // Y = X X^T (sigma^2 G G^T in the first segment, plus eps I)
    if ((s = product(0, -1, -1, kFbNone, 0.f, kFbNone, 0.f, 1.f, r, seg == 0 ? p->fast_eps : 0.f,
                     seg == 0, seg)) != PE_OK) return s;
    float q = 1.0f;
    for (int j = 0; j < k; ++j) {
      const float a = p->abc[3 * (t0 + j)], b = p->abc[3 * (t0 + j) + 1], cc = p->abc[3 * (t0 + j) + 2];
      // B_t = b R + c R^2 (into D directly on the segment's first step, D_1 = B_1)
      const int bdst = j == 0 ? dcur : kFbB;
      if ((s = product(1, r, r, r, b, kFbNone, 0.f, cc, bdst, 0.f, 0, seg)) != PE_OK) return s;
      if (j > 0) {
        const int dn = dcur == kFbD0 ? kFbD1 : kFbD0;
        if ((s = product(1, dcur, kFbB, dcur, a, kFbB, q, 1.f, dn, 0.f, 0, seg)) != PE_OK) return s;
        dcur = dn;
      }
      if (j + 1 < k) {
        const int rn = r == kFbR0 ? kFbR1 : kFbR0;
        if ((s = product(1, r, bdst, kFbNone, 0.f, kFbNone, 0.f, 1.f, kFbP, 0.f, 0, seg)) != PE_OK) return s;
        if ((s = product(1, kFbP, bdst, r, a * a, kFbP, 2.f * a, 1.f, rn, 0.f, 0, seg)) != PE_OK) return s;
        r = rn;
      }
      q *= a;
    }
    // X <- q X + D X
    KArgs u = base_args(p);
    set_phase(p, &u, PH_UPD, c);
    u.t = seg;
    u.last = t0 + k >= p->T;
    u.a = q;
    u.b = u.c = 0.0f;
    u.fast = 1;
    u.fp_ = dcur;
    if ((e = launch_gemm(kF32, kTileSmall, 2, u, kGemmGridCap, st)) != hipSuccess)
      return hip_fail(e, "fast update");
  }
  return PE_OK;
}

// power method on each matrix's step-1 Gram matrix and the init coefficients
pe_status enqueue_power(const pe_plan* p, hipStream_t st) {
  KArgs a = base_args(p);
  hipError_t e;
  if ((e = launch_power(kF32, 0, a, st)) != hipSuccess) return hip_fail(e, "power init");
  for (int it = 0; it < p->spectral_init; ++it) {
    for (int c = 0; c < kNCls; ++c) {
      if (!p->L.totals[PH_PW][c]) continue;
      set_phase(p, &a, PH_PW, c);
      if ((e = launch_power(cls_prec(c), 1, a, st)) != hipSuccess) return hip_fail(e, "power matvec");
    }
    a.last = it == p->spectral_init - 1;
    if ((e = launch_power(kF32, 2, a, st)) != hipSuccess) return hip_fail(e, "power norm");
  }
  return PE_OK;
}

pe_status enqueue_steps(const pe_plan* p, hipStream_t st, int fallback) {
  if (p->fast_restart > 0) return enqueue_fast(p, st);
  pe_status s = enqueue_norm(p, st, fallback);
  if (s != PE_OK) return s;
  for (int t = 0; t < p->T + p->t0; ++t)
    for (int kind = 0; kind < 3; ++kind) {
      if (t < p->t0 && kind == 1 && (s = enqueue_power(p, st)) != PE_OK) return s;
      if ((s = enqueue_gemm(p, t, kind, st, fallback)) != PE_OK) return s;
      if (p->learned && !fallback && t == 0 && kind == 1 && (s = enqueue_select(p, st)) != PE_OK)
        return s;
    }
  return PE_OK;
}

pe_status enqueue(const pe_plan* p, hipStream_t st) {
  if (phase_total(p->L, PH_PREP) == 0) return PE_OK;
  pe_status s = enqueue_steps(p, st, 0);
  if (s != PE_OK || !p->learned || !(p->tau > 0.0f)) return s;
  // estimate ||X X^T - I||_2 of every result; re-run the failed ones with class 4
  KArgs a = base_args(p);
  hipError_t e = launch_est(a, kEstIters, st, offs_ptr(p, PH_EST_A, 0), p->L.totals[PH_EST_A][0],
                            offs_ptr(p, PH_EST_B, 0), p->L.totals[PH_EST_B][0]);
  if (e != hipSuccess) return hip_fail(e, "estimate launch");
  return enqueue_steps(p, st, 1);
}

pe_status plan_init(pe_plan* p, int count, const pe_matrix* mats, const pe_opts* o, void* ws,
                    size_t ws_bytes, hipStream_t st) {
  pe_status s = validate(count, mats, o);
  if (s != PE_OK) return s;
  p->count = count;
  p->fp8_steps = o->compute == PE_COMPUTE_FP8 ? o->fp8_steps : 0;
  p->T = o->T;
  p->norm_mode = o->norm_mode;
  p->spectral_init = o->spectral_init;
  p->t0 = o->spectral_init > 0 ? 1 : 0;
  p->muon_beta = o->muon_beta;
  p->muon_lr = o->muon_lr;
  p->muon_wd = o->muon_wd;
  p->fast_restart = o->fast_restart;
  p->fast_eps = o->fast_eps;
  p->abc.resize(3 * o->T);
  for (int i = 0; i < 3 * o->T; ++i) p->abc[i] = (float)o->abc[i];
  p->learned = learned_mode(o);
  p->mlp = o->predictor;
  p->force_class = o->force_class;
  p->tau = o->fallback_tau;
  Layout sizing;
  build_layout(count, mats, o, nullptr, &sizing);
  if (phase_total(sizing, PH_PREP) == 0) return PE_OK;  // nothing but empty matrices
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < sizing.bytes) return PE_EWORKSPACE;
  build_layout(count, mats, o, (char*)ws, &p->L);
  warm_launch_grids();
  return upload(p, (char*)ws, st);
}

}  // namespace

// ------------------------------------------------ allocation-free entry point
// pe_polar_noalloc keeps its workspace in this file-scope device array instead
// of the caller's: one copy per device, allocated when the code object is
// loaded there and held until the process ends.  In host code `scratch` is
// only a stand-in for the symbol; its device address comes from
// hipGetSymbolAddress, queried once per device (with that device current) and
// cached.
static __device__ __align__(256) char scratch[PE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

pe_status scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) {
    g_last_error = "device index beyond the scratch table";
    return PE_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PE_OK;
}
}  // namespace

// ----------------------------------------------------------------- C ABI
extern "C" {

size_t pe_workspace_size(int32_t count, const pe_matrix* mats, const pe_opts* opts) {
  if (validate(count, mats, opts) != PE_OK) return 0;
  Layout L;
  build_layout(count, mats, opts, nullptr, &L);
  return L.bytes;
}

pe_status pe_polar_batched(int32_t count, const pe_matrix* mats, const pe_opts* opts, void* ws,
                           size_t ws_bytes, void* stream) {
  g_last_error.clear();
  hipStream_t st = (hipStream_t)stream;
  pe_plan p;
  pe_status s = plan_init(&p, count, mats, opts, ws, ws_bytes, st);
  if (s != PE_OK) return s;
  return enqueue(&p, st);
}

pe_status pe_polar(const pe_matrix* mat, const pe_opts* opts, void* ws, size_t ws_bytes, void* stream) {
  if (!mat) return PE_EINVAL;
  return pe_polar_batched(1, mat, opts, ws, ws_bytes, stream);
}

pe_status pe_polar_noalloc(const pe_matrix* mat, const pe_opts* opts, void* stream) {
  g_last_error.clear();
  if (!mat) return PE_EINVAL;
  pe_status s = validate(1, mat, opts);
  if (s != PE_OK) return s;
  Layout sizing;
  build_layout(1, mat, opts, nullptr, &sizing);
  if (sizing.bytes > (size_t)PE_NOALLOC_SCRATCH_BYTES) {
    char buf[160];
    snprintf(buf, sizeof buf, "pe_polar_noalloc: this matrix needs %zu bytes of workspace, the static "
             "scratch holds %zu", sizing.bytes, (size_t)PE_NOALLOC_SCRATCH_BYTES);
    g_last_error = buf;
    return PE_EWORKSPACE;
  }
  void* ws = nullptr;
  if ((s = scratch_address(&ws)) != PE_OK) return s;
  return pe_polar(mat, opts, ws, (size_t)PE_NOALLOC_SCRATCH_BYTES, stream);
}

pe_status pe_plan_create(int32_t count, const pe_matrix* mats, const pe_opts* opts, void* ws,
                         size_t ws_bytes, void* stream, pe_plan** plan) {
  g_last_error.clear();
  if (!plan) return PE_EINVAL;
  *plan = nullptr;
  pe_plan* p = new pe_plan();
  pe_status s = plan_init(p, count, mats, opts, ws, ws_bytes, (hipStream_t)stream);
  if (s != PE_OK) {
    delete p;
    return s;
  }
  *plan = p;
  return PE_OK;
}

pe_status pe_plan_launch(pe_plan* p, void* stream, int32_t use_graph) {
  g_last_error.clear();
  if (!p) return PE_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (!use_graph) return enqueue(p, st);
  hipError_t e;
  if (!p->exec) {
    // capture on a private stream (the caller's may be the legacy default stream)
    if ((e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "capture stream");
    // order the capture after the caller's pending work (tables were uploaded there)
    if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "sync before capture");
    if ((e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(e, "begin capture");
    pe_status s = enqueue(p, p->cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(p->cap_stream, &g);
    if (s != PE_OK) {
      if (g) hipGraphDestroy(g);
      return s;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    p->graph = g;
    if ((e = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
      p->exec = nullptr;
      return hip_fail(e, "graph instantiate");
    }
  }
  if ((e = hipGraphLaunch(p->exec, st)) != hipSuccess) return hip_fail(e, "graph launch");
  return PE_OK;
}

pe_status pe_plan_launch_phase(pe_plan* p, int32_t step, int32_t phase, void* stream) {
  g_last_error.clear();
  if (!p || step < 0 || step >= p->T + p->t0 || phase < 0 || phase > 3) return PE_EINVAL;
  // a learned plan's step 1 also selects the class between its phases
  if (p->learned) return PE_EUNSUPPORTED;
  if (phase_total(p->L, PH_PREP) == 0) return PE_OK;
  hipStream_t st = (hipStream_t)stream;
  if (phase == 0) return enqueue_norm(p, st);
  return enqueue_gemm(p, step, phase - 1, st);
}

pe_status pe_plan_destroy(pe_plan* p) {
  if (!p) return PE_OK;
  if (p->exec) hipGraphExecDestroy(p->exec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->cap_stream) hipStreamDestroy(p->cap_stream);
  delete p;
  return PE_OK;
}

pe_status pe_plan_selection(pe_plan* p, void* stream, int32_t* classes, float* feats, float* est,
                            int32_t* flags) {
  g_last_error.clear();
  if (!p) return PE_EINVAL;
  if (!p->learned) return PE_EINVAL;
  if (p->count == 0) return PE_OK;
  hipStream_t st = (hipStream_t)stream;
  std::vector<int32_t> rec((size_t)p->count * kSelWords);
  const char* src = (const char*)p->d_descs - p->L.descs_off + p->L.sel_off;
  hipError_t e = hipMemcpyAsync(rec.data(), src, rec.size() * 4, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(e, "selection copy");
  for (int i = 0; i < p->count; ++i) {
    const int32_t* r = rec.data() + (size_t)i * kSelWords;
    const bool run = p->L.descs[i].syrk_nt > 0;  // empty matrices have no record
    if (classes) classes[i] = run ? r[0] : -1;
    if (flags) flags[i] = run ? r[1] : 0;
    if (feats) {
      if (run) memcpy(feats + (size_t)i * kFeat, r + 16, kFeat * 4);
      else memset(feats + (size_t)i * kFeat, 0, kFeat * 4);
    }
    if (est) est[i] = run ? *(const float*)(r + 32) : 0.0f;
  }
  return PE_OK;
}

size_t pe_mlp_workspace_size(int32_t B) {
  if (B <= 0) return 0;
  const size_t nblk = (size_t)(B + 63) / 64;
  return align_up(nblk * kMlpParams * 4) + align_up(nblk * 4);
}

pe_status pe_mlp_forward(const float* params, const float* feats, int32_t B, float* logits,
                         void* stream) {
  g_last_error.clear();
  if (B < 0 || (B > 0 && (!params || !feats || !logits))) return PE_EINVAL;
  if (B == 0) return PE_OK;
  hipError_t e = launch_mlp_forward(params, feats, B, logits, (hipStream_t)stream);
  return e == hipSuccess ? PE_OK : hip_fail(e, "mlp forward");
}

static pe_status mlp_grad_common(const float* params, const float* feats, const int32_t* labels,
                                 int32_t B, float* grad, float* loss, float* upd, float* m, float* v,
                                 int32_t step, float lr, void* ws, size_t ws_bytes, void* stream) {
  g_last_error.clear();
  if (B <= 0 || !params || !feats || !labels) return PE_EINVAL;
  const size_t need = pe_mlp_workspace_size(B);
  if (!ws || ((uintptr_t)ws & 255) || ws_bytes < need) return PE_EWORKSPACE;
  const size_t nblk = (size_t)(B + 63) / 64;
  float* part = (float*)ws;
  float* part_loss = (float*)((char*)ws + align_up(nblk * kMlpParams * 4));
  hipError_t e = launch_mlp_grad(params, feats, labels, B, part, part_loss, grad, loss, upd, m, v,
                                 step, lr, (hipStream_t)stream);
  return e == hipSuccess ? PE_OK : hip_fail(e, "mlp grad");
}

pe_status pe_mlp_grad(const float* params, const float* feats, const int32_t* labels, int32_t B,
                      float* grad, float* loss, void* ws, size_t ws_bytes, void* stream) {
  if (!grad) return PE_EINVAL;
  return mlp_grad_common(params, feats, labels, B, grad, loss, nullptr, nullptr, nullptr, 0, 0.0f,
                         ws, ws_bytes, stream);
}

pe_status pe_mlp_train_step(float* params, float* m, float* v, int32_t step, float lr,
                            const float* feats, const int32_t* labels, int32_t B, float* loss,
                            void* ws, size_t ws_bytes, void* stream) {
  if (!m || !v || step < 1 || !(lr > 0.0f) || !std::isfinite(lr)) return PE_EINVAL;
  return mlp_grad_common(params, feats, labels, B, nullptr, loss, params, m, v, step, lr, ws,
                         ws_bytes, stream);
}

pe_status pe_quantize_e4m3(const void* x, int32_t x_dtype, void* q, int64_t n, float scale,
                           void* stream) {
  g_last_error.clear();
  if (n < 0 || (n > 0 && (!x || !q)) || (x_dtype != PE_F32 && x_dtype != PE_BF16)) return PE_EINVAL;
  if (!(scale > 0.0f) || !std::isfinite(scale)) return PE_EINVAL;
  if (n == 0) return PE_OK;
  hipError_t e = launch_quantize(x, x_dtype == PE_BF16, (uint8_t*)q, n, scale, (hipStream_t)stream);
  return e == hipSuccess ? PE_OK : hip_fail(e, "quantize launch");
}

int32_t pe_tile_count(void) { return 3; }

const char* pe_tile_name(int32_t tile_id) {
  switch (tile_id) {
    case 0: return "auto";
    case 1: return "bt128_w2x2_mfma16";
    case 2: return "bt256_w2x2_mfma32";
  }
  return nullptr;
}

pe_status pe_tile_table_load(const char* path) {
  if (!path) return PE_EINVAL;
  FILE* f = fopen(path, "r");
  if (!f) return PE_EINVAL;
  std::map<std::string, int> tab;
  char line[256];
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#' || line[0] == '\n') continue;
    char cls[128];
    int id = 0;
    if (sscanf(line, "%127s %d", cls, &id) != 2 || id < 1 || id > 2) {
      fclose(f);
      return PE_EINVAL;
    }
    tab[cls] = id;
  }
  fclose(f);
  std::lock_guard<std::mutex> lk(g_tab_mu);
  g_tile_table.swap(tab);
  return PE_OK;
}

const char* pe_shape_class(int32_t compute, int64_t m, int64_t n) {
  thread_local std::string s;
  if (m <= 0 || n <= 0) return "";
  s = shape_class(compute == PE_COMPUTE_F32 ? kF32 : kBF16, std::min(m, n), std::max(m, n));
  return s.c_str();
}

const char* pe_status_string(pe_status st) {
  switch (st) {
    case PE_OK: return "ok";
    case PE_EINVAL: return "invalid argument";
    case PE_EUNSUPPORTED: return "unsupported in this build";
    case PE_ENOCONV: return "Remez exchange did not converge";
    case PE_EWORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    case PE_EHIP: return "HIP runtime error";
  }
  return "unknown status";
}

const char* pe_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
