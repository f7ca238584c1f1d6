// gfx950 kernels of the Polar Express online stage (Section 3.5 and the
// Appendix A.1 listing: X_0 = G / (1.01 ||G||_F + 1e-7); per step
// A = X X^T, B = b A + c A^2, X = a X + B X).
//
// Kernels, each launched once per phase over the items of every matrix of a
// call ("grouped" launches; a single matrix is a group of one), each walking
// its items in a grid-stride loop:
//   prep_kernel   one HBM pass over G: orientation, sum of squares (FP32 per
//                 lane and item, FP64 fixed-order sum of the items' partials
//                 => deterministic),
//                 max |G|, and the unscaled copies of X_0 (bf16 paths: the bf16
//                 copy, plus an FP32 master unless the bf16 copy is exact;
//                 FP32 path: X_0 and X_0^T); the scale sigma is folded into
//                 step 1's epilogues (A_1 = sigma^2 G G^T, X_1 = sigma (a G +
//                 B_1 G)).
//   gemm_kernel   persistent blocks over block tiles of 128 (4 waves, 16x16x32
//                 MFMA, two blocks per CU) or 256 (8 waves in 2 x 4, 32x32x16
//                 MFMA, one block per CU); bf16 operands go from HBM straight
//                 into a four-stage LDS ring, FP32 accumulation.
//                 KIND_GRAM:  A = X X^T, upper-triangle tiles only, mirrored
//                             store (SYRK);
//                 KIND_A2:    B = b A + c A A^T (A symmetric, so A^2 = A A^T is
//                             again a SYRK), epilogue re-reads A;
//                 KIND_UPD:   X = a X + B X; the bf16 paths read X_t itself
//                             (k along its rows) with transposing LDS reads,
//                             the FP32 path reads X^T; writes the FP32 master
//                             and the other bf16 copy (FP32 path: the next
//                             X^T), or the caller's output on the last step
//                             (KIND_UPD_LAST); KIND_UPD0 is the first update
//                             reading X_0 from its exact bf16 copy.
//                 In the e4m3 steps the Gram-side products read e4m3 copies
//                 (quant_kernel) on the 256 tile, or convert bf16 operands
//                 while staging them on the 128 tile.
//                 Split-K for the Gram-side products writes partial tiles;
//                 splitk_reduce_kernel sums them in split order (deterministic)
//                 and runs the same epilogue.
// The Gram-side GEMMs are "NT": C[i][j] = sum_k P[i][k] Q[j][k] with both
// operands row-major along k, which is what the MFMA lane layout wants; the
// bf16 update's second operand is row-major along n and is transposed by
// the LDS reads.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "pe_device.h"

namespace pe {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef short i16x4 __attribute__((ext_vector_type(4)));

// Streaming (non-temporal) stores and loads, for data that a launch touches
// once: outputs that only later launches read should not displace from the L2
// the operand panels that neighbouring tiles of the same launch re-read.
template <typename T>
__device__ __forceinline__ void st_stream(T* p, T v) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void st_stream(uint2* p, uint2 v) {
  __builtin_nontemporal_store((u32x2){v.x, v.y}, (u32x2*)p);
}
// streaming only where S holds; an ordinary store otherwise
template <bool S, typename T>
__device__ __forceinline__ void st_hint(T* p, T v) {
  if constexpr (S) st_stream(p, v);
  else *p = v;
}

// KIND_UPD0: the first update when X_0 is exactly its bf16 copy (MatDesc::x0b)
enum Kind : int { KIND_GRAM = 0, KIND_A2 = 1, KIND_UPD = 2, KIND_UPD_LAST = 3, KIND_UPD0 = 4 };

// Descriptor pointers are generic; loads through these global-address-space
// views compile to global_load (not flat_load), which keeps vmcnt/lgkmcnt apart.
#define PE_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ const PE_GLOBAL T* gview(const T* p) {
  return (const PE_GLOBAL T*)p;
}
template <typename T>
__device__ __forceinline__ PE_GLOBAL T* gview_w(T* p) {
  return (PE_GLOBAL T*)p;
}

// ---------------------------------------------------------------- helpers
__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ int find_mat(const int32_t* offs, int count, int item) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offs[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}


// In the fallback re-run only the matrices whose estimate failed are recomputed.
__device__ __forceinline__ bool skip_matrix(const KArgs& args, const MatDesc& d) {
  return args.fallback && (d.flagp == nullptr || *d.flagp == 0);
}

// Learned path: the matrix's class schedule has ended (step t >= its T'); its
// kernels skip it, and the last step only copies X to the caller's output.
__device__ __forceinline__ bool past_schedule(const KArgs& args, const MatDesc& d) {
  if (!args.sel_steps || !d.selp) return false;
  int cls = *d.selp;
  if (cls < 0 || cls >= kClasses) cls = args.fixed_class;
  return args.t >= args.sel_steps[cls];
}

// bf16 operand copies of the iterate (bf16 / e4m3 paths): step t reads X_t
// from one of the two buffers, in the Gram product and as the k-rows of B X,
// while its update writes X_{t+1} into the other (every tile of the update
// reads all of X_t, so it cannot be overwritten in place)
__device__ __forceinline__ const uint16_t* xb_cur(const KArgs& args, const MatDesc& d) {
  return (const uint16_t*)((args.t & 1) ? d.Xb1 : d.Xb);
}
__device__ __forceinline__ uint16_t* xb_next(const KArgs& args, const MatDesc& d) {
  return (uint16_t*)((args.t & 1) ? d.Xb : d.Xb1);
}

__device__ __forceinline__ void step_coef(const KArgs& args, const MatDesc& d, float* a, float* b,
                                          float* c) {
  if (args.init_step) {
    // spectrum-aware init: the cubic chosen per matrix from its power bound
    *a = d.scal[kScInitA];
    *b = d.scal[kScInitB];
    *c = 0.0f;
  } else if (args.sel_coef) {
    // the class slot is written before any product that reads coefficients
    // (finalize: fixed class; select: the chosen one); an out-of-range value
    // still falls back to the fixed class instead of leaving the table
    int cls = *d.selp;
    if (cls < 0 || cls >= kClasses) cls = args.fixed_class;
    const float* p = args.sel_coef + ((size_t)cls * args.tmax + args.t) * 3;
    *a = p[0]; *b = p[1]; *c = p[2];
  } else {
    *a = args.a; *b = args.b; *c = args.c;
  }
}

// ------------------------------------------------------------------ prep
// One 64 x 64 tile of the oriented, padded X per iteration of the block loop.
// Thread t owns two 8-element row chunks of the source block (rows t/8 and
// t/8 + 32, columns 8*(t%8)..+8) and, after an LDS transpose, the matching
// chunks of the transposed block.  Each tile writes its own partial sum of
// squares (FP64) and max |G|; finalize_kernel reduces them in fixed order.
__device__ __forceinline__ void load8(const MatDesc& d, int gr, int gc, int srn, int scn, float (&v)[8]) {
  if (gr < srn && d.g_vec && gc + 8 <= scn) {
    const size_t off = (size_t)gr * d.ldg + gc;
    if (d.g_bf16) {
      const u32x4 c = *(const PE_GLOBAL u32x4*)(gview((const uint16_t*)d.G) + off);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        v[2 * e] = __uint_as_float(c[e] << 16);
        v[2 * e + 1] = __uint_as_float(c[e] & 0xffff0000u);
      }
    } else {
      const PE_GLOBAL f32x4* q = (const PE_GLOBAL f32x4*)(gview((const float*)d.G) + off);
      const f32x4 c0 = q[0], c1 = q[1];
#pragma unroll
      for (int e = 0; e < 4; ++e) { v[e] = c0[e]; v[4 + e] = c1[e]; }
    }
    return;
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    float x = 0.0f;
    if (gr < srn && gc + e < scn) {
      const size_t off = (size_t)gr * d.ldg + gc + e;
      x = d.g_bf16 ? bf2f(((const uint16_t*)d.G)[off]) : ((const float*)d.G)[off];
    }
    v[e] = x;
  }
}

template <int P>
__device__ __forceinline__ void store8_f32(float* dst, const float (&v)[8]) {
  st_stream((f32x4*)dst, f32x4{v[0], v[1], v[2], v[3]});
  st_stream((f32x4*)(dst + 4), f32x4{v[4], v[5], v[6], v[7]});
}
__device__ __forceinline__ void store8_bf16(uint16_t* dst, const float (&v)[8]) {
  u32x4 w;
#pragma unroll
  for (int e = 0; e < 4; ++e) w[e] = (uint32_t)f2bf(v[2 * e]) | ((uint32_t)f2bf(v[2 * e + 1]) << 16);
  st_stream((u32x4*)dst, w);
}

// row-major X row chunk: fp32 master (unless the bf16 copy holds X_0
// exactly) and (bf16 paths) the bf16 operand copy of X_0 (the first of the
// two buffers)
template <int P>
__device__ __forceinline__ void store_x_chunk(const MatDesc& d, size_t o, const float (&v)[8]) {
  if (P == kF32 || !d.x0b) store8_f32<P>(d.Xf + o, v);
  if (P != kF32) store8_bf16((uint16_t*)d.Xb + o, v);
}
// X^T chunk, the fp32 path's operand of B X: row n, columns i..i+7
__device__ __forceinline__ void store_xt_chunk(const MatDesc& d, int n, int i, const float (&v)[8]) {
  store8_f32<kF32>((float*)d.XT0 + (size_t)n * d.sp + i, v);
}

template <int P>
__global__ __launch_bounds__(kThreads) void prep_kernel(KArgs args) {
  __shared__ float tile[kPrepTile][kPrepTile + 1];
  __shared__ float red_s[kThreads / 64];
  __shared__ float red_f[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rr = tid >> 3, cc = (tid & 7) * 8;
  // one item = kPrepGroup consecutive 64 x 64 tiles (row-major tile order);
  // the partial sums of an item are reduced once, in a fixed order
  for (int item = blockIdx.x; item < args.total; item += gridDim.x) {
    const int mi = find_mat(args.offs, args.count, item);
    const MatDesc& d = args.descs[mi];
    if (skip_matrix(args, d)) continue;
    const int local = item - args.offs[mi];
    const int ntk = d.Lp / kPrepTile;
    const int srn = d.trans ? d.L : d.s, scn = d.trans ? d.s : d.L;
    // sum of squares in FP32 per lane and within the item; the items' partials
    // are summed across the matrix in FP64 (finalize_kernel)
    float ss = 0.0f;
    float amax = 0.0f;
#pragma unroll 1
    for (int u = 0; u < kPrepGroup; ++u) {
      const int tix = local * kPrepGroup + u;
      const int i0 = (tix / ntk) * kPrepTile;   // rows of X (s side)
      const int k0 = (tix % ntk) * kPrepTile;   // cols of X (L side)
      // source block in G's own layout
      const int sr0 = d.trans ? k0 : i0, sc0 = d.trans ? i0 : k0;
      float v[2][8];
#pragma unroll
      for (int j = 0; j < 2; ++j) load8(d, sr0 + rr + 32 * j, sc0 + cc, srn, scn, v[j]);
      if (d.M) {
        // Muon momentum (Section 1.1): M <- beta M + (1 - beta) G in place, and
        // the iteration runs on the new M (padding stays zero).  The thread's
        // 16 values are all loaded before any is stored (16-byte accesses when
        // the row chunk is inside the matrix and aligned).
        const bool mvec = ((uintptr_t)d.M % 16 == 0) && (d.ldm % 4 == 0);
        float mo[2][8];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int gr = sr0 + rr + 32 * j;
          const PE_GLOBAL float* mrow = gview(d.M) + (size_t)gr * d.ldm + sc0 + cc;
          if (gr < srn && mvec && sc0 + cc + 8 <= scn) {
            const f32x4 lo = *(const PE_GLOBAL f32x4*)mrow, hi = *(const PE_GLOBAL f32x4*)(mrow + 4);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              mo[j][e] = lo[e];
              mo[j][e + 4] = hi[e];
            }
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) mo[j][e] = (gr < srn && sc0 + cc + e < scn) ? mrow[e] : 0.0f;
          }
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int gr = sr0 + rr + 32 * j;
          PE_GLOBAL float* mrow = gview_w(d.M) + (size_t)gr * d.ldm + sc0 + cc;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            mo[j][e] = __builtin_fmaf(args.mbeta, mo[j][e], (1.0f - args.mbeta) * v[j][e]);
            if (gr < srn && sc0 + cc + e < scn) v[j][e] = mo[j][e];
          }
          if (gr < srn && mvec && sc0 + cc + 8 <= scn) {
            *(PE_GLOBAL f32x4*)mrow = (f32x4){mo[j][0], mo[j][1], mo[j][2], mo[j][3]};
            *(PE_GLOBAL f32x4*)(mrow + 4) = (f32x4){mo[j][4], mo[j][5], mo[j][6], mo[j][7]};
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e)
              if (gr < srn && sc0 + cc + e < scn) mrow[e] = mo[j][e];
          }
        }
      }
      // a transposed copy of the block goes through LDS: X itself when G is
      // tall, X^T on the fp32 path (the bf16 paths read X_0 row-major only)
      const bool transpose = P == kF32 || d.trans;
      if (transpose && u > 0) __syncthreads();  // the previous tile's transposed reads are done
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int r = rr + 32 * j;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          if (transpose) tile[r][cc + e] = v[j][e];
          ss = __builtin_fmaf(v[j][e], v[j][e], ss);
          amax = fmaxf(amax, fabsf(v[j][e]));
        }
        if (!d.trans) store_x_chunk<P>(d, (size_t)(i0 + r) * d.Lp + k0 + cc, v[j]);
        else if (P == kF32) store_xt_chunk(d, k0 + r, i0 + cc, v[j]);
      }
      if (transpose) {
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int q = rr + 32 * j;
          float w[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) w[e] = tile[cc + e][q];
          if (!d.trans) store_xt_chunk(d, k0 + q, i0 + cc, w);
          else store_x_chunk<P>(d, (size_t)(i0 + q) * d.Lp + k0 + cc, w);
        }
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      ss += __shfl_xor(ss, off);
      amax = fmaxf(amax, __shfl_xor(amax, off));
    }
    if (lane == 0) { red_s[wave] = ss; red_f[wave] = amax; }
    __syncthreads();
    if (tid == 0) {
      d.red[local] = (double)((red_s[0] + red_s[1]) + (red_s[2] + red_s[3]));
      ((float*)(d.red + d.n_prep))[local] = fmaxf(fmaxf(red_f[0], red_f[1]), fmaxf(red_f[2], red_f[3]));
    }
    __syncthreads();  // the next item's first tile reuses the LDS tile and the reduction slots
  }
}

// One block per matrix: fixed-order reduction of the tile partials (the same
// result for any launch geometry), then sigma = 1 / (1.01 ||G||_F + 1e-7)
// (or 1 / (||G||_F + 1e-2)); clears the amax slots the FP8 steps accumulate into.
__global__ __launch_bounds__(kThreads) void finalize_kernel(KArgs args) {
  __shared__ double red_d[kThreads / 64];
  __shared__ float red_f[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int mi = blockIdx.x; mi < args.count; mi += gridDim.x) {
    const MatDesc& d = args.descs[mi];
    if (d.n_prep == 0 || skip_matrix(args, d)) continue;
    double acc = 0.0;
    float am = 0.0f;
    const float* rf = (const float*)(d.red + d.n_prep);
    for (int i = tid; i < d.n_prep; i += kThreads) {
      acc += d.red[i];
      am = fmaxf(am, rf[i]);
    }
    for (int off = 32; off > 0; off >>= 1) {
      acc += __shfl_xor(acc, off);
      am = fmaxf(am, __shfl_xor(am, off));
    }
    __syncthreads();
    if (lane == 0) { red_d[wave] = acc; red_f[wave] = am; }
    __syncthreads();
    if (tid == 0) {
      const double tot = (red_d[0] + red_d[1]) + (red_d[2] + red_d[3]);
      const double fro = sqrt(tot);
      const double sigma = args.norm_mode == 1 ? 1.0 / (fro + 1e-2) : 1.0 / (1.01 * fro + 1e-7);
      d.scal[kScScale] = (float)sigma;
      d.scal[kScAmaxG] = fmaxf(fmaxf(red_f[0], red_f[1]), fmaxf(red_f[2], red_f[3]));
      d.scal[kScFro] = (float)fro;
    }
    for (int i = kScAmaxX + tid; i < kScN; i += kThreads) d.scal[i] = 0.0f;
    // learned path, first pass: the class slot holds the fixed class until the
    // selection kernel overwrites it, and no matrix is marked for the re-run
    if (d.selp && !args.fallback && tid == 0) {
      *d.selp = args.fixed_class;
      *d.flagp = 0;
    }
  }
}

// ------------------------------------------------------------- GEMM core
// Block tile BT x BT (BT = 128 or 256) of MFMA fragments F x F, F = BT/8:
//   F = 16: v_mfma_f32_16x16x32_bf16 / v_mfma_f32_16x16x4_f32
//   F = 32: v_mfma_f32_32x32x16_bf16 / v_mfma_f32_32x32x2_f32
// (the wave grid per path is WaveCfg below).  The register-staged FP32 loop
// (gemm_nt_tile, 4 waves in 2 x 2, each a (BT/2) x (BT/2) tile of 4 x 4
// fragments) keeps 128 bytes of k per LDS row (32 fp32) plus a 16-byte pad
// (bank spread), for both operands, in two double-buffered stages; a lane
// reads its fragment as one 16-byte chunk: rows lane % F, k-chunk lane / F
// within a sub-step of F == 16 ? 64 : 32 bytes.
constexpr int kRowBytes = 144;

template <int BT>
struct TileCfg {
  static constexpr int F = BT / 8;                   // fragment edge
  static constexpr int OPB = BT * kRowBytes;         // bytes of one operand stage
  static constexpr int LDS = 4 * OPB;                // 2 operands x 2 stages
  static constexpr int SUBB = F == 16 ? 64 : 32;     // bytes of k per MFMA sub-step
  static constexpr int NSUB = 128 / SUBB;            // sub-steps per stage
  static constexpr int CPT = BT / 32;                // 16-byte chunks per thread per operand
  static constexpr int ACC = F == 16 ? 4 : 16;       // accumulator floats per fragment
  static constexpr int RG = F == 16 ? 1 : 4;         // groups of 4 consecutive rows per fragment
};

template <int N>
struct AccT;
template <>
struct AccT<4> { typedef f32x4 type; };
template <>
struct AccT<16> { typedef float type __attribute__((ext_vector_type(16))); };

// Waves of a GEMM block and their grid over the BT x BT tile: two wave rows
// of BT/2 tile rows each; WGN wave columns of WTN tile columns, each holding
// FN fragments of F x F.  The bf16 256 tile runs 8 waves (2 per SIMD, wave
// tile 128 x 64): one wave's LDS reads, barrier waits and epilogue memory
// latency then overlap the other's MFMAs.  The FP8 256 tile uses the same
// layout; every other path runs 4 waves.
template <int P, int BT>
struct WaveCfg {
  static constexpr int NW = ((P == kBF16 || P == kFP8) && BT == 256) ? 8 : 4;
  static constexpr int NT = NW * 64;
  static constexpr int WGN = NW / 2;
  static constexpr int F = BT / 8;
  static constexpr int FN = 8 / WGN;
  static constexpr int WTN = FN * F;
};

// The FP32 path stages its operands through registers (the bf16 and e4m3
// paths use the direct-to-LDS ring below): 32 fp32 of k per LDS stage, four
// per 16-byte chunk.
template <typename T>
struct OpT;
template <>
struct OpT<float> {
  static constexpr int kVec = 4;
  static constexpr int kBK = 32;
};

template <typename T, int BT, typename A>
__device__ __forceinline__ void mma_stage(const char* sA, const char* sB, int wm, int wn, int lane,
                                          A (&acc)[4][4]) {
  typedef TileCfg<BT> C;
  constexpr int F = C::F;
#pragma unroll
  for (int ks = 0; ks < C::NSUB; ++ks) {
    u32x4 fa[4], fb[4];
    const int koff = ks * C::SUBB + (lane / F) * 16;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      fa[f] = *(const u32x4*)(sA + (wm * (BT / 2) + f * F + (lane % F)) * kRowBytes + koff);
      fb[f] = *(const u32x4*)(sB + (wn * (BT / 2) + f * F + (lane % F)) * kRowBytes + koff);
    }
#pragma unroll
    for (int fm = 0; fm < 4; ++fm) {
#pragma unroll
      for (int fn = 0; fn < 4; ++fn) {
        const f32x4 a4 = __builtin_bit_cast(f32x4, fa[fm]);
        const f32x4 b4 = __builtin_bit_cast(f32x4, fb[fn]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if constexpr (F == 16)
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x4f32(a4[e], b4[e], acc[fm][fn], 0, 0, 0);
          else
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[e], b4[e], acc[fm][fn], 0, 0, 0);
        }
      }
    }
  }
}

// acc += P[rp0:rp0+BT, k0:k1] * Q[rq0:rq0+BT, k0:k1]^T, (k1 - k0) % BK == 0.
template <typename T, int BT, typename A>
__device__ __forceinline__ void gemm_nt_tile(const T* __restrict__ P, const T* __restrict__ Q,
                                             int64_t ld, int rp0, int rq0, int k0, int k1,
                                             char* smem, A (&acc)[4][4]) {
  static_assert(sizeof(T) == 4, "register-staged tiles serve the FP32 path");
  typedef TileCfg<BT> C;
  constexpr int BK = OpT<T>::kBK, VEC = OpT<T>::kVec, CPT = C::CPT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // chunk c = tid + 256 j: row c / 8, 16-byte column c % 8
  const int crow = tid >> 3, ccol = tid & 7;
  const PE_GLOBAL T* pP = gview(P) + (size_t)(rp0 + crow) * ld + k0 + ccol * VEC;
  const PE_GLOBAL T* pQ = gview(Q) + (size_t)(rq0 + crow) * ld + k0 + ccol * VEC;
  const size_t jstride = (size_t)32 * ld;  // 32 rows between a thread's chunks
  u32x4 ra[CPT], rb[CPT];
  const int nk = (k1 - k0) / BK;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    ra[j] = *(const PE_GLOBAL u32x4*)(pP + j * jstride);
    rb[j] = *(const PE_GLOBAL u32x4*)(pQ + j * jstride);
  }
  const int soff = crow * kRowBytes + ccol * 16;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    *(u32x4*)(smem + soff + j * 32 * kRowBytes) = ra[j];
    *(u32x4*)(smem + C::OPB + soff + j * 32 * kRowBytes) = rb[j];
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    // prefetch the next stage (the last iteration re-reads its own stage, which
    // keeps the loop free of branches around the register buffers)
    const size_t adv = (size_t)(kt + 1 < nk ? kt + 1 : kt) * BK;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      ra[j] = *(const PE_GLOBAL u32x4*)(pP + adv + j * jstride);
      rb[j] = *(const PE_GLOBAL u32x4*)(pQ + adv + j * jstride);
    }
    // keep the prefetch at the top of the stage: a whole stage of MFMA work
    // then covers its latency
    __builtin_amdgcn_sched_barrier(0);
    const char* cur = smem + (kt & 1) * 2 * C::OPB;
    mma_stage<T, BT>(cur, cur + C::OPB, wm, wn, lane, acc);
    char* nxt = smem + ((kt + 1) & 1) * 2 * C::OPB;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      *(u32x4*)(nxt + soff + j * 32 * kRowBytes) = ra[j];
      *(u32x4*)(nxt + C::OPB + soff + j * 32 * kRowBytes) = rb[j];
    }
    __syncthreads();
  }
}

// ------------------------------------------------- bf16 direct-to-LDS main loop
// The bf16 path's main loop.  Operands go from HBM straight into LDS with
// global_load_lds_dwordx4 (lane i of a wave writes 16 bytes at LDS base + 16 i),
// so no registers stage them and no wait on a load sits in front of an LDS
// store.  Stages hold 32 k (64 bytes per row, unpadded) in a ring of four; the
// loads of stage kt + 3 are in flight while stage kt is multiplied.  A row's
// four 16-byte chunks are stored XOR-swizzled by (row / 4) % 4, which spreads
// the fragment reads of consecutive rows over all banks.
template <int BT>
struct DlCfg {
  static constexpr int F = BT / 8;
  static constexpr int BK = 32;                  // k per stage
  static constexpr int NS = 4;                   // stages in the LDS ring
  static constexpr int ROWB = 64;                // bytes per row per stage
  static constexpr int OPB = BT * ROWB;          // one operand, one stage
  static constexpr int STB = 2 * OPB;            // one stage
  static constexpr int LDS = NS * STB;
  static constexpr int NW = WaveCfg<kBF16, BT>::NW;
  static constexpr int IPW = OPB / 1024 / NW;    // 1-KB loads per wave per operand per stage
  static constexpr int LPS = 2 * IPW;            // load instructions per wave per stage
};

__device__ __forceinline__ int dl_swz(int row, int chunk) { return chunk ^ ((row >> 2) & 3); }

// s_waitcnt vmcnt(n) (gfx9 encoding: vmcnt[3:0] | vmcnt[5:4] << 14; exp/lgkm at max)
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Workgroup barrier that orders LDS accesses for the compiler without the
// memory fences of __syncthreads (which would also wait for every
// outstanding global load): the empty asm statements with a memory clobber
// keep the compiler from moving loads or stores across the s_barrier; the
// hardware ordering comes from the explicit waits placed before it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// The update's second operand can also be X itself, row-major with k along
// its rows (XR): a stage then holds 32 rows of X (k) by BT columns (n), and
// the fragments are read with transposing LDS reads.  16-byte chunk c of
// stage row r sits at chunk c ^ xr_swz(r): each transposing read covers four
// consecutive rows per 16 lanes, and the swizzle puts them on distinct banks.
template <int BT>
__device__ __forceinline__ int xr_swz(int r) {
  return BT == 256 ? (r & 3) << 2 : ((r & 3) | (((r >> 3) & 1) << 2)) << 1;
}

// P is row-major (row stride ld); Q has row stride ldQ and kbQ elements between
// consecutive 32-deep k blocks (row-major: ldQ = ld, kbQ = 32).  XR: Q is
// row-major X, k along its rows (row stride ldQ), already offset to the
// tile's first column.
template <int BT, bool XR = false>
__device__ __forceinline__ void dl_issue_stage(const PE_GLOBAL uint16_t* P, const PE_GLOBAL uint16_t* Q,
                                               int64_t ld, int64_t ldQ, int64_t kbQ, int kofs, char* slot,
                                               int wave, int lane) {
  typedef DlCfg<BT> C;
  static_assert(C::BK == 32, "one k block per stage");
  if constexpr (XR) {
    constexpr int CPR = BT / 8;                      // 16-byte chunks per stage row
#pragma unroll
    for (int j = 0; j < C::IPW; ++j) {
      const int blk = wave * C::IPW + j;            // 1-KB block = 64 / CPR rows
      const int row = blk * (64 / CPR) + lane / CPR;
      const int lc = (lane % CPR) ^ xr_swz<BT>(row);  // logical chunk this lane fetches
      const PE_GLOBAL uint16_t* g = Q + (size_t)(kofs + row) * ldQ + lc * 8;
      __builtin_amdgcn_global_load_lds((const void*)g,
                                       (__attribute__((address_space(3))) void*)(slot + C::OPB + blk * 1024),
                                       16, 0, 0);
    }
  }
#pragma unroll
  for (int op = 0; op < (XR ? 1 : 2); ++op) {
    const PE_GLOBAL uint16_t* base = op == 0 ? P : Q;
    const int64_t rs = op == 0 ? ld : ldQ;
    const int64_t kb = op == 0 ? 32 : kbQ;
#pragma unroll
    for (int j = 0; j < C::IPW; ++j) {
      const int blk = wave * C::IPW + j;            // 1-KB block = 16 rows
      const int row = blk * 16 + (lane >> 2);
      const int lc = dl_swz(row, lane & 3);          // logical chunk this lane fetches
      const PE_GLOBAL uint16_t* g = base + (size_t)row * rs + (size_t)(kofs >> 5) * kb + lc * 8;
      __builtin_amdgcn_global_load_lds((const void*)g,
                                       (__attribute__((address_space(3))) void*)(slot + op * C::OPB + blk * 1024),
                                       16, 0, 0);
    }
  }
}

// Transposing read of an XR stage (rows k, BT columns n): with every 16
// lanes addressing rows r0..r0+3 (lane q: row r0 + q / 4, columns n0 + 4 (q % 4)
// .. + 3), lane q receives the four k values of column n0 + q.
template <int BT>
__device__ __forceinline__ u32x2 xr_read(const char* sB, int r, int nn) {
  const char* p = sB + r * (BT * 2) + (((nn >> 3) ^ xr_swz<BT>(r)) << 4) + (nn & 4) * 2;
  return __builtin_bit_cast(u32x2, __builtin_amdgcn_ds_read_tr16_b64_v4i16(
                                       (__attribute__((address_space(3))) i16x4*)(p)));
}

template <int BT, typename A, bool XR = false>
__device__ __forceinline__ void dl_mma_stage(const char* sA, const char* sB, int wm, int wn, int lane,
                                             A (&acc)[4][4]) {
  constexpr int F = BT / 8;
  constexpr int NSUB = F == 16 ? 1 : 2;          // MFMA k-steps per 32-k stage
  static_assert(!XR || F == 16, "XR stage reads: 128 tile here, 256 tile in dl_read_frags32");
#pragma unroll
  for (int ks = 0; ks < NSUB; ++ks) {
    u32x4 fa[4], fb[4];
    const int lc = F == 16 ? (lane >> 4) : (2 * ks + (lane >> 5));
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const int ra = wm * (BT / 2) + f * F + (lane % F);
      const int rb = wn * (BT / 2) + f * F + (lane % F);
      fa[f] = *(const u32x4*)(sA + ra * 64 + dl_swz(ra, lc) * 16);
      if constexpr (XR) {
        // 16x16x32: lane l takes k = 8 (l / 16) .. + 7 of column l % 16
        const int r = 8 * (lane >> 4) + ((lane & 15) >> 2);
        const int nn = wn * (BT / 2) + f * F + 4 * (lane & 3);
        const u32x2 lo = xr_read<BT>(sB, r, nn), hi = xr_read<BT>(sB, r + 4, nn);
        fb[f] = (u32x4){lo[0], lo[1], hi[0], hi[1]};
      } else {
        fb[f] = *(const u32x4*)(sB + rb * 64 + dl_swz(rb, lc) * 16);
      }
    }
#pragma unroll
    for (int fm = 0; fm < 4; ++fm)
#pragma unroll
      for (int fn = 0; fn < 4; ++fn) {
        if constexpr (F == 16)
          acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              __builtin_bit_cast(bf16x8, fa[fm]), __builtin_bit_cast(bf16x8, fb[fn]), acc[fm][fn], 0, 0, 0);
        else
          acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
              __builtin_bit_cast(bf16x8, fa[fm]), __builtin_bit_cast(bf16x8, fb[fn]), acc[fm][fn], 0, 0, 0);
      }
  }
}

// s_waitcnt lgkmcnt(0) with vmcnt and expcnt left at their maxima
__device__ __forceinline__ void wait_lgkm0() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Fragments of one 16-deep k-step of the 256 tile (32x32x16 MFMA, 8 waves):
// rows lane % 32 of four 32-row fragments of the first operand and two of the
// second, 16-byte chunk 2 * sub + lane / 32 of the stage's 64-byte row.
struct Frags32 {
  u32x4 a[4], b[2];
};

template <bool XR = false>
__device__ __forceinline__ void dl_read_frags32(const char* stage, int sub, int wm, int wn, int lane,
                                                Frags32& f) {
  constexpr int OPB = DlCfg<256>::OPB;
  const int lc = 2 * sub + (lane >> 5);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int ra = wm * 128 + i * 32 + (lane & 31);
    f.a[i] = *(const u32x4*)(stage + ra * 64 + dl_swz(ra, lc) * 16);
  }
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if constexpr (XR) {
      // 32x32x16: lane l takes k = 16 sub + 8 (l / 32) .. + 7 of column l % 32
      // of the fragment, whose columns are 32 wn + 128 i .. (upd_col)
      const int r = 16 * sub + 8 * (lane >> 5) + ((lane & 15) >> 2);
      const int nn = wn * 32 + i * 128 + 16 * ((lane >> 4) & 1) + 4 * (lane & 3);
      const u32x2 lo = xr_read<256>(stage + OPB, r, nn), hi = xr_read<256>(stage + OPB, r + 4, nn);
      f.b[i] = (u32x4){lo[0], lo[1], hi[0], hi[1]};
    } else {
      const int rb = wn * 64 + i * 32 + (lane & 31);
      f.b[i] = *(const u32x4*)(stage + OPB + rb * 64 + dl_swz(rb, lc) * 16);
    }
  }
}

template <typename A>
__device__ __forceinline__ void dl_mfma32(const Frags32& f, A (&acc)[4][2]) {
#pragma unroll
  for (int fm = 0; fm < 4; ++fm)
#pragma unroll
    for (int fn = 0; fn < 2; ++fn)
      acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, f.a[fm]),
                                                            __builtin_bit_cast(bf16x8, f.b[fn]), acc[fm][fn], 0, 0, 0);
}

// acc += P[rp0:+BT, k0:k1] * Q[rq0:+BT, k0:k1]^T (bf16), k0 and k1 multiples of 32;
// Q's layout as for dl_issue_stage (XR: acc += P[rp0:+BT, k0:k1] * Q[k0:k1, rq0:+BT])
template <int BT, typename A, int FN, bool XR = false>
__device__ __forceinline__ void gemm_nt_tile_dl(const uint16_t* __restrict__ P,
                                                const uint16_t* __restrict__ Q, int64_t ld, int64_t ldQ,
                                                int64_t kbQ, int rp0, int rq0, int k0, int k1, char* smem,
                                                A (&acc)[4][FN]) {
  typedef DlCfg<BT> C;
  typedef WaveCfg<kBF16, BT> W;
  static_assert(FN == W::FN, "accumulator grid");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / W::WGN, wn = wave % W::WGN;
  const PE_GLOBAL uint16_t* pP = gview(P) + (size_t)rp0 * ld + k0;
  const PE_GLOBAL uint16_t* pQ = XR ? gview(Q) + (size_t)k0 * ldQ + rq0
                                    : gview(Q) + (size_t)rq0 * ldQ + (size_t)(k0 >> 5) * kbQ;
  const int nk = (k1 - k0) / C::BK;
  // prologue: stages 0..NS-2 in flight (a stage past the end re-reads the last
  // one, which keeps the count of outstanding loads per iteration fixed)
  __syncthreads();  // the previous tile's readers are done with the ring
#pragma unroll
  for (int s = 0; s < C::NS - 1; ++s) {
    const int ks = s < nk ? s : nk - 1;
    dl_issue_stage<BT, XR>(pP, pQ, ld, ldQ, kbQ, ks * C::BK, smem + s * C::STB, wave, lane);
  }
  if constexpr (BT == 128) {
    static_assert(W::NW == 4 && FN == 4, "128 tile: 4 waves");
    for (int kt = 0; kt < nk; ++kt) {
      // this wave's loads of stage kt are done once at most NS-2 later stages are pending
      wait_vmcnt<(C::NS - 2) * C::LPS>();
      lds_barrier();  // everyone's loads of stage kt landed; stage kt-1's slot is free
      {
        const int ks = kt + C::NS - 1 < nk ? kt + C::NS - 1 : nk - 1;
        dl_issue_stage<BT, XR>(pP, pQ, ld, ldQ, kbQ, ks * C::BK, smem + ((kt + C::NS - 1) % C::NS) * C::STB, wave, lane);
      }
      const char* cur = smem + (kt % C::NS) * C::STB;
      dl_mma_stage<BT, A, XR>(cur, cur + C::OPB, wm, wn, lane, acc);
    }
  } else {
    // 256 tile, two 16-deep k-steps per stage, software-pipelined: the
    // fragments of the next k-step are read from LDS while the MFMAs of the
    // current one run, and the stage barrier sits between the two halves, so
    // neither LDS latency nor the barrier stands between two MFMA groups.
    // Explicit waits at the end of each half leave nothing in flight at the
    // loop header, and scheduling fences keep the compiler's scheduler from
    // re-serialising reads and MFMAs.
    static_assert(BT == 256 && W::NW == 8, "pipelined loop is written for the 8-wave 256 tile");
    wait_vmcnt<(C::NS - 2) * C::LPS>();
    lds_barrier();  // stage 0 visible
    Frags32 f0, f1;
    dl_read_frags32<XR>(smem, 0, wm, wn, lane, f0);
    wait_lgkm0();
    for (int kt = 0; kt < nk; ++kt) {
      const char* cur = smem + (kt % C::NS) * C::STB;
      __builtin_amdgcn_sched_barrier(0);
      dl_read_frags32<XR>(cur, 1, wm, wn, lane, f1);
      dl_mfma32(f0, acc);
      // the LDS reads (6, or 8 with transposing reads) spread over the 8 MFMAs
      constexpr int NRD = XR ? 8 : 6;
#pragma unroll
      for (int q = 0; q < NRD; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
      }
      if constexpr (NRD < 8) __builtin_amdgcn_sched_group_barrier(0x008, 8 - NRD, 0);
      __builtin_amdgcn_sched_barrier(0);
      wait_lgkm0();
      // own loads of stage kt+1 landed; after the barrier everyone's have, and
      // every wave has finished reading stage kt-1's slot (its last reads were
      // waited for before this wave's previous barrier)
      wait_vmcnt<(C::NS - 3) * C::LPS>();
      lds_barrier();
      __builtin_amdgcn_sched_barrier(0);
      {
        const int ks = kt + C::NS - 1 < nk ? kt + C::NS - 1 : nk - 1;
        dl_issue_stage<BT, XR>(pP, pQ, ld, ldQ, kbQ, ks * C::BK, smem + ((kt + C::NS - 1) % C::NS) * C::STB, wave, lane);
      }
      const int nx = kt + 1 < nk ? kt + 1 : kt;
      dl_read_frags32<XR>(smem + (nx % C::NS) * C::STB, 0, wm, wn, lane, f0);
      dl_mfma32(f1, acc);
      // 4 direct-to-LDS loads and the LDS reads spread over the 8 MFMAs
      static_assert(C::LPS == 4, "load count per stage");
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x010, 1, 1);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 1);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 1);
      }
#pragma unroll
      for (int q = 4; q < NRD; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 1);
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 1);
      }
      if constexpr (NRD < 8) __builtin_amdgcn_sched_group_barrier(0x008, 8 - NRD, 1);
      __builtin_amdgcn_sched_barrier(0);
      wait_lgkm0();
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  wait_vmcnt<0>();  // no LDS write may still be in flight when the ring is reused
}

// Persistent blocks take items b, b + G, b + 2G, ... (G = gridDim.x).  Blocks
// are dispatched round-robin over the 8 XCDs (block b on XCD b % 8), each with
// its own L2.  When G is a multiple of 8, this permutation gives the G/8 blocks
// of XCD x, at round k, the contiguous positions
// [kG + x G/8, kG + (x+1) G/8) of the item order, so tiles that share operand
// panels run on the same L2.  The last, partial round keeps the identity.
__device__ __forceinline__ int xcd_item(int item, int total) {
  const int G = gridDim.x;
  if ((G & 7) != 0) return item;
  const int round = item / G, b = item - round * G;
  if ((round + 1) * G > total) return item;
  return round * G + (b & 7) * (G >> 3) + (b >> 3);
}

// Tile (tm, tn) of an nb x nbn grid from a position in "banded" order: bands of
// GM tile rows, tm fastest inside a band, so consecutive positions form
// GM-tall blocks that share both operand panels.
__device__ __forceinline__ void banded_decode(int local, int nb, int nbn, int* tm, int* tn) {
  constexpr int GM = 8;
  const int band = local / (GM * nbn);
  const int first = band * GM;
  const int rows = min(GM, nb - first);
  const int r = local - band * GM * nbn;
  *tm = first + r % rows;
  *tn = r / rows;
}

// upper-triangle tile index -> (ti, tj), ti <= tj, row-major over ti
__device__ __forceinline__ void tri_decode(int u, int nb, int* ti, int* tj) {
  int r = 0, rowlen = nb;
  while (u >= rowlen) { u -= rowlen; ++r; --rowlen; }
  *ti = r;
  *tj = r + u;
}

// Upper-triangle tile (ti <= tj) from a position in banded order: bands of
// GM tile rows; inside a band, columns left to right, the band's rows (those
// with ti <= tj) fastest.  Consecutive positions then share column panels and
// cycle through GM row panels, as in banded_decode, so the tiles that one XCD
// runs together touch few distinct operand panels.  A band of R rows starting
// at row r0 holds R(R+1)/2 tiles in its first R columns, then R per column.
__device__ __forceinline__ void tri_decode_banded(int u, int nb, int* ti, int* tj) {
  constexpr int GM = 8;
  int r0 = 0;
  for (;;) {
    const int R = min(GM, nb - r0);
    const int tri = R * (R + 1) / 2;
    const int cnt = tri + (nb - r0 - R) * R;
    if (u < cnt) {
      if (u < tri) {
        int c = 0;
        while ((c + 1) * (c + 2) / 2 <= u) ++c;
        *tj = r0 + c;
        *ti = r0 + (u - c * (c + 1) / 2);
      } else {
        const int v = u - tri;
        *tj = r0 + R + v / R;
        *ti = r0 + v % R;
      }
      return;
    }
    u -= cnt;
    r0 += R;
  }
}

// inverse of tri_decode (row-major index, used for per-tile partial sums)
__device__ __forceinline__ int tri_index(int ti, int tj, int nb) {
  return ti * nb - (ti * (ti - 1)) / 2 + (tj - ti);
}

__device__ __forceinline__ void split_range(int K, int split, int ksp, int BK, int* k0, int* k1) {
  int per = (K + split - 1) / split;
  per = (per + BK - 1) / BK * BK;
  *k0 = min(K, ksp * per);
  *k1 = min(K, *k0 + per);
}

// Wave-level max of non-negative floats, one atomic per wave.
__device__ __forceinline__ void wave_amax_atomic(float v, float* slot) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) atomicMax((unsigned int*)slot, __float_as_uint(v));
}

__device__ __forceinline__ uint2 pack4_bf16(const float (&v)[4]) {
  uint2 pk;
  pk.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
  pk.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
  return pk;
}

// ------------------------------------------------------------- FP8 (e4m3)
// Per-tensor scale: the largest power of two q with amax * 1.01 * q <= 448, so
// x * q is exact and never exceeds the largest e4m3 magnitude (the 1.01 covers
// the bf16 rounding of values whose maximum was taken in fp32).
__device__ __forceinline__ float fp8_scale(float amax) {
  if (!(amax > 0.0f) || !(amax < 3.0e38f)) return 1.0f;
  int e;
  frexpf(448.0f / (amax * 1.01f), &e);
  return ldexpf(1.0f, e - 1);
}

// four floats -> four OCP e4m3 bytes (hardware conversion, round to nearest even)
__device__ __forceinline__ uint32_t pack4_e4m3(float f0, float f1, float f2, float f3) {
  int w = __builtin_amdgcn_cvt_pk_fp8_f32(f0, f1, 0, false);
  w = __builtin_amdgcn_cvt_pk_fp8_f32(f2, f3, w, true);
  return (uint32_t)w;
}

// eight bf16 (one 16-byte chunk) scaled by q -> eight e4m3 bytes
__device__ __forceinline__ uint2 bf16x8_to_e4m3(u32x4 c, float q) {
  uint2 r;
  r.x = pack4_e4m3(__uint_as_float(c[0] << 16) * q, __uint_as_float(c[0] & 0xffff0000u) * q,
                   __uint_as_float(c[1] << 16) * q, __uint_as_float(c[1] & 0xffff0000u) * q);
  r.y = pack4_e4m3(__uint_as_float(c[2] << 16) * q, __uint_as_float(c[2] & 0xffff0000u) * q,
                   __uint_as_float(c[3] << 16) * q, __uint_as_float(c[3] & 0xffff0000u) * q);
  return r;
}

// FP8 stage layout: the bf16 operand is read from HBM and quantised on its way
// into LDS.  BT = 128: 128 k per stage, 16x16x128 f8f6f4 MFMA (lane: 32 bytes
// at k = 32*(lane/16)); BT = 256: 64 k per stage, 32x32x64 f8f6f4 MFMA (lane:
// 32 bytes at k = 32*(lane/32)).  Rows carry a 16-byte pad.
template <int BT>
struct Fp8Cfg {
  static constexpr int F = BT / 8;
  static constexpr int KQ = BT == 128 ? 128 : 64;   // k per stage
  static constexpr int ROWB = KQ + 16;              // LDS bytes per row
  static constexpr int OPB = BT * ROWB;
  static constexpr int LDS = 4 * OPB;
  static constexpr int CPR = KQ / 8;                // 16-byte bf16 chunks per row
  static constexpr int CPT = BT * CPR / kThreads;   // chunks per thread per operand (8)
  static constexpr int RSTRIDE = kThreads / CPR;    // rows between a thread's chunks
};

template <int BT, typename A>
__device__ __forceinline__ void mma_stage_fp8(const char* sA, const char* sB, int wm, int wn,
                                              int lane, A (&acc)[4][4]) {
  typedef Fp8Cfg<BT> C;
  constexpr int F = C::F;
  i32x8 fa[4], fb[4];
  const int koff = (lane / F) * 32;
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    const char* pa = sA + (wm * (BT / 2) + f * F + (lane % F)) * C::ROWB + koff;
    const char* pb = sB + (wn * (BT / 2) + f * F + (lane % F)) * C::ROWB + koff;
    const u32x4 a0 = *(const u32x4*)pa, a1 = *(const u32x4*)(pa + 16);
    const u32x4 b0 = *(const u32x4*)pb, b1 = *(const u32x4*)(pb + 16);
    fa[f] = i32x8{(int)a0[0], (int)a0[1], (int)a0[2], (int)a0[3],
                  (int)a1[0], (int)a1[1], (int)a1[2], (int)a1[3]};
    fb[f] = i32x8{(int)b0[0], (int)b0[1], (int)b0[2], (int)b0[3],
                  (int)b1[0], (int)b1[1], (int)b1[2], (int)b1[3]};
  }
#pragma unroll
  for (int fm = 0; fm < 4; ++fm) {
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
      // format 0 = e4m3 for both operands, E8M0 block scales 127 = 1.0
      if constexpr (F == 16)
        acc[fm][fn] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(fa[fm], fb[fn], acc[fm][fn],
                                                                       0, 0, 0, 127, 0, 127);
      else
        acc[fm][fn] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fa[fm], fb[fn], acc[fm][fn],
                                                                      0, 0, 0, 127, 0, 127);
    }
  }
}

// acc += q(P)[rp0:+BT, k0:k1] * q(Q)[rq0:+BT, k0:k1]^T with bf16 operands in HBM
// quantised to e4m3 with scales qp, qq; (k1 - k0) % KQ == 0.
template <int BT, typename A>
__device__ __forceinline__ void gemm_nt_tile_fp8(const uint16_t* __restrict__ P,
                                                 const uint16_t* __restrict__ Q, int64_t ld,
                                                 int rp0, int rq0, int k0, int k1, float qp, float qq,
                                                 char* smem, A (&acc)[4][4]) {
  typedef Fp8Cfg<BT> C;
  constexpr int CPT = C::CPT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int crow = tid / C::CPR, ccol = tid % C::CPR;
  const PE_GLOBAL uint16_t* pP = gview(P) + (size_t)(rp0 + crow) * ld + k0 + ccol * 8;
  const PE_GLOBAL uint16_t* pQ = gview(Q) + (size_t)(rq0 + crow) * ld + k0 + ccol * 8;
  const size_t jstride = (size_t)C::RSTRIDE * ld;
  u32x4 ra[CPT], rb[CPT];
  const int nk = (k1 - k0) / C::KQ;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    ra[j] = *(const PE_GLOBAL u32x4*)(pP + j * jstride);
    rb[j] = *(const PE_GLOBAL u32x4*)(pQ + j * jstride);
  }
  const int soff = crow * C::ROWB + ccol * 8;
#pragma unroll
  for (int j = 0; j < CPT; ++j) {
    *(uint2*)(smem + soff + j * C::RSTRIDE * C::ROWB) = bf16x8_to_e4m3(ra[j], qp);
    *(uint2*)(smem + C::OPB + soff + j * C::RSTRIDE * C::ROWB) = bf16x8_to_e4m3(rb[j], qq);
  }
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const size_t adv = (size_t)(kt + 1 < nk ? kt + 1 : kt) * C::KQ;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      ra[j] = *(const PE_GLOBAL u32x4*)(pP + adv + j * jstride);
      rb[j] = *(const PE_GLOBAL u32x4*)(pQ + adv + j * jstride);
    }
    // keep the prefetch at the top of the stage: a whole stage of MFMA work
    // then covers its latency
    __builtin_amdgcn_sched_barrier(0);
    const char* cur = smem + (kt & 1) * 2 * C::OPB;
    mma_stage_fp8<BT>(cur, cur + C::OPB, wm, wn, lane, acc);
    char* nxt = smem + ((kt + 1) & 1) * 2 * C::OPB;
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
      *(uint2*)(nxt + soff + j * C::RSTRIDE * C::ROWB) = bf16x8_to_e4m3(ra[j], qp);
      *(uint2*)(nxt + C::OPB + soff + j * C::RSTRIDE * C::ROWB) = bf16x8_to_e4m3(rb[j], qq);
    }
    __syncthreads();
  }
}

// ---------------------------------------- FP8 Gram-side main loop, 256 tile
// Once a step's operand maximum is known (X_t: the previous update or the norm
// pass; A_t: the Gram epilogue), a quantisation pass writes its e4m3 copy
// e4m3(q x) (quant_kernel); the product then streams one byte per element
// through the direct-to-LDS ring (64 k per 64-byte row, one
// v_mfma_scale_f32_32x32x64_f8f6f4 k-step per stage), half the bytes of the
// bf16 ring, and the epilogue multiplies by 1/q^2.  The conversion
// v_cvt_scalef32_pk_fp8_bf16 computes e4m3(x / scale) with round to nearest
// even (two values per instruction); scale = 1/q, a power of two, makes it
// e4m3(q x) exactly.
__device__ __forceinline__ int cvt4_e4m3(uint32_t u0, uint32_t u1, float inv_q) {
  i16x2 r = {0, 0};
  r = __builtin_amdgcn_cvt_scalef32_pk_fp8_bf16(r, __builtin_bit_cast(bf16x2, u0), inv_q, false);
  r = __builtin_amdgcn_cvt_scalef32_pk_fp8_bf16(r, __builtin_bit_cast(bf16x2, u1), inv_q, true);
  return __builtin_bit_cast(int, r);
}

// Direct-to-LDS issue of one 64-k stage of two e4m3 operands (64 bytes per
// row: the same row geometry and swizzle as a 32-k bf16 stage).
__device__ __forceinline__ void dl_issue_stage_q8(const PE_GLOBAL uint8_t* P, const PE_GLOBAL uint8_t* Q,
                                                  int64_t ld, int kofs, char* slot, int wave, int lane) {
  typedef DlCfg<256> C;
#pragma unroll
  for (int op = 0; op < 2; ++op) {
    const PE_GLOBAL uint8_t* base = op == 0 ? P : Q;
#pragma unroll
    for (int j = 0; j < C::IPW; ++j) {
      const int blk = wave * C::IPW + j;            // 1-KB block = 16 rows
      const int row = blk * 16 + (lane >> 2);
      const int lc = dl_swz(row, lane & 3);
      const PE_GLOBAL uint8_t* g = base + (size_t)row * ld + kofs + lc * 16;
      __builtin_amdgcn_global_load_lds((const void*)g,
                                       (__attribute__((address_space(3))) void*)(slot + op * C::OPB + blk * 1024),
                                       16, 0, 0);
    }
  }
}

// e4m3 fragments of one 64-k stage for v_mfma_scale_f32_32x32x64_f8f6f4:
// lane l holds row l % 32 and k = 32 (l / 32) + 0..31, i.e. the 16-byte
// chunks 2 (l / 32) and 2 (l / 32) + 1 of its 64-byte row.
struct FragsQ8 {
  i32x8 a[4], b[2];
};

__device__ __forceinline__ i32x8 q8_row(const char* op, int row, int kh) {
  const char* r = op + row * 64;
  const u32x4 c0 = *(const u32x4*)(r + dl_swz(row, 2 * kh) * 16);
  const u32x4 c1 = *(const u32x4*)(r + dl_swz(row, 2 * kh + 1) * 16);
  return i32x8{(int)c0[0], (int)c0[1], (int)c0[2], (int)c0[3], (int)c1[0], (int)c1[1], (int)c1[2], (int)c1[3]};
}

__device__ __forceinline__ void q8_read(const char* st, int wm, int wn, int lane, FragsQ8& f) {
  constexpr int OPB = DlCfg<256>::OPB;
  const int kh = lane >> 5;
#pragma unroll
  for (int i = 0; i < 4; ++i) f.a[i] = q8_row(st, wm * 128 + i * 32 + (lane & 31), kh);
#pragma unroll
  for (int i = 0; i < 2; ++i) f.b[i] = q8_row(st + OPB, wn * 64 + i * 32 + (lane & 31), kh);
}

template <typename A>
__device__ __forceinline__ void q8_mfma(const FragsQ8& f, A (&acc)[4][2]) {
#pragma unroll
  for (int fm = 0; fm < 4; ++fm)
#pragma unroll
    for (int fn = 0; fn < 2; ++fn)
      // format 0 = e4m3 for both operands, E8M0 block scales 127 = 1.0
      acc[fm][fn] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(f.a[fm], f.b[fn], acc[fm][fn],
                                                                    0, 0, 0, 127, 0, 127);
}

// acc += P[rp0:+256, k0:k1] * Q[rq0:+256, k0:k1]^T with e4m3 operands in HBM
// (already scaled by the quantisation pass); (k1 - k0) % 64 == 0.  Ring of
// four 64-k stages (32 KB each), three in flight.  One fragment set per wave
// (two would not fit beside the 128 accumulators); the second wave on each
// SIMD covers the LDS latency.
template <typename A>
__device__ __forceinline__ void gemm_nt_tile_dl_q8(const uint8_t* __restrict__ P,
                                                   const uint8_t* __restrict__ Q, int64_t ld, int rp0,
                                                   int rq0, int k0, int k1, char* smem, A (&acc)[4][2]) {
  typedef DlCfg<256> C;
  typedef WaveCfg<kFP8, 256> W;
  static_assert(W::NW == 8 && C::NS == 4 && C::LPS == 4, "ring of the 8-wave 256 tile");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / W::WGN, wn = wave % W::WGN;
  const PE_GLOBAL uint8_t* pP = (const PE_GLOBAL uint8_t*)P + (size_t)rp0 * ld + k0;
  const PE_GLOBAL uint8_t* pQ = (const PE_GLOBAL uint8_t*)Q + (size_t)rq0 * ld + k0;
  const int nk = (k1 - k0) / 64;
  __syncthreads();  // the previous tile's readers are done with the ring
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int ks = s < nk ? s : nk - 1;
    dl_issue_stage_q8(pP, pQ, ld, ks * 64, smem + s * C::STB, wave, lane);
  }
  for (int s = 0; s < nk; ++s) {
    // own loads of stage s landed (stages s+1, s+2 may be pending); after the
    // barrier everyone's have, and every wave has finished stage s-1, whose
    // slot takes stage s+3
    wait_vmcnt<2 * C::LPS>();
    lds_barrier();
    {
      const int ks = s + 3 < nk ? s + 3 : nk - 1;
      dl_issue_stage_q8(pP, pQ, ld, ks * 64, smem + ((s + 3) & 3) * C::STB, wave, lane);
    }
    FragsQ8 f;
    q8_read(smem + (s & 3) * C::STB, wm, wn, lane, f);
    q8_mfma(f, acc);
  }
  wait_vmcnt<0>();  // no LDS write may still be in flight when the ring is reused
}

// Scale of step t's Gram-side operand (kind GRAM: X_t, kind A2: A_t).
__device__ __forceinline__ float fp8_operand_scale(const MatDesc& d, int kind, int t) {
  float amax;
  if (kind == KIND_GRAM)
    amax = t == 0 ? d.scal[kScAmaxG] : __uint_as_float(((const uint32_t*)d.scal)[kScAmaxX + t]);
  else
    amax = __uint_as_float(((const uint32_t*)d.scal)[kScAmaxA + t]);
  return fp8_scale(amax);
}

// ------------------------------------------------------------- epilogues
// Accumulator element (fm, fn, g, r) is C[row][col] of the block tile with
//   F = 16: row = wm*BT/2 + fm*16 + 4*(lane/16) + r,           col = wn*BT/2 + fn*16 + lane%16
//   F = 32: row = wm*BT/2 + fm*32 + 8*g + 4*(lane/32) + r,     col = wn*WTN + fn*32 + lane%32
// with acc register index 4*g + r (WTN = BT/2 with 4 waves, BT/4 with 8); each
// (fm, fn, g) is four consecutive rows.
template <int BT>
__device__ __forceinline__ int acc_row(int wm, int fm, int g, int lane) {
  constexpr int F = TileCfg<BT>::F;
  return F == 16 ? wm * (BT / 2) + fm * 16 + 4 * (lane >> 4)
                 : wm * (BT / 2) + fm * 32 + 8 * g + 4 * (lane >> 5);
}
template <int P, int BT>
__device__ __forceinline__ int acc_col(int wn, int fn, int lane) {
  constexpr int F = TileCfg<BT>::F;
  return wn * WaveCfg<P, BT>::WTN + fn * F + (lane % F);
}
// Tile column of an update accumulator.  The bf16 256 tile's update spreads a
// wave's two fragment columns 128 apart (wave wn: columns 32 wn + 128 fn ..):
// the fragments' transposing reads from the swizzled X stage then differ by a
// constant offset, which the LDS instructions take as an immediate.
template <int P, int BT>
__device__ __forceinline__ int upd_col(int wn, int fn, int lane) {
  if constexpr (P != kF32 && BT == 256) return wn * 32 + fn * 128 + (lane & 31);
  else return acc_col<P, BT>(wn, fn, lane);
}

// The epilogues read one FP32 matrix (A for B = bA + cA^2, X for X = aX + BX)
// at the accumulator positions and write others, possibly the same buffer.
// A lane's inputs of one fragment row fm (4 fragments) are loaded before the
// stores of the previous row are issued, so the loads of a row overlap instead
// of each one waiting behind the stores the compiler must keep ahead of it.
template <int P, int BT>
struct FragRow {
  float x[WaveCfg<P, BT>::FN][TileCfg<BT>::RG][4];  // [fn][row group][r]
};

template <bool NT, typename S>
__device__ __forceinline__ float load_as_float(const S* p) {
  const S v = NT ? __builtin_nontemporal_load(p) : *p;
  if constexpr (sizeof(S) == 2) return bf2f(v);
  else return v;
}

// S = float or uint16_t (bf16); NT: streaming loads (data read once per launch)
template <int P, int BT, typename S, bool NT = false>
__device__ __forceinline__ void load_frag_row(const S* __restrict__ src, size_t ld, int row0,
                                              int col0, int wm, int wn, int fm, int lane,
                                              FragRow<P, BT>& f) {
#pragma unroll
  for (int fn = 0; fn < WaveCfg<P, BT>::FN; ++fn)
#pragma unroll
    for (int g = 0; g < TileCfg<BT>::RG; ++g) {
      const size_t o = (size_t)(row0 + acc_row<BT>(wm, fm, g, lane)) * ld + col0 + acc_col<P, BT>(wn, fn, lane);
#pragma unroll
      for (int r = 0; r < 4; ++r) f.x[fn][g][r] = load_as_float<NT>(src + o + (size_t)r * ld);
    }
}

// red: LDS scratch of at least 4 * NW doubles for the epilogue's block
// reductions (the GEMM kernel gives a tail of its one LDS array, past the
// operand ring and the staging area: a kernel with a single LDS object keeps
// the compiler's LDS-DMA wait tracking from turning into a full vmcnt(0) wait
// after every stage's loads).
// A is exactly symmetric as stored (a tile's mirror holds the same bf16
// values, and a diagonal tile sums the same products in the same order at (i,j)
// and (j,i)), so the four consecutive rows i..i+3 of a lane at column j are the
// contiguous A[j][i..i+3]: one 8-byte load instead of four 2-byte ones.
template <int P, int BT>
__device__ __forceinline__ void load_frag_row_sym(const uint16_t* __restrict__ A, size_t ld, int row0,
                                                  int col0, int wm, int wn, int fm, int lane,
                                                  FragRow<P, BT>& f) {
#pragma unroll
  for (int fn = 0; fn < WaveCfg<P, BT>::FN; ++fn)
#pragma unroll
    for (int g = 0; g < TileCfg<BT>::RG; ++g) {
      const size_t o = (size_t)(col0 + acc_col<P, BT>(wn, fn, lane)) * ld + row0 + acc_row<BT>(wm, fm, g, lane);
      const u32x2 w = *gview((const u32x2*)(A + o));
      f.x[fn][g][0] = __uint_as_float(w[0] << 16);
      f.x[fn][g][1] = __uint_as_float(w[0] & 0xffff0000u);
      f.x[fn][g][2] = __uint_as_float(w[1] << 16);
      f.x[fn][g][3] = __uint_as_float(w[1] & 0xffff0000u);
    }
}

// A transposed bf16 tile of the 256 tile (the update's X^T, a SYRK tile's
// mirror) staged in the operand ring: 256 rows of 256 bf16, padded to 528
// bytes so a 16-byte-aligned row start spreads the column-wise writes over the
// banks
constexpr int kXtStageRow = 528;
constexpr int kXtStageBytes = 256 * kXtStageRow;

// STAGE (bf16 operands of the 256 tile): the tile goes to LDS transposed,
// column by column, and leaves it as whole rows twice: the staged rows are the
// mirror tile's rows, and the tile's own rows are gathered from the staged
// columns with transposing LDS reads (ds_read_b64_tr_b16: within each 16
// lanes, lane 4a+j receives element j of the 8-byte rows addressed by lanes a,
// a+4, a+8, a+12).  Stored directly, the mirror would leave the L2 in 8-byte
// pieces of 64 rows per instruction and the tile in 2-byte ones.
template <int P, int BT, bool STAGE, typename A, int FN>
__device__ __forceinline__ void epi_syrk(const KArgs& args, const MatDesc& d, int kind, int ti,
                                         int tj, float deq, const A (&acc)[4][FN], double* red,
                                         char* smem) {
  typedef TileCfg<BT> C;
  typedef WaveCfg<P, BT> W;
  static_assert(FN == W::FN, "accumulator grid");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / W::WGN, wn = wave % W::WGN;
  const size_t sp = d.sp;
  // only B = bA + cA^2 needs the step's coefficients
  float a = 0.0f, b = 0.0f, c = 0.0f;
  if (kind == KIND_A2 && !args.raw_a2) step_coef(args, d, &a, &b, &c);
  float alpha = deq;
  if (kind == KIND_GRAM && args.t == 0) {
    const float sg = d.scal[kScScale];
    alpha *= sg * sg;
  }
  const float calpha = c * deq;
  // B - beta I: the shift leaves the diagonal of the real s x s block
  const bool shifted = kind == KIND_A2 && !args.raw_a2;
  const float beta = shifted ? shift_beta(d, b, c) : 0.0f;
  if (shifted && ti == 0 && tj == 0 && threadIdx.x == 0) d.scal[kScBeta] = beta;
  float amax = 0.0f;
  float trs = 0.0f, frs = 0.0f;  // Gram: this lane's share of tr(A) and of ||A||_F^2 over the tile
  // learned path: this lane's share of the tile's moment partials (FP32; the
  // tiles' partials are summed in FP64 by the selection kernel)
  float mom[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  // the A^2 kinds read A: FP32 on the fp32 path, its bf16 copy otherwise
  const bool reads_a = kind == KIND_A2;
  typedef typename std::conditional<P == kF32, float, uint16_t>::type AT;
  const AT* Asrc = P == kF32 ? (const AT*)d.Af : (const AT*)d.As;
  static_assert(!STAGE || (P != kF32 && BT == 256), "mirror staging: bf16 tiles of 256");
  const bool stage = STAGE && !(kind == KIND_A2 && args.raw_a2);
  if (stage) __syncthreads();  // every wave is done with the operand ring
  FragRow<P, BT> pre[2];
  auto load_a = [&](int fm, FragRow<P, BT>& f) {
    if constexpr (P == kF32) load_frag_row<P, BT>(Asrc, sp, ti * BT, tj * BT, wm, wn, fm, lane, f);
    else load_frag_row_sym<P, BT>((const uint16_t*)Asrc, sp, ti * BT, tj * BT, wm, wn, fm, lane, f);
  };
  if (reads_a) load_a(0, pre[0]);
#pragma unroll
  for (int fm = 0; fm < 4; ++fm) {
    if (reads_a && fm + 1 < 4) load_a(fm + 1, pre[(fm + 1) & 1]);
    const FragRow<P, BT>& cur = pre[fm & 1];
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
#pragma unroll
      for (int g = 0; g < C::RG; ++g) {
        const int i = ti * BT + acc_row<BT>(wm, fm, g, lane);
        const int j = tj * BT + acc_col<P, BT>(wn, fn, lane);
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const size_t o = (size_t)(i + r) * sp + j;
          const float x = acc[fm][fn][4 * g + r];
          if (kind == KIND_GRAM) {
            v[r] = alpha * x;
            if (P == kF32) d.Af[o] = v[r];
            else if constexpr (!STAGE) ((uint16_t*)d.As)[o] = f2bf(v[r]);
            // the spectrum-aware init's power method reads an FP32 copy of A
            if (P != kF32 && args.init_step) d.Af[o] = v[r];
            amax = fmaxf(amax, fabsf(v[r]));
            // (staged tiles take their sum of squares from LDS during the copy-out)
            if constexpr (!STAGE) frs = __builtin_fmaf(v[r], v[r], frs);
          } else if (args.raw_a2) {
            // learned path, step 1: keep A^2 and accumulate tr(A^k) partials;
            // the combine kernel forms B once the schedule class is known
            const float a2 = deq * x;
            const float av = cur.x[fn][g][r];
            v[r] = a2;
            d.A2f[o] = a2;
            if (ti == tj && i + r == j) mom[0] += av;
            mom[1] = __builtin_fmaf(av, av, mom[1]);
            mom[2] = __builtin_fmaf(av, a2, mom[2]);
            mom[3] = __builtin_fmaf(a2, a2, mom[3]);
          } else {
            // same operation order as the learned path's combine kernel
            v[r] = __builtin_fmaf(calpha, x, b * cur.x[fn][g][r]);
            if (ti == tj && i + r == j && j < d.s) v[r] -= beta;
            if (P == kF32) ((float*)d.Bs)[o] = v[r];
            else if constexpr (!STAGE) ((uint16_t*)d.Bs)[o] = f2bf(v[r]);
          }
        }
        if (P != kF32 && kind == KIND_GRAM && args.init_step && ti != tj)
          *(float4*)(d.Af + (size_t)j * sp + i) = make_float4(v[0], v[1], v[2], v[3]);
        if (ti != tj && kind == KIND_A2 && args.raw_a2) {
          *(float4*)(d.A2f + (size_t)j * sp + i) = make_float4(v[0], v[1], v[2], v[3]);
        } else if (stage) {
          *(uint2*)(smem + (j - tj * BT) * kXtStageRow + (i - ti * BT) * 2) = pack4_bf16(v);
        } else if (ti != tj) {
          // mirrored tile: row j, columns i..i+3 (contiguous)
          const size_t o = (size_t)j * sp + i;
          if (kind == KIND_GRAM) {
            if (P == kF32) *(float4*)(d.Af + o) = make_float4(v[0], v[1], v[2], v[3]);
            else *(uint2*)((uint16_t*)d.As + o) = pack4_bf16(v);
          } else {
            if (P == kF32) *(float4*)((float*)d.Bs + o) = make_float4(v[0], v[1], v[2], v[3]);
            else *(uint2*)((uint16_t*)d.Bs + o) = pack4_bf16(v);
          }
        }
      }
    }
  }
  if constexpr (STAGE) if (stage) {
    __syncthreads();
    uint16_t* dst = (uint16_t*)(kind == KIND_GRAM ? d.As : d.Bs);
    if (ti != tj) {
      // mirror rows j = tj*BT + r, columns ti*BT .. +255: 256 rows x 32 chunks of 16 bytes
      uint16_t* mir = dst + (size_t)tj * BT * sp + (size_t)ti * BT;
      for (int ch = threadIdx.x; ch < 256 * 32; ch += W::NT) {
        const int r = ch >> 5, cc = ch & 31;
        *(u32x4*)(mir + (size_t)r * sp + cc * 8) = *(const u32x4*)(smem + r * kXtStageRow + cc * 16);
      }
    }
    // the tile's own rows: each 16 lanes take tile columns 8 jb .. 8 jb + 7
    // (staged rows) of 16 tile rows (staged columns) per step; lane s then
    // holds row 16 ib + s, eight columns, as one 16-byte store
    static_assert(W::NT / 16 == 32, "one 16-lane group per 8 columns");
    const int jb = threadIdx.x >> 4, s = threadIdx.x & 15;
    uint16_t* own = dst + (size_t)ti * BT * sp + (size_t)tj * BT + 8 * jb;
#pragma unroll 4
    for (int ib = 0; ib < 16; ++ib) {
      u32x2 h[2];
#pragma unroll
      for (int rd = 0; rd < 2; ++rd) {
        const char* p = smem + (8 * jb + 4 * rd + (s >> 2)) * kXtStageRow + (16 * ib + 4 * (s & 3)) * 2;
        h[rd] = __builtin_bit_cast(u32x2, __builtin_amdgcn_ds_read_tr16_b64_v4i16(
                                              (__attribute__((address_space(3))) i16x4*)(p)));
      }
      *(u32x4*)(own + (size_t)(16 * ib + s) * sp) = (u32x4){h[0][0], h[0][1], h[1][0], h[1][1]};
      if (kind == KIND_GRAM) {
#pragma unroll
        for (int rd = 0; rd < 2; ++rd)
#pragma unroll
          for (int e = 0; e < 2; ++e) {
            const float lo = __uint_as_float(h[rd][e] << 16), hi = __uint_as_float(h[rd][e] & 0xffff0000u);
            frs = __builtin_fmaf(lo, lo, frs);
            frs = __builtin_fmaf(hi, hi, frs);
          }
      }
    }
    // (the next tile's prologue starts with a barrier before it refills the ring)
  }
  // the A^2 product of the same step quantises A with this maximum
  if (kind == KIND_GRAM && args.fp8) wave_amax_atomic(amax, d.scal + kScAmaxA + args.t);
  if (kind == KIND_GRAM) {
    // the tile's partials of tr(A) and ||A||_F^2 (an off-diagonal tile also
    // stands for its mirror), summed in a fixed order; the diagonal is read
    // back once the tile is stored (from the staging area, else from memory:
    // the block's own stores are visible to it after the barrier)
    float* rf = (float*)red;
    __syncthreads();  // tile stored; the previous tile's reader of rf is done
    // (the init step's F^2 = tr A feeds w^2 = F^2 - z^2, which cancels: it
    // takes the FP32 copy of A, not the bf16 one)
    if (ti == tj && threadIdx.x < BT) {
      const int q = threadIdx.x;
      if (P == kF32 || args.init_step) trs = d.Af[(size_t)(ti * BT + q) * sp + tj * BT + q];
      else if constexpr (STAGE) trs = bf2f(*(const uint16_t*)(smem + q * kXtStageRow + q * 2));
      else trs = bf2f(((const uint16_t*)d.As)[(size_t)(ti * BT + q) * sp + tj * BT + q]);
    }
    for (int off = 32; off > 0; off >>= 1) {
      trs += __shfl_xor(trs, off);
      frs += __shfl_xor(frs, off);
    }
    if (lane == 0) {
      rf[2 * wave] = trs;
      rf[2 * wave + 1] = frs;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      float t0 = 0.0f, t1 = 0.0f;
#pragma unroll
      for (int w = 0; w < W::NW; ++w) {
        t0 += rf[2 * w];
        t1 += rf[2 * w + 1];
      }
      const int tileid = tri_index(ti, tj, d.nb);
      d.trp[2 * tileid] = t0;
      d.trp[2 * tileid + 1] = (ti == tj ? 1.0f : 2.0f) * t1;
    }
  }
  if (kind == KIND_A2 && args.raw_a2) {
    // fixed-order block reduction of the tile's moment partials
    // (an off-diagonal tile also stands for its mirror: weight 2 except on tr A)
    const int tileid = tri_index(ti, tj, d.nb);
    const float wgt = ti == tj ? 1.0f : 2.0f;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float x = mom[k];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
      mom[k] = x;
    }
    float* rf = (float*)red;
    __syncthreads();
    if (lane == 0)
      for (int k = 0; k < 4; ++k) rf[k * W::NW + wave] = mom[k];
    __syncthreads();
    if (threadIdx.x < 4) {
      const int k = threadIdx.x;
      float t = 0.0f;
#pragma unroll
      for (int w = 0; w < W::NW; ++w) t += rf[k * W::NW + w];
      d.mom[(size_t)tileid * 4 + k] = k == 0 ? t : wgt * t;
    }
  }
}


// STAGE (last step only): the bf16 output or the Muon weights go through an
// LDS tile (stage_out below); X0B (first step, MatDesc::x0b): X_0 is read
// from its exact bf16 copy instead of an FP32 master.  Each form is an
// instantiation of its own, so that every loop stays small enough to unroll
// fully and index the accumulators with constants.
template <int P, int BT, bool LAST, bool STAGE, bool X0B, typename A, int FN>
__device__ __forceinline__ void epi_update(const KArgs& args, const MatDesc& d, int tm, int tn,
                                           const A (&acc)[4][FN], char* smem) {
  typedef TileCfg<BT> C;
  typedef WaveCfg<P, BT> W;
  static_assert(FN == W::FN, "accumulator grid");
  // the last step stages a bf16 output tile the same way, in the caller's
  // orientation, and stores whole rows (ragged edges element by element); the
  // Muon weight step then reads and writes W by whole rows too, from the
  // staged bf16 X (the values a bf16 output holds)
  constexpr bool stage_out = STAGE;
  static_assert(!STAGE || (LAST && P != kF32 && BT == 256), "staged output: last step, bf16 256 tile");
  // Streaming loads and stores on the 256 tile, which serves matrices whose
  // iterates are far larger than the caches: its outputs are read by later
  // launches only, and streaming keeps the L2 for the operand panels.  The 128
  // tile serves small matrices, whose working set stays in the caches from one
  // launch to the next, so it keeps ordinary loads and stores.
  constexpr bool kStream = BT == 256;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / W::WGN, wn = wave % W::WGN;
  float a, b, c;
  step_coef(args, d, &a, &b, &c);
  // the B operand holds B - beta I (a matrix past its schedule copies X: a = 1)
  if (!args.fast && !past_schedule(args, d)) a += d.scal[kScBeta];
  const float alpha = (args.t == 0) ? d.scal[kScScale] : 1.0f;
  const size_t Lp = d.Lp, sp = d.sp;
  void* XTn = (args.t & 1) ? d.XT0 : d.XT1;   // fp32 path
  uint16_t* Xbn = P != kF32 ? xb_next(args, d) : nullptr;
  float amax = 0.0f;
  if (stage_out) __syncthreads();  // every wave is done with the operand ring
  // FP32 inputs prefetched one piece ahead: 16 values per lane, i.e. one
  // fragment of the 256 tile (four row groups) or a fragment row of the 128
  // tile (FN fragments of one row group); a whole fragment row of the 256 tile
  // would spill
  constexpr int PF = BT == 256 ? 1 : FN;  // fragments per piece
  constexpr int NPIECE = 4 * FN / PF;
  float pre[2][PF][C::RG][4];
  auto load_piece = [&](int u, float (&dst)[PF][C::RG][4]) {
    const int fm = u * PF / FN, fn0 = u * PF % FN;
#pragma unroll
    for (int f = 0; f < PF; ++f)
#pragma unroll
      for (int g = 0; g < C::RG; ++g) {
        const size_t o = (size_t)(tm * BT + acc_row<BT>(wm, fm, g, lane)) * Lp + tn * BT +
                         upd_col<P, BT>(wn, fn0 + f, lane);
        if constexpr (X0B) {
          // X_0 in bf16, also the operand other tiles are reading: ordinary loads
          const uint16_t* x0 = xb_cur(args, d);
#pragma unroll
          for (int r = 0; r < 4; ++r) dst[f][g][r] = load_as_float<false>(x0 + o + (size_t)r * Lp);
        } else {
#pragma unroll
          for (int r = 0; r < 4; ++r) dst[f][g][r] = load_as_float<kStream>(d.Xf + o + (size_t)r * Lp);
        }
      }
  };
  load_piece(0, pre[0]);
#pragma unroll
  for (int u = 0; u < NPIECE; ++u) {
    if (u + 1 < NPIECE) load_piece(u + 1, pre[(u + 1) & 1]);
#pragma unroll
    for (int f = 0; f < PF; ++f) {
      const int fm = u * PF / FN, fn = u * PF % FN + f;
      const float (&cur)[C::RG][4] = pre[u & 1][f];
#pragma unroll
      for (int g = 0; g < C::RG; ++g) {
        const int i = tm * BT + acc_row<BT>(wm, fm, g, lane);
        const int n = tn * BT + upd_col<P, BT>(wn, fn, lane);
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) v[r] = alpha * (a * cur[g][r] + acc[fm][fn][4 * g + r]);
        if constexpr (!LAST) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const size_t o = (size_t)(i + r) * Lp + n;
            st_hint<kStream>(d.Xf + o, v[r]);
            if (P != kF32) Xbn[o] = f2bf(v[r]);
            amax = fmaxf(amax, fabsf(v[r]));
          }
          if constexpr (P == kF32)
            st_hint<kStream>((f32x4*)((float*)XTn + (size_t)n * sp + i), (f32x4){v[0], v[1], v[2], v[3]});
        } else if constexpr (STAGE) {
          // tile-local (row, col) in the caller's layout: (i, n), or (n, i) when transposed
          const int li = i - tm * BT, ln = n - tn * BT;
          if (d.trans) {
            *(uint2*)(smem + ln * kXtStageRow + li * 2) = pack4_bf16(v);
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) *(uint16_t*)(smem + (li + r) * kXtStageRow + ln * 2) = f2bf(v[r]);
          }
        } else if (n < d.L) {
          // Muon weight step W <- (1 - lr wd) W - lr X_T: the group's four
          // weights are loaded together, before any of them is stored
          float wv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
          if (d.W) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              if (i + r < d.s) {
                const size_t o = d.trans ? (size_t)n * d.ldw + (i + r) : (size_t)(i + r) * d.ldw + n;
                wv[r] = d.w_bf16 ? bf2f(gview((const uint16_t*)d.W)[o]) : gview((const float*)d.W)[o];
              }
            }
          }
          const float keep = 1.0f - args.mlr * args.mwd;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (i + r < d.s) {
              if (d.Out) {
                const size_t o = d.trans ? (size_t)n * d.ldo + (i + r) : (size_t)(i + r) * d.ldo + n;
                if (d.out_bf16) st_hint<kStream>((uint16_t*)d.Out + o, f2bf(v[r]));
                else st_hint<kStream>((float*)d.Out + o, v[r]);
              }
              if (d.W) {
                const size_t o = d.trans ? (size_t)n * d.ldw + (i + r) : (size_t)(i + r) * d.ldw + n;
                const float w = __builtin_fmaf(-args.mlr, v[r], keep * wv[r]);
                if (d.w_bf16) *gview_w((uint16_t*)d.W + o) = f2bf(w);
                else *gview_w((float*)d.W + o) = w;
              }
            }
          }
        }
      }
    }
  }
  if (!LAST && args.fp8_next) wave_amax_atomic(amax, d.scal + kScAmaxX + args.t + 1);
  if (stage_out) {
    __syncthreads();
    // staged rows are output rows: i (or n when transposed) from the tile's first row
    const int row0 = d.trans ? tn * BT : tm * BT, col0 = d.trans ? tm * BT : tn * BT;
    const int rows = d.trans ? d.L : d.s, cols = d.trans ? d.s : d.L;
    uint16_t* out = (uint16_t*)d.Out;
    const float keep = 1.0f - args.mlr * args.mwd;
    const bool w_vec = ((uintptr_t)d.W % 16 == 0) && (d.ldw % (d.w_bf16 ? 8 : 4) == 0);
    // each thread takes kGrp chunks of 8 row elements at a time: the group's
    // weights are all loaded before any of them is stored
    constexpr int kGrp = 4;
    static_assert((256 * 32) % (W::NT * kGrp) == 0, "staged chunks split evenly");
    for (int c0 = 0; c0 < 256 * 32; c0 += W::NT * kGrp) {
      float wv[kGrp][8];
      if (d.W) {
#pragma unroll
        for (int q = 0; q < kGrp; ++q) {
          const int ch = c0 + q * W::NT + threadIdx.x;
          const int gr = row0 + (ch >> 5), gc = col0 + (ch & 31) * 8;
          const size_t o = (size_t)gr * d.ldw + gc;
          if (gr < rows && gc + 8 <= cols && w_vec) {
            if (d.w_bf16) {
              const u32x4 raw = *(const PE_GLOBAL u32x4*)(gview((const uint16_t*)d.W) + o);
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                wv[q][2 * e] = bf2f((uint16_t)(raw[e] & 0xffffu));
                wv[q][2 * e + 1] = bf2f((uint16_t)(raw[e] >> 16));
              }
            } else {
              const PE_GLOBAL f32x4* wq = (const PE_GLOBAL f32x4*)(gview((const float*)d.W) + o);
              const f32x4 lo = wq[0], hi = wq[1];
#pragma unroll
              for (int e = 0; e < 4; ++e) {
                wv[q][e] = lo[e];
                wv[q][e + 4] = hi[e];
              }
            }
          } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) {
              wv[q][e] = 0.0f;
              if (gr < rows && gc + e < cols)
                wv[q][e] = d.w_bf16 ? bf2f(gview((const uint16_t*)d.W)[o + e]) : gview((const float*)d.W)[o + e];
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < kGrp; ++q) {
        const int ch = c0 + q * W::NT + threadIdx.x;
        const int r = ch >> 5, c8 = (ch & 31) * 8;
        const int gr = row0 + r, gc = col0 + c8;
        if (gr >= rows || gc >= cols) continue;
        const u32x4 xs = *(const u32x4*)(smem + r * kXtStageRow + c8 * 2);
        if (d.Out) {
          uint16_t* dst = out + (size_t)gr * d.ldo + gc;
          if (d.o_vec && gc + 8 <= cols) {
            st_hint<kStream>((u32x4*)dst, xs);
          } else {
            for (int e = 0; e < 8 && gc + e < cols; ++e)
              st_hint<kStream>(dst + e, (uint16_t)(xs[e >> 1] >> (16 * (e & 1))));
          }
        }
        if (d.W) {
          // Muon weight step W <- (1 - lr wd) W - lr X_T
          float w[8];
#pragma unroll
          for (int e = 0; e < 8; ++e)
            w[e] = __builtin_fmaf(-args.mlr, bf2f((uint16_t)(xs[e >> 1] >> (16 * (e & 1)))), keep * wv[q][e]);
          const size_t o = (size_t)gr * d.ldw + gc;
          if (gc + 8 <= cols && w_vec) {
            if (d.w_bf16) {
              u32x4 pk;
#pragma unroll
              for (int e = 0; e < 4; ++e) pk[e] = (uint32_t)f2bf(w[2 * e]) | ((uint32_t)f2bf(w[2 * e + 1]) << 16);
              *(PE_GLOBAL u32x4*)(gview_w((uint16_t*)d.W) + o) = pk;
            } else {
              PE_GLOBAL f32x4* wq = (PE_GLOBAL f32x4*)(gview_w((float*)d.W) + o);
              wq[0] = (f32x4){w[0], w[1], w[2], w[3]};
              wq[1] = (f32x4){w[4], w[5], w[6], w[7]};
            }
          } else {
            for (int e = 0; e < 8 && gc + e < cols; ++e) {
              if (d.w_bf16) gview_w((uint16_t*)d.W)[o + e] = f2bf(w[e]);
              else gview_w((float*)d.W)[o + e] = w[e];
            }
          }
        }
      }
    }
  }
}

// ------------------------------------------------------------- kernels
template <int P, int KIND, int BT>
__global__ __launch_bounds__((WaveCfg<P, BT>::NT), (BT == 128 ? 2 : 1)) void gemm_kernel(KArgs args) {
  using T = typename std::conditional<P == kF32, float, uint16_t>::type;
  typedef TileCfg<BT> C;
  typedef WaveCfg<P, BT> W;
  typedef typename AccT<C::ACC>::type Acc;
  constexpr int BK = P == kFP8 ? Fp8Cfg<BT>::KQ : (P == kBF16 ? DlCfg<BT>::BK : OpT<float>::kBK);
  constexpr bool UPD = KIND == KIND_UPD || KIND == KIND_UPD_LAST || KIND == KIND_UPD0;
  // direct-to-LDS operand ring (the FP8 instantiations run their updates in bf16)
  constexpr bool DL = P == kBF16 || (P == kFP8 && (BT == 256 || UPD));
  constexpr int LDSB0 = DL ? DlCfg<BT>::LDS : (P == kFP8 ? Fp8Cfg<BT>::LDS : C::LDS);
  // the bf16 256 tile stages a SYRK tile's mirror, or the last step's output
  // tile, in the same buffer
  constexpr bool kStageMirror = P != kF32 && BT == 256;
  constexpr int LDSB = (BT == 256 && P != kF32 && KIND != KIND_UPD && KIND != KIND_UPD0 && LDSB0 < kXtStageBytes)
                           ? kXtStageBytes : LDSB0;
  // SYRK kinds: a small tail past the ring for the epilogue's block reductions
  constexpr int kRedTail = (KIND == KIND_GRAM || KIND == KIND_A2) ? 256 : 0;
  static_assert(kRedTail == 0 || kRedTail >= 4 * W::NW * 8, "moment reduction fits the tail");
  __shared__ __attribute__((aligned(16))) char smem[LDSB + kRedTail];
  for (int slot = blockIdx.x; slot < args.total; slot += gridDim.x) {
    const int item = xcd_item(slot, args.total);
    const int pos = find_mat(args.offs, args.count, item);
    const MatDesc& d = args.descs[args.ord ? args.ord[pos] : pos];
    if (skip_matrix(args, d)) continue;
    const bool past = past_schedule(args, d);
    if (past && KIND != KIND_UPD_LAST) continue;
    const int local = item - args.offs[pos];
    Acc acc[4][W::FN];
#pragma unroll
    for (int fm = 0; fm < 4; ++fm)
#pragma unroll
      for (int fn = 0; fn < W::FN; ++fn) acc[fm][fn] = Acc{};
    if constexpr (UPD) {
      int tm, tn;
      banded_decode(local, d.nb, d.nbL, &tm, &tn);
      const T* Bop = args.fast ? (const T*)d.fb[args.fp_] : (const T*)d.Bs;
      // (the update always runs in bf16; the FP8 instantiation shares the bf16 loop)
      // the bf16 paths read X_t itself (row-major, k along its rows), the fp32
      // path its transpose; a matrix past its schedule: no product, the
      // epilogue copies X
      if (past) {
      } else if constexpr (DL)
        gemm_nt_tile_dl<BT, Acc, W::FN, true>((const uint16_t*)Bop, xb_cur(args, d), d.sp, d.Lp, 0, tm * BT,
                                               tn * BT, 0, d.sp, smem, acc);
      else
        gemm_nt_tile<T, BT>(Bop, (const T*)((args.t & 1) ? d.XT1 : d.XT0), d.sp, tm * BT, tn * BT, 0, d.sp,
                            smem, acc);
      if constexpr (KIND == KIND_UPD_LAST && P != kF32 && BT == 256) {
        if (d.Out ? d.out_bf16 != 0 : d.W != nullptr)
          epi_update<P, BT, true, true, false>(args, d, tm, tn, acc, smem);
        else
          epi_update<P, BT, true, false, false>(args, d, tm, tn, acc, smem);
      } else if constexpr (KIND == KIND_UPD0) {
        static_assert(P != kF32, "X_0 from a bf16 copy: bf16 paths only");
        epi_update<P, BT, false, false, true>(args, d, tm, tn, acc, smem);
      } else {
        epi_update<P, BT, KIND == KIND_UPD_LAST, false, false>(args, d, tm, tn, acc, smem);
      }
    } else {
      const int split = KIND == KIND_GRAM ? d.gram_split : d.a2_split;
      const int tile = local / split, ksp = local % split;
      int ti, tj;
      tri_decode_banded(tile, d.nb, &ti, &tj);
      const T* Op;
      int K;
      if (KIND == KIND_GRAM) {
        Op = (P == kF32) ? (const T*)d.Xf : (const T*)xb_cur(args, d);
        K = d.Lp;
      } else {
        Op = (P == kF32) ? (const T*)d.Af : (const T*)d.As;
        K = d.sp;
      }
      int k0, k1;
      split_range(K, split, ksp, BK, &k0, &k1);
      // a degree-3 step (c = 0 in the fixed schedule) needs no A^2: the
      // epilogue forms B = b A - beta I from an empty product
      if (KIND == KIND_A2 && !args.sel_coef && args.c == 0.0f) k1 = k0;
      float deq = 1.0f;
      if constexpr (P == kFP8) {
        const float q = fp8_operand_scale(d, KIND, args.t);
        deq = 1.0f / (q * q);
        if constexpr (BT == 256) {
          // e4m3 copies written by the quantisation pass (scale q already applied)
          const uint8_t* Oq = KIND == KIND_GRAM ? d.Xq : d.Aq;
          if (k1 > k0) gemm_nt_tile_dl_q8(Oq, Oq, K, ti * BT, tj * BT, k0, k1, smem, acc);
        } else {
          if (k1 > k0) gemm_nt_tile_fp8<BT>(Op, Op, K, ti * BT, tj * BT, k0, k1, q, q, smem, acc);
        }
      } else if constexpr (P == kBF16) {
        if (k1 > k0)
          gemm_nt_tile_dl<BT>((const uint16_t*)Op, (const uint16_t*)Op, K, K, 32, ti * BT, tj * BT, k0, k1,
                              smem, acc);
      } else {
        if (k1 > k0) gemm_nt_tile<T, BT>(Op, Op, K, ti * BT, tj * BT, k0, k1, smem, acc);
      }
      if (split == 1) {
        epi_syrk<P, BT, kStageMirror>(args, d, KIND, ti, tj, deq, acc, (double*)(smem + LDSB), smem);
      } else {
        // partial tile: float4 q of thread t at ((tile*split + ksp)*Q + q)*NT + t
        constexpr int Q = 4 * W::FN * C::ACC / 4;
        float4* part = (float4*)d.part + ((size_t)(tile * split + ksp) * Q) * W::NT;
#pragma unroll
        for (int fm = 0; fm < 4; ++fm)
#pragma unroll
          for (int fn = 0; fn < W::FN; ++fn)
#pragma unroll
            for (int g = 0; g < C::ACC / 4; ++g) {
              const int q = (fm * W::FN + fn) * (C::ACC / 4) + g;
              part[q * W::NT + threadIdx.x] =
                  make_float4(acc[fm][fn][4 * g], acc[fm][fn][4 * g + 1], acc[fm][fn][4 * g + 2],
                              acc[fm][fn][4 * g + 3]);
            }
      }
    }
  }
}

// ------------------------------------------------ fast rectangular iteration
// Appendix G, Algorithm 4, restarted every k steps, on FP32 operands and the
// 128 tile.  Within a segment the library carries Q_t = (prod a) I + D_t and
// R_t = Y Q_{t-1}^2 as polynomials in the segment's Gram matrix Y (all
// symmetric and commuting), so every product is a symmetric s x s product
// computed on upper-triangle tiles and mirrored:
//   B_t = b R_t + c R_t^2                       (SYRK of R_t)
//   D_t = a_t D_{t-1} + q_{t-1} B_t + D_{t-1} B_t   (D_1 = B_1, q_t = prod a)
//   P   = R_t B_t,  R_{t+1} = a_t^2 R_t + 2 a_t P + P B_t   (= R_t h_t(R_t)^2)
// and the segment ends with X <- q X + D X (the update kernel with a = q and
// D as its B operand).  One epilogue serves every product:
//   out = cacc * acc + c1 * E1 + c2 * E2 + cdiag * I   (cdiag on the real rows)
template <int BT>
__device__ __forceinline__ void epi_fast(const KArgs& args, const MatDesc& d, int ti, int tj,
                                         const f32x4 (&acc)[4][4]) {
  typedef WaveCfg<kF32, BT> W;
  static_assert(BT == 128 && W::FN == 4 && TileCfg<BT>::RG == 1, "FP32 128 tile");
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave / W::WGN, wn = wave % W::WGN;
  const size_t sp = d.sp;
  float ca = args.cacc;
  if (args.fscale) {
    const float sg = d.scal[kScScale];
    ca *= sg * sg;
  }
  const float* E1 = args.fe1 >= 0 ? d.fb[args.fe1] : nullptr;
  const float* E2 = args.fe2 >= 0 ? d.fb[args.fe2] : nullptr;
  float* out = d.fb[args.fout];
#pragma unroll
  for (int fm = 0; fm < 4; ++fm)
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
      const int i = ti * BT + acc_row<BT>(wm, fm, 0, lane);
      const int j = tj * BT + acc_col<kF32, BT>(wn, fn, lane);
      float v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const size_t o = (size_t)(i + r) * sp + j;
        float x = ca * acc[fm][fn][r];
        if (E1) x = __builtin_fmaf(args.c1, E1[o], x);
        if (E2) x = __builtin_fmaf(args.c2, E2[o], x);
        if (i + r == j && j < d.s) x += args.cdiag;
        v[r] = x;
        out[o] = x;
      }
      // mirrored tile: row j, columns i..i+3
      if (ti != tj) *(float4*)(out + (size_t)j * sp + i) = make_float4(v[0], v[1], v[2], v[3]);
    }
}

// KIND_GRAM: Y = X X^T from the FP32 master; KIND_A2: a symmetric product
// fb[fp_] fb[fq_]^T (both symmetric, so this is fb[fp_] fb[fq_]).  Items are
// the upper-triangle tiles of each matrix (no split-K).
template <int KIND>
__global__ __launch_bounds__(256, 2) void gemm_fast_kernel(KArgs args) {
  typedef TileCfg<128> C;
  __shared__ __attribute__((aligned(16))) char smem[C::LDS];
  for (int slot = blockIdx.x; slot < args.total; slot += gridDim.x) {
    const int item = xcd_item(slot, args.total);
    const int pos = find_mat(args.offs, args.count, item);
    const MatDesc& d = args.descs[pos];
    const int local = item - args.offs[pos];
    int ti, tj;
    tri_decode_banded(local, d.nb, &ti, &tj);
    f32x4 acc[4][4];
#pragma unroll
    for (int fm = 0; fm < 4; ++fm)
#pragma unroll
      for (int fn = 0; fn < 4; ++fn) acc[fm][fn] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (KIND == KIND_GRAM)
      gemm_nt_tile<float, 128>(d.Xf, d.Xf, d.Lp, ti * 128, tj * 128, 0, d.Lp, smem, acc);
    else
      gemm_nt_tile<float, 128>(d.fb[args.fp_], d.fb[args.fq_], d.sp, ti * 128, tj * 128, 0, d.sp, smem, acc);
    epi_fast<128>(args, d, ti, tj, acc);
  }
}

// ------------------------------------------------ spectrum-aware init
// Power method on the step-1 Gram matrix A = X X^T (appendix on matrices with
// large spectral gaps, k = 1): v_0 = the sign vector of Knuth's hash of the
// index (+-1/sqrt(s)), v <- A v / ||A v||; after the last step
// z = sqrt(||A v||) <= sigma_1, F^2 = tr A, w = sqrt(F^2 - z^2), and when
// z > w the cubic through (w, 1) and (z, 1):
//   a = (z^2 + z w + w^2) / (z w (z + w)),  b = -1 / (z w (z + w))
// (identity otherwise) is applied as an extra first step X <- a X + b A X.
// Vectors: d.vec[0, sp) = v, d.vec[sp, 2 sp) = y.
__global__ __launch_bounds__(256) void pw_init_kernel(KArgs args) {
  for (int mi = blockIdx.x; mi < args.count; mi += gridDim.x) {
    const MatDesc& d = args.descs[mi];
    if (d.syrk_nt == 0) continue;
    const float sc = rsqrtf((float)d.s);
    for (int i = threadIdx.x; i < d.sp; i += blockDim.x) {
      const uint32_t h = (uint32_t)i * 2654435761u;
      d.vec[i] = i < d.s ? ((h & 0x80000000u) ? -sc : sc) : 0.0f;
    }
  }
}

// y = A v: one wave per row, four rows per item, from the FP32 A (the fp32
// path's own A; on the bf16 paths the copy the init step's Gram epilogue
// writes: w^2 = tr A - z^2 cancels, and its error grows as z^2 / w^2 times
// that of z, which bf16 A would make useless)
__global__ __launch_bounds__(256) void pw_matvec_kernel(KArgs args) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int item = blockIdx.x; item < args.total; item += gridDim.x) {
    const int mi = find_mat(args.offs, args.count, item);
    const MatDesc& d = args.descs[mi];
    const int r = (item - args.offs[mi]) * 4 + wave;
    if (r >= d.sp) continue;
    const float* v = d.vec;
    float acc = 0.0f;
    const float* row = d.Af + (size_t)r * d.sp;
    for (int j = lane; j < d.sp; j += 64) acc = __builtin_fmaf(row[j], v[j], acc);
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0) d.vec[d.sp + r] = acc;
  }
}

// v = y / ||y|| (fixed-order block reduction); after the last power step the
// init coefficients
__global__ __launch_bounds__(256) void pw_norm_kernel(KArgs args) {
  __shared__ float red[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int mi = blockIdx.x; mi < args.count; mi += gridDim.x) {
    const MatDesc& d = args.descs[mi];
    if (d.syrk_nt == 0) continue;
    const float* y = d.vec + d.sp;
    float ss = 0.0f;
    for (int i = threadIdx.x; i < d.sp; i += blockDim.x) ss = __builtin_fmaf(y[i], y[i], ss);
    for (int off = 32; off > 0; off >>= 1) ss += __shfl_xor(ss, off);
    __syncthreads();
    if (lane == 0) red[wave] = ss;
    __syncthreads();
    const float nrm = sqrtf((red[0] + red[1]) + (red[2] + red[3]));
    const float inv = nrm > 0.0f ? 1.0f / nrm : 0.0f;
    for (int i = threadIdx.x; i < d.sp; i += blockDim.x) d.vec[i] = y[i] * inv;
    if (threadIdx.x == 0) d.scal[kScPowN] = nrm;
    if (args.last && wave == 0) {
      // F^2 = tr A from the Gram epilogue's per-tile partials (shift_beta with
      // b = s, c = 0 returns exactly their fixed-order sum)
      const float F2 = shift_beta(d, (float)d.s, 0.0f);
      if (lane == 0) {
        float a = 1.0f, b = 0.0f;
        const float z = sqrtf(nrm), w2 = F2 - nrm;
        if (z > 0.0f && w2 > 0.0f) {
          const float w = sqrtf(w2);
          if (z > w) {
            const float den = z * w * (z + w);
            a = (z * z + z * w + w * w) / den;
            b = -1.0f / den;
          }
        }
        d.scal[kScInitA] = a;
        d.scal[kScInitB] = b;
      }
    }
  }
}

// e4m3 copy of step t's Gram-side operand (KIND_GRAM: X_t from Xb into Xq;
// KIND_A2: A_t from As into Aq) with the step's per-tensor scale.  One item is
// 16384 elements (four chunks of 16 per thread, all loads issued first); the
// padded sizes are multiples of 65536.
template <int KIND>
__global__ __launch_bounds__(kThreads) void quant_kernel(KArgs args) {
  constexpr int kChunks = 4;
  for (int item = blockIdx.x; item < args.total; item += gridDim.x) {
    const int mi = find_mat(args.offs, args.count, item);
    const MatDesc& d = args.descs[mi];
    if (skip_matrix(args, d) || past_schedule(args, d)) continue;
    const size_t base = (size_t)(item - args.offs[mi]) * kChunks * kThreads * 16;
    const uint16_t* src = KIND == KIND_GRAM ? xb_cur(args, d) : (const uint16_t*)d.As;
    uint8_t* dst = KIND == KIND_GRAM ? d.Xq : d.Aq;
    const float inv_q = 1.0f / fp8_operand_scale(d, KIND, args.t);
    u32x4 c[kChunks][2];
#pragma unroll
    for (int k = 0; k < kChunks; ++k) {
      const size_t e0 = base + ((size_t)k * kThreads + threadIdx.x) * 16;
      c[k][0] = *(const PE_GLOBAL u32x4*)(gview(src) + e0);
      c[k][1] = *(const PE_GLOBAL u32x4*)(gview(src) + e0 + 8);
    }
#pragma unroll
    for (int k = 0; k < kChunks; ++k) {
      const size_t e0 = base + ((size_t)k * kThreads + threadIdx.x) * 16;
      const u32x4 o = {(uint32_t)cvt4_e4m3(c[k][0][0], c[k][0][1], inv_q), (uint32_t)cvt4_e4m3(c[k][0][2], c[k][0][3], inv_q),
                       (uint32_t)cvt4_e4m3(c[k][1][0], c[k][1][1], inv_q), (uint32_t)cvt4_e4m3(c[k][1][2], c[k][1][3], inv_q)};
      st_stream((u32x4*)(dst + e0), o);
    }
  }
}

template <int P, int KIND, int BT>
__global__ __launch_bounds__((WaveCfg<P, BT>::NT)) void splitk_reduce_kernel(KArgs args) {
  typedef TileCfg<BT> C;
  typedef WaveCfg<P, BT> W;
  typedef typename AccT<C::ACC>::type Acc;
  constexpr int Q = 4 * W::FN * C::ACC / 4;
  __shared__ double red[4 * W::NW];
  for (int item = blockIdx.x; item < args.total; item += gridDim.x) {
    const int mi = find_mat(args.offs, args.count, item);
    const MatDesc& d = args.descs[mi];
    if (skip_matrix(args, d) || past_schedule(args, d)) continue;
    const int tile = item - args.offs[mi];
    const int split = KIND == KIND_GRAM ? d.gram_split : d.a2_split;
    int ti, tj;
    tri_decode_banded(tile, d.nb, &ti, &tj);
    Acc acc[4][W::FN];
    const float4* part = (const float4*)d.part + ((size_t)tile * split * Q) * W::NT;
#pragma unroll
    for (int fm = 0; fm < 4; ++fm)
#pragma unroll
      for (int fn = 0; fn < W::FN; ++fn)
#pragma unroll
        for (int g = 0; g < C::ACC / 4; ++g) {
          const int q = (fm * W::FN + fn) * (C::ACC / 4) + g;
          float4 s = part[q * W::NT + threadIdx.x];
          for (int k = 1; k < split; ++k) {
            const float4 p = part[((size_t)k * Q + q) * W::NT + threadIdx.x];
            s.x += p.x; s.y += p.y; s.z += p.z; s.w += p.w;
          }
          acc[fm][fn][4 * g] = s.x;
          acc[fm][fn][4 * g + 1] = s.y;
          acc[fm][fn][4 * g + 2] = s.z;
          acc[fm][fn][4 * g + 3] = s.w;
        }
    float deq = 1.0f;
    if constexpr (P == kFP8) {
      const float q = fp8_operand_scale(d, KIND, args.t);
      deq = 1.0f / (q * q);
    }
    epi_syrk<P, BT, false>(args, d, KIND, ti, tj, deq, acc, red, nullptr);
  }
}

// q[i] = e4m3(x[i] * scale) with the conversion the FP8 path uses.
// bf16 input with a power-of-two scale takes the instruction of the FP8
// steps' quantisation pass (e4m3(x / (1/scale)), exact); other inputs scale in
// fp32 and convert with v_cvt_pk_fp8_f32.
__global__ void quantize_e4m3_kernel(const void* x, int x_bf16, uint8_t* q, int64_t n, float scale,
                                     int pow2) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (x_bf16 && pow2) {
      const uint32_t u = ((const uint16_t*)x)[i];
      q[i] = (uint8_t)((uint32_t)cvt4_e4m3(u, 0u, 1.0f / scale) & 0xffu);
    } else {
      const float v = x_bf16 ? bf2f(((const uint16_t*)x)[i]) : ((const float*)x)[i];
      q[i] = (uint8_t)(pack4_e4m3(v * scale, 0.0f, 0.0f, 0.0f) & 0xffu);
    }
  }
}

__global__ void put_words_kernel(PutChunk c) {
  for (int i = threadIdx.x; i < c.nwords; i += blockDim.x) c.dst[i] = c.w[i];
}

// ------------------------------------------------------------- launchers
hipError_t launch_finalize(const KArgs& a, hipStream_t st) {
  const int g = a.count < 1024 ? (a.count > 0 ? a.count : 1) : 1024;
  hipLaunchKernelGGL(finalize_kernel, dim3(g), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_put(const PutChunk& c, hipStream_t st) {
  hipLaunchKernelGGL(put_words_kernel, dim3(1), dim3(kThreads), 0, st, c);
  return hipGetLastError();
}

// Blocks of a kernel that fit on the device at once (occupancy calculator x CU
// count), cached per device and kernel; 0 if the runtime cannot say.  A
// grid-stride kernel launched with more blocks than this runs the surplus in
// a second round that leaves most of the device idle.
static int resident_blocks(const void* kernel, int threads) {
  constexpr int kDev = 16, kSlots = 64;
  static const void* keys[kDev][kSlots];
  static int vals[kDev][kSlots];
  static std::mutex mu;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDev) return 0;
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < kSlots; ++i) {
    if (keys[dev][i] == kernel) return vals[dev][i];
    if (keys[dev][i]) continue;
    int ncu = 0, per = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess) {
      (void)hipGetLastError();  // a failed query must not read as a failed launch
      return 0;
    }
    keys[dev][i] = kernel;
    vals[dev][i] = per * ncu;
    return vals[dev][i];
  }
  return 0;
}

template <typename K>
static int grid_for(int total, int cap, K kernel, int threads) {
  const int res = resident_blocks(reinterpret_cast<const void*>(kernel), threads);
  if (res > 0 && res < cap) cap = res;
  return total < cap ? (total > 0 ? total : 1) : cap;
}

template <int P, int BT>
static void warm_t() {
  constexpr int nt = WaveCfg<P, BT>::NT;
  resident_blocks(reinterpret_cast<const void*>(gemm_kernel<P, KIND_GRAM, BT>), nt);
  resident_blocks(reinterpret_cast<const void*>(gemm_kernel<P, KIND_A2, BT>), nt);
  resident_blocks(reinterpret_cast<const void*>(gemm_kernel<P, KIND_UPD, BT>), nt);
  resident_blocks(reinterpret_cast<const void*>(gemm_kernel<P, KIND_UPD_LAST, BT>), nt);
  if constexpr (P != kF32) resident_blocks(reinterpret_cast<const void*>(gemm_kernel<P, KIND_UPD0, BT>), nt);
  resident_blocks(reinterpret_cast<const void*>(splitk_reduce_kernel<P, KIND_GRAM, BT>), nt);
  resident_blocks(reinterpret_cast<const void*>(splitk_reduce_kernel<P, KIND_A2, BT>), nt);
}

// Fills the resident-block cache of the current device, so that launches
// recorded into a graph later make no runtime queries.
void warm_launch_grids() {
  resident_blocks(reinterpret_cast<const void*>(gemm_fast_kernel<KIND_GRAM>), 256);
  resident_blocks(reinterpret_cast<const void*>(gemm_fast_kernel<KIND_A2>), 256);
  resident_blocks(reinterpret_cast<const void*>(prep_kernel<kF32>), kThreads);
  resident_blocks(reinterpret_cast<const void*>(prep_kernel<kBF16>), kThreads);
  resident_blocks(reinterpret_cast<const void*>(quant_kernel<KIND_GRAM>), kThreads);
  resident_blocks(reinterpret_cast<const void*>(quant_kernel<KIND_A2>), kThreads);
  warm_t<kF32, 128>();
  warm_t<kF32, 256>();
  warm_t<kBF16, 128>();
  warm_t<kBF16, 256>();
  warm_t<kFP8, 128>();
  warm_t<kFP8, 256>();
}

hipError_t launch_prep(int prec, const KArgs& a, int grid_cap, hipStream_t st) {
  auto k = prec == kF32 ? prep_kernel<kF32> : prep_kernel<kBF16>;
  hipLaunchKernelGGL(k, dim3(grid_for(a.total, grid_cap, k, kThreads)), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

template <int P, int BT>
static void launch_gemm_t(int kind, const KArgs& a, int cap, hipStream_t st) {
  auto k = kind == KIND_GRAM ? gemm_kernel<P, KIND_GRAM, BT>
         : kind == KIND_A2   ? gemm_kernel<P, KIND_A2, BT>
         : !a.last           ? gemm_kernel<P, KIND_UPD, BT>
                             : gemm_kernel<P, KIND_UPD_LAST, BT>;
  if constexpr (P != kF32)
    if (kind == KIND_UPD && !a.last && a.x0b) k = gemm_kernel<P, KIND_UPD0, BT>;
  constexpr int nt = WaveCfg<P, BT>::NT;
  hipLaunchKernelGGL(k, dim3(grid_for(a.total, cap, k, nt)), dim3(nt), 0, st, a);
}

template <int P, int BT>
static void launch_reduce_t(int kind, const KArgs& a, int cap, hipStream_t st) {
  auto k = kind == KIND_GRAM ? splitk_reduce_kernel<P, KIND_GRAM, BT> : splitk_reduce_kernel<P, KIND_A2, BT>;
  constexpr int nt = WaveCfg<P, BT>::NT;
  hipLaunchKernelGGL(k, dim3(grid_for(a.total, cap, k, nt)), dim3(nt), 0, st, a);
}

hipError_t launch_gemm(int prec, int bt, int kind, const KArgs& a, int grid_cap, hipStream_t st) {
  const int g = grid_cap;
  if (prec == kFP8 && kind != KIND_UPD) {
    if (bt == 256) launch_gemm_t<kFP8, 256>(kind, a, g, st);
    else launch_gemm_t<kFP8, 128>(kind, a, g, st);
  } else if (prec == kF32) {
    if (bt == 256) launch_gemm_t<kF32, 256>(kind, a, g, st);
    else launch_gemm_t<kF32, 128>(kind, a, g, st);
  } else {
    if (bt == 256) launch_gemm_t<kBF16, 256>(kind, a, g, st);
    else launch_gemm_t<kBF16, 128>(kind, a, g, st);
  }
  return hipGetLastError();
}

hipError_t launch_power(int prec, int phase, const KArgs& a, hipStream_t st) {
  const int g = a.count < 1024 ? (a.count > 0 ? a.count : 1) : 1024;
  if (phase == 0) {
    hipLaunchKernelGGL(pw_init_kernel, dim3(g), dim3(256), 0, st, a);
  } else if (phase == 1) {
    (void)prec;
    const int gm = a.total < 2048 ? (a.total > 0 ? a.total : 1) : 2048;
    hipLaunchKernelGGL(pw_matvec_kernel, dim3(gm), dim3(256), 0, st, a);
  } else {
    hipLaunchKernelGGL(pw_norm_kernel, dim3(g), dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

hipError_t launch_fast(int kind, const KArgs& a, int grid_cap, hipStream_t st) {
  auto k = kind == KIND_GRAM ? gemm_fast_kernel<KIND_GRAM> : gemm_fast_kernel<KIND_A2>;
  hipLaunchKernelGGL(k, dim3(grid_for(a.total, grid_cap, k, 256)), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_quant(int kind, const KArgs& a, int grid_cap, hipStream_t st) {
  auto k = kind == KIND_GRAM ? quant_kernel<KIND_GRAM> : quant_kernel<KIND_A2>;
  hipLaunchKernelGGL(k, dim3(grid_for(a.total, grid_cap, k, kThreads)), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_reduce(int prec, int bt, int kind, const KArgs& a, int grid_cap, hipStream_t st) {
  const int g = grid_cap;
  if (prec == kFP8) {
    if (bt == 256) launch_reduce_t<kFP8, 256>(kind, a, g, st);
    else launch_reduce_t<kFP8, 128>(kind, a, g, st);
  } else if (prec == kF32) {
    if (bt == 256) launch_reduce_t<kF32, 256>(kind, a, g, st);
    else launch_reduce_t<kF32, 128>(kind, a, g, st);
  } else {
    if (bt == 256) launch_reduce_t<kBF16, 256>(kind, a, g, st);
    else launch_reduce_t<kBF16, 128>(kind, a, g, st);
  }
  return hipGetLastError();
}

hipError_t launch_quantize(const void* x, int x_bf16, uint8_t* q, int64_t n, float scale,
                           hipStream_t st) {
  const int64_t blocks = (n + kThreads - 1) / kThreads;
  const int g = (int)(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  int e2 = 0;
  const int pow2 = frexpf(scale, &e2) == 0.5f;
  hipLaunchKernelGGL(quantize_e4m3_kernel, dim3(g), dim3(kThreads), 0, st, x, x_bf16, q, n, scale, pow2);
  return hipGetLastError();
}

}  // namespace pe
