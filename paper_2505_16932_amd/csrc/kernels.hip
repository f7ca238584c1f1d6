// gfx950 kernels of the Polar Express online stage (Section 3.5 and the
// Appendix A.1 listing: X_0 = G / (1.01 ||G||_F + 1e-7); per step
// A = X X^T, B = b A + c A^2, X = a X + B X).
//
// Three kernel families, each launched once per phase over the tiles of every
// matrix of a call ("grouped" launches; a single matrix is a group of one):
//   prep_kernel   one HBM pass over G: orientation, sum of squares (FP64 per
//                 lane, fixed-order cross-block reduction => deterministic),
//                 max |G|, and the unscaled FP32 / bf16 / transposed copies of
//                 X_0; the scale sigma is folded into step 1's epilogues
//                 (A_1 = sigma^2 G G^T, X_1 = sigma (a G + B_1 G)).
//   gemm_kernel   128x128 block tiles, 4 wave64 in 2x2, bf16 16x16x32 or
//                 fp32 16x16x4 MFMA, FP32 accumulation, LDS double buffer.
//                 KIND_GRAM:  A = X X^T, upper-triangle tiles only, mirrored
//                             store (SYRK);
//                 KIND_A2:    B = b A + c A A^T (A symmetric, so A^2 = A A^T is
//                             again a SYRK), epilogue re-reads A;
//                 KIND_UPD:   X = a X + B X with X^T as the K-contiguous
//                             operand; writes the FP32 master, the bf16 copy
//                             and the next X^T, or the caller's output on the
//                             last step.
//                 Split-K for the Gram-side products writes partial tiles;
//                 splitk_reduce_kernel sums them in split order (deterministic)
//                 and runs the same epilogue.
// All three GEMMs are "NT": C[i][j] = sum_k P[i][k] Q[j][k] with both operands
// row-major along k, which is what the MFMA lane layout wants.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pe_device.h"

namespace pe {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

enum Kind : int { KIND_GRAM = 0, KIND_A2 = 1, KIND_UPD = 2, KIND_UPD_LAST = 3 };

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


__device__ __forceinline__ void step_coef(const KArgs& args, const MatDesc& d, float* a, float* b,
                                          float* c) {
  if (args.sel_coef) {
    const float* p = args.sel_coef + ((size_t)d.sel * args.tmax + args.t) * 3;
    *a = p[0]; *b = p[1]; *c = p[2];
  } else {
    *a = args.a; *b = args.b; *c = args.c;
  }
}

// ------------------------------------------------------------------ prep
// One 64x64 tile of the oriented, padded X per iteration of the block loop.
template <int P>
__global__ __launch_bounds__(kThreads) void prep_kernel(KArgs args) {
  __shared__ float tile[kPrepTile][kPrepTile + 1];
  __shared__ double red_d[kThreads / 64];
  __shared__ float red_f[kThreads / 64];
  __shared__ int last_flag;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int item = blockIdx.x; item < args.total; item += gridDim.x) {
    const int mi = find_mat(args.offs, args.count, item);
    const MatDesc& d = args.descs[mi];
    const int local = item - args.offs[mi];
    const int ntk = d.Lp / kPrepTile;
    const int i0 = (local / ntk) * kPrepTile;   // rows of X (s side)
    const int k0 = (local % ntk) * kPrepTile;   // cols of X (L side)
    // source block: rows r, cols c of G's own layout
    const int sr0 = d.trans ? k0 : i0, sc0 = d.trans ? i0 : k0;
    const int srn = d.trans ? d.L : d.s, scn = d.trans ? d.s : d.L;  // valid extents in G layout
    double ss = 0.0;
    float amax = 0.0f;
    const int cq = (tid & 15) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = (tid >> 4) + 16 * j;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int gr = sr0 + r, gc = sc0 + cq + e;
        float x = 0.0f;
        if (gr < srn && gc < scn) {
          const size_t off = (size_t)gr * d.ldg + gc;
          x = d.g_bf16 ? bf2f(((const uint16_t*)d.G)[off]) : ((const float*)d.G)[off];
        }
        v[e] = x;
        tile[r][cq + e] = x;
        ss += (double)x * (double)x;
        amax = fmaxf(amax, fabsf(x));
      }
      // direct output: the buffer whose row layout matches G's
      if (!d.trans) {
        const size_t o = (size_t)(i0 + r) * d.Lp + k0 + cq;
        if (P == kF32) {
          *(float4*)(d.Xf + o) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
          *(float4*)(d.Xf + o) = make_float4(v[0], v[1], v[2], v[3]);
          uint2 pk;
          pk.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
          pk.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
          *(uint2*)((uint16_t*)d.Xb + o) = pk;
        }
      } else {
        const size_t o = (size_t)(k0 + r) * d.sp + i0 + cq;
        if (P == kF32) {
          *(float4*)((float*)d.XT0 + o) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
          uint2 pk;
          pk.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
          pk.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
          *(uint2*)((uint16_t*)d.XT0 + o) = pk;
        }
      }
    }
    __syncthreads();
    // transposed output from LDS
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = (tid >> 4) + 16 * j;
      float v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = tile[cq + e][r];
      if (!d.trans) {
        // XT[k][i]: row k = k0 + r, cols i0 + cq..
        const size_t o = (size_t)(k0 + r) * d.sp + i0 + cq;
        if (P == kF32) {
          *(float4*)((float*)d.XT0 + o) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
          uint2 pk;
          pk.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
          pk.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
          *(uint2*)((uint16_t*)d.XT0 + o) = pk;
        }
      } else {
        const size_t o = (size_t)(i0 + r) * d.Lp + k0 + cq;
        *(float4*)(d.Xf + o) = make_float4(v[0], v[1], v[2], v[3]);
        if (P != kF32) {
          uint2 pk;
          pk.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
          pk.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
          *(uint2*)((uint16_t*)d.Xb + o) = pk;
        }
      }
    }
    // block reduction of this tile's sum of squares and max, fixed order
    for (int off = 32; off > 0; off >>= 1) {
      ss += __shfl_xor(ss, off);
      amax = fmaxf(amax, __shfl_xor(amax, off));
    }
    if (lane == 0) { red_d[wave] = ss; red_f[wave] = amax; }
    __syncthreads();
    if (tid == 0) {
      const double s4 = (red_d[0] + red_d[1]) + (red_d[2] + red_d[3]);
      const float a4 = fmaxf(fmaxf(red_f[0], red_f[1]), fmaxf(red_f[2], red_f[3]));
      d.red[local] = s4;
      ((float*)(d.red + d.n_prep))[local] = a4;
      __threadfence();
      const uint32_t prev = atomicAdd(&d.cnt[0], 1u);
      last_flag = (prev == (uint32_t)d.n_prep - 1u);
    }
    __syncthreads();
    if (last_flag) {
      // the block that finished this matrix's last tile reduces all partials
      __threadfence();
      double acc = 0.0;
      float am = 0.0f;
      const volatile double* rd = d.red;
      const volatile float* rf = (const volatile float*)(d.red + d.n_prep);
      for (int i = tid; i < d.n_prep; i += kThreads) {
        acc += rd[i];
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
        d.cnt[0] = 0u;
      }
      // clear the amax slots the later steps accumulate into
      for (int i = kScAmaxX + tid; i < kScN; i += kThreads) d.scal[i] = 0.0f;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- GEMM core
// Block tile BT x BT (BT = 128 or 256), 4 wave64 in a 2 x 2 grid, each wave a
// (BT/2) x (BT/2) tile of 4 x 4 MFMA fragments of F x F, F = BT/8:
//   F = 16: v_mfma_f32_16x16x32_bf16 / v_mfma_f32_16x16x4_f32
//   F = 32: v_mfma_f32_32x32x16_bf16 / v_mfma_f32_32x32x2_f32
// One LDS stage holds 128 bytes of k per row (64 bf16 or 32 fp32) plus a
// 16-byte pad (bank spread), for both operands; two stages are double-buffered.
// A lane reads its fragment as one 16-byte chunk: rows lane % F, k-chunk
// lane / F within a sub-step of F == 16 ? 64 : 32 bytes.
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

template <typename T>
struct OpT;
template <>
struct OpT<uint16_t> {  // bf16
  static constexpr int kVec = 8;   // elements per 16-byte chunk
  static constexpr int kBK = 64;   // k per LDS stage (128 bytes)
};
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
        if constexpr (sizeof(T) == 2) {
          if constexpr (F == 16)
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                __builtin_bit_cast(bf16x8, fa[fm]), __builtin_bit_cast(bf16x8, fb[fn]), acc[fm][fn],
                0, 0, 0);
          else
            acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(bf16x8, fa[fm]), __builtin_bit_cast(bf16x8, fb[fn]), acc[fm][fn],
                0, 0, 0);
        } else {
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
}

// acc += P[rp0:rp0+BT, k0:k1] * Q[rq0:rq0+BT, k0:k1]^T, (k1 - k0) % BK == 0.
template <typename T, int BT, typename A>
__device__ __forceinline__ void gemm_nt_tile(const T* __restrict__ P, const T* __restrict__ Q,
                                             int64_t ld, int rp0, int rq0, int k0, int k1,
                                             char* smem, A (&acc)[4][4]) {
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

// upper-triangle tile index -> (ti, tj), ti <= tj, row-major over ti
__device__ __forceinline__ void tri_decode(int u, int nb, int* ti, int* tj) {
  int r = 0, rowlen = nb;
  while (u >= rowlen) { u -= rowlen; ++r; --rowlen; }
  *ti = r;
  *tj = r + u;
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

// ------------------------------------------------------------- epilogues
// Accumulator element (fm, fn, g, r) is C[row][col] of the block tile with
//   F = 16: row = wm*BT/2 + fm*16 + 4*(lane/16) + r,           col = wn*BT/2 + fn*16 + lane%16
//   F = 32: row = wm*BT/2 + fm*32 + 8*g + 4*(lane/32) + r,     col = wn*BT/2 + fn*32 + lane%32
// with acc register index 4*g + r; each (fm, fn, g) is four consecutive rows.
template <int BT>
__device__ __forceinline__ int acc_row(int wm, int fm, int g, int lane) {
  constexpr int F = TileCfg<BT>::F;
  return F == 16 ? wm * (BT / 2) + fm * 16 + 4 * (lane >> 4)
                 : wm * (BT / 2) + fm * 32 + 8 * g + 4 * (lane >> 5);
}
template <int BT>
__device__ __forceinline__ int acc_col(int wn, int fn, int lane) {
  constexpr int F = TileCfg<BT>::F;
  return wn * (BT / 2) + fn * F + (lane % F);
}

template <int P, int BT, typename A>
__device__ __forceinline__ void epi_syrk(const KArgs& args, const MatDesc& d, int kind, int ti,
                                         int tj, const A (&acc)[4][4]) {
  typedef TileCfg<BT> C;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const size_t sp = d.sp;
  float a, b, c;
  step_coef(args, d, &a, &b, &c);
  float alpha = 1.0f;
  if (kind == KIND_GRAM && args.t == 0) {
    const float sg = d.scal[kScScale];
    alpha = sg * sg;
  }
  float amax = 0.0f;
#pragma unroll
  for (int fm = 0; fm < 4; ++fm) {
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
#pragma unroll
      for (int g = 0; g < C::RG; ++g) {
        const int i = ti * BT + acc_row<BT>(wm, fm, g, lane);
        const int j = tj * BT + acc_col<BT>(wn, fn, lane);
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const size_t o = (size_t)(i + r) * sp + j;
          const float x = acc[fm][fn][4 * g + r];
          if (kind == KIND_GRAM) {
            v[r] = alpha * x;
            d.Af[o] = v[r];
            if (P != kF32) ((uint16_t*)d.As)[o] = f2bf(v[r]);
            amax = fmaxf(amax, fabsf(v[r]));
          } else {
            v[r] = b * d.Af[o] + c * x;
            if (P == kF32) ((float*)d.Bs)[o] = v[r];
            else ((uint16_t*)d.Bs)[o] = f2bf(v[r]);
          }
        }
        if (ti != tj) {
          // mirrored tile: row j, columns i..i+3 (contiguous)
          const size_t o = (size_t)j * sp + i;
          if (kind == KIND_GRAM) {
            *(float4*)(d.Af + o) = make_float4(v[0], v[1], v[2], v[3]);
            if (P != kF32) *(uint2*)((uint16_t*)d.As + o) = pack4_bf16(v);
          } else {
            if (P == kF32) *(float4*)((float*)d.Bs + o) = make_float4(v[0], v[1], v[2], v[3]);
            else *(uint2*)((uint16_t*)d.Bs + o) = pack4_bf16(v);
          }
        }
      }
    }
  }
  if (kind == KIND_GRAM && P == kFP8) wave_amax_atomic(amax, d.scal + kScAmaxA + args.t);
}

template <int P, int BT, bool LAST, typename A>
__device__ __forceinline__ void epi_update(const KArgs& args, const MatDesc& d, int tm, int tn,
                                           const A (&acc)[4][4]) {
  typedef TileCfg<BT> C;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  float a, b, c;
  step_coef(args, d, &a, &b, &c);
  const float alpha = (args.t == 0) ? d.scal[kScScale] : 1.0f;
  const size_t Lp = d.Lp, sp = d.sp;
  void* XTn = (args.t & 1) ? d.XT0 : d.XT1;
  float amax = 0.0f;
#pragma unroll
  for (int fm = 0; fm < 4; ++fm) {
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
#pragma unroll
      for (int g = 0; g < C::RG; ++g) {
        const int i = tm * BT + acc_row<BT>(wm, fm, g, lane);
        const int n = tn * BT + acc_col<BT>(wn, fn, lane);
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const size_t o = (size_t)(i + r) * Lp + n;
          v[r] = alpha * (a * d.Xf[o] + acc[fm][fn][4 * g + r]);
        }
        if constexpr (!LAST) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const size_t o = (size_t)(i + r) * Lp + n;
            d.Xf[o] = v[r];
            if (P != kF32) ((uint16_t*)d.Xb)[o] = f2bf(v[r]);
            amax = fmaxf(amax, fabsf(v[r]));
          }
          const size_t ot = (size_t)n * sp + i;
          if (P == kF32) *(float4*)((float*)XTn + ot) = make_float4(v[0], v[1], v[2], v[3]);
          else *(uint2*)((uint16_t*)XTn + ot) = pack4_bf16(v);
        } else if (n < d.L) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            if (i + r < d.s) {
              const size_t o = d.trans ? (size_t)n * d.ldo + (i + r) : (size_t)(i + r) * d.ldo + n;
              if (d.out_bf16) ((uint16_t*)d.Out)[o] = f2bf(v[r]);
              else ((float*)d.Out)[o] = v[r];
            }
          }
        }
      }
    }
  }
  if (!LAST && args.fp8_next) wave_amax_atomic(amax, d.scal + kScAmaxX + args.t + 1);
}

// ------------------------------------------------------------- kernels
template <int P, int KIND, int BT>
__global__ __launch_bounds__(kThreads, BT == 128 ? 2 : 1) void gemm_kernel(KArgs args) {
  using T = typename std::conditional<P == kF32, float, uint16_t>::type;
  typedef TileCfg<BT> C;
  typedef typename AccT<C::ACC>::type Acc;
  constexpr int BK = OpT<T>::kBK;
  __shared__ __attribute__((aligned(16))) char smem[C::LDS];
  for (int item = blockIdx.x; item < args.total; item += gridDim.x) {
    const int mi = find_mat(args.offs, args.count, item);
    const MatDesc& d = args.descs[mi];
    const int local = item - args.offs[mi];
    Acc acc[4][4];
#pragma unroll
    for (int fm = 0; fm < 4; ++fm)
#pragma unroll
      for (int fn = 0; fn < 4; ++fn) acc[fm][fn] = Acc{};
    if constexpr (KIND == KIND_UPD || KIND == KIND_UPD_LAST) {
      const int tm = local % d.nb, tn = local / d.nb;
      const T* Bop = (const T*)d.Bs;
      const T* XTc = (const T*)((args.t & 1) ? d.XT1 : d.XT0);
      gemm_nt_tile<T, BT>(Bop, XTc, d.sp, tm * BT, tn * BT, 0, d.sp, smem, acc);
      epi_update<P, BT, KIND == KIND_UPD_LAST>(args, d, tm, tn, acc);
    } else {
      const int split = KIND == KIND_GRAM ? d.gram_split : d.a2_split;
      const int tile = local / split, ksp = local % split;
      int ti, tj;
      tri_decode(tile, d.nb, &ti, &tj);
      const T* Op;
      int K;
      if (KIND == KIND_GRAM) {
        Op = (P == kF32) ? (const T*)d.Xf : (const T*)d.Xb;
        K = d.Lp;
      } else {
        Op = (P == kF32) ? (const T*)d.Af : (const T*)d.As;
        K = d.sp;
      }
      int k0, k1;
      split_range(K, split, ksp, BK, &k0, &k1);
      if (k1 > k0) gemm_nt_tile<T, BT>(Op, Op, K, ti * BT, tj * BT, k0, k1, smem, acc);
      if (split == 1) {
        epi_syrk<P, BT>(args, d, KIND, ti, tj, acc);
      } else {
        // partial tile: float4 q of thread t at ((tile*split + ksp)*Q + q)*256 + t
        constexpr int Q = 16 * C::ACC / 4;
        float4* part = (float4*)d.part + ((size_t)(tile * split + ksp) * Q) * kThreads;
#pragma unroll
        for (int fm = 0; fm < 4; ++fm)
#pragma unroll
          for (int fn = 0; fn < 4; ++fn)
#pragma unroll
            for (int g = 0; g < C::ACC / 4; ++g) {
              const int q = (fm * 4 + fn) * (C::ACC / 4) + g;
              part[q * kThreads + threadIdx.x] =
                  make_float4(acc[fm][fn][4 * g], acc[fm][fn][4 * g + 1], acc[fm][fn][4 * g + 2],
                              acc[fm][fn][4 * g + 3]);
            }
      }
    }
  }
}

template <int P, int KIND, int BT>
__global__ __launch_bounds__(kThreads) void splitk_reduce_kernel(KArgs args) {
  typedef TileCfg<BT> C;
  typedef typename AccT<C::ACC>::type Acc;
  constexpr int Q = 16 * C::ACC / 4;
  for (int item = blockIdx.x; item < args.total; item += gridDim.x) {
    const int mi = find_mat(args.offs, args.count, item);
    const MatDesc& d = args.descs[mi];
    const int tile = item - args.offs[mi];
    const int split = KIND == KIND_GRAM ? d.gram_split : d.a2_split;
    int ti, tj;
    tri_decode(tile, d.nb, &ti, &tj);
    Acc acc[4][4];
    const float4* part = (const float4*)d.part + ((size_t)tile * split * Q) * kThreads;
#pragma unroll
    for (int fm = 0; fm < 4; ++fm)
#pragma unroll
      for (int fn = 0; fn < 4; ++fn)
#pragma unroll
        for (int g = 0; g < C::ACC / 4; ++g) {
          const int q = (fm * 4 + fn) * (C::ACC / 4) + g;
          float4 s = part[q * kThreads + threadIdx.x];
          for (int k = 1; k < split; ++k) {
            const float4 p = part[((size_t)k * Q + q) * kThreads + threadIdx.x];
            s.x += p.x; s.y += p.y; s.z += p.z; s.w += p.w;
          }
          acc[fm][fn][4 * g] = s.x;
          acc[fm][fn][4 * g + 1] = s.y;
          acc[fm][fn][4 * g + 2] = s.z;
          acc[fm][fn][4 * g + 3] = s.w;
        }
    epi_syrk<P, BT>(args, d, KIND, ti, tj, acc);
  }
}

// Clears the per-matrix arrival counters and amax slots at the start of every
// run, so no state carries over between calls or graph replays.
__global__ void init_kernel(const MatDesc* descs, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const MatDesc& d = descs[i];
  if (!d.cnt) return;
  for (int k = 0; k < 4; ++k) d.cnt[k] = 0u;
  for (int k = kScAmaxX; k < kScN; ++k) d.scal[k] = 0.0f;
}

__global__ void put_words_kernel(PutChunk c) {
  for (int i = threadIdx.x; i < c.nwords; i += blockDim.x) c.dst[i] = c.w[i];
}

// ------------------------------------------------------------- launchers
hipError_t launch_init(const MatDesc* descs, int count, hipStream_t st) {
  hipLaunchKernelGGL(init_kernel, dim3((count + kThreads - 1) / kThreads), dim3(kThreads), 0, st, descs, count);
  return hipGetLastError();
}

hipError_t launch_put(const PutChunk& c, hipStream_t st) {
  hipLaunchKernelGGL(put_words_kernel, dim3(1), dim3(kThreads), 0, st, c);
  return hipGetLastError();
}

static int grid_for(int total, int cap) { return total < cap ? (total > 0 ? total : 1) : cap; }

hipError_t launch_prep(int prec, const KArgs& a, int grid_cap, hipStream_t st) {
  const int g = grid_for(a.total, grid_cap);
  if (prec == kF32) hipLaunchKernelGGL(prep_kernel<kF32>, dim3(g), dim3(kThreads), 0, st, a);
  else hipLaunchKernelGGL(prep_kernel<kBF16>, dim3(g), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

template <int P, int BT>
static void launch_gemm_t(int kind, const KArgs& a, int g, hipStream_t st) {
  if (kind == KIND_GRAM)
    hipLaunchKernelGGL((gemm_kernel<P, KIND_GRAM, BT>), dim3(g), dim3(kThreads), 0, st, a);
  else if (kind == KIND_A2)
    hipLaunchKernelGGL((gemm_kernel<P, KIND_A2, BT>), dim3(g), dim3(kThreads), 0, st, a);
  else if (!a.last)
    hipLaunchKernelGGL((gemm_kernel<P, KIND_UPD, BT>), dim3(g), dim3(kThreads), 0, st, a);
  else
    hipLaunchKernelGGL((gemm_kernel<P, KIND_UPD_LAST, BT>), dim3(g), dim3(kThreads), 0, st, a);
}

template <int P, int BT>
static void launch_reduce_t(int kind, const KArgs& a, int g, hipStream_t st) {
  if (kind == KIND_GRAM)
    hipLaunchKernelGGL((splitk_reduce_kernel<P, KIND_GRAM, BT>), dim3(g), dim3(kThreads), 0, st, a);
  else
    hipLaunchKernelGGL((splitk_reduce_kernel<P, KIND_A2, BT>), dim3(g), dim3(kThreads), 0, st, a);
}

hipError_t launch_gemm(int prec, int bt, int kind, const KArgs& a, int grid_cap, hipStream_t st) {
  const int g = grid_for(a.total, grid_cap);
  if (prec == kF32) {
    if (bt == 256) launch_gemm_t<kF32, 256>(kind, a, g, st);
    else launch_gemm_t<kF32, 128>(kind, a, g, st);
  } else {
    if (bt == 256) launch_gemm_t<kBF16, 256>(kind, a, g, st);
    else launch_gemm_t<kBF16, 128>(kind, a, g, st);
  }
  return hipGetLastError();
}

hipError_t launch_reduce(int prec, int bt, int kind, const KArgs& a, int grid_cap, hipStream_t st) {
  const int g = grid_for(a.total, grid_cap);
  if (prec == kF32) {
    if (bt == 256) launch_reduce_t<kF32, 256>(kind, a, g, st);
    else launch_reduce_t<kF32, 128>(kind, a, g, st);
  } else {
    if (bt == 256) launch_reduce_t<kBF16, 256>(kind, a, g, st);
    else launch_reduce_t<kBF16, 128>(kind, a, g, st);
  }
  return hipGetLastError();
}

}  // namespace pe
