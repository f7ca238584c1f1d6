// Learned choice of the lower bound l (one of eight precomputed schedules) and
// its fallback.
//
// The paper fixes l = 1e-3 because a cheap lower bound on sigma_min is not
// available (Section 3.3); a wrong l costs iterations, not correctness.  Here a
// small MLP (16 -> 64 -> 64 -> 8, ReLU, FP32) reads moments of the step-1 Gram
// matrix, m_k = tr(A^k) for k = 1..4 (A = X_0 X_0^T, accumulated by the step-1
// Gram and A^2 epilogues), and picks the schedule class per matrix on the
// device.  After the last step a power iteration estimates ||X X^T - I||_2;
// matrices above the threshold are recomputed from G with the fixed l = 1e-3
// schedule (all kernels of that re-run skip the other matrices).
//
// Training kernels: per-sample forward/backward in registers, per-block
// gradient sums in fixed order, then a fixed-order sum over blocks and Adam.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pe_device.h"

namespace pe {

// ------------------------------------------------------------------ MLP
// Parameter layout: W1 [16 x 64] (row = input), b1 [64], W2 [64 x 64], b2 [64],
// W3 [64 x 8], b3 [8].
constexpr int oW1 = 0;
constexpr int ob1 = oW1 + kFeat * kMlpH;
constexpr int oW2 = ob1 + kMlpH;
constexpr int ob2 = oW2 + kMlpH * kMlpH;
constexpr int oW3 = ob2 + kMlpH;
constexpr int ob3 = oW3 + kMlpH * kClasses;
static_assert(ob3 + kClasses == kMlpParams, "parameter layout");

constexpr int kMlpBlock = 64;   // samples (threads) per block

// forward pass of one sample; h1, h2 keep the post-ReLU activations
__device__ __forceinline__ void mlp_forward1(const float* P, const float* x, float* h1, float* h2,
                                             float* logits) {
  for (int j = 0; j < kMlpH; ++j) {
    float z = P[ob1 + j];
    for (int i = 0; i < kFeat; ++i) z += x[i] * P[oW1 + i * kMlpH + j];
    h1[j] = z > 0.0f ? z : 0.0f;
  }
  for (int j = 0; j < kMlpH; ++j) {
    float z = P[ob2 + j];
    for (int i = 0; i < kMlpH; ++i) z += h1[i] * P[oW2 + i * kMlpH + j];
    h2[j] = z > 0.0f ? z : 0.0f;
  }
  for (int j = 0; j < kClasses; ++j) {
    float z = P[ob3 + j];
    for (int i = 0; i < kMlpH; ++i) z += h2[i] * P[oW3 + i * kClasses + j];
    logits[j] = z;
  }
}

__global__ __launch_bounds__(kMlpBlock) void mlp_forward_kernel(const float* params, const float* feats,
                                                                int B, float* logits) {
  __shared__ float P[kMlpParams];
  for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) P[i] = params[i];
  __syncthreads();
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  float x[kFeat], h1[kMlpH], h2[kMlpH], lg[kClasses];
  for (int i = 0; i < kFeat; ++i) x[i] = feats[(size_t)s * kFeat + i];
  mlp_forward1(P, x, h1, h2, lg);
  for (int j = 0; j < kClasses; ++j) logits[(size_t)s * kClasses + j] = lg[j];
}

// Per block: sum over its samples of the gradient of the cross-entropy (not
// yet divided by B) and of the loss, written to part[block][...].
__global__ __launch_bounds__(kMlpBlock) void mlp_grad_kernel(const float* params, const float* feats,
                                                             const int32_t* labels, int B, float* part,
                                                             float* part_loss) {
  __shared__ float P[kMlpParams];
  __shared__ float sx[kMlpBlock][kFeat];
  __shared__ float sh1[kMlpBlock][kMlpH];
  __shared__ float sh2[kMlpBlock][kMlpH];
  __shared__ float sd1[kMlpBlock][kMlpH];
  __shared__ float sd2[kMlpBlock][kMlpH];
  __shared__ float sd3[kMlpBlock][kClasses];
  __shared__ float sloss[kMlpBlock];
  const int t = threadIdx.x;
  for (int i = t; i < kMlpParams; i += blockDim.x) P[i] = params[i];
  __syncthreads();
  const int s = blockIdx.x * kMlpBlock + t;
  const bool valid = s < B;
  float x[kFeat], h1[kMlpH], h2[kMlpH], lg[kClasses];
  for (int i = 0; i < kFeat; ++i) x[i] = valid ? feats[(size_t)s * kFeat + i] : 0.0f;
  mlp_forward1(P, x, h1, h2, lg);
  // softmax cross-entropy
  float mx = lg[0];
  for (int j = 1; j < kClasses; ++j) mx = fmaxf(mx, lg[j]);
  float den = 0.0f, p[kClasses];
  for (int j = 0; j < kClasses; ++j) { p[j] = expf(lg[j] - mx); den += p[j]; }
  const int y = valid ? labels[s] : 0;
  float d3[kClasses];
  for (int j = 0; j < kClasses; ++j) {
    p[j] /= den;
    d3[j] = valid ? p[j] - (j == y ? 1.0f : 0.0f) : 0.0f;
  }
  sloss[t] = valid ? -logf(fmaxf(p[y], 1e-30f)) : 0.0f;
  // backward through the two hidden layers
  float d2[kMlpH];
  for (int i = 0; i < kMlpH; ++i) {
    float g = 0.0f;
    for (int j = 0; j < kClasses; ++j) g += d3[j] * P[oW3 + i * kClasses + j];
    d2[i] = h2[i] > 0.0f ? g : 0.0f;
  }
  for (int i = 0; i < kMlpH; ++i) {
    float g = 0.0f;
    for (int j = 0; j < kMlpH; ++j) g += d2[j] * P[oW2 + i * kMlpH + j];
    sd1[t][i] = h1[i] > 0.0f ? g : 0.0f;
  }
  for (int i = 0; i < kFeat; ++i) sx[t][i] = valid ? x[i] : 0.0f;
  for (int i = 0; i < kMlpH; ++i) {
    sh1[t][i] = valid ? h1[i] : 0.0f;
    sh2[t][i] = valid ? h2[i] : 0.0f;
    sd2[t][i] = d2[i];
  }
  for (int j = 0; j < kClasses; ++j) sd3[t][j] = d3[j];
  __syncthreads();
  // parameter gradients: sum over the block's samples in sample order
  float* out = part + (size_t)blockIdx.x * kMlpParams;
  for (int q = t; q < kMlpParams; q += blockDim.x) {
    float g = 0.0f;
    if (q < ob1) {
      const int i = q / kMlpH, j = q % kMlpH;
      for (int n = 0; n < kMlpBlock; ++n) g += sx[n][i] * sd1[n][j];
    } else if (q < oW2) {
      const int j = q - ob1;
      for (int n = 0; n < kMlpBlock; ++n) g += sd1[n][j];
    } else if (q < ob2) {
      const int i = (q - oW2) / kMlpH, j = (q - oW2) % kMlpH;
      for (int n = 0; n < kMlpBlock; ++n) g += sh1[n][i] * sd2[n][j];
    } else if (q < oW3) {
      const int j = q - ob2;
      for (int n = 0; n < kMlpBlock; ++n) g += sd2[n][j];
    } else if (q < ob3) {
      const int i = (q - oW3) / kClasses, j = (q - oW3) % kClasses;
      for (int n = 0; n < kMlpBlock; ++n) g += sh2[n][i] * sd3[n][j];
    } else {
      const int j = q - ob3;
      for (int n = 0; n < kMlpBlock; ++n) g += sd3[n][j];
    }
    out[q] = g;
  }
  if (t == 0) {
    float l = 0.0f;
    for (int n = 0; n < kMlpBlock; ++n) l += sloss[n];
    part_loss[blockIdx.x] = l;
  }
}

// Sum the block partials in block order, divide by B; optionally one Adam step
// (beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected, step counted from 1).
__global__ void mlp_reduce_kernel(const float* part, const float* part_loss, int nblk, int B,
                                  float* grad_out, float* loss_out, float* params, float* m, float* v,
                                  int step, float lr) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q == 0 && loss_out) {
    float l = 0.0f;
    for (int b = 0; b < nblk; ++b) l += part_loss[b];
    *loss_out = l / (float)B;
  }
  if (q >= kMlpParams) return;
  float g = 0.0f;
  for (int b = 0; b < nblk; ++b) g += part[(size_t)b * kMlpParams + q];
  g /= (float)B;
  if (grad_out) grad_out[q] = g;
  if (params) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float mq = b1 * m[q] + (1.0f - b1) * g;
    const float vq = b2 * v[q] + (1.0f - b2) * g * g;
    m[q] = mq;
    v[q] = vq;
    const float mh = mq / (1.0f - powf(b1, (float)step));
    const float vh = vq / (1.0f - powf(b2, (float)step));
    params[q] -= lr * mh / (sqrtf(vh) + 1e-8f);
  }
}

// ----------------------------------------------------- features and selection
// Must agree with the host feature code used for training (learned.py); FP32
// here (FP64 on the device is kept to the norm's cross-block sum).
__device__ void features_from_moments(int s, int L, const float* m, float* f) {
  const float m1 = fmaxf(m[0], 1e-37f), m2 = fmaxf(m[1], 1e-37f), m3 = fmaxf(m[2], 1e-37f),
              m4 = fmaxf(m[3], 1e-37f);
  const float ls = logf((float)(s > 1 ? s : 1)), lL = logf((float)(L > 1 ? L : 1));
  const float l1 = logf(m1), l2 = logf(m2), l3 = logf(m3), l4 = logf(m4);
  const float den = fmaxf(ls, 1e-3f);
  f[0] = ls / 8.0f;
  f[1] = lL / 8.0f;
  f[2] = lL - ls;
  f[3] = l1;
  f[4] = l2 / 4.0f;
  f[5] = l3 / 8.0f;
  f[6] = l4 / 8.0f;
  f[7] = (2.0f * l1 - l2) / den;
  f[8] = (2.0f * l2 - l4) / den;
  f[9] = l1 + l3 - 2.0f * l2;
  f[10] = l2 + l4 - 2.0f * l3;
  f[11] = l4 / 8.0f - l1 / 2.0f;
  f[12] = (2.0f * l1 - l2) / 8.0f;
  f[13] = (2.0f * l2 - l4) / 8.0f;
  f[14] = ls - (2.0f * l1 - l2);
  f[15] = 1.0f;
}

// One block per matrix: reduce the tile moments (fixed order), features, MLP,
// argmax (first maximum wins, i.e. the larger l on ties), store the class.
__global__ __launch_bounds__(64) void select_kernel(KArgs args) {
  __shared__ float P[kMlpParams];
  __shared__ float red[4][64];
  if (args.mlp)
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) P[i] = args.mlp[i];
  __syncthreads();
  for (int mi = blockIdx.x; mi < args.count; mi += gridDim.x) {
    const MatDesc& d = args.descs[mi];
    if (!d.selp) continue;
    float acc[4] = {0, 0, 0, 0};
    for (int u = threadIdx.x; u < d.syrk_nt; u += blockDim.x)
      for (int k = 0; k < 4; ++k) acc[k] += d.mom[(size_t)u * 4 + k];
    for (int k = 0; k < 4; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
      float m[4];
      for (int k = 0; k < 4; ++k) {
        float t = 0.0f;
        for (int i = 0; i < 64; ++i) t += red[k][i];
        m[k] = t;
      }
      float f[kFeat];
      features_from_moments(d.s, d.L, m, f);
      for (int i = 0; i < kFeat; ++i) d.feat[i] = f[i];
      int cls = args.fixed_class;
      if (args.force_class >= 0) {
        cls = args.force_class;
      } else if (args.mlp) {
        float h1[kMlpH], h2[kMlpH], lg[kClasses];
        mlp_forward1(P, f, h1, h2, lg);
        cls = 0;
        for (int j = 1; j < kClasses; ++j)
          if (lg[j] > lg[cls]) cls = j;
      }
      *d.selp = cls;
      *d.flagp = 0;
    }
    __syncthreads();
  }
}

// B - beta I, B = b_c A + c_c A^2, over the padded s x s block once the class
// is known (beta = tr(B)/s from the step-1 Gram partials, as in the fused A^2
// epilogue; the diagonal is shifted on the real s rows only).
template <int P>
__global__ __launch_bounds__(256) void combine_kernel(KArgs args) {
  for (int item = blockIdx.x; item < args.total; item += gridDim.x) {
    int lo = 0, hi = args.count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (args.offs[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const MatDesc& d = args.descs[lo];
    const int row = item - args.offs[lo];  // one row of the s x s block per item
    int cls = *d.selp;
    if (cls < 0 || cls >= kClasses) cls = args.fixed_class;
    const float* cf = args.sel_coef + ((size_t)cls * args.tmax + args.t) * 3;
    const float b = cf[1], c = cf[2];
    const float beta = shift_beta(d, b, c);
    if (row == 0 && threadIdx.x == 0) d.scal[kScBeta] = beta;
    const size_t base = (size_t)row * d.sp;
    for (int j = threadIdx.x; j < d.sp; j += blockDim.x) {
      const float av = P == kF32 ? d.Af[base + j]
                                 : __uint_as_float((uint32_t)((const uint16_t*)d.As)[base + j] << 16);
      // same operation order as the fused A^2 epilogue (there c * deq, deq = 1)
      float v = __builtin_fmaf(c, d.A2f[base + j], b * av);
      if (j == row && row < d.s) v -= beta;
      if (P == kF32) ((float*)d.Bs)[base + j] = v;
      else {
        uint32_t u = __float_as_uint(v);
        u += 0x7fffu + ((u >> 16) & 1u);
        ((uint16_t*)d.Bs)[base + j] = (uint16_t)(u >> 16);
      }
    }
  }
}

// ------------------------------------------------ ||X X^T - I||_2 estimate
// Power iteration on M = X X^T - I with X the oriented s x L result, read from
// the caller's output (element (i, k) of X is Out[i][k], or Out[k][i] for tall
// inputs).  Per iteration: w = X^T v, y = X w, v <- (y - v) / ||y - v||.
__device__ __forceinline__ float out_at(const MatDesc& d, size_t r, size_t c) {
  const size_t o = r * d.ldo + c;
  if (d.out_bf16) return __uint_as_float((uint32_t)((const uint16_t*)d.Out)[o] << 16);
  return ((const float*)d.Out)[o];
}

// deterministic start vector: a hash of (matrix, index) -> +-1 / sqrt(s)
__global__ void est_init_kernel(KArgs args) {
  for (int mi = blockIdx.x; mi < args.count; mi += gridDim.x) {
    const MatDesc& d = args.descs[mi];
    if (!d.selp) continue;
    const float sc = rsqrtf((float)d.s);
    for (int i = threadIdx.x; i < d.s; i += blockDim.x) {
      uint32_t h = (uint32_t)i * 2654435761u ^ (uint32_t)mi * 40503u;
      h ^= h >> 15; h *= 2246822519u; h ^= h >> 13;
      d.vec[i] = (h & 1u) ? sc : -sc;
    }
  }
}

// Matrix-vector products over the output matrix (m x n, row-major, ld):
//  row dot:  y[r] = sum_c Out[r][c] x[c]       one wave per row
//  col acc:  y[c] = sum_r Out[r][c] x[r]       64 columns per block, 4 row groups
// phase 0 computes w = X^T v (length L), phase 1 computes y = X w (length s).
__global__ __launch_bounds__(256) void est_matvec_kernel(KArgs args) {
  __shared__ float part[4][64];
  for (int item = blockIdx.x; item < args.total; item += gridDim.x) {
    int lo = 0, hi = args.count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (args.offs[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const MatDesc& d = args.descs[lo];
    const int local = item - args.offs[lo];
    float* v = d.vec;                 // [sp]
    float* y = d.vec + d.sp;          // [sp]
    float* w = d.vec + 2 * (size_t)d.sp;  // [Lp]
    const float* x = args.est_phase == 0 ? v : w;
    float* dst = args.est_phase == 0 ? w : y;
    // row-dot when the product runs along Out's rows
    const bool rowdot = (args.est_phase == 0) == (d.trans != 0);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (rowdot) {
      const int r = local * 4 + wave;
      const int nrow = d.m, ncol = d.n;
      float acc = 0.0f;
      if (r < nrow)
        for (int c = lane; c < ncol; c += 64) acc += out_at(d, r, c) * x[c];
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
      if (lane == 0 && r < nrow) dst[r] = acc;
    } else {
      const int c = local * 64 + lane;
      float acc = 0.0f;
      if (c < d.n)
        for (int r = wave; r < d.m; r += 4) acc += out_at(d, r, c) * x[r];
      part[wave][lane] = acc;
      __syncthreads();
      if (wave == 0 && c < d.n) dst[c] = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
      __syncthreads();
    }
  }
}

// v <- (y - v) / ||y - v||; est = ||y - v|| (|v| = 1).  On the last iteration
// also decide the fallback.
__global__ __launch_bounds__(256) void est_norm_kernel(KArgs args, int last) {
  __shared__ float red[4];
  for (int mi = blockIdx.x; mi < args.count; mi += gridDim.x) {
    const MatDesc& d = args.descs[mi];
    if (!d.selp) continue;
    float* v = d.vec;
    const float* y = d.vec + d.sp;
    float acc = 0.0f;
    for (int i = threadIdx.x; i < d.s; i += blockDim.x) {
      const float z = y[i] - v[i];
      acc += z * z;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    const float nrm = sqrtf((red[0] + red[1]) + (red[2] + red[3]));
    __syncthreads();
    const float inv = nrm > 0.0f ? 1.0f / nrm : 0.0f;
    for (int i = threadIdx.x; i < d.s; i += blockDim.x) v[i] = (y[i] - v[i]) * inv;
    if (threadIdx.x == 0) {
      d.est[0] = nrm;
      if (last) {
        const int fail = (args.tau > 0.0f) && (nrm > args.tau) && (*d.selp != args.fixed_class);
        *d.flagp = fail;
        d.est[1] = (float)fail;
        if (fail) *d.selp = args.fixed_class;
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- launchers
hipError_t launch_mlp_forward(const float* params, const float* feats, int B, float* logits,
                              hipStream_t st) {
  hipLaunchKernelGGL(mlp_forward_kernel, dim3((B + kMlpBlock - 1) / kMlpBlock), dim3(kMlpBlock), 0,
                     st, params, feats, B, logits);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* params, const float* feats, const int32_t* labels, int B,
                           float* part, float* part_loss, float* grad_out, float* loss_out,
                           float* upd_params, float* m, float* v, int step, float lr, hipStream_t st) {
  const int nblk = (B + kMlpBlock - 1) / kMlpBlock;
  hipLaunchKernelGGL(mlp_grad_kernel, dim3(nblk), dim3(kMlpBlock), 0, st, params, feats, labels, B,
                     part, part_loss);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, part,
                     part_loss, nblk, B, grad_out, loss_out, upd_params, m, v, step, lr);
  return hipGetLastError();
}

hipError_t launch_select(const KArgs& a, hipStream_t st) {
  const int g = a.count < 1024 ? (a.count > 0 ? a.count : 1) : 1024;
  hipLaunchKernelGGL(select_kernel, dim3(g), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_combine(int prec, const KArgs& a, hipStream_t st) {
  const int g = a.total < 4096 ? (a.total > 0 ? a.total : 1) : 4096;
  if (prec == kF32) hipLaunchKernelGGL(combine_kernel<kF32>, dim3(g), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(combine_kernel<kBF16>, dim3(g), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_est(const KArgs& a, int iters, hipStream_t st, const int32_t* offs_a, int total_a,
                      const int32_t* offs_b, int total_b) {
  const int gm = a.count < 1024 ? (a.count > 0 ? a.count : 1) : 1024;
  hipLaunchKernelGGL(est_init_kernel, dim3(gm), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  for (int it = 0; it < iters && e == hipSuccess; ++it) {
    KArgs b = a;
    b.est_phase = 0;
    b.offs = offs_a;
    b.total = total_a;
    hipLaunchKernelGGL(est_matvec_kernel, dim3(total_a < 8192 ? (total_a > 0 ? total_a : 1) : 8192),
                       dim3(256), 0, st, b);
    b.est_phase = 1;
    b.offs = offs_b;
    b.total = total_b;
    hipLaunchKernelGGL(est_matvec_kernel, dim3(total_b < 8192 ? (total_b > 0 ? total_b : 1) : 8192),
                       dim3(256), 0, st, b);
    hipLaunchKernelGGL(est_norm_kernel, dim3(gm), dim3(256), 0, st, a, it == iters - 1 ? 1 : 0);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace pe
