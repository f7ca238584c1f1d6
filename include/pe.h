/*
 * pe.h -- C ABI of the MI355X (gfx950) Polar Express library.
 *
 * Polar Express (Amsel, Persson, Musco, Gower, arXiv 2505.16932) approximates
 * polar(M) = U V^T (eq. matrixsign) by a composition of odd quintics
 * p_t(x) = a_t x + b_t x^3 + c_t x^5 chosen greedily to be minimax optimal on
 * [l_t, u_t] (Theorem 1), applied to a normalised input (Section 3.5,
 * Algorithm 1 and the Appendix A.1 listing):
 *     X_0 = G / (1.01 ||G||_F + 1e-7)
 *     for t = 1..T:  A = X X^T;  B = b_t A + c_t A^2;  X = a_t X + B X
 * with X oriented so that the Gram matrix A is formed on the smaller side.
 *
 * Conventions for every entry point:
 *  - Matrices are dense row-major: element (i, j) of an m x n matrix with
 *    leading dimension ld sits at base[i * ld + j], ld >= n.
 *  - G, X and the workspace are DEVICE pointers owned by the caller (for
 *    example PyTorch tensors).  The library never allocates device memory on
 *    the compute path; it never frees caller memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    All GPU entry points are asynchronous on that stream unless stated.
 *  - No exceptions cross the ABI; every entry point returns a pe_status and
 *    pe_status_string() describes it.  Device faults surface at the caller's
 *    next synchronisation.
 *  - X must not alias G or the workspace.  Concurrent calls on different
 *    streams must use different workspaces.
 *  - Non-finite input: a NaN or infinite entry of G makes its ||G||_F, and
 *    with it the scale of X_0, NaN or zero times infinity, so every entry of
 *    that matrix's result is NaN.  The calls are asynchronous and report no
 *    status for it; other matrices of a batched call are not affected.
 */
#ifndef PE_H
#define PE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PE_OK = 0,
  PE_EINVAL = 1,        /* invalid argument (null pointer, bad size, bad ld, bad l or T) */
  PE_EUNSUPPORTED = 2,  /* valid request this build does not implement */
  PE_ENOCONV = 3,       /* the Remez exchange did not converge */
  PE_EWORKSPACE = 4,    /* workspace missing, too small or misaligned (256 B) */
  PE_EHIP = 5           /* a HIP runtime call failed (message: pe_last_error) */
} pe_status;

/* Storage type of G and X. */
typedef enum { PE_F32 = 0, PE_BF16 = 1 } pe_dtype;

/* Arithmetic of the online stage.
 *  PE_COMPUTE_F32 : FP32 operands on FP32 MFMA, FP32 accumulation.
 *  PE_COMPUTE_BF16: FP32 master iterate; bf16 MFMA operands (X, A, B);
 *                   FP32 accumulation and FP32 epilogues.  Every path
 *                   evaluates the update as (a_t + beta) X + (B - beta I) X,
 *                   beta = tr(B) / s (the same polynomial; it moves the part
 *                   of B X that cancels against a_t X out of the bf16 product).
 *                   Matrices with min(m, n) < 16 run with FP32 operands.
 *  PE_COMPUTE_FP8 : as BF16, but in the first `fp8_steps` steps the two
 *                   Gram-side products (X X^T and A A^T) take OCP e4m3
 *                   operands with one per-tensor scale each (amax -> 448),
 *                   FP32 accumulation; the remaining steps are bf16. */
typedef enum { PE_COMPUTE_F32 = 0, PE_COMPUTE_BF16 = 1, PE_COMPUTE_FP8 = 2 } pe_compute;

/* ---------------------------------------------------------------------------
 * Offline stage: the coefficient schedule (host, FP64, synchronous,
 * thread-safe, no GPU).
 *
 * Theorem 1 (greedy is optimal) with the degree-5 Remez exchange of
 * Appendix E (Algorithm 3, eq. linearsystem) and the finite-precision changes
 * of Section 3.4 / Appendix F:
 *   u_1 = 1, l_1 = ell;  for t = 1..T:
 *     p_t = minimax odd quintic for 1 on [max(l_t, cushion*u_t), u_t]
 *           (Newton-Schulz (15/8, -10/8, 3/8) once the interval's ratio is
 *           within eps^(1/3) of 1, Algorithm 3's degenerate branch);
 *     p_t <- p_t * 2 / (p_t(l_t) + p_t(u_t))   (p(l_t), p(u_t) symmetric about 1)
 *     l_{t+1} = p_t(l_t),  u_{t+1} = 2 - l_{t+1}      (eq. newbounds)
 *   then every non-Newton-Schulz step is replaced by p_t(x / safety).
 * The default cushion applies Appendix F's ratio-1/10 rule to the image: the
 * r for which the minimax quintic on [r, 1] maps it onto an interval of ratio
 * 1/10 (levelled error 9/11), found by bisection (0.0240732742418276...).
 * cushion < 0 selects Algorithm 1's rule [max(l_t, u_t/10), u_t] (no re-centring).
 * ------------------------------------------------------------------------- */
typedef struct {
  double cushion;          /* default: the ratio-1/10 root above; 0 = pure greedy */
  double safety;           /* default 1.01; 1.0 = off */
  int32_t safety_on_last;  /* default 1; 0 = leave the last step unscaled */
} pe_coeff_opts;

/* Fill *opts with the defaults above. */
void pe_coeff_opts_default(pe_coeff_opts* opts);

/* ell in (0, 1), 1 <= T <= 64.
 *   abc       out, host, 3*T doubles: (a_t, b_t, c_t) for t = 1..T.
 *   bounds    out, host, nullable, 2*(T+1) doubles: l_1, u_1, ..., l_{T+1}, u_{T+1}.
 *   err_bound out, host, nullable: 1 - l_{T+1}, the worst-case spectral error
 *             on [ell, 1] of the composite before the safety factor (eq. optimal).
 *   iters     out, host, nullable, T ints: Remez exchanges per step (0 = NS5).
 * Returns PE_EINVAL on bad arguments, PE_ENOCONV if an exchange fails. */
pe_status pe_coeffs(double ell, int32_t T, const pe_coeff_opts* opts, double* abc,
                    double* bounds, double* err_bound, int32_t* iters);

/* Degree-3 schedule (Appendix E, eq. deg3_solution; Theorem 1): the greedy
 * composition of closed-form minimax cubics, safety factor as above (opts'
 * cushion is ignored).  abc receives T triples (a_t, b_t, 0), usable wherever
 * a degree-5 schedule is (the online stage skips the A^2 product of a step
 * whose c_t is 0).  bounds / err_bound as for pe_coeffs.  PE_EINVAL on bad
 * arguments. */
pe_status pe_coeffs_cubic(double ell, int32_t T, const pe_coeff_opts* opts, double* abc,
                          double* bounds, double* err_bound);

/* ---------------------------------------------------------------------------
 * Online stage.
 * ------------------------------------------------------------------------- */
typedef struct {
  const void* G;       /* device, m x n, leading dimension ldg (elements), dtype g_dtype */
  void* X;             /* device, m x n output, leading dimension ldx, dtype x_dtype;
                          may be NULL when W is given */
  int64_t m, n;        /* m, n >= 0; m = 0 or n = 0 is a no-op */
  int64_t ldg, ldx;    /* >= n */
  int32_t g_dtype;     /* pe_dtype */
  int32_t x_dtype;     /* pe_dtype */
  /* Muon step fused around the iteration (Section 1.1, eq. muon), optional:
   *   M <- beta M + (1 - beta) G   (in place; the iteration then runs on M)
   *   W <- (1 - lr wd) W - lr X_T  (in place, in the last step's epilogue)
   * with beta, lr, wd from pe_opts.  M: device FP32, m x n, leading dimension
   * ldm >= n, or NULL (the iteration runs on G).  W: device, m x n, ldw >= n,
   * dtype w_dtype, or NULL.  Not with the learned fallback (fallback_tau > 0),
   * whose re-run would apply the step twice. */
  float* M;
  int64_t ldm;
  void* W;
  int64_t ldw;
  int32_t w_dtype;
} pe_matrix;

typedef struct {
  int32_t T;           /* number of steps, 1..64 */
  const double* abc;   /* host, 3*T doubles (for example from pe_coeffs) */
  int32_t compute;     /* pe_compute */
  int32_t fp8_steps;   /* PE_COMPUTE_FP8 only: leading steps in e4m3 (0..T-1) */
  int32_t norm_mode;   /* 0: X_0 = G/(1.01||G||_F + 1e-7) (Appendix A.1 listing);
                          1: X_0 = G/(||G||_F + 1e-2) (Algorithm 1) */
  int32_t tile;        /* 0 = library choice (autotuned table if loaded), else a
                          tile id from pe_tile_count()/pe_tile_name(): 1 the
                          128 tile, 2 the 256 tile; other values PE_EINVAL */
  /* Learned schedule (optional).  With `predictor` (device pointer to
   * PE_MLP_PARAMS floats, see pe_mlp_*) or force_class >= 0, each matrix runs
   * one of PE_CLASSES schedules (l, T'): (1e-1, 2), (1e-1, 3), (3e-2, 3),
   * (1e-2, 4), class 4 = `abc` for all T steps, (3e-3, 4), (3e-4, T),
   * (1e-4, T), the others from pe_coeffs(l, T) with default options and cut
   * to min(T', T) steps (a matrix whose schedule has ended skips the later
   * steps' products; its X passes through).  The class is chosen on the
   * device from tr(A^k), k = 1..4, of the step-1 Gram matrix.  Afterwards
   * ||X X^T - I||_2 is estimated by power iteration; matrices above
   * fallback_tau (> 0) that did not run class 4 are recomputed from G with it. */
  const float* predictor;  /* device, PE_MLP_PARAMS floats, or NULL */
  int32_t force_class;     /* -1: the network's choice; 0..7: this class (tests) */
  float fallback_tau;      /* <= 0: no estimate and no fallback */
  /* Split-K of the two Gram-side products (A = X X^T, A^2).  When a launch
   * has fewer than 64 upper-triangle tiles of a (precision, tile) class, each
   * tile's k range is split into partial tiles (the Gram keeping at least 4
   * k-stages per part, A^2 at least 16), summed in split order by a
   * reduction kernel that runs the epilogue (deterministic).  0 = library
   * choice (up to 64), 1 = never split, n in 2..64 = at most n.  The
   * automatic factor depends on the whole call, so a matrix's result agrees
   * across calls and settings up to the FP32 summation order; with split_k = 1
   * it is the same bits in any call.  PE_EINVAL outside 0..64. */
  int32_t split_k;
  /* Fast rectangular iteration (Appendix G, Algorithm 4): with fast_restart =
   * k >= 1 the T steps run in segments of k steps, each computing the
   * composite as Q X with Q a polynomial in the segment's Gram matrix Y (two
   * products with the long side per segment instead of two per step); the
   * first segment's Y is Y + fast_eps I (the paper's guard, 1e-3; 0 keeps
   * the composite of the ordinary iteration exactly).  FP32 compute only
   * (with bf16 operands the accumulated Q loses the 3e-2 accuracy bar on
   * general spectra), no learned choice of l; PE_EUNSUPPORTED otherwise.
   * The segment's final X <- q X + D X cancels with q = prod a_t, so its
   * rounding grows with k: restarts every 3 steps (the paper's choice, q <=
   * 130 for the l = 1e-3 schedule) keep FP32 within 2e-4 of the FP64
   * Algorithm 4; k = 5 loses FP32 accuracy altogether.  0 = the ordinary
   * iteration. */
  int32_t fast_restart;
  float fast_eps;
  /* Muon hyperparameters (used where a pe_matrix carries M or W): momentum
   * coefficient beta in [0, 1), learning rate lr, decoupled weight decay wd. */
  float muon_beta;
  float muon_lr;
  float muon_wd;
  /* Spectrum-aware initialisation (appendix on matrices with large spectral
   * gaps, k = 1): > 0 runs that many power-method steps on the first Gram
   * matrix A = X_0 X_0^T (from a fixed sign vector) for z <= sigma_1, and when
   * z > w = sqrt(||X_0||_F^2 - z^2) applies the cubic through (w, 1) and
   * (z, 1) as an extra first step before the T scheduled ones (per matrix, on
   * the device).  Not with FP8 steps, the learned choice of l or the fast
   * iteration (PE_EUNSUPPORTED).  0 = off. */
  int32_t spectral_init;
} pe_opts;

#define PE_CLASSES 8
#define PE_FIXED_CLASS 4
#define PE_FEATURES 16
/* MLP 16 -> 64 -> 64 -> 8, ReLU, softmax cross-entropy.  Flat FP32 layout:
 * W1 [16 x 64] (row = input), b1 [64], W2 [64 x 64], b2 [64], W3 [64 x 8], b3 [8]. */
#define PE_MLP_PARAMS 5768

/* Bytes of device workspace needed by pe_polar / pe_polar_batched / a plan
 * for these matrices and options (0 on invalid input).  Workspace must be
 * 256-byte aligned; its contents need no initialisation. */
size_t pe_workspace_size(int32_t count, const pe_matrix* mats, const pe_opts* opts);

/* One matrix: X = PolarExpress(G).  Asynchronous on `stream`.  A zero G
 * gives a zero X (the 1e-7 guard of the normalisation).  Values are not
 * checked (the call does not synchronise): a NaN or infinite entry makes the
 * matrix's norm, and so its whole X, NaN, and in a batched call only that
 * matrix's; finite entries must keep the FP32 per-tile sums of squares of the
 * norm pass finite (|g| below about 1e17). */
pe_status pe_polar(const pe_matrix* mat, const pe_opts* opts, void* ws, size_t ws_bytes,
                   void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): pe_polar
 * with the workspace taken from a static device array of
 * PE_NOALLOC_SCRATCH_BYTES inside the library (one per device, allocated when
 * the library's code object is loaded on that device and held until the
 * process ends).  The caller still owns G and X.  Same kernels, workspace
 * layout and results as pe_polar.  Returns PE_EWORKSPACE (message in
 * pe_last_error) when the matrix needs more workspace than the array holds
 * (pe_workspace_size tells), and otherwise what pe_polar returns.  Every call
 * on one device shares that device's array, so calls that overlap on a device
 * (different streams or threads without ordering) race; calls ordered on one
 * stream do not.  No hipMalloc, hipFree or other allocating call is made. */
#define PE_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
pe_status pe_polar_noalloc(const pe_matrix* mat, const pe_opts* opts, void* stream);

/* A list of matrices of uneven shapes in grouped launches: each phase (norm,
 * Gram, A^2 + combine, update) is one persistent launch over the tiles of all
 * matrices.  The tile tables are written into the workspace by small kernels
 * on `stream` (no host synchronisation); a plan does that once for repeated
 * calls on the same matrices. */
pe_status pe_polar_batched(int32_t count, const pe_matrix* mats, const pe_opts* opts,
                           void* ws, size_t ws_bytes, void* stream);

/* Plans: the grouped launches of pe_polar_batched with the tile tables built
 * and uploaded once and the whole T-step sequence captured as a hipGraph on
 * the first launch.  The plan keeps the pointers it was created with; the
 * caller keeps G, X and ws alive and unchanged in shape while it exists. */
typedef struct pe_plan pe_plan;
pe_status pe_plan_create(int32_t count, const pe_matrix* mats, const pe_opts* opts, void* ws,
                         size_t ws_bytes, void* stream, pe_plan** plan);
/* use_graph = 1: replay the captured graph; 0: launch the kernels eagerly. */
pe_status pe_plan_launch(pe_plan* plan, void* stream, int32_t use_graph);
pe_status pe_plan_destroy(pe_plan* plan);

/* Diagnostic: enqueue one phase of one step of a plan on `stream`, eagerly,
 * so that a profiler or timer can measure that kernel alone.  phase: 0 = norm
 * and copies of X_0, 1 = Gram product (with its split-K reduction),
 * 2 = A^2 + combine (with its reduction), 3 = update X = aX + BX.  The phase
 * reads whatever the plan's buffers hold (run pe_plan_launch first); the
 * buffers are left in an unspecified state, the caller's X untouched unless
 * step = T-1 and phase = 3.  PE_EINVAL for a bad step or phase;
 * PE_EUNSUPPORTED for a plan with the learned choice of l. */
pe_status pe_plan_launch_phase(pe_plan* plan, int32_t step, int32_t phase, void* stream);

/* The e4m3 conversion of the FP8 path, for checking it: q[i] = e4m3(x[i] * scale)
 * (OCP E4M3, round to nearest even; |x[i] * scale| must not exceed 448, which the
 * FP8 path guarantees by choosing scale as the largest power of two with
 * 1.01 * max|x| * scale <= 448).  x: device, n elements of x_dtype; q: device,
 * n bytes.  Asynchronous on `stream`.  PE_EINVAL for bad pointers, n < 0, or a
 * non-positive or non-finite scale. */
pe_status pe_quantize_e4m3(const void* x, int32_t x_dtype, void* q, int64_t n, float scale,
                           void* stream);

/* After a learned plan's launch: per matrix the class used, the 16 features,
 * the ||X X^T - I||_2 estimate and the fallback flag (host outputs, each
 * nullable; classes/flags count ints, feats count*16 and est count floats;
 * an empty matrix reports class -1).  One copy from the plan's workspace,
 * ordered on `stream` after the work already queued there (the launch's
 * stream), then a synchronisation of that stream only. */
pe_status pe_plan_selection(pe_plan* plan, void* stream, int32_t* classes, float* feats, float* est,
                            int32_t* flags);

/* ---------------------------------------------------------------------------
 * Training kernels of the l-predictor (device pointers, FP32, asynchronous).
 * feats: B x 16 row-major; labels: B class indices.  Workspace for B samples:
 * pe_mlp_workspace_size(B) bytes (256-byte aligned).
 * ------------------------------------------------------------------------- */
size_t pe_mlp_workspace_size(int32_t B);
/* logits: B x 8 */
pe_status pe_mlp_forward(const float* params, const float* feats, int32_t B, float* logits,
                         void* stream);
/* grad: PE_MLP_PARAMS, mean cross-entropy gradient; loss: 1 float (nullable) */
pe_status pe_mlp_grad(const float* params, const float* feats, const int32_t* labels, int32_t B,
                      float* grad, float* loss, void* ws, size_t ws_bytes, void* stream);
/* one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected; step >= 1) in
 * place on params with moment buffers m, v (PE_MLP_PARAMS each, zero at step 1) */
pe_status pe_mlp_train_step(float* params, float* m, float* v, int32_t step, float lr,
                            const float* feats, const int32_t* labels, int32_t B, float* loss,
                            void* ws, size_t ws_bytes, void* stream);

/* Tile configurations compiled into the library (0 = auto, 1 = 128 x 128,
 * 2 = 256 x 256) and the autotuned table (written by
 * paper_2505_16932_amd/autotune.py); loading a table replaces the previous one. */
int32_t pe_tile_count(void);
const char* pe_tile_name(int32_t tile_id);
/* Lines "<shape-class>_<regime> <tile-id>" ('#' starts a comment); tile-id 1
 * or 2; regime xN for calls of at least 3e12 algorithmic FLOP per step
 * (sum of 3 s^2 L + s^3) or with more than 1024 update tiles of 256, x1
 * otherwise.  With a table
 * loaded and opts.tile = 0, each matrix of a call takes its class's tile, and
 * every phase of the call launches once per (precision, tile) class present;
 * matrices whose class is missing take the built-in rule (256 for s >= 512 in
 * calls with at least 256 update tiles of 256, else 128).  FP32 matrices use
 * the 128 tile unless opts.tile forces 256.  PE_EINVAL on a malformed file. */
pe_status pe_tile_table_load(const char* path);
/* Shape class of an m x n matrix for the compute mode (the table's key). */
const char* pe_shape_class(int32_t compute, int64_t m, int64_t n);

const char* pe_status_string(pe_status st);
/* Text of the last HIP error seen by this thread (empty if none). */
const char* pe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PE_H */
