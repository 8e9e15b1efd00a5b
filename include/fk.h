/*
 * fk.h - C ABI of libfastkernel: Fourier-basis kernel ridge regression with
 * type-1 / type-2 non-uniform FFTs on AMD Instinct MI355X (gfx950).
 *
 * The method (Doumeche, Bach, Biau, Boyer, "Fast kernel methods: Sobolev,
 * physics-informed, and additive models", arXiv 2509.02649):
 *
 *   theta = (n^-1 Phi^* Phi + lambda M^* M)^-1 n^-1 Phi^* Y          (eq. kenrel_reg, Sec. 2.1)
 *
 * on the truncated Fourier basis exp(i k.x), ||k||_inf <= m (Sec. 2.2), where
 * x are torus radians (x = pi X_raw / (2L)).  Sec. 2.3 observes that
 * n^-1 Phi^* Phi is the multilevel Toeplitz matrix Sigma[k, l] = M[l - k] with
 * generator M[q] = n^-1 sum_j exp(+i q.X_j), ||q||_inf <= 2m, and that
 * n^-1 Phi^* Y = (n^-1 sum_j Y_j exp(-i k.X_j))_k; both are type-1 NUFFTs.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Points X are structure-of-arrays [d][n] (row a holds coordinate a of all
 *   points), in radians; each coordinate must lie in [-2 pi, 2 pi) and is
 *   folded onto the torus [-pi, pi).  Targets Y are [ntgt][n].  X and Y have
 *   the same dtype (FK_F32 or FK_F64).
 * - Mode arrays are complex128, interleaved (re, im), row-major over the
 *   multi-index (k_1, ..., k_d), each coordinate running -m..m (k_d fastest).
 *   N = (2m+1)^d.  The generator M runs over -2m..2m: (4m+1)^d entries.
 * - All array pointers are DEVICE pointers owned by the caller (unless a
 *   parameter says "host").  The library never frees them and keeps no
 *   reference to them after the call returns.
 * - Scratch memory is caller-provided: query its size with the matching
 *   *_workspace_size function and pass a device buffer of at least that many
 *   bytes (256-byte aligned).  The library allocates no device memory inside
 *   compute calls except its small per-context plan tables (created on first
 *   use of a shape and freed by fk_destroy).
 * - Work is enqueued on the context's HIP stream (the additive model's
 *   transforms also on a second stream of the context, created at first use
 *   with the default priority and joined back before the call returns).
 *   Every compute entry point returns after synchronising that stream, and
 *   device-detected conditions (NaN input, out-of-range input, non-positive
 *   pivot, no convergence) become the returned status there.  The fits
 *   synchronise once per refinement step (its residual norms, which come back
 *   with the error flags of every stage before it, decide whether another step
 *   runs; with refine_tol below 1e-8 the first solve's check is skipped, since
 *   an FP32-class solve does not reach such a tolerance without refinement) and
 *   once at the end; a first use of an untuned large shape also
 *   synchronises around its timed trials.  Host-side argument checks return
 *   FK_EINVAL before anything is enqueued.
 * - A context must not be used by two threads at once; distinct contexts are
 *   independent.  No exception crosses this ABI.
 * - Repeatability: the dense stage (fk_solve, the solve of fk_fit, the
 *   gradients) gives the same bits for the same inputs and launch shapes; the
 *   type-1 sums (fk_gram) accumulate with FP64 atomics and agree between runs
 *   to FP64 rounding.
 */
#ifndef FASTKERNEL_FK_H
#define FASTKERNEL_FK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FK_OK = 0,
  FK_EINVAL = 1,   /* invalid argument (checked on the host, nothing enqueued) */
  FK_ERANGE = 2,   /* a coordinate outside [-2 pi, 2 pi) */
  FK_ENAN = 3,     /* a NaN or Inf among X or Y */
  FK_ENOTPD = 4,   /* the system matrix lost positive definiteness in FP32 */
  FK_ENOCONV = 5,  /* FP64 iterative refinement did not reach its tolerance */
  FK_ENOMEM = 6,   /* workspace smaller than the queried size */
  FK_EHIP = 7      /* a HIP runtime call failed */
} fk_status;

typedef enum { FK_F32 = 0, FK_F64 = 1 } fk_dtype;

typedef struct fk_ctx fk_ctx;

/* Penalty lambda M^* M of eq. (kenrel_reg). */
typedef enum {
  FK_PEN_SOBOLEV = 0,         /* diag 1 + ||k||_2^(2s)            (Sec. 3.1, matrix S) */
  FK_PEN_SOBOLEV_BESSEL = 1,  /* diag (1 + ||k||_2^2)^s           (an equivalent Sobolev norm, Sec. 3.1) */
  FK_PEN_IDENTITY = 2,        /* diag 1, the low-bias estimator     (Sec. 3.2, Prop. low-bias) */
  FK_PEN_DIAG = 3,            /* diag p, p given by the caller (host array of N doubles, p_k > 0,
                                 p_{-k} = p_k) */
  FK_PEN_HEAT_BOX = 4,        /* d = 2, modes (k_t, k_x): FK_PEN_PDE_BOX for the heat operator d_t - d_xx
                                 (D_k = i k_t + k_x^2) with s = 1 (alpha, coef unused) */
  FK_PEN_PDE_BOX = 5          /* d = 1 or 2, the physics-informed penalty of Sec. 4 (tractable domains):
                                   lambda diag(1 + ||k||^(2s)) + mu D^* C D
                                 for the linear constant-coefficient operator sum_t coef[t] d^alpha[t]:
                                   D_k = sum_t coef[t] prod_a (i k_a)^alpha[t][a]  (its action on exp(i k.x)),
                                   C[k, l] = (2 pi)^-d prod_a int_{lo_a}^{hi_a} exp(i (l_a - k_a) u) du,
                                 the Fourier matrix of the box [lo, hi] (radians), so that theta^* C theta =
                                 (2 pi)^-d int_box |f_theta|^2 and theta^* D^* C D theta =
                                 (2 pi)^-d int_box |sum_t coef[t] d^alpha[t] f_theta|^2 */
} fk_pen_kind;

typedef struct {
  int kind;            /* fk_pen_kind */
  double s;            /* Sobolev order for FK_PEN_SOBOLEV / _BESSEL / _PDE_BOX (s >= 0) */
  const double* p;     /* host, N weights for FK_PEN_DIAG, else NULL */
  double mu;           /* FK_PEN_HEAT_BOX / _PDE_BOX: weight of the PDE term (>= 0) */
  double box_lo[2];    /* FK_PEN_HEAT_BOX / _PDE_BOX: box corners in radians (entries 0..d-1 used, */
  double box_hi[2];    /*   box_lo[a] < box_hi[a]) */
  int nterms;          /* FK_PEN_PDE_BOX: number of operator terms, 1..16 */
  const int* alpha;    /* FK_PEN_PDE_BOX: host, nterms x d derivative orders, each 0..8 */
  const double* coef;  /* FK_PEN_PDE_BOX: host, nterms finite real coefficients */
} fk_penalty;

/* Options; zero-initialised means defaults. */
typedef struct {
  double eps;          /* spreading accuracy target per dimension (default 2e-7) */
  int max_refine;      /* FP64 refinement iterations cap (default 8; 0 = none) */
  double refine_tol;   /* relative FP64 residual target (default 1e-10) */
  int keep_factors;    /* 1: keep Cholesky factors in the workspace for fk_heldout_mse /
                          fk_fit_backward (always on; field reserved) */
  int autotune;        /* launch-shape autotuning (see "Autotuning" below): 0 = as the FK_AUTOTUNE
                          environment variable says (default: tune), 1 = built-in shapes only,
                          2 = re-measure even when the table has an entry, 3 = tune at first use */
} fk_options;

/* Per-call report, filled by fk_fit / fk_gram when non-NULL. */
typedef struct {
  int status;          /* same as the return value */
  int bad_index;       /* failing lambda index for FK_ENOTPD / FK_ENOCONV, else -1 */
  int refine_iters;    /* FP64 refinement iterations performed */
  int w;               /* spreading kernel width (grid points per dimension) */
  int nf;              /* fine-grid size per dimension */
  int bin;             /* bin edge (grid points) of the binned spread: > 0 FP64-atomic spread,
                          < 0 matrix-core spread over |bin| x |bin| cells, 0 = unbinned (1-D) */
  double beta;         /* exponential-of-semicircle shape parameter */
  double resid_rel;    /* max over (lambda, target) of ||b - A theta|| / ||b|| in FP64 */
  float t_sort_ms, t_spread_ms, t_fft_ms, t_assemble_ms, t_factor_ms, t_solve_ms, t_total_ms;
                       /* stage times (HIP events).  On the call that tunes a dense shape (see
                          "Autotuning") the trials run inside the assembly interval, whose last
                          factorization is kept, so t_factor_ms is then about 0 */
  double spread_kernel_ms;   /* device time of the spreading kernel alone */
} fk_fit_info;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t; NULL = the default stream). */
fk_status fk_create(fk_ctx** ctx, int device, void* hip_stream);
fk_status fk_destroy(fk_ctx* ctx);
fk_status fk_set_stream(fk_ctx* ctx, void* hip_stream);
fk_status fk_set_options(fk_ctx* ctx, const fk_options* opt);
const char* fk_status_string(fk_status s);

/* ---------------------------------------------------------------- type-1 stage
 * fk_gram: the Gram generator and the right-hand sides (Sec. 2.3):
 *   M_out[q] = n^-1 sum_j exp(+i q.X_j),          q in {-2m..2m}^d,  complex128 (4m+1)^d
 *   b_out[t][k] = n^-1 sum_j Y[t][j] exp(-i k.X_j),   k in {-m..m}^d,  complex128 ntgt x N
 * computed by exponential-of-semicircle spreading onto an oversampled grid, an
 * FFT and deconvolution.  d in {1, 2, 3}; 1 <= m <= 64 (m <= 31 and ntgt <= 8 for d = 3, whose
 * spread adds into an FP64 grid of up to 256^3 per channel by FP64 atomics); 0 <= ntgt <= 32 (Y may be NULL
 * when ntgt = 0); n >= 1, and n <= 2^32 - 1 for d = 2 with ntgt <= 16 (point positions
 * are 32-bit in the bin sort; larger n returns FK_EINVAL). */
fk_status fk_gram_workspace_size(fk_ctx* ctx, int d, int64_t n, int ntgt, int m, size_t* bytes);
fk_status fk_gram(fk_ctx* ctx, int d, int64_t n, fk_dtype dtype, const void* X, int ntgt,
                  const void* Y, int m, double* M_out, double* b_out,
                  void* ws, size_t ws_bytes, fk_fit_info* info);

/* ---------------------------------------------------------------- solve
 * fk_solve: theta[l][t] = (Sigma + lambda_l M^*M)^-1 b[t] for every lambda in `lambdas`
 * (host array, nlam >= 1, each > 0) and every right-hand side t (eq. kenrel_reg), from
 * the generator M (device, complex128 (4m+1)^d) and b (device, complex128 ntgt x N).
 * The Hermitian system is solved in its equivalent real cosine/sine form by a blocked
 * Cholesky of its diagonally equilibrated FP32 matrix per lambda, batched over lambda
 * (finished panels kept as pairs of FP16 halves, about 22 significant bits, their
 * products accumulated in FP32 on the matrix cores), with FP64 iterative refinement.
 * theta_out: device complex128 [nlam][ntgt][N].
 * The workspace also keeps the factors, the FP64 real-form Gram and the real-form
 * solutions for fk_heldout_mse / fk_fit_backward on the same workspace. */
fk_status fk_solve_workspace_size(fk_ctx* ctx, int d, int m, int ntgt, int nlam, size_t* bytes);
fk_status fk_solve(fk_ctx* ctx, int d, int m, const double* M, int ntgt, const double* b,
                   const double* lambdas, int nlam, const fk_penalty* pen,
                   double* theta_out, void* ws, size_t ws_bytes, fk_fit_info* info);

/* ---------------------------------------------------------------- restriction to a smaller m
 * fk_restrict: the generator and right-hand sides for m_to <= m_from from those for m_from.
 * M[q] and b_k (Sec. 2.3) do not depend on m: a smaller basis keeps the frequencies
 * ||q||_inf <= 2 m_to and ||k||_inf <= m_to, the centred sub-blocks.  So one type-1 stage at the
 * largest m of a sweep (over m, or over s with m tied to s) serves every smaller m.
 * d = 1, 2 or 3; 1 <= m_to <= m_from <= 255; 0 <= ntgt.  Device complex128: M_in (4m_from+1)^d,
 * b_in ntgt x (2m_from+1)^d, M_out (4m_to+1)^d, b_out ntgt x (2m_to+1)^d (b may be NULL when
 * ntgt = 0); outputs must not overlap inputs.  Synchronises the context's stream. */
fk_status fk_restrict(fk_ctx* ctx, int d, int m_from, int m_to, int ntgt, const double* M_in,
                      const double* b_in, double* M_out, double* b_out);

/* ---------------------------------------------------------------- iterative solve
 * The paper's own route to theta (Sec. 2.3, "Matrix inversion"): conjugate gradients on
 * (Sigma + lambda P) theta = b, where each product with Sigma[k, l] = M[l - k] (Sec. 2.3,
 * "Covariance matrix") costs O(m^d log m) through an FFT of its circulant embedding
 * (length Lf = the next power of two >= 4m + 1 per dimension).
 *
 * fk_toeplitz_apply: y[v] = Sigma x[v] for nvec vectors.  d = 1, 2 or 3; 1 <= m <= 255
 * (m <= 63 for d = 3).  M: device complex128, (4m+1)^d entries, as fk_gram writes it;
 * x, y: device complex128 [nvec][N], N = (2m+1)^d, not overlapping.
 * Workspace: fk_toeplitz_apply_workspace_size bytes of device memory, owned by the caller.
 *
 * fk_solve_cg: all nlam x ntgt systems, lambda_l > 0, iterate together from theta = 0 with
 * the Jacobi preconditioner M[0] + lambda_l p_k; system (l, t) stops at the first
 * iteration where the recursively updated residual has ||r|| <= tol ||b_t||
 * (0 < tol < 1), or after maxit iterations.  A zero right-hand side gives theta = 0 in 0
 * iterations.  P must be diagonal: FK_PEN_SOBOLEV, _SOBOLEV_BESSEL, _IDENTITY or _DIAG (NULL
 * = FK_PEN_SOBOLEV with s = 1); FK_PEN_HEAT_BOX returns FK_EINVAL (use fk_solve).
 * M, b, theta_out: device, layouts as in fk_solve (theta_out [nlam][ntgt][N]).
 * iters (host, may be NULL): iterations of the slowest system.  relres (host, nlam x ntgt
 * doubles, may be NULL): final ||b - A theta|| / ||b|| recomputed with one more product.
 * ntgt * nlam <= 65536.  The call synchronises the context's stream every 4 iterations.
 * Returns FK_ENOCONV when some system has not met tol after maxit iterations (theta_out then
 * holds the last iterates), FK_ENOTPD when <p, A p> <= 0 for some system (A not positive
 * definite in FP64), FK_ENAN when b holds a NaN or Inf or a NaN reaches <p, A p>, FK_EINVAL
 * when the centre M[0] is not positive. */
fk_status fk_toeplitz_apply_workspace_size(fk_ctx* ctx, int d, int m, int nvec, size_t* bytes);
fk_status fk_toeplitz_apply(fk_ctx* ctx, int d, int m, const double* M, int nvec, const double* x,
                            double* y, void* ws, size_t ws_bytes);
fk_status fk_solve_cg_workspace_size(fk_ctx* ctx, int d, int m, int ntgt, int nlam, size_t* bytes);
fk_status fk_solve_cg(fk_ctx* ctx, int d, int m, const double* M, int ntgt, const double* b,
                      const double* lambdas, int nlam, const fk_penalty* pen, double tol, int maxit,
                      double* theta_out, int* iters, double* relres, void* ws, size_t ws_bytes);

/* fk_solve_cg_collocation: the physics-informed estimator on a domain without a closed-form
 * Fourier matrix (Sec. 4, intractable domains): the same iteration on
 *   (Sigma + lambda P + mu D^* Sigma_r D) theta = b,
 * where Sigma_r[k, l] = Mr[l - k] is the Gram of n_r collocation points sampled over the domain
 * (Mr: device complex128, (4m+1)^d entries, the generator fk_gram returns for those points with
 * no targets) and D = diag(Dsym) is the operator's symbol on exp(i k.x) (Dsym: device complex128
 * [N]; for sum_alpha a_alpha d^alpha it is sum_alpha a_alpha prod_l (i k_l)^alpha_l).  mu >= 0.
 * Each iteration takes two FFT products; the preconditioner is
 * M[0] + lambda p_k + mu |D_k|^2 Mr[0].  Other arguments, results and errors as fk_solve_cg; the
 * workspace is fk_solve_cg_collocation_workspace_size bytes. */
fk_status fk_solve_cg_collocation_workspace_size(fk_ctx* ctx, int d, int m, int ntgt, int nlam,
                                                 size_t* bytes);
fk_status fk_solve_cg_collocation(fk_ctx* ctx, int d, int m, const double* M, int ntgt, const double* b,
                                  const double* lambdas, int nlam, const fk_penalty* pen, double mu,
                                  const double* Mr, const double* Dsym, double tol, int maxit,
                                  double* theta_out, int* iters, double* relres, void* ws, size_t ws_bytes);

/* fk_fit = fk_gram followed by fk_solve (one workspace holding both). */
fk_status fk_fit_workspace_size(fk_ctx* ctx, int d, int64_t n, int ntgt, int m, int nlam,
                                size_t* bytes);
fk_status fk_fit(fk_ctx* ctx, int d, int64_t n, fk_dtype dtype, const void* X, int ntgt,
                 const void* Y, int m, const double* lambdas, int nlam, const fk_penalty* pen,
                 double* theta_out, void* ws, size_t ws_bytes, fk_fit_info* info);

/* fk_fit_kept: fk_fit with its two parts in two workspaces: ws_solve (solve_bytes of
 * fk_fit_kept_workspace_size, the same layout as fk_solve's workspace) keeps the factors, the FP64
 * real-form Gram and the solutions for fk_heldout_mse / fk_fit_backward (see "Kept factors"), and
 * ws_scratch (scratch_bytes) holds M, b and the type-1 stage's buffers, free again when the call
 * returns.  So a caller keeping the factors of several fits keeps only their ws_solve buffers, and
 * shares one scratch buffer.  The two buffers must not overlap (FK_EINVAL).  Results and errors as
 * fk_fit; the stage and the solve run without a synchronisation between them. */
fk_status fk_fit_kept_workspace_size(fk_ctx* ctx, int d, int64_t n, int ntgt, int m, int nlam,
                                     size_t* solve_bytes, size_t* scratch_bytes);
fk_status fk_fit_kept(fk_ctx* ctx, int d, int64_t n, fk_dtype dtype, const void* X, int ntgt,
                      const void* Y, int m, const double* lambdas, int nlam, const fk_penalty* pen,
                      double* theta_out, void* ws_solve, size_t ws_solve_bytes, void* ws_scratch,
                      size_t ws_scratch_bytes, fk_fit_info* info);

/* ---------------------------------------------------------------- type-2 stage
 * fk_predict: out[t][j] = Re sum_k theta[t][k] exp(+i k.Xq_j) (the estimator of
 * Sec. 2.1 evaluated at new points), by deconvolution, an inverse FFT onto an
 * oversampled grid and exponential-of-semicircle interpolation.  theta is device
 * complex128 [ntheta][N] (Hermitian-symmetric for a real f; the imaginary part of
 * the sum is dropped); out is device float32 [ntheta][nq].  d in {1, 2, 3} (d = 3: m <= 31,
 * ntheta <= 64, oversampled grid up to 128^3 per coefficient set). */
fk_status fk_predict_workspace_size(fk_ctx* ctx, int d, int m, int ntheta, size_t* bytes);
fk_status fk_predict(fk_ctx* ctx, int d, int m, int ntheta, const double* theta, int64_t nq,
                     fk_dtype dtype, const void* Xq, float* out, void* ws, size_t ws_bytes);

/* fk_predict_noalloc: fk_predict without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as fk_predict, computed by the same kernels.  It
 * calls no hipMalloc / hipFree: its intermediates (the deconvolution table and the oversampled
 * grids) live in one library-owned device array of 64 MiB per device, resolved by fk_create and held
 * until the process ends.  Shapes whose fk_predict_workspace_size exceeds
 * fk_predict_noalloc_max_bytes() return FK_ENOMEM (nothing enqueued); d = 2 with m = 32 fits up to
 * 266 coefficient sets.  Every call on a device shares that array and leaves its contents there:
 * calls that overlap in time on one device (several streams, threads or contexts) race and must be
 * serialised by the caller. */
fk_status fk_predict_noalloc(fk_ctx* ctx, int d, int m, int ntheta, const double* theta, int64_t nq,
                             fk_dtype dtype, const void* Xq, float* out);
size_t fk_predict_noalloc_max_bytes(void);

/* ---------------------------------------------------------------- held-out loss and gradients
 * Kept factors.  fk_solve and fk_fit leave, at the start of their workspace, the factors of
 * every lambda (in the format above), the FP64 real-form Gram and the solutions; a successful call (FK_OK or
 * FK_ENOCONV) registers that workspace (its address and the shape d, m, nlam, ntgt).  Any later
 * library call that writes a workspace overlapping it (fk_gram, fk_solve, fk_fit, fk_predict,
 * the additive and iterative entry points, from any context) removes the registration, and
 * fk_heldout_mse / fk_fit_backward then return FK_EINVAL instead of reading overwritten factors.
 * Writes into the buffer from outside the library are not seen: the caller must not reuse the
 * workspace memory while it wants the gradients.
 *
 * After fk_solve (or fk_fit) on workspace `ws`, with the held-out Gram generator Mv
 * (device complex128 (4m+1)^d), right-hand sides bv (device complex128 ntgt x N) and
 * yv2[t] = n_v^-1 sum_j Yv[t][j]^2 (device, ntgt doubles):
 *   mse[l][t] = theta^* Sigma_v theta - 2 Re(bv^* theta) + yv2[t]
 *             = n_v^-1 sum_j |f_theta(Xv_j) - Yv[t][j]|^2          (device, nlam x ntgt doubles)
 * This is not in the paper; it makes the lambda grid search of Sec. 5 differentiable. */
fk_status fk_heldout_mse(fk_ctx* ctx, int d, int m, int ntgt, int nlam, const double* Mv,
                         const double* bv, const double* yv2, double* mse_out,
                         void* ws, size_t ws_bytes);

/* fk_mean_square: out[t] = n^-1 sum_j Y[t][j]^2 in FP64 (device, ntgt doubles), the constant
 * term of the held-out loss above.  Y is device [ntgt][n] (fp32 or fp64); n >= 1. */
fk_status fk_mean_square(fk_ctx* ctx, int ntgt, int64_t n, fk_dtype dtype, const void* Y, double* out);

/* fk_fit_backward: the gradients of a real loss Loss(mse, theta) through theta = A_l^-1 b_t, where
 * mse is the held-out loss above.  Complex gradients follow the Wirtinger convention:
 * dLoss/dconj(theta), the vector G with dLoss = 2 Re(G^* dtheta) (PyTorch's .grad of a complex
 * tensor is 2 G).  Inputs:
 *   grad_mse[l][t] = dLoss/dmse[l][t]                        (device, nlam x ntgt doubles)
 *   grad_theta_in[l][t][k] = dLoss/dconj(theta) from every other use of theta (device complex128
 *                    nlam x ntgt x N, or NULL for none); only its Hermitian-symmetric part acts, as
 *                    theta stays Hermitian-symmetric (real data) for every lambda and p.
 * With g = Sigma_v theta - bv (= d mse / d conj(theta)), G = grad_mse * g + grad_theta_in and the
 * adjoint u = A_l^-1 G (solved with the kept factors and FP64 refinement):
 *   grad_loglam[l] = sum_t -2 lambda_l Re(u^* P theta)                  (device, nlam)
 *   grad_p[k]      = sum_{l,t} -lambda_l Re(conj(u_k) theta_k + conj(u_-k) theta_-k)
 *                    (device, N; only for diagonal penalties, else left untouched; may be NULL).
 *                    The weights are tied (p_{-k} = p_k is required), so this is the gradient
 *                    projected onto symmetric weights: grad_p[k] = grad_p[-k] = half of dLoss/dq for
 *                    the common value q = p_k = p_{-k}.  For a Hermitian-symmetric G it equals
 *                    -2 lambda_l Re(conj(u_k) theta_k) summed over (l, t).
 *   grad_theta[l][t] = grad_mse[l][t] * g   (device complex128, may be NULL: the Wirtinger gradient
 *                    of the mse term with respect to conj(theta), theta held fixed)
 * Requires the fk_heldout_mse call on the same workspace after its fk_solve / fk_fit (FK_EINVAL
 * otherwise, see "Kept factors").  Returns FK_ENAN if the adjoint right-hand sides are not finite. */
fk_status fk_fit_backward(fk_ctx* ctx, int d, int m, int ntgt, int nlam, const double* grad_mse,
                          const double* grad_theta_in, double* grad_loglam, double* grad_p,
                          double* grad_theta, void* ws, size_t ws_bytes);

/* ---------------------------------------------------------------- additive model (Sec. 5)
 * fk_additive_gram: block Gram B (device complex128, [d(2m+1)]^2 row-major) with blocks
 *   B[a,b][k,l] = n^-1 sum_j exp(-i k X_ja + i l X_jb)
 * (diagonal blocks from 1-D type-1 transforms, off-diagonal blocks from 2-D type-1
 * transforms at the points (X_a, X_b)) and the stacked right-hand side
 * b_out[t][a(2m+1) + k] = n^-1 sum_j Y[t][j] exp(-i k X_ja).  2 <= d <= 16, m <= 64. */
fk_status fk_additive_gram_workspace_size(fk_ctx* ctx, int d, int64_t n, int ntgt, int m,
                                          size_t* bytes);
fk_status fk_additive_gram(fk_ctx* ctx, int d, int64_t n, fk_dtype dtype, const void* X, int ntgt,
                           const void* Y, int m, double* B_out, double* b_out,
                           void* ws, size_t ws_bytes, fk_fit_info* info);

/* fk_additive_fit: theta = (B + lambda blockdiag(p))^-1 b, p_k = 1 + |k|^(2s) per
 * component (s = 0 gives the low-bias identity of Prop. low-bias additive), theta_out
 * device complex128 [nlam][ntgt][d(2m+1)]. */
fk_status fk_additive_fit_workspace_size(fk_ctx* ctx, int d, int64_t n, int ntgt, int m, int nlam,
                                         size_t* bytes);
fk_status fk_additive_fit(fk_ctx* ctx, int d, int64_t n, fk_dtype dtype, const void* X, int ntgt,
                          const void* Y, int m, const double* lambdas, int nlam, double s,
                          double* theta_out, void* ws, size_t ws_bytes, fk_fit_info* info);

/* ---------------------------------------------------------------- autotuning
 * Launch shapes of the large stages are chosen by measurement (not in the paper: its grid search,
 * Sec. 5, repeats one type-1 stage and many solves, so their speed is what the search costs):
 *   - the 2-D type-1 stage with 0..16 targets and n >= 2^22 points: the bin edge of the channel-row
 *     spread (2 or 4 cells), points per spreading workgroup, workgroups of the first sort pass and
 *     points per slice of the second;
 *   - the dense solve with Np^2 nlam >= 2^28 (Np = N rounded up to 64): workgroups per
 *     triangular-solve launch and whether block columns are factored in pairs.
 * A table entry of a dense shape may also hold diag64=1 (never chosen by the tuner): the 64 x 64
 * diagonal blocks of the factorization are then factored in FP64 instead of FP32 (slower; the
 * FP32 default matches an FP32 LAPACK factorization's accuracy).
 * At the first call of a shape without a table entry the library times each candidate (coordinate
 * descent, one knob at a time, on the call's own data, a type-1 candidate as the better of two runs;
 * the call then runs with the fastest) and
 * records "<arch> <stage> <shape> = <knob>=<value> ... ms=<time>" in a process-wide table; every
 * candidate is a correct configuration, so results differ only by rounding.  Environment:
 * FK_AUTOTUNE_CACHE = path of a text file read at the first lookup and appended with each new
 * entry; FK_AUTOTUNE = off | force (or fk_options.autotune).  Entries may be written by hand to pin
 * a configuration.
 *
 * fk_autotune_load: merge the entries of a table file (lines "<key> = <knob>=<int> ...", '#'
 *   comments; malformed lines are skipped).  Host only; FK_EINVAL if the file cannot be read.
 * fk_autotune_table: the table as text (one entry per line, sorted by key) into buf (host, cap
 *   bytes, NUL-terminated); *len = its length without the NUL.  buf = NULL only queries len;
 *   FK_EINVAL if cap is too small.
 * fk_autotune_clear: empty the table (the cache file is not read again in this process). */
fk_status fk_autotune_load(const char* path);
fk_status fk_autotune_table(char* buf, size_t cap, size_t* len);
fk_status fk_autotune_clear(void);

/* ---------------------------------------------------------------- synthetic inputs
 * fk_generate_uniform: X[a][j] = (float)(lo_a + (hi_a - lo_a) * u), u = (w >> 8) 2^-24
 * with w the Philox4x32-10 word a (a < 4) of counter (j + start, 0, 0, 0) >> ..., key = seed
 * (the counter layout of the test-suite generator); and
 * fk_generate_targets: Y[t][j] = (float)(sin((t+1) x1) cos(x2) + sigma * z_t(j)) with
 * z_t Box-Muller on words 0, 1 of stream t + 1.  Device float32 outputs.  Used to
 * materialise large inputs in device memory before a timed fit. */
fk_status fk_generate_uniform(fk_ctx* ctx, uint64_t seed, int d, int64_t n, int64_t start,
                              const double* lo, const double* hi, float* X);
fk_status fk_generate_targets(fk_ctx* ctx, uint64_t seed, int ntgt, int64_t n, int64_t start,
                              const float* X, double sigma, float* Y);

#ifdef __cplusplus
}
#endif
#endif /* FASTKERNEL_FK_H */
