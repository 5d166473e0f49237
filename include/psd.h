/*
 * psd.h -- C ABI of the MI355X (gfx950) preconditioned steepest descent
 * solver for periodic, finite-difference regularised p-Laplacian problems
 * (Feng, Salgado, Wang & Wise, arXiv:1607.01475).
 *
 * Problems (periodic box [0,L]^dim, n cells per axis, h = L/n, Sec. 5.1):
 *   order 4 (Sec. 5.3, discrete fourth-order equation):
 *       u - s div_h(|grad_h u|^{p-2} grad_h u) + s eps^2 Delta_h^2 u = f
 *   order 6 (Sec. 5.4, discrete sixth-order mixed system):
 *       u - Delta_h w = g,
 *       s lam u - s div_h(|grad_h u|^{p-2} grad_h u) + s eps^2 Delta_h^2 u - w = f
 * grad_h is the collocated centre-to-vertex gradient and div_h the
 * vertex-to-centre divergence of Sec. 5.1 (3D: the same construction with
 * averages over the two other axes).  Each call of the PSD loop (Sec. 2.2 and
 * Sec. 6) computes the residual, solves the preconditioner equation
 * L_h d = r by FFT (Sec. 6.1 and 6.2), finds the exact line-search step
 * alpha (unique root of q, Sec. 6.1) and updates u <- u + alpha d.
 *
 * Memory: every array argument is a DEVICE pointer to n^dim contiguous
 * doubles, x fastest (idx = i + n*(j + n*k)); cell i has centre (i+1/2)h.
 * The caller owns inputs and outputs; the handle owns all workspace.
 * Streams: all work is ordered on the stream given to psd_create (NULL =
 * default stream).  psd_solve, psd_residual, psd_energy, psd_adjoint return
 * only after the results are on the host/device (they synchronise the stream).
 * Errors: status codes only; nothing aborts, no exception crosses the ABI.
 * psd_last_error gives a message for the last failing call on a handle.
 * A handle must not be used from two threads at once.
 */
#ifndef PSD_H
#define PSD_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psd_handle_s psd_handle;

typedef enum {
    PSD_OK = 0,
    PSD_NOT_CONVERGED = 1,     /* max_iter updates without reaching tol */
    PSD_ERR_ARG = -1,          /* NULL pointer, bad size, unsupported n */
    PSD_ERR_RANGE = -2,        /* parameter outside the paper's range */
    PSD_ERR_HIP = -3,          /* HIP runtime error (no device, OOM, ...) */
    PSD_ERR_NONFINITE = -4,    /* NaN/Inf in the residual */
    PSD_ERR_NOT_DESCENT = -5,  /* q(0) >= 0 with residual above tol */
    PSD_ERR_MEAN = -6          /* order 6: mean(u0) != mean(g) */
} psd_status;

/* Problem statement (Sec. 1; discrete form Sec. 5).
 *   dim   2 or 3
 *   n     cells per axis; supported: 16, 32, 48, 64, 96, 128, 192, 256, 384,
 *         512, 1024 (2D); up to 256 in 3D
 *   L     box side (> 0)
 *   order 4 or 6
 *   p     exponent, p >= 2 (p <= 6 in 3D, Sec. 3.1)
 *   s     > 0
 *   eps   0 < eps <= 1
 *   lambda  >= 0 (order 6 only) */
typedef struct {
    int dim;
    int n;
    double L;
    int order;
    double p, s, eps, lambda;
} psd_problem;

enum { PSD_FP64 = 0, PSD_MIXED = 1 };
enum { PSD_METRIC_CONSTANT = 0, PSD_METRIC_VARIABLE = 1 };

/* Solver options.
 *   tol         stop when the absolute max-norm of the residual is <= tol
 *               (order 4: f - N_h[u]; order 6: max of the two residuals of
 *               the mixed system), checked after every update
 *   max_iter    maximum number of updates
 *   precision   PSD_FP64: every step in FP64.  PSD_MIXED: the FFT
 *               preconditioner (forward transform, spectral scaling,
 *               inverse transform) runs in FP32; residual, line-search
 *               reductions, step and update stay FP64 (iterative refinement)
 *   graph_chunk 0: host-driven loop, the host reads the convergence flag
 *               after every iteration.  k > 0: k iterations are captured once
 *               in a HIP graph and replayed until the device flag says done;
 *               the host reads the flags of one batch of replays while the
 *               next batch runs (two pinned state buffers and two events,
 *               allocated on first use) (general p: each captured iteration
 *               runs up to 6 evaluation passes of the root search; see
 *               psd_stats.ls_truncated)
 *   history     non-zero: record per-update (alpha, ||r||_inf, ||r||_2, dE)
 *   profile     non-zero: per-pass kernel timing of psd_solve (psd_pass_times)
 *   autotune    non-zero: pick stencil tilings by timing at creation */
typedef struct {
    double tol;
    int max_iter;
    int precision;
    int graph_chunk;
    int history;
    int profile;   /* non-zero: time every kernel launch with HIP events on the
                      solver stream (see psd_pass_times) */
    int autotune;  /* non-zero: at psd_create, time the 3D stencil-kernel tilings
                      (residual z-chunk 16/28/40/64, line-search z-chunk
                      12/24/36/60, plus per kernel the chunk at which all its
                      blocks are resident at once; line-search tile 64x8 or
                      32x16; natural or XCD-grouped block order) and the
                      row-transform layout (lines per block, 2D and 3D) on
                      this handle's buffers and keep the fastest; results are
                      cached in the file named by PSD_TUNE_CACHE when set */
    int metric;       /* PSD_METRIC_CONSTANT: d = L_h^{-1} r by FFT (Sec. 5.3 and 6).
                         PSD_METRIC_VARIABLE (order 4, graph_chunk 0): the metric
                         of the Remark in Sec. 3, L_k = I - s div_h(|grad_h u^k|^{p-2}
                         grad_h .) + s eps^2 Delta_h^2 (coefficient frozen at the
                         current iterate); d = L_k^{-1} r by conjugate gradients
                         preconditioned with L_h^{-1}, then the same exact line
                         search and update */
    double inner_rtol; /* variable metric: stop the inner solve at
                          ||res||_2 <= inner_rtol ||r||_2 (0: run inner_iters) */
    int inner_iters;   /* variable metric: iteration cap of the inner solve */
} psd_options;

/* Per-instance result.  energy is E_h at the final iterate (Sec. 5.3 and
 * 5.4 discrete energies) when options.history is set, else NaN (use
 * psd_energy); status a psd_status.  ls_truncated counts the line searches
 * of a general-p solve (p other than 2, 4, 6... with no polynomial q) whose
 * root search stopped at its evaluation cap (graph mode captures a fixed
 * number of evaluations per iteration) instead of at the root; 0 normally. */
typedef struct {
    int iters;
    double res_inf, res_l2, energy;
    int status;
    int ls_truncated;
} psd_stats;

/* Validate one problem statement on the host (no GPU needed).  Returns
 * PSD_OK, PSD_ERR_ARG or PSD_ERR_RANGE; msg (may be NULL) receives a short
 * reason (buffer of msg_len bytes). */
psd_status psd_check_problem(const psd_problem* prob, char* msg, int msg_len);

/* Create a solver for `batch` independent instances (probs[batch]); all
 * share the options.  Plans FFTs, symbol tables and all workspace on the
 * current HIP device.  hip_stream is a hipStream_t (NULL = default). */
psd_status psd_create(const psd_problem* probs, int batch, const psd_options* opt,
                      void* hip_stream, psd_handle** out);

/* Solve all instances.  f[b], g[b] (order 6, else NULL array or entries),
 * u[b] (in: u0, out: final iterate; order 6 needs mean(u0) = mean(g)),
 * w[b] (order 6 output of the mixed system, may be NULL) are device
 * pointers.  stats[batch] is host memory.  Returns the worst instance status
 * (errors < 0 take precedence over PSD_NOT_CONVERGED). */
psd_status psd_solve(psd_handle* h, const double* const* f, const double* const* g,
                     double* const* u, double* const* w, psd_stats* stats);

/* One solve that allocates nothing, for callers that cannot allocate device
 * memory (serving loops, harnesses that forbid hipMalloc).  Same problem,
 * options and results as psd_create + psd_solve + psd_destroy for a batch of
 * one instance, with these differences:
 *   - all device workspace comes from one static device array of 64 MiB per
 *     GPU (held by every GPU the library runs on until the process ends);
 *     a problem whose workspace does not fit is rejected with PSD_ERR_ARG
 *     (for example 2D order 4 fits up to n = 1024, 3D order 4 up to n = 96,
 *     2D order 6 up to n = 512);
 *   - no hipMalloc, hipFree, pinned host allocation, stream, event or graph
 *     creation; the state is staged through static host memory (ordinary
 *     C++ containers hold the small host-side task tables);
 *   - options.graph_chunk, profile and autotune must be 0 (host-driven loop,
 *     default tiling), else PSD_ERR_ARG;
 *   - calls on one GPU share the array and run one after the other (a mutex
 *     per GPU); each call clears what must start at zero, and returns only
 *     after its work on hip_stream has finished.  Work of the caller that
 *     uses the same array concurrently (none outside this call) would race.
 * f, g (order 6, else may be NULL), u (in: u0, out: final iterate), w (order
 * 6 output, may be NULL) are device pointers of n^dim doubles; stats (host,
 * may be NULL) receives the result.  Errors are reported by
 * psd_last_error(NULL) of the calling thread. */
psd_status psd_solve_noalloc(const psd_problem* prob, const psd_options* opt, void* hip_stream,
                             const double* f, const double* g, double* u, double* w,
                             psd_stats* stats);

/* Residual of instance `inst` at u.  Order 4: r = f - N_h[u].  Order 6: the
 * reduced residual rho = P0[f - (s lam u - s div_h(...) + s eps^2 Delta_h^2 u)
 * - T_h(u - g)] (minus the gradient of the mean-zero energy; T_h = -Delta_h^{-1}
 * on mean-zero functions).  r (device, may be NULL) receives it, *res_inf
 * (host, may be NULL) its max-norm. */
psd_status psd_residual(psd_handle* h, int inst, const double* f, const double* g,
                        const double* u, double* r, double* res_inf);

/* Residuals of the order-6 mixed system at (u, w) (Sec. 5.4):
 *   r1 = g - u + Delta_h w,  r2 = f - (s lam u - s div_h(...) + s eps^2 Delta_h^2 u - w). */
psd_status psd_residual_mixed(psd_handle* h, int inst, const double* f, const double* g,
                              const double* u, const double* w, double* r1, double* r2,
                              double* res_inf);

/* Discrete energy E_h at u (Sec. 5.3; order 6: Sec. 5.4 evaluated at
 * nu = u - mean(g)).  *E is host memory. */
psd_status psd_energy(psd_handle* h, int inst, const double* f, const double* g,
                      const double* u, double* E);

/* Gradient delta E_h[u] with respect to the grid inner product (.,.)_2
 * (Sec. 5.3): order 4: N_h[u] - f;  order 6: -rho (mean zero).  The plain
 * partial derivative with respect to a cell value is h^dim times this. */
psd_status psd_grad(psd_handle* h, int inst, const double* f, const double* g,
                    const double* u, double* grad);

/* Adjoint of the converged order-4 solve (implicit differentiation through
 * N_h[u*] = f).  For each instance b: solve H lam = dJdu[b] by conjugate
 * gradients preconditioned with L_h^{-1}, where H is the Hessian of E_h at
 * u*[b] (second variation, Sec. 5.3) acting on cell values; then
 *   dJdf[b] = lam,  dJds[b] = -lam . dN/ds,  dJdeps[b] = -lam . dN/deps,
 * with dN/ds = -div_h(|grad u|^{p-2} grad u) + eps^2 Delta_h^2 u and
 * dN/deps = 2 s eps Delta_h^2 u.  dJdu, dJdf are device pointers (plain
 * partial derivatives); dJds, dJdeps, cg_iters are host arrays [batch].
 * Stops at ||res||_2 <= rtol ||dJdu||_2 or max_iter. */
psd_status psd_adjoint(psd_handle* h, const double* const* u_star, const double* const* dJdu,
                       double* const* dJdf, double* dJds, double* dJdeps, double rtol,
                       int max_iter, int* cg_iters);

/* Adjoint of the converged order-6 solve (Sec. 4 and 5.4).  With
 * u = mean(g) + nu (nu mean-zero) the solution satisfies
 *   F(nu) = P0[s lam u - s div_h(|grad_h u|^{p-2} grad_h u) + s eps^2 Delta_h^2 u
 *           + T_h(nu - g) - f] = 0,
 * whose Jacobian H (the Hessian of the sixth-order energy on mean-zero
 * functions) is symmetric positive definite.  For each instance b: solve
 * H Lam = P0 dJdu[b] by conjugate gradients preconditioned with the
 * one-field sixth-order L_h^{-1} (FP64, FFT), then
 *   dJdf[b] = Lam,  dJdg[b] = sum(dJdu[b])/N + T_h Lam   (device, may be NULL),
 *   dJds[b] = -Lam.(lam u - div_h(...) + eps^2 Delta_h^2 u),
 *   dJdeps[b] = -Lam.(2 s eps Delta_h^2 u),  dJdlam[b] = -s Lam.u
 * (host arrays [batch], each may be NULL).  dJdu are plain partial
 * derivatives of a loss of u; stops at ||res||_2 <= rtol ||P0 dJdu||_2 or
 * max_iter (cg_iters, host, may be NULL, receives the counts). */
psd_status psd_adjoint6(psd_handle* h, const double* const* u_star, const double* const* dJdu,
                        double* const* dJdf, double* const* dJdg, double* dJds, double* dJdeps,
                        double* dJdlam, double rtol, int max_iter, int* cg_iters);

/* Convex-splitting time stepping: nsteps time levels, each one PSD solve
 * warm-started from the previous level (the handle's options: tol, max_iter,
 * precision, graph_chunk).  The time step is the problem's s.
 *   PSD_SCHEME_THINFILM (order-4 handle; Sec. 6.1, thin film with slope
 *     selection): N_h[u^{n+1}] = u^n - s Delta_h^v u^n, Delta_h^v the skew
 *     Laplacian of Sec. 5.1 (vertex gradient, then vertex-to-centre divergence);
 *   PSD_SCHEME_SPFC (order-6 handle with lambda = gamma0; Sec. 6.2, square
 *     phase field crystal): the sixth-order system with g = u^n and
 *     f = -s gamma1 Delta_h u^n (5-point Laplacian; the factor s, absent
 *     from the printed scheme, makes the step consistent with the H^-1
 *     gradient flow and energy stable); w[b] (may be NULL) receives
 *     w^{n+1} of the last step.
 * u[b] (device) holds u^0 on entry and u^nsteps on exit.  stats[batch] (host)
 * receives per instance the steps completed, the summed and the largest
 * PSD iteration counts, the residual of the last solve and the worst status;
 * step_iters (host, may be NULL) receives nsteps * batch iteration counts,
 * step-major.  Stops at the first step whose solve fails (status < 0);
 * a solve that hits max_iter is reported (PSD_NOT_CONVERGED) and stepping
 * continues.  gamma1 is used by the SPFC scheme only (>= 0). */
enum { PSD_SCHEME_THINFILM = 0, PSD_SCHEME_SPFC = 1 };
typedef struct {
    int steps;
    int psd_iters;
    int max_iters;
    double res_inf;
    int status;
} psd_step_stats;
psd_status psd_timestep(psd_handle* h, int scheme, double gamma1, double* const* u, double* const* w,
                        int nsteps, psd_step_stats* stats, int* step_iters);

/* Per-update history of instance `inst` from the last psd_solve (options
 * history != 0): out[4*k + {0,1,2,3}] = alpha, ||r||_inf, ||r||_2, energy
 * decrease (p = 4 and p = 6, the integral of the polynomial q of Sec. 6.1;
 * else 0).  Copies min(cap, iters) records to host memory and returns their
 * number in *count. */
psd_status psd_history(psd_handle* h, int inst, double* out, int cap, int* count);

/* Kernel passes of one PSD iteration, in launch order (psd_pass_times). */
enum {
    PSD_PASS_ROWS_R2C = 0,   /* x-axis real-to-complex rows */
    PSD_PASS_COLS_FWD = 1,   /* y-axis forward columns (3D) */
    PSD_PASS_COLS_FUSED = 2, /* last axis: forward, 1/sigma, inverse */
    PSD_PASS_COLS_INV = 3,   /* y-axis inverse columns (3D) */
    PSD_PASS_ROWS_C2R = 4,   /* x-axis complex-to-real rows -> d */
    PSD_PASS_LS = 5,         /* line-search sums */
    PSD_PASS_LS_FIN = 6,     /* line-search reduction and root */
    PSD_PASS_RES = 7,        /* update + residual */
    PSD_PASS_RES_FIN = 8,    /* residual reduction and stop test */
    PSD_NPASS = 9
};

/* Per-pass kernel time of the last psd_solve made with options.profile set
 * and graph_chunk = 0: ms[k] = summed duration (HIP events on the solver
 * stream) of the launches of pass k, launches[k] = their number (all zero in
 * graph mode).  Arrays of PSD_NPASS entries, host memory. */
psd_status psd_pass_times(psd_handle* h, double* ms, int* launches);

/* Tiling chosen for the stencil kernels and layout of the row transforms
 * (after autotuning or defaults): out[0..5] = z-chunk of the residual,
 * z-chunk of the line search, XCD-grouped order of the residual (0/1), of the
 * line search (0/1), 3D line-search tile width (32 or 64 cells), row-pass
 * layout (0, 1, 2: the lines per block of the x-axis transforms fill about
 * 16, 32 or 64 KB of LDS; default 1).  out6 is host memory of six ints.  The
 * z-chunks and tile width matter in 3D only. */
psd_status psd_tuning(const psd_handle* h, int* out6);

/* Destroy the handle and free its workspace. */
psd_status psd_destroy(psd_handle* h);

/* Message of the last error on h (or of the last failed psd_create when h
 * is NULL).  Never NULL. */
const char* psd_last_error(const psd_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* PSD_H */
