/* sgpdeconv.h -- C ABI of the MI355X (gfx950) SGP / Richardson-Lucy library.
 *
 * Method: Prato, Cavicchioli, Zanni, Boccacci, Bertero, "Efficient
 * deconvolution methods for astronomical imaging: algorithms and IDL-GPU
 * codes", A&A 539, A133 (2012).  Given detected images g_j, PSFs K_j and
 * backgrounds b_j, the calls below return f >= 0 minimising the
 * Kullback-Leibler divergence J_0(f; g) of Sect. 1 Eq. (divergence) (summed
 * over the images, Sect. 2.3 Eq. (multipleKL)) by scaled gradient projection
 * (Sect. 2.1, Algorithm 1) or by the Richardson-Lucy iteration (Sect. 1,
 * Eq. (RL); Sect. 2.3 Eq. (multipleRL); Sect. 2.4 Eq. (boundaryRL)).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Array pointers are DEVICE pointers (hipMalloc / torch CUDA tensors on the
 *   current HIP device), float32, C-contiguous row-major with x fastest.
 *   Image stacks are [p][ny][nx].  The caller owns every array; the library
 *   never frees or keeps them after return.  Inputs are never modified; f is
 *   overwritten.
 * - Every PSF has the size of its FFT domain, its centre at (NY/2, NX/2), and
 *   is normalised to unit volume by the library (Sect. 1; Sect. 2.4: over the
 *   broader domain).  Negative or non-finite PSF entries, or a zero sum, give
 *   SGP_E_BAD_PSF.
 * - The background is a map (b_map, same layout as g) or, when b_map is NULL,
 *   one constant per image (Sect. 1: b is a known array).  g must be finite
 *   and >= 0 (SGP_E_BAD_DATA); b must be >= 0 (SGP_E_BAD_DATA).
 * - FFT lengths (ny, nx; NY, NX for the boundary call) must be one of
 *   16 32 64 128 256 512 1024 2048 80 160 320 640 1280; anything else gives
 *   SGP_E_UNSUPPORTED_SIZE.
 * - Calls are ordered on hip_stream (NULL = the null stream) and synchronous
 *   on return: the report is filled in and f is ready.  A call allocates the
 *   workspace it needs (kept in a per-shape cache until sgp_release_cache).
 *   Calls are thread-safe; concurrent calls on one device serialise.
 * - Return value: 0 on success; positive warnings leave a valid f;
 *   negative errors leave f unspecified.  sgp_last_error() gives a
 *   thread-local message for the last failing call.  No exception crosses
 *   the ABI.
 */
#ifndef SGPDECONV_H
#define SGPDECONV_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define SGP_OK 0
#define SGP_W_MAXITER 1            /* max_iter reached before the requested stop rule */
#define SGP_W_ARMIJO_EXHAUSTED 2   /* backtracking cap hit (Algorithm 1, step 5) */
#define SGP_W_STATIONARY 3         /* grad^T d = 0: f is stationary */
#define SGP_W_FLUX_UNCONVERGED 4   /* flux constraint: in some iteration the Newton passes for the
                                      projection multiplier ended before its root, so that direction
                                      was projected with sum above the prescribed flux (count in
                                      sgp_report.flux_unconverged) */
#define SGP_E_INVALID_ARG -1
#define SGP_E_UNSUPPORTED_SIZE -2
#define SGP_E_BAD_PSF -3
#define SGP_E_BAD_DATA -4
#define SGP_E_HIP -5
#define SGP_E_NUMERIC -6           /* NaN / Inf appeared mid-run */
#define SGP_E_NO_DEVICE -7

/* stopping rules, Sect. 3.3 (bitmask; the first rule met ends the run) */
#define SGP_STOP_FIXED 1           /* max_iter iterations */
#define SGP_STOP_CONV 2            /* Eq. (convergence): |J(k+1) - J(k)| <= tol J(k) */
#define SGP_STOP_DISCREPANCY 4     /* Eq. (discrepancy): 2 J / (p ny nx) <= disc_target */
#define SGP_STOP_RMSE 8            /* Sect. 3.3, minimum of the relative reconstruction error
                                      rho = ||f - f_true||_2 / ||f_true||_2 (simulation studies; needs
                                      f_true): rho is evaluated as each iterate is formed, over the
                                      object domain, and at its first increase the previous iterate,
                                      the minimum, is returned (with its KL and iteration count).
                                      Single problems only (not sgp_batch_deconv / the mosaic). */

/* stop reasons reported in sgp_report.stop_reason */
#define SGP_REASON_MAXITER 0
#define SGP_REASON_CONV 1
#define SGP_REASON_DISCREPANCY 2
#define SGP_REASON_RMSE 3
#define SGP_REASON_STATIONARY 4
#define SGP_REASON_ARMIJO 5
#define SGP_REASON_NUMERIC 6

/* initial point, Sect. 3.1 */
#define SGP_INIT_FLAT 0   /* (mean) background-subtracted flux / (ny nx), on R only */
#define SGP_INIT_ZERO 1   /* not valid for RL, whose iterates stay at 0 */
#define SGP_INIT_DATA 2   /* g (g_1 for several images), embedded on R */
#define SGP_INIT_USER 3   /* f0 below (device pointer, [NY][NX]); negative values clipped */
#define SGP_INIT_WARM 4   /* f0 (e.g. a learned warm start), replaced by the flat start when its
                             KL is larger; sgp_report.used_fallback tells which was used */

/* per-iteration trace columns (one row of SGP_TRACE_COLS doubles per iteration) */
#define SGP_TRACE_COLS 20
enum {
  SGP_TR_K = 0, SGP_TR_ALPHA, SGP_TR_GD, SGP_TR_BACKTRACKS, SGP_TR_LAMBDA, SGP_TR_J,
  SGP_TR_A, SGP_TR_C1, SGP_TR_C2, SGP_TR_E, SGP_TR_ALPHA1, SGP_TR_ALPHA2, SGP_TR_BB1_BRANCH,
  SGP_TR_BB2_BRANCH, SGP_TR_ALT_BRANCH, SGP_TR_TAU, SGP_TR_ALPHA_NEXT, SGP_TR_FLUX_MU
};

/* Solver parameters.  sgp_params_init() fills in the paper's defaults
 * (Sect. 3.2: beta 1e-4, theta 0.4, alpha0 1.3, tau1 0.5, alpha_max 1e5,
 * alpha_min 1e-5, M_alpha 3; adaptive (L1, L2)). */
typedef struct sgp_params {
  int max_iter;          /* cap on iterations (default 1000) */
  int stop;              /* SGP_STOP_* bitmask (default SGP_STOP_FIXED) */
  double tol;            /* Eq. (convergence) tolerance (default 1e-4) */
  double disc_target;    /* b of Eq. (discrepancy) (default 1.0) */
  int init;              /* SGP_INIT_* (default SGP_INIT_FLAT) */
  const float* f0;       /* SGP_INIT_USER start, device pointer [NY][NX] */
  double beta, theta;    /* Armijo parameters, Algorithm 1 step 5 */
  double alpha0, alpha_min, alpha_max, tau1; /* steplength rules, Sect. 2.1 */
  int m_alpha;           /* memory of Eq. (alphadef), 1..8 (default 3) */
  int n_bb2_only;        /* iterations using Eq. (alphadef) before alternation (default 20) */
  int auto_bounds;       /* 1: (L1, L2) by the Sect. 3.2 rule; 0: use L1, L2 below */
  double L1, L2;         /* scaling bounds of Eq. (Dk) when auto_bounds = 0 */
  int flux_constraint;   /* 1: project onto {f >= 0, sum f = flux} in the D^-1 metric (SGP only;
                            the constraint set named in Sect. 2), else onto f >= 0 */
  double flux;           /* flux of the constraint; < 0: mean over images of sum_S (g - b) */
  double sigma_R;        /* threshold sigma of Eq. (Rdef) (default 1e-3) */
  int max_backtracks;    /* Armijo reductions allowed, 0..40 (default 40) */
  double* trace;         /* optional HOST buffer [(max_iter + 1) * SGP_TRACE_COLS] doubles */
  double rl_alpha;       /* RL only: exponent a of the multiplicative relaxation, Sect. 1
                            Eq. (RL1), f <- f o q^a with q the RL factor of Eqs. (RL),
                            (multipleRL), (boundaryRL); in (0, 8], default 1 (plain RL;
                            the paper cites convergence for a < 2).  Other values are
                            rejected with SGP_E_INVALID_ARG, as is a != 1 for SGP / OSEM. */
  const float* f_true;   /* SGP_STOP_RMSE: the true object, device pointer [NY][NX] (the
                            object domain; [ny][nx] for periodic problems); else unused */
  int rl_line_search;    /* RL only: 1 = the linear relaxation of Sect. 1 Eq. (RL2),
                            f <- f + lam d along the RL direction d = -(M_R / w) o f o grad J
                            (the RL step minus f) with lam >= 1 by the Armijo rule of
                            Algorithm 1 (beta, theta): the first step tried is the largest
                            keeping f >= 0, at most rl_lambda_cap, then theta times the last
                            while above 1; lam = 1 (the RL step) when none passes.  0 (default):
                            the RL iteration.  Not with rl_alpha != 1. */
  double rl_lambda_cap;  /* largest step of that line search, >= 1 (default 10) */
} sgp_params;

typedef struct sgp_report {
  int iters;             /* iterations performed */
  int stop_reason;       /* SGP_REASON_* */
  int backtracks;        /* total Armijo reductions */
  int used_fallback;     /* SGP_INIT_WARM: 1 if the flat start replaced f0 */
  double kl;             /* J_0 at the returned f */
  double discrepancy;    /* 2 J_0 / (p ny nx) */
  double flux;           /* sum of f */
  double L1, L2;         /* scaling bounds used */
  double seconds;        /* wall time of the call */
  int flux_unconverged;  /* flux constraint: iterations whose multiplier had not converged after
                            the Newton passes (then the return code is at least
                            SGP_W_FLUX_UNCONVERGED) */
} sgp_report;

/* Fills *p with the defaults above.  Returns SGP_E_INVALID_ARG on NULL. */
int sgp_params_init(sgp_params* p);

/* Richardson-Lucy, Sect. 1 Eq. (RL) with a periodic convolution A f = K * f.
 * g, f: [ny][nx]; psf: [ny][nx]; b_map: [ny][nx] or NULL (then b_const).
 * Uses max_iter, stop, tol, disc_target, init, f0, trace of *prm; one
 * iteration costs two FFT convolutions. */
int rl_deconv(const float* g, const float* psf, const float* b_map, float b_const,
              int ny, int nx, const sgp_params* prm, float* f, sgp_report* rep,
              void* hip_stream);

/* SGP for one image (Sect. 2.1 Algorithm 1 with the RL scaling Eq. (Dk) and
 * the gradient of Sect. 2.2 Eq. (KLgrad)).  Arguments as rl_deconv. */
int sgp_deconv(const float* g, const float* psf, const float* b_map, float b_const,
               int ny, int nx, const sgp_params* prm, float* f, sgp_report* rep,
               void* hip_stream);

/* sgp_deconv for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same problem, arguments, iteration and results as sgp_deconv, but every
 * workspace buffer lives in one static device array of 64 MiB that the
 * library holds on each GPU it runs on until the process ends (enough for
 * about 2 million pixels: up to 2048 x 1024 or 1024 x 1024; larger sizes give
 * SGP_E_INVALID_ARG with the size needed).  The call allocates no device or
 * pinned host memory, creates no stream or graph (each iteration is launched
 * on hip_stream) and is synchronous on return.  prm->trace must be NULL.
 * Every call on a GPU shares that GPU's array, which keeps the previous
 * call's contents; calls from one process are serialised, but calls that
 * overlap on one GPU (e.g. from several processes) race. */
int sgp_deconv_noalloc(const float* g, const float* psf, const float* b_map, float b_const,
                       int ny, int nx, const sgp_params* prm, float* f, sgp_report* rep,
                       void* hip_stream);

/* SGP for p images of one object (Sect. 2.3 Eqs. (multipleKL),
 * (multiplegradient); scaling f/p).  g, psf, b_map: [p][ny][nx];
 * b_const: HOST array of p constants (used when b_map is NULL); f: [ny][nx].
 * 1 <= p <= 8. */
int sgp_multi_deconv(const float* g, const float* psf, const float* b_map,
                     const float* b_const, int p, int ny, int nx,
                     const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream);

/* RL for p images (Sect. 2.3 Eq. (multipleRL)); arguments as sgp_multi_deconv. */
int rl_multi_deconv(const float* g, const float* psf, const float* b_map,
                    const float* b_const, int p, int ny, int nx,
                    const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream);

/* SGP with boundary-effect correction (Sect. 2.4): the object lives on the
 * NY x NX domain Sbar, the images g_j ([p][ny][nx], with b_map likewise) are
 * observed on the window S at rows oy..oy+ny-1, columns ox..ox+nx-1 of Sbar.
 * psf: [p][NY][NX].  A_j = M_S o (K_j * (M_R o .)) (Eq. (projection)), the
 * weights alpha_j = A_j^T 1 before M_R, R by Eq. (Rdef) with sigma_R, scaling
 * Eq. (Dkbound).  f: [NY][NX] (zero outside R on return). */
int sgp_boundary_deconv(const float* g, const float* psf, const float* b_map,
                        const float* b_const, int p, int ny, int nx, int NY, int NX,
                        int oy, int ox, const sgp_params* prm, float* f,
                        sgp_report* rep, void* hip_stream);

/* RL with boundary-effect correction (Sect. 2.4 Eq. (boundaryRL)). */
int rl_boundary_deconv(const float* g, const float* psf, const float* b_map,
                       const float* b_const, int p, int ny, int nx, int NY, int NX,
                       int oy, int ox, const sgp_params* prm, float* f,
                       sgp_report* rep, void* hip_stream);

/* OSEM, ordered subsets over the p images (Sect. 2.3 Algorithm 2,
 * Eq. (OSEMstep)): every iteration cycles over the images,
 * h <- h o A_j^T (g_j / (A_j h + b_j)), j = 1..p.  Arguments, layouts and
 * errors as sgp_multi_deconv; the flux constraint and SGP_INIT_ZERO are
 * rejected (SGP_E_INVALID_ARG).  The KL divergence of every iterate f^(k) is
 * formed over all images for the stop rules and the report. */
int osem_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                int ny, int nx, const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream);

/* OSEM with boundary-effect correction (Sect. 2.4 Eq. (boundaryOSEM)):
 * h <- (M_R / alpha_j) o h o A_j^T (g_j / (A_j h + b_j)), alpha_j = A_j^T 1
 * before M_R.  Arguments as sgp_boundary_deconv. */
int osem_boundary_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                         int ny, int nx, int NY, int NX, int oy, int ox, const sgp_params* prm, float* f,
                         sgp_report* rep, void* hip_stream);

/* Operator application for checks and callers that build their own loops:
 * out = A_j x (adjoint = 0) or A_j^T x (adjoint = 1) for the periodic
 * operator of Sect. 1 (K_j unit-volume, centred).  x, out: [ny][nx];
 * psf: [ny][nx]. */
int sgp_apply_operator(const float* psf, const float* x, int ny, int nx, int adjoint,
                       float* out, void* hip_stream);

/* ---------------------------------------------------------------------------
 * Stepping interface.  A solver owns its workspace; create() runs the setup of
 * the one-shot calls above (validation, transfer functions, weights, start,
 * and for SGP the RL step that sets (L1, L2) and the first gradient);
 * step() advances by up to n iterations (fewer if a stop rule fires) and can
 * be called repeatedly, continuing exactly where the previous call stopped;
 * report() fills the report of the iterations so far.  The iteration loop is
 * captured once as a HIP graph of `block` iterations and replayed.
 * ------------------------------------------------------------------------- */
#define SGP_KIND_RL 0
#define SGP_KIND_SGP 1
#define SGP_KIND_OSEM 2

typedef struct sgp_problem {
  const float* g;        /* device [p][ny][nx] */
  const float* psf;      /* device [p][NY][NX] */
  const float* b_map;    /* device [p][ny][nx] or NULL */
  const float* b_const;  /* HOST [p], used when b_map is NULL */
  int p, ny, nx;
  int NY, NX, oy, ox;    /* object domain; NY = ny, NX = nx, oy = ox = 0 when periodic */
  int boundary;          /* 1: Sect. 2.4 boundary-effect correction */
} sgp_problem;

typedef struct sgp_solver sgp_solver;

/* kind: SGP_KIND_RL, SGP_KIND_SGP or SGP_KIND_OSEM.  f: device [NY][NX], the iterate, owned
 * by the caller and updated in place by step().  The parameters are copied;
 * prm->trace (if set) must stay valid until sgp_solver_destroy. */
int sgp_solver_create(int kind, const sgp_problem* prob, const sgp_params* prm, float* f,
                      void* hip_stream, sgp_solver** out);
/* Runs up to n more iterations; *done (optional) becomes 1 once a stop rule
 * or max_iter has ended the run.  Synchronous on return. */
int sgp_solver_step(sgp_solver* s, int n, int* done);
/* Captures (without running any iteration) the HIP graphs that a later
 * sgp_solver_step(s, n, ...) replays: a latency-sensitive caller moves the
 * capture out of that call.  step() captures them itself when absent; a
 * solver keeps every graph it has captured until it is destroyed. */
int sgp_solver_prepare(sgp_solver* s, int n);
int sgp_solver_report(sgp_solver* s, sgp_report* rep);
/* SGP only: copies the gradient of J_0 at the current iterate, as the solver
 * carries it (Sect. 2.2 Eq. (KLgrad), Sect. 2.3 Eq. (multiplegradient),
 * Sect. 2.4 Eq. (gradientboundary): the start's gradient plus the change of
 * every step, in float32), into out (device [NY][NX], caller-owned), so that
 * one iteration can be re-run elsewhere from the solver's own state.
 * SGP_E_INVALID_ARG for another kind or a batched solver.  Synchronous. */
int sgp_solver_gradient(sgp_solver* s, float* out);
/* Kernel timing of later step() calls (HIP events around every launch on the
 * solver's stream; graphs are not used while enabled).  ms[i] receives the
 * summed milliseconds and counts[i] the launches of kernel class i:
 * see SGP_KCLASS_*; ncls is the array length. */
#define SGP_KCLASS_ROW_DIR 0      /* scaling, projection, direction + row FFT */
#define SGP_KCLASS_COL_CONV 1     /* column FFT x K x IFFT */
#define SGP_KCLASS_ROW_AD 2       /* row IFFT -> A d, Armijo candidates */
#define SGP_KCLASS_ARMIJO_MORE 3  /* Armijo test of lambda = 1, theta; further candidates only when both fail */
#define SGP_KCLASS_ROW_UPD 4      /* update f, A f, residual change + row FFT */
#define SGP_KCLASS_COL_CORR 5     /* column FFT x conj K x IFFT, summed over images */
#define SGP_KCLASS_ROW_GRAD 6     /* row IFFT -> gradient, BB sums */
#define SGP_KCLASS_ROW_RATIO 7    /* RL: row IFFT -> ratio, KL -> row FFT */
#define SGP_KCLASS_ROW_RLUPD 8    /* RL: row IFFT -> update -> row FFT */
#define SGP_KCLASS_ROW_FIN 9      /* one-workgroup finish of a row reduction (the BB steplength rule) */
#define SGP_KCLASS_COUNT 10
int sgp_solver_set_timing(sgp_solver* s, int enable);
/* Graph replay of the iteration loop (default on); off launches every kernel
 * from the host. */
int sgp_solver_set_graph(sgp_solver* s, int enable);
int sgp_solver_timing(sgp_solver* s, double* ms, long long* counts, int ncls);
int sgp_solver_destroy(sgp_solver* s);

/* Many single-image problems in one run (images of uneven sizes, periodic
 * or boundary-corrected).  probs[i]: p = 1, b_map = NULL (constant
 * background b_const[0]); boundary problems give their FFT domain and window
 * (NY, NX, oy, ox).  f[i]: device [NY][NX] iterate of problem i; f0: NULL or
 * per-problem starts for SGP_INIT_USER / SGP_INIT_WARM.  Problems of one
 * shape (window, domain and offsets) form one batched solver (every launch
 * covers all of them); all shapes advance together in one HIP graph of
 * parallel branches, replayed until every problem has met its own stop rule.
 * reps: n reports (optional).  Returns the most severe per-problem code.
 * kind: SGP_KIND_SGP, _RL or _OSEM. */
int sgp_batch_deconv(int kind, const sgp_problem* probs, int n, float* const* f, const float* const* f0,
                     const sgp_params* prm, sgp_report* reps, void* hip_stream);

/* Mosaic of boundary-corrected subdomains (the second experiment of
 * Sect. 4.1; Sect. 2.4 for each subdomain).  The H x W image g (device,
 * row-major) is cut into core x core tiles (H, W multiples of core); tile
 * (i, j) is reconstructed from the window of g that extends the tile by
 * `margin` pixels towards its neighbours (clipped at the image edge), placed
 * at the centre of an N x N FFT domain with the N x N PSF psf (device, centre
 * (N/2, N/2)) and constant background b, by the boundary-corrected method
 * `kind` (SGP_KIND_SGP, _RL or _OSEM); all windows run as one batch and the
 * tile cores are written into f (device H x W).  Needs core + 2 margin <= N
 * and N a supported FFT size.  rep (optional): iterations and stop reason of
 * the longest-running tile, KL and backtracks summed over the tiles, the
 * largest tile discrepancy.  Staging memory is allocated per call.  Errors as
 * sgp_batch_deconv. */
int sgp_mosaic_deconv(int kind, const float* g, int H, int W, const float* psf, int N, float b, int core,
                      int margin, const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream);

/* The steplength rule of Sect. 2.1 exactly as the device runs it, callable on
 * the host for validation.  k: index of the iteration just completed;
 * alpha: steplength used in it; Q/nQ: memory of alpha^(2) values (oldest
 * first); a, c1, c2, e: the sums s'D^-2 s, s'D^-1 z, s'D z, z'D^2 z.
 * out (16 doubles): alpha1, alpha2, alpha_next, tau_next, alternation branch,
 * BB1 branch, BB2 branch, nQ, then the updated Q. */
int sgp_steplength_rule(const sgp_params* prm, int k, double alpha, double tau, const double* Q,
                        int nQ, double a, double c1, double c2, double e, double* out);

/* The multiplier of the flux-constrained projection (the constraint set
 * {x >= 0, sum x = c} of Sect. 2, projected in the D^-1 metric:
 * x_i = max(0, z_i - mu D_i) with sum x = c) found exactly as the device finds
 * it, callable on the host for validation: the all-active step, then up to
 * max_steps Newton steps on phi(mu) = sum_i max(0, z_i - mu D_i) - c, each
 * with the device's FP64 sums and finalisers.  z, D: HOST arrays of n
 * doubles (D >= 0; pixels with D = 0 are held at max(0, z)).  *mu receives
 * the multiplier, *steps (optional) the Newton steps taken, *converged
 * (optional) 1 if the active set stopped changing (mu is then the root).
 * Returns SGP_W_FLUX_UNCONVERGED when the last allowed step ended before the
 * root (the solver allows 8 per iteration), SGP_E_NUMERIC on a non-finite
 * multiplier, SGP_E_INVALID_ARG on bad arguments. */
int sgp_flux_multiplier(const double* z, const double* D, long long n, double c, int max_steps, double* mu,
                        int* steps, int* converged);

/* ---------------------------------------------------------------------------
 * FFT tile schedule and its autotuner.  The FFTs are the main cost of an
 * iteration (Sect. 3.4, Sect. 5).  Each length L has four tile variants
 * 0..3 for its row passes and for its column passes: bit 1 selects the
 * transform plan (points per thread and radix sequence), bit 0 the
 * workgroup shape:
 *   plan 0: four points per thread from 128 to 1280 (radix 4 passes, one
 *           radix 8 or 5 pass where the length needs it), eight at 2048
 *           (8,8,8,4), the radix-5-first plans of the other 5 * 2^k lengths;
 *   plan 1: eight points per thread from 128 to 1024 (radix 8 first);
 *           lengths without a second plan run plan 0;
 *   rows    shape 0: as many row pairs per workgroup as fit 1024 threads
 *                    (at most the 8-row block); shape 1: half as many;
 *   columns shape 0: as many columns as fit 256 threads (at least one) and
 *                    40 KB of LDS; shape 1: twice as many (512 threads, 1024
 *                    for a one-column tile) where the LDS tile allows, else
 *                    half as many.
 * A shape that cannot differ at some L (it would leave a wavefront partly
 * empty or overflow the LDS) equals shape 0 there.  All variants compute
 * the same per-pixel arithmetic; another plan rounds the transforms
 * differently (to the FP32 accuracy of the FFT), another shape may add the
 * FP64 per-workgroup partial sums in another grouping.  The schedule is one
 * process-wide table indexed by L (variant 0 where unset); a solver or
 * one-shot call reads it when it starts (rows of length NX, columns of
 * length NY) and keeps those variants.  Table calls are thread-safe.
 * ------------------------------------------------------------------------- */

/* Shape of tile variant `variant` (0..3) at FFT length L: threads per
 * workgroup and row pairs of the row kernel, threads and columns of the
 * column kernel (each output optional); its transforms take
 * L * row_pairs / row_threads points per thread.  Host only, no device
 * needed.  SGP_E_UNSUPPORTED_SIZE for a length the library has no FFT for,
 * SGP_E_INVALID_ARG for a variant outside 0..3. */
int sgp_tile_info(int L, int variant, int* row_threads, int* row_pairs, int* col_threads, int* col_width);
/* Sets / reads the variants used for rows and for columns of length L. */
int sgp_set_tile_schedule(int L, int row_variant, int col_variant);
int sgp_get_tile_schedule(int L, int* row_variant, int* col_variant);
/* Writes the table to a text file (a comment line, then one line
 * "L row_variant col_variant" per length set) / reads such a file and
 * applies every line.  A malformed line, unsupported length or variant
 * outside 0..3 fails the whole load with SGP_E_INVALID_ARG (naming the line)
 * and applies nothing; so does a file that cannot be opened. */
int sgp_save_tile_schedule(const char* path);
int sgp_load_tile_schedule(const char* path);
/* Autotuner: times `iters` SGP iterations of the caller's problem (periodic,
 * multi-image or boundary, as for sgp_solver_create; 1 <= iters <= 100000)
 * under every distinct combination of row variant (length NX) and column
 * variant (length NY): one untimed call that captures the graph, then three
 * timed calls of `iters` iterations each, whose least wall time per
 * iteration is the combination's time (a multiple of 32 iterations, the
 * graph block, times whole graph replays).  The fastest combination is
 * chosen unless it is within 1% of (0,0), which then stays; the choice is
 * set in the table and returned in *row_variant / *col_variant (optional).
 * ms (optional, 16 doubles): ms per iteration of (row, column) = (r, c) at
 * ms[4 r + c]; -1 for a combination equal to one already timed (a variant
 * that runs the same kernels as a lower one).
 * f: device [NY][NX], caller-owned scratch that is overwritten.  The problem
 * must run 4 iters iterations without a stop (fixed-count SGP: only a
 * numerical failure stops it), otherwise SGP_E_INVALID_ARG.  On any error
 * the table is left as it was.  While it runs, the table holds the
 * combination being timed: solvers that other threads create meanwhile get
 * that combination (correct results, possibly not the fastest shape).
 * Synchronous on return. */
int sgp_autotune(const sgp_problem* prob, float* f, int iters, int* row_variant, int* col_variant, double* ms,
                 void* hip_stream);

/* Releases every cached workspace of the calling process on the current device. */
int sgp_release_cache(void);

const char* sgp_strerror(int code);
const char* sgp_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SGPDECONV_H */
