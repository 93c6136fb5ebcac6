// Shared host/device definitions of the SGP deconvolution library.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sgp {

constexpr int kMaxP = 8;          // images per problem (multi-image deconvolution)
constexpr int kMaxCand = 41;      // Armijo candidates theta^0 .. theta^40
constexpr int kTraceCols = 20;    // columns of the per-iteration trace
constexpr int kTile = 8;          // rows per block of the spectrum layout
constexpr int kRP = 4;            // row pairs per row-kernel workgroup (kTile / 2)
constexpr int kPixThreads = 256;  // threads of the pointwise kernels
constexpr int kMaxPixBlocks = 1024;

// stop-rule bits (Sect. 3.3)
enum { STOP_FIXED = 1, STOP_CONV = 2, STOP_DISCREPANCY = 4, STOP_RMSE = 8 };
// stop reasons reported back
enum { REASON_MAXITER = 0, REASON_CONV = 1, REASON_DISCREPANCY = 2, REASON_RMSE = 3,
       REASON_STATIONARY = 4, REASON_ARMIJO = 5, REASON_NUMERIC = 6 };
// start options (Sect. 3.1)
enum { INIT_FLAT = 0, INIT_ZERO = 1, INIT_DATA = 2, INIT_USER = 3, INIT_WARM = 4 };
// data validation flags
enum { FLAG_BAD_DATA = 1, FLAG_BAD_PSF = 2, FLAG_BAD_BG = 4 };

// Trace columns, one row per iteration (the same fields as the oracle's log).
enum { TR_K = 0, TR_ALPHA, TR_GD, TR_BACK, TR_LAM, TR_J, TR_A, TR_C1, TR_C2, TR_E,
       TR_A1, TR_A2, TR_BR1, TR_BR2, TR_ALT, TR_TAU, TR_ALPHA_NEXT, TR_FLUXMU };

// Device-resident solver state: parameters, scalars and flags.  Written by
// the single finalising thread of each reduction, read by every workgroup of
// the following kernels.
struct DevState {
  // parameters
  int max_iter, stop, m_alpha, n_bb2_only, auto_bounds, max_backtracks, flux_constraint, trace_on;
  int init, p;
  double tol, disc_target, beta, theta, alpha0, alpha_min, alpha_max, tau1, L1p, L2p, sigma_R, flux;
  // iteration scalars
  double alpha, tau, L1, L2, J, Jprev, gd, lam, flux_c;
  double Q[8];
  int nQ, k, done, reason, need_more, nback, total_back, flags;
  int pause, k_stop;  // a stepping call stops (resumably) once k reaches k_stop
  double lam_tab[kMaxCand];
  double psf_scale[kMaxP];
  double norm_disc;  // 2 / (p |S|), Eq. (discrepancy)
  double cflat, ymin, ymax;
  double fsum;       // sum of f (PIX_FSUM)
  double J_alt;      // KL of the flat start when a given start is judged against it
  int used_fallback; // the given start was replaced by the flat one
  double mu;         // flux-projection multiplier
  double flux_fixed; // sum of max(0, z) over pixels with D = 0
  double flux_cnt;   // active-set size at the current mu
  int flux_done;     // Newton iteration for mu has converged
  int flux_unconv;   // iterations whose multiplier had not converged after the last Newton pass
  double* trace;     // [max_iter + 1][kTraceCols] or null
  double rl_alpha;   // exponent of the relaxed RL step, Eq. (RL1) (1: RL)
  int f_pending;     // an accepted step waits for f += lam d (taken by the
                     // gradient pass, also after a stop; cleared after it)
  int spec_ok;       // lambda = 1 accepted: the update the A d pass made for it stands
  // reconstruction-error stop (Sect. 3.3)
  double rms_prev;   // rho of the last iterate evaluated
  int rms_k;         // iteration count at which rho was last evaluated (-1: none)
  int rms_back;      // the run ended past the minimum: the previous iterate is returned
  // linear relaxation of RL, Eq. (RL2): the SGP iteration with alpha = 1,
  // D = (M_R / w) f, no steplength rule, and an Armijo search from the
  // largest step keeping f >= 0 down to 1
  int rl2;
  double lam_cap;    // largest step tried
  double lam_bound;  // largest step keeping f >= 0 (min over d < 0 of f / -d)
};

// Kernel arguments (passed by value).
struct Args {
  int NY, NX;            // FFT domain Sbar
  int ny, nx, oy, ox;    // observed window S inside Sbar
  int p;                 // number of images
  int nblk;              // workgroups taking part in this launch's reduction
  int iter;              // 1: iteration kernel, exits when the solver is done
  int flag;              // op-specific switch
  int jsel;              // op-specific image index
  const float* g;        // [p][ny][nx]
  const float* bmap;     // [p][ny][nx] or null
  const float* bvec;     // [p] constant backgrounds in device memory (used when bmap is null)
  float* f;              // [NY][NX] iterate
  float* grad;           // [NY][NX]
  float* d;              // [NY][NX]
  const float* invw;     // [NY][NX] M_R / alpha, or null for the scalar invw_s
  float invw_s;
  float* Af;             // [p][ny][nx]
  float* Af2;            // [p][ny][nx] second A f: SGP iteration k reads Af (k even) or Af2
                         // (k odd) and writes the other
  float* Ad;             // [p][ny][nx]
  float2* spec;          // [p][NY * NX / 2] row-blocked half spectra
  float2* khat;          // [p][NY * NX / 2] transfer functions / (NY NX)
  float2* knyq;          // [p][NY]       Nyquist column of each transfer function
  const float* psf;      // [p][NY][NX]
  float* aux;            // [p][NY][NX] scratch field (boundary weights)
  const float* src;      // generic input field
  const float* ftrue;    // [NY][NX] true object of the reconstruction-error stop, or null
  const float2* tw_row;  // twiddles for length NX
  const float2* tw_col;  // twiddles for length NY
  double* part;          // reduction partials [slot][nblk]
  unsigned* counter;     // arrival counter of the reduction
  DevState* st;
  // batched launches (nbatch > 0): item blockIdx.z takes its data through the
  // pointer tables and offsets below (see batch_view)
  int nbatch;
  const float* const* gtab;   // [nbatch] observed image of each item
  float* const* ftab;         // [nbatch] iterate of each item
  const float* const* psftab; // [nbatch] PSF of each item
  const float* const* srctab; // [nbatch] user start of each item, or null
  const int* zmap;            // [gridDim.z] item of each grid-z slice (null: slice = item)
  // deferred second reduction stage: 1 + the row op whose partials (fin_nblk
  // workgroups) this launch finalises first (0: none)
  int fin_op;
  int fin_nblk;
  // image range of a launch: row launches work on images j0 + blockIdx.y,
  // column launches on images j0 .. j0 + jn - 1 (jn = 0: all p)
  int j0, jn;
  long long item_field;       // NY*NX: grad, d
  long long item_obs;         // p*ny*nx: Af, Ad
  long long item_spec;        // p*NY*NX/2: spec, khat
  long long item_nyq;         // p*NY: knyq
  long long item_part;        // partials per item
};

// Row-kernel operations: pointwise work fused into the row FFT passes.
enum RowOp {
  ROW_PSF = 0,      // fwd: shifted, scaled PSF  -> spec[j]
  ROW_MASKS,        // fwd: M_S                   -> spec[0]
  ROW_STORE,        // inv: spec[j]               -> aux[j]
  ROW_FIELD,        // fwd: src                   -> spec[0]
  ROW_RATIO,        // inv+fwd: A_j f -> rho_j, KL (RL step / setup)
  ROW_RLUPD,        // inv+fwd: RL update of f    -> spec[0]
  ROW_SETUPGRAD,    // inv: gradient at f0, min/max of one RL step (bounds)
  ROW_DIR,          // fwd: scaling, projection, direction d -> spec[0]
  ROW_AD,           // inv+fwd: A_j d, Armijo candidates lambda = 1, theta, and the
                    // update for lambda = 1: A_j f + A_j d, KL, delta rho_j -> spec[j]
  ROW_UPD,          // fwd: the update for an accepted lambda other than 1 (else no work)
  ROW_GRAD,         // inv: gradient change z, new gradient, BB sums
  ROW_NOPS
};

// Column-kernel modes.
enum ColMode {
  COL_FWD = 0,      // spec[j] -> khat[j], knyq[j]   (setup)
  COL_CONV,         // spec[0] -> spec[j] = K_j x (or conj K_j x)
  COL_CORRSUM,      // spec[j] -> spec[0] = sum_j conj(K_j) x_j
  COL_CORR1,        // COL_CORRSUM for p = 1 (fewer registers)
  COL_CONV1,        // COL_CONV of one image (fewer registers)
  COL_NMODES
};

// Pointwise (non-FFT) kernels.
enum PixOp {
  PIX_VALIDATE = 0, // g, b checks
  PIX_PSFSUM,       // PSF sum, sign and finiteness (image jsel)
  PIX_FLATSUM,      // sum_S (g - b) over all images -> flat start value
  PIX_INITF,        // write the start image
  PIX_INVW,         // boundary: R mask and M_R / alpha from aux (alpha_j)
  PIX_ARMIJO,       // Armijo test of lambda = 1, theta; if both fail, further theta^m
  PIX_FLUX_INIT,    // flux projection: all-active multiplier and bracket
  PIX_FLUX_NEWTON,  // flux projection: one Newton step on the multiplier
  PIX_FSUM,         // sum of f (flux of the start image)
  PIX_FSCALE,       // scale f to the prescribed flux
  PIX_CHOOSE,       // keep the given start or fall back to the flat one (lower KL wins)
  PIX_INVWJ,        // boundary OSEM: per-image weights M_R / alpha_j from aux
  PIX_FCOPY,        // reconstruction-error stop: f -> d (the iterate before an update)
  PIX_RMSE,         // reconstruction-error stop: rho of the current f, stop at its first increase
  PIX_RL2MAX,       // Eq. (RL2): largest step keeping f + lam d >= 0, and the step candidates
  PIX_RL2ZERO,      // Eq. (RL2): a step at that bound zeroes the pixels that bound it
  PIX_NOPS
};

__host__ __device__ inline long long spec_elems(int NY, int NX) { return (long long)NY * (NX / 2); }

}  // namespace sgp
