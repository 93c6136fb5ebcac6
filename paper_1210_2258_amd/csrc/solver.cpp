// Host side of the library: argument validation, per-shape workspace plans,
// the setup sequence and the iteration loops of RL and SGP, and the C ABI.
//
// Each iteration is a fixed sequence of kernel launches with no host round
// trip; the scalar decisions (Armijo, Barzilai-Borwein, stopping) are taken
// on the device by the finalising workgroup of each reduction.  The host
// reads the device "done" flag once every block of iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>

#include "../../include/sgpdeconv.h"
#include "common.hpp"
#include "launch.hpp"

namespace sgp {

static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define SGP_HIP(x)                                                                    \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) return fail(SGP_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

enum Kind { KIND_RL = 0, KIND_SGP = 1, KIND_OP = 2 };

struct PlanKey {
  int kind, p, NY, NX, ny, nx, oy, ox, boundary, dev;
  bool operator<(const PlanKey& o) const {
    return std::tie(kind, p, NY, NX, ny, nx, oy, ox, boundary, dev) <
           std::tie(o.kind, o.p, o.NY, o.NX, o.ny, o.nx, o.oy, o.ox, o.boundary, o.dev);
  }
};

struct Plan {
  PlanKey key{};
  float* grad = nullptr;
  float* d = nullptr;
  float* invw = nullptr;
  float* Af = nullptr;
  float* Ad = nullptr;
  float* aux = nullptr;
  float2* spec = nullptr;
  float2* khat = nullptr;
  float2* knyq = nullptr;
  float2* tw_row = nullptr;
  float2* tw_col = nullptr;
  double* part = nullptr;
  unsigned* counter = nullptr;
  DevState* st = nullptr;
  DevState* host_st = nullptr;  // pinned
  double* trace = nullptr;
  int trace_rows = 0;

  ~Plan() {
    void* ptrs[] = {grad, d, invw, Af, Ad, aux, spec, khat, knyq, tw_row, tw_col, part, counter, st, trace};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
    if (host_st) (void)hipHostFree(host_st);
  }
};

static std::mutex g_mutex;
static std::map<PlanKey, std::unique_ptr<Plan>> g_plans;

static size_t part_capacity(const PlanKey& k) {
  const size_t row_blocks = (size_t)(k.NY / kTile) * k.p;
  return std::max<size_t>((size_t)(kMaxCand) * kMaxPixBlocks, 8 * row_blocks);
}

template <class T>
static int dalloc(T** p, size_t n) {
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess) return fail(SGP_E_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  return 0;
}

static int get_plan(const PlanKey& key, hipStream_t s, Plan** out) {
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    *out = it->second.get();
    return 0;
  }
  auto pl = std::make_unique<Plan>();
  pl->key = key;
  const size_t nF = (size_t)key.NY * key.NX;
  const size_t nS = (size_t)key.ny * key.nx;
  const size_t nSpec = (size_t)spec_elems(key.NY, key.NX);
  int rc;
  if ((rc = dalloc(&pl->grad, nF))) return rc;
  if ((rc = dalloc(&pl->d, nF))) return rc;
  if (key.boundary) {
    if ((rc = dalloc(&pl->invw, nF))) return rc;
    if ((rc = dalloc(&pl->aux, nF * key.p))) return rc;
  } else if (key.kind == KIND_OP) {
    if ((rc = dalloc(&pl->aux, nF))) return rc;
  }
  if ((rc = dalloc(&pl->Af, nS * key.p))) return rc;
  if (key.kind == KIND_SGP && (rc = dalloc(&pl->Ad, nS * key.p))) return rc;
  if ((rc = dalloc(&pl->spec, nSpec * key.p))) return rc;
  if ((rc = dalloc(&pl->khat, nSpec * key.p))) return rc;
  if ((rc = dalloc(&pl->knyq, (size_t)key.NY * key.p))) return rc;
  if ((rc = dalloc(&pl->tw_row, (size_t)key.NX))) return rc;
  if ((rc = dalloc(&pl->tw_col, (size_t)key.NY))) return rc;
  if ((rc = dalloc(&pl->part, part_capacity(key)))) return rc;
  if ((rc = dalloc(&pl->counter, 1))) return rc;
  if ((rc = dalloc(&pl->st, 1))) return rc;
  SGP_HIP(hipHostMalloc((void**)&pl->host_st, sizeof(DevState), hipHostMallocDefault));
  SGP_HIP(hipMemsetAsync(pl->counter, 0, sizeof(unsigned), s));
  launch_twiddle(pl->tw_row, key.NX, s);
  launch_twiddle(pl->tw_col, key.NY, s);
  SGP_HIP(hipGetLastError());
  *out = pl.get();
  g_plans[key] = std::move(pl);
  return 0;
}

struct Problem {
  const float* g = nullptr;
  const float* psf = nullptr;
  const float* bmap = nullptr;
  float b[kMaxP] = {0};
  int p = 1, ny = 0, nx = 0, NY = 0, NX = 0, oy = 0, ox = 0;
  bool boundary = false;
};

static void defaults(sgp_params* p) {
  std::memset(p, 0, sizeof(*p));
  p->max_iter = 1000;
  p->stop = SGP_STOP_FIXED;
  p->tol = 1e-4;
  p->disc_target = 1.0;
  p->init = SGP_INIT_FLAT;
  p->f0 = nullptr;
  p->beta = 1e-4;
  p->theta = 0.4;
  p->alpha0 = 1.3;
  p->alpha_min = 1e-5;
  p->alpha_max = 1e5;
  p->tau1 = 0.5;
  p->m_alpha = 3;
  p->n_bb2_only = 20;
  p->auto_bounds = 1;
  p->L1 = 1e-10;
  p->L2 = 1e10;
  p->flux_constraint = 0;
  p->flux = -1.0;
  p->sigma_R = 1e-3;
  p->max_backtracks = 40;
  p->trace = nullptr;
}

static int check_params(const sgp_params& p, int kind) {
  if (p.max_iter < 0) return fail(SGP_E_INVALID_ARG, "max_iter must be >= 0");
  if (p.stop & ~(SGP_STOP_FIXED | SGP_STOP_CONV | SGP_STOP_DISCREPANCY))
    return fail(SGP_E_INVALID_ARG, "unknown stop bits");
  if (!(p.tol >= 0)) return fail(SGP_E_INVALID_ARG, "tol must be >= 0");
  if (!(p.disc_target > 0)) return fail(SGP_E_INVALID_ARG, "disc_target must be > 0");
  if (p.init < SGP_INIT_FLAT || p.init > SGP_INIT_USER) return fail(SGP_E_INVALID_ARG, "unknown init");
  if (p.init == SGP_INIT_USER && !p.f0) return fail(SGP_E_INVALID_ARG, "SGP_INIT_USER needs f0");
  if (kind == KIND_RL && p.init == SGP_INIT_ZERO)
    return fail(SGP_E_INVALID_ARG, "RL cannot start from the zero image");
  if (kind == KIND_SGP) {
    if (!(p.beta > 0 && p.beta < 1)) return fail(SGP_E_INVALID_ARG, "beta must be in (0,1)");
    if (!(p.theta > 0 && p.theta < 1)) return fail(SGP_E_INVALID_ARG, "theta must be in (0,1)");
    if (!(p.alpha_min > 0 && p.alpha_min < p.alpha_max)) return fail(SGP_E_INVALID_ARG, "need 0 < alpha_min < alpha_max");
    if (!(p.alpha0 >= p.alpha_min && p.alpha0 <= p.alpha_max)) return fail(SGP_E_INVALID_ARG, "alpha0 outside [alpha_min, alpha_max]");
    if (!(p.tau1 > 0 && p.tau1 < 1)) return fail(SGP_E_INVALID_ARG, "tau1 must be in (0,1)");
    if (p.m_alpha < 1 || p.m_alpha > 8) return fail(SGP_E_INVALID_ARG, "m_alpha must be in 1..8");
    if (p.n_bb2_only < 0) return fail(SGP_E_INVALID_ARG, "n_bb2_only must be >= 0");
    if (!p.auto_bounds && !(p.L1 > 0 && p.L1 < p.L2)) return fail(SGP_E_INVALID_ARG, "need 0 < L1 < L2");
    if (p.max_backtracks < 0 || p.max_backtracks > kMaxCand - 1)
      return fail(SGP_E_INVALID_ARG, "max_backtracks must be in 0..40");
  }
  if (p.flux_constraint) return fail(SGP_E_INVALID_ARG, "flux_constraint is not available in this build");
  if (!(p.sigma_R > 0)) return fail(SGP_E_INVALID_ARG, "sigma_R must be > 0");
  return 0;
}

static int check_problem(const Problem& pb) {
  if (!pb.g || !pb.psf) return fail(SGP_E_INVALID_ARG, "g and psf must be non-null");
  if (pb.p < 1 || pb.p > kMaxP) return fail(SGP_E_INVALID_ARG, "p must be in 1..8");
  if (pb.ny <= 0 || pb.nx <= 0 || pb.NY <= 0 || pb.NX <= 0) return fail(SGP_E_INVALID_ARG, "sizes must be positive");
  if (!size_supported(pb.NY) || !size_supported(pb.NX))
    return fail(SGP_E_UNSUPPORTED_SIZE, "FFT lengths must be in {16..2048 powers of 2, 80, 160, 320, 640, 1280}");
  if (pb.boundary) {
    if (pb.oy < 0 || pb.ox < 0 || pb.oy + pb.ny > pb.NY || pb.ox + pb.nx > pb.NX)
      return fail(SGP_E_INVALID_ARG, "observed window S must lie inside the object domain");
  } else if (pb.ny != pb.NY || pb.nx != pb.NX || pb.oy || pb.ox) {
    return fail(SGP_E_INVALID_ARG, "periodic problems have S = Sbar");
  }
  if (!pb.bmap)
    for (int j = 0; j < pb.p; ++j)
      if (!(pb.b[j] >= 0) || !std::isfinite(pb.b[j])) return fail(SGP_E_BAD_DATA, "background must be finite and >= 0");
  return 0;
}

static int current_device(int* dev) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(SGP_E_NO_DEVICE, "no HIP device available");
  SGP_HIP(hipGetDevice(dev));
  return 0;
}

struct Launcher {
  Args base;
  hipStream_t s;
  int NY, NX;
  void row(int op, int jc, int iter, int flag = 0) {
    Args a = base;
    a.nblk = (NY / kTile) * jc;
    a.iter = iter;
    a.flag = flag;
    launch_row(NX, op, dim3(NY / kTile, jc), a, s);
  }
  void col(int mode, int conj, int jc, int iter) {
    Args a = base;
    const int C = col_width(NY);
    a.iter = iter;
    launch_col(NY, mode, conj, dim3((NX / 2 + C - 1) / C, jc), a, s);
  }
  void pix(int op, long long n, int iter, int jsel = 0) {
    Args a = base;
    long long nb = (n + kPixThreads - 1) / kPixThreads;
    nb = std::max<long long>(1, std::min<long long>(nb, kMaxPixBlocks));
    a.nblk = (int)nb;
    a.iter = iter;
    a.jsel = jsel;
    launch_pix(op, dim3((unsigned)nb), a, s);
  }
};

static int read_state(Plan* pl, hipStream_t s) {
  SGP_HIP(hipMemcpyAsync(pl->host_st, pl->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  SGP_HIP(hipStreamSynchronize(s));
  return 0;
}

// Setup shared by every solver: validation of data and PSFs, transfer
// functions, boundary weights.  On return the state's flags are checked.
static int setup_common(Plan* pl, Launcher& L, const Problem& pb) {
  const long long nS = (long long)pb.ny * pb.nx, nF = (long long)pb.NY * pb.NX;
  L.pix(PIX_VALIDATE, pb.p * nS, 0);
  for (int j = 0; j < pb.p; ++j) L.pix(PIX_PSFSUM, nF, 0, j);
  SGP_HIP(hipGetLastError());
  int rc;
  if ((rc = read_state(pl, L.s))) return rc;
  const int fl = pl->host_st->flags;
  if (fl & FLAG_BAD_PSF) return fail(SGP_E_BAD_PSF, "PSF has negative or non-finite entries or a non-positive sum");
  if (fl & FLAG_BAD_DATA) return fail(SGP_E_BAD_DATA, "g must be finite and >= 0");
  if (fl & FLAG_BAD_BG) return fail(SGP_E_BAD_DATA, "background map must be finite and >= 0");
  // transfer functions K_j / (NY NX): shifted PSF -> row FFT -> column FFT
  L.row(ROW_PSF, pb.p, 0);
  L.col(COL_FWD, 0, pb.p, 0);
  if (pb.boundary) {
    // alpha_j = K_j correlated with M_S, then R and M_R / alpha
    L.row(ROW_MASKS, 1, 0);
    L.col(COL_CONV, 1, 1, 0);
    L.row(ROW_STORE, pb.p, 0);
    Args save = L.base;
    L.base.d = pl->invw;
    L.pix(PIX_INVW, nF, 0);
    L.base = save;
  }
  SGP_HIP(hipGetLastError());
  return 0;
}

static void fill_state(DevState& h, const sgp_params& p, const Problem& pb, double* trace) {
  std::memset(&h, 0, sizeof(h));
  h.max_iter = p.max_iter;
  h.stop = p.stop;
  h.m_alpha = p.m_alpha;
  h.n_bb2_only = p.n_bb2_only;
  h.auto_bounds = p.auto_bounds;
  h.max_backtracks = p.max_backtracks;
  h.flux_constraint = p.flux_constraint;
  h.trace_on = trace ? 1 : 0;
  h.trace = trace;
  h.init = p.init;
  h.p = pb.p;
  h.tol = p.tol;
  h.disc_target = p.disc_target;
  h.beta = p.beta;
  h.theta = p.theta;
  h.alpha0 = p.alpha0;
  h.alpha_min = p.alpha_min;
  h.alpha_max = p.alpha_max;
  h.tau1 = p.tau1;
  h.L1p = p.L1;
  h.L2p = p.L2;
  h.sigma_R = p.sigma_R;
  h.flux = p.flux;
  h.norm_disc = 2.0 / ((double)pb.p * (double)pb.ny * (double)pb.nx);
  h.alpha = p.alpha0;
  h.tau = p.tau1;
  h.lam = 1.0;
  h.L1 = p.L1;
  h.L2 = p.L2;
}

static int finish(Plan* pl, Launcher& L, const sgp_params& prm, const Problem& pb, sgp_report* rep,
                  std::chrono::steady_clock::time_point t0, int kind) {
  int rc;
  if ((rc = read_state(pl, L.s))) return rc;
  const DevState& h = *pl->host_st;
  if (prm.trace && pl->trace) {
    SGP_HIP(hipMemcpy(prm.trace, pl->trace, sizeof(double) * kTraceCols * (size_t)(prm.max_iter + 1),
                      hipMemcpyDeviceToHost));
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (rep) {
    rep->iters = h.k;
    rep->stop_reason = h.reason;
    rep->backtracks = h.total_back;
    rep->used_fallback = 0;
    rep->kl = h.J;
    rep->discrepancy = h.norm_disc * h.J;
    rep->flux = std::nan("");
    rep->L1 = h.L1;
    rep->L2 = h.L2;
    rep->seconds = secs;
  }
  (void)kind;
  switch (h.reason) {
    case REASON_NUMERIC: return fail(SGP_E_NUMERIC, "non-finite value during the iteration");
    case REASON_ARMIJO: return SGP_W_ARMIJO_EXHAUSTED;
    case REASON_STATIONARY: return SGP_W_STATIONARY;
    case REASON_MAXITER: return (prm.stop & (SGP_STOP_CONV | SGP_STOP_DISCREPANCY)) ? SGP_W_MAXITER : SGP_OK;
    default: return SGP_OK;
  }
}

static int solve(int kind, const Problem& pb, const sgp_params* prm_in, float* f, sgp_report* rep,
                 void* stream) {
  const auto t0 = std::chrono::steady_clock::now();
  sgp_params prm;
  if (prm_in) prm = *prm_in;
  else defaults(&prm);
  int rc;
  if (!f) return fail(SGP_E_INVALID_ARG, "f must be non-null");
  if ((rc = check_problem(pb))) return rc;
  if ((rc = check_params(prm, kind))) return rc;
  int dev;
  if ((rc = current_device(&dev))) return rc;
  std::lock_guard<std::mutex> lock(g_mutex);
  hipStream_t s = (hipStream_t)stream;
  PlanKey key{kind, pb.p, pb.NY, pb.NX, pb.ny, pb.nx, pb.oy, pb.ox, pb.boundary ? 1 : 0, dev};
  Plan* pl;
  if ((rc = get_plan(key, s, &pl))) return rc;
  if (prm.trace) {
    const int rows = prm.max_iter + 1;
    if (pl->trace_rows < rows) {
      if (pl->trace) (void)hipFree(pl->trace);
      pl->trace = nullptr;
      pl->trace_rows = 0;
      if ((rc = dalloc(&pl->trace, (size_t)rows * kTraceCols))) return rc;
      pl->trace_rows = rows;
    }
    SGP_HIP(hipMemsetAsync(pl->trace, 0, sizeof(double) * kTraceCols * rows, s));
  }
  fill_state(*pl->host_st, prm, pb, prm.trace ? pl->trace : nullptr);
  SGP_HIP(hipMemcpyAsync(pl->st, pl->host_st, sizeof(DevState), hipMemcpyHostToDevice, s));

  Launcher L;
  std::memset(&L.base, 0, sizeof(L.base));
  Args& a = L.base;
  a.NY = pb.NY; a.NX = pb.NX; a.ny = pb.ny; a.nx = pb.nx; a.oy = pb.oy; a.ox = pb.ox; a.p = pb.p;
  a.g = pb.g; a.bmap = pb.bmap;
  for (int j = 0; j < kMaxP; ++j) a.b[j] = pb.b[j];
  a.f = f; a.grad = pl->grad; a.d = pl->d;
  a.invw = pb.boundary ? pl->invw : nullptr;
  a.invw_s = 1.0f / (float)pb.p;
  a.Af = pl->Af; a.Ad = pl->Ad; a.spec = pl->spec; a.khat = pl->khat; a.knyq = pl->knyq;
  a.psf = pb.psf; a.aux = pl->aux; a.src = prm.f0;
  a.tw_row = pl->tw_row; a.tw_col = pl->tw_col;
  a.part = pl->part; a.counter = pl->counter; a.st = pl->st;
  L.s = s; L.NY = pb.NY; L.NX = pb.NX;

  if ((rc = setup_common(pl, L, pb))) return rc;
  const long long nS = (long long)pb.ny * pb.nx, nF = (long long)pb.NY * pb.NX;
  if (prm.init == SGP_INIT_FLAT) L.pix(PIX_FLATSUM, pb.p * nS, 0);
  L.pix(PIX_INITF, nF, 0);
  // spectrum of f^(0)
  a.src = f;
  L.row(ROW_FIELD, 1, 0);
  SGP_HIP(hipGetLastError());

  const int block = 8;  // iterations between host checks of the done flag
  if (kind == KIND_SGP) {
    // one RL step from f^(0): A_j f^(0), J(f^(0)), grad J(f^(0)), (L1, L2)
    L.col(COL_CONV, 0, 1, 0);
    L.row(ROW_RATIO, pb.p, 0, 1);
    L.col(COL_CORRSUM, 1, 1, 0);
    L.row(ROW_SETUPGRAD, 1, 0);
    SGP_HIP(hipGetLastError());
    for (int it = 0; it < prm.max_iter; it += block) {
      const int nb = std::min(block, prm.max_iter - it);
      for (int b = 0; b < nb; ++b) {
        L.row(ROW_DIR, 1, 1);
        L.col(COL_CONV, 0, 1, 1);
        L.row(ROW_AD, pb.p, 1);
        L.pix(PIX_ARMIJO_MORE, pb.p * nS, 1);
        L.row(ROW_UPD, pb.p, 1);
        L.col(COL_CORRSUM, 1, 1, 1);
        L.row(ROW_GRAD, 1, 1);
      }
      SGP_HIP(hipGetLastError());
      if ((rc = read_state(pl, s))) return rc;
      if (pl->host_st->done) break;
    }
  } else {
    for (int it = 0; it <= prm.max_iter; it += block) {
      const int nb = std::min(block, prm.max_iter + 1 - it);
      for (int b = 0; b < nb; ++b) {
        L.col(COL_CONV, 0, 1, 1);
        L.row(ROW_RATIO, pb.p, 1, 0);
        L.col(COL_CORRSUM, 1, 1, 1);
        L.row(ROW_RLUPD, 1, 1);
      }
      SGP_HIP(hipGetLastError());
      if ((rc = read_state(pl, s))) return rc;
      if (pl->host_st->done) break;
    }
  }
  return finish(pl, L, prm, pb, rep, t0, kind);
}

static int apply_operator(const float* psf, const float* x, int ny, int nx, int adjoint, float* out,
                          void* stream) {
  if (!psf || !x || !out) return fail(SGP_E_INVALID_ARG, "null pointer");
  Problem pb;
  pb.g = x;  // validated like data only for finiteness of the PSF; x may be signed
  pb.psf = psf;
  pb.p = 1; pb.ny = pb.NY = ny; pb.nx = pb.NX = nx;
  int rc;
  if ((rc = check_problem(pb))) return rc;
  int dev;
  if ((rc = current_device(&dev))) return rc;
  std::lock_guard<std::mutex> lock(g_mutex);
  hipStream_t s = (hipStream_t)stream;
  PlanKey key{KIND_OP, 1, ny, nx, ny, nx, 0, 0, 0, dev};
  Plan* pl;
  if ((rc = get_plan(key, s, &pl))) return rc;
  sgp_params prm;
  defaults(&prm);
  fill_state(*pl->host_st, prm, pb, nullptr);
  SGP_HIP(hipMemcpyAsync(pl->st, pl->host_st, sizeof(DevState), hipMemcpyHostToDevice, s));
  Launcher L;
  std::memset(&L.base, 0, sizeof(L.base));
  Args& a = L.base;
  a.NY = ny; a.NX = nx; a.ny = ny; a.nx = nx; a.p = 1;
  a.psf = psf; a.spec = pl->spec; a.khat = pl->khat; a.knyq = pl->knyq; a.aux = pl->aux;
  a.tw_row = pl->tw_row; a.tw_col = pl->tw_col; a.part = pl->part; a.counter = pl->counter; a.st = pl->st;
  a.invw_s = 1.f;
  L.s = s; L.NY = ny; L.NX = nx;
  L.pix(PIX_PSFSUM, (long long)ny * nx, 0, 0);
  if ((rc = read_state(pl, s))) return rc;
  if (pl->host_st->flags & FLAG_BAD_PSF) return fail(SGP_E_BAD_PSF, "PSF has negative or non-finite entries or a non-positive sum");
  L.row(ROW_PSF, 1, 0);
  L.col(COL_FWD, 0, 1, 0);
  a.src = x;
  L.row(ROW_FIELD, 1, 0);
  L.col(COL_CONV, adjoint ? 1 : 0, 1, 0);
  L.row(ROW_STORE, 1, 0);
  SGP_HIP(hipGetLastError());
  SGP_HIP(hipMemcpyAsync(out, pl->aux, sizeof(float) * (size_t)ny * nx, hipMemcpyDeviceToDevice, s));
  SGP_HIP(hipStreamSynchronize(s));
  return 0;
}

}  // namespace sgp

using namespace sgp;

static void fill_b(Problem& pb, const float* b_const, int p) {
  for (int j = 0; j < p && j < kMaxP; ++j) pb.b[j] = b_const ? b_const[j] : 0.f;
}

extern "C" {

int sgp_params_init(sgp_params* p) {
  if (!p) return fail(SGP_E_INVALID_ARG, "null params");
  defaults(p);
  return SGP_OK;
}

static int single(int kind, const float* g, const float* psf, const float* b_map, float b_const, int ny,
                  int nx, const sgp_params* prm, float* f, sgp_report* rep, void* stream) {
  Problem pb;
  pb.g = g; pb.psf = psf; pb.bmap = b_map; pb.b[0] = b_const;
  pb.p = 1; pb.ny = pb.NY = ny; pb.nx = pb.NX = nx;
  return solve(kind, pb, prm, f, rep, stream);
}

int rl_deconv(const float* g, const float* psf, const float* b_map, float b_const, int ny, int nx,
              const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream) {
  try { return single(KIND_RL, g, psf, b_map, b_const, ny, nx, prm, f, rep, hip_stream); }
  catch (...) { return fail(SGP_E_HIP, "internal error"); }
}

int sgp_deconv(const float* g, const float* psf, const float* b_map, float b_const, int ny, int nx,
               const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream) {
  try { return single(KIND_SGP, g, psf, b_map, b_const, ny, nx, prm, f, rep, hip_stream); }
  catch (...) { return fail(SGP_E_HIP, "internal error"); }
}

static int multi(int kind, const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                 int ny, int nx, const sgp_params* prm, float* f, sgp_report* rep, void* stream) {
  if (!b_map && !b_const) return fail(SGP_E_INVALID_ARG, "need b_map or b_const");
  if (p < 1 || p > kMaxP) return fail(SGP_E_INVALID_ARG, "p must be in 1..8");
  Problem pb;
  pb.g = g; pb.psf = psf; pb.bmap = b_map;
  fill_b(pb, b_const, p);
  pb.p = p; pb.ny = pb.NY = ny; pb.nx = pb.NX = nx;
  return solve(kind, pb, prm, f, rep, stream);
}

int sgp_multi_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                     int ny, int nx, const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream) {
  try { return multi(KIND_SGP, g, psf, b_map, b_const, p, ny, nx, prm, f, rep, hip_stream); }
  catch (...) { return fail(SGP_E_HIP, "internal error"); }
}

int rl_multi_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                    int ny, int nx, const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream) {
  try { return multi(KIND_RL, g, psf, b_map, b_const, p, ny, nx, prm, f, rep, hip_stream); }
  catch (...) { return fail(SGP_E_HIP, "internal error"); }
}

static int bnd(int kind, const float* g, const float* psf, const float* b_map, const float* b_const, int p,
               int ny, int nx, int NY, int NX, int oy, int ox, const sgp_params* prm, float* f,
               sgp_report* rep, void* stream) {
  if (!b_map && !b_const) return fail(SGP_E_INVALID_ARG, "need b_map or b_const");
  if (p < 1 || p > kMaxP) return fail(SGP_E_INVALID_ARG, "p must be in 1..8");
  Problem pb;
  pb.g = g; pb.psf = psf; pb.bmap = b_map;
  fill_b(pb, b_const, p);
  pb.p = p; pb.ny = ny; pb.nx = nx; pb.NY = NY; pb.NX = NX; pb.oy = oy; pb.ox = ox;
  pb.boundary = true;
  return solve(kind, pb, prm, f, rep, stream);
}

int sgp_boundary_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                        int ny, int nx, int NY, int NX, int oy, int ox, const sgp_params* prm, float* f,
                        sgp_report* rep, void* hip_stream) {
  try { return bnd(KIND_SGP, g, psf, b_map, b_const, p, ny, nx, NY, NX, oy, ox, prm, f, rep, hip_stream); }
  catch (...) { return fail(SGP_E_HIP, "internal error"); }
}

int rl_boundary_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                       int ny, int nx, int NY, int NX, int oy, int ox, const sgp_params* prm, float* f,
                       sgp_report* rep, void* hip_stream) {
  try { return bnd(KIND_RL, g, psf, b_map, b_const, p, ny, nx, NY, NX, oy, ox, prm, f, rep, hip_stream); }
  catch (...) { return fail(SGP_E_HIP, "internal error"); }
}

int sgp_apply_operator(const float* psf, const float* x, int ny, int nx, int adjoint, float* out,
                       void* hip_stream) {
  try { return apply_operator(psf, x, ny, nx, adjoint, out, hip_stream); }
  catch (...) { return fail(SGP_E_HIP, "internal error"); }
}

int sgp_release_cache(void) {
  std::lock_guard<std::mutex> lock(g_mutex);
  (void)hipDeviceSynchronize();
  g_plans.clear();
  return SGP_OK;
}

const char* sgp_strerror(int code) {
  switch (code) {
    case SGP_OK: return "success";
    case SGP_W_MAXITER: return "warning: iteration cap reached before the stop rule";
    case SGP_W_ARMIJO_EXHAUSTED: return "warning: Armijo backtracking exhausted";
    case SGP_W_STATIONARY: return "warning: stationary point (grad^T d = 0)";
    case SGP_E_INVALID_ARG: return "invalid argument";
    case SGP_E_UNSUPPORTED_SIZE: return "unsupported FFT size";
    case SGP_E_BAD_PSF: return "bad PSF";
    case SGP_E_BAD_DATA: return "bad data";
    case SGP_E_HIP: return "HIP runtime error";
    case SGP_E_NUMERIC: return "numerical failure (NaN/Inf)";
    case SGP_E_NO_DEVICE: return "no HIP device";
    default: return "unknown code";
  }
}

const char* sgp_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
