// Host side of the library: argument validation, per-shape workspaces, the
// setup sequence, the iteration loops of RL and SGP (captured as HIP graphs),
// and the C ABI.
//
// Each iteration is a fixed sequence of kernel launches with no host round
// trip; the scalar decisions (Armijo, Barzilai-Borwein, stopping) are taken
// on the device by the finalising workgroup of each reduction.  The host
// reads the device state once per replayed block of iterations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <type_traits>
#include <array>
#include <vector>

#include "../../include/sgpdeconv.h"
#include "common.hpp"
#include "finalize.hpp"
#include "launch.hpp"

namespace sgp {

static thread_local std::string g_last_error;

static int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

void record_error(const std::string& msg) { g_last_error = msg; }

#define SGP_HIP(x)                                                                    \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) return fail(SGP_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

enum Kind { KIND_RL = SGP_KIND_RL, KIND_SGP = SGP_KIND_SGP, KIND_OSEM = SGP_KIND_OSEM, KIND_OP = 3 };
// RL and OSEM share the multiplicative update and the per-iterate KL pass
static bool em_kind(int kind) { return kind == KIND_RL || kind == KIND_OSEM; }

struct PlanKey {
  int kind, p, NY, NX, ny, nx, oy, ox, boundary, dev;
  int nitems = 1;  // batched problems of this shape
  bool operator<(const PlanKey& o) const {
    return std::tie(kind, p, NY, NX, ny, nx, oy, ox, boundary, dev, nitems) <
           std::tie(o.kind, o.p, o.NY, o.NX, o.ny, o.nx, o.oy, o.ox, o.boundary, o.dev, o.nitems);
  }
};

// Device workspace of one problem shape.
struct Plan {
  PlanKey key{};
  float* grad = nullptr;
  float* d = nullptr;
  float* invw = nullptr;
  float* invwj = nullptr;  // boundary OSEM: [p][NY][NX] per-image weights M_R / alpha_j
  float* Af = nullptr;
  float* Af2 = nullptr;  // SGP: the second A f buffer (iterations alternate)
  float* Ad = nullptr;
  float* aux = nullptr;
  float2* spec = nullptr;
  float2* khat = nullptr;
  float2* knyq = nullptr;
  float2* tw_row[2] = {nullptr, nullptr};  // twiddle tables of transform plans 0 and 1, rows (length NX)
  float2* tw_col[2] = {nullptr, nullptr};  // and columns (length NY)
  double* part = nullptr;
  unsigned* counter = nullptr;
  DevState* st = nullptr;
  DevState* host_st = nullptr;  // pinned, one per item
  double* trace = nullptr;
  int trace_rows = 0;
  // batched items: device pointer tables
  const float** gtab = nullptr;
  float** ftab = nullptr;
  const float** psftab = nullptr;
  const float** srctab = nullptr;
  float* btab = nullptr;
  int* zmap = nullptr;

  bool external = false;  // carved from the static workspace: nothing to free

  ~Plan() {
    if (external) return;
    void* ptrs[] = {grad, d, invw, invwj, Af, Af2, Ad, aux, spec, khat, knyq, tw_row[0], tw_row[1], tw_col[0],
                    tw_col[1], part, counter, st, trace,
                    (void*)gtab, (void*)ftab, (void*)psftab, (void*)srctab, btab, zmap};
    for (void* q : ptrs)
      if (q) (void)hipFree(q);
    if (host_st) (void)hipHostFree(host_st);
  }
};

static std::mutex g_mutex;
static std::map<PlanKey, std::unique_ptr<Plan>> g_plans;

// Internal stream and ordering event of the one-shot calls, one pair per
// device, kept for the process (creating a stream costs more than a small
// solve's setup).  The calls hold g_mutex, so they never share it at once.
struct SharedStream {
  hipStream_t s = nullptr;
  hipEvent_t e = nullptr;
};
static std::map<int, SharedStream> g_streams;
static int shared_stream(int dev, SharedStream** out) {
  SharedStream& ss = g_streams[dev];
  if (!ss.s) SGP_HIP(hipStreamCreateWithFlags(&ss.s, hipStreamNonBlocking));
  if (!ss.e) SGP_HIP(hipEventCreateWithFlags(&ss.e, hipEventDisableTiming));
  *out = &ss;
  return 0;
}

// workgroups of the Armijo kernel (its rare candidate pass)
#ifndef SGP_ARM_BLOCKS
#define SGP_ARM_BLOCKS 512
#endif
constexpr int kArmBlocks = SGP_ARM_BLOCKS;

static size_t part_capacity(const PlanKey& k) {
  // row kernels: at most NY / 2 workgroups per image and 4 slots; the Armijo
  // kernel keeps ROW_AD's 3 slots and adds 8 slots of its own
  const size_t row_blocks = (size_t)(k.NY / 2) * k.p;
  return std::max<size_t>({(size_t)(kMaxCand) * kMaxPixBlocks, 4 * row_blocks,
                           3 * row_blocks + (size_t)8 * kArmBlocks});
}

template <class T>
static int dalloc(T** p, size_t n) {
  if (n == 0) n = 1;
  hipError_t e = hipMalloc((void**)p, n * sizeof(T));
  if (e != hipSuccess) return fail(SGP_E_HIP, std::string("hipMalloc: ") + hipGetErrorString(e));
  return 0;
}

static int make_plan(const PlanKey& key, hipStream_t s, std::unique_ptr<Plan>& pl) {
  pl = std::make_unique<Plan>();
  pl->key = key;
  const size_t n = (size_t)key.nitems;
  const size_t nF = (size_t)key.NY * key.NX * n;
  const size_t nS = (size_t)key.ny * key.nx * n;
  const size_t nSpec = (size_t)spec_elems(key.NY, key.NX) * n;
  int rc;
  if ((rc = dalloc(&pl->grad, nF))) return rc;
  if ((rc = dalloc(&pl->d, nF))) return rc;
  if (key.boundary) {
    if ((rc = dalloc(&pl->invw, nF))) return rc;
    if ((rc = dalloc(&pl->aux, nF * key.p))) return rc;
    if (key.kind == KIND_OSEM && (rc = dalloc(&pl->invwj, nF * key.p))) return rc;
  } else if (key.kind == KIND_OP) {
    if ((rc = dalloc(&pl->aux, nF))) return rc;
  }
  if ((rc = dalloc(&pl->Af, nS * key.p))) return rc;
  if (key.kind == KIND_SGP && (rc = dalloc(&pl->Ad, nS * key.p))) return rc;
  if (key.kind == KIND_SGP && (rc = dalloc(&pl->Af2, nS * key.p))) return rc;
  if ((rc = dalloc(&pl->spec, nSpec * key.p))) return rc;
  if ((rc = dalloc(&pl->khat, nSpec * key.p))) return rc;
  if ((rc = dalloc(&pl->knyq, (size_t)key.NY * key.p * n))) return rc;
  for (int a = 0; a < 2; ++a) {
    if ((rc = dalloc(&pl->tw_row[a], (size_t)key.NX))) return rc;
    if ((rc = dalloc(&pl->tw_col[a], (size_t)key.NY))) return rc;
  }
  if ((rc = dalloc(&pl->part, part_capacity(key) * n))) return rc;
  if ((rc = dalloc(&pl->counter, n))) return rc;
  if ((rc = dalloc(&pl->st, n))) return rc;
  if (n > 1) {
    if ((rc = dalloc(&pl->gtab, n))) return rc;
    if ((rc = dalloc(&pl->ftab, n))) return rc;
    if ((rc = dalloc(&pl->psftab, n))) return rc;
    if ((rc = dalloc(&pl->srctab, n))) return rc;
    if ((rc = dalloc(&pl->zmap, n))) return rc;
  }
  if ((rc = dalloc(&pl->btab, std::max<size_t>(n, kMaxP)))) return rc;
  SGP_HIP(hipHostMalloc((void**)&pl->host_st, sizeof(DevState) * n, hipHostMallocDefault));
  SGP_HIP(hipMemsetAsync(pl->counter, 0, sizeof(unsigned) * n, s));
  for (int a = 0; a < 2; ++a) {
    launch_twiddle(pl->tw_row[a], key.NX, a, s);
    launch_twiddle(pl->tw_col[a], key.NY, a, s);
  }
  SGP_HIP(hipGetLastError());
  return 0;
}

// ------------------------------------------------ static workspace
// Workspace of the entry point that allocates nothing (sgp_deconv_noalloc):
// one file-scope device array, one copy per GPU, kept until the process ends.
// Host code never passes the array's name to a kernel (on the host it names
// a stand-in, not device memory); it uses the device address that
// hipGetSymbolAddress returns for the current device.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static char* g_scratch_ptr[kMaxDevices];  // device address of scratch, per device
static std::mutex g_scratch_mutex;          // one call on the static workspace at a time

static int scratch_address(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(SGP_E_INVALID_ARG, "device index beyond the static workspace table");
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SGP_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)ptr;
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

// Lays out the workspace of one single-image periodic problem (the fields of
// make_plan with nitems = 1) from base; returns the bytes used.  With base
// null only the size is computed.
static size_t carve_plan(const PlanKey& key, char* base, Plan& pl) {
  size_t off = 0;
  auto take = [&](auto** p, size_t n) {
    using T = std::remove_reference_t<decltype(**p)>;
    off = (off + 255) & ~size_t(255);
    if (base) *p = (T*)(base + off);
    off += std::max<size_t>(n, 1) * sizeof(T);
  };
  const size_t nF = (size_t)key.NY * key.NX, nS = (size_t)key.ny * key.nx;
  const size_t nSpec = (size_t)spec_elems(key.NY, key.NX);
  take(&pl.grad, nF);
  take(&pl.d, nF);
  take(&pl.Af, nS * key.p);
  take(&pl.Ad, nS * key.p);
  take(&pl.Af2, nS * key.p);
  take(&pl.spec, nSpec * key.p);
  take(&pl.khat, nSpec * key.p);
  take(&pl.knyq, (size_t)key.NY * key.p);
  for (int a = 0; a < 2; ++a) {
    take(&pl.tw_row[a], (size_t)key.NX);
    take(&pl.tw_col[a], (size_t)key.NY);
  }
  take(&pl.part, part_capacity(key));
  take(&pl.counter, 1);
  take(&pl.st, 1);
  take(&pl.btab, (size_t)kMaxP);
  return off;
}

// A plan of the same shape made for at least key.nitems items serves: item
// strides do not depend on the item count, and a launch covers only the
// items it is given (the smallest such plan is taken, so repeated batches of
// varying sizes do not pile up workspaces).
static int cached_plan(const PlanKey& key, hipStream_t s, Plan** out) {
  auto it = g_plans.lower_bound(key);
  if (it != g_plans.end()) {
    PlanKey k = it->first;
    k.nitems = key.nitems;
    if (!(k < key) && !(key < k)) {
      *out = it->second.get();
      return 0;
    }
  }
  std::unique_ptr<Plan> pl;
  int rc = make_plan(key, s, pl);
  if (rc) return rc;
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
  p->rl_alpha = 1.0;
  p->f_true = nullptr;
  p->rl_line_search = 0;
  p->rl_lambda_cap = 10.0;
}

static int check_params(const sgp_params& p, int kind) {
  if (p.max_iter < 0) return fail(SGP_E_INVALID_ARG, "max_iter must be >= 0");
  if (p.stop & ~(SGP_STOP_FIXED | SGP_STOP_CONV | SGP_STOP_DISCREPANCY | SGP_STOP_RMSE))
    return fail(SGP_E_INVALID_ARG, "unknown stop bits");
  if ((p.stop & SGP_STOP_RMSE) && !p.f_true)
    return fail(SGP_E_INVALID_ARG, "SGP_STOP_RMSE needs f_true (the true object)");
  if (!(p.tol >= 0)) return fail(SGP_E_INVALID_ARG, "tol must be >= 0");
  if (!(p.disc_target > 0)) return fail(SGP_E_INVALID_ARG, "disc_target must be > 0");
  if (p.init < SGP_INIT_FLAT || p.init > SGP_INIT_WARM) return fail(SGP_E_INVALID_ARG, "unknown init");
  if ((p.init == SGP_INIT_USER || p.init == SGP_INIT_WARM) && !p.f0)
    return fail(SGP_E_INVALID_ARG, "SGP_INIT_USER / SGP_INIT_WARM need f0");
  if (em_kind(kind) && p.init == SGP_INIT_ZERO)
    return fail(SGP_E_INVALID_ARG, "RL / OSEM cannot start from the zero image");
  if (p.rl_line_search) {
    if (kind != KIND_RL) return fail(SGP_E_INVALID_ARG, "rl_line_search (Eq. (RL2)) applies to RL only");
    if (p.rl_alpha != 1.0) return fail(SGP_E_INVALID_ARG, "rl_line_search and rl_alpha != 1 exclude each other");
    if (!(p.rl_lambda_cap >= 1.0 && p.rl_lambda_cap <= 1e6))
      return fail(SGP_E_INVALID_ARG, "rl_lambda_cap must be in [1, 1e6]");
  }
  if (kind == KIND_SGP || p.rl_line_search) {
    if (!(p.beta > 0 && p.beta < 1)) return fail(SGP_E_INVALID_ARG, "beta must be in (0,1)");
    if (!(p.theta > 0 && p.theta < 1)) return fail(SGP_E_INVALID_ARG, "theta must be in (0,1)");
  }
  if (kind == KIND_SGP) {
    if (!(p.alpha_min > 0 && p.alpha_min < p.alpha_max)) return fail(SGP_E_INVALID_ARG, "need 0 < alpha_min < alpha_max");
    if (!(p.alpha0 >= p.alpha_min && p.alpha0 <= p.alpha_max)) return fail(SGP_E_INVALID_ARG, "alpha0 outside [alpha_min, alpha_max]");
    if (!(p.tau1 > 0 && p.tau1 < 1)) return fail(SGP_E_INVALID_ARG, "tau1 must be in (0,1)");
    if (p.m_alpha < 1 || p.m_alpha > 8) return fail(SGP_E_INVALID_ARG, "m_alpha must be in 1..8");
    if (p.n_bb2_only < 0) return fail(SGP_E_INVALID_ARG, "n_bb2_only must be >= 0");
    if (!p.auto_bounds && !(p.L1 > 0 && p.L1 < p.L2)) return fail(SGP_E_INVALID_ARG, "need 0 < L1 < L2");
    if (p.max_backtracks < 0 || p.max_backtracks > kMaxCand - 1)
      return fail(SGP_E_INVALID_ARG, "max_backtracks must be in 0..40");
  }
  if (p.flux_constraint && kind != KIND_SGP) return fail(SGP_E_INVALID_ARG, "the flux constraint applies to SGP only");
  if (!(p.rl_alpha > 0 && p.rl_alpha <= 8)) return fail(SGP_E_INVALID_ARG, "rl_alpha must be in (0, 8]");
  if (p.rl_alpha != 1.0 && kind != KIND_RL) return fail(SGP_E_INVALID_ARG, "rl_alpha (Eq. (RL1)) applies to RL only");
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

// Tile schedule: the workgroup-shape variant of the row and column kernels
// of each FFT length, process-wide (every device is the same part).  A solver
// reads it when it is created and keeps its variants for its lifetime.
constexpr int kTileVariants = 4;  // tile variants per length: bit 0 workgroup shape, bit 1 transform plan
struct TileChoice {
  int row = 0, col = 0;
};
static std::mutex g_tile_mutex;
static std::map<int, TileChoice> g_tile;

static void tile_schedule(int L, int* row, int* col) {
  std::lock_guard<std::mutex> lock(g_tile_mutex);
  auto it = g_tile.find(L);
  const TileChoice c = it == g_tile.end() ? TileChoice{} : it->second;
  if (row) *row = c.row;
  if (col) *col = c.col;
}

static void set_tile_schedule(int L, int row, int col) {
  std::lock_guard<std::mutex> lock(g_tile_mutex);
  g_tile[L] = TileChoice{row, col};
}

// Launch helper; optionally brackets every launch with HIP events.
struct Launcher {
  Args base;
  hipStream_t s = nullptr;
  int NY = 0, NX = 0;
  int vrow = 0, vcol = 0;  // tile variants of the row (length NX) and column (length NY) kernels
  int nz = 1;  // batched items (grid z)
  bool timing = false;
  struct Mark { hipEvent_t a, b; int cls; };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
  size_t used = 0;

  hipEvent_t ev() {
    if (used == pool.size()) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      pool.push_back(e);
    }
    return pool[used++];
  }
  void begin(int cls, hipEvent_t& a) {
    if (timing && cls >= 0) {
      a = ev();
      (void)hipEventRecord(a, s);
    }
  }
  void end(int cls, hipEvent_t a) {
    if (timing && cls >= 0) {
      hipEvent_t b = ev();
      (void)hipEventRecord(b, s);
      marks.push_back({a, b, cls});
    }
  }
  int row_nblk = 0;  // workgroups of the last row launch (its partials)
  // Row kernel.  The iteration ops (row_fin_deferred) leave their reduction
  // partials; fin = true finishes it in a one-workgroup launch, otherwise the
  // next col() / pix() launch must be given the op as fin_op.
  void row(int op, int jc, int iter, int flag = 0, int cls = -1, bool fin = false) {
    Args a = base;
    const int gx = NY / (2 * row_pairs(NX, vrow));
    a.nblk = gx * jc;
    row_nblk = a.nblk;
    a.iter = iter;
    a.flag = flag;
    hipEvent_t e0 = nullptr;
    begin(cls, e0);
    launch_row(NX, vrow, op, dim3(gx, jc, nz), a, s);
    end(cls, e0);
    if (fin) {
      begin(cls >= 0 ? SGP_KCLASS_ROW_FIN : -1, e0);
      launch_row_fin(op, nz, a, s);
      end(cls >= 0 ? SGP_KCLASS_ROW_FIN : -1, e0);
    }
  }
  void col(int mode, int conj, int jc, int iter, int cls = -1, int fin_op = -1) {
    Args a = base;
    const int C = col_width(NY, vcol);
    a.fin_op = fin_op + 1;
    a.fin_nblk = row_nblk;
    a.iter = iter;
    hipEvent_t e0 = nullptr;
    begin(cls, e0);
    launch_col(NY, vcol, mode, conj, dim3((NX / 2 + C - 1) / C, jc, nz), a, s);
    end(cls, e0);
  }
  void pix(int op, long long n, int iter, int jsel = 0, int cls = -1, int fin_op = -1) {
    Args a = base;
    a.fin_op = fin_op + 1;
    a.fin_nblk = row_nblk;
    long long nb = (n + kPixThreads - 1) / kPixThreads;
    // the extra Armijo candidates are rarely needed: a small grid keeps the
    // usual early exit cheap (one workgroup per 2048 pixels of an item, at
    // most kArmBlocks; the same grid per item in single and batched runs,
    // so their sums group alike)
    const long long cap = op == PIX_ARMIJO ? std::min<long long>(kArmBlocks, (n + 2047) / 2048) : kMaxPixBlocks;
    nb = std::max<long long>(1, std::min<long long>(nb, cap));
    a.nblk = (int)nb;
    a.iter = iter;
    a.jsel = jsel;
    hipEvent_t e0 = nullptr;
    begin(cls, e0);
    launch_pix(op, dim3((unsigned)nb, 1, nz), a, s);
    end(cls, e0);
  }
  ~Launcher() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

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
  h.flux_c = p.flux;
  h.norm_disc = 2.0 / ((double)pb.p * (double)pb.ny * (double)pb.nx);
  h.rl_alpha = p.rl_alpha;
  h.alpha = p.alpha0;
  h.tau = p.tau1;
  h.lam = 1.0;
  h.L1 = p.L1;
  h.L2 = p.L2;
  h.k_stop = 0;
  h.rms_k = -1;
  if (p.rl_line_search) {
    // Eq. (RL2) on the SGP iteration: alpha = 1 and D = (M_R / w) o f
    // (bounds 0 and a value no float reaches) make the projected step the
    // RL step, d the RL direction; the candidates come from fin_rl2max
    h.rl2 = 1;
    h.lam_cap = p.rl_lambda_cap;
    h.auto_bounds = 0;
    h.L1p = 0.0;
    h.L2p = 3.0e38;
    h.alpha0 = 1.0;
    h.alpha = 1.0;
  }
}

}  // namespace sgp

// A solver: workspace, problem, parameters, launch state and graph.
struct sgp_solver {
  int kind = 0;
  sgp::Problem pb;
  sgp_params prm{};
  float* f = nullptr;
  hipStream_t user = nullptr;
  hipStream_t s = nullptr;  // internal stream (capturable)
  sgp::Plan* pl = nullptr;
  std::unique_ptr<sgp::Plan> owned;
  sgp::Launcher L;
  // captured iteration blocks, by length: full blocks and the remainder of
  // a step() call each replay a graph of exactly their iteration count
  std::map<int, std::pair<hipGraph_t, hipGraphExec_t>> graphs;
  bool use_graph = true;
  bool done = false;
  int nitems = 1;  // batched problems (same shape), item i's iterate is fs[i]
  std::vector<float*> fs;
  std::chrono::steady_clock::time_point t0;
  double ms[SGP_KCLASS_COUNT] = {0};
  long long cnt[SGP_KCLASS_COUNT] = {0};

  bool own_stream = true;   // false: the per-device stream of the one-shot calls
  bool restored = false;    // the reconstruction-error stop's minimum has been put back into f
  ~sgp_solver() {
    for (auto& kv : graphs) {
      (void)hipGraphExecDestroy(kv.second.second);
      (void)hipGraphDestroy(kv.second.first);
    }
    if (s && own_stream) (void)hipStreamDestroy(s);
  }
};

namespace sgp {

static int read_state(sgp_solver* S) {
  SGP_HIP(hipMemcpyAsync(S->pl->host_st, S->pl->st, sizeof(DevState) * S->nitems, hipMemcpyDeviceToHost, S->s));
  SGP_HIP(hipStreamSynchronize(S->s));
  return 0;
}

static bool all_done(const sgp_solver* S) {
  for (int i = 0; i < S->nitems; ++i)
    if (!S->pl->host_st[i].done) return false;
  return true;
}

// Points the field input of ROW_FIELD / PIX_INITF at the iterate f (or the
// user start) of every item.
static void src_iterate(sgp_solver* S) {
  if (S->nitems > 1) S->L.base.srctab = (const float* const*)S->pl->ftab;
  else S->L.base.src = S->f;
}
static void src_user(sgp_solver* S) {
  if (S->nitems > 1) S->L.base.srctab = S->pl->srctab;
  else S->L.base.src = S->prm.f0;
}

// Newton steps allowed for the flux multiplier per iteration (each exits at
// once after convergence, typically within 4 steps)
constexpr int kFluxNewton = 8;

// one iteration of the solver's loop
static void enqueue_iteration(sgp_solver* S) {
  Launcher& L = S->L;
  const int p = S->pb.p;
  const long long nS = (long long)S->pb.ny * S->pb.nx;
  const long long nF = (long long)S->pb.NY * S->pb.NX;
  // Sect. 3.3 reconstruction-error stop: the iterate before each update is
  // kept, and rho of the new one is tested
  const bool rms = (S->prm.stop & SGP_STOP_RMSE) != 0;
  if (S->kind == KIND_SGP) {
    if (S->prm.flux_constraint) {
      L.pix(PIX_FLUX_INIT, nF, 1, 0, SGP_KCLASS_ROW_DIR);
      for (int t = 0; t < kFluxNewton; ++t) {
        // the last pass counts an iteration whose multiplier is still not at the root
        const int save = L.base.flag;
        L.base.flag = t == kFluxNewton - 1 ? 1 : 0;
        L.pix(PIX_FLUX_NEWTON, nF, 1, 0, SGP_KCLASS_ROW_DIR);
        L.base.flag = save;
      }
    }
    // Eq. (RL2): the step candidates, from the largest keeping f >= 0
    if (S->prm.rl_line_search) L.pix(PIX_RL2MAX, nF, 1);
    // each row kernel's reduction is finished at the start of the next launch
    // (the direction and update sums by the column kernels, the Armijo test by
    // the Armijo kernel), the BB sums by a one-workgroup launch
    L.row(ROW_DIR, 1, 1, 0, SGP_KCLASS_ROW_DIR);
    L.col(COL_CONV, 0, 1, 1, SGP_KCLASS_COL_CONV, ROW_DIR);
    L.row(ROW_AD, p, 1, 0, SGP_KCLASS_ROW_AD);
    L.pix(PIX_ARMIJO, p * nS, 1, 0, SGP_KCLASS_ARMIJO_MORE, ROW_AD);
    L.row(ROW_UPD, p, 1, 0, SGP_KCLASS_ROW_UPD);
    L.col(COL_CORRSUM, 1, 1, 1, SGP_KCLASS_COL_CORR, ROW_UPD);
    if (rms) L.pix(PIX_FCOPY, nF, 1);  // the iterate before f <- f + lambda d
    if (S->prm.rl_line_search) L.pix(PIX_RL2ZERO, nF, 1);
    L.row(ROW_GRAD, 1, 1, 0, SGP_KCLASS_ROW_GRAD, true);
    if (rms) L.pix(PIX_RMSE, nF, 1, 1);
  } else if (S->kind == KIND_RL) {
    L.col(COL_CONV, 0, 1, 1, SGP_KCLASS_COL_CONV);
    L.row(ROW_RATIO, p, 1, 0, SGP_KCLASS_ROW_RATIO);
    L.col(COL_CORRSUM, 1, 1, 1, SGP_KCLASS_COL_CORR);
    if (rms) L.pix(PIX_FCOPY, nF, 1);
    L.row(ROW_RLUPD, 1, 1, 0, SGP_KCLASS_ROW_RLUPD);
    if (rms) L.pix(PIX_RMSE, nF, 1, 0);
  } else {
    // OSEM (Algorithm 2): the KL of f^(k) over all images (the stop rules),
    // whose ratio pass also serves the first sub-step; then for each image j
    // h <- w_j o h o A_j^T (g_j / (A_j h + b_j)), w_j = 1 (periodic) or
    // M_R / alpha_j (Eq. boundaryOSEM)
    L.col(COL_CONV, 0, 1, 1, SGP_KCLASS_COL_CONV);
    L.row(ROW_RATIO, p, 1, 0, SGP_KCLASS_ROW_RATIO);
    const Args save = L.base;
    for (int j = 0; j < p; ++j) {
      L.base.j0 = j;
      L.base.jn = 1;
      if (j > 0) {
        L.col(COL_CONV, 0, 1, 1, SGP_KCLASS_COL_CONV);
        L.row(ROW_RATIO, 1, 1, 4, SGP_KCLASS_ROW_RATIO);
      }
      L.col(COL_CORRSUM, 1, 1, 1, SGP_KCLASS_COL_CORR);
      L.base.j0 = 0;
      L.base.jn = 0;
      if (S->pb.boundary) L.base.invw = S->pl->invwj + (long long)j * nF;
      else L.base.invw_s = 1.0f;
      if (rms && j == 0) L.pix(PIX_FCOPY, nF, 1);  // f^(k) before the first sub-step
      L.row(ROW_RLUPD, 1, 1, 0, SGP_KCLASS_ROW_RLUPD);
      L.base = save;
    }
    if (rms) L.pix(PIX_RMSE, nF, 1, 0);
  }
}

// Setup: validation of data and PSFs, transfer functions, boundary weights,
// start image, and for SGP one RL step giving A_j f0, J(f0), grad J(f0) and
// (L1, L2).
static int setup(sgp_solver* S) {
  Launcher& L = S->L;
  const Problem& pb = S->pb;
  const long long nS = (long long)pb.ny * pb.nx, nF = (long long)pb.NY * pb.NX;
  // the data checks are read back with the rest of the setup (one host
  // synchronisation): on bad data the setup kernels compute non-finite values
  // in bounds, and the call fails before any iteration
  L.pix(PIX_VALIDATE, pb.p * nS, 0);
  for (int j = 0; j < pb.p; ++j) L.pix(PIX_PSFSUM, nF, 0, j);
  SGP_HIP(hipGetLastError());
  int rc;
  // transfer functions K_j / (NY NX): shifted PSF -> row FFT -> column FFT
  L.row(ROW_PSF, pb.p, 0);
  L.col(COL_FWD, 0, pb.p, 0);
  if (pb.boundary) {
    // alpha_j = K_j correlated with M_S, then R and M_R / alpha
    L.row(ROW_MASKS, 1, 0);
    L.col(COL_CONV, 1, 1, 0);
    L.row(ROW_STORE, pb.p, 0);
    Args save = L.base;
    L.base.d = S->pl->invw;
    L.pix(PIX_INVW, nF, 0);
    if (S->kind == KIND_OSEM) {
      L.base.d = S->pl->invwj;
      L.pix(PIX_INVWJ, nF, 0);
    }
    L.base = save;
  }
  const int init = S->prm.init;
  if (init == SGP_INIT_FLAT || init == SGP_INIT_WARM || S->prm.flux_constraint) L.pix(PIX_FLATSUM, pb.p * nS, 0);
  if (init == SGP_INIT_WARM) {
    // J of the flat start (kept aside), then J of the given start; each item
    // keeps the given start only if its KL is not larger
    L.pix(PIX_INITF, nF, 0, INIT_FLAT);
    src_iterate(S);
    L.row(ROW_FIELD, 1, 0);
    L.col(COL_CONV, 0, 1, 0);
    L.row(ROW_RATIO, pb.p, 0, 2);
    src_user(S);
    L.pix(PIX_INITF, nF, 0, INIT_USER);
    src_iterate(S);
    L.row(ROW_FIELD, 1, 0);
    L.col(COL_CONV, 0, 1, 0);
    L.row(ROW_RATIO, pb.p, 0, 0);
    L.pix(PIX_CHOOSE, nF, 0);
  } else {
    src_user(S);
    L.pix(PIX_INITF, nF, 0, init);
  }
  if (S->prm.flux_constraint) {  // the start image is put on the constraint set
    L.pix(PIX_FSUM, nF, 0);
    L.pix(PIX_FSCALE, nF, 0);
  }
  src_iterate(S);
  L.row(ROW_FIELD, 1, 0);
  if (S->kind == KIND_SGP) {
    L.col(COL_CONV, 0, 1, 0);
    L.row(ROW_RATIO, pb.p, 0, 1);
    L.col(COL_CORRSUM, 1, 1, 0);
    L.row(ROW_SETUPGRAD, 1, 0);
  }
  if (S->prm.stop & SGP_STOP_RMSE) L.pix(PIX_RMSE, nF, 0);  // rho^(0)
  SGP_HIP(hipGetLastError());
  if ((rc = read_state(S))) return rc;
  for (int i = 0; i < S->nitems; ++i) {
    const int fl = S->pl->host_st[i].flags;
    const std::string who = S->nitems > 1 ? " (batch item " + std::to_string(i) + ")" : "";
    if (fl & FLAG_BAD_PSF) return fail(SGP_E_BAD_PSF, "PSF has negative or non-finite entries or a non-positive sum" + who);
    if (fl & FLAG_BAD_DATA) return fail(SGP_E_BAD_DATA, "g must be finite and >= 0" + who);
    if (fl & FLAG_BAD_BG) return fail(SGP_E_BAD_DATA, "background map must be finite and >= 0" + who);
  }
  S->done = all_done(S);
  return 0;
}

// The graph of `block` iterations, captured on first use and kept.
static int block_graph(sgp_solver* S, int block, hipGraphExec_t* out) {
  auto it = S->graphs.find(block);
  if (it != S->graphs.end()) {
    *out = it->second.second;
    return 0;
  }
  SGP_HIP(hipStreamBeginCapture(S->s, hipStreamCaptureModeThreadLocal));
  for (int b = 0; b < block; ++b) enqueue_iteration(S);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(S->s, &g);
  if (e != hipSuccess) return fail(SGP_E_HIP, std::string("graph capture: ") + hipGetErrorString(e));
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    return fail(SGP_E_HIP, std::string("graph instantiation: ") + hipGetErrorString(e));
  }
  S->graphs[block] = {g, x};
  *out = x;
  return 0;
}

// Iterations of a step(n) call and how they are replayed: blocks of 32 (16
// with an early stop rule, so that the state is read often enough), then
// one block of the remainder.
struct StepPlan {
  int iters, block, full, rem;
  bool early;
};
static StepPlan step_plan(const sgp_solver* S, int n) {
  StepPlan p;
  p.early = (S->prm.stop & (SGP_STOP_CONV | SGP_STOP_DISCREPANCY | SGP_STOP_RMSE)) != 0;
  p.iters = em_kind(S->kind) ? n + 1 : n;  // RL / OSEM evaluate J once more before pausing
  p.block = std::min(p.iters, p.early ? 16 : 32);
  p.full = p.block > 0 ? p.iters / p.block : 0;
  p.rem = p.block > 0 ? p.iters % p.block : 0;
  return p;
}

// Captures the graphs a later step(n) call replays, so that no capture falls
// inside that call.
static int prepare(sgp_solver* S, int n) {
  if (n < 0) return fail(SGP_E_INVALID_ARG, "n must be >= 0");
  const StepPlan p = step_plan(S, n);
  if (!S->use_graph || p.iters == 0) return 0;
  hipGraphExec_t x;
  int rc;
  if ((rc = block_graph(S, p.block, &x))) return rc;
  if (p.rem && (rc = block_graph(S, p.rem, &x))) return rc;
  return 0;
}

static int step(sgp_solver* S, int n, int* done_out) {
  if (n < 0) return fail(SGP_E_INVALID_ARG, "n must be >= 0");
  int rc;
  if (S->done || n == 0) {
    if (done_out) *done_out = S->done ? 1 : 0;
    return 0;
  }
  launch_resume(S->pl->st, n, S->nitems, S->s);
  if (em_kind(S->kind)) {
    // the spectrum of f is rebuilt so a resumed RL / OSEM call starts from f
    src_iterate(S);
    S->L.row(ROW_FIELD, 1, 0);
  }
  const StepPlan sp = step_plan(S, n);
  const bool early = sp.early;
  const int iters = sp.iters;
  if (S->L.timing || !S->use_graph) {
    for (int it = 0; it < iters; ++it) {
      enqueue_iteration(S);
      if (early && (it % 16) == 15) {
        if ((rc = read_state(S))) return rc;
        if (all_done(S)) break;
      }
    }
    SGP_HIP(hipGetLastError());
    SGP_HIP(hipStreamSynchronize(S->s));
    for (auto& m : S->L.marks) {
      float t = 0;
      SGP_HIP(hipEventElapsedTime(&t, m.a, m.b));
      S->ms[m.cls] += t;
      S->cnt[m.cls] += 1;
    }
    S->L.marks.clear();
    S->L.used = 0;
  } else {
    // a run with an early stop replays blocks of 16 iterations and reads the
    // state after each of the first four (a short run then ends with no
    // replay of iterations that only exit), later after every second one
    hipGraphExec_t gfull = nullptr, grem = nullptr;
    if ((rc = block_graph(S, sp.block, &gfull))) return rc;
    if (sp.rem && (rc = block_graph(S, sp.rem, &grem))) return rc;
    const int reps = sp.full + (sp.rem ? 1 : 0);
    for (int r = 0; r < reps; ++r) {
      SGP_HIP(hipGraphLaunch(r < sp.full ? gfull : grem, S->s));
      if (early && r + 1 < reps && (r < 4 || (r % 2) == 1)) {
        if ((rc = read_state(S))) return rc;
        if (all_done(S)) break;
      }
    }
  }
  if ((rc = read_state(S))) return rc;
  S->done = all_done(S);
  // Sect. 3.3: a run stopped past the minimum of the reconstruction error
  // returns the iterate kept before the last update (one problem per solver)
  if (S->done && !S->restored && S->pl->host_st[0].rms_back) {
    SGP_HIP(hipMemcpyAsync(S->f, S->pl->d, sizeof(float) * (size_t)S->pb.NY * S->pb.NX, hipMemcpyDeviceToDevice,
                           S->s));
    SGP_HIP(hipStreamSynchronize(S->s));
    S->restored = true;
  }
  if (done_out) *done_out = S->done ? 1 : 0;
  return 0;
}

static int item_code(const sgp_solver* S, const DevState& h) {
  int code = SGP_OK;
  if (h.done) {
    switch (h.reason) {
      case REASON_NUMERIC: return fail(SGP_E_NUMERIC, "non-finite value during the iteration");
      case REASON_ARMIJO: code = SGP_W_ARMIJO_EXHAUSTED; break;
      case REASON_STATIONARY: code = SGP_W_STATIONARY; break;
      case REASON_MAXITER:
        code = (S->prm.stop & (SGP_STOP_CONV | SGP_STOP_DISCREPANCY)) ? SGP_W_MAXITER : SGP_OK;
        break;
      default: break;
    }
  }
  if (h.flux_unconv > 0) code = std::max(code, (int)SGP_W_FLUX_UNCONVERGED);
  return code;
}

static void fill_report(const sgp_solver* S, const DevState& h, sgp_report* rep) {
  rep->iters = h.k;
  rep->stop_reason = h.reason;
  rep->backtracks = h.total_back;
  rep->used_fallback = h.used_fallback;
  rep->kl = h.J;
  rep->discrepancy = h.norm_disc * h.J;
  rep->flux = h.fsum;
  rep->L1 = h.L1;
  rep->L2 = h.L2;
  rep->flux_unconverged = h.flux_unconv;
  rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - S->t0).count();
}

// Fills reps[0..nitems) and returns the most severe item code (errors first,
// then the largest warning).
static int report(sgp_solver* S, sgp_report* rep) {
  int rc;
  S->L.pix(PIX_FSUM, (long long)S->pb.NY * S->pb.NX, 0);
  if ((rc = read_state(S))) return rc;
  if (S->prm.trace && S->pl->trace) {
    SGP_HIP(hipMemcpy(S->prm.trace, S->pl->trace,
                      sizeof(double) * kTraceCols * (size_t)(S->prm.max_iter + 1), hipMemcpyDeviceToHost));
  }
  int worst = SGP_OK;
  for (int i = 0; i < S->nitems; ++i) {
    const DevState& h = S->pl->host_st[i];
    if (rep) fill_report(S, h, rep + i);
    const int c = item_code(S, h);
    if (c < 0 ? (worst >= 0 || c < worst) : (worst >= 0 && c > worst)) worst = c;
  }
  return worst;
}

static int to_problem(const sgp_problem* pr, Problem& pb) {
  if (!pr) return fail(SGP_E_INVALID_ARG, "null problem");
  if (pr->p < 1 || pr->p > kMaxP) return fail(SGP_E_INVALID_ARG, "p must be in 1..8");
  if (!pr->b_map && !pr->b_const) return fail(SGP_E_INVALID_ARG, "need b_map or b_const");
  pb.g = pr->g; pb.psf = pr->psf; pb.bmap = pr->b_map;
  for (int j = 0; j < pr->p; ++j) pb.b[j] = pr->b_const ? pr->b_const[j] : 0.f;
  pb.p = pr->p; pb.ny = pr->ny; pb.nx = pr->nx;
  pb.boundary = pr->boundary != 0;
  if (pb.boundary) {
    pb.NY = pr->NY; pb.NX = pr->NX; pb.oy = pr->oy; pb.ox = pr->ox;
  } else {
    pb.NY = pr->ny; pb.NX = pr->nx; pb.oy = pb.ox = 0;
  }
  return 0;
}

// Builds a solver for one problem or for a batch of problems of one shape
// (item i: problem items[i], iterate fs[i], start f0s[i]).  With `cached` the
// workspace comes from the per-shape cache (one-shot calls, serialised by the
// caller), otherwise the solver owns it.
static int create_items(int kind, const std::vector<Problem>& items, const std::vector<float*>& fs,
                        const std::vector<const float*>& f0s, const sgp_params* prm_in, void* stream,
                        bool cached, std::unique_ptr<sgp_solver>& out, bool shared = false,
                        Plan* ext = nullptr) {
  auto S = std::make_unique<sgp_solver>();
  S->t0 = std::chrono::steady_clock::now();
  if (prm_in) S->prm = *prm_in;
  else defaults(&S->prm);
  int rc;
  const int n = (int)items.size();
  if (n < 1) return fail(SGP_E_INVALID_ARG, "no problem given");
  for (int i = 0; i < n; ++i)
    if (!fs[i]) return fail(SGP_E_INVALID_ARG, "f must be non-null");
  if (kind != KIND_RL && kind != KIND_SGP && kind != KIND_OSEM) return fail(SGP_E_INVALID_ARG, "unknown solver kind");
  for (const Problem& q : items)
    if ((rc = check_problem(q))) return rc;
  if (n > 1) {
    if ((S->prm.init == SGP_INIT_USER || S->prm.init == SGP_INIT_WARM))
      for (int i = 0; i < n; ++i)
        if (!f0s[i]) return fail(SGP_E_INVALID_ARG, "SGP_INIT_USER / SGP_INIT_WARM need a start for every item");
    S->prm.trace = nullptr;  // no per-iteration trace for batches
    if (S->prm.stop & SGP_STOP_RMSE)
      return fail(SGP_E_INVALID_ARG, "SGP_STOP_RMSE takes one problem (one true object), not a batch");
    if (S->prm.f0 == nullptr && (S->prm.init == SGP_INIT_USER || S->prm.init == SGP_INIT_WARM))
      S->prm.f0 = f0s[0];
  }
  if ((rc = check_params(S->prm, kind))) return rc;
  // the linear relaxation of RL (Eq. (RL2)) runs the SGP iteration (see fill_state)
  if (kind == KIND_RL && S->prm.rl_line_search) kind = KIND_SGP;
  int dev;
  if ((rc = current_device(&dev))) return rc;
  const Problem& pb = items[0];
  S->kind = kind;
  S->pb = pb;
  S->f = fs[0];
  S->nitems = n;
  S->fs = fs;
  S->user = (hipStream_t)stream;
  // order the internal stream after the caller's stream
  if (ext) {  // the static workspace: every launch goes on the caller's stream
    S->s = S->user;
    S->own_stream = false;
  } else if (shared) {
    SharedStream* ss;
    if ((rc = shared_stream(dev, &ss))) return rc;
    S->s = ss->s;
    S->own_stream = false;
    SGP_HIP(hipEventRecord(ss->e, S->user));
    SGP_HIP(hipStreamWaitEvent(S->s, ss->e, 0));
  } else {
    SGP_HIP(hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking));
    hipEvent_t e;
    SGP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    SGP_HIP(hipEventRecord(e, S->user));
    SGP_HIP(hipStreamWaitEvent(S->s, e, 0));
    SGP_HIP(hipEventDestroy(e));
  }
  PlanKey key{kind, pb.p, pb.NY, pb.NX, pb.ny, pb.nx, pb.oy, pb.ox, pb.boundary ? 1 : 0, dev};
  key.nitems = n;
  if (ext) {
    S->pl = ext;
  } else if (cached) {
    if ((rc = cached_plan(key, S->s, &S->pl))) return rc;
  } else {
    if ((rc = make_plan(key, S->s, S->owned))) return rc;
    S->pl = S->owned.get();
  }
  Plan* pl = S->pl;
  if (S->prm.trace) {
    const int rows = S->prm.max_iter + 1;
    if (pl->trace_rows < rows) {
      if (pl->trace) (void)hipFree(pl->trace);
      pl->trace = nullptr;
      pl->trace_rows = 0;
      if ((rc = dalloc(&pl->trace, (size_t)rows * kTraceCols))) return rc;
      pl->trace_rows = rows;
    }
    SGP_HIP(hipMemsetAsync(pl->trace, 0, sizeof(double) * kTraceCols * rows, S->s));
  }
  for (int i = 0; i < n; ++i) fill_state(pl->host_st[i], S->prm, items[i], S->prm.trace ? pl->trace : nullptr);
  SGP_HIP(hipMemcpyAsync(pl->st, pl->host_st, sizeof(DevState) * n, hipMemcpyHostToDevice, S->s));

  Launcher& L = S->L;
  std::memset(&L.base, 0, sizeof(L.base));
  Args& a = L.base;
  a.NY = pb.NY; a.NX = pb.NX; a.ny = pb.ny; a.nx = pb.nx; a.oy = pb.oy; a.ox = pb.ox; a.p = pb.p;
  a.g = pb.g; a.bmap = pb.bmap;
  a.f = fs[0]; a.grad = pl->grad; a.d = pl->d;
  a.invw = pb.boundary ? pl->invw : nullptr;
  a.invw_s = 1.0f / (float)pb.p;
  a.Af = pl->Af; a.Af2 = pl->Af2; a.Ad = pl->Ad; a.spec = pl->spec; a.khat = pl->khat; a.knyq = pl->knyq;
  a.psf = pb.psf; a.aux = pl->aux; a.src = S->prm.f0;
  a.ftrue = (S->prm.stop & SGP_STOP_RMSE) ? S->prm.f_true : nullptr;
  a.part = pl->part; a.counter = pl->counter; a.st = pl->st;
  a.bvec = pl->btab;
  if (n == 1) SGP_HIP(hipMemcpy(pl->btab, pb.b, sizeof(float) * pb.p, hipMemcpyHostToDevice));
  if (n > 1) {
    std::vector<const float*> gt(n), pt(n), st0(n);
    std::vector<float> bt(n);
    for (int i = 0; i < n; ++i) {
      gt[i] = items[i].g;
      pt[i] = items[i].psf;
      st0[i] = f0s.empty() ? nullptr : f0s[i];
      bt[i] = items[i].b[0];
    }
    SGP_HIP(hipMemcpy(pl->gtab, gt.data(), sizeof(float*) * n, hipMemcpyHostToDevice));
    SGP_HIP(hipMemcpy(pl->ftab, fs.data(), sizeof(float*) * n, hipMemcpyHostToDevice));
    SGP_HIP(hipMemcpy(pl->psftab, pt.data(), sizeof(float*) * n, hipMemcpyHostToDevice));
    SGP_HIP(hipMemcpy(pl->srctab, st0.data(), sizeof(float*) * n, hipMemcpyHostToDevice));
    SGP_HIP(hipMemcpy(pl->btab, bt.data(), sizeof(float) * n, hipMemcpyHostToDevice));
    a.nbatch = n;
    a.gtab = pl->gtab;
    a.ftab = pl->ftab;
    a.psftab = pl->psftab;
    a.srctab = pl->srctab;
    PlanKey k1 = key;
    k1.nitems = 1;
    a.item_field = (long long)pb.NY * pb.NX;
    a.item_obs = (long long)pb.p * pb.ny * pb.nx;
    a.item_spec = (long long)pb.p * spec_elems(pb.NY, pb.NX);
    a.item_nyq = (long long)pb.p * pb.NY;
    a.item_part = (long long)part_capacity(k1);
  }
  L.s = S->s; L.NY = pb.NY; L.NX = pb.NX; L.nz = n;
  tile_schedule(pb.NX, &L.vrow, nullptr);
  tile_schedule(pb.NY, nullptr, &L.vcol);
  a.tw_row = pl->tw_row[plan_of(pb.NX, L.vrow)];  // the tables of the transform plans the variants run
  a.tw_col = pl->tw_col[plan_of(pb.NY, L.vcol)];
  if ((rc = setup(S.get()))) return rc;
  out = std::move(S);
  return 0;
}

static int create(int kind, const Problem& pb, const sgp_params* prm_in, float* f, void* stream, bool cached,
                  std::unique_ptr<sgp_solver>& out, bool shared = false) {
  return create_items(kind, std::vector<Problem>{pb}, std::vector<float*>{f},
                      std::vector<const float*>{prm_in ? prm_in->f0 : nullptr}, prm_in, stream, cached, out,
                      shared);
}

// Many problems in one run: problems are grouped by shape, each group is one
// batched solver (every kernel launch covers all its items, grid z = item),
// and the groups advance together: one HIP graph holds a block of iterations
// of every group as parallel branches and is replayed until every item has
// met its stop rule.
static int batch_run(int kind, const sgp_problem* probs, int n, float* const* fout, const float* const* f0s,
                     const sgp_params* prm, sgp_report* reps, void* stream) {
  if (!probs || n < 1 || !fout) return fail(SGP_E_INVALID_ARG, "need n >= 1 problems and outputs");
  std::map<std::array<int, 7>, std::vector<int>> groups;  // by shape: ny, nx, NY, NX, oy, ox, boundary
  std::vector<Problem> all(n);
  int rc;
  for (int i = 0; i < n; ++i) {
    if ((rc = to_problem(&probs[i], all[i]))) return rc;
    if (all[i].p != 1 || all[i].bmap)
      return fail(SGP_E_INVALID_ARG, "batched problems must be single images with constant background");
    const Problem& q = all[i];
    groups[{q.ny, q.nx, q.NY, q.NX, q.oy, q.ox, q.boundary}].push_back(i);
  }
  std::lock_guard<std::mutex> lock(g_mutex);
  std::vector<std::unique_ptr<sgp_solver>> sol;
  std::vector<std::vector<int>> idx;
  for (auto& kv : groups) {
    std::vector<Problem> items;
    std::vector<float*> fs;
    std::vector<const float*> f0v;
    for (int i : kv.second) {
      items.push_back(all[i]);
      fs.push_back(fout[i]);
      f0v.push_back(f0s ? f0s[i] : nullptr);
    }
    std::unique_ptr<sgp_solver> S;
    if ((rc = create_items(kind, items, fs, f0v, prm, stream, true, S))) return rc;
    sol.push_back(std::move(S));
    idx.push_back(kv.second);
  }
  const int max_iter = sol[0]->prm.max_iter;
  const int iters = em_kind(kind) ? max_iter + 1 : max_iter;
  hipStream_t s0 = sol[0]->s;
  for (auto& S : sol) launch_resume(S->pl->st, max_iter, S->nitems, S->s);
  // the first group's stream carries the graph; the others fork from it
  std::vector<hipEvent_t> ev(2 * sol.size());
  for (auto& e : ev) SGP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  for (size_t c = 1; c < sol.size(); ++c) {  // setup and resume of every group precede the graph
    SGP_HIP(hipEventRecord(ev[c], sol[c]->s));
    SGP_HIP(hipStreamWaitEvent(s0, ev[c], 0));
  }
  const int block = std::min(iters, 16);
  const size_t ng = sol.size();
  std::vector<char> live(ng, 1);  // groups with items still running
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
  auto drop_graph = [&]() {
    if (ge) (void)hipGraphExecDestroy(ge);
    if (g) (void)hipGraphDestroy(g);
    ge = nullptr;
    g = nullptr;
  };
  // one block of iterations of every live group, as parallel branches
  auto capture = [&]() -> int {
    drop_graph();
    SGP_HIP(hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal));
    SGP_HIP(hipEventRecord(ev[0], s0));
    for (size_t c = 1; c < ng; ++c)
      if (live[c]) SGP_HIP(hipStreamWaitEvent(sol[c]->s, ev[0], 0));
    for (size_t c = 0; c < ng; ++c)
      if (live[c])
        for (int b = 0; b < block; ++b) enqueue_iteration(sol[c].get());
    for (size_t c = 1; c < ng; ++c)
      if (live[c]) {
        SGP_HIP(hipEventRecord(ev[ng + c], sol[c]->s));
        SGP_HIP(hipStreamWaitEvent(s0, ev[ng + c], 0));
      }
    hipError_t ce = hipStreamEndCapture(s0, &g);
    if (ce != hipSuccess) return fail(SGP_E_HIP, std::string("graph capture: ") + hipGetErrorString(ce));
    SGP_HIP(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
    return 0;
  };
  if ((rc = capture())) return rc;
  const int reps_n = (iters + block - 1) / block;
  std::vector<int> act;
  for (int r = 0; r < reps_n; ++r) {
    SGP_HIP(hipGraphLaunch(ge, s0));
    if (r % 4 == 3 || r + 1 == reps_n) {  // stop once every item has stopped
      SGP_HIP(hipStreamSynchronize(s0));
      bool done = true, recapture = false;
      for (size_t c = 0; c < ng; ++c) {
        if (!live[c]) continue;
        sgp_solver* S = sol[c].get();
        if ((rc = read_state(S))) return rc;
        act.clear();
        for (int i = 0; i < S->nitems; ++i)
          if (!S->pl->host_st[i].done) act.push_back(i);
        if (act.empty()) {
          live[c] = 0;
          recapture = true;
          continue;
        }
        done = false;
        // once half of a group's launch covers stopped items, launch over the
        // running ones only (grid z through the slice map)
        if (S->nitems > 1 && 2 * (int)act.size() <= S->L.nz) {
          SGP_HIP(hipMemcpy(S->pl->zmap, act.data(), sizeof(int) * act.size(), hipMemcpyHostToDevice));
          S->L.base.zmap = S->pl->zmap;
          S->L.nz = (int)act.size();
          recapture = true;
        }
      }
      if (done) break;
      if (recapture && r + 1 < reps_n && (rc = capture())) return rc;
    }
  }
  SGP_HIP(hipStreamSynchronize(s0));
  drop_graph();
  for (auto& e : ev) (void)hipEventDestroy(e);
  for (auto& S : sol) {  // reports see every item again
    S->L.base.zmap = nullptr;
    S->L.nz = S->nitems;
  }
  int worst = SGP_OK;
  std::vector<sgp_report> tmp;
  for (size_t c = 0; c < sol.size(); ++c) {
    tmp.resize(sol[c]->nitems);
    const int code = report(sol[c].get(), tmp.data());
    if (code < 0 ? (worst >= 0 || code < worst) : (worst >= 0 && code > worst)) worst = code;
    if (reps)
      for (int t = 0; t < sol[c]->nitems; ++t) reps[idx[c][t]] = tmp[t];
  }
  return worst;
}

static int one_shot(int kind, const Problem& pb, const sgp_params* prm, float* f, sgp_report* rep, void* stream) {
  std::lock_guard<std::mutex> lock(g_mutex);
  std::unique_ptr<sgp_solver> S;
  int rc = create(kind, pb, prm, f, stream, true, S, true);
  if (rc) return rc;
  const int n = S->prm.max_iter;
  if ((rc = step(S.get(), n, nullptr))) return rc;
  return report(S.get(), rep);
}

// sgp_deconv on the static workspace: no device or pinned-host allocation,
// no graph (every iteration is launched on the caller's stream), no
// internal stream.
static int deconv_noalloc(const float* g, const float* psf, const float* b_map, float b_const, int ny, int nx,
                          const sgp_params* prm, float* f, sgp_report* rep, void* stream) {
  Problem pb;
  pb.g = g; pb.psf = psf; pb.bmap = b_map; pb.b[0] = b_const;
  pb.p = 1; pb.ny = pb.NY = ny; pb.nx = pb.NX = nx;
  int rc;
  if ((rc = check_problem(pb))) return rc;
  if (prm && prm->trace) return fail(SGP_E_INVALID_ARG, "sgp_deconv_noalloc keeps no trace (prm->trace must be NULL)");
  int dev;
  if ((rc = current_device(&dev))) return rc;
  PlanKey key{KIND_SGP, 1, ny, nx, ny, nx, 0, 0, 0, dev};
  Plan sizing;
  sizing.external = true;
  const size_t need = carve_plan(key, nullptr, sizing);
  if (need > kScratchBytes)
    return fail(SGP_E_INVALID_ARG, "a " + std::to_string(ny) + " x " + std::to_string(nx) + " problem needs " +
                                       std::to_string((need + (1 << 20) - 1) >> 20) + " MiB of workspace; the static "
                                       "workspace of sgp_deconv_noalloc holds " +
                                       std::to_string(kScratchBytes >> 20) + " MiB (about 2 million pixels)");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  char* base = nullptr;
  if ((rc = scratch_address(dev, &base))) return rc;
  Plan pl;
  pl.external = true;
  pl.key = key;
  carve_plan(key, base, pl);
  DevState host_state;
  pl.host_st = &host_state;
  hipStream_t s = (hipStream_t)stream;
  // the workspace keeps the previous call's contents: the reduction counter
  // must start at zero (every other buffer is written before it is read);
  // cleared by a fill kernel, so the call records no memset node
  launch_zero(pl.counter, 1, s);
  for (int a = 0; a < 2; ++a) {
    launch_twiddle(pl.tw_row[a], nx, a, s);
    launch_twiddle(pl.tw_col[a], ny, a, s);
  }
  SGP_HIP(hipGetLastError());
  std::unique_ptr<sgp_solver> S;
  rc = create_items(KIND_SGP, std::vector<Problem>{pb}, std::vector<float*>{f},
                    std::vector<const float*>{prm ? prm->f0 : nullptr}, prm, stream, false, S, false, &pl);
  if (rc) return rc;
  S->use_graph = false;
  if ((rc = step(S.get(), S->prm.max_iter, nullptr))) return rc;
  rc = report(S.get(), rep);
  S->pl = nullptr;
  return rc;
}

static int apply_operator(const float* psf, const float* x, int ny, int nx, int adjoint, float* out,
                          void* stream) {
  if (!psf || !x || !out) return fail(SGP_E_INVALID_ARG, "null pointer");
  Problem pb;
  pb.g = x;
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
  if ((rc = cached_plan(key, s, &pl))) return rc;
  sgp_params prm;
  defaults(&prm);
  fill_state(*pl->host_st, prm, pb, nullptr);
  SGP_HIP(hipMemcpyAsync(pl->st, pl->host_st, sizeof(DevState), hipMemcpyHostToDevice, s));
  Launcher L;
  std::memset(&L.base, 0, sizeof(L.base));
  Args& a = L.base;
  a.NY = ny; a.NX = nx; a.ny = ny; a.nx = nx; a.p = 1;
  a.psf = psf; a.spec = pl->spec; a.khat = pl->khat; a.knyq = pl->knyq; a.aux = pl->aux;
  a.part = pl->part; a.counter = pl->counter; a.st = pl->st;
  a.invw_s = 1.f;
  L.s = s; L.NY = ny; L.NX = nx;
  tile_schedule(nx, &L.vrow, nullptr);
  tile_schedule(ny, nullptr, &L.vcol);
  a.tw_row = pl->tw_row[plan_of(nx, L.vrow)];
  a.tw_col = pl->tw_col[plan_of(ny, L.vcol)];
  L.pix(PIX_PSFSUM, (long long)ny * nx, 0, 0);
  SGP_HIP(hipMemcpyAsync(pl->host_st, pl->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  SGP_HIP(hipStreamSynchronize(s));
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

extern "C" {

int sgp_params_init(sgp_params* p) {
  if (!p) return fail(SGP_E_INVALID_ARG, "null params");
  defaults(p);
  return SGP_OK;
}

// Mosaic of boundary-corrected subdomains: every core x core tile of the
// image is reconstructed from a window extended by `margin` pixels towards its
// neighbours (clipped at the image edge), placed at the centre of an N x N
// FFT domain; all windows run as one batch and the cores are stitched.
static int mosaic_run(int kind, const float* g, int H, int W, const float* psf, int N, float b, int core,
                      int margin, const sgp_params* prm, float* f, sgp_report* rep, void* stream) {
  if (!g || !psf || !f) return fail(SGP_E_INVALID_ARG, "null pointer");
  if (prm && (prm->stop & SGP_STOP_RMSE))
    return fail(SGP_E_INVALID_ARG, "SGP_STOP_RMSE takes one problem (one true object), not a mosaic");
  if (core < 1 || margin < 0 || H < core || W < core || H % core || W % core)
    return fail(SGP_E_INVALID_ARG, "H and W must be positive multiples of core, margin >= 0");
  if (core + 2 * margin > N) return fail(SGP_E_INVALID_ARG, "a window (core + 2 margin) must fit in N");
  if (!size_supported(N)) return fail(SGP_E_UNSUPPORTED_SIZE, "unsupported FFT size N");
  if (!(b >= 0) || !std::isfinite(b)) return fail(SGP_E_BAD_DATA, "background must be finite and >= 0");
  hipStream_t s = (hipStream_t)stream;
  struct Tile { int cy, cx, y0, y1, x0, x1, oy, ox; };
  std::vector<Tile> tiles;
  for (int i = 0; i < H / core; ++i)
    for (int j = 0; j < W / core; ++j) {
      Tile t;
      t.cy = i * core;
      t.cx = j * core;
      t.y0 = std::max(0, t.cy - margin);
      t.y1 = std::min(H, t.cy + core + margin);
      t.x0 = std::max(0, t.cx - margin);
      t.x1 = std::min(W, t.cx + core + margin);
      t.oy = (N - (t.y1 - t.y0)) / 2;
      t.ox = (N - (t.x1 - t.x0)) / 2;
      tiles.push_back(t);
    }
  const int n = (int)tiles.size();
  // staging: the windows (contiguous) and the per-tile iterates on N x N
  size_t gtot = 0;
  std::vector<size_t> goff(n);
  for (int t = 0; t < n; ++t) {
    goff[t] = gtot;
    gtot += (size_t)(tiles[t].y1 - tiles[t].y0) * (tiles[t].x1 - tiles[t].x0);
  }
  float* gst = nullptr;
  float* fst = nullptr;
  int rc = 0;
  if ((rc = dalloc(&gst, gtot))) return rc;
  if ((rc = dalloc(&fst, (size_t)n * N * N))) {
    (void)hipFree(gst);
    return rc;
  }
  std::vector<sgp_problem> probs(n);
  std::vector<float*> fp(n);
  std::vector<sgp_report> reps(n);
  const float bc[1] = {b};
  hipError_t e = hipSuccess;
  for (int t = 0; t < n && e == hipSuccess; ++t) {
    const Tile& q = tiles[t];
    const int wy = q.y1 - q.y0, wx = q.x1 - q.x0;
    e = hipMemcpy2DAsync(gst + goff[t], sizeof(float) * wx, g + (size_t)q.y0 * W + q.x0, sizeof(float) * W,
                         sizeof(float) * wx, wy, hipMemcpyDeviceToDevice, s);
    sgp_problem& pr = probs[t];
    pr.g = gst + goff[t];
    pr.psf = psf;
    pr.b_map = nullptr;
    pr.b_const = bc;
    pr.p = 1;
    pr.ny = wy;
    pr.nx = wx;
    pr.NY = N;
    pr.NX = N;
    pr.oy = q.oy;
    pr.ox = q.ox;
    pr.boundary = 1;
    fp[t] = fst + (size_t)t * N * N;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) rc = fail(SGP_E_HIP, std::string("window copy: ") + hipGetErrorString(e));
  if (!rc) rc = batch_run(kind, probs.data(), n, fp.data(), nullptr, prm, reps.data(), stream);
  if (rc >= 0) {
    for (int t = 0; t < n && e == hipSuccess; ++t) {
      const Tile& q = tiles[t];
      const int ry = q.oy + (q.cy - q.y0), rx = q.ox + (q.cx - q.x0);
      e = hipMemcpy2DAsync(f + (size_t)q.cy * W + q.cx, sizeof(float) * W, fp[t] + (size_t)ry * N + rx,
                           sizeof(float) * N, sizeof(float) * core, core, hipMemcpyDeviceToDevice, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) rc = fail(SGP_E_HIP, std::string("stitching: ") + hipGetErrorString(e));
  }
  if (rep && rc >= 0) {
    // the tile that ran longest gives iters and stop_reason; KL values and
    // backtracks are summed over the tiles (windows overlap), the
    // discrepancy is the largest of the tiles'
    sgp_report r{};
    for (int t = 0; t < n; ++t) {
      if (t == 0 || reps[t].iters > r.iters) {
        r.iters = reps[t].iters;
        r.stop_reason = reps[t].stop_reason;
      }
      r.backtracks += reps[t].backtracks;
      r.used_fallback += reps[t].used_fallback;
      r.kl += reps[t].kl;
      r.discrepancy = std::max(r.discrepancy, reps[t].discrepancy);
      r.seconds = std::max(r.seconds, reps[t].seconds);
    }
    r.L1 = reps[0].L1;
    r.L2 = reps[0].L2;
    *rep = r;
  }
  (void)hipFree(gst);
  (void)hipFree(fst);
  return rc;
}

#define SGP_GUARD(expr)                                      \
  try {                                                      \
    return (expr);                                           \
  } catch (...) {                                            \
    return fail(SGP_E_HIP, "internal error");                \
  }

static int single(int kind, const float* g, const float* psf, const float* b_map, float b_const, int ny,
                  int nx, const sgp_params* prm, float* f, sgp_report* rep, void* stream) {
  Problem pb;
  pb.g = g; pb.psf = psf; pb.bmap = b_map; pb.b[0] = b_const;
  pb.p = 1; pb.ny = pb.NY = ny; pb.nx = pb.NX = nx;
  return one_shot(kind, pb, prm, f, rep, stream);
}

int rl_deconv(const float* g, const float* psf, const float* b_map, float b_const, int ny, int nx,
              const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream) {
  SGP_GUARD(single(KIND_RL, g, psf, b_map, b_const, ny, nx, prm, f, rep, hip_stream));
}

int sgp_deconv(const float* g, const float* psf, const float* b_map, float b_const, int ny, int nx,
               const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream) {
  SGP_GUARD(single(KIND_SGP, g, psf, b_map, b_const, ny, nx, prm, f, rep, hip_stream));
}

static int stack(int kind, const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                 int ny, int nx, int NY, int NX, int oy, int ox, int boundary, const sgp_params* prm, float* f,
                 sgp_report* rep, void* stream) {
  sgp_problem pr{g, psf, b_map, b_const, p, ny, nx, NY, NX, oy, ox, boundary};
  Problem pb;
  int rc = to_problem(&pr, pb);
  if (rc) return rc;
  return one_shot(kind, pb, prm, f, rep, stream);
}

int sgp_deconv_noalloc(const float* g, const float* psf, const float* b_map, float b_const, int ny, int nx,
                       const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream) {
  SGP_GUARD(deconv_noalloc(g, psf, b_map, b_const, ny, nx, prm, f, rep, hip_stream));
}

int sgp_multi_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                     int ny, int nx, const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream) {
  SGP_GUARD(stack(KIND_SGP, g, psf, b_map, b_const, p, ny, nx, ny, nx, 0, 0, 0, prm, f, rep, hip_stream));
}

int rl_multi_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                    int ny, int nx, const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream) {
  SGP_GUARD(stack(KIND_RL, g, psf, b_map, b_const, p, ny, nx, ny, nx, 0, 0, 0, prm, f, rep, hip_stream));
}

int sgp_boundary_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                        int ny, int nx, int NY, int NX, int oy, int ox, const sgp_params* prm, float* f,
                        sgp_report* rep, void* hip_stream) {
  SGP_GUARD(stack(KIND_SGP, g, psf, b_map, b_const, p, ny, nx, NY, NX, oy, ox, 1, prm, f, rep, hip_stream));
}

int rl_boundary_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                       int ny, int nx, int NY, int NX, int oy, int ox, const sgp_params* prm, float* f,
                       sgp_report* rep, void* hip_stream) {
  SGP_GUARD(stack(KIND_RL, g, psf, b_map, b_const, p, ny, nx, NY, NX, oy, ox, 1, prm, f, rep, hip_stream));
}

int osem_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p, int ny,
                int nx, const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream) {
  SGP_GUARD(stack(KIND_OSEM, g, psf, b_map, b_const, p, ny, nx, ny, nx, 0, 0, 0, prm, f, rep, hip_stream));
}

int osem_boundary_deconv(const float* g, const float* psf, const float* b_map, const float* b_const, int p,
                         int ny, int nx, int NY, int NX, int oy, int ox, const sgp_params* prm, float* f,
                         sgp_report* rep, void* hip_stream) {
  SGP_GUARD(stack(KIND_OSEM, g, psf, b_map, b_const, p, ny, nx, NY, NX, oy, ox, 1, prm, f, rep, hip_stream));
}

int sgp_apply_operator(const float* psf, const float* x, int ny, int nx, int adjoint, float* out,
                       void* hip_stream) {
  SGP_GUARD(apply_operator(psf, x, ny, nx, adjoint, out, hip_stream));
}

static int solver_create(int kind, const sgp_problem* prob, const sgp_params* prm, float* f, void* stream,
                         sgp_solver** out) {
  if (!out) return fail(SGP_E_INVALID_ARG, "null output pointer");
  *out = nullptr;
  Problem pb;
  int rc = to_problem(prob, pb);
  if (rc) return rc;
  std::unique_ptr<sgp_solver> S;
  if ((rc = create(kind, pb, prm, f, stream, false, S))) return rc;
  *out = S.release();
  return 0;
}

int sgp_solver_create(int kind, const sgp_problem* prob, const sgp_params* prm, float* f, void* hip_stream,
                      sgp_solver** out) {
  SGP_GUARD(solver_create(kind, prob, prm, f, hip_stream, out));
}

int sgp_solver_step(sgp_solver* s, int n, int* done) {
  if (!s) return fail(SGP_E_INVALID_ARG, "null solver");
  SGP_GUARD(step(s, n, done));
}

int sgp_solver_prepare(sgp_solver* s, int n) {
  if (!s) return fail(SGP_E_INVALID_ARG, "null solver");
  SGP_GUARD(prepare(s, n));
}

int sgp_solver_report(sgp_solver* s, sgp_report* rep) {
  if (!s) return fail(SGP_E_INVALID_ARG, "null solver");
  SGP_GUARD(report(s, rep));
}

int sgp_solver_gradient(sgp_solver* s, float* out) {
  if (!s || !out) return fail(SGP_E_INVALID_ARG, "null solver or output");
  if (s->kind != KIND_SGP || s->nitems != 1 || s->prm.rl_line_search)
    return fail(SGP_E_INVALID_ARG, "the gradient is kept by single-problem SGP solvers only");
  hipError_t e = hipMemcpyAsync(out, s->pl->grad, sizeof(float) * (size_t)s->pb.NY * s->pb.NX,
                                hipMemcpyDeviceToDevice, s->s);
  if (e == hipSuccess) e = hipStreamSynchronize(s->s);
  if (e != hipSuccess) return fail(SGP_E_HIP, std::string("gradient copy: ") + hipGetErrorString(e));
  return 0;
}

int sgp_solver_set_timing(sgp_solver* s, int enable) {
  if (!s) return fail(SGP_E_INVALID_ARG, "null solver");
  s->L.timing = enable != 0;
  for (int i = 0; i < SGP_KCLASS_COUNT; ++i) {
    s->ms[i] = 0;
    s->cnt[i] = 0;
  }
  return 0;
}

int sgp_solver_set_graph(sgp_solver* s, int enable) {
  if (!s) return fail(SGP_E_INVALID_ARG, "null solver");
  s->use_graph = enable != 0;
  return 0;
}

int sgp_solver_timing(sgp_solver* s, double* ms, long long* counts, int ncls) {
  if (!s || !ms || !counts) return fail(SGP_E_INVALID_ARG, "null pointer");
  for (int i = 0; i < ncls && i < SGP_KCLASS_COUNT; ++i) {
    ms[i] = s->ms[i];
    counts[i] = s->cnt[i];
  }
  return 0;
}

int sgp_solver_destroy(sgp_solver* s) {
  if (!s) return 0;
  (void)hipStreamSynchronize(s->s);
  delete s;
  return 0;
}

int sgp_batch_deconv(int kind, const sgp_problem* probs, int n, float* const* f, const float* const* f0,
                     const sgp_params* prm, sgp_report* reps, void* hip_stream) {
  SGP_GUARD(batch_run(kind, probs, n, f, f0, prm, reps, hip_stream));
}

int sgp_mosaic_deconv(int kind, const float* g, int H, int W, const float* psf, int N, float b, int core,
                      int margin, const sgp_params* prm, float* f, sgp_report* rep, void* hip_stream) {
  SGP_GUARD(mosaic_run(kind, g, H, W, psf, N, b, core, margin, prm, f, rep, hip_stream));
}

int sgp_steplength_rule(const sgp_params* prm, int k, double alpha, double tau, const double* Q, int nQ,
                        double a, double c1, double c2, double e, double* out) {
  if (!prm || !out || nQ < 0 || nQ > 8 || (nQ > 0 && !Q)) return fail(SGP_E_INVALID_ARG, "bad arguments");
  DevState st;
  std::memset(&st, 0, sizeof(st));
  st.m_alpha = prm->m_alpha;
  st.n_bb2_only = prm->n_bb2_only;
  st.alpha_min = prm->alpha_min;
  st.alpha_max = prm->alpha_max;
  st.alpha = alpha;
  st.tau = tau;
  st.k = k + 1;          // iterations completed
  st.nQ = std::min(nQ, prm->m_alpha);
  for (int i = 0; i < st.nQ; ++i) st.Q[i] = Q[nQ - st.nQ + i];
  const BBInfo r = bb_rule(&st, a, c1, c2, e);
  out[0] = r.a1;
  out[1] = r.a2;
  out[2] = r.next;
  out[3] = st.tau;
  out[4] = r.alt;
  out[5] = r.br1;
  out[6] = r.br2;
  out[7] = st.nQ;
  for (int i = 0; i < 8; ++i) out[8 + i] = i < st.nQ ? st.Q[i] : 0.0;
  return 0;
}

int sgp_flux_multiplier(const double* z, const double* D, long long n, double c, int max_steps, double* mu,
                        int* steps, int* converged) {
  if (!z || !D || n < 1 || max_steps < 0 || !mu) return fail(SGP_E_INVALID_ARG, "bad arguments");
  DevState st;
  std::memset(&st, 0, sizeof(st));
  st.flux_c = c;
  // the sums of the all-active pass (PIX_FLUX_INIT), in the same order and precision
  double t[5] = {0.0, 0.0, __builtin_inf(), 0.0, 0.0};
  for (long long i = 0; i < n; ++i) {
    if (D[i] > 0.0) {
      t[0] += z[i];
      t[1] += D[i];
      t[2] = std::fmin(t[2], z[i] / D[i]);
      t[4] += 1.0;
    } else {
      t[3] += std::fmax(0.0, z[i]);
    }
  }
  fin_flux_init(&st, t);
  int k = 0;
  for (; k < max_steps && !st.flux_done && !st.done; ++k) {  // the Newton passes (PIX_FLUX_NEWTON)
    double u[3] = {0.0, 0.0, 0.0};
    for (long long i = 0; i < n; ++i) {
      if (D[i] > 0.0 && z[i] - st.mu * D[i] > 0.0) {
        u[0] += z[i];
        u[1] += D[i];
        u[2] += 1.0;
      }
    }
    fin_flux_newton(&st, u, k == max_steps - 1);
  }
  *mu = st.mu;
  if (steps) *steps = k;
  if (converged) *converged = st.flux_done;
  if (st.done) return fail(SGP_E_NUMERIC, "non-finite multiplier");
  return st.flux_unconv > 0 ? SGP_W_FLUX_UNCONVERGED : SGP_OK;
}

// ------------------------------------------------------------ tile schedule
int sgp_tile_info(int L, int variant, int* row_threads_out, int* row_pairs_out, int* col_threads_out,
                  int* col_width_out) {
  if (!size_supported(L)) return fail(SGP_E_UNSUPPORTED_SIZE, "unsupported FFT length " + std::to_string(L));
  if (variant < 0 || variant >= kTileVariants) return fail(SGP_E_INVALID_ARG, "tile variant must be in 0..3");
  if (row_threads_out) *row_threads_out = row_threads(L, variant);
  if (row_pairs_out) *row_pairs_out = row_pairs(L, variant);
  if (col_threads_out) *col_threads_out = col_threads(L, variant);
  if (col_width_out) *col_width_out = col_width(L, variant);
  return SGP_OK;
}

int sgp_set_tile_schedule(int L, int row_variant, int col_variant) {
  if (!size_supported(L)) return fail(SGP_E_UNSUPPORTED_SIZE, "unsupported FFT length " + std::to_string(L));
  if (row_variant < 0 || row_variant >= kTileVariants || col_variant < 0 || col_variant >= kTileVariants)
    return fail(SGP_E_INVALID_ARG, "tile variants must be in 0..3");
  set_tile_schedule(L, row_variant, col_variant);
  return SGP_OK;
}

int sgp_get_tile_schedule(int L, int* row_variant, int* col_variant) {
  if (!size_supported(L)) return fail(SGP_E_UNSUPPORTED_SIZE, "unsupported FFT length " + std::to_string(L));
  tile_schedule(L, row_variant, col_variant);
  return SGP_OK;
}

static const char* kTileHeader = "# sgpdeconv tile schedule v2: length row_variant col_variant (0..3)";

int sgp_save_tile_schedule(const char* path) {
  if (!path) return fail(SGP_E_INVALID_ARG, "null path");
  std::map<int, TileChoice> copy;
  {
    std::lock_guard<std::mutex> lock(g_tile_mutex);
    copy = g_tile;
  }
  FILE* fp = std::fopen(path, "w");
  if (!fp) return fail(SGP_E_INVALID_ARG, std::string("cannot write ") + path);
  std::fprintf(fp, "%s\n", kTileHeader);
  for (const auto& kv : copy) std::fprintf(fp, "%d %d %d\n", kv.first, kv.second.row, kv.second.col);
  const bool ok = std::fclose(fp) == 0;
  return ok ? SGP_OK : fail(SGP_E_INVALID_ARG, std::string("cannot write ") + path);
}

int sgp_load_tile_schedule(const char* path) {
  if (!path) return fail(SGP_E_INVALID_ARG, "null path");
  FILE* fp = std::fopen(path, "r");
  if (!fp) return fail(SGP_E_INVALID_ARG, std::string("cannot read ") + path);
  std::map<int, TileChoice> parsed;
  char line[256];
  int lineno = 0, rc = SGP_OK;
  while (std::fgets(line, sizeof line, fp)) {
    ++lineno;
    const char* q = line;
    while (*q == ' ' || *q == '\t') ++q;
    if (*q == '#' || *q == '\n' || *q == '\r' || *q == 0) continue;
    int L, r, c;
    char extra;
    if (std::sscanf(q, "%d %d %d %c", &L, &r, &c, &extra) != 3 || !size_supported(L) || r < 0 ||
        r >= kTileVariants || c < 0 || c >= kTileVariants) {
      rc = fail(SGP_E_INVALID_ARG, std::string(path) + ":" + std::to_string(lineno) +
                                       ": expected 'length row_variant col_variant' with a supported length "
                                       "and variants in 0..3");
      break;
    }
    parsed[L] = TileChoice{r, c};
  }
  std::fclose(fp);
  if (rc) return rc;  // nothing applied
  for (const auto& kv : parsed) set_tile_schedule(kv.first, kv.second.row, kv.second.col);
  return SGP_OK;
}

// Times `iters` SGP iterations of the caller's problem under one tile
// combination: a warm-up call (graph capture), then `reps` timed calls;
// returns the least milliseconds per iteration (the run least disturbed).
static int time_combo(const sgp_problem* prob, float* f, int iters, int reps, void* stream, double* ms) {
  sgp_params prm;
  defaults(&prm);
  prm.stop = SGP_STOP_FIXED;
  prm.max_iter = iters * (reps + 1);
  sgp_solver* S = nullptr;
  int rc = solver_create(KIND_SGP, prob, &prm, f, stream, &S);
  if (rc < 0) return rc;
  std::unique_ptr<sgp_solver, int (*)(sgp_solver*)> guard(S, sgp_solver_destroy);
  int done = 0;
  if ((rc = step(S, iters, &done)) < 0) return rc;
  std::vector<double> t;
  for (int r = 0; r < reps && !done; ++r) {
    const auto t0 = std::chrono::steady_clock::now();
    if ((rc = step(S, iters, &done)) < 0) return rc;
    const auto t1 = std::chrono::steady_clock::now();
    t.push_back(std::chrono::duration<double, std::milli>(t1 - t0).count() / iters);
  }
  sgp_report rep;
  if ((rc = report(S, &rep)) < 0) return rc;
  if (rep.iters != iters * (reps + 1))
    return fail(SGP_E_INVALID_ARG, "the problem stopped after " + std::to_string(rep.iters) +
                                       " iterations while being timed (tune on a problem that runs " +
                                       std::to_string(iters * (reps + 1)) + " SGP iterations)");
  *ms = *std::min_element(t.begin(), t.end());
  return SGP_OK;
}

static int autotune(const sgp_problem* prob, float* f, int iters, int* row_variant, int* col_variant, double* ms,
                    void* hip_stream) {
  if (!prob || !f) return fail(SGP_E_INVALID_ARG, "null problem or f");
  if (iters < 1 || iters > 100000) return fail(SGP_E_INVALID_ARG, "iters must be in [1, 100000]");
  const int LX = prob->boundary ? prob->NX : prob->nx;
  const int LY = prob->boundary ? prob->NY : prob->ny;
  if (!size_supported(LX) || !size_supported(LY))
    return fail(SGP_E_UNSUPPORTED_SIZE, "unsupported FFT size " + std::to_string(LY) + " x " + std::to_string(LX));
  int prev_row, prev_col;  // restored if a timing run fails
  tile_schedule(LX, &prev_row, nullptr);
  tile_schedule(LY, nullptr, &prev_col);
  // a variant that runs the same kernels as a lower one is not timed
  auto same_row = [&](int v, int w) {
    return plan_of(LX, v) == plan_of(LX, w) && row_pairs(LX, v) == row_pairs(LX, w) &&
           row_threads(LX, v) == row_threads(LX, w);
  };
  auto same_col = [&](int v, int w) {
    return plan_of(LY, v) == plan_of(LY, w) && col_width(LY, v) == col_width(LY, w) &&
           col_threads(LY, v) == col_threads(LY, w);
  };
  auto distinct = [&](int v, bool row) {
    for (int w = 0; w < v; ++w)
      if (row ? same_row(v, w) : same_col(v, w)) return false;
    return true;
  };
  constexpr int NC = kTileVariants * kTileVariants;
  double t[NC];
  for (double& x : t) x = -1.0;
  int best = -1, rc = SGP_OK;
  for (int combo = 0; combo < NC; ++combo) {
    const int vr = combo / kTileVariants, vc = combo % kTileVariants;
    if (!distinct(vr, true) || !distinct(vc, false)) continue;  // equal to a combination already timed
    {
      std::lock_guard<std::mutex> lock(g_tile_mutex);
      g_tile[LX].row = vr;
      g_tile[LY].col = vc;
    }
    if ((rc = time_combo(prob, f, iters, 3, hip_stream, &t[combo])) < 0) break;
    if (best < 0 || t[combo] < t[best]) best = combo;
  }
  // the default shape stays unless the fastest is more than 1% faster, so
  // that timing noise between near-equal shapes keeps variant 0
  if (rc >= 0 && t[best] > 0.99 * t[0]) best = 0;
  {
    std::lock_guard<std::mutex> lock(g_tile_mutex);
    if (rc < 0) {
      g_tile[LX].row = prev_row;
      g_tile[LY].col = prev_col;
    } else {
      g_tile[LX].row = best / kTileVariants;
      g_tile[LY].col = best % kTileVariants;
    }
  }
  if (rc < 0) return rc;
  if (row_variant) *row_variant = best / kTileVariants;
  if (col_variant) *col_variant = best % kTileVariants;
  if (ms)
    for (int i = 0; i < NC; ++i) ms[i] = t[i];
  return SGP_OK;
}

int sgp_autotune(const sgp_problem* prob, float* f, int iters, int* row_variant, int* col_variant, double* ms,
                 void* hip_stream) {
  SGP_GUARD(autotune(prob, f, iters, row_variant, col_variant, ms, hip_stream));
}

int sgp_release_cache(void) {
  std::lock_guard<std::mutex> lock(g_mutex);
  (void)hipDeviceSynchronize();
  g_plans.clear();
  for (auto& kv : g_streams) {
    if (kv.second.e) (void)hipEventDestroy(kv.second.e);
    if (kv.second.s) (void)hipStreamDestroy(kv.second.s);
  }
  g_streams.clear();
  return SGP_OK;
}

const char* sgp_strerror(int code) {
  switch (code) {
    case SGP_OK: return "success";
    case SGP_W_MAXITER: return "warning: iteration cap reached before the stop rule";
    case SGP_W_ARMIJO_EXHAUSTED: return "warning: Armijo backtracking exhausted";
    case SGP_W_STATIONARY: return "warning: stationary point (grad^T d = 0)";
    case SGP_W_FLUX_UNCONVERGED: return "warning: flux-projection multiplier not converged in some iteration";
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
