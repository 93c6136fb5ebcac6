// Test infrastructure: a CPU stand-in for the HIP runtime and the kernel
// launchers, so that the library's host code (solver.cpp) runs under
// AddressSanitizer without a GPU.
// Device memory is host memory; streams are synchronous; graphs record and
// replay the launcher calls.  The iteration end (launch_row_fin of the
// gradient pass) advances each item's counter and stops items at a
// per-item iteration count, so the batch driver's compaction paths run.
#include <hip/hip_runtime.h>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>
#include "launch.hpp"

using Rec = std::vector<std::function<void()>>;
static bool g_cap = false;
static Rec* g_rec = nullptr;
static void run_or_rec(std::function<void()> fn) {
  if (g_cap) g_rec->push_back(std::move(fn));
  else fn();
}

extern "C" {
hipError_t hipMalloc(void** p, size_t n) { *p = calloc(1, n ? n : 1); return hipSuccess; }
hipError_t hipFree(void* p) { free(p); return hipSuccess; }
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { *p = calloc(1, n ? n : 1); return hipSuccess; }
hipError_t hipHostFree(void* p) { free(p); return hipSuccess; }
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) { memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  run_or_rec([=] { memmove(d, s, n); });
  return hipSuccess;
}
hipError_t hipMemcpy2DAsync(void* d, size_t dp, const void* s, size_t sp, size_t w, size_t h, hipMemcpyKind,
                            hipStream_t) {
  run_or_rec([=] {
    for (size_t r = 0; r < h; ++r) memmove((char*)d + r * dp, (const char*)s + r * sp, w);
  });
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  run_or_rec([=] { memset(d, v, n); });
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) { *s = (hipStream_t)malloc(16); return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { free((void*)s); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned int) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t* e) { *e = (hipEvent_t)malloc(16); return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned int) { *e = (hipEvent_t)malloc(16); return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e) { free((void*)e); return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) { *ms = 0.f; return hipSuccess; }
hipError_t hipGetDevice(int* d) { *d = 0; return hipSuccess; }
hipError_t hipGetDeviceCount(int* n) { *n = 1; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "shim error"; }
hipError_t hipGetSymbolAddress(void** p, const void* sym) { *p = (void*)sym; return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) {
  if (g_cap) { fprintf(stderr, "nested capture\n"); abort(); }
  g_cap = true;
  g_rec = new Rec();
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
  g_cap = false;
  *g = (hipGraph_t)g_rec;
  g_rec = nullptr;
  return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  *e = (hipGraphExec_t) new Rec(*(Rec*)g);
  return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t e, hipStream_t) {
  for (auto& f : *(Rec*)e) f();
  return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t e) { delete (Rec*)e; return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete (Rec*)g; return hipSuccess; }
void** __hipRegisterFatBinary(const void*) { static void* h[4]; return h; }
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterVar(void**, char*, char*, const char*, int, size_t, int, int) {}
}

namespace sgp {
bool size_supported(int L) { return L >= 16 && L <= 2048; }
int row_pairs(int L, int v) { int rp = 1024 / (L / 8); rp = rp < 1 ? 1 : rp > 4 ? 4 : rp; return v == 1 && rp >= 2 ? rp / 2 : rp; }
int row_threads(int L, int v) { return row_pairs(L, v) * (L / 8); }
int col_width(int L, int v) { return v == 1 ? 2 : 1; }
int col_threads(int L, int v) { return col_width(L, v) * (L / 8); }
// iteration count at which batched item b stops (the harness expects it)
int shim_target(int b) { return 2 + (b * 37) % 90; }
void launch_row(int, int, int, dim3, const Args&, hipStream_t) {}
void launch_col(int, int, int, int, dim3, const Args&, hipStream_t) {}
void launch_pix(int, dim3, const Args&, hipStream_t) {}
void launch_twiddle(float2*, int, int, hipStream_t) {}
int plan_of(int, int v) { return (v >> 1) & 1; }
void launch_zero(unsigned* c, int n, hipStream_t) { run_or_rec([=] { memset(c, 0, sizeof(unsigned) * n); }); }
void launch_resume(DevState* st, int n, int nitems, hipStream_t) {
  run_or_rec([=] {
    for (int i = 0; i < nitems; ++i) { st[i].pause = 0; st[i].k_stop = st[i].k + n; }
  });
}
void launch_row_fin(int op, int nz, const Args& a_in, hipStream_t) {
  const Args a = a_in;
  if (op != ROW_GRAD && op != ROW_RLUPD) return;
  run_or_rec([=] {
    for (int z = 0; z < nz; ++z) {
      const int b = a.zmap ? a.zmap[z] : z;
      DevState& s = a.st[b];
      if (s.done || s.pause) continue;
      s.k++;
      if (s.k >= shim_target(b)) { s.done = 1; s.reason = 2; }
      else if (s.k >= s.max_iter) { s.done = 1; s.reason = 0; }
      else if (s.k >= s.k_stop) s.pause = 1;
    }
  });
}
}  // namespace sgp
