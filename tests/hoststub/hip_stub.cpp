// Host-only stand-in for the HIP runtime and the kernel launch wrappers, for
// running the library's host code (handles, block tables, graph bookkeeping,
// tuner, adjoint schedule, checkpoints) on the CPU under AddressSanitizer.
//
// Device memory is ordinary heap memory, so every host-side copy, memset and
// table upload that overruns an allocation is caught by the sanitizer;
// streams, events, graphs and graph executables are heap objects that are
// checked for use after destruction and destroyed twice.  Kernel launches do
// nothing: results are meaningless, only memory safety of the host code is
// tested.  Test infrastructure, never linked into the library.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <set>

#include "../../paper_2202_12147_amd/csrc/adjoint.h"
#include "../../paper_2202_12147_amd/csrc/common.h"

namespace {
constexpr unsigned kLive = 0x5ca1ab1e;
std::set<const void*> g_live;  // every live stream, event, graph and executable

[[noreturn]] void die(const char* what, const void* p) {
  std::fprintf(stderr, "hip_stub: %s %p\n", what, p);
  std::abort();
}
void check(const void* p, const char* what) {
  if (p && !g_live.count(p)) die(what, p);
}
}  // namespace

struct ihipStream_t {
  unsigned magic = kLive;
  bool capturing = false;
};
struct ihipEvent_t {
  unsigned magic = kLive;
};
struct ihipGraph {
  unsigned magic = kLive;
};
struct hipGraphExec {
  unsigned magic = kLive;
};

template <class T>
static T* make() {
  T* p = new T;
  g_live.insert(p);
  return p;
}
template <class T>
static hipError_t destroy(T* p, const char* what) {
  if (!p) return hipErrorInvalidValue;
  check(p, what);
  g_live.erase(p);
  delete p;
  return hipSuccess;
}

extern "C" {
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* pi, hipDeviceAttribute_t, int) {
  *pi = 256;
  return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
hipError_t hipGetLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "stub error"; }

hipError_t hipMalloc(void** p, size_t n) {
  *p = std::calloc(n ? n : 1, 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  std::free(p);
  return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
  std::memcpy(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
  check(s, "copy on a destroyed stream");
  std::memcpy(dst, src, n);
  return hipSuccess;
}
hipError_t hipMemset(void* dst, int v, size_t n) {
  std::memset(dst, v, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* dst, int v, size_t n, hipStream_t s) {
  check(s, "memset on a destroyed stream");
  std::memset(dst, v, n);
  return hipSuccess;
}

hipError_t hipStreamCreate(hipStream_t* s) {
  *s = make<ihipStream_t>();
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) { return destroy(s, "stream destroyed twice"); }
hipError_t hipStreamSynchronize(hipStream_t s) {
  check(s, "synchronize on a destroyed stream");
  return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
  check(s, "wait on a destroyed stream");
  check(e, "wait for a destroyed event");
  return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
  check(s, "capture on a destroyed stream");
  if (!s || s->capturing) return hipErrorIllegalState;
  s->capturing = true;
  return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
  check(s, "end capture on a destroyed stream");
  if (!s || !s->capturing) return hipErrorIllegalState;
  s->capturing = false;
  *g = make<ihipGraph>();
  return hipSuccess;
}

hipError_t hipEventCreate(hipEvent_t* e) {
  *e = make<ihipEvent_t>();
  return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) { return destroy(e, "event destroyed twice"); }
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  check(e, "record of a destroyed event");
  check(s, "record on a destroyed stream");
  return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
  check(e, "synchronize on a destroyed event");
  return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
  check(a, "elapsed time of a destroyed event");
  check(b, "elapsed time of a destroyed event");
  *ms = 1.0f;
  return hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
  check(g, "instantiate of a destroyed graph");
  *x = make<hipGraphExec>();
  return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) { return destroy(g, "graph destroyed twice"); }
hipError_t hipGraphExecDestroy(hipGraphExec_t x) { return destroy(x, "graph executable destroyed twice"); }
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
  if (!x) die("launch of a null graph executable", x);
  check(x, "launch of a destroyed graph executable");
  check(s, "graph launch on a destroyed stream");
  return hipSuccess;
}
}  // extern "C"

// Kernel launch wrappers of the library: no device work.
namespace lbmib {
namespace {
double g_scratch[4 * kNoAllocParts];
}
void launch_stream_collide(const Dev&, int, int, int, int, int, int, int, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1) {
  check(s, "launch on a destroyed stream");
  check(e0, "launch stamping a destroyed event");
  check(e1, "launch stamping a destroyed event");
}
void launch_stream_collide_mom(const Dev&, int, int, hipStream_t s) { check(s, "launch on a destroyed stream"); }
void launch_tick(const Dev&, int, hipStream_t s) { check(s, "launch on a destroyed stream"); }
void launch_velocity(const Dev&, int, int, float*, float*, hipStream_t s) { check(s, "launch"); }
void launch_average_out(const Dev&, int, int64_t, float*, hipStream_t s) { check(s, "launch"); }
void launch_conserved(const Dev&, int, int, double* partial, int nparts, double* out, hipStream_t s,
                      double mass0) {
  check(s, "launch");
  std::memset(partial, 0, sizeof(double) * 4 * nparts);  // the partial sums the launch would write
  out[0] = mass0;
  out[1] = out[2] = out[3] = 0.0;
}
hipError_t resolve_conserved_scratch(int, double** out) {
  *out = g_scratch;
  return hipSuccess;
}
void launch_bead_stats(const Dev&, int, hipStream_t s) { check(s, "launch"); }
void launch_stats_forces(const Dev&, int, hipStream_t s) { check(s, "launch"); }
void launch_marker_force_total(const Dev&, float*, hipStream_t s) { check(s, "launch"); }
void launch_spread(const Dev&, hipStream_t s) { check(s, "launch"); }
void launch_interp_advance(const Dev&, hipStream_t s) { check(s, "launch"); }
void launch_bead_centres(const Dev&, double* out, hipStream_t s) {
  check(s, "launch");
  (void)out;
}
void launch_copy(const void*, void*, int64_t, hipStream_t s) { check(s, "launch"); }
void launch_adj_init(const Dev&, const Adj&, hipStream_t s) { check(s, "launch"); }
void launch_adj_collide(const Dev&, const Adj&, int, int, hipStream_t s) { check(s, "launch"); }
void launch_adj_gather(const Dev&, const Adj&, hipStream_t s) { check(s, "launch"); }
void launch_adj_bead(const Dev&, const Adj&, hipStream_t s) { check(s, "launch"); }
void launch_adj_tangent(const Dev&, const Adj&, hipStream_t s) { check(s, "launch"); }
void launch_set_step(int64_t*, int64_t, hipStream_t s) { check(s, "launch"); }
}  // namespace lbmib
