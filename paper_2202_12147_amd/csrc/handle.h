// Internal host-side handle shared by the runtime translation units (not part
// of the C-ABI: callers see lbm_handle only as an opaque pointer).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/lbmib.h"
#include "common.h"

namespace lbmib {

constexpr int kGraphChunk = 32;  // steps per captured graph
// Step graphs of every count 1..kGraphChunk: a call of n steps replays the
// graph of n mod kGraphChunk steps once, then the chunk graph n / kGraphChunk
// times, so a call of up to 32 steps is one graph (one fork and join of the
// two streams; a 20-step call 59.3-60.1 against 61.5-61.8 us per step with
// the binary split into graphs of 4 and 16 steps).

template <class T>
T* dev_alloc(size_t n, int& rc) {
  void* p = nullptr;
  if (n == 0) n = 1;
  if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) {
    rc = LBM_ENOMEM;
    return nullptr;
  }
  return static_cast<T*>(p);
}

}  // namespace lbmib

namespace lbmib {
namespace rt {
struct AdjWork;
}
}  // namespace lbmib

using lbmib::Bead;
using lbmib::BeadState;
using lbmib::Box;
using lbmib::Dev;
using lbmib::Swimmer;

struct lbm_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int storage = LBM_FP32_SHIFTED, width = 3;
  float fp16_scale = 1.0f;
  bool use_graphs = true;
  std::string err;

  // host model
  std::vector<Box> boxes;
  std::vector<Bead> beads;
  std::vector<Swimmer> swimmers;
  std::vector<double> pos0;  // [nm][3] initial marker positions
  std::vector<int> marker_bead;
  std::vector<int> marker_info;  // [nm][4], see Dev::marker_info
  std::vector<int> tri;      // [ntri][3] global vertex ids
  std::vector<double> G0;    // [ntri][3]
  std::vector<double> hingeth0;
  std::vector<int> hinge;    // [nh][4]
  int nm = 0;
  int64_t nodes = 0, pstride = 0;
  int ntiles = 0, sc_blocks = 0, spread_blocks = 0, out_blocks = 0;
  int sc_block = 512, sc_remap = 0, sc_resident = 1;  // stream-collide launch shape (set per handle at creation)
  int ncu = 256;                                        // compute units of the device
  bool uploaded = false, stepped = false;
  int64_t host_step = 0;  // steps enqueued

  // device buffers
  void* pop[2] = {nullptr, nullptr};
  float *F = nullptr, *u = nullptr, *uout = nullptr;
  double* avg_sums = nullptr;     // time-average sums [3][pstride] (allocated on first use)
  int* stamp = nullptr;
  Box* d_boxes = nullptr;
  int* d_block_box = nullptr;     // 256-node block -> box
  int* d_sc_block_box = nullptr;  // stream-collide block -> box (sized for block 128)
  int* d_sc_box_block0 = nullptr; // first stream-collide block of each box
  int64_t sc_table_cap = 0;       // stream-collide blocks at block 128: sum over boxes of ceil(n / 128)
  int64_t* d_step = nullptr;
  double* d_pos = nullptr;
  float *d_U = nullptr, *d_fm = nullptr, *d_fmem = nullptr, *d_gvol = nullptr;
  lbmib::BeadTerms* d_bterms = nullptr;  // [beads]
  Bead* d_beads = nullptr;
  BeadState* d_bstate = nullptr;
  Swimmer* d_swimmers = nullptr;
  int *d_marker_bead = nullptr, *d_tri = nullptr, *d_hinge = nullptr;
  int4* d_marker_info = nullptr;
  double *d_G0 = nullptr, *d_theta0 = nullptr;
  float *d_G0inv = nullptr, *d_A0 = nullptr, *d_idet = nullptr;
  int *d_lane_elem = nullptr, *d_lane_v = nullptr;
  int* d_overflow = nullptr;
  int* d_spread_info = nullptr;  // [spread block][8], see Dev::spread_info
  int *d_near = nullptr, *d_near_list = nullptr, *d_near_count = nullptr;
  int* d_work = nullptr;           // persistent bulk block counters (kWorkCounters)
  bool need_prologue = true;
  hipStream_t side = nullptr;      // IBM chain, forked from `stream` every step
  std::vector<hipEvent_t> step_events;  // per chunk step: bulk done, near blocks done; + one fork
  double *d_partial = nullptr, *d_out = nullptr, *d_centres = nullptr;
  double* conserved_scratch = nullptr;  // the device's static scratch (not owned)
  std::vector<void*> allocs;

  Dev dev{};
  lbmib::rt::AdjWork* adj = nullptr;  // adjoint buffers, kept between calls
  hipGraphExec_t g_steps[lbmib::kGraphChunk + 1] = {};  // g_steps[c]: c steps

  bool timing = false;
  double timed_ms = 0;
  int64_t timed_launches = 0;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;

  int fail(int code, const std::string& msg) {
    err = msg;
    return code;
  }
  int hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return LBM_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return LBM_EDEVICE;
  }
  template <class T>
  T* alloc(size_t n, int& rc) {
    T* p = lbmib::dev_alloc<T>(n, rc);
    if (p) allocs.push_back(p);
    return p;
  }
};

namespace lbmib {
namespace rt {

int element_bytes(const lbm_handle* h);
// Device buffers and mesh tables, once, before the first step.
int upload(lbm_handle* h);
// Bead regions and near blocks of the current markers when stepping resumes.
int prologue(lbm_handle* h);
// LBM_EOVERFLOW when a bead outgrew its tiles or the near list overflowed.
int check_overflow(lbm_handle* h);
// Free the adjoint buffers of a handle.
void adjoint_release(lbm_handle* h);

// Device copy of every buffer that stepping changes.
struct Snapshot {
  std::vector<std::pair<void*, size_t>> parts;
  char* mem = nullptr;
  int64_t host_step = 0;
};
void snapshot_parts(lbm_handle* h, Snapshot& S);
size_t snapshot_bytes(const Snapshot& S);
// take = true: state -> snapshot; false: snapshot -> state.  Synchronizes.
int snapshot_copy(lbm_handle* h, Snapshot& S, bool take);

}  // namespace rt
}  // namespace lbmib
