// Host side of the discrete adjoint: checkpointed forward run, segment
// recompute recording (rho, u) per step, and the reverse sweep.
//
// The forward run is plain stepping (lbm_step) with the populations, markers
// and bead statistics copied aside every K steps.  Segments are then taken in
// reverse order: the segment's forward steps are recomputed from its
// checkpoint on scratch buffers (lbm_step's concurrent bulk / near-block
// schedule, so the trajectory is bitwise the forward one), keeping per step the markers, the
// bead statistics, the marker forces, the force density with its tile stamps
// and (rho, u) of every node; then its reverse steps run from last to first.
// The handle's own state is only touched by the forward run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <vector>

#include "adjoint.h"
#include "handle.h"

using namespace lbmib;

namespace lbmib {
namespace rt {

// Reverse-sweep buffers, kept on the handle between calls.
struct AdjWork {
  int64_t nck = 0;
  int K = 0;
  std::vector<void*> allocs;
  float* ck_pop = nullptr;      // [nck][19][pstride]
  double* ck_pos = nullptr;     // [nck][3][nm]
  BeadState* ck_bst = nullptr;  // [nck][nbeads]
  float* P = nullptr;           // [2][19][pstride] recompute populations
  float* L = nullptr;           // [2][19][pstride] adjoint populations
  float4* mom = nullptr;        // [K][nodes]
  double* pslab = nullptr;      // [K+1][3][nm]
  BeadState* bslab = nullptr;   // [K+1][nbeads]
  float* fslab = nullptr;       // [K][3][nm] marker forces
  float* Fslab = nullptr;       // [K][3][pstride] force density of each step (active tiles)
  int* stslab = nullptr;        // [K][ntiles] tile stamps of each step
  float *u = nullptr, *lu = nullptr, *lF = nullptr;  // [3][pstride]
  float* U = nullptr;           // [3][nm]
  int64_t* step = nullptr;
  int* overflow = nullptr;
  // near-block marks of every segment step (blocks of kScBlock nodes): flags
  // [K+1][kNearSlots][nsc], lists [K+1][2][max_near], counts [K+1][2]; entry i holds
  // the marks step i's launches read (made by step i-1's bead statistics)
  int nsc = 0, max_near = 0;
  int *nflag = nullptr, *nlist = nullptr, *ncount = nullptr, *count_sink = nullptr;
  BeadState* bsink = nullptr;   // bead statistics of the segment-start marking
  hipStream_t side = nullptr;
  hipEvent_t ev[10] = {};
  std::map<int64_t, hipGraphExec_t> graphs;  // segment graphs by 2 * length + parity
  double *lr = nullptr, *lfm = nullptr, *ltmp = nullptr, *bsum = nullptr, *grad = nullptr;
  float* lr32 = nullptr;

  ~AdjWork() {
    if (side) (void)hipStreamSynchronize(side);
    for (auto& kv : graphs)
      if (kv.second) (void)hipGraphExecDestroy(kv.second);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (side) (void)hipStreamDestroy(side);
    for (void* p : allocs) (void)hipFree(p);
  }
  template <class T>
  T* alloc(size_t n, int& rc) {
    if (rc) return nullptr;
    T* p = dev_alloc<T>(n, rc);
    if (p) allocs.push_back(p);
    return p;
  }
};

void adjoint_release(lbm_handle* h) {
  delete h->adj;
  h->adj = nullptr;
}

namespace {

int ensure_work(lbm_handle* h, int64_t nck, int K) {
  if (h->adj && h->adj->nck >= nck && h->adj->K == K) return LBM_OK;
  adjoint_release(h);
  auto* w = new AdjWork;
  int rc = LBM_OK;
  const size_t ps = (size_t)h->pstride, nm = (size_t)h->nm, nb = h->beads.size();
  w->nck = nck;
  w->K = K;
  w->ck_pop = w->alloc<float>((size_t)nck * kQ * ps, rc);
  w->ck_pos = w->alloc<double>((size_t)nck * 3 * nm, rc);
  w->ck_bst = w->alloc<BeadState>((size_t)nck * nb, rc);
  w->P = w->alloc<float>(2 * kQ * ps, rc);
  w->L = w->alloc<float>(2 * kQ * ps, rc);
  w->mom = w->alloc<float4>((size_t)K * h->nodes, rc);
  w->pslab = w->alloc<double>((size_t)(K + 1) * 3 * nm, rc);
  w->bslab = w->alloc<BeadState>((size_t)(K + 1) * nb, rc);
  w->fslab = w->alloc<float>((size_t)K * 3 * nm, rc);
  w->Fslab = w->alloc<float>((size_t)K * 3 * ps, rc);
  w->stslab = w->alloc<int>((size_t)K * h->ntiles, rc);
  w->u = w->alloc<float>(3 * ps, rc);
  w->lu = w->alloc<float>(3 * ps, rc);
  w->lF = w->alloc<float>(3 * ps, rc);
  w->U = w->alloc<float>(3 * nm, rc);
  w->step = w->alloc<int64_t>(1, rc);
  // near-block bound of the scratch launches (as set_near_bounds, blocks of kScBlock)
  w->nsc = (int)((h->nodes + kScBlock - 1) / kScBlock);
  int64_t mx = 0;
  for (const Bead& b : h->beads) {
    const Box& B = h->boxes[b.box];
    const int64_t sx = std::min<int64_t>(b.tiles_x * kTile + 4, B.nx);
    const int64_t sy = std::min<int64_t>(b.tiles_y * kTile + 4, B.ny);
    const int64_t sz = std::min<int64_t>(b.tiles_z * kTile + 4, B.nz);
    mx += sy * sz * (sx / kScBlock + 2);
  }
  w->max_near = (int)std::max<int64_t>(1, std::min<int64_t>(mx, w->nsc));
  w->nflag = w->alloc<int>((size_t)(K + 1) * kNearSlots * w->nsc, rc);
  w->nlist = w->alloc<int>((size_t)(K + 1) * 2 * w->max_near, rc);
  w->ncount = w->alloc<int>((size_t)(K + 1) * 2, rc);
  w->count_sink = w->alloc<int>(2, rc);
  w->bsink = w->alloc<BeadState>(nb, rc);
  w->overflow = w->alloc<int>(1, rc);
  w->lr = w->alloc<double>(3 * nm, rc);
  w->lfm = w->alloc<double>(3 * nm, rc);
  w->ltmp = w->alloc<double>(3 * nm, rc);
  w->bsum = w->alloc<double>(4 * nb, rc);
  w->grad = w->alloc<double>(4, rc);
  w->lr32 = w->alloc<float>(3 * nm, rc);
  if (!rc) rc = h->hip(hipStreamCreate(&w->side), "hipStreamCreate");
  for (hipEvent_t& e : w->ev)
    if (!rc) rc = h->hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreateWithFlags");
  if (rc) {
    delete w;
    return h->fail(rc, "adjoint workspace allocation failed");
  }
  h->adj = w;
  return LBM_OK;
}

// The scratch view reading (and, for bead statistics, writing) the near-block
// marks of segment step i.
Dev near_view(const Dev& base, const AdjWork& w, int i) {
  Dev d = base;
  d.near = w.nflag + (size_t)i * kNearSlots * w.nsc;
  d.near_list = w.nlist + (size_t)i * 2 * w.max_near;
  d.near_count = w.ncount + (size_t)i * 2;
  return d;
}

Dev with_near(Dev d, const Dev& n) {
  d.near = n.near;
  d.near_list = n.near_list;
  d.near_count = n.near_count;
  return d;
}

// Advection of segment step i: markers of pslab[i] into pslab[i+1]; the
// near-count reset of the advection kernel goes to a sink (every entry's
// counts are cleared at segment start).
Dev advect_view(const Dev& base, const AdjWork& w, int i, size_t nm) {
  Dev d = base;
  d.sub = i + 1;
  d.pos = w.pslab + i * 3 * nm;
  d.pos_next = w.pslab + (i + 1) * 3 * nm;
  d.near_count = w.count_sink;
  return d;
}

// Everything of one segment after its checkpoint is in place: near marks of
// its first step, the recompute, the reverse sweep.  Depends on the segment
// only through its length m and the parity par of its first step.
void enqueue_segment(lbm_handle* h, AdjWork& w, const Dev& dS, Adj a, int m, int par, int nblocks) {
  const size_t ps = (size_t)h->pstride, nm = (size_t)h->nm, nb = h->beads.size();
  const size_t popn = kQ * ps;
  hipStream_t s = h->stream;
  // near marks of the segment's first step from the checkpoint's markers (into entry 0),
  // bead statistics discarded
  {
    Dev d = near_view(dS, w, 0);
    d.pos = w.pslab;
    d.bstate_prev = w.bslab;
    d.bstate = w.bsink;
    launch_bead_stats(d, -1, s);
  }
  hipStream_t S = w.side;
  hipEvent_t* ev = w.ev;
  (void)hipEventRecord(ev[8], s);
  (void)hipStreamWaitEvent(S, ev[8], 0);
  // Recompute, as lbm_step's concurrent schedule: the side stream advects
  // step i-1, then runs step i's bead statistics, forces, spreading and
  // near-block launch (after the bulk launch of step i-1); the main stream
  // runs the bulk launch of step i (after the near-block launch of step i-1).
  // Step i reads the markers of pslab[i], advects them into pslab[i+1],
  // writes its bead statistics to bslab[i+1] taking the previous centres
  // (the volume's reference point) from bslab[i], and marks the near blocks
  // of step i+1 into entry i+1.
  for (int i = 0; i < m; ++i) {
    Dev d = dS;
    d.sub = i;
    d.pos = w.pslab + i * 3 * nm;
    d.bstate_prev = w.bslab + i * nb;
    d.bstate = w.bslab + (i + 1) * nb;
    d.fm = w.fslab + i * 3 * nm;
    d.F = w.Fslab + (size_t)i * 3 * ps;
    d.stamp = w.stslab + (size_t)i * h->ntiles;
    d.mom = w.mom + (size_t)i * h->nodes;
    hipEvent_t bulk_now = ev[i & 1], bulk_prev = ev[(i + 1) & 1];
    hipEvent_t near_now = ev[2 + (i & 1)], near_prev = ev[2 + ((i + 1) & 1)];
    if (i > 0) launch_interp_advance(advect_view(dS, w, i - 1, nm), S);
    const Dev dm = with_near(d, near_view(dS, w, i + 1));
    launch_bead_stats(dm, 0, S);
    launch_vertex_forces(dm, S);
    launch_spread(dm, S);
    const Dev dr = with_near(d, near_view(dS, w, i));
    if (i > 0) (void)hipStreamWaitEvent(s, near_prev, 0);
    launch_stream_collide_mom(dr, kLaunchBulk, nblocks, s);
    (void)hipEventRecord(bulk_now, s);
    if (i > 0) (void)hipStreamWaitEvent(S, bulk_prev, 0);
    launch_stream_collide_mom(dr, kLaunchActive, nblocks, S);
    (void)hipEventRecord(near_now, S);
  }
  (void)hipEventRecord(ev[8], s);
  (void)hipStreamWaitEvent(S, ev[8], 0);
  launch_interp_advance(advect_view(dS, w, m - 1, nm), S);
  (void)hipEventRecord(ev[9], S);
  (void)hipStreamWaitEvent(s, ev[9], 0);
  // Reverse steps of the segment, last to first.  The main stream runs the adjoint
  // collide of the blocks away from the swimmers; the side stream spreads
  // lambda_u, runs the near blocks, then the marker adjoints.  Bulk i reads
  // (and its parity is read by) near-block launch i+1; near-block launch i
  // likewise pairs with bulk i+1.
  (void)hipEventRecord(ev[8], s);
  (void)hipStreamWaitEvent(S, ev[8], 0);
  for (int i = m - 1; i >= 0; --i) {
    const int n = par + i;  // the parity of the step index is all that is used
    Dev d = dS;
    d.sub = i;
    d.pos = w.pslab + i * 3 * nm;
    d.bstate = w.bslab + (i + 1) * nb;
    d.fm = w.fslab + i * 3 * nm;
    d.F = w.Fslab + (size_t)i * 3 * ps;  // F_n, kept by the recompute
    d.stamp = w.stslab + (size_t)i * h->ntiles;
    const Dev dr = with_near(d, near_view(dS, w, i));
    a.Lsrc = w.L + ((n + 1) & 1) * popn;
    a.Ldst = w.L + (n & 1) * popn;
    a.mom = w.mom + (size_t)i * h->nodes;
    const bool first = i == m - 1;
    hipEvent_t bulk_now = ev[4 + (i & 1)], bulk_prev = ev[4 + ((i + 1) & 1)];
    hipEvent_t near_now = ev[6 + (i & 1)], near_prev = ev[6 + ((i + 1) & 1)];
    if (!first) (void)hipStreamWaitEvent(s, near_prev, 0);
    launch_adj_collide(dr, a, kLaunchBulk, nblocks, s);
    (void)hipEventRecord(bulk_now, s);
    Dev dl = d;
    dl.fm = w.lr32;
    dl.F = w.lu;
    launch_spread(dl, S);  // lambda_u = S(r_n) lambda_r(n+1), same tiles as F_n
    if (!first) (void)hipStreamWaitEvent(S, bulk_prev, 0);
    launch_adj_collide(dr, a, kLaunchActive, nblocks, S);
    (void)hipEventRecord(near_now, S);
    launch_adj_gather(d, a, S);
    launch_adj_bead(d, a, S);
    launch_adj_tangent(d, a, S);
  }
  (void)hipEventRecord(ev[9], S);
  (void)hipStreamWaitEvent(s, ev[9], 0);
}

// Segments replay captured HIP graphs (one per length and parity) when the
// handle steps with graphs, else enqueue directly.
int enqueue_or_replay(lbm_handle* h, AdjWork& w, const Dev& dS, const Adj& a, int m, int par, int nblocks) {
  if (!h->use_graphs) {
    enqueue_segment(h, w, dS, a, m, par, nblocks);
    return h->hip(hipGetLastError(), "adjoint launch");
  }
  const int64_t key = 2 * (int64_t)m + par;
  hipGraphExec_t& g = w.graphs[key];
  if (!g) {
    hipGraph_t graph = nullptr;
    int rc = h->hip(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (rc) return rc;
    enqueue_segment(h, w, dS, a, m, par, nblocks);
    rc = h->hip(hipStreamEndCapture(h->stream, &graph), "hipStreamEndCapture");
    if (!rc) rc = h->hip(hipGraphInstantiate(&g, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) {
      g = nullptr;
      return rc;
    }
  }
  return h->hip(hipGraphLaunch(g, h->stream), "hipGraphLaunch");
}

// Copy on the handle's stream.
int dcopy(lbm_handle* h, void* dst, const void* src, size_t bytes) {
  return h->hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, h->stream), "hipMemcpyAsync");
}

int run(lbm_handle* h, const lbm_adjoint_desc* ad, double* J, double* grad) {
  const int64_t T = ad->steps;
  const int K = (int)std::min<int64_t>(ad->checkpoint, T);
  const int64_t nck = (T + K - 1) / K;
  int rc = upload(h);
  if (!rc) rc = prologue(h);
  if (!rc) rc = ensure_work(h, nck, K);
  if (rc) return rc;
  AdjWork& w = *h->adj;
  const size_t ps = (size_t)h->pstride, nm = (size_t)h->nm, nb = h->beads.size();
  const size_t popn = kQ * ps;
  hipStream_t s = h->stream;

  // forward run with checkpoints
  std::vector<double> X0(3 * h->swimmers.size()), XT(X0.size());
  rc = lbm_get_swimmer_centres(h, X0.data());
  if (rc) return rc;
  const int64_t t0 = h->host_step;
  for (int64_t c = 0; c < nck; ++c) {
    const int64_t n0 = t0 + c * K, m = std::min<int64_t>(K, T - c * K);
    rc = dcopy(h, w.ck_pop + c * popn, h->pop[n0 & 1], sizeof(float) * popn);
    if (!rc) rc = dcopy(h, w.ck_pos + c * 3 * nm, h->d_pos, sizeof(double) * 3 * nm);
    if (!rc) rc = dcopy(h, w.ck_bst + c * nb, h->d_bstate, sizeof(BeadState) * nb);
    if (!rc) rc = lbm_step(h, m);
    if (rc) return rc;
  }
  rc = lbm_get_swimmer_centres(h, XT.data());
  if (rc) return rc;
  *J = XT[3 * ad->swimmer] - X0[3 * ad->swimmer];

  // scratch views of the state for the recompute and the reverse sweep
  Dev dS = h->dev;
  dS.pop[0] = w.P;
  dS.pop[1] = w.P + popn;
  dS.u = w.u;
  dS.step = w.step;
  dS.U = w.U;
  dS.overflow = w.overflow;
  dS.nsc = w.nsc;
  dS.sc_bs = kScBlock;
  dS.max_near = w.max_near;
  Adj a{};
  a.lu = w.lu;
  a.lF = w.lF;
  a.lr = w.lr;
  a.lr32 = w.lr32;
  a.lfm = w.lfm;
  a.ltmp = w.ltmp;
  a.bsum = w.bsum;
  a.grad = w.grad;
  a.swimmer = ad->swimmer;
  rc = h->hip(hipMemsetAsync(w.L, 0, sizeof(float) * 2 * popn, s), "hipMemsetAsync");
  if (!rc) rc = h->hip(hipMemsetAsync(w.stslab, 0x80, sizeof(int) * (size_t)K * h->ntiles, s), "hipMemsetAsync");
  if (!rc)
    rc = h->hip(hipMemsetAsync(w.nflag, 0x80, sizeof(int) * (size_t)(K + 1) * kNearSlots * w.nsc, s), "hipMemsetAsync");
  if (!rc) rc = h->hip(hipMemsetAsync(w.overflow, 0, sizeof(int), s), "hipMemsetAsync");
  if (rc) return rc;
  launch_adj_init(dS, a, s);
  const int nblocks = (int)((h->nodes + kScBlock - 1) / kScBlock);

  for (int64_t c = nck - 1; c >= 0; --c) {
    const int64_t n0 = t0 + c * K;
    const int m = (int)std::min<int64_t>(K, T - c * K);
    rc = dcopy(h, w.P + (n0 & 1) * popn, w.ck_pop + c * popn, sizeof(float) * popn);
    if (!rc) rc = dcopy(h, w.pslab, w.ck_pos + c * 3 * nm, sizeof(double) * 3 * nm);
    if (!rc) rc = dcopy(h, w.bslab, w.ck_bst + c * nb, sizeof(BeadState) * nb);
    if (!rc) rc = h->hip(hipMemsetAsync(w.ncount, 0, sizeof(int) * (size_t)(K + 1) * 2, s), "hipMemsetAsync");
    if (rc) return rc;
    launch_set_step(w.step, n0, s);
    rc = enqueue_or_replay(h, w, dS, a, m, (int)(n0 & 1), nblocks);
    if (rc) return rc;
    rc = h->hip(hipGetLastError(), "adjoint launch");
    if (rc) return rc;
  }
  int ov = 0;
  rc = h->hip(hipMemcpyAsync(grad, w.grad, sizeof(double) * 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  if (!rc) rc = h->hip(hipMemcpyAsync(&ov, w.overflow, sizeof(int), hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  if (!rc) rc = h->hip(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (rc) return rc;
  if (ov) return h->fail(LBM_EOVERFLOW, "bead region or near list overflow in the adjoint recompute");
  return LBM_OK;
}

}  // namespace
}  // namespace rt
}  // namespace lbmib

extern "C" {

int lbm_swimmer_set_params(lbm_handle* h, int32_t swimmer, double A, double B, double alpha, double k) {
  if (!h || swimmer < 0 || swimmer >= (int32_t)h->swimmers.size()) return LBM_EINVAL;
  Swimmer& S = h->swimmers[swimmer];
  S.A = A;
  S.B = B;
  S.alpha = alpha;
  S.k[0] = S.k[1] = k;
  if (!h->uploaded) return LBM_OK;
  int rc = h->hip(hipMemcpyAsync(h->d_swimmers + swimmer, &S, sizeof(Swimmer), hipMemcpyHostToDevice, h->stream),
                  "hipMemcpyAsync");
  if (rc) return rc;
  return h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
}

int lbm_adjoint(lbm_handle* h, const lbm_adjoint_desc* desc, double* J, double grad[4]) {
  if (!h || !desc || !J || !grad) return LBM_EINVAL;
  if (desc->steps < 1 || desc->checkpoint < 1) return h->fail(LBM_EINVAL, "adjoint needs steps >= 1 and checkpoint >= 1");
  if (desc->swimmer < 0 || desc->swimmer >= (int32_t)h->swimmers.size())
    return h->fail(LBM_EINVAL, "adjoint objective: no such swimmer");
  if (h->boxes.size() != 1) return h->fail(LBM_EINVAL, "adjoint: single-box handles only");
  if (h->storage != LBM_FP32_SHIFTED) return h->fail(LBM_EINVAL, "adjoint: FP32 storage only");
  if (h->boxes[0].forcing != kGuo) return h->fail(LBM_EINVAL, "adjoint: Guo forcing only");
  int rc = rt::upload(h);
  if (rc) return rc;
  rt::Snapshot snap;
  if (desc->rewind) {
    rc = rt::prologue(h);
    if (rc) return rc;
    rt::snapshot_parts(h, snap);
    if (hipMalloc(&snap.mem, rt::snapshot_bytes(snap)) != hipSuccess)
      return h->fail(LBM_ENOMEM, "adjoint snapshot allocation failed");
    rc = rt::snapshot_copy(h, snap, true);
  }
  if (!rc) rc = rt::run(h, desc, J, grad);
  if (desc->rewind) {
    const int rc2 = rt::snapshot_copy(h, snap, false);
    if (!rc) rc = rc2;
    (void)hipFree(snap.mem);
  }
  return rc;
}

}  // extern "C"
