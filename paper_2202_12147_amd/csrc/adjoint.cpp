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
// Segment storage is double-buffered: the recompute of segment c - 1 runs on
// its own pair of streams while the reverse sweep of segment c runs on the
// handle's stream and the adjoint side stream.
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

// Storage of one recomputed segment (two of them alternate).
struct AdjSet {
  float* P = nullptr;           // [2][19][pstride] recompute populations
  float4* mom = nullptr;        // [K][nodes]
  double* pslab = nullptr;      // [K+1][3][nm]
  BeadState* bslab = nullptr;   // [K+1][nbeads]
  float* fslab = nullptr;       // [K][3][nm] marker forces
  float* Fslab = nullptr;       // [K][3][pstride] force density of each step (active tiles)
  int* stslab = nullptr;        // [K][ntiles] tile stamps of each step
  float* u = nullptr;           // [3][pstride] velocity at forced nodes
  float* U = nullptr;           // [3][nm]
  int64_t* step = nullptr;      // step index of the segment's first step
  // near-block marks of every segment step (blocks of kScBlock nodes): flags
  // [K+1][kNearSlots][nsc], lists [K+1][2][max_near], counts [K+1][2]; entry i holds
  // the marks step i's launches read (made by step i-1's bead statistics)
  int *nflag = nullptr, *nlist = nullptr, *ncount = nullptr, *count_sink = nullptr;
  BeadState* bsink = nullptr;   // bead statistics of the segment-start marking
};

// Reverse-sweep buffers, kept on the handle between calls.
struct AdjWork {
  int64_t nck = 0;
  int K = 0;
  std::vector<void*> allocs;
  float* ck_pop = nullptr;      // [nck][19][pstride]
  double* ck_pos = nullptr;     // [nck][3][nm]
  BeadState* ck_bst = nullptr;  // [nck][nbeads]
  AdjSet set[2];
  float* L = nullptr;           // [2][19][pstride] adjoint populations
  float *lu = nullptr, *lF = nullptr;  // [3][pstride]
  int* overflow = nullptr;
  int nsc = 0, max_near = 0;
  hipStream_t side = nullptr;            // reverse sweep: side stream (main: the handle's)
  hipStream_t rmain = nullptr, rside = nullptr;  // recompute
  hipEvent_t ev[12] = {};  // 0-3, 8, 9: recompute; 4-7, 10, 11: reverse
  hipEvent_t rec_done[2] = {}, rev_done[2] = {}, start = nullptr;
  // recompute graphs by (length, set); reverse-sweep graphs by (objective
  // swimmer, length, parity, set): the swimmer is a kernel argument of the
  // reverse sweep's bead kernels
  std::map<int64_t, hipGraphExec_t> rgraphs, vgraphs;
  double *lr = nullptr, *lfm = nullptr, *ltmp = nullptr, *bsum = nullptr, *grad = nullptr;
  float* lr32 = nullptr;

  ~AdjWork() {
    for (hipStream_t q : {side, rmain, rside})
      if (q) (void)hipStreamSynchronize(q);
    for (auto* g : {&rgraphs, &vgraphs})
      for (auto& kv : *g)
        if (kv.second) (void)hipGraphExecDestroy(kv.second);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    for (hipEvent_t e : {rec_done[0], rec_done[1], rev_done[0], rev_done[1], start})
      if (e) (void)hipEventDestroy(e);
    for (hipStream_t q : {side, rmain, rside})
      if (q) (void)hipStreamDestroy(q);
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
  for (AdjSet& S : w->set) {
    S.P = w->alloc<float>(2 * kQ * ps, rc);
    S.mom = w->alloc<float4>((size_t)K * h->nodes, rc);
    S.pslab = w->alloc<double>((size_t)(K + 1) * 3 * nm, rc);
    S.bslab = w->alloc<BeadState>((size_t)(K + 1) * nb, rc);
    S.fslab = w->alloc<float>((size_t)K * 3 * nm, rc);
    S.Fslab = w->alloc<float>((size_t)K * 3 * ps, rc);
    S.stslab = w->alloc<int>((size_t)K * h->ntiles, rc);
    S.u = w->alloc<float>(3 * ps, rc);
    S.U = w->alloc<float>(3 * nm, rc);
    S.step = w->alloc<int64_t>(1, rc);
    S.nflag = w->alloc<int>((size_t)(K + 1) * kNearSlots * w->nsc, rc);
    S.nlist = w->alloc<int>((size_t)(K + 1) * 2 * w->max_near, rc);
    S.ncount = w->alloc<int>((size_t)(K + 1) * 2, rc);
    S.count_sink = w->alloc<int>(2, rc);
    S.bsink = w->alloc<BeadState>(nb, rc);
  }
  w->L = w->alloc<float>(2 * kQ * ps, rc);
  w->lu = w->alloc<float>(3 * ps, rc);
  w->lF = w->alloc<float>(3 * ps, rc);
  w->overflow = w->alloc<int>(1, rc);
  w->lr = w->alloc<double>(3 * nm, rc);
  w->lfm = w->alloc<double>(3 * nm, rc);
  w->ltmp = w->alloc<double>(3 * nm, rc);
  w->bsum = w->alloc<double>(4 * nb, rc);
  w->grad = w->alloc<double>(4, rc);
  w->lr32 = w->alloc<float>(3 * nm, rc);
  for (hipStream_t* q : {&w->side, &w->rmain, &w->rside})
    if (!rc) rc = h->hip(hipStreamCreate(q), "hipStreamCreate");
  for (hipEvent_t& e : w->ev)
    if (!rc) rc = h->hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreateWithFlags");
  for (hipEvent_t* e : {&w->rec_done[0], &w->rec_done[1], &w->rev_done[0], &w->rev_done[1], &w->start})
    if (!rc) rc = h->hip(hipEventCreateWithFlags(e, hipEventDisableTiming), "hipEventCreateWithFlags");
  if (rc) {
    delete w;
    return h->fail(rc, "adjoint workspace allocation failed");
  }
  h->adj = w;
  return LBM_OK;
}

// The scratch view reading (and, for bead statistics, writing) the near-block
// marks of segment step i.
Dev near_view(const Dev& base, const AdjWork& w, const AdjSet& S, int i) {
  Dev d = base;
  d.near = S.nflag + (size_t)i * kNearSlots * w.nsc;
  d.near_list = S.nlist + (size_t)i * 2 * w.max_near;
  d.near_count = S.ncount + (size_t)i * 2;
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
Dev advect_view(const Dev& base, const AdjSet& S, int i, size_t nm) {
  Dev d = base;
  d.sub = i + 1;
  d.pos = S.pslab + i * 3 * nm;
  d.pos_next = S.pslab + (i + 1) * 3 * nm;
  d.near_count = S.count_sink;
  return d;
}

// The state view of a segment set: its populations, velocity, marker
// velocities and step counter.
Dev set_view(const Dev& dS, const AdjSet& S, size_t popn) {
  Dev d = dS;
  d.pop[0] = S.P;
  d.pop[1] = S.P + popn;
  d.u = S.u;
  d.step = S.step;
  d.U = S.U;
  return d;
}

// Recompute of one segment from its checkpoint (already in the set), on the
// streams s (main) and S2 (side): near marks of its first step, then the
// steps as lbm_step's concurrent schedule -- the side stream advects step
// i-1 and runs step i's bead statistics, forces, spreading and near-block
// launch (after the bulk launch of step i-1), the main stream the bulk launch
// of step i (after the near-block launch of step i-1).  Step i reads the
// markers of pslab[i], advects them into pslab[i+1], writes its bead
// statistics to bslab[i+1] taking the previous centres (the volume's
// reference point) from bslab[i], and marks the near blocks of step i+1 into
// entry i+1.
void enqueue_recompute(lbm_handle* h, AdjWork& w, const AdjSet& St, const Dev& dS, int m, int nblocks,
                       hipStream_t s, hipStream_t S2) {
  const size_t ps = (size_t)h->pstride, nm = (size_t)h->nm, nb = h->beads.size();
  hipEvent_t* ev = w.ev;
  {
    // near marks of the segment's first step from the checkpoint's markers
    // (into entry 0), bead statistics discarded
    Dev d = near_view(dS, w, St, 0);
    d.pos = St.pslab;
    d.bstate_prev = St.bslab;
    d.bstate = St.bsink;
    launch_bead_stats(d, -1, s);
  }
  (void)hipEventRecord(ev[8], s);
  (void)hipStreamWaitEvent(S2, ev[8], 0);
  for (int i = 0; i < m; ++i) {
    Dev d = dS;
    d.sub = i;
    d.pos = St.pslab + i * 3 * nm;
    d.bstate_prev = St.bslab + i * nb;
    d.bstate = St.bslab + (i + 1) * nb;
    d.fm = St.fslab + i * 3 * nm;
    d.F = St.Fslab + (size_t)i * 3 * ps;
    d.stamp = St.stslab + (size_t)i * h->ntiles;
    d.mom = St.mom + (size_t)i * h->nodes;
    hipEvent_t bulk_now = ev[i & 1], bulk_prev = ev[(i + 1) & 1];
    hipEvent_t near_now = ev[2 + (i & 1)], near_prev = ev[2 + ((i + 1) & 1)];
    if (i > 0) launch_interp_advance(advect_view(dS, St, i - 1, nm), S2);
    const Dev dm = with_near(d, near_view(dS, w, St, i + 1));
    launch_stats_forces(dm, 0, S2);
    launch_spread(dm, S2);
    launch_marker_force_total(dm, dm.fm, S2);  // the step's total forces, read by the reverse sweep
    const Dev dr = with_near(d, near_view(dS, w, St, i));
    if (i > 0) (void)hipStreamWaitEvent(s, near_prev, 0);
    launch_stream_collide_mom(dr, kLaunchBulk, nblocks, s);
    (void)hipEventRecord(bulk_now, s);
    if (i > 0) (void)hipStreamWaitEvent(S2, bulk_prev, 0);
    launch_stream_collide_mom(dr, kLaunchActive, nblocks, S2);
    (void)hipEventRecord(near_now, S2);
  }
  launch_interp_advance(advect_view(dS, St, m - 1, nm), S2);
  (void)hipEventRecord(ev[9], S2);
  (void)hipStreamWaitEvent(s, ev[9], 0);
}

// Reverse steps of a segment, last to first, on the streams s (main) and S2
// (side).  The main stream runs the adjoint collide of the blocks away from
// the swimmers; the side stream spreads lambda_u, runs the near blocks, then
// the marker adjoints.  Bulk i reads (and its parity is read by) near-block
// launch i+1; near-block launch i likewise pairs with bulk i+1.
void enqueue_reverse(lbm_handle* h, AdjWork& w, const AdjSet& St, const Dev& dS, Adj a, int m, int par,
                     int nblocks, hipStream_t s, hipStream_t S2) {
  const size_t ps = (size_t)h->pstride, nm = (size_t)h->nm, nb = h->beads.size();
  const size_t popn = kQ * ps;
  hipEvent_t* ev = w.ev;
  (void)hipEventRecord(ev[10], s);
  (void)hipStreamWaitEvent(S2, ev[10], 0);
  for (int i = m - 1; i >= 0; --i) {
    const int n = par + i;  // the parity of the step index is all that is used
    Dev d = dS;
    d.sub = i;
    d.pos = St.pslab + i * 3 * nm;
    d.bstate = St.bslab + (i + 1) * nb;
    d.fm = St.fslab + i * 3 * nm;
    d.F = St.Fslab + (size_t)i * 3 * ps;  // F_n, kept by the recompute
    d.stamp = St.stslab + (size_t)i * h->ntiles;
    const Dev dr = with_near(d, near_view(dS, w, St, i));
    a.Lsrc = w.L + ((n + 1) & 1) * popn;
    a.Ldst = w.L + (n & 1) * popn;
    a.mom = St.mom + (size_t)i * h->nodes;
    const bool first = i == m - 1;
    hipEvent_t bulk_now = ev[4 + (i & 1)], bulk_prev = ev[4 + ((i + 1) & 1)];
    hipEvent_t near_now = ev[6 + (i & 1)], near_prev = ev[6 + ((i + 1) & 1)];
    if (!first) (void)hipStreamWaitEvent(s, near_prev, 0);
    launch_adj_collide(dr, a, kLaunchBulk, nblocks, s);
    (void)hipEventRecord(bulk_now, s);
    Dev dl = d;
    dl.fm = w.lr32;
    dl.spread_raw = 1;
    dl.F = w.lu;
    launch_spread(dl, S2);  // lambda_u = S(r_n) lambda_r(n+1), same tiles as F_n
    if (!first) (void)hipStreamWaitEvent(S2, bulk_prev, 0);
    launch_adj_collide(dr, a, kLaunchActive, nblocks, S2);
    (void)hipEventRecord(near_now, S2);
    launch_adj_gather(d, a, S2);
    launch_adj_bead(d, a, S2);
    launch_adj_tangent(d, a, S2);
  }
  (void)hipEventRecord(ev[11], S2);
  (void)hipStreamWaitEvent(s, ev[11], 0);
}

// Enqueue (or replay the captured graph of) one part on its main stream.
template <class F>
int enqueue_or_replay(lbm_handle* h, std::map<int64_t, hipGraphExec_t>& graphs, int64_t key, hipStream_t s,
                      F&& enqueue) {
  if (!h->use_graphs) {
    enqueue();
    return h->hip(hipGetLastError(), "adjoint launch");
  }
  hipGraphExec_t& g = graphs[key];
  if (!g) {
    hipGraph_t graph = nullptr;
    int rc = h->hip(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (rc) return rc;
    enqueue();
    rc = h->hip(hipStreamEndCapture(s, &graph), "hipStreamEndCapture");
    if (!rc) rc = h->hip(hipGraphInstantiate(&g, graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    if (graph) (void)hipGraphDestroy(graph);
    if (rc) {
      g = nullptr;
      return rc;
    }
  }
  return h->hip(hipGraphLaunch(g, s), "hipGraphLaunch");
}

// Copy on stream s.
int dcopy(lbm_handle* h, void* dst, const void* src, size_t bytes, hipStream_t s) {
  return h->hip(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
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
    rc = dcopy(h, w.ck_pop + c * popn, h->pop[n0 & 1], sizeof(float) * popn, s);
    if (!rc) rc = dcopy(h, w.ck_pos + c * 3 * nm, h->d_pos, sizeof(double) * 3 * nm, s);
    if (!rc) rc = dcopy(h, w.ck_bst + c * nb, h->d_bstate, sizeof(BeadState) * nb, s);
    if (!rc) rc = lbm_step(h, m);
    if (rc) return rc;
  }
  rc = lbm_get_swimmer_centres(h, XT.data());
  if (rc) return rc;
  *J = XT[3 * ad->swimmer] - X0[3 * ad->swimmer];

  // scratch views of the state for the recompute and the reverse sweep
  Dev dS = h->dev;
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
  for (const AdjSet& St : w.set) {
    if (!rc) rc = h->hip(hipMemsetAsync(St.stslab, 0x80, sizeof(int) * (size_t)K * h->ntiles, s), "hipMemsetAsync");
    if (!rc)
      rc = h->hip(hipMemsetAsync(St.nflag, 0x80, sizeof(int) * (size_t)(K + 1) * kNearSlots * w.nsc, s),
                  "hipMemsetAsync");
  }
  if (!rc) rc = h->hip(hipMemsetAsync(w.overflow, 0, sizeof(int), s), "hipMemsetAsync");
  if (rc) return rc;
  launch_adj_init(set_view(dS, w.set[0], popn), a, s);
  const int nblocks = (int)((h->nodes + kScBlock - 1) / kScBlock);
  // the recompute streams start after everything above
  rc = h->hip(hipEventRecord(w.start, s), "hipEventRecord");
  if (!rc) rc = h->hip(hipStreamWaitEvent(w.rmain, w.start, 0), "hipStreamWaitEvent");
  if (rc) return rc;

  // Recompute of segment c into set c % 2 on the recompute streams, after the
  // reverse sweep that last read that set (segment c + 2).
  auto recompute = [&](int64_t c) -> int {
    const int k = (int)(c & 1);
    const AdjSet& St = w.set[k];
    const int64_t n0 = t0 + c * K;
    const int m = (int)std::min<int64_t>(K, T - c * K);
    hipStream_t r = w.rmain;
    int e = LBM_OK;
    if (c + 2 < nck) e = h->hip(hipStreamWaitEvent(r, w.rev_done[k], 0), "hipStreamWaitEvent");
    if (!e) e = dcopy(h, St.P + (n0 & 1) * popn, w.ck_pop + c * popn, sizeof(float) * popn, r);
    if (!e) e = dcopy(h, St.pslab, w.ck_pos + c * 3 * nm, sizeof(double) * 3 * nm, r);
    if (!e) e = dcopy(h, St.bslab, w.ck_bst + c * nb, sizeof(BeadState) * nb, r);
    if (!e) e = h->hip(hipMemsetAsync(St.ncount, 0, sizeof(int) * (size_t)(K + 1) * 2, r), "hipMemsetAsync");
    if (e) return e;
    launch_set_step(St.step, n0, r);
    const Dev dv = set_view(dS, St, popn);
    e = enqueue_or_replay(h, w.rgraphs, 4 * (int64_t)m + k, r,
                          [&] { enqueue_recompute(h, w, St, dv, m, nblocks, r, w.rside); });
    if (!e) e = h->hip(hipEventRecord(w.rec_done[k], r), "hipEventRecord");
    return e;
  };
  rc = recompute(nck - 1);
  for (int64_t c = nck - 1; c >= 0 && !rc; --c) {
    if (c > 0) rc = recompute(c - 1);
    if (rc) break;
    const int k = (int)(c & 1);
    const int64_t n0 = t0 + c * K;
    const int m = (int)std::min<int64_t>(K, T - c * K);
    rc = h->hip(hipStreamWaitEvent(s, w.rec_done[k], 0), "hipStreamWaitEvent");
    if (rc) break;
    const Dev dv = set_view(dS, w.set[k], popn);
    const int64_t vkey = ((int64_t)ad->swimmer << 40) | (4 * (int64_t)m + 2 * (int64_t)(n0 & 1) + k);
    rc = enqueue_or_replay(h, w.vgraphs, vkey, s,
                           [&] { enqueue_reverse(h, w, w.set[k], dv, a, m, (int)(n0 & 1), nblocks, s, w.side); });
    if (!rc) rc = h->hip(hipEventRecord(w.rev_done[k], s), "hipEventRecord");
  }
  if (rc) return rc;
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
  if (h->dev.uavg) return h->fail(LBM_ESTATE, "adjoint: stop the velocity average first (lbm_average_begin(h, 0))");
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
