// Host runtime behind the C-ABI of include/lbmib.h: handle lifetime, bead
// meshes, device buffers, step sequencing (direct launches or replayed HIP
// graphs), observables and checkpoints.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/lbmib.h"
#include "common.h"

using namespace lbmib;

namespace {

constexpr int kGraphChunk = 32;  // steps per captured graph
constexpr int kReduceParts = 1024;
constexpr uint32_t kMagic = 0x4c424d31;  // "LBM1"

// ---- meshes ------------------------------------------------------------------
struct Mesh {
  std::vector<double> v;  // [nv][3], unit sphere
  std::vector<int> t;     // [ntri][3], counter-clockwise seen from outside
};

void unit(double* p) {
  const double len = std::sqrt(p[0] * p[0] + p[1] * p[1] + p[2] * p[2]);
  p[0] = p[0] / len;
  p[1] = p[1] / len;
  p[2] = p[2] / len;
}

// Icosahedron refined `level` times (paper Sec. 2.2): every triangle (a,b,c)
// splits into (a,ab,ca), (b,bc,ab), (c,ca,bc), (ab,bc,ca) with the edge
// midpoints created in the order ab, bc, ca and projected onto the unit
// sphere.  The base solid has vertices at the cyclic permutations of
// (0, +-1, +-golden ratio), which makes the mesh mirror symmetric in x, y, z.
Mesh icosphere(int level) {
  const double g = 1.6180339887498948482;
  Mesh M;
  const double base[12][3] = {{-1, g, 0}, {1, g, 0}, {-1, -g, 0}, {1, -g, 0},
                              {0, -1, g}, {0, 1, g}, {0, -1, -g}, {0, 1, -g},
                              {g, 0, -1}, {g, 0, 1}, {-g, 0, -1}, {-g, 0, 1}};
  const int faces[20][3] = {{0, 11, 5}, {0, 5, 1},  {0, 1, 7},   {0, 7, 10}, {0, 10, 11},
                            {1, 5, 9},  {5, 11, 4}, {11, 10, 2}, {10, 7, 6}, {7, 1, 8},
                            {3, 9, 4},  {3, 4, 2},  {3, 2, 6},   {3, 6, 8},  {3, 8, 9},
                            {4, 9, 5},  {2, 4, 11}, {6, 2, 10},  {8, 6, 7},  {9, 8, 1}};
  for (auto& p : base) {
    double q[3] = {p[0], p[1], p[2]};
    unit(q);
    M.v.insert(M.v.end(), q, q + 3);
  }
  for (auto& f : faces) M.t.insert(M.t.end(), f, f + 3);
  for (int l = 0; l < level; ++l) {
    std::unordered_map<uint64_t, int> mid;
    auto get = [&](int a, int b) {
      const uint64_t key = (uint64_t)std::min(a, b) << 32 | (uint32_t)std::max(a, b);
      auto it = mid.find(key);
      if (it != mid.end()) return it->second;
      const int id = (int)(M.v.size() / 3);
      double q[3];
      for (int k = 0; k < 3; ++k) q[k] = (M.v[3 * a + k] + M.v[3 * b + k]) * 0.5;
      unit(q);
      M.v.insert(M.v.end(), q, q + 3);
      mid.emplace(key, id);
      return id;
    };
    std::vector<int> nt;
    nt.reserve(M.t.size() * 4);
    for (size_t f = 0; f < M.t.size(); f += 3) {
      const int a = M.t[f], b = M.t[f + 1], c = M.t[f + 2];
      const int ab = get(a, b), bc = get(b, c), ca = get(c, a);
      const int add[12] = {a, ab, ca, b, bc, ab, c, ca, bc, ab, bc, ca};
      nt.insert(nt.end(), add, add + 12);
    }
    M.t.swap(nt);
  }
  return M;
}

double dihedral(const double* x1, const double* x2, const double* x3, const double* x4) {
  const double e[3] = {x2[0] - x1[0], x2[1] - x1[1], x2[2] - x1[2]};
  const double a[3] = {x3[0] - x1[0], x3[1] - x1[1], x3[2] - x1[2]};
  const double b[3] = {x4[0] - x2[0], x4[1] - x2[1], x4[2] - x2[2]};
  const double nA[3] = {e[1] * a[2] - e[2] * a[1], e[2] * a[0] - e[0] * a[2], e[0] * a[1] - e[1] * a[0]};
  const double nB[3] = {-(e[1] * b[2] - e[2] * b[1]), -(e[2] * b[0] - e[0] * b[2]),
                        -(e[0] * b[1] - e[1] * b[0])};
  const double E = std::sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  const double c[3] = {nA[1] * nB[2] - nA[2] * nB[1], nA[2] * nB[0] - nA[0] * nB[2],
                       nA[0] * nB[1] - nA[1] * nB[0]};
  return std::atan2((c[0] * e[0] + c[1] * e[1] + c[2] * e[2]) / E,
                    nA[0] * nB[0] + nA[1] * nB[1] + nA[2] * nB[2]);
}

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

const char* kErrNames[] = {"ok", "invalid argument", "out of memory", "HIP runtime error",
                           "call not allowed in this state", "non-finite conserved sums",
                           "file I/O error", "bead outgrew its reserved tile region"};

}  // namespace

struct lbm_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  lbm_grid grid{};
  double tau = 1.0;
  int forcing = LBM_GUO, storage = LBM_FP32_SHIFTED, width = 3;
  float fp16_scale = 1.0f;
  bool use_graphs = true;
  std::string err;

  // host model
  std::vector<Box> boxes;
  std::vector<Bead> beads;
  std::vector<Swimmer> swimmers;
  std::vector<double> pos0;  // [nm][3] initial marker positions
  std::vector<int> marker_bead;
  std::vector<int> tri;      // [ntri][3] global vertex ids
  std::vector<double> G0;    // [ntri][3]
  std::vector<double> hingeth0;
  std::vector<int> hinge;    // [nh][4]
  int nm = 0;
  int64_t nodes = 0, pstride = 0;
  int ntiles = 0, sc_blocks = 0, spread_blocks = 0, out_blocks = 0;
  int sc_block = 256, sc_remap = 1, sc_resident = 0;  // stream-collide launch shape
  int ncu = 256;                                        // compute units of the device
  bool uploaded = false, stepped = false;
  int64_t host_step = 0;  // steps enqueued

  // device buffers
  void* pop[2] = {nullptr, nullptr};
  float *F = nullptr, *u = nullptr, *uout = nullptr;
  int* stamp = nullptr;
  Box* d_boxes = nullptr;
  int* d_block_box = nullptr;
  int64_t* d_step = nullptr;
  double* d_pos = nullptr;
  float *d_U = nullptr, *d_fm = nullptr;
  Bead* d_beads = nullptr;
  BeadState* d_bstate = nullptr;
  Swimmer* d_swimmers = nullptr;
  int *d_marker_bead = nullptr, *d_tri = nullptr, *d_hinge = nullptr;
  double *d_G0 = nullptr, *d_theta0 = nullptr;
  float *d_G0inv = nullptr, *d_A0 = nullptr, *d_idet = nullptr;
  int *d_lane_elem = nullptr, *d_lane_v = nullptr;
  int* d_overflow = nullptr;
  int* d_spread_bead = nullptr;
  int *d_near = nullptr, *d_near_list = nullptr, *d_near_count = nullptr;
  bool need_prologue = true;
  hipStream_t side = nullptr;      // IBM chain, forked from `stream` every step
  std::vector<hipEvent_t> fork_join;
  double *d_partial = nullptr, *d_out = nullptr, *d_centres = nullptr;
  std::vector<void*> allocs;

  Dev dev{};
  hipGraphExec_t g_chunk = nullptr, g_one = nullptr;

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
    T* p = dev_alloc<T>(n, rc);
    if (p) allocs.push_back(p);
    return p;
  }
};

namespace {

int element_bytes(const lbm_handle* h) { return h->storage == LBM_FP16_SHIFTED ? 2 : 4; }

// Candidate tiles reserved per axis for a bead: the node span of its stencils
// with 25% room for deformation, in tiles, for any alignment.
int reserved_tiles(double radius, int width, int T) {
  const int span = (int)std::floor(2.0 * radius * 1.25) + width + 2;
  return std::min(T, (span + kTile - 2) / kTile + 1);
}

// Stream-collide block geometry and the bound on near blocks: per bead the
// marked node box is its reserved tile span plus two nodes each side.
void set_near_bounds(lbm_handle* h) {
  Dev& d = h->dev;
  d.nsc = h->sc_blocks;
  d.sc_bs = h->sc_block;
  int64_t mx = 0;
  const Box& B = h->boxes[0];
  for (const Bead& b : h->beads) {
    const int64_t sx = std::min<int64_t>(b.tiles_x * kTile + 4, B.nx);
    const int64_t sy = std::min<int64_t>(b.tiles_y * kTile + 4, B.ny);
    const int64_t sz = std::min<int64_t>(b.tiles_z * kTile + 4, B.nz);
    mx += sy * sz * (sx / h->sc_block + 2);
  }
  d.max_near = (int)std::max<int64_t>(1, std::min<int64_t>(mx, d.nsc));
}

int upload(lbm_handle* h) {
  if (h->uploaded) return LBM_OK;
  int rc = LBM_OK;
  const int nm = h->nm;
  const int ntri = (int)h->tri.size() / 3, nh = (int)h->hinge.size() / 4;
  // per-triangle reference geometry and per-vertex incidence lists
  std::vector<double> G0(3 * (size_t)ntri);
  std::vector<float> Gi(3 * (size_t)ntri), A0(ntri), idet(ntri);
  std::vector<int> tri(3 * (size_t)ntri), hinge(4 * (size_t)nh);
  std::vector<std::vector<int>> vt(nm), vh(nm);
  for (int t = 0; t < ntri; ++t) {
    const double G11 = h->G0[3 * t], G12 = h->G0[3 * t + 1], G22 = h->G0[3 * t + 2];
    const double det = G11 * G22 - G12 * G12;
    G0[t] = G11;
    G0[ntri + t] = G12;
    G0[2 * ntri + t] = G22;
    Gi[t] = (float)(G22 / det);
    Gi[ntri + t] = (float)(-G12 / det);
    Gi[2 * ntri + t] = (float)(G11 / det);
    A0[t] = (float)(0.5 * std::sqrt(det));
    idet[t] = (float)(1.0 / det);
    for (int k = 0; k < 3; ++k) {
      tri[k * ntri + t] = h->tri[3 * t + k];
      vt[h->tri[3 * t + k]].push_back(3 * t + k);
    }
  }
  for (int e = 0; e < nh; ++e)
    for (int k = 0; k < 4; ++k) {
      hinge[k * nh + e] = h->hinge[4 * e + k];
      vh[h->hinge[4 * e + k]].push_back(4 * e + k);
    }
  std::vector<int> lane_elem(32 * (size_t)nm, -1);
  std::vector<int> lane_v(4 * 32 * (size_t)nm, 0);
  for (int m = 0; m < nm; ++m) {
    // the node-force kernel gives each node 8 triangle and 24 hinge lanes
    if (vt[m].size() > 8 || vh[m].size() > 24)
      return h->fail(LBM_EINVAL, "mesh node with more than 8 triangles or 24 hinges");
    for (size_t k = 0; k < vt[m].size(); ++k) {
      const int e = vt[m][k], t = e / 3;
      const size_t l = 32 * (size_t)m + k;
      lane_elem[l] = e;
      for (int q = 0; q < 3; ++q) lane_v[4 * l + q] = h->tri[3 * t + q];
    }
    for (size_t k = 0; k < vh[m].size(); ++k) {
      const int e = vh[m][k], hh = e / 4;
      const size_t l = 32 * (size_t)m + 8 + k;
      lane_elem[l] = e;
      for (int q = 0; q < 4; ++q) lane_v[4 * l + q] = h->hinge[4 * hh + q];
    }
  }
  std::vector<double> pos(3 * (size_t)nm);
  for (int m = 0; m < nm; ++m)
    for (int k = 0; k < 3; ++k) pos[(size_t)k * nm + m] = h->pos0[3 * (size_t)m + k];
  // spread candidate blocks
  std::vector<int> spread_bead;
  for (size_t b = 0; b < h->beads.size(); ++b) {
    Bead& B = h->beads[b];
    B.tile_block0 = (int)spread_bead.size();
    const int cnt = B.tiles_x * B.tiles_y * B.tiles_z;
    spread_bead.insert(spread_bead.end(), cnt, (int)b);
  }
  h->spread_blocks = (int)spread_bead.size();
  h->boxes[0].bead0 = 0;
  h->boxes[0].nbeads = (int)h->beads.size();

  auto put = [&](void* dst, const void* src, size_t bytes) {
    if (rc != LBM_OK || bytes == 0) return;
    rc = h->hip(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy");
  };
  h->d_pos = h->alloc<double>(3 * (size_t)nm, rc);
  h->d_U = h->alloc<float>(3 * (size_t)nm, rc);
  h->d_fm = h->alloc<float>(3 * (size_t)nm, rc);
  h->d_beads = h->alloc<Bead>(h->beads.size(), rc);
  h->d_bstate = h->alloc<BeadState>(h->beads.size(), rc);
  h->d_swimmers = h->alloc<Swimmer>(h->swimmers.size(), rc);
  h->d_marker_bead = h->alloc<int>(nm, rc);
  h->d_tri = h->alloc<int>(tri.size(), rc);
  h->d_G0 = h->alloc<double>(G0.size(), rc);
  h->d_G0inv = h->alloc<float>(Gi.size(), rc);
  h->d_A0 = h->alloc<float>(A0.size(), rc);
  h->d_idet = h->alloc<float>(idet.size(), rc);
  h->d_hinge = h->alloc<int>(hinge.size(), rc);
  h->d_theta0 = h->alloc<double>(2 * h->hingeth0.size(), rc);
  h->d_lane_elem = h->alloc<int>(lane_elem.size(), rc);
  h->d_lane_v = h->alloc<int>(lane_v.size(), rc);
  h->d_spread_bead = h->alloc<int>(spread_bead.size(), rc);
  h->d_centres = h->alloc<double>(3 * h->beads.size(), rc);
  // near-block buffers, sized for the smallest stream-collide block (128)
  const int64_t nsc_max = (h->nodes + 127) / 128;
  h->d_near = h->alloc<int>(2 * (size_t)nsc_max, rc);
  h->d_near_list = h->alloc<int>(2 * (size_t)nsc_max, rc);
  h->d_near_count = h->alloc<int>(2, rc);
  if (rc != LBM_OK) return h->fail(rc, "device allocation for markers failed");
  put(h->d_boxes, h->boxes.data(), sizeof(Box) * h->boxes.size());
  put(h->d_pos, pos.data(), sizeof(double) * pos.size());
  if (rc == LBM_OK && nm > 0) {
    rc = h->hip(hipMemset(h->d_U, 0, sizeof(float) * 3 * nm), "hipMemset");
    if (rc == LBM_OK) rc = h->hip(hipMemset(h->d_fm, 0, sizeof(float) * 3 * nm), "hipMemset");
  }
  put(h->d_beads, h->beads.data(), sizeof(Bead) * h->beads.size());
  {
    // initial bead state: centre of the stress-free mesh, reference volume
    std::vector<BeadState> st(h->beads.size());
    for (size_t b = 0; b < h->beads.size(); ++b) {
      const Bead& B = h->beads[b];
      double c[3] = {0, 0, 0};
      for (int i = 0; i < B.nv; ++i)
        for (int q = 0; q < 3; ++q) c[q] += h->pos0[3 * (size_t)(B.first + i) + q];
      for (int q = 0; q < 3; ++q) st[b].c[q] = c[q] / B.nv;
      st[b].V = B.V0;
    }
    put(h->d_bstate, st.data(), sizeof(BeadState) * st.size());
  }
  put(h->d_swimmers, h->swimmers.data(), sizeof(Swimmer) * h->swimmers.size());
  put(h->d_marker_bead, h->marker_bead.data(), sizeof(int) * nm);
  put(h->d_tri, tri.data(), sizeof(int) * tri.size());
  put(h->d_G0, G0.data(), sizeof(double) * G0.size());
  put(h->d_G0inv, Gi.data(), sizeof(float) * Gi.size());
  put(h->d_A0, A0.data(), sizeof(float) * A0.size());
  put(h->d_idet, idet.data(), sizeof(float) * idet.size());
  put(h->d_hinge, hinge.data(), sizeof(int) * hinge.size());
  {
    std::vector<double> cs(2 * (size_t)nh);
    for (int e = 0; e < nh; ++e) {
      cs[e] = std::cos(h->hingeth0[e]);
      cs[nh + e] = std::sin(h->hingeth0[e]);
    }
    put(h->d_theta0, cs.data(), sizeof(double) * cs.size());
  }
  put(h->d_lane_elem, lane_elem.data(), sizeof(int) * lane_elem.size());
  put(h->d_lane_v, lane_v.data(), sizeof(int) * lane_v.size());
  put(h->d_spread_bead, spread_bead.data(), sizeof(int) * spread_bead.size());
  if (rc != LBM_OK) return rc;

  Dev& d = h->dev;
  d.pos = h->d_pos;
  d.U = h->d_U;
  d.fm = h->d_fm;
  d.nm = nm;
  d.beads = h->d_beads;
  d.nbeads = (int)h->beads.size();
  d.bstate = h->d_bstate;
  d.swimmers = h->d_swimmers;
  d.nswimmers = (int)h->swimmers.size();
  d.marker_bead = h->d_marker_bead;
  d.tri = h->d_tri;
  d.G0 = h->d_G0;
  d.G0inv = h->d_G0inv;
  d.A0 = h->d_A0;
  d.idetG0 = h->d_idet;
  d.hinge = h->d_hinge;
  d.th0cs = h->d_theta0;
  d.ntri = ntri;
  d.nh = nh;
  d.lane_elem = h->d_lane_elem;
  d.lane_v = reinterpret_cast<const int4*>(h->d_lane_v);
  d.spread_blocks = h->spread_blocks;
  d.spread_bead = h->d_spread_bead;
  d.near = h->d_near;
  d.near_list = h->d_near_list;
  d.near_count = h->d_near_count;
  d.tile_box = nullptr;
  set_near_bounds(h);
  if (!h->swimmers.empty()) {
    rc = h->hip(hipStreamCreate(&h->side), "hipStreamCreate");
    if (rc) return rc;
    h->fork_join.resize(2 * kGraphChunk);
    for (auto& e : h->fork_join) {
      rc = h->hip(hipEventCreateWithFlags(&e, hipEventDisableTiming), "hipEventCreateWithFlags");
      if (rc) return rc;
    }
  }
  h->uploaded = true;
  h->need_prologue = true;
  return LBM_OK;
}

// Two timing events for one launch (nullptr when timing is off).
void timing_pair(lbm_handle* h, hipEvent_t* e0, hipEvent_t* e1) {
  *e0 = *e1 = nullptr;
  if (!h->timing) return;
  if (h->ev_used + 2 > h->ev_pool.size()) {
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      (void)hipEventCreate(&e);
      h->ev_pool.push_back(e);
    }
  }
  *e0 = h->ev_pool[h->ev_used++];
  *e1 = h->ev_pool[h->ev_used++];
}

// Enqueue `count` steps.  Without swimmers each step is one full-grid
// stream-collide launch.  With swimmers, step k forks the IBM chain onto the
// side stream -- advection of the previous step, bead statistics, nodal
// forces, spreading -- while the main stream streams and collides every node
// away from the swimmers; the active-tile launch then joins both and advances
// the step counter.  The last step's advection closes the sequence, so the
// markers are current whenever the sequence ends.
void enqueue_steps(lbm_handle* h, int64_t count) {
  Dev d = h->dev;
  if (h->swimmers.empty()) {
    for (int64_t i = 0; i < count; ++i) {
      d.sub = (int)i;
      hipEvent_t e0, e1;
      timing_pair(h, &e0, &e1);
      launch_stream_collide(d, h->storage, kLaunchAll, h->sc_block, h->sc_blocks, h->sc_remap, 0, h->ncu, h->stream,
                            e0, e1);
    }
    launch_tick(d, (int)count, h->stream);
    return;
  }
  if (h->sc_resident < 0) {
    // serial order: the immersed-boundary chain, then the full grid
    for (int64_t i = 0; i < count; ++i) {
      d.sub = (int)i;
      launch_bead_stats(d, 0, h->stream);
      launch_vertex_forces(d, h->stream);
      launch_spread(d, h->stream);
      hipEvent_t e0, e1;
      timing_pair(h, &e0, &e1);
      launch_stream_collide(d, h->storage, kLaunchAll, h->sc_block, h->sc_blocks, h->sc_remap, 0, h->ncu, h->stream,
                            e0, e1);
      d.sub = (int)i + 1;
      launch_interp_advance(d, h->stream);
    }
    launch_tick(d, (int)count, h->stream);
    return;
  }
  for (int64_t i = 0; i < count; ++i) {
    hipEvent_t fork = h->fork_join[2 * (i % kGraphChunk)], join = h->fork_join[2 * (i % kGraphChunk) + 1];
    (void)hipEventRecord(fork, h->stream);
    (void)hipStreamWaitEvent(h->side, fork, 0);
    d.sub = (int)i;
    if (i > 0) launch_interp_advance(d, h->side);
    launch_bead_stats(d, 0, h->side);
    launch_vertex_forces(d, h->side);
    launch_spread(d, h->side);
    (void)hipEventRecord(join, h->side);
    hipEvent_t e0, e1;
    timing_pair(h, &e0, &e1);
    launch_stream_collide(d, h->storage, kLaunchBulk, h->sc_block, h->sc_blocks, h->sc_remap, h->sc_resident,
                          h->ncu, h->stream, e0, e1);
    (void)hipStreamWaitEvent(h->stream, join, 0);
    timing_pair(h, &e0, &e1);
    launch_stream_collide(d, h->storage, kLaunchActive, h->sc_block, h->sc_blocks, 0, 0, h->ncu, h->stream, e0, e1);
  }
  d.sub = (int)count;
  launch_interp_advance(d, h->stream);
  launch_tick(d, (int)count, h->stream);
}

// Before stepping resumes: bead regions of the current markers and the near
// tiles under the previous step's parity, so the first step can split the
// grid into bulk and active parts.  Eager, never captured.
int prologue(lbm_handle* h) {
  if (!h->need_prologue || h->swimmers.empty()) return LBM_OK;
  int rc = h->hip(hipMemsetAsync(h->d_near, 0x80, sizeof(int) * 2 * h->dev.nsc, h->stream), "hipMemsetAsync");
  if (!rc) rc = h->hip(hipMemsetAsync(h->d_near_count, 0, sizeof(int) * 2, h->stream), "hipMemsetAsync");
  if (rc) return rc;
  launch_bead_stats(h->dev, -1, h->stream);
  rc = h->hip(hipGetLastError(), "prologue launch");
  if (!rc) h->need_prologue = false;
  return rc;
}

int capture(lbm_handle* h, int steps, hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  int rc = h->hip(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
  if (rc) return rc;
  enqueue_steps(h, steps);
  rc = h->hip(hipStreamEndCapture(h->stream, &g), "hipStreamEndCapture");
  if (rc) return rc;
  rc = h->hip(hipGraphInstantiate(out, g, nullptr, nullptr, 0), "hipGraphInstantiate");
  (void)hipGraphDestroy(g);
  return rc;
}

void harvest_timing(lbm_handle* h) {
  if (h->ev_used == 0) return;
  (void)hipStreamSynchronize(h->stream);
  for (size_t i = 0; i + 1 < h->ev_used; i += 2) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, h->ev_pool[i], h->ev_pool[i + 1]);
    h->timed_ms += ms;
    h->timed_launches += 1;
  }
  h->ev_used = 0;
}

int check_overflow(lbm_handle* h) {
  if (!h->uploaded || h->swimmers.empty()) return LBM_OK;
  int ov = 0;
  int rc = h->hip(hipMemcpyAsync(&ov, h->d_overflow, sizeof(int), hipMemcpyDeviceToHost, h->stream),
                  "hipMemcpyAsync");
  if (rc) return rc;
  rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  if (ov & 1) return h->fail(LBM_EOVERFLOW, "a bead outgrew its reserved tile region");
  if (ov & 2) return h->fail(LBM_EOVERFLOW, "near-block list overflow");
  return LBM_OK;
}

}  // namespace

// =============================================================================
extern "C" {

const char* lbm_strerror(int code) {
  const int i = -code;
  if (i < 0 || i >= (int)(sizeof(kErrNames) / sizeof(kErrNames[0]))) return "unknown error";
  return kErrNames[i];
}

const char* lbm_last_error(const lbm_handle* h) { return h ? h->err.c_str() : "null handle"; }

int lbm_create(const lbm_grid* grid, double tau, int forcing, const lbm_opts* opts,
               lbm_handle** out) {
  if (!out || !grid) return LBM_EINVAL;
  *out = nullptr;
  if (!(tau > 0.5) || !std::isfinite(tau)) return LBM_EINVAL;
  if (grid->nx < 16 || grid->ny < 16 || grid->nz < 16) return LBM_EINVAL;
  if ((int64_t)grid->nx * grid->ny * grid->nz >= (int64_t)1 << 31) return LBM_EINVAL;
  if (forcing != LBM_GUO && forcing != LBM_SHAN_CHEN) return LBM_EINVAL;
  lbm_opts o{LBM_FP32_SHIFTED, 3, 1.0f, 1, nullptr};
  if (opts) o = *opts;
  if (o.storage != LBM_FP32_SHIFTED && o.storage != LBM_FP16_SHIFTED) return LBM_EINVAL;
  if (o.delta_width < 2 || o.delta_width > 4) return LBM_EINVAL;
  if (o.fp16_scale == 0.0f) o.fp16_scale = 1.0f;
  {
    int e;
    std::frexp(o.fp16_scale, &e);
    if (!(o.fp16_scale > 0.0f) || std::ldexp(1.0, e - 1) != o.fp16_scale) return LBM_EINVAL;
  }
  auto* h = new lbm_handle();
  h->grid = *grid;
  h->tau = tau;
  h->forcing = forcing;
  h->storage = o.storage;
  h->width = o.delta_width;
  h->fp16_scale = o.fp16_scale;
  h->use_graphs = o.use_graphs != 0;
  int rc = h->hip(hipGetDevice(&h->device), "hipGetDevice");
  if (!rc) rc = h->hip(hipDeviceGetAttribute(&h->ncu, hipDeviceAttributeMultiprocessorCount, h->device),
                      "hipDeviceGetAttribute");
  if (rc) {
    delete h;
    return rc;
  }
  if (o.stream) {
    h->stream = static_cast<hipStream_t>(o.stream);
  } else {
    rc = h->hip(hipStreamCreate(&h->stream), "hipStreamCreate");
    if (rc) {
      delete h;
      return rc;
    }
    h->own_stream = true;
  }
  Box B{};
  B.nx = grid->nx;
  B.ny = grid->ny;
  B.nz = grid->nz;
  B.tx = (B.nx + kTile - 1) / kTile;
  B.ty = (B.ny + kTile - 1) / kTile;
  B.tz = (B.nz + kTile - 1) / kTile;
  B.node0 = 0;
  B.n = (int64_t)B.nx * B.ny * B.nz;
  B.tile0 = 0;
  B.block0 = 0;
  B.forcing = forcing;
  B.tau = (float)tau;
  B.omega = (float)(1.0 / tau);
  h->boxes.push_back(B);
  h->nodes = B.n;
  h->pstride = (B.n + 127) / 128 * 128;
  h->ntiles = B.tx * B.ty * B.tz;
  h->out_blocks = (int)((B.n + kScBlock - 1) / kScBlock);
  h->sc_blocks = (int)((B.n + h->sc_block - 1) / h->sc_block);

  const size_t eb = element_bytes(h);
  h->pop[0] = h->alloc<char>(eb * kQ * h->pstride, rc);
  h->pop[1] = h->alloc<char>(eb * kQ * h->pstride, rc);
  h->F = h->alloc<float>(3 * h->pstride, rc);
  h->u = h->alloc<float>(3 * h->pstride, rc);
  h->stamp = h->alloc<int>(h->ntiles, rc);
  h->d_boxes = h->alloc<Box>(1, rc);
  h->d_step = h->alloc<int64_t>(1, rc);
  h->d_overflow = h->alloc<int>(1, rc);
  h->d_partial = h->alloc<double>(4 * kReduceParts, rc);
  h->d_out = h->alloc<double>(4, rc);
  if (rc) {
    lbm_destroy(h);
    return LBM_ENOMEM;
  }
  rc = h->hip(hipMemset(h->pop[0], 0, eb * kQ * h->pstride), "hipMemset");
  if (!rc) rc = h->hip(hipMemset(h->pop[1], 0, eb * kQ * h->pstride), "hipMemset");
  if (!rc) rc = h->hip(hipMemset(h->F, 0, sizeof(float) * 3 * h->pstride), "hipMemset");
  if (!rc) rc = h->hip(hipMemset(h->u, 0, sizeof(float) * 3 * h->pstride), "hipMemset");
  if (!rc) rc = h->hip(hipMemset(h->stamp, 0x80, sizeof(int) * h->ntiles), "hipMemset");
  if (!rc) rc = h->hip(hipMemset(h->d_step, 0, sizeof(int64_t)), "hipMemset");
  if (!rc) rc = h->hip(hipMemset(h->d_overflow, 0, sizeof(int)), "hipMemset");
  if (!rc) rc = h->hip(hipMemcpy(h->d_boxes, h->boxes.data(), sizeof(Box), hipMemcpyHostToDevice), "hipMemcpy");
  if (!rc) rc = h->hip(hipDeviceSynchronize(), "hipDeviceSynchronize");
  if (rc) {
    lbm_destroy(h);
    return rc;
  }
  Dev& d = h->dev;
  d.pop[0] = h->pop[0];
  d.pop[1] = h->pop[1];
  d.pstride = h->pstride;
  d.F = h->F;
  d.u = h->u;
  d.stamp = h->stamp;
  d.boxes = h->d_boxes;
  d.nboxes = 1;
  d.block_box = nullptr;
  d.step = h->d_step;
  d.sub = 0;
  d.fp16_scale = h->fp16_scale;
  d.fp16_inv = 1.0f / h->fp16_scale;
  d.width = h->width;
  d.overflow = h->d_overflow;
  *out = h;
  return LBM_OK;
}

int lbm_destroy(lbm_handle* h) {
  if (!h) return LBM_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->g_chunk) (void)hipGraphExecDestroy(h->g_chunk);
  if (h->g_one) (void)hipGraphExecDestroy(h->g_one);
  for (auto e : h->ev_pool) (void)hipEventDestroy(e);
  for (auto e : h->fork_join) (void)hipEventDestroy(e);
  if (h->side) (void)hipStreamDestroy(h->side);
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return LBM_OK;
}

int lbm_swimmer_add(lbm_handle* h, const lbm_bead_desc beads[3], const lbm_spring_desc springs[2],
                    const lbm_actuation_desc* act, int32_t* id) {
  if (!h || !beads || !springs || !act) return LBM_EINVAL;
  if (h->stepped || h->uploaded) return h->fail(LBM_ESTATE, "swimmers must be added before the first step");
  if (!(act->period > 0)) return h->fail(LBM_EINVAL, "actuation period must be positive");
  const int minedge = std::min(h->grid.nx, std::min(h->grid.ny, h->grid.nz));
  for (int k = 0; k < 3; ++k) {
    if (!(beads[k].radius > 0) || beads[k].level < 0 || beads[k].level > 5)
      return h->fail(LBM_EINVAL, "bead radius must be positive and level in 0..5");
    if (2.0 * beads[k].radius * 1.25 + h->width + 2 > minedge / 1.5)
      return h->fail(LBM_EINVAL, "bead too large for the box");
  }
  Swimmer S{};
  const int sw = (int)h->swimmers.size();
  const Box& B = h->boxes[0];
  for (int k = 0; k < 3; ++k) {
    const lbm_bead_desc& bd = beads[k];
    const Mesh M = icosphere(bd.level);
    const int nv = (int)M.v.size() / 3, nt = (int)M.t.size() / 3;
    Bead b{};
    b.first = h->nm;
    b.nv = nv;
    b.tri0 = (int)h->tri.size() / 3;
    b.ntri = nt;
    b.box = 0;
    b.swimmer = sw;
    b.slot = k;
    b.tiles_x = reserved_tiles(bd.radius, h->width, B.tx);
    b.tiles_y = reserved_tiles(bd.radius, h->width, B.ty);
    b.tiles_z = reserved_tiles(bd.radius, h->width, B.tz);
    b.ks = (float)bd.kappa_s;
    b.C = (float)bd.C;
    b.kt = (float)(2.0 * bd.kappa_b / std::sqrt(3.0));
    b.kv = (float)bd.kappa_v;
    std::vector<double> x(3 * (size_t)nv);
    for (int i = 0; i < nv; ++i)
      for (int q = 0; q < 3; ++q) x[3 * i + q] = bd.centre[q] + bd.radius * M.v[3 * i + q];
    // reference metric per triangle
    double cx = 0, cy = 0, cz = 0;
    for (int i = 0; i < nv; ++i) {
      cx += x[3 * i];
      cy += x[3 * i + 1];
      cz += x[3 * i + 2];
    }
    cx /= nv;
    cy /= nv;
    cz /= nv;
    double V = 0;
    for (int t = 0; t < nt; ++t) {
      const double* p0 = &x[3 * M.t[3 * t]];
      const double* p1 = &x[3 * M.t[3 * t + 1]];
      const double* p2 = &x[3 * M.t[3 * t + 2]];
      const double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
      const double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
      h->G0.push_back(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
      h->G0.push_back(e1[0] * e2[0] + e1[1] * e2[1] + e1[2] * e2[2]);
      h->G0.push_back(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
      for (int q = 0; q < 3; ++q) h->tri.push_back(b.first + M.t[3 * t + q]);
      const double a[3] = {p0[0] - cx, p0[1] - cy, p0[2] - cz};
      const double bb[3] = {p1[0] - cx, p1[1] - cy, p1[2] - cz};
      const double c[3] = {p2[0] - cx, p2[1] - cy, p2[2] - cz};
      V += a[0] * (bb[1] * c[2] - bb[2] * c[1]) + a[1] * (bb[2] * c[0] - bb[0] * c[2]) +
           a[2] * (bb[0] * c[1] - bb[1] * c[0]);
    }
    b.V0 = V / 6.0;
    // hinges: each undirected edge once, from the face holding it as lo->hi
    std::unordered_map<uint64_t, int> opposite;  // directed edge a->b -> third vertex
    for (int t = 0; t < nt; ++t)
      for (int q = 0; q < 3; ++q) {
        const uint32_t a = M.t[3 * t + q], c = M.t[3 * t + (q + 1) % 3];
        opposite[(uint64_t)a << 32 | c] = M.t[3 * t + (q + 2) % 3];
      }
    for (int t = 0; t < nt; ++t)
      for (int q = 0; q < 3; ++q) {
        const int a = M.t[3 * t + q], c = M.t[3 * t + (q + 1) % 3];
        if (a > c) continue;
        const int x3 = M.t[3 * t + (q + 2) % 3];
        const int x4 = opposite.at((uint64_t)(uint32_t)c << 32 | (uint32_t)a);
        const int ids[4] = {a, c, x3, x4};
        for (int r = 0; r < 4; ++r) h->hinge.push_back(b.first + ids[r]);
        h->hingeth0.push_back(dihedral(&x[3 * a], &x[3 * c], &x[3 * x3], &x[3 * x4]));
      }
    h->pos0.insert(h->pos0.end(), x.begin(), x.end());
    h->marker_bead.insert(h->marker_bead.end(), nv, (int)h->beads.size());
    S.bead[k] = (int)h->beads.size();
    h->beads.push_back(b);
    h->nm += nv;
  }
  for (int s = 0; s < 2; ++s) {
    S.k[s] = springs[s].k;
    S.L0[s] = springs[s].L0;
  }
  S.A = act->A;
  S.B = act->B;
  S.omega = 2.0 * M_PI / act->period;
  S.alpha = act->alpha;
  S.phi0 = act->phi0;
  h->swimmers.push_back(S);
  if (id) *id = sw;
  return LBM_OK;
}

int lbm_set_body_force(lbm_handle* h, const double g[3]) {
  if (!h || !g) return LBM_EINVAL;
  for (auto& B : h->boxes) {
    B.gx = (float)g[0];
    B.gy = (float)g[1];
    B.gz = (float)g[2];
  }
  int rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  return h->hip(hipMemcpy(h->d_boxes, h->boxes.data(), sizeof(Box) * h->boxes.size(),
                          hipMemcpyHostToDevice), "hipMemcpy");
}

int lbm_step(lbm_handle* h, int64_t n) {
  if (!h || n < 0) return LBM_EINVAL;
  int rc = upload(h);
  if (rc) return rc;
  rc = prologue(h);
  if (rc) return rc;
  h->stepped = true;
  if (h->timing || !h->use_graphs) {
    for (int64_t done = 0; done < n; done += kGraphChunk) enqueue_steps(h, std::min<int64_t>(kGraphChunk, n - done));
    h->host_step += n;
    if (h->timing && h->ev_used > 256) harvest_timing(h);
    return h->hip(hipGetLastError(), "kernel launch");
  }
  int64_t left = n;
  if (left >= kGraphChunk && !h->g_chunk) {
    rc = capture(h, kGraphChunk, &h->g_chunk);
    if (rc) return rc;
  }
  while (left >= kGraphChunk) {
    rc = h->hip(hipGraphLaunch(h->g_chunk, h->stream), "hipGraphLaunch");
    if (rc) return rc;
    left -= kGraphChunk;
  }
  if (left > 0 && !h->g_one) {
    rc = capture(h, 1, &h->g_one);
    if (rc) return rc;
  }
  for (; left > 0; --left) {
    rc = h->hip(hipGraphLaunch(h->g_one, h->stream), "hipGraphLaunch");
    if (rc) return rc;
  }
  h->host_step += n;
  return LBM_OK;
}

int lbm_sync(lbm_handle* h) {
  if (!h) return LBM_EINVAL;
  int rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  return check_overflow(h);
}

int64_t lbm_time(const lbm_handle* h) { return h ? h->host_step : -1; }
int32_t lbm_n_markers(const lbm_handle* h) { return h ? h->nm : -1; }
int32_t lbm_n_swimmers(const lbm_handle* h) { return h ? (int32_t)h->swimmers.size() : -1; }

int lbm_get_bead_centres(lbm_handle* h, double* out) {
  if (!h || !out) return LBM_EINVAL;
  if (h->beads.empty()) return LBM_OK;
  int rc = upload(h);
  if (rc) return rc;
  launch_bead_centres(h->dev, h->d_centres, h->stream);
  rc = h->hip(hipMemcpyAsync(out, h->d_centres, sizeof(double) * 3 * h->beads.size(),
                             hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync");
  if (rc) return rc;
  rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  return check_overflow(h);
}

int lbm_get_swimmer_centres(lbm_handle* h, double* out) {
  if (!h || !out) return LBM_EINVAL;
  std::vector<double> R(3 * h->beads.size());
  int rc = lbm_get_bead_centres(h, R.data());
  if (rc) return rc;
  for (size_t s = 0; s < h->swimmers.size(); ++s)
    for (int q = 0; q < 3; ++q) {
      const Swimmer& S = h->swimmers[s];
      out[3 * s + q] = (R[3 * S.bead[0] + q] + R[3 * S.bead[1] + q] + R[3 * S.bead[2] + q]) / 3.0;
    }
  return LBM_OK;
}

int lbm_get_markers(lbm_handle* h, double* out) {
  if (!h || !out) return LBM_EINVAL;
  if (h->nm == 0) return LBM_OK;
  int rc = upload(h);
  if (rc) return rc;
  std::vector<double> tmp(3 * (size_t)h->nm);
  rc = h->hip(hipMemcpyAsync(tmp.data(), h->d_pos, sizeof(double) * tmp.size(), hipMemcpyDeviceToHost,
                             h->stream), "hipMemcpyAsync");
  if (!rc) rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  for (int m = 0; m < h->nm; ++m)
    for (int q = 0; q < 3; ++q) out[3 * (size_t)m + q] = tmp[(size_t)q * h->nm + m];
  return LBM_OK;
}

static int get_marker_f32(lbm_handle* h, const float* src, double* out) {
  if (!h || !out) return LBM_EINVAL;
  if (h->nm == 0) return LBM_OK;
  int rc = upload(h);
  if (rc) return rc;
  std::vector<float> tmp(3 * (size_t)h->nm);
  rc = h->hip(hipMemcpyAsync(tmp.data(), src, sizeof(float) * tmp.size(), hipMemcpyDeviceToHost,
                             h->stream), "hipMemcpyAsync");
  if (!rc) rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  for (int m = 0; m < h->nm; ++m)
    for (int q = 0; q < 3; ++q) out[3 * (size_t)m + q] = tmp[(size_t)q * h->nm + m];
  return LBM_OK;
}

int lbm_get_marker_velocities(lbm_handle* h, double* out) {
  if (!h) return LBM_EINVAL;
  int rc = upload(h);
  if (rc) return rc;
  return get_marker_f32(h, h->d_U, out);
}

int lbm_get_marker_forces(lbm_handle* h, double* out) {
  if (!h) return LBM_EINVAL;
  int rc = upload(h);
  if (rc) return rc;
  return get_marker_f32(h, h->d_fm, out);
}

static int get_macro(lbm_handle* h, float* dst, int on_device, bool vel) {
  if (!h || !dst) return LBM_EINVAL;
  const size_t comps = vel ? 3 : 1;
  const size_t bytes = sizeof(float) * comps * h->nodes;
  float* target = dst;
  int rc = LBM_OK;
  if (!on_device) {
    if (!h->uout) {
      h->uout = h->alloc<float>(3 * h->nodes, rc);
      if (rc) return h->fail(rc, "velocity staging allocation failed");
    }
    target = h->uout;
  }
  launch_velocity(h->dev, h->storage, h->out_blocks, vel ? target : nullptr, vel ? nullptr : target,
                  h->stream);
  rc = h->hip(hipGetLastError(), "k_velocity launch");
  if (rc) return rc;
  if (!on_device) {
    rc = h->hip(hipMemcpyAsync(dst, target, bytes, hipMemcpyDeviceToHost, h->stream), "hipMemcpyAsync");
    if (rc) return rc;
  }
  return h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
}

int lbm_get_velocity(lbm_handle* h, float* dst, int on_device) { return get_macro(h, dst, on_device, true); }
int lbm_get_density(lbm_handle* h, float* dst, int on_device) { return get_macro(h, dst, on_device, false); }

int lbm_get_conserved(lbm_handle* h, double out[4]) {
  if (!h || !out) return LBM_EINVAL;
  launch_conserved(h->dev, h->storage, h->d_partial, kReduceParts, h->d_out, h->stream);
  int rc = h->hip(hipMemcpyAsync(out, h->d_out, sizeof(double) * 4, hipMemcpyDeviceToHost, h->stream),
                  "hipMemcpyAsync");
  if (!rc) rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  out[0] += (double)h->nodes;  // sum of the weights: one per node
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(out[k])) return h->fail(LBM_ENONFINITE, "non-finite mass or momentum");
  return LBM_OK;
}

int lbm_set_populations(lbm_handle* h, const double* dev) {
  if (!h || !dev) return LBM_EINVAL;
  if (h->stepped) return h->fail(LBM_ESTATE, "populations can only be set before the first step");
  const int64_t N = h->nodes;
  const int cur = 0;  // step counter is 0 before stepping
  if (h->storage == LBM_FP16_SHIFTED) {
    std::vector<_Float16> buf(kQ * (size_t)h->pstride, (_Float16)0);
    for (int q = 0; q < kQ; ++q)
      for (int64_t n = 0; n < N; ++n)
        buf[q * h->pstride + n] = (_Float16)((float)dev[q * N + n] * h->fp16_scale);
    return h->hip(hipMemcpy(h->pop[cur], buf.data(), buf.size() * 2, hipMemcpyHostToDevice), "hipMemcpy");
  }
  std::vector<float> buf(kQ * (size_t)h->pstride, 0.0f);
  for (int q = 0; q < kQ; ++q)
    for (int64_t n = 0; n < N; ++n) buf[q * h->pstride + n] = (float)dev[q * N + n];
  return h->hip(hipMemcpy(h->pop[cur], buf.data(), buf.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
}

int lbm_get_populations(lbm_handle* h, double* dev) {
  if (!h || !dev) return LBM_EINVAL;
  int rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  const int cur = (int)(h->host_step & 1);
  const int64_t N = h->nodes;
  if (h->storage == LBM_FP16_SHIFTED) {
    std::vector<_Float16> buf(kQ * (size_t)h->pstride);
    rc = h->hip(hipMemcpy(buf.data(), h->pop[cur], buf.size() * 2, hipMemcpyDeviceToHost), "hipMemcpy");
    if (rc) return rc;
    for (int q = 0; q < kQ; ++q)
      for (int64_t n = 0; n < N; ++n) dev[q * N + n] = (double)((float)buf[q * h->pstride + n] / h->fp16_scale);
    return LBM_OK;
  }
  std::vector<float> buf(kQ * (size_t)h->pstride);
  rc = h->hip(hipMemcpy(buf.data(), h->pop[cur], buf.size() * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  if (rc) return rc;
  for (int q = 0; q < kQ; ++q)
    for (int64_t n = 0; n < N; ++n) dev[q * N + n] = (double)buf[q * h->pstride + n];
  return LBM_OK;
}

// ---- checkpoint -------------------------------------------------------------------
namespace {
struct CkptHeader {
  uint32_t magic, version;
  int32_t nx, ny, nz, storage, width, forcing, nm, nbeads;
  double tau;
  int64_t step;
};

int io_blob(lbm_handle* h, FILE* f, void* dptr, size_t bytes, bool save) {
  std::vector<char> buf(bytes);
  if (save) {
    int rc = h->hip(hipMemcpy(buf.data(), dptr, bytes, hipMemcpyDeviceToHost), "hipMemcpy");
    if (rc) return rc;
    if (fwrite(buf.data(), 1, bytes, f) != bytes) return h->fail(LBM_EIO, "short write");
    return LBM_OK;
  }
  if (fread(buf.data(), 1, bytes, f) != bytes) return h->fail(LBM_EIO, "short read");
  return h->hip(hipMemcpy(dptr, buf.data(), bytes, hipMemcpyHostToDevice), "hipMemcpy");
}

int checkpoint(lbm_handle* h, const char* path, bool save) {
  if (!h || !path) return LBM_EINVAL;
  int rc = upload(h);
  if (rc) return rc;
  rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  FILE* f = fopen(path, save ? "wb" : "rb");
  if (!f) return h->fail(LBM_EIO, std::string("cannot open ") + path);
  CkptHeader hd{kMagic, 1, h->grid.nx, h->grid.ny, h->grid.nz, h->storage, h->width, h->forcing,
                h->nm, (int32_t)h->beads.size(), h->tau, h->host_step};
  if (save) {
    if (fwrite(&hd, sizeof hd, 1, f) != 1) rc = h->fail(LBM_EIO, "short write");
  } else {
    CkptHeader in{};
    if (fread(&in, sizeof in, 1, f) != 1) rc = h->fail(LBM_EIO, "short read");
    else if (in.magic != kMagic || in.version != 1 || in.nx != hd.nx || in.ny != hd.ny || in.nz != hd.nz ||
             in.storage != hd.storage || in.width != hd.width || in.forcing != hd.forcing ||
             in.nm != hd.nm || in.nbeads != hd.nbeads || in.tau != hd.tau)
      rc = h->fail(LBM_EINVAL, "checkpoint does not match this handle");
    else
      h->host_step = in.step;
  }
  const size_t pb = (size_t)element_bytes(h) * kQ * h->pstride;
  if (!rc) rc = io_blob(h, f, h->pop[0], pb, save);
  if (!rc) rc = io_blob(h, f, h->pop[1], pb, save);
  if (!rc) rc = io_blob(h, f, h->F, sizeof(float) * 3 * h->pstride, save);
  if (!rc) rc = io_blob(h, f, h->u, sizeof(float) * 3 * h->pstride, save);
  if (!rc) rc = io_blob(h, f, h->stamp, sizeof(int) * h->ntiles, save);
  if (!rc) rc = io_blob(h, f, h->d_step, sizeof(int64_t), save);
  if (!rc && h->nm > 0) {
    rc = io_blob(h, f, h->d_pos, sizeof(double) * 3 * h->nm, save);
    if (!rc) rc = io_blob(h, f, h->d_U, sizeof(float) * 3 * h->nm, save);
    if (!rc) rc = io_blob(h, f, h->d_fm, sizeof(float) * 3 * h->nm, save);
    if (!rc) rc = io_blob(h, f, h->d_bstate, sizeof(BeadState) * h->beads.size(), save);
  }
  fclose(f);
  if (!rc && !save) {
    h->stepped = true;
    h->need_prologue = true;
  }
  return rc;
}
}  // namespace

int lbm_save(lbm_handle* h, const char* path) { return checkpoint(h, path, true); }
int lbm_load(lbm_handle* h, const char* path) { return checkpoint(h, path, false); }

// ---- measurement -------------------------------------------------------------------
int lbm_set_kernel_timing(lbm_handle* h, int on) {
  if (!h) return LBM_EINVAL;
  harvest_timing(h);
  h->timing = on != 0;
  h->timed_ms = 0;
  h->timed_launches = 0;
  return LBM_OK;
}

int lbm_kernel_time(lbm_handle* h, double* ms, int64_t* launches) {
  if (!h) return LBM_EINVAL;
  harvest_timing(h);
  if (ms) *ms = h->timed_ms;
  if (launches) *launches = h->timed_launches;
  return LBM_OK;
}

int lbm_probe_copy_bandwidth(int64_t bytes, int iters, double* gbs) {
  if (bytes < 16 * 1024 || iters < 1 || !gbs) return LBM_EINVAL;
  bytes = bytes / 16 * 16;
  void *a = nullptr, *b = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = LBM_OK;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess) rc = LBM_ENOMEM;
  if (!rc && (hipStreamCreate(&s) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
              hipEventCreate(&e1) != hipSuccess))
    rc = LBM_EDEVICE;
  if (!rc && hipMemsetAsync(a, 0, bytes, s) != hipSuccess) rc = LBM_EDEVICE;
  if (!rc) {
    launch_copy(a, b, bytes, s);  // warm up
    (void)hipEventRecord(e0, s);
    for (int i = 0; i < iters; ++i) launch_copy(i & 1 ? b : a, i & 1 ? a : b, bytes, s);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) rc = LBM_EDEVICE;
  }
  if (!rc) {
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    *gbs = 2.0 * (double)bytes * iters / (ms * 1e-3) / 1e9;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (s) (void)hipStreamDestroy(s);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  return rc;
}

int lbm_set_stream_collide_launch(lbm_handle* h, int block, int xcd_remap, int resident) {
  if (!h || (block != 128 && block != 256 && block != 512) || resident < -1 || resident > 64) return LBM_EINVAL;
  if (h->boxes.size() != 1) return h->fail(LBM_ESTATE, "launch shape of a batch is set by its tuner");
  int rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  h->sc_block = block;
  h->sc_remap = xcd_remap ? 1 : 0;
  h->sc_resident = resident;
  h->sc_blocks = (int)((h->nodes + block - 1) / block);
  set_near_bounds(h);
  h->need_prologue = true;
  if (h->g_chunk) (void)hipGraphExecDestroy(h->g_chunk);
  if (h->g_one) (void)hipGraphExecDestroy(h->g_one);
  h->g_chunk = h->g_one = nullptr;
  return LBM_OK;
}

int64_t lbm_bytes_per_step(const lbm_handle* h) {
  return h ? (int64_t)2 * kQ * element_bytes(h) * h->nodes : -1;
}

}  // extern "C"
