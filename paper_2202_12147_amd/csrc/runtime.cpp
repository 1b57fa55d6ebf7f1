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
#include "handle.h"

using namespace lbmib;

namespace {

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

const char* kErrNames[] = {"ok", "invalid argument", "out of memory", "HIP runtime error",
                           "call not allowed in this state", "non-finite conserved sums",
                           "file I/O error", "bead outgrew its reserved tile region"};

}  // namespace

namespace {

int element_bytes(const lbm_handle* h) { return h->storage == LBM_FP16_SHIFTED ? 2 : 4; }

// D3Q19 weight of population q in FP32 (the rounding the device uses).
float lattice_weight(int q) { return q == 0 ? 1.0f / 3.0f : (q < 7 ? 1.0f / 18.0f : 1.0f / 36.0f); }

// Candidate tiles reserved per axis for a bead: the node span of its stencils
// with 25% room for deformation, in tiles, for any alignment.
int reserved_tiles(double radius, int width, int n, int T) {
  const int span = (int)std::floor(2.0 * radius * 1.25) + width + 2;
  // an edge that is not a whole number of tiles ends in a short tile, which a
  // run of nodes across it may touch on top of the whole tiles
  const int shorter = n % kTile ? 1 : 0;
  return std::min(T, (span + kTile - 2) / kTile + 1 + shorter);
}

// Host layout of population deviations: box after box, each [19][n_box];
// device index pop_index(q, node0_b + n) (256-node population blocks).
// With the in-place storage the current state's f*_q(x) sits in slot q of
// node x + c_q after an even number of steps (and initially), in slot
// opposite(q) of node x after an odd number.
template <class F>
void for_each_population(const lbm_handle* h, F f) {
  const bool inplace = h->storage == LBM_FP32_INPLACE, odd = (h->host_step & 1) != 0;
  for (const Box& B : h->boxes) {
    const int64_t hoff = kQ * B.node0;
    for (int q = 0; q < kQ; ++q)
      for (int64_t n = 0; n < B.n; ++n) {
        int64_t di = pop_index(q, B.node0 + n);
        if (inplace && odd) {
          di = pop_index(opposite(q), B.node0 + n);
        } else if (inplace) {
          const int64_t x = n % B.nx, y = (n / B.nx) % B.ny, z = n / ((int64_t)B.nx * B.ny);
          const int64_t xs = (x + kLatticeC[q][0] + B.nx) % B.nx, ys = (y + kLatticeC[q][1] + B.ny) % B.ny,
                        zs = (z + kLatticeC[q][2] + B.nz) % B.nz;
          di = pop_index(q, B.node0 + xs + B.nx * (ys + B.ny * zs));
        }
        f(hoff + q * B.n + n, di, q);
      }
  }
}

// Geometry signature of a handle (FNV-1a over box shapes, relaxation times,
// forcing, storage, kernel width and markers): keys checkpoints and the tuner
// cache.
uint64_t signature(const lbm_handle* h) {
  uint64_t x = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) x = (x ^ c[i]) * 1099511628211ull;
  };
  for (const Box& B : h->boxes) {
    const int dims[4] = {B.nx, B.ny, B.nz, B.forcing};
    mix(dims, sizeof dims);
    mix(&B.tau, sizeof B.tau);
  }
  const int rest[3] = {h->storage, h->width, h->nm};
  mix(rest, sizeof rest);
  return x;
}

// Stream-collide block tables for the current block size: first block of each
// box and block -> box (device copies used only when there are several boxes).
int build_sc_tables(lbm_handle* h) {
  std::vector<int> first(h->boxes.size()), owner;
  int blocks = 0;
  for (size_t b = 0; b < h->boxes.size(); ++b) {
    first[b] = blocks;
    const int nb = (int)((h->boxes[b].n + h->sc_block - 1) / h->sc_block);
    owner.insert(owner.end(), nb, (int)b);
    blocks += nb;
  }
  h->sc_blocks = blocks;
  if (h->boxes.size() > 1) {
    if ((int64_t)owner.size() > h->sc_table_cap) return h->fail(LBM_EINVAL, "block table too small");
    int rc = h->hip(hipMemcpy(h->d_sc_block_box, owner.data(), sizeof(int) * owner.size(), hipMemcpyHostToDevice),
                    "hipMemcpy");
    if (!rc) rc = h->hip(hipMemcpy(h->d_sc_box_block0, first.data(), sizeof(int) * first.size(),
                                   hipMemcpyHostToDevice), "hipMemcpy");
    if (rc) return rc;
  }
  h->dev.sc_block_box = h->d_sc_block_box;
  h->dev.sc_box_block0 = h->d_sc_box_block0;
  return LBM_OK;
}

// Stream-collide block geometry and the bound on near blocks: per bead the
// marked node box is its reserved tile span plus two nodes each side.
void set_near_bounds(lbm_handle* h) {
  Dev& d = h->dev;
  d.nsc = h->sc_blocks;
  d.sc_bs = h->sc_block;
  int64_t mx = 0;
  for (const Bead& b : h->beads) {
    const Box& B = h->boxes[b.box];
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
  for (Box& B : h->boxes) {
    B.bead0 = 0;
    B.nbeads = 0;
  }
  for (size_t b = 0; b < h->beads.size(); ++b) {
    Box& B = h->boxes[h->beads[b].box];
    if (B.nbeads == 0) B.bead0 = (int)b;
    B.nbeads += 1;
  }
  // spread candidate blocks, spread_parts(beads) per reserved tile of each
  // bead (each kTile / parts z layers): {bead, box, first bead of the box,
  // beads of the box}, {tile offsets kx, ky, kz, part}
  const int parts = spread_parts((int)h->beads.size());
  std::vector<int> spread_info;
  for (size_t b = 0; b < h->beads.size(); ++b) {
    Bead& Bd = h->beads[b];
    const Box& B = h->boxes[Bd.box];
    Bd.tile_block0 = (int)(spread_info.size() / 8);
    for (int kz = 0; kz < Bd.tiles_z; ++kz)
      for (int ky = 0; ky < Bd.tiles_y; ++ky)
        for (int kx = 0; kx < Bd.tiles_x; ++kx)
          for (int part = 0; part < parts; ++part) {
            const int e[8] = {(int)b, Bd.box, B.bead0, B.nbeads, kx, ky, kz, part};
            spread_info.insert(spread_info.end(), e, e + 8);
          }
  }
  h->spread_blocks = (int)(spread_info.size() / 8);

  auto put = [&](void* dst, const void* src, size_t bytes) {
    if (rc != LBM_OK || bytes == 0) return;
    rc = h->hip(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice), "hipMemcpy");
  };
  h->d_pos = h->alloc<double>(3 * (size_t)nm, rc);
  h->d_U = h->alloc<float>(3 * (size_t)nm, rc);
  h->d_fm = h->alloc<float>(3 * (size_t)nm, rc);
  h->d_fmem = h->alloc<float>(3 * (size_t)nm, rc);
  h->d_gvol = h->alloc<float>(3 * (size_t)nm, rc);
  h->d_bterms = h->alloc<BeadTerms>(h->beads.size(), rc);
  h->d_beads = h->alloc<Bead>(h->beads.size(), rc);
  h->d_bstate = h->alloc<BeadState>(h->beads.size(), rc);
  h->d_swimmers = h->alloc<Swimmer>(h->swimmers.size(), rc);
  h->d_marker_bead = h->alloc<int>(nm, rc);
  h->d_marker_info = h->alloc<int4>(nm, rc);
  h->d_tri = h->alloc<int>(tri.size(), rc);
  h->d_G0 = h->alloc<double>(G0.size(), rc);
  h->d_G0inv = h->alloc<float>(Gi.size(), rc);
  h->d_A0 = h->alloc<float>(A0.size(), rc);
  h->d_idet = h->alloc<float>(idet.size(), rc);
  h->d_hinge = h->alloc<int>(hinge.size(), rc);
  h->d_theta0 = h->alloc<double>(2 * h->hingeth0.size(), rc);
  h->d_lane_elem = h->alloc<int>(lane_elem.size(), rc);
  h->d_lane_v = h->alloc<int>(lane_v.size(), rc);
  h->d_spread_info = h->alloc<int>(spread_info.size(), rc);
  h->d_centres = h->alloc<double>(3 * h->beads.size(), rc);
  // near-block buffers, sized for the smallest stream-collide block (128):
  // every box starts a new block, so the bound is the sum over the boxes of
  // ceil(n / 128), not ceil(nodes / 128)
  const int64_t nsc_max = h->sc_table_cap;
  h->d_near = h->alloc<int>(kNearSlots * (size_t)nsc_max, rc);
  h->d_near_list = h->alloc<int>(2 * (size_t)nsc_max, rc);
  h->d_near_count = h->alloc<int>(2, rc);
  h->d_work = h->alloc<int>(kWorkCounters, rc);
  if (rc != LBM_OK) return h->fail(rc, "device allocation for markers failed");
  put(h->d_boxes, h->boxes.data(), sizeof(Box) * h->boxes.size());
  put(h->d_pos, pos.data(), sizeof(double) * pos.size());
  if (rc == LBM_OK && nm > 0) {
    rc = h->hip(hipMemset(h->d_U, 0, sizeof(float) * 3 * nm), "hipMemset");
    if (rc == LBM_OK) rc = h->hip(hipMemset(h->d_fm, 0, sizeof(float) * 3 * nm), "hipMemset");
    if (rc == LBM_OK) rc = h->hip(hipMemset(h->d_fmem, 0, sizeof(float) * 3 * nm), "hipMemset");
    if (rc == LBM_OK) rc = h->hip(hipMemset(h->d_gvol, 0, sizeof(float) * 3 * nm), "hipMemset");
    if (rc == LBM_OK) rc = h->hip(hipMemset(h->d_bterms, 0, sizeof(BeadTerms) * h->beads.size()), "hipMemset");
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
  put(h->d_marker_info, h->marker_info.data(), sizeof(int4) * nm);
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
  put(h->d_spread_info, spread_info.data(), sizeof(int) * spread_info.size());
  if (rc != LBM_OK) return rc;

  Dev& d = h->dev;
  d.pos = h->d_pos;
  d.U = h->d_U;
  d.fm = h->d_fm;
  d.fmem = h->d_fmem;
  d.gvol = h->d_gvol;
  d.spread_raw = 0;
  d.bterms = h->d_bterms;
  d.nm = nm;
  d.beads = h->d_beads;
  d.nbeads = (int)h->beads.size();
  d.bstate = h->d_bstate;
  d.swimmers = h->d_swimmers;
  d.nswimmers = (int)h->swimmers.size();
  d.marker_bead = h->d_marker_bead;
  d.marker_info = h->d_marker_info;
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
  d.spread_info = reinterpret_cast<const int4*>(h->d_spread_info);
  d.near = h->d_near;
  d.near_list = h->d_near_list;
  d.near_count = h->d_near_count;
  d.work = h->d_work;
  d.tile_box = nullptr;
  set_near_bounds(h);
  if (!h->swimmers.empty()) {
    rc = h->hip(hipStreamCreate(&h->side), "hipStreamCreate");
    if (rc) return rc;
    h->step_events.resize(2 * kGraphChunk + 2);  // per step bulk and near, the fork, the tail
    for (auto& e : h->step_events) {
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
// stream-collide launch.  With swimmers the side stream runs the IBM chain of
// each step -- advection of the previous step, bead statistics, nodal forces,
// spreading -- and then the near-block launch, while the main stream streams
// and collides every node away from the swimmers.  The last step's advection
// closes the sequence on the main stream after a join, so the markers are
// current whenever the sequence ends; one kernel advances the step counter.
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
      launch_stats_forces(d, 0, h->stream);
      launch_spread(d, h->stream);
      launch_marker_force_total(d, d.fm, h->stream);
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
  // The near-block launch of step n needs the spreading of step n and the
  // populations of step n - 1 (bulk and near blocks), not the bulk launch of
  // step n; the bulk launch of step n needs the near blocks of step n - 1.
  // Each stream waits on the other with a lag of one step, so in the steady
  // state the bulk launches run back to back.
  hipEvent_t fork = h->step_events[2 * kGraphChunk];
  (void)hipEventRecord(fork, h->stream);
  (void)hipStreamWaitEvent(h->side, fork, 0);
  hipEvent_t prev_bulk = nullptr, prev_near = nullptr;
  for (int64_t i = 0; i < count; ++i) {
    hipEvent_t ev_bulk = h->step_events[2 * (i % kGraphChunk)], ev_near = h->step_events[2 * (i % kGraphChunk) + 1];
    d.sub = (int)i;
    if (i > 0) launch_interp_advance(d, h->side);
    launch_stats_forces(d, kNoMark, h->side);  // the near-block launch marks the next step's blocks
    launch_spread(d, h->side);                 // and forms the markers' total forces
    if (prev_near) (void)hipStreamWaitEvent(h->stream, prev_near, 0);
    hipEvent_t e0, e1;
    timing_pair(h, &e0, &e1);
    launch_stream_collide(d, h->storage, kLaunchBulk, h->sc_block, h->sc_blocks, h->sc_remap, h->sc_resident,
                          h->ncu, h->stream, e0, e1);
    (void)hipEventRecord(ev_bulk, h->stream);
    if (prev_bulk) (void)hipStreamWaitEvent(h->side, prev_bulk, 0);
    timing_pair(h, &e0, &e1);
    Dev dn = d;
    dn.near_mark = 1;
    launch_stream_collide(dn, h->storage, kLaunchActive, h->sc_block, h->sc_blocks, 0, 0, h->ncu, h->side, e0, e1);
    (void)hipEventRecord(ev_near, h->side);
    prev_bulk = ev_bulk;
    prev_near = ev_near;
  }
  // the last advection follows the last near-block launch on the side
  // stream, where it overlaps the tail of the last bulk launch, and the main
  // stream joins after it (20-step call 58.7 against 60.0 us per step, long
  // runs 56.5 against 57.0 with it on the main stream after the join)
  d.sub = (int)count;
  hipEvent_t tail = h->step_events[2 * kGraphChunk + 1];
  launch_interp_advance(d, h->side);
  (void)hipEventRecord(tail, h->side);
  (void)hipStreamWaitEvent(h->stream, tail, 0);
  launch_tick(d, (int)count, h->stream);
}

// Before stepping resumes: bead regions of the current markers and the near
// tiles under the previous step's parity, so the first step can split the
// grid into bulk and active parts, and zeroed block counters for the
// persistent bulk launch.  Eager, never captured.
int prologue(lbm_handle* h) {
  if (!h->need_prologue || h->swimmers.empty()) return LBM_OK;
  int rc = h->hip(hipMemsetAsync(h->d_near, 0x80, sizeof(int) * kNearSlots * h->dev.nsc, h->stream), "hipMemsetAsync");
  if (!rc) rc = h->hip(hipMemsetAsync(h->d_near_count, 0, sizeof(int) * 2, h->stream), "hipMemsetAsync");
  if (!rc) rc = h->hip(hipMemsetAsync(h->d_work, 0, sizeof(int) * kWorkCounters, h->stream), "hipMemsetAsync");
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

// Drop the captured step graphs (kernel arguments or launch shapes changed);
// the next graph-replayed call captures them again.
void drop_graphs(lbm_handle* h) {
  for (auto& g : h->g_steps) {
    if (g) (void)hipGraphExecDestroy(g);
    g = nullptr;
  }
}

// Point the stream-collide launches at the time-average state.  Captured
// graphs hold the previous kernel arguments, so they are dropped and
// recaptured on the next step.
int set_average(lbm_handle* h, double* sums, int64_t t0, int every) {
  int rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  h->dev.uavg = sums;
  h->dev.avg_t0 = t0;
  h->dev.avg_every = every;
  drop_graphs(h);
  return LBM_OK;
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

}  // extern "C"

namespace {

// Box descriptors as lbm_batch_create accepts them; *nodes receives the
// total node count.
int check_boxes(const lbm_box_desc* boxes, int nboxes, int64_t* nodes) {
  if (!boxes || nboxes < 1) return LBM_EINVAL;
  int64_t total = 0;
  for (int b = 0; b < nboxes; ++b) {
    const lbm_box_desc& d = boxes[b];
    if (!(d.tau > 0.5) || !std::isfinite(d.tau)) return LBM_EINVAL;
    if (d.grid.nx < 16 || d.grid.ny < 16 || d.grid.nz < 16) return LBM_EINVAL;
    // node offsets within a box are 32-bit in the kernels (a lane index plus a
    // neighbour offset of up to n nodes), so a box stays 2^16 below 2^31
    if ((int64_t)d.grid.nx * d.grid.ny * d.grid.nz > ((int64_t)1 << 31) - ((int64_t)1 << 16)) return LBM_EINVAL;
    if (d.forcing != LBM_GUO && d.forcing != LBM_SHAN_CHEN) return LBM_EINVAL;
    total += (int64_t)d.grid.nx * d.grid.ny * d.grid.nz;
  }
  if (total >= (int64_t)1 << 31) return LBM_EINVAL;
  *nodes = total;
  return LBM_OK;
}

bool valid_storage(int storage) {
  return storage == LBM_FP32_SHIFTED || storage == LBM_FP16_SHIFTED || storage == LBM_FP32_PLAIN ||
         storage == LBM_FP32_INPLACE;
}

// Population sets a storage keeps: one updated in place, else two.
int population_sets(int storage) { return storage == LBM_FP32_INPLACE ? 1 : 2; }

// The node fields in one allocation: the population sets (0 and 1, or the
// one in-place set), then the body-force density and the velocity
// ([3][pstride] float32 each).  Every part is a multiple of 256 bytes long
// (pstride is a multiple of the 256-node population block), so each starts
// 256-byte aligned.
struct FieldLayout {
  size_t pop, vec, total;  // bytes of one population set, of F (or u), of all
  int sets;
};

FieldLayout field_layout(int64_t nodes, int storage) {
  const int64_t pstride = (nodes + kPopBlock - 1) / kPopBlock * kPopBlock;
  FieldLayout L;
  L.sets = population_sets(storage);
  L.pop = (size_t)(storage == LBM_FP16_SHIFTED ? 2 : 4) * kQ * (size_t)pstride;
  L.vec = sizeof(float) * 3 * (size_t)pstride;
  L.total = L.sets * L.pop + 2 * L.vec;
  return L;
}

int create_boxes(const lbm_box_desc* boxes, int nboxes, const lbm_opts* opts, lbm_handle** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  int64_t total = 0;
  if (int rc = check_boxes(boxes, nboxes, &total)) return rc;
  lbm_opts o{LBM_FP32_SHIFTED, 3, 1.0f, 1, nullptr, nullptr, 0};
  if (opts) o = *opts;
  if (!valid_storage(o.storage)) return LBM_EINVAL;
  // the in-place set is addressed with 32-bit byte offsets
  if (o.storage == LBM_FP32_INPLACE && field_layout(total, o.storage).pop >= ((size_t)1 << 32)) return LBM_EINVAL;
  if (o.field_memory) {
    if (((uintptr_t)o.field_memory & 255) != 0) return LBM_EINVAL;
    if (o.field_bytes < 0 || (uint64_t)o.field_bytes < field_layout(total, o.storage).total) return LBM_EINVAL;
  }
  if (o.delta_width < 2 || o.delta_width > 4) return LBM_EINVAL;
  if (o.fp16_scale == 0.0f) o.fp16_scale = 1.0f;
  {
    int e;
    std::frexp(o.fp16_scale, &e);
    if (!(o.fp16_scale > 0.0f) || std::ldexp(1.0, e - 1) != o.fp16_scale) return LBM_EINVAL;
  }
  auto* h = new lbm_handle();
  h->storage = o.storage;
  h->width = o.delta_width;
  h->fp16_scale = o.fp16_scale;
  h->use_graphs = o.use_graphs != 0;
  int rc = h->hip(hipGetDevice(&h->device), "hipGetDevice");
  if (!rc) rc = h->hip(hipDeviceGetAttribute(&h->ncu, hipDeviceAttributeMultiprocessorCount, h->device),
                      "hipDeviceGetAttribute");
  // device address of the static scratch of the allocation-free conserved
  // sums, looked up once per device while it is current
  if (!rc) rc = h->hip(resolve_conserved_scratch(h->device, &h->conserved_scratch), "hipGetSymbolAddress");
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
  int64_t node0 = 0;
  int tile0 = 0, block0 = 0;
  int64_t sc_cap = 0;
  std::vector<int> block_box;
  for (int b = 0; b < nboxes; ++b) {
    const lbm_box_desc& d = boxes[b];
    Box B{};
    B.nx = d.grid.nx;
    B.ny = d.grid.ny;
    B.nz = d.grid.nz;
    B.tx = (B.nx + kTile - 1) / kTile;
    B.ty = (B.ny + kTile - 1) / kTile;
    B.tz = (B.nz + kTile - 1) / kTile;
    B.node0 = node0;
    B.n = (int64_t)B.nx * B.ny * B.nz;
    B.tile0 = tile0;
    B.block0 = block0;
    B.forcing = d.forcing;
    B.tau = (float)d.tau;
    B.omega = (float)(1.0 / d.tau);
    B.div_nx = make_divisor((uint32_t)B.nx);
    B.div_ny = make_divisor((uint32_t)B.ny);
    const int nb = (int)((B.n + kScBlock - 1) / kScBlock);
    block_box.insert(block_box.end(), nb, b);
    node0 += B.n;
    tile0 += B.tx * B.ty * B.tz;
    block0 += nb;
    sc_cap += (B.n + 127) / 128;
    h->boxes.push_back(B);
  }
  h->nodes = node0;
  h->pstride = (node0 + kPopBlock - 1) / kPopBlock * kPopBlock;
  h->ntiles = tile0;
  h->out_blocks = block0;
  h->sc_table_cap = sc_cap;
  // default stream-collide launch shape, the fastest measured on MI355X:
  // one box, FP32 storage: one persistent 512-node workgroup per CU claiming
  // blocks in round-robin order (128^3 swimmer step 62.3 us, 82 us at the
  // non-persistent shape); FP16 storage: two persistent 256-node workgroups
  // per CU; batches: non-persistent 512-node workgroups in block order
  // (64-box ensemble 707.6 us per step against 731.5 us XCD-remapped)
  if (nboxes > 1) {
    h->sc_block = 512;
    h->sc_remap = 0;
    h->sc_resident = 0;
  } else if (h->storage == LBM_FP16_SHIFTED) {
    h->sc_block = 256;
    h->sc_remap = 0;
    h->sc_resident = 2;
  } else {
    h->sc_block = 512;
    h->sc_remap = 0;
    h->sc_resident = 1;
  }

  const size_t eb = element_bytes(h);
  if (o.field_memory) {
    // the caller's memory, laid out as field_layout says; never freed here
    const FieldLayout L = field_layout(h->nodes, h->storage);
    char* base = static_cast<char*>(o.field_memory);
    h->pop[0] = base;
    h->pop[1] = base + (L.sets - 1) * L.pop;
    h->F = reinterpret_cast<float*>(base + L.sets * L.pop);
    h->u = reinterpret_cast<float*>(base + L.sets * L.pop + L.vec);
  } else {
    h->pop[0] = h->alloc<char>(eb * kQ * h->pstride, rc);
    // the in-place storage names its one set twice
    h->pop[1] = population_sets(h->storage) == 2 ? h->alloc<char>(eb * kQ * h->pstride, rc) : h->pop[0];
    h->F = h->alloc<float>(3 * h->pstride, rc);
    h->u = h->alloc<float>(3 * h->pstride, rc);
  }
  h->stamp = h->alloc<int>(h->ntiles, rc);
  h->d_boxes = h->alloc<Box>(nboxes, rc);
  h->d_step = h->alloc<int64_t>(1, rc);
  h->d_overflow = h->alloc<int>(1, rc);
  h->d_partial = h->alloc<double>(4 * kReduceParts, rc);
  h->d_out = h->alloc<double>(4, rc);
  if (nboxes > 1) {
    h->d_block_box = h->alloc<int>(block_box.size(), rc);
    h->d_sc_block_box = h->alloc<int>(sc_cap, rc);
    h->d_sc_box_block0 = h->alloc<int>(nboxes, rc);
  }
  if (rc) {
    lbm_destroy(h);
    return LBM_ENOMEM;
  }
  if (h->storage == LBM_FP32_PLAIN) {
    // rest state f = w (the shifted forms store g = 0)
    std::vector<float> rest(kQ * (size_t)h->pstride);
    for (int64_t i = 0; i < (int64_t)rest.size(); ++i) rest[i] = lattice_weight((int)((i / kPopBlock) % kQ));
    rc = h->hip(hipMemcpy(h->pop[0], rest.data(), rest.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
    if (!rc) rc = h->hip(hipMemcpy(h->pop[1], rest.data(), rest.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
  } else {
    rc = h->hip(hipMemset(h->pop[0], 0, eb * kQ * h->pstride), "hipMemset");
    if (!rc) rc = h->hip(hipMemset(h->pop[1], 0, eb * kQ * h->pstride), "hipMemset");
  }
  if (!rc) rc = h->hip(hipMemset(h->F, 0, sizeof(float) * 3 * h->pstride), "hipMemset");
  if (!rc) rc = h->hip(hipMemset(h->u, 0, sizeof(float) * 3 * h->pstride), "hipMemset");
  if (!rc) rc = h->hip(hipMemset(h->stamp, 0x80, sizeof(int) * h->ntiles), "hipMemset");
  if (!rc) rc = h->hip(hipMemset(h->d_step, 0, sizeof(int64_t)), "hipMemset");
  if (!rc) rc = h->hip(hipMemset(h->d_overflow, 0, sizeof(int)), "hipMemset");
  if (!rc) rc = h->hip(hipMemcpy(h->d_boxes, h->boxes.data(), sizeof(Box) * nboxes, hipMemcpyHostToDevice),
                       "hipMemcpy");
  if (!rc && nboxes > 1)
    rc = h->hip(hipMemcpy(h->d_block_box, block_box.data(), sizeof(int) * block_box.size(), hipMemcpyHostToDevice),
                "hipMemcpy");
  if (!rc) rc = build_sc_tables(h);
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
  d.nboxes = nboxes;
  d.block_box = h->d_block_box;
  d.step = h->d_step;
  d.sub = 0;
  d.fp16_scale = h->fp16_scale;
  d.small_pops = population_sets(h->storage) * kQ * h->pstride * (int64_t)element_bytes(h) <= kWriteThroughBytes ? 1 : 0;
  d.pops32 = kQ * h->pstride * (int64_t)element_bytes(h) < ((int64_t)1 << 32) ? 1 : 0;
  d.fp16_inv = 1.0f / h->fp16_scale;
  d.width = h->width;
  d.overflow = h->d_overflow;
  *out = h;
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_create(const lbm_grid* grid, double tau, int forcing, const lbm_opts* opts,
               lbm_handle** out) {
  if (!grid) return LBM_EINVAL;
  lbm_box_desc b{*grid, tau, forcing};
  return create_boxes(&b, 1, opts, out);
}

int lbm_batch_create(const lbm_box_desc* boxes, int32_t nboxes, const lbm_opts* opts, lbm_handle** out) {
  return create_boxes(boxes, nboxes, opts, out);
}

int lbm_field_bytes(const lbm_box_desc* boxes, int32_t nboxes, int32_t storage, int64_t* bytes) {
  if (!bytes || !valid_storage(storage)) return LBM_EINVAL;
  int64_t nodes = 0;
  if (int rc = check_boxes(boxes, nboxes, &nodes)) return rc;
  *bytes = (int64_t)field_layout(nodes, storage).total;
  return LBM_OK;
}

int32_t lbm_n_boxes(const lbm_handle* h) { return h ? (int32_t)h->boxes.size() : -1; }

int lbm_destroy(lbm_handle* h) {
  if (!h) return LBM_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  drop_graphs(h);
  for (auto e : h->ev_pool) (void)hipEventDestroy(e);
  for (auto e : h->step_events) (void)hipEventDestroy(e);
  if (h->side) (void)hipStreamDestroy(h->side);
  rt::adjoint_release(h);
  for (void* p : h->allocs) (void)hipFree(p);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return LBM_OK;
}

int lbm_swimmer_add(lbm_handle* h, const lbm_bead_desc beads[3], const lbm_spring_desc springs[2],
                    const lbm_actuation_desc* act, int32_t* id) {
  return lbm_batch_swimmer_add(h, 0, beads, springs, act, id);
}

int lbm_batch_swimmer_add(lbm_handle* h, int32_t box, const lbm_bead_desc beads[3],
                          const lbm_spring_desc springs[2], const lbm_actuation_desc* act, int32_t* id) {
  if (!h || !beads || !springs || !act) return LBM_EINVAL;
  if (box < 0 || box >= (int)h->boxes.size()) return h->fail(LBM_EINVAL, "box index out of range");
  if (!h->beads.empty() && h->beads.back().box > box)
    return h->fail(LBM_EINVAL, "swimmers must be added in non-decreasing box order");
  if (h->stepped || h->uploaded) return h->fail(LBM_ESTATE, "swimmers must be added before the first step");
  if (!(act->period > 0)) return h->fail(LBM_EINVAL, "actuation period must be positive");
  const Box& BX = h->boxes[box];
  const int minedge = std::min(BX.nx, std::min(BX.ny, BX.nz));
  for (int k = 0; k < 3; ++k) {
    if (!(beads[k].radius > 0) || beads[k].level < 0 || beads[k].level > 5)
      return h->fail(LBM_EINVAL, "bead radius must be positive and level in 0..5");
    if (2.0 * beads[k].radius * 1.25 + h->width + 2 > minedge / 1.5)
      return h->fail(LBM_EINVAL, "bead too large for the box");
  }
  Swimmer S{};
  const int sw = (int)h->swimmers.size();
  const Box& B = h->boxes[box];
  for (int k = 0; k < 3; ++k) {
    const lbm_bead_desc& bd = beads[k];
    const Mesh M = icosphere(bd.level);
    const int nv = (int)M.v.size() / 3, nt = (int)M.t.size() / 3;
    Bead b{};
    b.first = h->nm;
    b.nv = nv;
    b.tri0 = (int)h->tri.size() / 3;
    b.ntri = nt;
    b.box = box;
    b.swimmer = sw;
    b.slot = k;
    b.tiles_x = reserved_tiles(bd.radius, h->width, B.nx, B.tx);
    b.tiles_y = reserved_tiles(bd.radius, h->width, B.ny, B.ty);
    b.tiles_z = reserved_tiles(bd.radius, h->width, B.nz, B.tz);
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
    for (int j = 0; j < nv; ++j) {
      const int info[4] = {(int)h->beads.size(), b.box, (int)h->swimmers.size() * 4 + k,
                           (int)h->beads.size() - k};
      h->marker_info.insert(h->marker_info.end(), info, info + 4);
    }
    // bead_terms (device) relies on swimmer s owning beads 3s .. 3s + 2
    if ((int)h->beads.size() != 3 * (int)h->swimmers.size() + k) return h->fail(LBM_ESTATE, "bead numbering");
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
  // every graph a call can replay is captured on the first call that steps,
  // so no later call (of any step count) pays for a capture
  for (int c = 1; c <= kGraphChunk && n > 0; ++c)
    if (!h->g_steps[c] && (rc = capture(h, c, &h->g_steps[c]))) return rc;
  // the remainder's graph first, then the full chunks (the smaller graph
  // reaches the GPU sooner; the 128^3 workload: 60.05 against 60.33 us per
  // step over 2000 steps with the remainder last)
  const int64_t rest = n % kGraphChunk;
  if (rest)
    if ((rc = h->hip(hipGraphLaunch(h->g_steps[rest], h->stream), "hipGraphLaunch"))) return rc;
  for (int64_t c = 0; c < n / kGraphChunk; ++c)
    if ((rc = h->hip(hipGraphLaunch(h->g_steps[kGraphChunk], h->stream), "hipGraphLaunch"))) return rc;
  h->host_step += n;
  return LBM_OK;
}

int lbm_batch_step(lbm_handle* h, int64_t n) { return lbm_step(h, n); }

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
  if (!h) return LBM_EINVAL;
  if (h->beads.empty()) return LBM_OK;  // nothing to write (out may be null)
  if (!out) return LBM_EINVAL;
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
  if (!h) return LBM_EINVAL;
  if (h->swimmers.empty()) return LBM_OK;  // nothing to write (out may be null)
  if (!out) return LBM_EINVAL;
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
  if (!h) return LBM_EINVAL;
  if (h->nm == 0) return LBM_OK;  // nothing to write (out may be null)
  if (!out) return LBM_EINVAL;
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
  if (!h) return LBM_EINVAL;
  if (h->nm == 0) return LBM_OK;  // nothing to write (out may be null)
  if (!out) return LBM_EINVAL;
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

static int get_macro(lbm_handle* h, int box, float* dst, int on_device, bool vel) {
  if (!h || !dst) return LBM_EINVAL;
  if (box < 0 || box >= (int)h->boxes.size()) return h->fail(LBM_EINVAL, "box index out of range");
  const Box& B = h->boxes[box];
  const size_t comps = vel ? 3 : 1;
  const size_t bytes = sizeof(float) * comps * B.n;
  int rc = LBM_OK;
  float* target = dst;
  const bool direct = on_device && h->boxes.size() == 1;
  if (!direct) {
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
  if (!direct) {
    const float* src = target + comps * B.node0;
    rc = h->hip(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                               h->stream), "hipMemcpyAsync");
    if (rc) return rc;
  }
  return h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
}

int lbm_get_velocity(lbm_handle* h, float* dst, int on_device) { return get_macro(h, 0, dst, on_device, true); }
int lbm_get_density(lbm_handle* h, float* dst, int on_device) { return get_macro(h, 0, dst, on_device, false); }
int lbm_batch_get_velocity(lbm_handle* h, int32_t box, float* dst, int on_device) {
  return get_macro(h, box, dst, on_device, true);
}

int lbm_get_conserved(lbm_handle* h, double out[4]) { return lbm_batch_get_conserved(h, -1, out); }

int lbm_batch_get_conserved(lbm_handle* h, int32_t box, double out[4]) {
  if (!h || !out) return LBM_EINVAL;
  if (box < -1 || box >= (int)h->boxes.size()) return h->fail(LBM_EINVAL, "box index out of range");
  launch_conserved(h->dev, h->storage, box, h->d_partial, kReduceParts, h->d_out, h->stream, 0.0);
  int rc = h->hip(hipMemcpyAsync(out, h->d_out, sizeof(double) * 4, hipMemcpyDeviceToHost, h->stream),
                  "hipMemcpyAsync");
  if (!rc) rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  out[0] += (double)(box < 0 ? h->nodes : h->boxes[box].n);  // sum of the weights: one per node
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(out[k])) return h->fail(LBM_ENONFINITE, "non-finite mass or momentum");
  return LBM_OK;
}

int lbm_batch_get_conserved_noalloc(lbm_handle* h, int32_t box, int32_t parts, double* dst) {
  if (!h || !dst) return LBM_EINVAL;
  if (box < -1 || box >= (int)h->boxes.size()) return h->fail(LBM_EINVAL, "box index out of range");
  if (parts < 1 || parts > kNoAllocParts)
    return h->fail(LBM_EINVAL, "parts must lie in 1..4096, the partial sums the static scratch holds");
  if (!h->conserved_scratch) return h->fail(LBM_ESTATE, "static scratch address not resolved");
  const double mass0 = (double)(box < 0 ? h->nodes : h->boxes[box].n);  // sum of the weights: one per node
  launch_conserved(h->dev, h->storage, box, h->conserved_scratch, parts, dst, h->stream, mass0);
  return h->hip(hipGetLastError(), "conserved-sum launch");
}

int lbm_set_populations(lbm_handle* h, const double* dev) {
  if (!h || !dev) return LBM_EINVAL;
  if (h->stepped) return h->fail(LBM_ESTATE, "populations can only be set before the first step");
  const int cur = 0;  // step counter is 0 before stepping
  if (h->storage == LBM_FP16_SHIFTED) {
    std::vector<_Float16> buf(kQ * (size_t)h->pstride, (_Float16)0);
    for_each_population(h, [&](int64_t hi, int64_t di, int) {
      buf[di] = (_Float16)((float)dev[hi] * h->fp16_scale);
    });
    return h->hip(hipMemcpy(h->pop[cur], buf.data(), buf.size() * 2, hipMemcpyHostToDevice), "hipMemcpy");
  }
  std::vector<float> buf(kQ * (size_t)h->pstride, 0.0f);
  if (h->storage == LBM_FP32_PLAIN)
    for (int64_t i = 0; i < (int64_t)buf.size(); ++i) buf[i] = lattice_weight((int)((i / kPopBlock) % kQ));
  if (h->storage == LBM_FP32_PLAIN)
    for_each_population(h, [&](int64_t hi, int64_t di, int q) { buf[di] = (float)(lattice_weight(q) + dev[hi]); });
  else
    for_each_population(h, [&](int64_t hi, int64_t di, int) { buf[di] = (float)dev[hi]; });
  return h->hip(hipMemcpy(h->pop[cur], buf.data(), buf.size() * 4, hipMemcpyHostToDevice), "hipMemcpy");
}

int lbm_get_populations(lbm_handle* h, double* dev) {
  if (!h || !dev) return LBM_EINVAL;
  int rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  const int cur = (int)(h->host_step & 1);
  if (h->storage == LBM_FP16_SHIFTED) {
    std::vector<_Float16> buf(kQ * (size_t)h->pstride);
    rc = h->hip(hipMemcpy(buf.data(), h->pop[cur], buf.size() * 2, hipMemcpyDeviceToHost), "hipMemcpy");
    if (rc) return rc;
    for_each_population(h, [&](int64_t hi, int64_t di, int) {
      dev[hi] = (double)((float)buf[di] / h->fp16_scale);
    });
    return LBM_OK;
  }
  std::vector<float> buf(kQ * (size_t)h->pstride);
  rc = h->hip(hipMemcpy(buf.data(), h->pop[cur], buf.size() * 4, hipMemcpyDeviceToHost), "hipMemcpy");
  if (rc) return rc;
  if (h->storage == LBM_FP32_PLAIN)
    for_each_population(h, [&](int64_t hi, int64_t di, int q) {
      dev[hi] = (double)buf[di] - (double)lattice_weight(q);
    });
  else
    for_each_population(h, [&](int64_t hi, int64_t di, int) { dev[hi] = (double)buf[di]; });
  return LBM_OK;
}

// ---- checkpoint -------------------------------------------------------------------
namespace {
struct CkptHeader {
  uint32_t magic, version;
  int32_t nboxes, storage, width, nm, nbeads, pad;
  uint64_t signature;
  int64_t nodes, step;
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
  CkptHeader hd{kMagic, 4, (int32_t)h->boxes.size(), h->storage, h->width, h->nm, (int32_t)h->beads.size(),
                0, signature(h), h->nodes, h->host_step};
  if (save) {
    if (fwrite(&hd, sizeof hd, 1, f) != 1) rc = h->fail(LBM_EIO, "short write");
  } else {
    CkptHeader in{};
    if (fread(&in, sizeof in, 1, f) != 1) rc = h->fail(LBM_EIO, "short read");
    else if (in.magic != kMagic || in.version != hd.version || in.nboxes != hd.nboxes ||
             in.storage != hd.storage || in.width != hd.width || in.nm != hd.nm || in.nbeads != hd.nbeads ||
             in.signature != hd.signature || in.nodes != hd.nodes)
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
int lbm_load(lbm_handle* h, const char* path) {
  int rc = checkpoint(h, path, false);
  if (!rc && h->dev.uavg) rc = set_average(h, nullptr, 0, 0);  // the step count jumped
  return rc;
}

// ---- time-averaged velocity ------------------------------------------------------------
int lbm_average_begin(lbm_handle* h, int32_t every) {
  if (!h || every < 0) return LBM_EINVAL;
  if (every == 0) return set_average(h, nullptr, 0, 0);
  int rc = LBM_OK;
  const size_t bytes = sizeof(double) * 3 * (size_t)h->pstride;
  if (!h->avg_sums) {
    h->avg_sums = h->alloc<double>(3 * (size_t)h->pstride, rc);
    if (rc) return h->fail(rc, "velocity average allocation failed");
  }
  rc = h->hip(hipMemsetAsync(h->avg_sums, 0, bytes, h->stream), "hipMemsetAsync");
  if (rc) return rc;
  return set_average(h, h->avg_sums, h->host_step, every);
}

int lbm_get_average_velocity(lbm_handle* h, int32_t box, float* dst, int on_device, int64_t* samples) {
  if (!h || !dst) return LBM_EINVAL;
  if (box < 0 || box >= (int)h->boxes.size()) return h->fail(LBM_EINVAL, "box index out of range");
  if (!h->dev.uavg) return h->fail(LBM_ESTATE, "no velocity average is running (lbm_average_begin)");
  const Box& B = h->boxes[box];
  const int64_t span = h->host_step - h->dev.avg_t0;
  const int64_t count = span > 0 ? (span + h->dev.avg_every - 1) / h->dev.avg_every : 0;
  int rc = LBM_OK;
  float* target = dst;
  const bool direct = on_device && h->boxes.size() == 1;
  if (!direct) {
    if (!h->uout) {
      h->uout = h->alloc<float>(3 * h->nodes, rc);
      if (rc) return h->fail(rc, "velocity staging allocation failed");
    }
    target = h->uout;
  }
  launch_average_out(h->dev, h->out_blocks, count, target, h->stream);
  rc = h->hip(hipGetLastError(), "k_average_out launch");
  if (rc) return rc;
  if (!direct) {
    rc = h->hip(hipMemcpyAsync(dst, target + 3 * B.node0, sizeof(float) * 3 * B.n,
                               on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, h->stream),
                "hipMemcpyAsync");
    if (rc) return rc;
  }
  rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  if (samples) *samples = count;
  return LBM_OK;
}

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
  int rc = h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
  if (rc) return rc;
  h->sc_block = block;
  h->sc_remap = xcd_remap ? 1 : 0;
  h->sc_resident = resident;
  rc = build_sc_tables(h);
  if (rc) return rc;
  set_near_bounds(h);
  h->need_prologue = true;
  drop_graphs(h);
  return LBM_OK;
}

}  // extern "C"

namespace lbmib {
namespace rt {

// Device copy of every buffer that stepping changes (tuner, adjoint rewind).

void snapshot_parts(lbm_handle* h, Snapshot& S) {
  const size_t pb = (size_t)element_bytes(h) * kQ * h->pstride;
  S.parts = {{h->pop[0], pb}, {h->pop[1], pb}, {h->F, sizeof(float) * 3 * h->pstride},
             {h->u, sizeof(float) * 3 * h->pstride}, {h->stamp, sizeof(int) * h->ntiles},
             {h->d_step, sizeof(int64_t)}, {h->d_overflow, sizeof(int)}};
  if (h->uploaded && h->nm > 0) {
    const size_t nsc_max = (size_t)h->sc_table_cap;
    S.parts.push_back({h->d_pos, sizeof(double) * 3 * h->nm});
    S.parts.push_back({h->d_U, sizeof(float) * 3 * h->nm});
    S.parts.push_back({h->d_fm, sizeof(float) * 3 * h->nm});
    S.parts.push_back({h->d_bstate, sizeof(BeadState) * h->beads.size()});
    S.parts.push_back({h->d_near, sizeof(int) * kNearSlots * nsc_max});
    S.parts.push_back({h->d_near_list, sizeof(int) * 2 * nsc_max});
    S.parts.push_back({h->d_near_count, sizeof(int) * 2});
  }
}

int snapshot_copy(lbm_handle* h, Snapshot& S, bool take) {
  size_t off = 0;
  for (auto& p : S.parts) {
    void* dst = take ? (void*)(S.mem + off) : p.first;
    const void* src = take ? p.first : (const void*)(S.mem + off);
    int rc = h->hip(hipMemcpyAsync(dst, src, p.second, hipMemcpyDeviceToDevice, h->stream), "hipMemcpyAsync");
    if (rc) return rc;
    off += (p.second + 255) / 256 * 256;
  }
  if (take)
    S.host_step = h->host_step;
  else
    h->host_step = S.host_step;
  h->need_prologue = true;
  return h->hip(hipStreamSynchronize(h->stream), "hipStreamSynchronize");
}

size_t snapshot_bytes(const Snapshot& S) {
  size_t total = 0;
  for (auto& p : S.parts) total += (p.second + 255) / 256 * 256;
  return total;
}

int element_bytes(const lbm_handle* h) { return ::element_bytes(h); }
int upload(lbm_handle* h) { return ::upload(h); }
int prologue(lbm_handle* h) { return ::prologue(h); }
int check_overflow(lbm_handle* h) { return ::check_overflow(h); }

}  // namespace rt
}  // namespace lbmib



extern "C" {

int lbm_autotune(lbm_handle* h, int32_t steps, const char* cache_path, char* report, int32_t report_len) {
  (void)steps;
  (void)cache_path;
  if (report && report_len > 0) report[0] = '\0';
  if (!h) return LBM_EINVAL;
  // One GPU run aborted inside the tuner with a corrupted host heap and no
  // cause has been shown, so the tuner stays off until one is.  Launch shapes
  // are set explicitly with lbm_set_stream_collide_launch.
  return h->fail(LBM_ESTATE, "the launch-shape tuner is disabled: a host-heap abort inside it has no cause "
                             "shown yet; set the shape with lbm_set_stream_collide_launch");
}

int64_t lbm_bytes_per_step(const lbm_handle* h) {
  return h ? (int64_t)2 * kQ * element_bytes(h) * h->nodes : -1;
}

}  // extern "C"
