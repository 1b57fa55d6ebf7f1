// Immersed-boundary and membrane kernels.
//
//   k_bead_stats      one workgroup per bead: bead centres (mean of the mesh
//                     nodes, Fig. 1 caption), enclosed volumes and the node
//                     region each bead's delta-kernel stencils can touch.
//   k_vertex_forces   32 lanes per mesh node: the membrane forces f = -dW/dr
//                     of the Skalak and Kantor-Nelson bending energies and the
//                     area-vector sum that the volume force scales (Sec. 2.2),
//                     gathered over the node's triangles and hinges (no
//                     atomics); no bead statistics needed.
//   k_stats_forces    both of the above in one launch.
//   (the spreading adds the bead terms: -pv times the area-vector sum and the
//   node's 1/N_v share of the bead's driving and spring force, bead_terms.h)
//   k_spread          two or four workgroups per 8x8x8 tile of a bead region
//                     (each a slab of its z layers): stages the
//                     stencil weights of the markers touching the tile in LDS
//                     (bead order, marker order) and accumulates
//                     F(x) = sum_m f_m Delta(x - r_m) node by node (Eq.
//                     spreading); deterministic, writes the whole tile, stamps
//                     it active for this step.
//   k_interp_advance  a group of 8/32/64 lanes per marker (2/3/4-point kernel):
//                     each lane weights one stencil node's velocity, a
//                     wavefront-shuffle reduction gives U = sum_x u Delta (Eq.
//                     interpolation), and the marker moves r += U.
//
// Delta kernel Delta(d) = phi(dx) phi(dy) phi(dz): the two-point linear kernel
// of Sec. 2.3, the three-point kernel of Roma, Peskin and Berger (1999) and the
// four-point kernel of Peskin (2002).  Stencil of n nodes starting at
// floor(r) (n = 2), floor(r + 1/2) - 1 (n = 3), floor(r) - 1 (n = 4); nodes
// outside it carry zero weight.
//
// Marker positions are FP64 (the per-step motion, ~1e-5 lattice units, is
// below FP32 resolution at box coordinates); differences of positions are
// formed in FP64 and the force arithmetic after that is FP32 except where a
// small difference of O(1) numbers decides the result (metric change of a
// triangle, dihedral angle change of a hinge, volume change).
#include "common.h"
#include "bead_terms.h"
#include "near_marks.h"

namespace lbmib {

namespace {

// Workgroup sizes of the bead-statistics and spreading kernels: wide when a
// handle has few beads (latency of a few workgroups dominates), small when it
// has many (they run beside the bulk stream-collide launch and must fit into
// the wave slots its retiring workgroups free).
constexpr int kStatsBlock = 256;
constexpr int kStatsBlockWide = 1024;
constexpr int kSpreadBlock = 256;
constexpr int kSpreadBlockWide = 512;
constexpr int kInterpBlock = 256;
// Bead statistics: meshes of up to this many nodes (four refinements) are
// staged in LDS for the volume sum; triangle ids loaded per round trip.
constexpr int kStatsLdsVerts = 2562;
constexpr int kStatsTriRounds = 5;

__device__ inline int pmod(int a, int b) {
  int r = a % b;
  return r < 0 ? r + b : r;
}

template <int NW>
__device__ inline float phi(float r) {
  r = fabsf(r);
  if constexpr (NW == 2) {
    return r < 1.0f ? 1.0f - r : 0.0f;
  } else if constexpr (NW == 3) {
    if (r <= 0.5f) return (1.0f + sqrtf(1.0f - 3.0f * r * r)) * (1.0f / 3.0f);
    if (r <= 1.5f) return (5.0f - 3.0f * r - sqrtf(fmaxf(0.0f, 1.0f - 3.0f * (1.0f - r) * (1.0f - r)))) * (1.0f / 6.0f);
    return 0.0f;
  } else {
    if (r <= 1.0f) return (3.0f - 2.0f * r + sqrtf(1.0f + 4.0f * r - 4.0f * r * r)) * 0.125f;
    if (r <= 2.0f) return (5.0f - 2.0f * r - sqrtf(fmaxf(0.0f, -7.0f + 12.0f * r - 4.0f * r * r))) * 0.125f;
    return 0.0f;
  }
}

// First stencil node of a marker coordinate.  The clamp keeps the integer
// conversion defined when a diverged run produces non-finite positions (fmax
// returns the finite operand for NaN); the bead-region check then reports it.
template <int NW>
__device__ inline int stencil_base(double r) {
  r = fmin(fmax(r, -1.0e9), 1.0e9);
  if constexpr (NW == 3) return (int)floor(r + 0.5) - 1;
  if constexpr (NW == 4) return (int)floor(r) - 1;
  return (int)floor(r);
}

__device__ inline double3 load_pos(const double* pos, int nm, int m) {
  return make_double3(pos[m], pos[nm + m], pos[2 * nm + m]);
}

// ---- wavefront reductions ---------------------------------------------------
// Within rows of 16 lanes by DPP moves: pairs and quads by quad permutations,
// then the mirrored half row and the mirrored row, after which every lane of
// a row holds the row's total.  Each step is a register move of the ALU; a
// shuffle routes every step through the LDS unit.
constexpr int kDppXor1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int kDppXor2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int kDppHalfMirror = 0x141;  // lane i <- lane 7 - i of its half row
constexpr int kDppMirror = 0x140;      // lane i <- lane 15 - i of its row

template <int CTRL>
__device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

enum { kRedSum, kRedMin, kRedMax };
template <int OP, typename T>
__device__ inline T red_op(T a, T b) {
  if constexpr (OP == kRedSum) return a + b;
  else if constexpr (OP == kRedMin) return fmin(a, b);  // a NaN operand is dropped
  else return fmax(a, b);
}

// The reduction over each aligned group of L lanes (L a power of two up to
// 64), the result in every lane of the group; the steps beyond a row of 16
// are shuffles.
template <int L, int OP = kRedSum, typename T>
__device__ inline T group_reduce(T v) {
  if constexpr (L >= 2) v = red_op<OP>(v, dpp_move<kDppXor1>(v));
  if constexpr (L >= 4) v = red_op<OP>(v, dpp_move<kDppXor2>(v));
  if constexpr (L >= 8) v = red_op<OP>(v, dpp_move<kDppHalfMirror>(v));
  if constexpr (L >= 16) v = red_op<OP>(v, dpp_move<kDppMirror>(v));
#pragma unroll
  for (int s = 16; s < L; s <<= 1) v = red_op<OP>(v, __shfl_xor(v, s, 64));
  return v;
}

// The reduction over the whole wavefront, the result in every lane: row
// totals by DPP, then the four rows read out and combined in a fixed order.
template <int OP>
__device__ inline double wave_reduce(double v) {
  v = group_reduce<16, OP>(v);
  double r[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    r[k] = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), 16 * k),
                            __builtin_amdgcn_readlane(__double2loint(v), 16 * k));
  return red_op<OP>(red_op<OP>(r[0], r[1]), red_op<OP>(r[2], r[3]));
}

// ---- block reductions -------------------------------------------------------
template <int BS>
__device__ inline double block_sum(double v, double* sh) {
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0;
  for (int i = 0; i < BS / 64; ++i) t += sh[i];
  return t;
}
// ---- bead statistics ----------------------------------------------------------
// One workgroup per bead: centre (mean of nodes), bounding box and enclosed
// volume, reduced in FP64 with wavefront shuffles, and from the box the node
// region the bead's stencils can touch (in 8^3 tiles).
template <int NW, int BS>
__device__ inline void bead_stats_block(const Dev& d, int b, int mark_offset) {
  constexpr int NWAVE = BS / 64;
  constexpr int NV = 10;  // sums x y z, min x y z, max x y z, volume
  __shared__ double part[NWAVE][NV];
  __shared__ int reg_lo[3], reg_hi[3];
  __shared__ double lpos[3][kStatsLdsVerts];
  const Bead Bd = d.beads[b];
  const Box Bx = d.boxes[Bd.box];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  // The enclosed volume 1/6 sum (r0-c).((r1-c) x (r2-c)) of a closed outward
  // surface does not depend on the reference point c; the previous step's
  // centre keeps the products small, and lets one pass reduce everything.
  const BeadState* prev = d.bstate_prev ? d.bstate_prev : d.bstate;
  const double cx = prev[b].c[0], cy = prev[b].c[1], cz = prev[b].c[2];
  double v[NV] = {0, 0, 0, 1e300, 1e300, 1e300, -1e300, -1e300, -1e300, 0};
  // The node positions are loaded once and, for meshes of up to
  // kStatsLdsVerts nodes, staged in LDS, where the volume sum reads the
  // triangle corners; the triangles' corner ids are loaded with the
  // positions, so the kernel makes one round trip to memory for its inputs
  // (it runs beside the bulk stream-collide launch, where trips are slow).
  const bool staged = Bd.nv <= kStatsLdsVerts;
  for (int i = threadIdx.x; i < Bd.nv; i += BS) {
    const double3 p = load_pos(d.pos, d.nm, Bd.first + i);
    if (staged) {
      lpos[0][i] = p.x;
      lpos[1][i] = p.y;
      lpos[2][i] = p.z;
    }
    v[0] += p.x;
    v[1] += p.y;
    v[2] += p.z;
    v[3] = fmin(v[3], p.x);
    v[4] = fmin(v[4], p.y);
    v[5] = fmin(v[5], p.z);
    v[6] = fmax(v[6], p.x);
    v[7] = fmax(v[7], p.y);
    v[8] = fmax(v[8], p.z);
  }
  for (int t0 = 0; t0 < Bd.ntri; t0 += kStatsTriRounds * BS) {
    int ids[kStatsTriRounds][3];
#pragma unroll
    for (int r = 0; r < kStatsTriRounds; ++r) {
      const int t = t0 + r * BS + (int)threadIdx.x;
      const int tt = Bd.tri0 + t;
      ids[r][0] = ids[r][1] = ids[r][2] = -1;
      if (t < Bd.ntri) {
        ids[r][0] = d.tri[tt];
        ids[r][1] = d.tri[d.ntri + tt];
        ids[r][2] = d.tri[2 * d.ntri + tt];
      }
    }
    if (staged) __syncthreads();  // positions staged (uniform: staged depends on the bead only)
#pragma unroll
    for (int r = 0; r < kStatsTriRounds; ++r) {
      if (ids[r][0] < 0) continue;
      double3 p0, p1, p2;
      if (staged) {
        const int i0 = ids[r][0] - Bd.first, i1 = ids[r][1] - Bd.first, i2 = ids[r][2] - Bd.first;
        p0 = make_double3(lpos[0][i0], lpos[1][i0], lpos[2][i0]);
        p1 = make_double3(lpos[0][i1], lpos[1][i1], lpos[2][i1]);
        p2 = make_double3(lpos[0][i2], lpos[1][i2], lpos[2][i2]);
      } else {
        p0 = load_pos(d.pos, d.nm, ids[r][0]);
        p1 = load_pos(d.pos, d.nm, ids[r][1]);
        p2 = load_pos(d.pos, d.nm, ids[r][2]);
      }
      const double ax = p0.x - cx, ay = p0.y - cy, az = p0.z - cz;
      const double bx = p1.x - cx, by = p1.y - cy, bz = p1.z - cz;
      const double qx = p2.x - cx, qy = p2.y - cy, qz = p2.z - cz;
      v[9] += ax * (by * qz - bz * qy) + ay * (bz * qx - bx * qz) + az * (bx * qy - by * qx);
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[k] = wave_reduce<kRedSum>(v[k]);
    v[3 + k] = wave_reduce<kRedMin>(v[3 + k]);
    v[6 + k] = wave_reduce<kRedMax>(v[6 + k]);
  }
  v[9] = wave_reduce<kRedSum>(v[9]);
  if (lane == 0)
    for (int k = 0; k < NV; ++k) part[wave][k] = v[k];
  __syncthreads();
  // each of the first NV threads folds one statistic over the wavefront
  // partials (independent LDS reads, issued back to back)
  if (threadIdx.x < NV) {
    const int k = threadIdx.x;
    double t = part[0][k];
    for (int w = 1; w < NWAVE; ++w) {
      const double x = part[w][k];
      t = (k < 3 || k == 9) ? t + x : (k < 6 ? fmin(t, x) : fmax(t, x));
    }
    part[0][k] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) t[k] = part[0][k];
    BeadState& st = d.bstate[b];
    const int T[3] = {Bx.tx, Bx.ty, Bx.tz};
    const int N[3] = {Bx.nx, Bx.ny, Bx.nz};
    const int reserved[3] = {Bd.tiles_x, Bd.tiles_y, Bd.tiles_z};
    for (int a = 0; a < 3; ++a) st.c[a] = t[a] / Bd.nv;
    st.V = t[9] / 6.0;
    for (int a = 0; a < 3; ++a) {
      st.lo[a] = stencil_base<NW>(t[3 + a]);
      st.hi[a] = stencil_base<NW>(t[6 + a]) + NW - 1;
      // Tiles from the wrapped first node, counted on in periodic tile order
      // (tile T follows tile T - 1): node lo + j lies in tile
      // (u / N) T + (u mod N) / kTile (mod T), u = (lo mod N) + j, which rises
      // by at most one per node, so the region's nodes fill the tile run
      // [t0, t0 + cnt) also on an edge that is not a whole number of tiles.
      // A region shorter than the edge wraps at most once.
      const int lw = pmod(st.lo[a], N[a]);
      const int hw = lw + (st.hi[a] - st.lo[a]);
      int t0 = lw / kTile;
      int cnt = T[a];
      if (hw < lw)
        cnt = 0;  // no region (non-finite positions)
      else if (hw - lw + 1 < N[a])
        cnt = (hw < N[a] ? hw / kTile : T[a] + (hw - N[a]) / kTile) - t0 + 1;
      if (cnt >= T[a]) {
        t0 = 0;
        cnt = T[a];
      }
      if (cnt > reserved[a]) {
        atomicOr(d.overflow, 1);
        cnt = reserved[a];
      }
      if (cnt < 0) cnt = 0;
      st.tlo[a] = t0;
      st.tcnt[a] = cnt;
      reg_lo[a] = st.lo[a];
      reg_hi[a] = st.hi[a];
    }
  }
  __syncthreads();
  // blocks the next step's stream-collide must treat as near this bead
  if (mark_offset != kNoMark) mark_near_blocks(d, Bx, Bd.box, reg_lo, reg_hi, *d.step + d.sub + mark_offset);
}

template <int NW, int BS>
__global__ __launch_bounds__(BS) void k_bead_stats(Dev d, int mark_offset) {
  bead_stats_block<NW, BS>(d, blockIdx.x, mark_offset);
}

// ---- membrane forces ------------------------------------------------------------
// Skalak force on corner `corner` of triangle t.  With
// Delta = g - G0 (metric change, formed in FP64), I1 = G0^-1 : Delta,
// I2 = (det g - det G0)/det G0 and the stress P = dW/dg written so that its
// O(1) parts cancel analytically:
//   P = ks A0/4 [(2 I1 + 2 C I2) G0^-1 + (2 C I2 - 2) adj(Delta)/det G0],
// dW/de1 = 2 (P11 e1 + P12 e2), dW/de2 = 2 (P12 e1 + P22 e2), e_a = r_a - r_0.
// The triangle's area vector (r1 - r0) x (r2 - r0), formed in FP64, goes to
// `area`: the volume force of the corner is -pv times it (bead_terms.h).
__device__ inline float3 triangle_corner(const Dev& d, const Bead& Bd, int t, int corner, int i0, int i1,
                                         int i2, float3& area) {
  const double3 p0 = load_pos(d.pos, d.nm, i0);
  const double3 p1 = load_pos(d.pos, d.nm, i1);
  const double3 p2 = load_pos(d.pos, d.nm, i2);
  const double e1x = p1.x - p0.x, e1y = p1.y - p0.y, e1z = p1.z - p0.z;
  const double e2x = p2.x - p0.x, e2y = p2.y - p0.y, e2z = p2.z - p0.z;
  const double G11d = d.G0[t], G12d = d.G0[d.ntri + t], G22d = d.G0[2 * d.ntri + t];
  const float D11 = (float)(e1x * e1x + e1y * e1y + e1z * e1z - G11d);
  const float D12 = (float)(e1x * e2x + e1y * e2y + e1z * e2z - G12d);
  const float D22 = (float)(e2x * e2x + e2y * e2y + e2z * e2z - G22d);
  const float G11 = (float)G11d, G12 = (float)G12d, G22 = (float)G22d;
  const float Gi11 = d.G0inv[t], Gi12 = d.G0inv[d.ntri + t], Gi22 = d.G0inv[2 * d.ntri + t];
  const float idet = d.idetG0[t];
  const float I1 = Gi11 * D11 + 2.0f * Gi12 * D12 + Gi22 * D22;
  const float I2 = (G11 * D22 + G22 * D11 - 2.0f * G12 * D12 + (D11 * D22 - D12 * D12)) * idet;
  const float k4 = 0.25f * Bd.ks * d.A0[t];
  const float a = k4 * (2.0f * I1 + 2.0f * Bd.C * I2);
  const float bq = k4 * (2.0f * Bd.C * I2 - 2.0f) * idet;
  const float P11 = a * Gi11 + bq * D22;
  const float P12 = a * Gi12 - bq * D12;
  const float P22 = a * Gi22 + bq * D11;
  const float e1[3] = {(float)e1x, (float)e1y, (float)e1z};
  const float e2[3] = {(float)e2x, (float)e2y, (float)e2z};
  float ca, cb;  // force = -(ca e1 + cb e2) from the Skalak energy
  if (corner == 1) {
    ca = 2.0f * P11;
    cb = 2.0f * P12;
  } else if (corner == 2) {
    ca = 2.0f * P12;
    cb = 2.0f * P22;
  } else {
    ca = -2.0f * (P11 + P12);
    cb = -2.0f * (P12 + P22);
  }
  area = make_float3((float)(e1y * e2z - e1z * e2y), (float)(e1z * e2x - e1x * e2z), (float)(e1x * e2y - e1y * e2x));
  return make_float3(-(ca * e1[0] + cb * e2[0]), -(ca * e1[1] + cb * e2[1]), -(ca * e1[2] + cb * e2[2]));
}

// Kantor-Nelson bending force -kt sin(theta - theta0) d theta / d x_role on one
// vertex of hinge h (x1, x2 shared edge; x3, x4 opposite).  With
// nA = (x2-x1) x (x3-x1), nB = (x1-x2) x (x4-x2), e = x2 - x1:
//   d theta/d x3 = -|e| nA/|nA|^2,  d theta/d x4 = -|e| nB/|nB|^2,
//   d theta/d x1 = -((x3-x2).e^) nA/|nA|^2 + ((x2-x4).e^) nB/|nB|^2,
//   d theta/d x2 = -((x1-x3).e^) nA/|nA|^2 + ((x4-x1).e^) nB/|nB|^2.
// sin(theta - theta0) = sin theta cos theta0 - cos theta sin theta0 with
// cos theta = nA.nB/(|nA||nB|), sin theta = (nA x nB).e^/(|nA||nB|), in FP64.
__device__ inline float3 bending_role(const Dev& d, const Bead& Bd, int h, int role, int4 v) {
  const int nh = d.nh;
  const double3 x1 = load_pos(d.pos, d.nm, v.x);
  const double3 x2 = load_pos(d.pos, d.nm, v.y);
  const double3 x3 = load_pos(d.pos, d.nm, v.z);
  const double3 x4 = load_pos(d.pos, d.nm, v.w);
  const double ex = x2.x - x1.x, ey = x2.y - x1.y, ez = x2.z - x1.z;
  const double ax = x3.x - x1.x, ay = x3.y - x1.y, az = x3.z - x1.z;
  const double bx = x4.x - x2.x, by = x4.y - x2.y, bz = x4.z - x2.z;
  const double nAx = ey * az - ez * ay, nAy = ez * ax - ex * az, nAz = ex * ay - ey * ax;
  const double nBx = -(ey * bz - ez * by), nBy = -(ez * bx - ex * bz), nBz = -(ex * by - ey * bx);
  const double nA2 = nAx * nAx + nAy * nAy + nAz * nAz;
  const double nB2 = nBx * nBx + nBy * nBy + nBz * nBz;
  const double E = sqrt(ex * ex + ey * ey + ez * ez);
  const double iE = 1.0 / E;
  const double ehx = ex * iE, ehy = ey * iE, ehz = ez * iE;
  const double cx = nAy * nBz - nAz * nBy, cy = nAz * nBx - nAx * nBz, cz = nAx * nBy - nAy * nBx;
  const double inorm = 1.0 / sqrt(nA2 * nB2);
  const double sn = (cx * ehx + cy * ehy + cz * ehz) * inorm;
  const double cs = (nAx * nBx + nAy * nBy + nAz * nBz) * inorm;
  const float dW = Bd.kt * (float)(sn * d.th0cs[h] - cs * d.th0cs[nh + h]);
  double ca, cb;  // d theta / d x_role = ca nA/|nA|^2 + cb nB/|nB|^2
  if (role == 2) {
    ca = -E;
    cb = 0;
  } else if (role == 3) {
    ca = 0;
    cb = -E;
  } else if (role == 0) {
    ca = -((x3.x - x2.x) * ehx + (x3.y - x2.y) * ehy + (x3.z - x2.z) * ehz);
    cb = (x2.x - x4.x) * ehx + (x2.y - x4.y) * ehy + (x2.z - x4.z) * ehz;
  } else {
    ca = -((x1.x - x3.x) * ehx + (x1.y - x3.y) * ehy + (x1.z - x3.z) * ehz);
    cb = (x4.x - x1.x) * ehx + (x4.y - x1.y) * ehy + (x4.z - x1.z) * ehz;
  }
  const float fa = (float)(ca / nA2), fb = (float)(cb / nB2);
  return make_float3(-dW * (fa * (float)nAx + fb * (float)nBx), -dW * (fa * (float)nAy + fb * (float)nBy),
                     -dW * (fa * (float)nAz + fb * (float)nBz));
}

// 32 lanes per mesh node: lanes 0..7 take the node's incident triangles
// (Skalak force and area vector), lanes 8..31 the hinges it belongs to (its
// own edges and the edges opposite it: bending); a fixed reduction tree sums
// them.  The result is the bead-independent part of the node force
// (bead_terms.h): the kernel reads no bead statistics, so it can run beside
// the statistics of the same step.
constexpr int kVertLanes = 32;
constexpr int kVertTriLanes = 8;
template <int BS>
__device__ inline void vertex_forces_block(const Dev& d, int blk) {
  const int gid = blk * BS + threadIdx.x;
  const int m = gid / kVertLanes, lane = gid % kVertLanes;
  float fx = 0, fy = 0, fz = 0, gx = 0, gy = 0, gz = 0;
  if (m < d.nm) {
    // every load below depends only on this first round of per-marker and
    // per-lane tables, so the kernel makes two dependent trips to memory
    const int4 mi = d.marker_info[m];
    const int e = d.lane_elem[gid];
    const int4 v = d.lane_v[gid];
    if (e >= 0) {
      const Bead Bd = d.beads[mi.x];
      float3 f;
      if (lane < kVertTriLanes) {
        float3 area;
        f = triangle_corner(d, Bd, e / 3, e % 3, v.x, v.y, v.z, area);
        gx = area.x;
        gy = area.y;
        gz = area.z;
      } else {
        f = bending_role(d, Bd, e / 4, e % 4, v);
      }
      fx = f.x;
      fy = f.y;
      fz = f.z;
    }
  }
  fx = group_reduce<kVertLanes>(fx);
  fy = group_reduce<kVertLanes>(fy);
  fz = group_reduce<kVertLanes>(fz);
  gx = group_reduce<kVertLanes>(gx);
  gy = group_reduce<kVertLanes>(gy);
  gz = group_reduce<kVertLanes>(gz);
  if (m < d.nm && lane == 0) {
    d.fmem[m] = fx;
    d.fmem[d.nm + m] = fy;
    d.fmem[2 * d.nm + m] = fz;
    d.gvol[m] = gx;
    d.gvol[d.nm + m] = gy;
    d.gvol[2 * d.nm + m] = gz;
  }
}

__global__ __launch_bounds__(256) void k_vertex_forces(Dev d) { vertex_forces_block<256>(d, blockIdx.x); }

// Bead statistics (the first nbeads workgroups) and the membrane forces (the
// rest) of one step in one launch: neither reads what the other writes.
template <int NW, int BS>
__global__ __launch_bounds__(BS) void k_stats_forces(Dev d, int mark_offset) {
  if ((int)blockIdx.x < d.nbeads)
    bead_stats_block<NW, BS>(d, blockIdx.x, mark_offset);
  else
    vertex_forces_block<BS>(d, (int)blockIdx.x - d.nbeads);
}

// Total force on every marker of step counter + sub into out (observables,
// the adjoint's recorded forces).
__global__ __launch_bounds__(256) void k_marker_force_total(Dev d, float* out) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= d.nm) return;
  const BeadTerms t = d.bterms[d.marker_info[m].x];
  float f[3];
  marker_total(d, m, t, f);
  out[m] = f[0];
  out[d.nm + m] = f[1];
  out[2 * d.nm + m] = f[2];
}

// ---- spreading --------------------------------------------------------------------

// Offset of a marker's stencil from the tile origin, taking the periodic image
// that meets the tile; returns false when no image meets it.
template <int NW>
__device__ inline bool stencil_offset(int base, int origin, int extent, int N, int& off) {
  const int r = pmod(base - origin, N);
  if (r < extent) {
    off = r;
    return true;
  }
  if (r >= N - NW + 1) {
    off = r - N;
    return true;
  }
  return false;
}

// One workgroup per part of a tile (spread_parts: four parts of two z layers
// for handles of few beads, two of four above; each workgroup adds only the
// markers whose stencils meet its part).  Those markers are compacted in (bead,
// marker) order; the thread that finds a marker stages its
// stencil offset, its per-axis kernel weights and its force in LDS.  Entry e
// goes to wavefront e % W (W wavefronts per workgroup), which adds the
// marker's stencil (one lane per stencil node, all distinct) into the
// wavefront's private LDS copy of the tile; the W copies are summed in
// wavefront order.  No atomics, fixed summation order: deterministic.
//
// The kernel runs beside the bulk stream-collide launch, where every
// dependent trip to memory is slow, so its loads are issued in three rounds:
// the block's table entry; the box and the tile regions and mesh ranges of
// all the box's beads (into LDS); then the positions and forces of every
// marker of the beads covering the tile, held in registers (kSpreadRounds
// chunks of BS markers per round trip) while the chunks are staged.
template <int NW>
struct SpreadEntry {
  int off;           // packed stencil offset from the tile origin, +8 per axis
  float w[3][NW];    // per-axis kernel weights of the stencil nodes
  float f[3];        // marker force
};

constexpr int kSpreadBeads = 64;   // beads per box held in LDS (more: read from memory)
constexpr int kSpreadRounds = 4;   // marker chunks loaded per round trip

// Tile region, mesh range and the force terms of the step (volume pressure,
// per-node share of the driving + spring force) of bead i of the box (LDS
// copy or memory).
struct SpreadBead {
  int tlo[3], tcnt[3], first, nv;
  BeadTerms t;
};

__device__ inline SpreadBead make_spread_bead(const Dev& d, int b, int64_t n) {
  const BeadState& s = d.bstate[b];
  const Bead& q = d.beads[b];
  SpreadBead r{{s.tlo[0], s.tlo[1], s.tlo[2]}, {s.tcnt[0], s.tcnt[1], s.tcnt[2]}, q.first, q.nv, {0.0f, {0.0f, 0.0f, 0.0f}}};
  if (!d.spread_raw) r.t = bead_terms(d, b, n);
  return r;
}

__device__ inline SpreadBead spread_bead(const Dev& d, const SpreadBead* sb, int bead0, int nb, int i, int64_t n) {
  if (nb <= kSpreadBeads) return sb[i];
  return make_spread_bead(d, bead0 + i, n);
}

__device__ inline bool covers(const SpreadBead& s, int tx, int ty, int tz, const Box& B) {
  return pmod(tx - s.tlo[0], B.tx) < s.tcnt[0] && pmod(ty - s.tlo[1], B.ty) < s.tcnt[1] &&
         pmod(tz - s.tlo[2], B.tz) < s.tcnt[2];
}


// PARTS workgroups per tile (spread_parts), each kTile / PARTS z layers
template <int NW, int BS, int PARTS>
__global__ __launch_bounds__(BS) void k_spread(Dev d) {
  static_assert(kTile % PARTS == 0, "whole z layers per spreading part");
  constexpr int kPartLayers = kTile / PARTS;
  constexpr int kPartNodes = kTile * kTile * kPartLayers;
  constexpr int kSpreadWaves = BS / 64;
  __shared__ float acc[kSpreadWaves][3][kPartNodes];
  __shared__ SpreadEntry<NW> ent[BS];
  __shared__ int wave_cnt[kSpreadWaves];
  __shared__ SpreadBead sb[kSpreadBeads];
  // round trip 1: the block's bead, box and candidate tile within the bead
  const int4 info = d.spread_info[2 * blockIdx.x];
  const int4 kk = d.spread_info[2 * blockIdx.x + 1];
  const int b = info.x, bead0 = info.z, nb = info.w, own = b - bead0;
  // round trip 2: the box and every bead of the box
  const Box B = d.boxes[info.y];
  const int64_t n = *d.step + d.sub;
  if (nb <= kSpreadBeads)
    for (int i = threadIdx.x; i < nb; i += BS) sb[i] = make_spread_bead(d, bead0 + i, n);
  __syncthreads();
  const SpreadBead S = spread_bead(d, sb, bead0, nb, own, n);
  // the first candidate block of each bead keeps its terms for the total
  // marker forces formed later in the step
  if (!d.spread_raw && threadIdx.x == 0 && kk.x == 0 && kk.y == 0 && kk.z == 0 && kk.w == 0) d.bterms[b] = S.t;
  if (kk.x >= S.tcnt[0] || kk.y >= S.tcnt[1] || kk.z >= S.tcnt[2]) return;
  const int tx = pmod(S.tlo[0] + kk.x, B.tx), ty = pmod(S.tlo[1] + kk.y, B.ty), tz = pmod(S.tlo[2] + kk.z, B.tz);
  for (int i = 0; i < own; ++i)
    if (covers(spread_bead(d, sb, bead0, nb, i, n), tx, ty, tz, B)) return;  // an earlier bead owns this tile
  // this workgroup's part: z layers [oz, oz + ez) of the tile, ez <= kPartLayers
  const int ox = tx * kTile, oy = ty * kTile, oz = tz * kTile + kPartLayers * kk.w;
  const int ex = min(kTile, B.nx - ox), ey = min(kTile, B.ny - oy), ez = min(kPartLayers, B.nz - oz);
  if (kk.w == 0 && threadIdx.x == 0) d.stamp[B.tile0 + tx + B.tx * (ty + B.ty * tz)] = (int)n;
  if (ez <= 0) return;  // an upper part of a short tile at the box's end holds no node
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  for (int w = 0; w < kSpreadWaves; ++w)
    for (int nd = threadIdx.x; nd < kPartNodes; nd += BS) {
      acc[w][0][nd] = 0.0f;
      acc[w][1][nd] = 0.0f;
      acc[w][2][nd] = 0.0f;
    }
  // stencil node of this lane (NW^3 <= 64 lanes used)
  const int sa = lane % NW, sb_ = (lane / NW) % NW, sc = lane / (NW * NW);
  // chunks (covering bead, first marker) in order: this bead, then the later
  // beads of the box that cover the tile; kSpreadRounds chunks per load round
  int cb = own, c0 = 0;  // next chunk to load
  SpreadBead Q = S;
  while (cb < nb) {
    double px[kSpreadRounds], py[kSpreadRounds], pz[kSpreadRounds];
    float fx[kSpreadRounds], fy[kSpreadRounds], fz[kSpreadRounds];
    int nvr[kSpreadRounds];  // markers of each loaded chunk's bead left from its first (0: no chunk)
    int nr = 0;
#pragma unroll
    for (int r = 0; r < kSpreadRounds; ++r) {
      nvr[r] = 0;
      px[r] = py[r] = pz[r] = 0.0;
      fx[r] = fy[r] = fz[r] = 0.0f;
      if (cb >= nb) continue;
      const int i = c0 + (int)threadIdx.x;
      nvr[r] = Q.nv - c0;
      if (i < Q.nv) {
        const int m = Q.first + i;
        px[r] = d.pos[m];
        py[r] = d.pos[d.nm + m];
        pz[r] = d.pos[2 * d.nm + m];
        if (d.spread_raw) {
          fx[r] = d.fm[m];
          fy[r] = d.fm[d.nm + m];
          fz[r] = d.fm[2 * d.nm + m];
        } else {
          fx[r] = total_force(d.fmem[m], d.gvol[m], Q.t.pv, Q.t.share[0]);
          fy[r] = total_force(d.fmem[d.nm + m], d.gvol[d.nm + m], Q.t.pv, Q.t.share[1]);
          fz[r] = total_force(d.fmem[2 * d.nm + m], d.gvol[2 * d.nm + m], Q.t.pv, Q.t.share[2]);
        }
      }
      ++nr;
      // advance to the next chunk: the rest of this bead, else the next
      // later bead that covers the tile
      c0 += BS;
      if (c0 >= Q.nv) {
        c0 = 0;
        for (++cb; cb < nb; ++cb) {
          Q = spread_bead(d, sb, bead0, nb, cb, n);
          if (covers(Q, tx, ty, tz, B)) break;
        }
      }
    }
#pragma unroll
    for (int r = 0; r < kSpreadRounds; ++r) {
      if (r >= nr) break;
      bool take = false;
      int offx = 0, offy = 0, offz = 0;
      int bx = 0, by = 0, bz = 0;
      if ((int)threadIdx.x < nvr[r]) {
        bx = stencil_base<NW>(px[r]);
        by = stencil_base<NW>(py[r]);
        bz = stencil_base<NW>(pz[r]);
        take = stencil_offset<NW>(bx, ox, ex, B.nx, offx) && stencil_offset<NW>(by, oy, ey, B.ny, offy) &&
               stencil_offset<NW>(bz, oz, ez, B.nz, offz);
      }
      const unsigned long long mask = __ballot(take);
      const int before = __popcll(mask & ((1ull << lane) - 1ull));
      __syncthreads();  // previous chunk's entries fully consumed
      if (lane == 0) wave_cnt[wave] = __popcll(mask);
      __syncthreads();
      int slot = before, total = 0;
      for (int w = 0; w < kSpreadWaves; ++w) {
        if (w < wave) slot += wave_cnt[w];
        total += wave_cnt[w];
      }
      if (take) {
        SpreadEntry<NW>& E = ent[slot];
        E.off = ((offx + 8) << 10) | ((offy + 8) << 5) | (offz + 8);
#pragma unroll
        for (int a = 0; a < NW; ++a) {
          E.w[0][a] = phi<NW>((float)((double)(bx + a) - px[r]));
          E.w[1][a] = phi<NW>((float)((double)(by + a) - py[r]));
          E.w[2][a] = phi<NW>((float)((double)(bz + a) - pz[r]));
        }
        E.f[0] = fx[r];
        E.f[1] = fy[r];
        E.f[2] = fz[r];
      }
      __syncthreads();
      if (lane < NW * NW * NW) {
        for (int e = wave; e < total; e += kSpreadWaves) {
          const SpreadEntry<NW>& E = ent[e];
          const int lx = ((E.off >> 10) & 31) - 8 + sa;
          const int ly = ((E.off >> 5) & 31) - 8 + sb_;
          const int lz = (E.off & 31) - 8 + sc;
          if ((unsigned)lx < (unsigned)ex && (unsigned)ly < (unsigned)ey && (unsigned)lz < (unsigned)ez) {
            const float w = E.w[0][sa] * E.w[1][sb_] * E.w[2][sc];
            const int node = lx + kTile * (ly + kTile * lz);  // lz < ez <= kPartLayers
            acc[wave][0][node] += w * E.f[0];
            acc[wave][1][node] += w * E.f[1];
            acc[wave][2][node] += w * E.f[2];
          }
        }
      }
    }
  }
  __syncthreads();
  for (int nd = threadIdx.x; nd < kPartNodes; nd += BS) {
    const int lx = nd % kTile, ly = (nd / kTile) % kTile, lz = nd / (kTile * kTile);
    if (lx < ex && ly < ey && lz < ez) {
      float ax = 0, ay = 0, az = 0;
      for (int w = 0; w < kSpreadWaves; ++w) {
        ax += acc[w][0][nd];
        ay += acc[w][1][nd];
        az += acc[w][2][nd];
      }
      const int64_t node = B.node0 + (int64_t)(oz + lz) * B.nx * B.ny + (int64_t)(oy + ly) * B.nx + (ox + lx);
      d.F[node] = ax;
      d.F[d.pstride + node] = ay;
      d.F[2 * d.pstride + node] = az;
    }
  }
}

// ---- interpolation and advection -----------------------------------------------------
template <int NW>
__global__ __launch_bounds__(kInterpBlock) void k_interp_advance(Dev d) {
  constexpr int L = NW == 2 ? 8 : (NW == 3 ? 32 : 64);
  // the next bead statistics (step *d.step + d.sub) list near blocks under
  // that step's parity; the list was last read by the active launch that
  // preceded this kernel
  if (blockIdx.x == 0 && threadIdx.x == 0) d.near_count[(int)((*d.step + d.sub) & 1)] = 0;
  const int gid = blockIdx.x * kInterpBlock + threadIdx.x;
  const int m = gid / L, lane = gid % L;
  float ux = 0, uy = 0, uz = 0;
  if (m < d.nm && lane < NW * NW * NW) {
    const int a = lane % NW, bb = (lane / NW) % NW, c = lane / (NW * NW);
    const double3 p = load_pos(d.pos, d.nm, m);
    Box B;
    if (d.nboxes == 1)
      B = d.boxes[0];
    else
      B = d.boxes[d.marker_info[m].y];
    const int bx = stencil_base<NW>(p.x) + a, by = stencil_base<NW>(p.y) + bb, bz = stencil_base<NW>(p.z) + c;
    const float w = phi<NW>((float)((double)bx - p.x)) * phi<NW>((float)((double)by - p.y)) *
                    phi<NW>((float)((double)bz - p.z));
    const int64_t node = B.node0 + ((int64_t)pmod(bz, B.nz) * B.ny + pmod(by, B.ny)) * B.nx + pmod(bx, B.nx);
    ux = w * d.u[node];
    uy = w * d.u[d.pstride + node];
    uz = w * d.u[2 * d.pstride + node];
  }
  ux = group_reduce<L>(ux);
  uy = group_reduce<L>(uy);
  uz = group_reduce<L>(uz);
  if (m < d.nm && lane == 0) {
    d.U[m] = ux;
    d.U[d.nm + m] = uy;
    d.U[2 * d.nm + m] = uz;
    double* out = d.pos_next ? d.pos_next : d.pos;
    out[m] = d.pos[m] + (double)ux;
    out[d.nm + m] = d.pos[d.nm + m] + (double)uy;
    out[2 * d.nm + m] = d.pos[2 * d.nm + m] + (double)uz;
  }
}

// Bead centres of the current marker positions (observable), FP64.
__global__ __launch_bounds__(kStatsBlock) void k_bead_centres(Dev d, double* out) {
  __shared__ double sh[kStatsBlock / 64];
  const Bead Bd = d.beads[blockIdx.x];
  double s[3] = {0, 0, 0};
  for (int i = threadIdx.x; i < Bd.nv; i += kStatsBlock) {
    const double3 p = load_pos(d.pos, d.nm, Bd.first + i);
    s[0] += p.x;
    s[1] += p.y;
    s[2] += p.z;
  }
  for (int a = 0; a < 3; ++a) {
    const double t = block_sum<kStatsBlock>(s[a], sh);
    if (threadIdx.x == 0) out[3 * blockIdx.x + a] = t / Bd.nv;
  }
}

}  // namespace

template <int BS>
static void launch_stats_bs(const Dev& d, int mark_offset, hipStream_t s) {
  if (d.width == 2) hipLaunchKernelGGL((k_bead_stats<2, BS>), dim3(d.nbeads), dim3(BS), 0, s, d, mark_offset);
  else if (d.width == 3) hipLaunchKernelGGL((k_bead_stats<3, BS>), dim3(d.nbeads), dim3(BS), 0, s, d, mark_offset);
  else hipLaunchKernelGGL((k_bead_stats<4, BS>), dim3(d.nbeads), dim3(BS), 0, s, d, mark_offset);
}

void launch_bead_stats(const Dev& d, int mark_offset, hipStream_t s) {
  if (d.nbeads <= kWideBeads)
    launch_stats_bs<kStatsBlockWide>(d, mark_offset, s);
  else
    launch_stats_bs<kStatsBlock>(d, mark_offset, s);
}

// Few beads: statistics and forces in one launch of wide workgroups; many
// beads: two launches (the statistics' LDS would otherwise cap the force
// workgroups per CU).
void launch_stats_forces(const Dev& d, int mark_offset, hipStream_t s) {
  if (d.nbeads <= kWideBeads) {
    constexpr int BS = kStatsBlockWide;
    const int grid = d.nbeads + (int)(((int64_t)d.nm * kVertLanes + BS - 1) / BS);
    if (d.width == 2) hipLaunchKernelGGL((k_stats_forces<2, BS>), dim3(grid), dim3(BS), 0, s, d, mark_offset);
    else if (d.width == 3) hipLaunchKernelGGL((k_stats_forces<3, BS>), dim3(grid), dim3(BS), 0, s, d, mark_offset);
    else hipLaunchKernelGGL((k_stats_forces<4, BS>), dim3(grid), dim3(BS), 0, s, d, mark_offset);
  } else {
    launch_stats_bs<kStatsBlock>(d, mark_offset, s);
    const int blocks = (int)(((int64_t)d.nm * kVertLanes + 255) / 256);
    hipLaunchKernelGGL(k_vertex_forces, dim3(blocks), dim3(256), 0, s, d);
  }
}

void launch_marker_force_total(const Dev& d, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_marker_force_total, dim3((d.nm + 255) / 256), dim3(256), 0, s, d, out);
}

template <int BS, int PARTS>
static void launch_spread_bs(const Dev& d, hipStream_t s) {
  if (d.width == 2) hipLaunchKernelGGL((k_spread<2, BS, PARTS>), dim3(d.spread_blocks), dim3(BS), 0, s, d);
  else if (d.width == 3) hipLaunchKernelGGL((k_spread<3, BS, PARTS>), dim3(d.spread_blocks), dim3(BS), 0, s, d);
  else hipLaunchKernelGGL((k_spread<4, BS, PARTS>), dim3(d.spread_blocks), dim3(BS), 0, s, d);
}

// the part count follows the same rule as the host's candidate-block table
void launch_spread(const Dev& d, hipStream_t s) {
  if (spread_parts(d.nbeads) == kSpreadPartsWide)
    launch_spread_bs<kSpreadBlockWide, kSpreadPartsWide>(d, s);
  else
    launch_spread_bs<kSpreadBlock, kSpreadPartsNarrow>(d, s);
}

void launch_interp_advance(const Dev& d, hipStream_t s) {
  const int L = d.width == 2 ? 8 : (d.width == 3 ? 32 : 64);
  const int blocks = (int)(((int64_t)d.nm * L + kInterpBlock - 1) / kInterpBlock);
  if (d.width == 2) hipLaunchKernelGGL(k_interp_advance<2>, dim3(blocks), dim3(kInterpBlock), 0, s, d);
  else if (d.width == 3) hipLaunchKernelGGL(k_interp_advance<3>, dim3(blocks), dim3(kInterpBlock), 0, s, d);
  else hipLaunchKernelGGL(k_interp_advance<4>, dim3(blocks), dim3(kInterpBlock), 0, s, d);
}

void launch_bead_centres(const Dev& d, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_bead_centres, dim3(d.nbeads), dim3(kStatsBlock), 0, s, d, out);
}

}  // namespace lbmib
