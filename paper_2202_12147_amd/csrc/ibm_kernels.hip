// Immersed-boundary and membrane kernels.
//
//   k_bead_stats      one workgroup per swimmer: bead centres (mean of the mesh
//                     nodes, Fig. 1 caption), enclosed volumes, the node region
//                     each bead's delta-kernel stencils can touch, and the
//                     driving + spring force on each bead (Sec. 2.2).
//   k_vertex_forces   one thread per mesh node: membrane forces f = -dW/dr of
//                     the Skalak, Kantor-Nelson bending and volume energies
//                     (Sec. 2.2), gathered over the node's triangles and hinges
//                     (no atomics), plus the node's 1/N_v share of the bead force.
//   k_spread          one workgroup per 8x8x8 tile of a bead region: stages the
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

namespace lbmib {

namespace {

constexpr int kStatsBlock = 256;
constexpr int kSpreadBlock = kTile * kTile * kTile;  // 512, one thread per node
constexpr int kInterpBlock = 256;

__device__ inline int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
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
template <int BS>
__device__ inline double block_min(double v, double* sh) {
  for (int s = 32; s > 0; s >>= 1) v = fmin(v, __shfl_xor(v, s, 64));
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = sh[0];
  for (int i = 1; i < BS / 64; ++i) t = fmin(t, sh[i]);
  return t;
}
template <int BS>
__device__ inline double block_max(double v, double* sh) {
  for (int s = 32; s > 0; s >>= 1) v = fmax(v, __shfl_xor(v, s, 64));
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = sh[0];
  for (int i = 1; i < BS / 64; ++i) t = fmax(t, sh[i]);
  return t;
}

// ---- bead statistics ----------------------------------------------------------
template <int NW>
__global__ __launch_bounds__(kStatsBlock) void k_bead_stats(Dev d) {
  __shared__ double sh[kStatsBlock / 64];
  __shared__ double cen[3][3];
  const Swimmer S = d.swimmers[blockIdx.x];
  const int64_t n = *d.step;
  for (int k = 0; k < 3; ++k) {
    const int b = S.bead[k];
    const Bead Bd = d.beads[b];
    double sx = 0, sy = 0, sz = 0;
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int i = threadIdx.x; i < Bd.nv; i += kStatsBlock) {
      const double3 p = load_pos(d.pos, d.nm, Bd.first + i);
      sx += p.x;
      sy += p.y;
      sz += p.z;
      mn[0] = fmin(mn[0], p.x);
      mn[1] = fmin(mn[1], p.y);
      mn[2] = fmin(mn[2], p.z);
      mx[0] = fmax(mx[0], p.x);
      mx[1] = fmax(mx[1], p.y);
      mx[2] = fmax(mx[2], p.z);
    }
    const double inv = 1.0 / Bd.nv;
    const double c[3] = {block_sum<kStatsBlock>(sx, sh) * inv, block_sum<kStatsBlock>(sy, sh) * inv,
                         block_sum<kStatsBlock>(sz, sh) * inv};
    double lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = block_min<kStatsBlock>(mn[a], sh);
      hi[a] = block_max<kStatsBlock>(mx[a], sh);
    }
    // enclosed volume, relative to the centre
    double v = 0;
    for (int t = threadIdx.x; t < Bd.ntri; t += kStatsBlock) {
      const int tt = Bd.tri0 + t;
      const double3 p0 = load_pos(d.pos, d.nm, d.tri[tt]);
      const double3 p1 = load_pos(d.pos, d.nm, d.tri[d.ntri + tt]);
      const double3 p2 = load_pos(d.pos, d.nm, d.tri[2 * d.ntri + tt]);
      const double ax = p0.x - c[0], ay = p0.y - c[1], az = p0.z - c[2];
      const double bx = p1.x - c[0], by = p1.y - c[1], bz = p1.z - c[2];
      const double qx = p2.x - c[0], qy = p2.y - c[1], qz = p2.z - c[2];
      v += ax * (by * qz - bz * qy) + ay * (bz * qx - bx * qz) + az * (bx * qy - by * qx);
    }
    v = block_sum<kStatsBlock>(v, sh) / 6.0;
    if (threadIdx.x == 0) {
      BeadState& st = d.bstate[b];
      const Box B = d.boxes[Bd.box];
      const int T[3] = {B.tx, B.ty, B.tz};
      const int reserved[3] = {Bd.tiles_x, Bd.tiles_y, Bd.tiles_z};
      for (int a = 0; a < 3; ++a) {
        st.c[a] = c[a];
        cen[k][a] = c[a];
        st.lo[a] = stencil_base<NW>(lo[a]);
        st.hi[a] = stencil_base<NW>(hi[a]) + NW - 1;
        int t0 = floor_div(st.lo[a], kTile);
        int cnt = floor_div(st.hi[a], kTile) - t0 + 1;
        if (cnt >= T[a]) {
          t0 = 0;
          cnt = T[a];
        }
        if (cnt > reserved[a]) {
          atomicOr(d.overflow, 1);
          cnt = reserved[a];
        }
        st.tlo[a] = t0;
        st.tcnt[a] = cnt;
      }
      st.V = v;
    }
    __syncthreads();
  }
  // driving forces (Sec. 2.2, Eq. ext forces) and harmonic springs between
  // bead centres: f1 = -k (|R1-R2| - L) (R1-R2)/|R1-R2|, f2 = -f1 - f3
  if (threadIdx.x == 0) {
    const double t = (double)n;
    const double f1 = S.A * sin(S.omega * t + S.phi0);
    const double f3 = S.B * sin(S.omega * t + S.phi0 + S.alpha);
    double fb[3][3] = {{f1, 0, 0}, {-f1 - f3, 0, 0}, {f3, 0, 0}};
    for (int sp = 0; sp < 2; ++sp) {
      const int outer = sp == 0 ? 0 : 2;
      const double dx = cen[outer][0] - cen[1][0], dy = cen[outer][1] - cen[1][1],
                   dz = cen[outer][2] - cen[1][2];
      const double len = sqrt(dx * dx + dy * dy + dz * dz);
      const double s = -S.k[sp] * (len - S.L0[sp]) / len;
      fb[outer][0] += s * dx;
      fb[outer][1] += s * dy;
      fb[outer][2] += s * dz;
      fb[1][0] -= s * dx;
      fb[1][1] -= s * dy;
      fb[1][2] -= s * dz;
    }
    for (int k = 0; k < 3; ++k)
      for (int a = 0; a < 3; ++a) d.bstate[S.bead[k]].fb[a] = fb[k][a];
  }
}

// ---- membrane forces ------------------------------------------------------------
// Skalak force on corner `corner` of triangle t.  With Delta = g - G0 (metric
// change, formed in FP64), I1 = G0^-1 : Delta, I2 = (det g - det G0)/det G0 and
// the stress P = dW/dg written so that the O(1) parts cancel analytically:
// P = ks A0/4 [(2 I1 + 2 C I2) G0^-1 + (2 C I2 - 2) adj(Delta)/det G0].
__device__ inline float3 skalak_corner(const Dev& d, const Bead& Bd, int t, int corner) {
  const int i0 = d.tri[t], i1 = d.tri[d.ntri + t], i2 = d.tri[2 * d.ntri + t];
  const double3 p0 = load_pos(d.pos, d.nm, i0);
  const double3 p1 = load_pos(d.pos, d.nm, i1);
  const double3 p2 = load_pos(d.pos, d.nm, i2);
  const double e1x = p1.x - p0.x, e1y = p1.y - p0.y, e1z = p1.z - p0.z;
  const double e2x = p2.x - p0.x, e2y = p2.y - p0.y, e2z = p2.z - p0.z;
  const float D11 = (float)(e1x * e1x + e1y * e1y + e1z * e1z - d.G0[t]);
  const float D12 = (float)(e1x * e2x + e1y * e2y + e1z * e2z - d.G0[d.ntri + t]);
  const float D22 = (float)(e2x * e2x + e2y * e2y + e2z * e2z - d.G0[2 * d.ntri + t]);
  const float G11 = (float)d.G0[t], G12 = (float)d.G0[d.ntri + t], G22 = (float)d.G0[2 * d.ntri + t];
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
  const float3 e1 = make_float3((float)e1x, (float)e1y, (float)e1z);
  const float3 e2 = make_float3((float)e2x, (float)e2y, (float)e2z);
  // dW/de1 = 2 (P11 e1 + P12 e2), dW/de2 = 2 (P12 e1 + P22 e2); e_a = r_a - r_0
  if (corner == 1)
    return make_float3(-2.0f * (P11 * e1.x + P12 * e2.x), -2.0f * (P11 * e1.y + P12 * e2.y),
                       -2.0f * (P11 * e1.z + P12 * e2.z));
  if (corner == 2)
    return make_float3(-2.0f * (P12 * e1.x + P22 * e2.x), -2.0f * (P12 * e1.y + P22 * e2.y),
                       -2.0f * (P12 * e1.z + P22 * e2.z));
  return make_float3(2.0f * ((P11 + P12) * e1.x + (P12 + P22) * e2.x),
                     2.0f * ((P11 + P12) * e1.y + (P12 + P22) * e2.y),
                     2.0f * ((P11 + P12) * e1.z + (P12 + P22) * e2.z));
}

// Kantor-Nelson bending force kt sin(theta - theta0) * (-d theta / d x_role) on
// one vertex of hinge h (x1, x2 shared edge; x3, x4 opposite).  With
// nA = (x2-x1) x (x3-x1), nB = (x1-x2) x (x4-x2), e = x2 - x1:
//   d theta/d x3 = -|e| nA/|nA|^2,  d theta/d x4 = -|e| nB/|nB|^2,
//   d theta/d x1 = -((x3-x2).e^) nA/|nA|^2 + ((x2-x4).e^) nB/|nB|^2,
//   d theta/d x2 = -((x1-x3).e^) nA/|nA|^2 + ((x4-x1).e^) nB/|nB|^2.
__device__ inline float3 bending_role(const Dev& d, const Bead& Bd, int h, int role) {
  const int nh = d.nh;
  const double3 x1 = load_pos(d.pos, d.nm, d.hinge[h]);
  const double3 x2 = load_pos(d.pos, d.nm, d.hinge[nh + h]);
  const double3 x3 = load_pos(d.pos, d.nm, d.hinge[2 * nh + h]);
  const double3 x4 = load_pos(d.pos, d.nm, d.hinge[3 * nh + h]);
  const double ex = x2.x - x1.x, ey = x2.y - x1.y, ez = x2.z - x1.z;
  const double ax = x3.x - x1.x, ay = x3.y - x1.y, az = x3.z - x1.z;
  const double bx = x4.x - x2.x, by = x4.y - x2.y, bz = x4.z - x2.z;
  // nA = e x a ; nB = (-e) x b
  const double nAx = ey * az - ez * ay, nAy = ez * ax - ex * az, nAz = ex * ay - ey * ax;
  const double nBx = -(ey * bz - ez * by), nBy = -(ez * bx - ex * bz), nBz = -(ex * by - ey * bx);
  const double nA2 = nAx * nAx + nAy * nAy + nAz * nAz;
  const double nB2 = nBx * nBx + nBy * nBy + nBz * nBz;
  const double E = sqrt(ex * ex + ey * ey + ez * ez);
  // signed angle from nA to nB about e
  const double cx = nAy * nBz - nAz * nBy, cy = nAz * nBx - nAx * nBz, cz = nAx * nBy - nAy * nBx;
  const double th = atan2((cx * ex + cy * ey + cz * ez) / E, nAx * nBx + nAy * nBy + nAz * nBz);
  const float dW = Bd.kt * (float)sin(th - (double)d.theta0[h]);
  double ca, cb;  // coefficients of nA/|nA|^2 and nB/|nB|^2 in d theta / d x_role
  const double ehx = ex / E, ehy = ey / E, ehz = ez / E;
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

__global__ __launch_bounds__(256) void k_vertex_forces(Dev d) {
  const int m = blockIdx.x * 256 + threadIdx.x;
  if (m >= d.nm) return;
  const int b = d.marker_bead[m];
  const Bead Bd = d.beads[b];
  const BeadState st = d.bstate[b];
  float fx = 0, fy = 0, fz = 0;
  // volume penalty: f = -kv (V - V0)/V0 dV/dr, dV/dr = 1/6 sum (r_b - c) x (r_c - c)
  const float pref = (float)(Bd.kv * (st.V - Bd.V0) / Bd.V0) * (1.0f / 6.0f);
  for (int k = d.vt_off[m]; k < d.vt_off[m + 1]; ++k) {
    const int e = d.vt[k];
    const int t = e / 3, corner = e % 3;
    const float3 f = skalak_corner(d, Bd, t, corner);
    fx += f.x;
    fy += f.y;
    fz += f.z;
    const int jb = d.tri[((corner + 1) % 3) * d.ntri + t];
    const int jc = d.tri[((corner + 2) % 3) * d.ntri + t];
    const double3 pb = load_pos(d.pos, d.nm, jb), pc = load_pos(d.pos, d.nm, jc);
    const float bx = (float)(pb.x - st.c[0]), by = (float)(pb.y - st.c[1]), bz = (float)(pb.z - st.c[2]);
    const float cx = (float)(pc.x - st.c[0]), cy = (float)(pc.y - st.c[1]), cz = (float)(pc.z - st.c[2]);
    fx -= pref * (by * cz - bz * cy);
    fy -= pref * (bz * cx - bx * cz);
    fz -= pref * (bx * cy - by * cx);
  }
  for (int k = d.vh_off[m]; k < d.vh_off[m + 1]; ++k) {
    const int e = d.vh[k];
    const float3 f = bending_role(d, Bd, e / 4, e % 4);
    fx += f.x;
    fy += f.y;
    fz += f.z;
  }
  const float inv = 1.0f / (float)Bd.nv;
  d.fm[m] = fx + (float)st.fb[0] * inv;
  d.fm[d.nm + m] = fy + (float)st.fb[1] * inv;
  d.fm[2 * d.nm + m] = fz + (float)st.fb[2] * inv;
}

// ---- spreading --------------------------------------------------------------------
__device__ inline bool covers(const BeadState& s, int tx, int ty, int tz, const Box& B) {
  return pmod(tx - s.tlo[0], B.tx) < s.tcnt[0] && pmod(ty - s.tlo[1], B.ty) < s.tcnt[1] &&
         pmod(tz - s.tlo[2], B.tz) < s.tcnt[2];
}

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

struct SpreadEntry {
  int ox, oy, oz;
  float wx[4], wy[4], wz[4];
  float f[3];
};

template <int NW>
__global__ __launch_bounds__(kSpreadBlock) void k_spread(Dev d) {
  __shared__ SpreadEntry ent[kSpreadBlock];
  __shared__ int wave_cnt[kSpreadBlock / 64];
  const int blk = blockIdx.x;
  const int b = d.spread_bead[blk];
  const Bead Bd = d.beads[b];
  const BeadState S = d.bstate[b];
  const int k = blk - Bd.tile_block0;
  const int kx = k % Bd.tiles_x, ky = (k / Bd.tiles_x) % Bd.tiles_y, kz = k / (Bd.tiles_x * Bd.tiles_y);
  if (kx >= S.tcnt[0] || ky >= S.tcnt[1] || kz >= S.tcnt[2]) return;
  const Box B = d.boxes[Bd.box];
  const int tx = pmod(S.tlo[0] + kx, B.tx), ty = pmod(S.tlo[1] + ky, B.ty), tz = pmod(S.tlo[2] + kz, B.tz);
  for (int b2 = B.bead0; b2 < b; ++b2)
    if (covers(d.bstate[b2], tx, ty, tz, B)) return;  // an earlier bead owns this tile
  const int64_t n = *d.step;
  const int ox = tx * kTile, oy = ty * kTile, oz = tz * kTile;
  const int ex = min(kTile, B.nx - ox), ey = min(kTile, B.ny - oy), ez = min(kTile, B.nz - oz);
  const int lx = threadIdx.x % kTile, ly = (threadIdx.x / kTile) % kTile, lz = threadIdx.x / (kTile * kTile);
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  float ax = 0, ay = 0, az = 0;
  for (int b2 = b; b2 < B.bead0 + B.nbeads; ++b2) {
    if (b2 != b && !covers(d.bstate[b2], tx, ty, tz, B)) continue;
    const Bead Q = d.beads[b2];
    for (int c0 = 0; c0 < Q.nv; c0 += kSpreadBlock) {
      const int i = c0 + (int)threadIdx.x;
      bool take = false;
      int offx = 0, offy = 0, offz = 0;
      double3 p = make_double3(0, 0, 0);
      if (i < Q.nv) {
        p = load_pos(d.pos, d.nm, Q.first + i);
        take = stencil_offset<NW>(stencil_base<NW>(p.x), ox, ex, B.nx, offx) &&
               stencil_offset<NW>(stencil_base<NW>(p.y), oy, ey, B.ny, offy) &&
               stencil_offset<NW>(stencil_base<NW>(p.z), oz, ez, B.nz, offz);
      }
      // deterministic compaction: slot = markers taken before this one
      const unsigned long long mask = __ballot(take);
      const int before = __popcll(mask & ((1ull << lane) - 1ull));
      if (lane == 0) wave_cnt[wave] = __popcll(mask);
      __syncthreads();
      int slot = before, total = 0;
      for (int w = 0; w < kSpreadBlock / 64; ++w) {
        if (w < wave) slot += wave_cnt[w];
        total += wave_cnt[w];
      }
      if (take) {
        SpreadEntry& E = ent[slot];
        E.ox = offx;
        E.oy = offy;
        E.oz = offz;
        const int bx = stencil_base<NW>(p.x), by = stencil_base<NW>(p.y), bz = stencil_base<NW>(p.z);
#pragma unroll
        for (int a = 0; a < NW; ++a) {
          E.wx[a] = phi<NW>((float)((double)(bx + a) - p.x));
          E.wy[a] = phi<NW>((float)((double)(by + a) - p.y));
          E.wz[a] = phi<NW>((float)((double)(bz + a) - p.z));
        }
        const int m = Q.first + i;
        E.f[0] = d.fm[m];
        E.f[1] = d.fm[d.nm + m];
        E.f[2] = d.fm[2 * d.nm + m];
      }
      __syncthreads();
      for (int e = 0; e < total; ++e) {
        const int ix = lx - ent[e].ox, iy = ly - ent[e].oy, iz = lz - ent[e].oz;
        if ((unsigned)ix < (unsigned)NW && (unsigned)iy < (unsigned)NW && (unsigned)iz < (unsigned)NW) {
          const float w = ent[e].wx[ix] * ent[e].wy[iy] * ent[e].wz[iz];
          ax += w * ent[e].f[0];
          ay += w * ent[e].f[1];
          az += w * ent[e].f[2];
        }
      }
      __syncthreads();
    }
  }
  if (lx < ex && ly < ey && lz < ez) {
    const int64_t node = B.node0 + (int64_t)(oz + lz) * B.nx * B.ny + (int64_t)(oy + ly) * B.nx + (ox + lx);
    d.F[node] = ax;
    d.F[d.pstride + node] = ay;
    d.F[2 * d.pstride + node] = az;
  }
  if (threadIdx.x == 0) d.stamp[B.tile0 + tx + B.tx * (ty + B.ty * tz)] = (int)n;
}

// ---- interpolation and advection -----------------------------------------------------
template <int NW>
__global__ __launch_bounds__(kInterpBlock) void k_interp_advance(Dev d) {
  constexpr int L = NW == 2 ? 8 : (NW == 3 ? 32 : 64);
  if (blockIdx.x == 0 && threadIdx.x == 0)
    atomicAdd(reinterpret_cast<unsigned long long*>(d.step), 1ull);
  const int gid = blockIdx.x * kInterpBlock + threadIdx.x;
  const int m = gid / L, lane = gid % L;
  float ux = 0, uy = 0, uz = 0;
  if (m < d.nm && lane < NW * NW * NW) {
    const int a = lane % NW, bb = (lane / NW) % NW, c = lane / (NW * NW);
    const double3 p = load_pos(d.pos, d.nm, m);
    const Box B = d.boxes[d.beads[d.marker_bead[m]].box];
    const int bx = stencil_base<NW>(p.x) + a, by = stencil_base<NW>(p.y) + bb, bz = stencil_base<NW>(p.z) + c;
    const float w = phi<NW>((float)((double)bx - p.x)) * phi<NW>((float)((double)by - p.y)) *
                    phi<NW>((float)((double)bz - p.z));
    const int64_t node = B.node0 + ((int64_t)pmod(bz, B.nz) * B.ny + pmod(by, B.ny)) * B.nx + pmod(bx, B.nx);
    ux = w * d.u[node];
    uy = w * d.u[d.pstride + node];
    uz = w * d.u[2 * d.pstride + node];
  }
#pragma unroll
  for (int s = L / 2; s > 0; s >>= 1) {
    ux += __shfl_xor(ux, s, 64);
    uy += __shfl_xor(uy, s, 64);
    uz += __shfl_xor(uz, s, 64);
  }
  if (m < d.nm && lane == 0) {
    d.U[m] = ux;
    d.U[d.nm + m] = uy;
    d.U[2 * d.nm + m] = uz;
    d.pos[m] += (double)ux;
    d.pos[d.nm + m] += (double)uy;
    d.pos[2 * d.nm + m] += (double)uz;
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

void launch_bead_stats(const Dev& d, hipStream_t s) {
  if (d.width == 2) hipLaunchKernelGGL(k_bead_stats<2>, dim3(d.nswimmers), dim3(kStatsBlock), 0, s, d);
  else if (d.width == 3) hipLaunchKernelGGL(k_bead_stats<3>, dim3(d.nswimmers), dim3(kStatsBlock), 0, s, d);
  else hipLaunchKernelGGL(k_bead_stats<4>, dim3(d.nswimmers), dim3(kStatsBlock), 0, s, d);
}

void launch_vertex_forces(const Dev& d, hipStream_t s) {
  hipLaunchKernelGGL(k_vertex_forces, dim3((d.nm + 255) / 256), dim3(256), 0, s, d);
}

void launch_spread(const Dev& d, hipStream_t s) {
  if (d.width == 2) hipLaunchKernelGGL(k_spread<2>, dim3(d.spread_blocks), dim3(kSpreadBlock), 0, s, d);
  else if (d.width == 3) hipLaunchKernelGGL(k_spread<3>, dim3(d.spread_blocks), dim3(kSpreadBlock), 0, s, d);
  else hipLaunchKernelGGL(k_spread<4>, dim3(d.spread_blocks), dim3(kSpreadBlock), 0, s, d);
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
