// Kernels of the discrete adjoint of one fused LBM-IBM step (reverse order).
//
//   k_adj_collide   every node: pulls the step-(n+1) population adjoints from
//                   the downstream neighbours (the transpose of pull
//                   streaming), forms the vector-Jacobian product of the
//                   BGK collision with Guo or Shan-Chen forcing (Eqs. lbe,
//                   lbm:equilibrium, sc) with respect to the pre-collision
//                   populations and the force density, and stores both.
//   k_adj_gather    a lane group per marker: transposed spreading
//                   (lambda_f = sum_x lambda_F Delta) and the position
//                   derivatives of the spreading and interpolation weights
//                   (Eqs. spreading, interpolation).
//   k_adj_bead      one workgroup per bead: sums of lambda_f over its nodes and
//                   the directional derivative of its volume.
//   k_adj_tangent   32 lanes per node: the Jacobian of the Skalak, bending,
//                   volume and spring forces (Sec. 2.2) applied to lambda_f in
//                   dual-number FP64 arithmetic, giving lambda_r(n); lane 0 of
//                   the first workgroup folds step n into dJ/d(A, B, alpha, k).
//
// Every force of the model except the driving term is minus the gradient of
// an energy, so its Jacobian is symmetric and the transposed product needed
// by the reverse sweep equals the forward directional derivative.
#include "adjoint.h"

#include <hip/hip_runtime.h>

namespace lbmib {

namespace {

constexpr double kW0 = 1.0 / 3.0, kW1 = 1.0 / 18.0, kW2 = 1.0 / 36.0;
constexpr int kBlock = 256;

__device__ inline int pmod(int a, int b) {
  int r = a % b;
  return r < 0 ? r + b : r;
}

__device__ inline double3 ld3(const double* p, int nm, int m) { return make_double3(p[m], p[nm + m], p[2 * nm + m]); }

// ---- adjoint collision and streaming --------------------------------------------
//
// With Lambda_i the adjoint of the post-collision population f*_i at node y,
// omega = 1/tau, s = 1 - omega/2 and the weighted moments
//   P0 = sum w_i Lambda_i,  P1 = sum w_i Lambda_i c_i,  P2 = sum w_i Lambda_i c_i c_i,
// the collision f*_i = (1 - omega) f_i + omega feq_i(rho, u)
//                    + s w_i [3 (c_i - u) + 9 (c_i.u) c_i].F,  u = (j + F/2)/rho
// has the adjoints
//   a   = omega [P0 + 3 u.P1 + 4.5 u.P2 u - 1.5 u.u P0]                (via rho)
//   b   = omega rho [3 P1 + 9 P2 u - 3 u P0] + s [9 P2 F - 3 F P0] + lambda_u
//   lambda_f,i = (1 - omega) Lambda_i + a + b.(c_i - u)/rho
//   lambda_F   = s [3 P1 - 3 u P0 + 9 P2 u] + b/(2 rho)
// where lambda_u is the interpolation adjoint spread onto the grid.  The
// streamed value f_i(x) = f*_{n-1,i}(x - c_i) makes the step-(n-1) adjoint
// at y equal lambda_f,i(y + c_i): each node pulls Lambda_i from y + c_i and
// stores its own lambda_f (reads shifted by one element, writes coalesced);
// same block layout as the populations.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_adj_collide(Dev d, Adj a, int nblocks) {
  const Box B = d.boxes[0];
  const int64_t n = *d.step + d.sub;
  const int64_t pn = n - 1;  // the near marks of step n were made at step n - 1
  const int pp = (int)(pn & 1), pf = near_slot(pn);
  int blk = blockIdx.x;
  if constexpr (MODE == kLaunchActive) {
    if ((int)blockIdx.x >= min(d.near_count[pp], d.max_near)) return;
    blk = d.near_list[pp * d.max_near + blockIdx.x];
  } else if constexpr (MODE == kLaunchBulk) {
    if (blk >= nblocks || d.near[pf * d.nsc + blk] == (int)pn) return;
  }
  const int id = blk * kBlock + threadIdx.x;
  if (id >= B.n) return;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int x = id % nx, yz = id / nx, y = yz % ny, z = yz / ny;
  const int sz = nx * ny;
  const int xm = (x == 0) ? nx - 1 : -1, xp = (x == nx - 1) ? -(nx - 1) : 1;
  const int ym = (y == 0) ? (ny - 1) * nx : -nx, yp = (y == ny - 1) ? -(ny - 1) * nx : nx;
  const int zm = (z == 0) ? (nz - 1) * sz : -sz, zp = (z == nz - 1) ? -(nz - 1) * sz : sz;
  // offset of y + c_i for the velocity set of the population planes
  const int off[kQ] = {0,       xp,      xm,      yp,      ym,      zp,      zm,
                       xp + yp, xm + ym, xp + ym, xm + yp, xp + zp, xm + zm, xp + zm, xm + zp,
                       yp + zp, ym + zm, yp + zm, ym + zp};
  const int64_t ps = d.pstride, base = B.node0 + id;
  float L[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) L[q] = __builtin_nontemporal_load(a.Lsrc + pop_index(q, base + off[q]));

  const float4 mu = a.mom[base];
  const float rho = mu.x, ux = mu.y, uy = mu.z, uz = mu.w;
  float Fx = B.gx, Fy = B.gy, Fz = B.gz, lux = 0.0f, luy = 0.0f, luz = 0.0f;
  const int tile = B.tile0 + (x / kTile) + B.tx * ((y / kTile) + B.ty * (z / kTile));
  // bulk blocks are never forced: the nodes of an active tile outside the
  // near blocks carry F = 0 and lambda_u = 0, and no stencil reads their
  // lambda_F (the side stream is rewriting lambda_u meanwhile)
  const bool forced = MODE != kLaunchBulk && d.stamp[tile] == (int)n;
  if (forced) {
    Fx += d.F[base];
    Fy += d.F[ps + base];
    Fz += d.F[2 * ps + base];
    lux = a.lu[base];
    luy = a.lu[ps + base];
    luz = a.lu[2 * ps + base];
  }

  // weighted moments of Lambda over the opposite pairs (+c, -c)
  const float w1 = (float)kW1, w2 = (float)kW2;
  float P0 = (float)kW0 * L[0];
  float Px = 0, Py = 0, Pz = 0, Pxx = 0, Pyy = 0, Pzz = 0, Pxy = 0, Pxz = 0, Pyz = 0;
  {
    const float s12 = L[1] + L[2], s34 = L[3] + L[4], s56 = L[5] + L[6];
    P0 += w1 * (s12 + s34 + s56);
    Px += w1 * (L[1] - L[2]);
    Py += w1 * (L[3] - L[4]);
    Pz += w1 * (L[5] - L[6]);
    Pxx += w1 * s12;
    Pyy += w1 * s34;
    Pzz += w1 * s56;
  }
  {
    const float s78 = L[7] + L[8], d78 = L[7] - L[8];      // ( 1,  1,  0)
    const float s910 = L[9] + L[10], d910 = L[9] - L[10];  // ( 1, -1,  0)
    const float sab = L[11] + L[12], dab = L[11] - L[12];  // ( 1,  0,  1)
    const float scd = L[13] + L[14], dcd = L[13] - L[14];  // ( 1,  0, -1)
    const float sef = L[15] + L[16], def = L[15] - L[16];  // ( 0,  1,  1)
    const float sgh = L[17] + L[18], dgh = L[17] - L[18];  // ( 0,  1, -1)
    P0 += w2 * (s78 + s910 + sab + scd + sef + sgh);
    Px += w2 * (d78 + d910 + dab + dcd);
    Py += w2 * (d78 - d910 + def + dgh);
    Pz += w2 * (dab - dcd + def - dgh);
    Pxx += w2 * (s78 + s910 + sab + scd);
    Pyy += w2 * (s78 + s910 + sef + sgh);
    Pzz += w2 * (sab + scd + sef + sgh);
    Pxy += w2 * (s78 - s910);
    Pxz += w2 * (sab - scd);
    Pyz += w2 * (sef - sgh);
  }
  const float om = B.omega, sh = 1.0f - 0.5f * om;
  const float ir = 1.0f / rho;
  // lambda_f,i = (1 - omega) Lambda_i + a0 + bt.c_i
  float a0, btx, bty, btz;
  if (B.forcing == kShanChen) {
    // Shan-Chen: the equilibrium at v = (j + tau F)/rho = u + (tau - 1/2) F/rho,
    // no source term; u (interpolated, adjoint lambda_u) stays (j + F/2)/rho:
    //   av  = omega [P0 + 3 v.P1 + 4.5 v.P2 v - 1.5 v.v P0]
    //   bv  = omega rho [3 P1 + 9 P2 v - 3 v P0]
    //   lambda_f,i = (1 - omega) Lambda_i + av + (bv.(c_i - v) + lambda_u.(c_i - u))/rho
    //   lambda_F   = (tau bv + lambda_u / 2)/rho
    const float kt = (B.tau - 0.5f) * ir;
    const float vx = ux + kt * Fx, vy = uy + kt * Fy, vz = uz + kt * Fz;
    const float P2vx = Pxx * vx + Pxy * vy + Pxz * vz;
    const float P2vy = Pxy * vx + Pyy * vy + Pyz * vz;
    const float P2vz = Pxz * vx + Pyz * vy + Pzz * vz;
    const float vv = vx * vx + vy * vy + vz * vz;
    const float av = om * (P0 + 3.0f * (vx * Px + vy * Py + vz * Pz) + 4.5f * (vx * P2vx + vy * P2vy + vz * P2vz) -
                           1.5f * vv * P0);
    const float orho = om * rho;
    const float bvx = orho * (3.0f * Px + 9.0f * P2vx - 3.0f * vx * P0);
    const float bvy = orho * (3.0f * Py + 9.0f * P2vy - 3.0f * vy * P0);
    const float bvz = orho * (3.0f * Pz + 9.0f * P2vz - 3.0f * vz * P0);
    if (forced) {
      a.lF[base] = (B.tau * bvx + 0.5f * lux) * ir;
      a.lF[ps + base] = (B.tau * bvy + 0.5f * luy) * ir;
      a.lF[2 * ps + base] = (B.tau * bvz + 0.5f * luz) * ir;
    }
    btx = (bvx + lux) * ir;
    bty = (bvy + luy) * ir;
    btz = (bvz + luz) * ir;
    a0 = av - ((bvx * vx + bvy * vy + bvz * vz) + (lux * ux + luy * uy + luz * uz)) * ir;
  } else {
    const float P2ux = Pxx * ux + Pxy * uy + Pxz * uz;
    const float P2uy = Pxy * ux + Pyy * uy + Pyz * uz;
    const float P2uz = Pxz * ux + Pyz * uy + Pzz * uz;
    const float P2Fx = Pxx * Fx + Pxy * Fy + Pxz * Fz;
    const float P2Fy = Pxy * Fx + Pyy * Fy + Pyz * Fz;
    const float P2Fz = Pxz * Fx + Pyz * Fy + Pzz * Fz;
    const float uu = ux * ux + uy * uy + uz * uz;
    const float aa = om * (P0 + 3.0f * (ux * Px + uy * Py + uz * Pz) + 4.5f * (ux * P2ux + uy * P2uy + uz * P2uz) -
                           1.5f * uu * P0);
    const float orho = om * rho;
    const float bx = orho * (3.0f * Px + 9.0f * P2ux - 3.0f * ux * P0) + sh * (9.0f * P2Fx - 3.0f * Fx * P0) + lux;
    const float by = orho * (3.0f * Py + 9.0f * P2uy - 3.0f * uy * P0) + sh * (9.0f * P2Fy - 3.0f * Fy * P0) + luy;
    const float bz = orho * (3.0f * Pz + 9.0f * P2uz - 3.0f * uz * P0) + sh * (9.0f * P2Fz - 3.0f * Fz * P0) + luz;
    if (forced) {
      const float h = 0.5f * ir;
      a.lF[base] = sh * (3.0f * Px - 3.0f * ux * P0 + 9.0f * P2ux) + h * bx;
      a.lF[ps + base] = sh * (3.0f * Py - 3.0f * uy * P0 + 9.0f * P2uy) + h * by;
      a.lF[2 * ps + base] = sh * (3.0f * Pz - 3.0f * uz * P0 + 9.0f * P2uz) + h * bz;
    }
    btx = bx * ir;
    bty = by * ir;
    btz = bz * ir;
    a0 = aa - (btx * ux + bty * uy + btz * uz);
  }
  const float k1 = 1.0f - om;
  const float cq[kQ] = {0.0f,       btx,        -btx,       bty,        -bty,       btz,        -btz,
                        btx + bty,  -btx - bty, btx - bty,  bty - btx,  btx + btz,  -btx - btz, btx - btz,
                        btz - btx,  bty + btz,  -bty - btz, bty - btz,  btz - bty};
  if (d.small_pops) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) stream_store(a.Ldst + pop_index(q, base), k1 * L[q] + a0 + cq[q]);
  } else {
#pragma unroll
    for (int q = 0; q < kQ; ++q) __builtin_nontemporal_store(k1 * L[q] + a0 + cq[q], a.Ldst + pop_index(q, base));
  }
}

// ---- transposed spreading and interpolation -----------------------------------------
// phi and d phi / d r in FP64 for the three kernels of Sec. 2.3.
template <int NW>
__device__ inline void phi_dphi(double r, double& p, double& dp) {
  const double ar = fabs(r), sg = r < 0 ? -1.0 : 1.0;
  p = 0.0;
  dp = 0.0;
  if constexpr (NW == 2) {
    if (ar < 1.0) {
      p = 1.0 - ar;
      dp = -sg;
    }
  } else if constexpr (NW == 3) {
    if (ar <= 0.5) {
      const double s = sqrt(1.0 - 3.0 * r * r);
      p = (1.0 + s) / 3.0;
      dp = -r / s;
    } else if (ar <= 1.5) {
      const double q = 1.0 - ar, s = sqrt(fmax(0.0, 1.0 - 3.0 * q * q));
      p = (5.0 - 3.0 * ar - s) / 6.0;
      dp = sg * (-3.0 - (s > 0.0 ? 3.0 * q / s : 0.0)) / 6.0;
    }
  } else {
    if (ar <= 1.0) {
      const double s = sqrt(1.0 + 4.0 * ar - 4.0 * ar * ar);
      p = (3.0 - 2.0 * ar + s) / 8.0;
      dp = sg * (-2.0 + (2.0 - 4.0 * ar) / s) / 8.0;
    } else if (ar <= 2.0) {
      const double s = sqrt(fmax(0.0, -7.0 + 12.0 * ar - 4.0 * ar * ar));
      p = (5.0 - 2.0 * ar - s) / 8.0;
      dp = sg * (-2.0 - (s > 0.0 ? (6.0 - 4.0 * ar) / s : 0.0)) / 8.0;
    }
  }
}

template <int NW>
__device__ inline int stencil_base(double r) {
  r = fmin(fmax(r, -1.0e9), 1.0e9);
  if constexpr (NW == 3) return (int)floor(r + 0.5) - 1;
  if constexpr (NW == 4) return (int)floor(r) - 1;
  return (int)floor(r);
}

// With t(x) = lambda_F(x).f_m + lambda_r(n+1)_m.u(x) and Delta(x - r) =
// phi(x1 - r1) phi(x2 - r2) phi(x3 - r3):
//   lambda_f,m  = sum_x lambda_F(x) Delta(x - r_m)
//   ltmp_m      = lambda_r(n+1)_m + sum_x t(x) d Delta(x - r_m)/d r_m.
template <int NW>
__global__ __launch_bounds__(kBlock) void k_adj_gather(Dev d, Adj a) {
  constexpr int L = NW == 2 ? 8 : (NW == 3 ? 32 : 64);
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int m = gid / L, lane = gid % L;
  double s[6] = {0, 0, 0, 0, 0, 0};
  if (m < d.nm && lane < NW * NW * NW) {
    const int ia = lane % NW, ib = (lane / NW) % NW, ic = lane / (NW * NW);
    const double3 p = ld3(d.pos, d.nm, m);
    const Box B = d.boxes[0];
    const int bx = stencil_base<NW>(p.x) + ia, by = stencil_base<NW>(p.y) + ib, bz = stencil_base<NW>(p.z) + ic;
    double px, dx, py, dy, pz, dz;
    phi_dphi<NW>((double)bx - p.x, px, dx);
    phi_dphi<NW>((double)by - p.y, py, dy);
    phi_dphi<NW>((double)bz - p.z, pz, dz);
    const double w = px * py * pz;
    const int64_t node = B.node0 + ((int64_t)pmod(bz, B.nz) * B.ny + pmod(by, B.ny)) * B.nx + pmod(bx, B.nx);
    const int64_t ps = d.pstride;
    const double lFx = a.lF[node], lFy = a.lF[ps + node], lFz = a.lF[2 * ps + node];
    const float4 mu = a.mom[node];
    const double t = lFx * (double)d.fm[m] + lFy * (double)d.fm[d.nm + m] + lFz * (double)d.fm[2 * d.nm + m] +
                     a.lr[m] * (double)mu.y + a.lr[d.nm + m] * (double)mu.z + a.lr[2 * d.nm + m] * (double)mu.w;
    s[0] = w * lFx;
    s[1] = w * lFy;
    s[2] = w * lFz;
    // d Delta(x - r)/d r_1 = -phi'(x1 - r1) phi(x2 - r2) phi(x3 - r3)
    s[3] = -t * dx * py * pz;
    s[4] = -t * px * dy * pz;
    s[5] = -t * px * py * dz;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k)
    for (int sh = L / 2; sh > 0; sh >>= 1) s[k] += __shfl_xor(s[k], sh, 64);
  if (m < d.nm && lane == 0) {
    const int nm = d.nm;
    a.lfm[m] = s[0];
    a.lfm[nm + m] = s[1];
    a.lfm[2 * nm + m] = s[2];
    a.ltmp[m] = a.lr[m] + s[3];
    a.ltmp[nm + m] = a.lr[nm + m] + s[4];
    a.ltmp[2 * nm + m] = a.lr[2 * nm + m] + s[5];
  }
}

// ---- per-bead sums -----------------------------------------------------------------------
__device__ inline double block_sum(double v, double* sh) {
  for (int s = 32; s > 0; s >>= 1) v += __shfl_xor(v, s, 64);
  const int w = threadIdx.x / 64, l = threadIdx.x % 64;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0;
  for (int i = 0; i < kBlock / 64; ++i) t += sh[i];
  return t;
}

// bsum[b] = (sum over the bead's nodes of lambda_f, dV[lambda_f]) with
// dV[v] = 1/6 sum_t v0.((x1-c) x (x2-c)) + v1.((x2-c) x (x0-c)) + v2.((x0-c) x (x1-c));
// the centre c can be any fixed point of a closed surface.
__global__ __launch_bounds__(kBlock) void k_adj_bead(Dev d, Adj a) {
  __shared__ double sh[kBlock / 64];
  const int b = blockIdx.x;
  const Bead Bd = d.beads[b];
  const int nm = d.nm;
  double v[4] = {0, 0, 0, 0};
  for (int i = threadIdx.x; i < Bd.nv; i += kBlock) {
    const int m = Bd.first + i;
    v[0] += a.lfm[m];
    v[1] += a.lfm[nm + m];
    v[2] += a.lfm[2 * nm + m];
  }
  const double* c = d.bstate[b].c;
  for (int t = threadIdx.x; t < Bd.ntri; t += kBlock) {
    const int tt = Bd.tri0 + t;
    const int i[3] = {d.tri[tt], d.tri[d.ntri + tt], d.tri[2 * d.ntri + tt]};
    double3 x[3], w[3];
    for (int k = 0; k < 3; ++k) {
      const double3 p = ld3(d.pos, nm, i[k]);
      x[k] = make_double3(p.x - c[0], p.y - c[1], p.z - c[2]);
      w[k] = ld3(a.lfm, nm, i[k]);
    }
    for (int k = 0; k < 3; ++k) {
      const double3 p = x[(k + 1) % 3], q = x[(k + 2) % 3];
      const double gx = p.y * q.z - p.z * q.y, gy = p.z * q.x - p.x * q.z, gz = p.x * q.y - p.y * q.x;
      v[3] += (w[k].x * gx + w[k].y * gy + w[k].z * gz) * (1.0 / 6.0);
    }
  }
  for (int k = 0; k < 4; ++k) {
    const double t = block_sum(v[k], sh);
    if (threadIdx.x == 0) a.bsum[4 * b + k] = t;
  }
}

// ---- force Jacobian ------------------------------------------------------------------------
// Dual numbers: value and directional derivative.
struct Dl {
  double v, d;
};
__device__ inline Dl operator+(Dl a, Dl b) { return {a.v + b.v, a.d + b.d}; }
__device__ inline Dl operator-(Dl a, Dl b) { return {a.v - b.v, a.d - b.d}; }
__device__ inline Dl operator-(Dl a) { return {-a.v, -a.d}; }
__device__ inline Dl operator*(Dl a, Dl b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ inline Dl operator*(double s, Dl a) { return {s * a.v, s * a.d}; }
__device__ inline Dl operator/(Dl a, Dl b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
__device__ inline Dl dsqrt(Dl a) {
  const double s = sqrt(a.v);
  return {s, 0.5 * a.d / s};
}

struct D3 {
  Dl x, y, z;
};
__device__ inline D3 operator+(const D3& a, const D3& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline D3 operator-(const D3& a, const D3& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline D3 operator*(Dl s, const D3& a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ inline Dl dot(const D3& a, const D3& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline D3 cross(const D3& a, const D3& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ inline D3 load_d3(const Dev& d, const Adj& a, int m) {
  const int nm = d.nm;
  return {{d.pos[m], a.lfm[m]}, {d.pos[nm + m], a.lfm[nm + m]}, {d.pos[2 * nm + m], a.lfm[2 * nm + m]}};
}

// Skalak force on corner `corner` of triangle t (the energy and the
// cancellation-free stress of the forward force kernel), differentiated.
__device__ inline double3 skalak_corner_tangent(const Dev& d, const Bead& Bd, int t, int corner, const D3* p) {
  const D3 e1 = p[1] - p[0], e2 = p[2] - p[0];
  const double G11 = d.G0[t], G12 = d.G0[d.ntri + t], G22 = d.G0[2 * d.ntri + t];
  const double det = G11 * G22 - G12 * G12, idet = 1.0 / det;
  const double Gi11 = G22 * idet, Gi12 = -G12 * idet, Gi22 = G11 * idet;
  const Dl D11 = dot(e1, e1) - Dl{G11, 0}, D12 = dot(e1, e2) - Dl{G12, 0}, D22 = dot(e2, e2) - Dl{G22, 0};
  const Dl I1 = Gi11 * D11 + (2.0 * Gi12) * D12 + Gi22 * D22;
  const Dl I2 = idet * (G11 * D22 + G22 * D11 - (2.0 * G12) * D12 + (D11 * D22 - D12 * D12));
  const double C = (double)Bd.C, k4 = 0.25 * (double)Bd.ks * 0.5 * sqrt(det);
  const Dl aa = k4 * (2.0 * I1 + (2.0 * C) * I2);
  const Dl bq = (k4 * idet) * ((2.0 * C) * I2 - Dl{2.0, 0});
  const Dl P11 = Gi11 * aa + bq * D22, P12 = Gi12 * aa - bq * D12, P22 = Gi22 * aa + bq * D11;
  Dl ca, cb;
  if (corner == 1) {
    ca = 2.0 * P11;
    cb = 2.0 * P12;
  } else if (corner == 2) {
    ca = 2.0 * P12;
    cb = 2.0 * P22;
  } else {
    ca = -2.0 * (P11 + P12);
    cb = -2.0 * (P12 + P22);
  }
  const D3 f = ca * e1 + cb * e2;
  return make_double3(-f.x.d, -f.y.d, -f.z.d);
}

// Kantor-Nelson force -kt sin(theta - theta0) d theta/d x_role of hinge h on
// its vertex `role` (x1, x2 shared edge; x3, x4 opposite), differentiated.
__device__ inline double3 bending_role_tangent(const Dev& d, const Bead& Bd, int h, int role, const D3* x) {
  const D3 e = x[1] - x[0], av = x[2] - x[0], bv = x[3] - x[1];
  const D3 nA = cross(e, av);
  const D3 nB0 = cross(e, bv);
  const D3 nB = {-nB0.x, -nB0.y, -nB0.z};
  const Dl nA2 = dot(nA, nA), nB2 = dot(nB, nB);
  const Dl E = dsqrt(dot(e, e));
  const D3 eh = (Dl{1.0, 0} / E) * e;
  const D3 c = cross(nA, nB);
  const Dl inorm = Dl{1.0, 0} / dsqrt(nA2 * nB2);
  const Dl sn = dot(c, eh) * inorm, cs = dot(nA, nB) * inorm;
  const double c0 = d.th0cs[h], s0 = d.th0cs[d.nh + h];
  const Dl dW = (double)Bd.kt * (c0 * sn - s0 * cs);
  Dl ca = {0, 0}, cb = {0, 0};
  if (role == 2) {
    ca = -E;
  } else if (role == 3) {
    cb = -E;
  } else if (role == 0) {
    ca = -dot(x[2] - x[1], eh);
    cb = dot(x[1] - x[3], eh);
  } else {
    ca = -dot(x[0] - x[2], eh);
    cb = dot(x[3] - x[0], eh);
  }
  const D3 g = (ca / nA2) * nA + (cb / nB2) * nB;
  const D3 f = dW * g;
  return make_double3(-f.x.d, -f.y.d, -f.z.d);
}

// 32 lanes per node (the force kernel's lane tables): lanes 0..7 the node's
// triangles (Skalak tangent; volume gradient G and its tangent), lanes 8..31
// its hinges.  Lane 0 adds the volume term
//   d f_vol = -(kv dV/V0) G - kv (V - V0)/V0 dG
// and the spring term through the bead centres, dR_b = bsum_b / N_v.
constexpr int kLanes = 32;
constexpr int kTriLanes = 8;
__global__ __launch_bounds__(kBlock) void k_adj_tangent(Dev d, Adj a) {
  const int gid = blockIdx.x * kBlock + threadIdx.x;
  const int m = gid / kLanes, lane = gid % kLanes;
  const int nm = d.nm;
  double s[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // force tangent, G, dG
  int b = 0;
  if (m < nm) {
    b = d.marker_bead[m];
    const int e = d.lane_elem[gid];
    const int4 v = d.lane_v[gid];
    if (e >= 0) {
      const Bead Bd = d.beads[b];
      if (lane < kTriLanes) {
        const int t = e / 3, corner = e % 3;
        const D3 p[3] = {load_d3(d, a, v.x), load_d3(d, a, v.y), load_d3(d, a, v.z)};
        const double3 f = skalak_corner_tangent(d, Bd, t, corner, p);
        s[0] = f.x;
        s[1] = f.y;
        s[2] = f.z;
        const double* c = d.bstate[b].c;
        const D3 cc = {{c[0], 0}, {c[1], 0}, {c[2], 0}};
        // the other two corners in counter-clockwise order, selected with
        // constant indices (a computed index would put p in scratch memory)
        D3 pb, pc;
        if (corner == 0) {
          pb = p[1] - cc;
          pc = p[2] - cc;
        } else if (corner == 1) {
          pb = p[2] - cc;
          pc = p[0] - cc;
        } else {
          pb = p[0] - cc;
          pc = p[1] - cc;
        }
        const D3 g = cross(pb, pc);
        s[3] = g.x.v * (1.0 / 6.0);
        s[4] = g.y.v * (1.0 / 6.0);
        s[5] = g.z.v * (1.0 / 6.0);
        s[6] = g.x.d * (1.0 / 6.0);
        s[7] = g.y.d * (1.0 / 6.0);
        s[8] = g.z.d * (1.0 / 6.0);
      } else {
        const D3 x[4] = {load_d3(d, a, v.x), load_d3(d, a, v.y), load_d3(d, a, v.z), load_d3(d, a, v.w)};
        const double3 f = bending_role_tangent(d, Bd, e / 4, e % 4, x);
        s[0] = f.x;
        s[1] = f.y;
        s[2] = f.z;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k)
    for (int sh = kLanes / 2; sh > 0; sh >>= 1) s[k] += __shfl_xor(s[k], sh, 64);
  if (m < nm && lane == 0) {
    const Bead Bd = d.beads[b];
    const double V = d.bstate[b].V, kv = (double)Bd.kv;
    const double pref = kv * (V - Bd.V0) / Bd.V0, dpref = kv * a.bsum[4 * b + 3] / Bd.V0;
    double t[3];
    for (int k = 0; k < 3; ++k) t[k] = s[k] - dpref * s[3 + k] - pref * s[6 + k];
    if (Bd.swimmer >= 0) {
      const Swimmer S = d.swimmers[Bd.swimmer];
      const double* R1 = d.bstate[S.bead[1]].c;
      const Bead B1 = d.beads[S.bead[1]];
      for (int sp = 0; sp < 2; ++sp) {
        const int outer = sp == 0 ? 0 : 2;
        if (Bd.slot != outer && Bd.slot != 1) continue;
        const Bead Bo = d.beads[S.bead[outer]];
        const double* Ro = d.bstate[S.bead[outer]].c;
        double dd[3], dD[3];
        for (int k = 0; k < 3; ++k) {
          dd[k] = Ro[k] - R1[k];
          dD[k] = a.bsum[4 * S.bead[outer] + k] / Bo.nv - a.bsum[4 * S.bead[1] + k] / B1.nv;
        }
        const double len = sqrt(dd[0] * dd[0] + dd[1] * dd[1] + dd[2] * dd[2]);
        const double dlen = (dd[0] * dD[0] + dd[1] * dD[1] + dd[2] * dD[2]) / len;
        const double sign = Bd.slot == outer ? 1.0 : -1.0;
        for (int k = 0; k < 3; ++k) {
          const double dfs = -S.k[sp] * (dlen * dd[k] / len + (len - S.L0[sp]) * (dD[k] / len - dd[k] * dlen / (len * len)));
          t[k] += sign * dfs / Bd.nv;
        }
      }
    }
    for (int k = 0; k < 3; ++k) {
      const double l = a.ltmp[k * nm + m] + t[k];
      a.lr[k * nm + m] = l;
      a.lr32[k * nm + m] = (float)l;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    // dJ/dtheta += sum over the swimmer's beads of Phi_b . d f_b/d theta, with
    // Phi_b = bsum_b / N_v the adjoint of bead b's total (driving + spring) force
    const Swimmer S = d.swimmers[a.swimmer];
    double Phi[3][3];
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) Phi[j][k] = a.bsum[4 * S.bead[j] + k] / d.beads[S.bead[j]].nv;
    const double tn = (double)(*d.step + d.sub);
    const double ph1 = S.omega * tn + S.phi0, ph3 = ph1 + S.alpha;
    a.grad[0] += sin(ph1) * (Phi[0][0] - Phi[1][0]);
    a.grad[1] += sin(ph3) * (Phi[2][0] - Phi[1][0]);
    a.grad[2] += S.B * cos(ph3) * (Phi[2][0] - Phi[1][0]);
    const double* R1 = d.bstate[S.bead[1]].c;
    double gk = 0;
    for (int sp = 0; sp < 2; ++sp) {
      const int outer = sp == 0 ? 0 : 2;
      const double* Ro = d.bstate[S.bead[outer]].c;
      const double dx = Ro[0] - R1[0], dy = Ro[1] - R1[1], dz = Ro[2] - R1[2];
      const double len = sqrt(dx * dx + dy * dy + dz * dz);
      const double c = -(len - S.L0[sp]) / len;  // d f_spring / d k = c (R_o - R_2)
      gk += c * (dx * (Phi[outer][0] - Phi[1][0]) + dy * (Phi[outer][1] - Phi[1][1]) + dz * (Phi[outer][2] - Phi[1][2]));
    }
    a.grad[3] += gk;
  }
}

__global__ void k_adj_init(Dev d, Adj a) {
  const int m = blockIdx.x * kBlock + threadIdx.x;
  if (m == 0)
    for (int k = 0; k < 4; ++k) a.grad[k] = 0.0;
  if (m >= d.nm) return;
  const int b = d.marker_bead[m];
  const Bead Bd = d.beads[b];
  const double lx = Bd.swimmer == a.swimmer ? 1.0 / (3.0 * Bd.nv) : 0.0;
  a.lr[m] = lx;
  a.lr[d.nm + m] = 0.0;
  a.lr[2 * d.nm + m] = 0.0;
  a.lr32[m] = (float)lx;
  a.lr32[d.nm + m] = 0.0f;
  a.lr32[2 * d.nm + m] = 0.0f;
}

__global__ void k_set_step(int64_t* step, int64_t value) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step = value;
}

}  // namespace

void launch_adj_init(const Dev& d, const Adj& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_init, dim3((d.nm + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d, a);
}

void launch_adj_collide(const Dev& d, const Adj& a, int mode, int nblocks, hipStream_t s) {
  if (mode == kLaunchActive)
    hipLaunchKernelGGL(k_adj_collide<kLaunchActive>, dim3(d.max_near), dim3(kBlock), 0, s, d, a, nblocks);
  else if (mode == kLaunchBulk)
    hipLaunchKernelGGL(k_adj_collide<kLaunchBulk>, dim3(nblocks), dim3(kBlock), 0, s, d, a, nblocks);
  else
    hipLaunchKernelGGL(k_adj_collide<kLaunchAll>, dim3(nblocks), dim3(kBlock), 0, s, d, a, nblocks);
}

void launch_adj_gather(const Dev& d, const Adj& a, hipStream_t s) {
  const int L = d.width == 2 ? 8 : (d.width == 3 ? 32 : 64);
  const int blocks = (int)(((int64_t)d.nm * L + kBlock - 1) / kBlock);
  if (d.width == 2) hipLaunchKernelGGL(k_adj_gather<2>, dim3(blocks), dim3(kBlock), 0, s, d, a);
  else if (d.width == 3) hipLaunchKernelGGL(k_adj_gather<3>, dim3(blocks), dim3(kBlock), 0, s, d, a);
  else hipLaunchKernelGGL(k_adj_gather<4>, dim3(blocks), dim3(kBlock), 0, s, d, a);
}

void launch_adj_bead(const Dev& d, const Adj& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_bead, dim3(d.nbeads), dim3(kBlock), 0, s, d, a);
}

void launch_adj_tangent(const Dev& d, const Adj& a, hipStream_t s) {
  const int blocks = (int)(((int64_t)d.nm * kLanes + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_adj_tangent, dim3(blocks), dim3(kBlock), 0, s, d, a);
}

void launch_set_step(int64_t* step, int64_t value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_step, dim3(1), dim3(64), 0, s, step, value);
}

}  // namespace lbmib
