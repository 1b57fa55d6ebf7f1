// Bead-level force terms shared by the immersed-boundary and lattice kernels
// (device code; included by the .hip files only).
//
// The force on a mesh node is split by what it depends on: the Skalak and
// bending parts and the area-vector sum of the node's triangles depend on the
// node's neighbourhood only; the volume-penalty pressure pv and the bead's
// driving + spring force depend on the bead statistics of the step
// (Sec. 2.2).  The volume force of a node is -pv times the sum over its
// triangles of (r_b - p) x (r_c - p) (corners counter-clockwise), which is
// the same for every reference point p on a closed mesh, since the edges
// r_c - r_b of the node's triangles close a loop; with p = r_a every term is
// the triangle's own area vector (r_1 - r_0) x (r_2 - r_0).
#pragma once

#include "common.h"

namespace lbmib {
namespace {

// Driving + spring force on bead `slot` of swimmer S at step n (Sec. 2.2):
// f1 = A sin(w n + phi0) x, f3 = B sin(w n + phi0 + alpha) x, f2 = -f1 - f3,
// springs f_o = -k (|R_o - R_2| - L) (R_o - R_2)/|R_o - R_2| on the outer
// beads with the opposite force on the middle one.
__device__ inline void bead_force(const Swimmer& S, int slot, int64_t n, const double* const* c, double* f) {
  const double t = (double)n;
  const double f1 = S.A * sin(S.omega * t + S.phi0);
  const double f3 = S.B * sin(S.omega * t + S.phi0 + S.alpha);
  f[0] = slot == 0 ? f1 : (slot == 2 ? f3 : -f1 - f3);
  f[1] = 0;
  f[2] = 0;
  const double* R2 = c[1];
  for (int sp = 0; sp < 2; ++sp) {
    const int outer = sp == 0 ? 0 : 2;
    if (slot != outer && slot != 1) continue;
    const double* Ro = c[outer];
    const double dx = Ro[0] - R2[0], dy = Ro[1] - R2[1], dz = Ro[2] - R2[2];
    const double len = sqrt(dx * dx + dy * dy + dz * dz);
    const double s = (slot == outer ? -1.0 : 1.0) * S.k[sp] * (len - S.L0[sp]) / len;
    f[0] += s * dx;
    f[1] += s * dy;
    f[2] += s * dz;
  }
}

// The bead terms of bead b at step n from the step's bead statistics:
// volume pressure pv = kv (V - V0)/(6 V0) and the per-node share of the
// bead's driving + spring force.

// Swimmer s owns beads 3s, 3s + 1, 3s + 2 (lbm_swimmer_add numbers them so),
// which lets every load below issue at once.
__device__ inline BeadTerms bead_terms(const Dev& d, int b, int64_t n) {
  const int sw = b / 3, slot = b - 3 * sw;
  const Bead& q = d.beads[b];
  const BeadState* st = d.bstate + 3 * sw;
  const Swimmer& S = d.swimmers[sw];
  const double* c[3] = {st[0].c, st[1].c, st[2].c};
  double f[3];
  bead_force(S, slot, n, c, f);
  const float inv = 1.0f / (float)q.nv;
  BeadTerms t;
  t.pv = (float)(q.kv * (d.bstate[b].V - q.V0) / (6.0 * q.V0));
  t.share[0] = (float)f[0] * inv;
  t.share[1] = (float)f[1] * inv;
  t.share[2] = (float)f[2] * inv;
  return t;
}

// One component of a node's total force from its split parts and its bead's
// terms; the explicit fmaf fixes the rounding wherever it is formed.
__device__ inline float total_force(float fmem, float gvol, float pv, float share) {
  return fmaf(-pv, gvol, fmem) + share;
}

// Total force on marker m.
__device__ inline void marker_total(const Dev& d, int m, const BeadTerms& t, float* f) {
  const int nm = d.nm;
#pragma unroll
  for (int a = 0; a < 3; ++a) f[a] = total_force(d.fmem[a * nm + m], d.gvol[a * nm + m], t.pv, t.share[a]);
}

}  // namespace
}  // namespace lbmib
