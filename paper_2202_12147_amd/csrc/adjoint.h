// Internal definitions of the discrete adjoint (reverse sweep of the fused
// LBM-IBM step).
//
// Forward step n (Sec. 2): F_n = S(r_n) f(r_n, n), streaming, moments
// u_n = (j + F_n/2)/rho, Guo-forced BGK collision, r_{n+1} = r_n + I(r_n) u_n.
// The reverse step n maps the adjoints of (f*_n, r_{n+1}) to those of
// (f*_{n-1}, r_n) and adds step n's share of dJ/dtheta; it needs (rho, u)_n
// at every node (recorded by the segment recompute), r_n, the marker forces
// of step n and the bead statistics of step n.
#pragma once

#include "common.h"

namespace lbmib {

struct Adj {
  const float* Lsrc;    // adjoint populations of step n+1 (population block layout)
  float* Ldst;          // adjoint populations of step n
  const float4* mom;    // (rho, u_x, u_y, u_z) of step n per node
  float* lu;            // lambda_u [3][pstride] (spread of lambda_r(n+1)); tiles stamped n
  float* lF;            // lambda_F [3][pstride], written in tiles stamped n
  double* lr;           // lambda_r [3][nm]: holds lambda_r(n+1), receives lambda_r(n)
  float* lr32;          // FP32 copy of lambda_r, the source of the lambda_u spread
  double* lfm;          // adjoint of the marker forces [3][nm]
  double* ltmp;         // [3][nm] lambda_r(n+1) plus the delta-gradient terms
  double* bsum;         // [nbeads][4]: sum of lfm over the bead's nodes, d V[lfm]
  double* grad;         // [4]: dJ/dA, dJ/dB, dJ/dalpha, dJ/dk
  int swimmer;          // objective and parameters: this swimmer
};

// lambda_r(T) = x^/(3 N_v) on the swimmer's nodes, zero elsewhere; grad = 0.
void launch_adj_init(const Dev& d, const Adj& a, hipStream_t s);
// Collision VJP and adjoint (push) streaming, in the launch modes of the
// forward stream-collide (kLaunchAll: every node; kLaunchBulk: blocks not
// marked near for step n; kLaunchActive: the near list), blocks of 256 nodes.
void launch_adj_collide(const Dev& d, const Adj& a, int mode, int nblocks, hipStream_t s);
// Transposed spreading and interpolation at the markers.
void launch_adj_gather(const Dev& d, const Adj& a, hipStream_t s);
// Per-bead sums of the force adjoint and the volume tangent.
void launch_adj_bead(const Dev& d, const Adj& a, hipStream_t s);
// Force-Jacobian product and the parameter-gradient update.
void launch_adj_tangent(const Dev& d, const Adj& a, hipStream_t s);
// *step = value (stream ordered).
void launch_set_step(int64_t* step, int64_t value, hipStream_t s);

}  // namespace lbmib
