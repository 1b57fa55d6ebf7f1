// Lattice kernels: fused pull stream-collide, macroscopic output, and the
// FP64 conservation reductions.
//
// Fluid model (paper Sec. 2.1): D3Q19 BGK, Eq. (lbe) with the second-order
// equilibrium of Eq. (lbm:equilibrium); moments rho = sum f, rho u_eq =
// sum f c + tau F for the Shan-Chen force scheme (Eq. sc), physical velocity
// rho u = sum f c + F/2.  The Guo scheme uses u in the equilibrium and adds
// (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i.u) c_i].F.
//
// Storage holds g_i = f_i - w_i (deviation from the rest state), so the
// O(1e-5) flow signal is not swamped by the O(1/3) weights in FP32; FP16
// storage holds g_i * S rounded to nearest even; the unshifted reference
// storage holds f_i.  Arithmetic is FP32 on g in all three.
//
// Streaming is "pull": node x gathers g*_i(x - c_i) from the source parity and
// writes its 19 post-collision values to the same node of the other parity,
// so every read and write of a wavefront covers consecutive x (coalesced);
// only the c_x = +-1 loads are shifted by one element.
#include <hip/hip_fp16.h>

#include "common.h"
#include "bead_terms.h"
#include "near_marks.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <mutex>

namespace lbmib {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Fourth word of a raw buffer resource on this architecture (32-bit data
// format; stride 0, so the range check is against the byte count)
constexpr int kBufferWord3 = 0x00020000;

constexpr float kW0 = 1.0f / 3.0f;
constexpr float kW1 = 1.0f / 18.0f;
constexpr float kW2 = 1.0f / 36.0f;

template <int ST>
struct PopIO;

__device__ constexpr float weight(int q) { return q == 0 ? kW0 : (q < 7 ? kW1 : kW2); }

// Load / store of population q as the deviation g = f - w_q.
template <>
struct PopIO<kFp32> {
  using T = float;
  using Raw = unsigned;
  static constexpr int kNtAux = 2;  // non-temporal buffer loads (the nt bit)
  __device__ static inline float decode(Raw r, int, float) { return __uint_as_float(r); }
  __device__ static inline float ld(const float* p, int, float) { return __builtin_nontemporal_load(p); }
  __device__ static inline float ld_cached(const float* p, int, float) { return *p; }
  __device__ static inline void st(float* p, int, float v, float) { __builtin_nontemporal_store(v, p); }
  __device__ static inline void st_wt(float* p, int, float v, float) { stream_store(p, v); }
};

template <>
struct PopIO<kFp16> {
  using T = __half;
  using Raw = unsigned short;
  static constexpr int kNtAux = 0;  // half loads stay plain (measured faster)
  __device__ static inline float decode(Raw r, int, float inv) { return __half2float(__ushort_as_half(r)) * inv; }
  __device__ static inline float ld(const __half* p, int, float inv) { return __half2float(*p) * inv; }
  __device__ static inline float ld_cached(const __half* p, int q, float inv) { return ld(p, q, inv); }
  __device__ static inline void st(__half* p, int, float v, float scale) { *p = __float2half_rn(v * scale); }
  __device__ static inline void st_wt(__half* p, int, float v, float scale) {
    stream_store(reinterpret_cast<unsigned short*>(p), __half_as_ushort(__float2half_rn(v * scale)));
  }
};

// Unshifted storage of f itself (rounded at the scale of w_q ~ 1/3): the
// reference that shows what the shifted forms gain.
template <>
struct PopIO<kFp32Plain> {
  using T = float;
  using Raw = unsigned;
  static constexpr int kNtAux = 2;
  __device__ static inline float decode(Raw r, int q, float) { return __uint_as_float(r) - weight(q); }
  __device__ static inline float ld(const float* p, int q, float) {
    return __builtin_nontemporal_load(p) - weight(q);
  }
  __device__ static inline float ld_cached(const float* p, int q, float) { return *p - weight(q); }
  __device__ static inline void st(float* p, int q, float v, float) { __builtin_nontemporal_store(v + weight(q), p); }
  __device__ static inline void st_wt(float* p, int q, float v, float) { stream_store(p, v + weight(q)); }
};

// In-place FP32 deviations: the element type and decoding of kFp32; its loads
// and stores are the buffer forms of sc_node_inplace.
template <>
struct PopIO<kFp32InPlace> : PopIO<kFp32> {};

// Offsets (in nodes, periodic wrap folded in) of the six face neighbours.
struct Nbr {
  int xm, xp, ym, yp, zm, zp;
};

__device__ inline Nbr neighbours(int x, int y, int z, int nx, int ny, int nz) {
  const int sz = nx * ny;
  Nbr o;
  o.xm = (x == 0) ? nx - 1 : -1;
  o.xp = (x == nx - 1) ? -(nx - 1) : 1;
  o.ym = (y == 0) ? (ny - 1) * nx : -nx;
  o.yp = (y == ny - 1) ? -(ny - 1) * nx : nx;
  o.zm = (z == 0) ? (nz - 1) * sz : -sz;
  o.zp = (z == nz - 1) ? -(nz - 1) * sz : sz;
  return o;
}

// Pull the 19 deviations of node `base` from the source populations.
// NTLD: non-temporal loads (populations of the last-level-cache size) or
// plain ones (larger sets: 2 % faster on 10 GB of populations, 8 % slower at
// 128^3).
template <int ST, bool NTLD = true, bool OFF32 = false>
__device__ inline void pull(const typename PopIO<ST>::T* __restrict__ src, int64_t base, const Nbr& o, float inv,
                            float* g, uint32_t set_bytes = 0) {
  using IO = PopIO<ST>;
  const int off[kQ] = {0,
                       o.xm, o.xp, o.ym, o.yp, o.zm, o.zp,
                       o.xm + o.ym, o.xp + o.yp, o.xm + o.yp, o.xp + o.ym,
                       o.xm + o.zm, o.xp + o.zp, o.xm + o.zp, o.xp + o.zm,
                       o.ym + o.zm, o.yp + o.zp, o.ym + o.zp, o.yp + o.zm};
  const int lane = (int)(base % kPopBlock);
  if constexpr (OFF32) {
    // A population set below 4 GiB (set_bytes): buffer loads with a 32-bit
    // byte offset per node and the population's constant offset split into a
    // scalar part (multiples of 4 KiB) and the instruction's immediate field,
    // so each load takes one offset register and no 64-bit address
    // arithmetic.  Node m sits at element (m / 256) * 19 * 256 + m % 256 =
    // m + 4608 (m >> 8) of population 0; in bytes, with M = m * sizeof(T):
    // M + 4608 sizeof(T) (M >> (8 + log2 sizeof(T))).  Per population: one
    // add (the neighbour's M), one shift, one 24-bit multiply-add
    // (m >> 8 < 2^23).
    using T = typename PopIO<ST>::T;
    using Raw = typename IO::Raw;
    constexpr uint32_t kSz = (uint32_t)sizeof(T);
    constexpr int kSh = 8 + (kSz == 4 ? 2 : kSz == 2 ? 1 : 0);
    constexpr uint32_t kBlockStep = (kQ - 1) * kPopBlock * kSz;
    constexpr int kAux = NTLD ? IO::kNtAux : 0;
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(src), (short)0, (int)set_bytes, kBufferWord3);
    const uint32_t M = (uint32_t)base * kSz;
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const uint32_t Mn = M + (uint32_t)off[q] * kSz;  // the neighbour's node, in bytes (wraps to in-box)
      const uint32_t b = __umul24(Mn >> kSh, kBlockStep) + Mn;
      const uint32_t c = (uint32_t)q * kPopBlock * kSz;  // population q's block offset
      Raw r;
      if constexpr (kSz == 2)
        r = __builtin_amdgcn_raw_buffer_load_b16(rs, b + (c & 4095u), c & ~4095u, kAux);
      else
        r = __builtin_amdgcn_raw_buffer_load_b32(rs, b + (c & 4095u), c & ~4095u, kAux);
      g[q] = IO::decode(r, q, inv);
    }
    return;
  } else {
  // larger sets: addresses relative to the node's own population block,
  // 32-bit lane and population offsets, one 64-bit multiply-add per
  // population for the block
  const typename PopIO<ST>::T* bp = src + (base / kPopBlock) * (int64_t)(kQ * kPopBlock);
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int rel = lane + off[q];
    const int db = rel >> 8;  // floor(rel / kPopBlock): arithmetic shift, kPopBlock = 256
    const typename PopIO<ST>::T* a = bp + (int64_t)db * (kQ * kPopBlock) + (q * kPopBlock + (rel & (kPopBlock - 1)));
    if constexpr (NTLD)
      g[q] = IO::ld(a, q, inv);
    else
      g[q] = IO::ld_cached(a, q, inv);
  }
  }
}

struct Moments {
  float drho, rho, jx, jy, jz;
};

__device__ inline Moments moments(const float* g) {
  Moments m;
  float s = g[0];
#pragma unroll
  for (int q = 1; q < kQ; ++q) s += g[q];
  m.drho = s;
  m.rho = 1.0f + s;
  m.jx = (g[1] - g[2]) + (g[7] - g[8]) + (g[9] - g[10]) + (g[11] - g[12]) + (g[13] - g[14]);
  m.jy = (g[3] - g[4]) + (g[7] - g[8]) - (g[9] - g[10]) + (g[15] - g[16]) + (g[17] - g[18]);
  m.jz = (g[5] - g[6]) + (g[11] - g[12]) - (g[13] - g[14]) + (g[15] - g[16]) - (g[17] - g[18]);
  return m;
}

// BGK collision of one direction pair (+c, -c) with weight w.
//   e    = c . u_eq, the equilibrium velocity projection
//   cu,cf = c . u and c . F (Guo source), uf = u . F
// Every sum of two products is written as an explicit fmaf: left to the
// compiler, which product is fused can differ between template instances of
// the caller and change the last bit, and the launch variants of the step
// must agree bit for bit.
// 1/rho from the hardware reciprocal (within one ulp; rho stays near 1 in
// these flows), in place of the correctly rounded division sequence
__device__ inline float inv_density(float rho) { return __builtin_amdgcn_rcpf(rho); }

// SRC = false: the source term is zero (no force at the node, or Shan-Chen
// forcing) and is left out of the arithmetic; the populations are the same
// as with the zero term added (up to the sign of an exact zero).
template <bool SRC>
__device__ inline void collide_pair(float& gp, float& gm, float w, float om, float drho, float rho,
                                    float usq15, float e, float src_a, float cu, float cf,
                                    float uf) {
  const float sym = w * (drho + rho * fmaf(4.5f * e, e, -usq15));
  const float wr3 = w * rho * 3.0f;
  const float eqp = fmaf(wr3, e, sym), eqm = fmaf(-wr3, e, sym);
  if constexpr (SRC) {
    // Guo source: src_a (1 - om/2) w [3 (c - u).F + 9 (c.u)(c.F)]
    const float sw = src_a * w;
    const float s_sym = sw * fmaf(9.0f * cu, cf, -3.0f * uf);
    const float sw3 = sw * 3.0f;
    const float sp = fmaf(sw3, cf, s_sym), sm = fmaf(-sw3, cf, s_sym);
    gp = gp + om * (eqp - gp) + sp;
    gm = gm + om * (eqm - gm) + sm;
  } else {
    gp = gp + om * (eqp - gp);
    gm = gm + om * (eqm - gm);
  }
}

// BGK collision of all 19 populations (with the Guo source when SRC).
template <bool SRC>
__device__ inline void collide_all(float* g, const Moments& m, float om, float ex, float ey, float ez, float src_a,
                                   float ux, float uy, float uz, float Fx, float Fy, float Fz) {
  const float usq15 = 1.5f * fmaf(ez, ez, fmaf(ey, ey, ex * ex));
  const float uf = SRC ? fmaf(uz, Fz, fmaf(uy, Fy, ux * Fx)) : 0.0f;
  // rest population
  {
    const float eq0 = kW0 * (m.drho - m.rho * usq15);
    if constexpr (SRC)
      g[0] = g[0] + om * (eq0 - g[0]) + src_a * kW0 * (-3.0f * uf);
    else
      g[0] = g[0] + om * (eq0 - g[0]);
  }
  // faces
  collide_pair<SRC>(g[1], g[2], kW1, om, m.drho, m.rho, usq15, ex, src_a, ux, Fx, uf);
  collide_pair<SRC>(g[3], g[4], kW1, om, m.drho, m.rho, usq15, ey, src_a, uy, Fy, uf);
  collide_pair<SRC>(g[5], g[6], kW1, om, m.drho, m.rho, usq15, ez, src_a, uz, Fz, uf);
  // edges
  collide_pair<SRC>(g[7], g[8], kW2, om, m.drho, m.rho, usq15, ex + ey, src_a, ux + uy, Fx + Fy, uf);
  collide_pair<SRC>(g[9], g[10], kW2, om, m.drho, m.rho, usq15, ex - ey, src_a, ux - uy, Fx - Fy, uf);
  collide_pair<SRC>(g[11], g[12], kW2, om, m.drho, m.rho, usq15, ex + ez, src_a, ux + uz, Fx + Fz, uf);
  collide_pair<SRC>(g[13], g[14], kW2, om, m.drho, m.rho, usq15, ex - ez, src_a, ux - uz, Fx - Fz, uf);
  collide_pair<SRC>(g[15], g[16], kW2, om, m.drho, m.rho, usq15, ey + ez, src_a, uy + uz, Fy + Fz, uf);
  collide_pair<SRC>(g[17], g[18], kW2, om, m.drho, m.rho, usq15, ey - ez, src_a, uy - uz, Fy - Fz, uf);
}

// Workgroup -> logical block.  Workgroups are handed to the 8 XCDs round
// robin; with `remap` each XCD instead receives one contiguous range of
// logical blocks, so the cache lines shared by neighbouring blocks (the
// x-shifted pulls straddle block edges) stay in one XCD's L2.
__device__ inline int logical_block(int remap, int nblocks) {
  if (!remap) return blockIdx.x;
  const int per = (int)gridDim.x / 8;  // grid is a multiple of 8 when remapping
  return (blockIdx.x % 8) * per + blockIdx.x / 8;
}

// One node of the fused step: pull, moments, forcing, BGK collision, store.
// `forced`: read F and write u at this node (its tile is active this step).
// `avg`: add u to the node's time-average sums (a sampled step).
// MOM: also record (rho, u) of the node in d.mom.
template <int ST, bool MOM = false, bool NTLD = true, bool OFF32 = false>
__device__ inline void sc_node(const Dev& d, const Box& B, int x, int y, int z, int64_t base,
                               int64_t n, bool forced, bool avg) {
  using IO = PopIO<ST>;
  using T = typename IO::T;
  const Nbr o = neighbours(x, y, z, B.nx, B.ny, B.nz);
  const T* __restrict__ src = static_cast<const T*>(d.pop[n & 1]);
  T* __restrict__ dst = static_cast<T*>(d.pop[(n + 1) & 1]);
  const int64_t ps = d.pstride;
  // a sampled step loads the node's sums with the pulls, so that their
  // latency overlaps (the persistent bulk launch runs two waves per SIMD)
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (avg) {
    a0 = d.uavg[base];
    a1 = d.uavg[ps + base];
    a2 = d.uavg[2 * ps + base];
  }
  float g[kQ];
  pull<ST, NTLD, OFF32>(src, base, o, d.fp16_inv, g, (uint32_t)(kQ * d.pstride * (int64_t)sizeof(T)));
  const Moments m = moments(g);

  float Fx = B.gx, Fy = B.gy, Fz = B.gz;
  if (forced) {
    Fx += d.F[base];
    Fy += d.F[ps + base];
    Fz += d.F[2 * ps + base];
  }
  const float ir = inv_density(m.rho);
  const float ux = (m.jx + 0.5f * Fx) * ir;
  const float uy = (m.jy + 0.5f * Fy) * ir;
  const float uz = (m.jz + 0.5f * Fz) * ir;
  if (forced) {
    d.u[base] = ux;
    d.u[ps + base] = uy;
    d.u[2 * ps + base] = uz;
  }
  if constexpr (MOM) {
    const f32x4 rec = {m.rho, ux, uy, uz};
    __builtin_nontemporal_store(rec, reinterpret_cast<f32x4*>(d.mom) + base);
  }
  float ex = ux, ey = uy, ez = uz, src_a = 1.0f - 0.5f * B.omega;
  if (B.forcing == kShanChen) {
    ex = (m.jx + B.tau * Fx) * ir;
    ey = (m.jy + B.tau * Fy) * ir;
    ez = (m.jz + B.tau * Fz) * ir;
    src_a = 0.0f;
  }
  // no force at the node (most nodes) or Shan-Chen forcing: no source term
  if (src_a != 0.0f && (Fx != 0.0f || Fy != 0.0f || Fz != 0.0f))
    collide_all<true>(g, m, B.omega, ex, ey, ez, src_a, ux, uy, uz, Fx, Fy, Fz);
  else
    collide_all<false>(g, m, B.omega, ex, ey, ez, src_a, ux, uy, uz, Fx, Fy, Fz);
  if constexpr (OFF32) {
    // 32-bit byte offsets from the set's start (see pull)
    // one offset register for all 19 stores: the population's q * 256
    // elements are a constant the store instruction carries
    constexpr uint32_t kSz = (uint32_t)sizeof(T);
    constexpr int kSh = 8 + (kSz == 4 ? 2 : kSz == 2 ? 1 : 0);
    const uint32_t M = (uint32_t)base * kSz;
    T* const bq = reinterpret_cast<T*>(reinterpret_cast<char*>(dst) + (__umul24(M >> kSh, (kQ - 1) * kPopBlock * kSz) + M));
    if (d.small_pops) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) IO::st_wt(bq + q * kPopBlock, q, g[q], d.fp16_scale);
    } else {
#pragma unroll
      for (int q = 0; q < kQ; ++q) IO::st(bq + q * kPopBlock, q, g[q], d.fp16_scale);
    }
  } else {
    T* const bq = dst + (base / kPopBlock) * (int64_t)(kQ * kPopBlock) + (int)(base % kPopBlock);
    if (d.small_pops) {
#pragma unroll
      for (int q = 0; q < kQ; ++q) IO::st_wt(bq + q * kPopBlock, q, g[q], d.fp16_scale);
    } else {
#pragma unroll
      for (int q = 0; q < kQ; ++q) IO::st(bq + q * kPopBlock, q, g[q], d.fp16_scale);
    }
  }
  if (avg) {
    double* __restrict__ acc = d.uavg;
    acc[base] = a0 + (double)ux;
    acc[ps + base] = a1 + (double)uy;
    acc[2 * ps + base] = a2 + (double)uz;
  }
}

// ---- in-place storage (one population set) ------------------------------------
// The AA access pattern (Bailey, Myre, Walsh, Lilja and Lerner, "Accelerating
// lattice Boltzmann fluid flow simulations using graphics processors", ICPP
// 2009): one set of deviations, updated in place.  With the state after an
// odd number of steps (and the initial state) holding f*_q(x) in slot q of
// node x + c_q, an even step n reads the incoming f_q(x) from its own slot q
// and writes f*_q(x) back to slot opposite(q) of the same node; after it,
// slot opposite(q) of node x holds f*_q(x), so an odd step reads f_q(x) =
// f*_q(x - c_q) from slot opposite(q) of node x - c_q and writes f*_q(x) to
// slot q of node x + c_q, which restores the first arrangement.  Every node
// reads and writes the same 19 slots and no other node touches them in that
// step, so the launches of one step (bulk and near blocks) may run
// concurrently, as with two sets.  The moments, forcing and collision are
// those of sc_node, so the results equal the two-set storage bit for bit.
// Loads and stores go through a buffer resource bounded by the set's size.

// Node offsets of the upstream neighbours x - c_q, periodic wrap folded in.
__device__ inline void upstream_offsets(const Nbr& o, int* off) {
  const int t[kQ] = {0,
                     o.xm, o.xp, o.ym, o.yp, o.zm, o.zp,
                     o.xm + o.ym, o.xp + o.yp, o.xm + o.yp, o.xp + o.ym,
                     o.xm + o.zm, o.xp + o.zp, o.xm + o.zp, o.xp + o.zm,
                     o.ym + o.zm, o.yp + o.zp, o.ym + o.zp, o.yp + o.zm};
#pragma unroll
  for (int q = 0; q < kQ; ++q) off[q] = t[q];
}

// Byte offset of population 0 of node byte offset M = m * 4 in the block layout
// (m + 4608 (m >> 8) elements, see pull).
__device__ inline uint32_t inplace_node_bytes(uint32_t M) {
  return __umul24(M >> 10, (uint32_t)((kQ - 1) * kPopBlock * 4)) + M;
}

__device__ inline __amdgpu_buffer_rsrc_t inplace_rsrc(const Dev& d) {
  return __builtin_amdgcn_make_buffer_rsrc(d.pop[0], (short)0, (int)(uint32_t)(kQ * d.pstride * 4), kBufferWord3);
}

// Slot q of the node at byte offset b (from inplace_node_bytes), as float.
__device__ inline float inplace_load(__amdgpu_buffer_rsrc_t rs, uint32_t b, int q) {
  const uint32_t c = (uint32_t)q * kPopBlock * 4u;
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(rs, b + (c & 4095u), c & ~4095u, 0));
}

// Stores written through (system-coherent, the sc0 sc1 bits) while the set
// is of the order of the last-level cache, non-temporal above.
template <int AUX>
__device__ inline void inplace_store(__amdgpu_buffer_rsrc_t rs, uint32_t b, int q, float v) {
  const uint32_t c = (uint32_t)q * kPopBlock * 4u;
  __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(v), rs, b + (c & 4095u), c & ~4095u, AUX);
}
constexpr int kAuxWriteThrough = 17;  // sc0 | sc1
constexpr int kAuxNonTemporal = 2;    // nt

// The state after `steps` steps, f*_q(x) of node x (byte offset M), into g.
__device__ inline void inplace_post(__amdgpu_buffer_rsrc_t rs, uint32_t M, const int* off, int64_t steps, float* g) {
  if (steps & 1) {
    const uint32_t b = inplace_node_bytes(M);
#pragma unroll
    for (int q = 0; q < kQ; ++q) g[q] = inplace_load(rs, b, opposite(q));
  } else {
#pragma unroll
    for (int q = 0; q < kQ; ++q) g[q] = inplace_load(rs, inplace_node_bytes(M + (uint32_t)off[opposite(q)] * 4u), q);
  }
}

template <int AUX>
__device__ inline void inplace_push(__amdgpu_buffer_rsrc_t rs, uint32_t M, const int* off, bool odd, const float* g) {
  if (!odd) {
    const uint32_t b = inplace_node_bytes(M);
#pragma unroll
    for (int q = 0; q < kQ; ++q) inplace_store<AUX>(rs, b, opposite(q), g[q]);
  } else {
#pragma unroll
    for (int q = 0; q < kQ; ++q) inplace_store<AUX>(rs, inplace_node_bytes(M + (uint32_t)off[opposite(q)] * 4u), q, g[q]);
  }
}

// SERIAL: a full-grid launch with no concurrent kernels, whose odd-step
// stores go plain (the L2 merges the partial lines of the neighbours'
// scattered runs: 128^3 FP32 launch 48.1 against 50.2 us written through);
// beside the immersed-boundary kernels they stay written through (plain:
// step 58.9 against 56.8 us, the L2 taken from the concurrent kernels).
template <bool SERIAL>
__device__ inline void sc_node_inplace(const Dev& d, const Box& B, int x, int y, int z, int64_t base, int64_t n,
                                       bool forced, bool avg) {
  const Nbr o = neighbours(x, y, z, B.nx, B.ny, B.nz);
  int off[kQ];
  upstream_offsets(o, off);
  const __amdgpu_buffer_rsrc_t rs = inplace_rsrc(d);
  const int64_t ps = d.pstride;
  const uint32_t M = (uint32_t)base * 4u;
  const bool odd = (n & 1) != 0;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  if (avg) {
    a0 = d.uavg[base];
    a1 = d.uavg[ps + base];
    a2 = d.uavg[2 * ps + base];
  }
  float g[kQ];
  if (!odd) {
    const uint32_t b = inplace_node_bytes(M);
#pragma unroll
    for (int q = 0; q < kQ; ++q) g[q] = inplace_load(rs, b, q);
  } else {
#pragma unroll
    for (int q = 0; q < kQ; ++q) g[q] = inplace_load(rs, inplace_node_bytes(M + (uint32_t)off[q] * 4u), opposite(q));
  }
  const Moments m = moments(g);
  float Fx = B.gx, Fy = B.gy, Fz = B.gz;
  if (forced) {
    Fx += d.F[base];
    Fy += d.F[ps + base];
    Fz += d.F[2 * ps + base];
  }
  const float ir = inv_density(m.rho);
  const float ux = (m.jx + 0.5f * Fx) * ir;
  const float uy = (m.jy + 0.5f * Fy) * ir;
  const float uz = (m.jz + 0.5f * Fz) * ir;
  if (forced) {
    d.u[base] = ux;
    d.u[ps + base] = uy;
    d.u[2 * ps + base] = uz;
  }
  float ex = ux, ey = uy, ez = uz, src_a = 1.0f - 0.5f * B.omega;
  if (B.forcing == kShanChen) {
    ex = (m.jx + B.tau * Fx) * ir;
    ey = (m.jy + B.tau * Fy) * ir;
    ez = (m.jz + B.tau * Fz) * ir;
    src_a = 0.0f;
  }
  if (src_a != 0.0f && (Fx != 0.0f || Fy != 0.0f || Fz != 0.0f))
    collide_all<true>(g, m, B.omega, ex, ey, ez, src_a, ux, uy, uz, Fx, Fy, Fz);
  else
    collide_all<false>(g, m, B.omega, ex, ey, ez, src_a, ux, uy, uz, Fx, Fy, Fz);
  if (!d.small_pops)
    inplace_push<kAuxNonTemporal>(rs, M, off, odd, g);
  else if (SERIAL && odd)
    inplace_push<0>(rs, M, off, true, g);
  else
    inplace_push<kAuxWriteThrough>(rs, M, off, odd, g);
  if (avg) {
    double* __restrict__ acc = d.uavg;
    acc[base] = a0 + (double)ux;
    acc[ps + base] = a1 + (double)uy;
    acc[2 * ps + base] = a2 + (double)uz;
  }
}

// Whether step n adds to the time-average sums (uniform over a launch).
__device__ inline bool avg_sampled(const Dev& d, int64_t n) {
  return d.uavg != nullptr && n >= d.avg_t0 && (n - d.avg_t0) % d.avg_every == 0;
}

// Launch modes of the fused step:
//   kScAll    every node of the grid; F and u where the node's tile is
//             stamped active for this step (used without concurrent IBM work);
//   kScBulk   every block except those marked near at the previous step,
//             never forced; persistent when `resident` > 0 (each XCD walks one
//             contiguous range of blocks, leaving workgroup slots free for the
//             concurrent immersed-boundary kernels);
//   kScActive one workgroup per listed near block, forced where the node's
//             tile is active.
constexpr int kScAll = kLaunchAll, kScBulk = kLaunchBulk, kScActive = kLaunchActive;

template <int ST, int BS, bool MOM = false, bool NTLD = true, bool SERIAL = false>
__device__ inline void sc_block(const Dev& d, int blk, int64_t n, bool bulk, bool avg) {
  const int b = d.nboxes == 1 ? 0 : d.sc_block_box[blk];
  const Box B = d.boxes[b];
  const int first = d.nboxes == 1 ? 0 : d.sc_box_block0[b];
  const int id = (blk - first) * BS + (int)threadIdx.x;
  if (id >= B.n) return;
  const int yz = (int)divide((uint32_t)id, B.div_nx);
  const int x = id - yz * B.nx;
  const int z = (int)divide((uint32_t)yz, B.div_ny);
  const int y = yz - z * B.ny;
  // nodes of the bulk launch are never forced: every node a stencil reaches
  // lies in a near block, and an active tile's other nodes carry F = 0
  bool forced = false;
  if (!bulk) {
    const int tile = B.tile0 + (x / kTile) + B.tx * ((y / kTile) + B.ty * (z / kTile));
    forced = d.stamp[tile] == (int)n;
  }
  // the two addressing forms as separate code (a population set below 4 GiB
  // takes 32-bit offsets; the in-place set always does)
  if constexpr (ST == kFp32InPlace) {
    static_assert(!MOM, "the in-place storage does not record moments");
    sc_node_inplace<SERIAL>(d, B, x, y, z, B.node0 + id, n, forced, avg);
  } else if (d.pops32) {
    sc_node<ST, MOM, NTLD, true>(d, B, x, y, z, B.node0 + id, n, forced, avg);
  } else {
    sc_node<ST, MOM, NTLD, false>(d, B, x, y, z, B.node0 + id, n, forced, avg);
  }
}

// AVG: the variant launched while a time average of u runs (the sampling
// test and the sums); without it the averaging code is compiled out.
template <int ST, int BS, int MODE, bool AVG, bool NTLD>
__global__ __launch_bounds__(BS) void k_stream_collide(Dev d, int remap, int nblocks, int resident) {
  const int64_t n = *d.step + d.sub;
  const int64_t pn = n - 1;  // the step whose bead statistics marked the near blocks
  const int pp = (int)(pn & 1), pf = near_slot(pn);
  const bool avg = AVG && avg_sampled(d, n);
  if constexpr (MODE == kScActive) {
    if ((int)blockIdx.x >= d.max_near + d.nbeads) {
      // the total force of each marker at step n (the observable; the
      // spreading formed the same sums from the split parts)
      const int m = ((int)blockIdx.x - d.max_near - d.nbeads) * BS + (int)threadIdx.x;
      if (m < d.nm) {
        const BeadTerms t = d.bterms[d.marker_info[m].x];
        float f[3];
        marker_total(d, m, t, f);
        d.fm[m] = f[0];
        d.fm[d.nm + m] = f[1];
        d.fm[2 * d.nm + m] = f[2];
      }
      return;
    }
    if ((int)blockIdx.x >= d.max_near) {
      // the near blocks of step n + 1 around bead blockIdx.x - max_near, from
      // the bead region its statistics kernel found at step n
      const int b = (int)blockIdx.x - d.max_near;
      const BeadState& st = d.bstate[b];
      const int box = d.beads[b].box;
      __shared__ int reg[6];
      if (threadIdx.x < 3) {
        reg[threadIdx.x] = st.lo[threadIdx.x];
        reg[3 + threadIdx.x] = st.hi[threadIdx.x];
      }
      __syncthreads();
      mark_near_blocks(d, d.boxes[box], box, reg, reg + 3, n);
      return;
    }
    const int cnt = min(d.near_count[pp], d.max_near);
    if ((int)blockIdx.x < cnt)
      sc_block<ST, BS, false, NTLD>(d, d.near_list[pp * d.max_near + blockIdx.x], n, false, avg);
  } else if constexpr (MODE == kScBulk) {
    // Persistent launches (resident > 0) walk the blocks statically here
    // (FP16 storage; FP32 launches k_stream_collide_claimed instead): FP16
    // blocks take half the time of FP32 ones and the FP16 step is bound by
    // the immersed-boundary chain, so claiming blocks costs more than it
    // balances (58.8 against 57.7 us per 128^3 step).  With `remap` each XCD
    // walks one contiguous range of blocks, else the blocks go grid-stride
    // (round robin over the XCDs).
    if (resident && remap) {
      const int per = (nblocks + 7) / 8;  // logical blocks per XCD
      const int xcd = blockIdx.x % 8, g8 = (int)gridDim.x / 8;
      for (int j = blockIdx.x / 8; j < per; j += g8) {
        const int blk = xcd * per + j;
        if (blk < nblocks && d.near[pf * d.nsc + blk] != (int)pn) sc_block<ST, BS, false, NTLD>(d, blk, n, true, avg);
      }
    } else if (resident) {
      for (int blk = blockIdx.x; blk < nblocks; blk += (int)gridDim.x)
        if (d.near[pf * d.nsc + blk] != (int)pn) sc_block<ST, BS, false, NTLD>(d, blk, n, true, avg);
    } else {
      const int blk = logical_block(remap, nblocks);
      if (blk < nblocks && d.near[pf * d.nsc + blk] != (int)pn) sc_block<ST, BS, false, NTLD>(d, blk, n, true, avg);
    }
  } else {
    const int blk = logical_block(remap, nblocks);
    if (blk < nblocks) sc_block<ST, BS, false, NTLD, true>(d, blk, n, false, avg);
  }
}

// Persistent bulk launch with claimed blocks (FP32 storage; the same launch
// mode and arguments as k_stream_collide<..., kScBulk, ...> with resident > 0;
// a kernel of its own so that the claim slots in LDS are not allocated by the
// other launches).
template <int ST, int BS, bool AVG, bool NTLD>
__global__ __launch_bounds__(BS) void k_stream_collide_claimed(Dev d, int remap, int nblocks, int resident) {
  // The workgroups of group g = blockIdx.x mod G (G = 8 when the grid allows:
  // the workgroups of one XCD) claim the group's blocks one at a time from
  // the group's counter, so workgroups slowed by the concurrent
  // immersed-boundary kernels take fewer blocks (128^3 FP32 step 62.7
  // against 69.9 us with a static split).  The group's blocks are g, g + G,
  // g + 2G, ... (round robin), or, with `remap`, one contiguous range per
  // group.  The claim of the next block is issued before the current block's
  // work, which hides its latency; two claim slots need one barrier per block.
  // Odd steps walk each group's blocks in reverse, so a step starts on the
  // blocks the previous one wrote last, the likeliest to be still in the
  // last-level cache (128^3 FP32 step 58.0 against 58.7 us; the full-grid
  // launch gains nothing from the same reversal, 50.8 against 49.9 us).
  (void)resident;
  const int64_t n = *d.step + d.sub;
  const int64_t pn = n - 1;  // the step whose bead statistics marked the near blocks
  const int pf = near_slot(pn);
  const bool avg = AVG && avg_sampled(d, n);
  __shared__ int next[2];
  const int G = min(kXcds, (int)gridDim.x), g = (int)blockIdx.x % G;
  const int per = (nblocks + G - 1) / G;
  int* const ctr = d.work + ((int)(n & 1) * kXcds + g) * kWorkStride;
  if ((int)blockIdx.x < G && threadIdx.x == 0)
    d.work[((int)((n + 1) & 1) * kXcds + (int)blockIdx.x) * kWorkStride] = 0;
  if (threadIdx.x == 0) next[0] = atomicAdd(ctr, 1);
  __syncthreads();
  for (int i = 0;; ++i) {
    const int j = next[i & 1];  // uniform over the workgroup
    if (j >= per) break;
    // slot (i + 1) & 1 was last read in iteration i - 1, before its barrier
    if (threadIdx.x == 0) next[(i + 1) & 1] = atomicAdd(ctr, 1);
    const int jj = (n & 1) ? per - 1 - j : j;
    const int blk = remap ? g * per + jj : g + G * jj;
    if (blk < nblocks && d.near[pf * d.nsc + blk] != (int)pn) sc_block<ST, BS, false, NTLD>(d, blk, n, true, avg);
    __syncthreads();
  }
}

// FP32, recording (rho, u) per node (adjoint segment recompute), in the
// three launch modes of k_stream_collide with workgroups of kScBlock nodes.
template <int MODE>
__global__ __launch_bounds__(kScBlock) void k_stream_collide_mom(Dev d, int nblocks) {
  const int64_t n = *d.step + d.sub;
  const int64_t pn = n - 1;
  const int pp = (int)(pn & 1), pf = near_slot(pn);
  if constexpr (MODE == kScActive) {
    const int cnt = min(d.near_count[pp], d.max_near);
    if ((int)blockIdx.x < cnt)
      sc_block<kFp32, kScBlock, true>(d, d.near_list[pp * d.max_near + blockIdx.x], n, false, false);
  } else if constexpr (MODE == kScBulk) {
    const int blk = blockIdx.x;
    if (blk < nblocks && d.near[pf * d.nsc + blk] != (int)pn) sc_block<kFp32, kScBlock, true>(d, blk, n, true, false);
  } else {
    if ((int)blockIdx.x < nblocks) sc_block<kFp32, kScBlock, true>(d, blockIdx.x, n, false, false);
  }
}

// Advance the step counter past an enqueued chunk of `count` steps.
__global__ void k_tick(int64_t* step, int count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step += count;
}

// u_n and rho_n of the last completed step n = step - 1 (zero before any step).
template <int ST>
__global__ __launch_bounds__(kScBlock) void k_velocity(Dev d, float* __restrict__ uo,
                                                        float* __restrict__ ro) {
  using T = typename PopIO<ST>::T;
  const int blk = blockIdx.x;
  const int b = d.nboxes == 1 ? 0 : d.block_box[blk];
  const Box B = d.boxes[b];
  const int id = (blk - B.block0) * kScBlock + (int)threadIdx.x;
  if (id >= B.n) return;
  const int64_t c = *d.step;
  // outputs box after box: velocity [box][3][n_box], density [box][n_box]
  const int64_t ob = 3 * B.node0 + id, nb = B.n, orho = B.node0 + id;
  if (c == 0) {
    if (uo) {
      uo[ob] = 0.0f;
      uo[nb + ob] = 0.0f;
      uo[2 * nb + ob] = 0.0f;
    }
    if (ro) ro[orho] = 1.0f;
    return;
  }
  const int64_t n = c - 1;
  const int nx = B.nx, ny = B.ny, nz = B.nz;
  const int x = id % nx;
  const int yz = id / nx;
  const int y = yz % ny;
  const int z = yz / ny;
  const Nbr o = neighbours(x, y, z, nx, ny, nz);
  const int64_t ps = d.pstride;
  const int64_t base = B.node0 + id;
  float g[kQ];
  // the incoming populations of step n (two sets: still in the set step n
  // read), or, in place, the post-collision ones, whose momentum is j + F
  // (the collision adds the force density once, Guo or Shan-Chen)
  float hf = 0.5f;
  if constexpr (ST == kFp32InPlace) {
    int off[kQ];
    upstream_offsets(o, off);
    inplace_post(inplace_rsrc(d), (uint32_t)base * 4u, off, c, g);
    hf = -0.5f;
  } else {
    const T* src = static_cast<const T*>(d.pop[n & 1]);
    pull<ST>(src, base, o, d.fp16_inv, g);
  }
  const Moments m = moments(g);
  float Fx = B.gx, Fy = B.gy, Fz = B.gz;
  const int tile = B.tile0 + (x / kTile) + B.tx * ((y / kTile) + B.ty * (z / kTile));
  if (d.stamp[tile] == (int)n) {
    Fx += d.F[base];
    Fy += d.F[ps + base];
    Fz += d.F[2 * ps + base];
  }
  const float ir = inv_density(m.rho);
  if (uo) {
    uo[ob] = (m.jx + hf * Fx) * ir;
    uo[nb + ob] = (m.jy + hf * Fy) * ir;
    uo[2 * nb + ob] = (m.jz + hf * Fz) * ir;
  }
  if (ro) ro[orho] = m.rho;
}

// Time-average of u: the FP64 sums over `count` sampled steps divided by the
// count (zero without samples), box after box as [box][3][n_box].
__global__ __launch_bounds__(kScBlock) void k_average_out(Dev d, int64_t count, float* __restrict__ uo) {
  const int blk = blockIdx.x;
  const int b = d.nboxes == 1 ? 0 : d.block_box[blk];
  const Box B = d.boxes[b];
  const int id = (blk - B.block0) * kScBlock + (int)threadIdx.x;
  if (id >= B.n) return;
  const int64_t ob = 3 * B.node0 + id, nb = B.n, base = B.node0 + id, ps = d.pstride;
  const double inv = count > 0 ? 1.0 / (double)count : 0.0;
  uo[ob] = (float)(d.uavg[base] * inv);
  uo[nb + ob] = (float)(d.uavg[ps + base] * inv);
  uo[2 * nb + ob] = (float)(d.uavg[2 * ps + base] * inv);
}

// Block sum of 4 doubles through wavefront shuffles, result in thread 0.
__device__ inline void block_sum4(double* v) {
  __shared__ double part[kScBlock / 64][4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    for (int s = 32; s > 0; s >>= 1) v[k] += __shfl_xor(v[k], s, 64);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0)
    for (int k = 0; k < 4; ++k) part[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 4; ++k) {
      double s = 0;
      for (int w = 0; w < kScBlock / 64; ++w) s += part[w][k];
      v[k] = s;
    }
  }
}

// Stage 1: per-block FP64 sums of g and g c over the current state.
template <int ST>
__global__ __launch_bounds__(kScBlock) void k_conserved_partial(Dev d, int box, double* __restrict__ part) {
  using IO = PopIO<ST>;
  using T = typename IO::T;
  const int64_t c = *d.step;
  const T* src = static_cast<const T*>(d.pop[c & 1]);
  double v[4] = {0, 0, 0, 0};
  for (int b = 0; b < d.nboxes; ++b) {
    if (box >= 0 && b != box) continue;
    const Box B = d.boxes[b];
    for (int64_t id = (int64_t)blockIdx.x * kScBlock + threadIdx.x; id < B.n;
         id += (int64_t)gridDim.x * kScBlock) {
      float g[kQ];
      if constexpr (ST == kFp32InPlace) {
        // each node's own 19 post-collision values, wherever they are stored
        const int x = (int)(id % B.nx), yz = (int)(id / B.nx), y = yz % B.ny, z = yz / B.ny;
        int off[kQ];
        upstream_offsets(neighbours(x, y, z, B.nx, B.ny, B.nz), off);
        inplace_post(inplace_rsrc(d), (uint32_t)(B.node0 + id) * 4u, off, c, g);
      } else {
#pragma unroll
        for (int q = 0; q < kQ; ++q) g[q] = IO::ld(src + pop_index(q, B.node0 + id), q, d.fp16_inv);
      }
      const Moments m = moments(g);
      v[0] += (double)m.drho;
      v[1] += (double)m.jx;
      v[2] += (double)m.jy;
      v[3] += (double)m.jz;
    }
  }
  block_sum4(v);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) part[4 * blockIdx.x + k] = v[k];
}

// Stage 2: one block folds the partials in a fixed order; `mass0` (the sum
// of the weights, one per node, or 0 when the caller adds it) is added to the
// mass sum last.
__global__ __launch_bounds__(kScBlock) void k_conserved_final(const double* __restrict__ part,
                                                               int nparts, double* __restrict__ out,
                                                               double mass0) {
  double v[4] = {0, 0, 0, 0};
  for (int i = threadIdx.x; i < nparts; i += kScBlock)
    for (int k = 0; k < 4; ++k) v[k] += part[4 * i + k];
  block_sum4(v);
  if (threadIdx.x == 0) {
    out[0] = v[0] + mass0;
    for (int k = 1; k < 4; ++k) out[k] = v[k];
  }
}

// Plain device copy, one 16-byte vector per thread over a grid that covers
// the buffer, non-temporal loads and stores: the achievable-bandwidth
// reference for the HBM roofline.
__global__ __launch_bounds__(256) void k_copy(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                              int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

}  // namespace

void launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s) {
  const int64_t n = bytes / 16;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, (int64_t)1 << 30);
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, s, static_cast<const f32x4*>(src),
                     static_cast<f32x4*>(dst), n);
}

// Launch through hipExtLaunchKernelGGL when timing: the start / stop events are
// stamped by the kernel's own dispatch packet, so the elapsed time is the
// kernel's duration without the cost of separate event packets.
template <class K>
static void launch_k(K kernel, int grid, int block, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, const Dev& d,
                     int remap, int nblocks, int resident) {
  if (ev0)
    hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, ev0, ev1, 0, d, remap, nblocks, resident);
  else
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, d, remap, nblocks, resident);
}

template <int ST, int MODE, bool AVG, bool NTLD>
static void launch_sc_mode(const Dev& d, int block, int nblocks, int remap, int resident, int ncu,
                           hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  int grid = remap ? (nblocks + 7) / 8 * 8 : nblocks;
  if (MODE == kScActive) grid = d.max_near + (d.near_mark ? d.nbeads + (d.nm + block - 1) / block : 0);
  if (MODE == kScBulk && resident > 0)
    grid = remap ? std::min(grid, ncu * resident) / 8 * 8 : std::min(grid, ncu * resident);
  if (MODE != kScBulk) resident = 0;
  if (MODE == kScBulk && resident > 0 && ST != kFp16) {
    if (block == 128)
      launch_k(k_stream_collide_claimed<ST, 128, AVG, NTLD>, grid, 128, s, ev0, ev1, d, remap, nblocks, resident);
    else if (block == 512)
      launch_k(k_stream_collide_claimed<ST, 512, AVG, NTLD>, grid, 512, s, ev0, ev1, d, remap, nblocks, resident);
    else
      launch_k(k_stream_collide_claimed<ST, 256, AVG, NTLD>, grid, 256, s, ev0, ev1, d, remap, nblocks, resident);
    return;
  }
  if (block == 128)
    launch_k(k_stream_collide<ST, 128, MODE, AVG, NTLD>, grid, 128, s, ev0, ev1, d, remap, nblocks, resident);
  else if (block == 512)
    launch_k(k_stream_collide<ST, 512, MODE, AVG, NTLD>, grid, 512, s, ev0, ev1, d, remap, nblocks, resident);
  else
    launch_k(k_stream_collide<ST, 256, MODE, AVG, NTLD>, grid, 256, s, ev0, ev1, d, remap, nblocks, resident);
}

template <int ST, bool AVG, bool NTLD>
static void launch_sc_ld(const Dev& d, int mode, int block, int nblocks, int remap, int resident,
                         int ncu, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (mode == kScBulk)
    launch_sc_mode<ST, kScBulk, AVG, NTLD>(d, block, nblocks, remap, resident, ncu, s, ev0, ev1);
  else if (mode == kScActive)
    launch_sc_mode<ST, kScActive, AVG, NTLD>(d, block, nblocks, remap, resident, ncu, s, ev0, ev1);
  else
    launch_sc_mode<ST, kScAll, AVG, NTLD>(d, block, nblocks, remap, resident, ncu, s, ev0, ev1);
}

// FP16 pulls are plain loads in either regime, and the in-place set has one
// load form (one instance each)
template <int ST, bool AVG>
static void launch_sc_avg(const Dev& d, int mode, int block, int nblocks, int remap, int resident,
                          int ncu, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if constexpr (ST == kFp16 || ST == kFp32InPlace)
    launch_sc_ld<ST, AVG, true>(d, mode, block, nblocks, remap, resident, ncu, s, ev0, ev1);
  else if (d.small_pops)
    launch_sc_ld<ST, AVG, true>(d, mode, block, nblocks, remap, resident, ncu, s, ev0, ev1);
  else
    launch_sc_ld<ST, AVG, false>(d, mode, block, nblocks, remap, resident, ncu, s, ev0, ev1);
}

template <int ST>
static void launch_sc_st(const Dev& d, int mode, int block, int nblocks, int remap, int resident,
                         int ncu, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (d.uavg)
    launch_sc_avg<ST, true>(d, mode, block, nblocks, remap, resident, ncu, s, ev0, ev1);
  else
    launch_sc_avg<ST, false>(d, mode, block, nblocks, remap, resident, ncu, s, ev0, ev1);
}

void launch_stream_collide(const Dev& d, int storage, int mode, int block, int nblocks, int remap,
                           int resident, int ncu, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  if (storage == kFp16)
    launch_sc_st<kFp16>(d, mode, block, nblocks, remap, resident, ncu, s, ev0, ev1);
  else if (storage == kFp32Plain)
    launch_sc_st<kFp32Plain>(d, mode, block, nblocks, remap, resident, ncu, s, ev0, ev1);
  else if (storage == kFp32InPlace)
    launch_sc_st<kFp32InPlace>(d, mode, block, nblocks, remap, resident, ncu, s, ev0, ev1);
  else
    launch_sc_st<kFp32>(d, mode, block, nblocks, remap, resident, ncu, s, ev0, ev1);
}

void launch_stream_collide_mom(const Dev& d, int mode, int nblocks, hipStream_t s) {
  if (mode == kScActive)
    hipLaunchKernelGGL(k_stream_collide_mom<kScActive>, dim3(d.max_near), dim3(kScBlock), 0, s, d, nblocks);
  else if (mode == kScBulk)
    hipLaunchKernelGGL(k_stream_collide_mom<kScBulk>, dim3(nblocks), dim3(kScBlock), 0, s, d, nblocks);
  else
    hipLaunchKernelGGL(k_stream_collide_mom<kScAll>, dim3(nblocks), dim3(kScBlock), 0, s, d, nblocks);
}

void launch_tick(const Dev& d, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_tick, dim3(1), dim3(64), 0, s, d.step, count);
}

void launch_velocity(const Dev& d, int storage, int nblocks, float* u_out, float* rho_out,
                     hipStream_t s) {
  if (storage == kFp16)
    hipLaunchKernelGGL(k_velocity<kFp16>, dim3(nblocks), dim3(kScBlock), 0, s, d, u_out, rho_out);
  else if (storage == kFp32Plain)
    hipLaunchKernelGGL(k_velocity<kFp32Plain>, dim3(nblocks), dim3(kScBlock), 0, s, d, u_out, rho_out);
  else if (storage == kFp32InPlace)
    hipLaunchKernelGGL(k_velocity<kFp32InPlace>, dim3(nblocks), dim3(kScBlock), 0, s, d, u_out, rho_out);
  else
    hipLaunchKernelGGL(k_velocity<kFp32>, dim3(nblocks), dim3(kScBlock), 0, s, d, u_out, rho_out);
}

void launch_average_out(const Dev& d, int nblocks, int64_t count, float* u_out, hipStream_t s) {
  hipLaunchKernelGGL(k_average_out, dim3(nblocks), dim3(kScBlock), 0, s, d, count, u_out);
}

void launch_conserved(const Dev& d, int storage, int box, double* partial, int nparts, double* out,
                      hipStream_t s, double mass0) {
  if (storage == kFp16)
    hipLaunchKernelGGL(k_conserved_partial<kFp16>, dim3(nparts), dim3(kScBlock), 0, s, d, box, partial);
  else if (storage == kFp32Plain)
    hipLaunchKernelGGL(k_conserved_partial<kFp32Plain>, dim3(nparts), dim3(kScBlock), 0, s, d, box, partial);
  else if (storage == kFp32InPlace)
    hipLaunchKernelGGL(k_conserved_partial<kFp32InPlace>, dim3(nparts), dim3(kScBlock), 0, s, d, box, partial);
  else
    hipLaunchKernelGGL(k_conserved_partial<kFp32>, dim3(nparts), dim3(kScBlock), 0, s, d, box, partial);
  hipLaunchKernelGGL(k_conserved_final, dim3(1), dim3(kScBlock), 0, s, partial, nparts, out, mass0);
}

// ---- static scratch of the allocation-free conserved sums ---------------------
// The partial sums of lbm_batch_get_conserved_noalloc live in this array, one
// copy per GPU for the life of the process.  In host code `scratch` names a
// host-side stand-in, not device memory: its address on a GPU comes from
// hipGetSymbolAddress, called once per device while that device is current.
static __device__ __align__(256) double scratch[4 * kNoAllocParts];

namespace {
constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
double* scratch_addr[kMaxDevices] = {};
}  // namespace

hipError_t resolve_conserved_scratch(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_addr[device]) {
    double* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_addr[device] = p;
  }
  *out = scratch_addr[device];
  return hipSuccess;
}

}  // namespace lbmib
