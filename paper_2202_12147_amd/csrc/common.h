// Internal definitions shared by the lbmib HIP translation units.
//
// Device layout (one allocation per array, all boxes of a batch concatenated):
//   populations  pop[parity][node / 256][q][node % 256]   blocks of 256 nodes,
//                                       the 19 populations of a block one
//                                       after the other (pop_index); FP32 or
//                                       FP16; pstride (node count rounded up to
//                                       256) nodes per parity
//   force        F[3][node]             FP32, valid only in active tiles
//   velocity     u[3][node]             FP32, valid only in active tiles
//   tile stamps  stamp[tile]            step index at which a tile was last
//                                       made active (8x8x8-node tiles)
//   markers      pos[3][marker]         FP64 absolute, unwrapped
//                U[3][marker], f[3][marker]  FP32
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmib {

constexpr int kQ = 19;
constexpr int kTile = 8;       // active-tile edge in nodes
// Spreading workgroups per tile, each kTile / parts z layers: four for
// handles of at most kWideBeads beads (wide 512-lane workgroups, latency of
// the few of them dominates), two above (256-lane workgroups beside a bulk
// launch that keeps the GPU busy)
constexpr int kWideBeads = 32;
constexpr int kSpreadPartsWide = 4;
constexpr int kSpreadPartsNarrow = 2;
__host__ __device__ constexpr int spread_parts(int nbeads) {
  return nbeads <= kWideBeads ? kSpreadPartsWide : kSpreadPartsNarrow;
}
constexpr int kScBlock = 256;  // stream-collide threads per block
// Near-block flags hold three step slots (step mod 3): the bead statistics of
// step n mark slot n mod 3 while the bulk launch of step n - 1, which may
// still be running, reads slot (n - 2) mod 3.  Lists and counts, read only by
// the near-block launch that precedes the next marking on the same stream,
// keep two (step parity).
constexpr int kNearSlots = 3;

// Store of a streamed population value, written through: a relaxed atomic
// store at system scope, which the compiler issues as a plain global store
// with the system-coherence bits (no L2 line allocated).  For the 19-way
// streaming writes of a lattice sweep this leaves the L2 to the pulls and to
// the immersed-boundary kernels running beside the sweep.  On MI355X it pays
// while the two population sets are of the order of the 256 MB last-level
// cache (128^3 FP32: 45.5 us per sweep against 54.3 us with non-temporal
// stores; 45.9 us with plain stores, which slow the concurrent kernels) and
// costs 6 % on a 7.7 GB batch, so handles use it up to kWriteThroughBytes of
// population storage (Dev::small_pops) and non-temporal stores above.
__device__ inline void stream_store(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ inline void stream_store(unsigned short* p, unsigned short v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
constexpr int64_t kWriteThroughBytes = int64_t(1) << 30;  // both population sets
__host__ __device__ inline int near_slot(int64_t v) {
  const int r = (int)(v % kNearSlots);
  return r < 0 ? r + kNearSlots : r;
}
constexpr int kPopBlock = 256; // nodes per population block (a power of two: shifts and masks)
// mark_offset of launch_bead_stats that leaves the near blocks unmarked (the
// near-block launch of the concurrent schedule marks them instead)
constexpr int kNoMark = -(1 << 30);
// Block counters of the persistent bulk launch: one per XCD (workgroups are
// dealt to the 8 XCDs round robin) and step parity, each on its own 128-byte
// line; Dev::work holds kWorkCounters ints.
constexpr int kXcds = 8;
constexpr int kWorkStride = 32;
constexpr int kWorkCounters = 2 * kXcds * kWorkStride;

// Element index of population q of global node `node`.  A wavefront's 64
// consecutive nodes read or write one contiguous 256-byte (FP32) run per
// population, and a 256-node block's 19 runs are adjacent, so the DRAM sees a
// few long streams instead of 19 planes far apart.
__host__ __device__ inline int64_t pop_index(int q, int64_t node) {
  return (node / kPopBlock) * (int64_t)(kQ * kPopBlock) + q * kPopBlock + (node % kPopBlock);
}

enum Forcing { kGuo = 0, kShanChen = 1 };
enum Storage { kFp32 = 0, kFp16 = 1, kFp32Plain = 2, kFp32InPlace = 3 };

// D3Q19 velocities c_q in the population order of the interface (0 rest,
// 1..6 faces, 7..18 edges, opposite directions adjacent), for host code.
constexpr int kLatticeC[kQ][3] = {{0, 0, 0},  {1, 0, 0},  {-1, 0, 0}, {0, 1, 0},   {0, -1, 0},
                                  {0, 0, 1},  {0, 0, -1}, {1, 1, 0},  {-1, -1, 0}, {1, -1, 0},
                                  {-1, 1, 0}, {1, 0, 1},  {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
                                  {0, 1, 1},  {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};
__host__ __device__ constexpr int opposite(int q) { return q == 0 ? 0 : ((q & 1) ? q + 1 : q - 1); }
enum ScLaunch { kLaunchAll = 0, kLaunchBulk = 1, kLaunchActive = 2 };

// Division of unsigned 32-bit numbers by an invariant d >= 1 through a
// multiply-high and two shifts (Granlund and Montgomery, "Division by
// invariant integers using multiplication", 1994, Fig. 4.1): with
// l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1,
// n / d = (t + ((n - t) >> min(l, 1))) >> max(l - 1, 0), t = (m n) >> 32.
struct Divisor {
  uint32_t m;
  int s1, s2;
};

__host__ __device__ inline Divisor make_divisor(uint32_t d) {
  int l = 0;
  while (((uint64_t)1 << l) < d) ++l;
  const uint64_t m = (((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1;
  return Divisor{(uint32_t)m, l < 1 ? l : 1, l > 1 ? l - 1 : 0};
}

__host__ __device__ inline uint32_t divide(uint32_t n, const Divisor& v) {
  const uint32_t t = (uint32_t)(((uint64_t)v.m * n) >> 32);
  return (t + ((n - t) >> v.s1)) >> v.s2;
}

// One periodic box.  A single-box handle has exactly one.
struct Box {
  int nx, ny, nz;
  int tx, ty, tz;       // tiles per axis (ceil(n / kTile))
  int64_t node0;        // first node of the box in the population planes
  int64_t n;            // nodes in the box
  int tile0;            // first tile of the box in the stamp array
  int block0;           // first 256-node block of the box
  int bead0, nbeads;    // beads of the box (contiguous)
  int forcing;
  float tau, omega;     // tau and 1/tau
  float gx, gy, gz;     // uniform body force density
  Divisor div_nx, div_ny;  // node id -> (x, y, z) without integer division
};

// Per-bead constant data.
struct Bead {
  int first, nv;        // markers [first, first+nv)
  int tri0, ntri;       // triangles
  int box, swimmer;
  int slot;             // 0, 1, 2 within the swimmer
  int tiles_x, tiles_y, tiles_z;  // reserved candidate tiles per axis
  int tile_block0;      // first spread block of this bead
  float ks, C, kt, kv;  // Skalak ks and C, Kantor-Nelson kt = 2 kb/sqrt 3, kv
  double V0;            // stress-free volume
};

struct Swimmer {
  int bead[3];
  double k[2], L0[2];
  double A, B, omega, alpha, phi0;
};

// Per-bead state recomputed every step.
struct BeadState {
  double c[3];          // centre (mean of nodes)
  double V;             // enclosed volume
  int lo[3], hi[3];     // region: nodes [lo, hi] (unwrapped) within the kernel
                        // support of some marker
  int tlo[3], tcnt[3];  // region in tiles: first tile (in the box), count (periodic)
};

// Per-bead force terms of a step from its bead statistics (bead_terms.h):
// volume pressure pv and the per-node share of the bead's driving + spring
// force.
struct BeadTerms {
  float pv;
  float share[3];
};

// Everything a kernel needs, passed by value.
struct Dev {
  // lattice
  void* pop[2];
  int64_t pstride;
  float* F;
  float* u;
  int* stamp;
  const Box* boxes;
  int nboxes;
  const int* block_box;  // 256-node block -> box (output and reduction kernels)
  const int* sc_block_box;   // stream-collide block -> box (tuned block size)
  const int* sc_box_block0;  // first stream-collide block of each box
  int64_t* step;         // device step counter: first step of the enqueued chunk
  int sub;               // offset of this launch's step within the chunk
  float fp16_scale, fp16_inv;
  // markers and meshes
  double* pos;           // [3][nm]
  float* U;              // [3][nm]
  float* fm;             // [3][nm] total force on each marker (after the step)
  // the force split by what it depends on, so the membrane part needs no
  // bead statistics of the step: fmem = Skalak + bending, gvol = sum of the
  // area vectors of the node's triangles; the total is
  // fmem - pv gvol + (driving + spring force of the bead) / N_v
  float* fmem;           // [3][nm]
  float* gvol;           // [3][nm]
  int spread_raw;        // 1: spread d.fm as given (the adjoint's lambda_r)
  // bead terms of the step (bead_terms.h), kept by the spreading kernel
  BeadTerms* bterms;     // [nbeads]
  int nm;
  int width;             // delta kernel support in nodes
  const Bead* beads;
  int nbeads;
  BeadState* bstate;
  const Swimmer* swimmers;
  int nswimmers;
  const int* marker_bead;
  // per marker: bead, box, swimmer * 4 + slot, first bead of the swimmer (one
  // 16-byte load gives a marker-level kernel every index it dereferences)
  const int4* marker_info;
  // triangles: vertex ids and reference metric (FP64) / inverse (FP32)
  const int* tri;        // [3][ntri]
  const double* G0;      // [3][ntri]: G11, G12, G22
  const float* G0inv;    // [3][ntri]
  const float* A0;       // [ntri] reference area
  const float* idetG0;   // [ntri] 1 / det G0
  // hinges: x1, x2 shared edge, x3, x4 opposite; stress-free dihedral angle
  // theta0 as (cos theta0, sin theta0)
  const int* hinge;      // [4][nh]
  const double* th0cs;   // [2][nh]
  int ntri, nh;
  // per node, 32 force lanes: lanes 0..7 incident triangles (element
  // tri*3 + corner, vertex ids i0 i1 i2), lanes 8..31 hinges (element
  // h*4 + role, vertex ids x1 x2 x3 x4); element -1 = idle lane
  const int* lane_elem;  // [nm * 32]
  const int4* lane_v;    // [nm * 32]
  // stream-collide blocks near the swimmers: flags near[step mod 3][block] =
  // step that marked the block, and per-parity block lists
  // (near_list[parity][i], near_count[parity]); a block is near when it holds
  // a node within two nodes of a bead's stencil region
  int* near;
  // persistent bulk launch: block counters work[parity][group * kWorkStride]
  // (zero before a step's launch; each launch zeroes the next step's)
  int* work;
  int* near_list;
  int* near_count;
  int max_near, nsc, sc_bs;
  // nonzero in the near-block launch of the concurrent schedule: nbeads extra
  // workgroups mark the near blocks of the next step from the bead regions of
  // this step (mark_near_blocks), off the bead-statistics kernel's path, and
  // further ones form each marker's total force (fm)
  int near_mark;
  // 1 when both population sets take at most kWriteThroughBytes: the
  // streaming stores are written through (stream_store) and the pulls are
  // non-temporal loads, which lets the last-level cache serve part of the
  // traffic; 0 above: non-temporal stores and plain (cached) pulls
  int small_pops;
  // 1 when one population set takes less than 4 GiB: stream-collide
  // addresses are 32-bit byte offsets from the set's start
  int pops32;
  const int* tile_box;   // tile -> box (batches only)
  int* overflow;         // set when a bead region outgrows its reserved tiles
  int spread_blocks;
  // per spread block (two per reserved tile of each bead), two int4:
  // {bead, box, first bead of the box, beads in the box}, {kx, ky, kz, part}:
  // the tile's offset within the bead's reserved tiles and which part
  // (kTile / spread_parts(beads) z layers) of the tile the block fills
  const int4* spread_info;
  // (rho, u) of every node, written by the moment-recording stream-collide
  // variant only (segment recompute of the adjoint)
  float4* mom;
  // time average of the fluid velocity (optional): FP64 sums uavg[3][node]
  // of the u of steps avg_t0, avg_t0 + avg_every, ...; null when off
  double* uavg;
  int64_t avg_t0;
  int avg_every;
  // optional out-of-place variants (adjoint segment recompute): advection
  // writes r + U to pos_next instead of pos, and bead statistics take the
  // previous centres from bstate_prev instead of bstate
  double* pos_next;
  const BeadState* bstate_prev;
};

// Launch wrappers (defined in the .hip files).
// ev0 / ev1 (optional): events stamped by the launch's own dispatch packet
void launch_stream_collide(const Dev& d, int storage, int mode, int block, int nblocks, int remap,
                           int resident, int ncu, hipStream_t s, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr);
// Stream-collide (FP32 storage, single box, workgroups of kScBlock nodes,
// launch mode kLaunchAll / kLaunchBulk / kLaunchActive) that also writes each
// node's (rho, u_x, u_y, u_z) to d.mom; nblocks = node blocks of the box.
void launch_stream_collide_mom(const Dev& d, int mode, int nblocks, hipStream_t s);
void launch_tick(const Dev& d, int count, hipStream_t s);
void launch_velocity(const Dev& d, int storage, int nblocks, float* u_out, float* rho_out,
                     hipStream_t s);
// Mean velocity from the sums d.uavg over `count` samples (zero when count is
// 0), written box after box as [box][3][n_box] like launch_velocity.
void launch_average_out(const Dev& d, int nblocks, int64_t count, float* u_out, hipStream_t s);
// Two-stage FP64 sums of f* and f* c: `nparts` workgroups write partial sums
// to partial[4 * nparts], one workgroup folds them into out[4] and adds mass0
// to out[0].
void launch_conserved(const Dev& d, int storage, int box, double* partial, int nparts, double* out,
                      hipStream_t s, double mass0);
// Partial sums held by the allocation-free conserved-sum call: a static device
// array of kNoAllocParts x 4 doubles per GPU.  resolve_conserved_scratch gives
// its address on `device`, which must be the current device on the first call
// for that device (the address is looked up once and kept).
constexpr int kNoAllocParts = 4096;
hipError_t resolve_conserved_scratch(int device, double** out);
// mark_offset: the near blocks of step (counter + sub + mark_offset) are
// marked from the new bead regions; kNoMark: not marked.
void launch_bead_stats(const Dev& d, int mark_offset, hipStream_t s);
// bead statistics and the split membrane forces (independent of each other),
// in one launch for handles of at most kWideBeads beads
void launch_stats_forces(const Dev& d, int mark_offset, hipStream_t s);
// total marker forces of step counter + sub from the split parts into out
void launch_marker_force_total(const Dev& d, float* out, hipStream_t s);
void launch_spread(const Dev& d, hipStream_t s);
void launch_interp_advance(const Dev& d, hipStream_t s);
void launch_bead_centres(const Dev& d, double* out, hipStream_t s);
void launch_copy(const void* src, void* dst, int64_t bytes, hipStream_t s);

}  // namespace lbmib
