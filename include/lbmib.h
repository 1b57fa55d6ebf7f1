/*
 * lbmib — MI355X (gfx950) lattice Boltzmann + immersed boundary + finite
 * element bead-spring microswimmer step.
 *
 * Method: Geyer et al., "Lattice Boltzmann Simulations of Two Linear
 * Microswimmers Using the Immersed Boundary Method" (arXiv 2202.12147),
 * Sec. 2.1 (D3Q19 BGK fluid, Eqs. lbe, lbm:equilibrium, sc), Sec. 2.2
 * (three-bead spring swimmer, driving and spring forces, Skalak / Helfrich /
 * volume membrane energies of icosphere beads), Sec. 2.3 (IBM spreading and
 * interpolation with a discrete delta kernel, Eqs. spreading and
 * interpolation).
 *
 * Conventions shared by every call:
 *   - Return value 0 on success, a negative LBM_E* code on error.  No C++
 *     exception crosses this boundary.  lbm_last_error() gives the message of
 *     the handle's most recent error.
 *   - Lattice units: node (i,j,k) sits at integer coordinates; lengths in
 *     lattice spacings, times in steps, rho0 = 1 (Sec. 2.1).
 *   - Lattice fields are laid out [component][z][y][x], x fastest.
 *   - Populations: D3Q19 with index 0 = rest, 1..6 = +x,-x,+y,-y,+z,-z,
 *     7..18 = (+1,+1,0),(-1,-1,0),(+1,-1,0),(-1,+1,0),(+1,0,+1),(-1,0,-1),
 *     (+1,0,-1),(-1,0,+1),(0,+1,+1),(0,-1,-1),(0,+1,-1),(0,-1,+1).  They
 *     cross the boundary as deviations g_i = f_i - w_i from the rest state
 *     (w_i the lattice weights of Sec. 2.1), in float64.
 *   - Marker (mesh node) arrays are [marker][xyz] in float64, unwrapped (they
 *     may leave the box; grid indices wrap periodically).
 *   - Pointers marked "device" must be device memory of the handle's device;
 *     "host" pointers are ordinary host memory.  The caller owns every buffer
 *     it passes; the handle owns its internal device memory and frees it in
 *     lbm_destroy.
 *   - All work is enqueued on the handle's stream.  Calls that return data to
 *     the host (or into caller device memory) synchronise that stream before
 *     returning.  One handle must not be used from two host threads at once.
 */
#ifndef LBMIB_H
#define LBMIB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---------------------------------------------------------- */
#define LBM_OK 0
#define LBM_EINVAL -1      /* invalid argument (bad size, enum, tau <= 1/2 ...) */
#define LBM_ENOMEM -2      /* device or host allocation failed */
#define LBM_EDEVICE -3     /* a HIP runtime call failed */
#define LBM_ESTATE -4      /* call not allowed in the current state */
#define LBM_ENONFINITE -5  /* NaN or Inf found in the conserved sums */
#define LBM_EIO -6         /* file could not be read or written */
#define LBM_EOVERFLOW -7   /* a bead outgrew the region reserved for it */

/* ---- enums ---------------------------------------------------------------- */
/* Body-force scheme.  SHAN_CHEN shifts the equilibrium velocity,
 * rho u_eq = sum f c + tau F (Sec. 2.1, Eq. sc), as the paper does.  GUO
 * uses u = (sum f c + F/2)/rho in the equilibrium plus the source term
 * (1 - 1/(2 tau)) w_i [3 (c_i - u) + 9 (c_i . u) c_i] . F.  In both the
 * physical velocity is rho u = sum f c + F/2 (Sec. 2.1). */
typedef enum { LBM_GUO = 0, LBM_SHAN_CHEN = 1 } lbm_forcing;

/* Population storage on the device; arithmetic is FP32 in all four.  The
 * shifted forms store the deviation g = f - w from the rest state;
 * FP16_SHIFTED stores g * scale rounded to nearest-even half precision.
 * FP32_PLAIN stores f itself, rounded at the scale of the weights (~1/3), a
 * reference that shows the precision the shift recovers.  FP32_INPLACE
 * stores the FP32 deviations in ONE population set updated in place (the
 * AA access pattern of Bailey et al., ICPP 2009: even steps read a node's
 * own slots and write them back reversed, odd steps read from and write to
 * the neighbours' slots), half the memory of the two-set pull scheme and
 * the same streaming and collision bit for bit; one set must stay below
 * 4 GiB (LBM_EINVAL otherwise).  Not for lbm_adjoint. */
typedef enum {
  LBM_FP32_SHIFTED = 0,
  LBM_FP16_SHIFTED = 1,
  LBM_FP32_PLAIN = 2,
  LBM_FP32_INPLACE = 3
} lbm_storage;

/* ---- descriptors ---------------------------------------------------------- */
typedef struct {
  int32_t nx, ny, nz; /* fully periodic box (Sec. 3) */
} lbm_grid;

typedef struct {
  int32_t storage;     /* lbm_storage */
  int32_t delta_width; /* IBM kernel support in nodes: 2 (two-point linear, Sec.
                          2.3), 3 (Roma-Peskin-Berger) or 4 (Peskin) */
  float fp16_scale;    /* power of two S for FP16_SHIFTED (0 = default 1) */
  int32_t use_graphs;  /* 1 = replay steps from captured HIP graphs */
  void* stream;        /* hipStream_t to enqueue on; NULL = own stream */
  /* Device memory for the node fields (both population sets, the body-force
   * density and the velocity), e.g. a tensor the caller allocated; NULL = the
   * handle allocates them.  At least lbm_field_bytes() bytes, 256-byte
   * aligned, on the handle's device.  The caller owns it, keeps it alive and
   * untouched until lbm_destroy, and frees it afterwards; lbm_create
   * overwrites it with the rest state.  The handle's other device memory
   * stays its own: mesh tables, bead, tile, block-flag and reduction
   * buffers (at most a few bytes per 128 nodes), and, made on first use, the
   * staging of lbm_get_velocity into host memory, the sums of the time
   * average and the adjoint's workspace. */
  void* field_memory;
  int64_t field_bytes; /* size of field_memory in bytes */
} lbm_opts;

typedef struct {
  double centre[3]; /* initial bead centre */
  double radius;    /* shell radius */
  int32_t level;    /* icosphere refinement level: 20*4^level triangles */
  double kappa_s;   /* Skalak shear modulus (Sec. 2.2) */
  double C;         /* Skalak area constant, kappa_a/kappa_s = 1 + 2C */
  double kappa_b;   /* Helfrich bending modulus (Kantor-Nelson discretised) */
  double kappa_v;   /* volume penalty modulus, Eq. (vol_cons) */
} lbm_bead_desc;

typedef struct {
  double k;  /* harmonic spring constant (Sec. 2.2) */
  double L0; /* equilibrium length L_spring */
} lbm_spring_desc;

typedef struct {
  double A;      /* amplitude on bead 1: f1 = A sin(w t + phi0) x (Sec. 2.2) */
  double B;      /* amplitude on bead 3: f3 = B sin(w t + phi0 + alpha) x */
  double period; /* T, w = 2 pi / T, t = step index */
  double alpha;  /* phase shift between the outer beads */
  double phi0;   /* common phase offset (0 in the paper) */
} lbm_actuation_desc;

typedef struct lbm_handle lbm_handle;

/* ---- lifetime --------------------------------------------------------------- */
/* Create a periodic D3Q19 BGK fluid at rest (rho = 1, u = 0), relaxation time
 * tau (Eq. lbe; viscosity nu = (tau - 1/2)/3, Sec. 2.1).  Requires tau > 1/2,
 * every grid edge >= 16, at most 2^31 - 2^16 nodes (a batch: per box, and
 * fewer than 2^31 in all), forcing and opts valid.  opts may be NULL (FP32,
 * 3-point kernel, graphs on, own stream, fields allocated by the handle).
 * *out receives the handle.  Errors: LBM_EINVAL (also: field_memory not
 * 256-byte aligned or field_bytes below lbm_field_bytes), LBM_ENOMEM,
 * LBM_EDEVICE. */
int lbm_create(const lbm_grid* grid, double tau, int forcing, const lbm_opts* opts,
               lbm_handle** out);

/* Release the handle's own device memory and the handle (not caller field
 * memory).  Accepts NULL. */
int lbm_destroy(lbm_handle* h);

/* Add one three-bead swimmer (Sec. 2.2, Fig. 1): beads[0..2] in order along
 * the swimmer, springs[0] joins beads 0-1, springs[1] joins beads 2-1, the
 * driving forces act along x.  Each bead is an icosphere (an icosahedron
 * refined `level` times, new vertices projected onto the sphere) whose
 * initial shape is stress-free.  Allowed only before the first lbm_step
 * (LBM_ESTATE afterwards).  *id (may be NULL) receives the swimmer index.
 * Errors: LBM_EINVAL (radius <= 0, level outside 0..5, bead larger than a
 * third of the box), LBM_ESTATE, LBM_ENOMEM, LBM_EDEVICE. */
int lbm_swimmer_add(lbm_handle* h, const lbm_bead_desc beads[3],
                    const lbm_spring_desc springs[2], const lbm_actuation_desc* act,
                    int32_t* id);

/* Uniform body force density added to F at every node (test and drag setups). */
int lbm_set_body_force(lbm_handle* h, const double g[3]);

/* ---- stepping ---------------------------------------------------------------- */
/* Advance n time steps, asynchronously on the handle's stream.  One step:
 * bead centres, driving + spring + membrane forces, spreading (Eq.
 * spreading), fused stream-collide (Eq. lbe), interpolation (Eq.
 * interpolation) and marker advection r += U.  Errors: LBM_EINVAL (n < 0),
 * LBM_EDEVICE. */
int lbm_step(lbm_handle* h, int64_t n);

/* Block until all enqueued work is done; reports LBM_EOVERFLOW if a bead
 * outgrew its reserved tile region during the steps. */
int lbm_sync(lbm_handle* h);

/* ---- observables (synchronous) ---------------------------------------------- */
int64_t lbm_time(const lbm_handle* h);    /* steps taken */
int32_t lbm_n_markers(const lbm_handle* h);
int32_t lbm_n_swimmers(const lbm_handle* h);

/* Swimmer centres x_cm = mean of the three bead centres (Eq. vel_swim), each
 * bead centre the mean of its mesh nodes; host out[n_swimmers*3], float64. */
int lbm_get_swimmer_centres(lbm_handle* h, double* out);
/* Bead centres, host out[3*n_swimmers*3], float64. */
int lbm_get_bead_centres(lbm_handle* h, double* out);
/* Marker positions, host out[n_markers*3], float64 (unwrapped). */
int lbm_get_markers(lbm_handle* h, double* out);
/* Interpolated marker velocities of the last step, host out[n_markers*3]. */
int lbm_get_marker_velocities(lbm_handle* h, double* out);
/* Total nodal forces f_tot of the last step (Sec. 2.2), host out[n_markers*3]. */
int lbm_get_marker_forces(lbm_handle* h, double* out);

/* Physical fluid velocity u_n = (sum f c + F/2)/rho of the last completed
 * step n (the velocity the markers were advected with), dst[3][nz][ny][nx]
 * float32; on_device = 1: dst is device memory, 0: host memory.  Before the
 * first step it is zero. */
int lbm_get_velocity(lbm_handle* h, float* dst, int on_device);
/* Density rho_n of the last completed step, dst[nz][ny][nx] float32. */
int lbm_get_density(lbm_handle* h, float* dst, int on_device);

/* Time-averaged fluid velocity, the quantity of the period-averaged flow
 * fields in the results (Sec. 3, Figs. 3, 6 and 9: the average over one
 * swimming period).  lbm_average_begin(h, every), every >= 1, starts a new
 * average: from the next step on, that step and every every-th step after it
 * add their physical velocity u (as lbm_get_velocity) to per-node float64
 * sums held on the device (24 bytes per node, allocated on first use, freed
 * by lbm_destroy); every = 1 samples every step.  The stream-collide launches
 * add u as they compute it: a sampled step moves 48 more bytes per node.
 * every = 0 stops the average.  lbm_load stops it (the sums and the
 * sampling schedule are not part of a checkpoint), and lbm_adjoint fails
 * with LBM_ESTATE while one runs.  Errors: LBM_EINVAL (every < 0), LBM_ENOMEM. */
int lbm_average_begin(lbm_handle* h, int32_t every);
/* Mean of the sampled velocities of box `box` (0 for a single box), dst
 * [3][nz][ny][nx] float32, device (on_device = 1) or host memory; zero when
 * no step has been sampled yet.  *samples (if non-NULL) receives the number
 * of steps averaged.  Synchronous.  LBM_ESTATE when no average is running,
 * LBM_EINVAL for a box out of range. */
int lbm_get_average_velocity(lbm_handle* h, int32_t box, float* dst, int on_device, int64_t* samples);

/* out[0] = sum over nodes and populations of f*, out[1..3] = sum f* c, of the
 * current post-collision state, reduced in float64 on the device.
 * LBM_ENONFINITE if any sum is NaN or Inf. */
int lbm_get_conserved(lbm_handle* h, double out[4]);

/* Population deviations g = f* - w of the current post-collision state,
 * host float64 [19][nz][ny][nx] (for a batch, box after box, each
 * [19][nz][ny][nx]).  set: before the first step only. */
int lbm_set_populations(lbm_handle* h, const double* dev);
int lbm_get_populations(lbm_handle* h, double* dev);

/* ---- batches of independent boxes -------------------------------------------- */
/* One periodic box of a batch: its own grid, relaxation time and forcing. */
typedef struct {
  lbm_grid grid;
  double tau;
  int32_t forcing; /* lbm_forcing */
} lbm_box_desc;

/* Create a handle stepping `nboxes` independent periodic boxes together: every
 * step is one pass of the method over all boxes (shared launches, one graph).
 * Each box starts at rest.  Box b's nodes follow box b-1's in the population
 * planes.  Validation as lbm_create per box.  lbm_step, lbm_sync,
 * lbm_get_swimmer_centres, lbm_get_bead_centres, lbm_get_markers and the
 * checkpoint calls act on the whole batch; swimmers are numbered across boxes
 * in the order they were added.  Errors: as lbm_create. */
int lbm_batch_create(const lbm_box_desc* boxes, int32_t nboxes, const lbm_opts* opts,
                     lbm_handle** out);

/* Bytes of caller field memory (lbm_opts.field_memory) that a handle over
 * these boxes with this storage (lbm_storage) needs: two population sets
 * (one with FP32_INPLACE; 19 values per node, 4 bytes each, 2 with
 * FP16_SHIFTED) plus 3 float32 of
 * body force and 3 of velocity per node, each part padded to the population
 * blocks of 256 nodes.  Host-only; no device is touched.  Errors: LBM_EINVAL
 * (boxes that lbm_batch_create would reject, unknown storage, NULL bytes). */
int lbm_field_bytes(const lbm_box_desc* boxes, int32_t nboxes, int32_t storage, int64_t* bytes);
/* Add a swimmer (as lbm_swimmer_add) to box `box`.  Swimmers must be added in
 * non-decreasing box order (LBM_EINVAL otherwise). */
int lbm_batch_swimmer_add(lbm_handle* h, int32_t box, const lbm_bead_desc beads[3],
                          const lbm_spring_desc springs[2], const lbm_actuation_desc* act,
                          int32_t* id);
int32_t lbm_n_boxes(const lbm_handle* h);
/* Advance every box of a batch n steps: the same call as lbm_step (which
 * accepts batch handles too), under the batch's name. */
int lbm_batch_step(lbm_handle* h, int64_t n);
/* Velocity (layout as lbm_get_velocity) of one box of the batch. */
int lbm_batch_get_velocity(lbm_handle* h, int32_t box, float* dst, int on_device);
/* Conserved sums (as lbm_get_conserved) of one box; box = -1 sums all boxes. */
int lbm_batch_get_conserved(lbm_handle* h, int32_t box, double out[4]);

/* For callers that cannot allocate device memory or wait on the host (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the conserved sums of lbm_batch_get_conserved (box = -1: all
 * boxes), enqueued on the handle's stream without allocating and without
 * synchronising.  dst: caller device memory of 4 float64, receives
 * dst[0] = sum f* (the weights included, one per node) and dst[1..3] =
 * sum f* c once the stream reaches the work; no finiteness check (read dst
 * after synchronising the stream).  parts: workgroups of the first reduction
 * stage, 1..4096 (lbm_batch_get_conserved uses 1024, and gives the same bits
 * at that value).  Their partial sums go to one static device array of the
 * library, 4096 x 4 float64 = 128 KiB per GPU, held until the process ends
 * and shared by every call on that GPU: calls that overlap on one GPU (two
 * streams or two host threads) race on it.  Every call overwrites the
 * `parts` entries it reads, so nothing has to start at zero.
 * Errors: LBM_EINVAL (null handle or dst, box out of range, parts outside
 * 1..4096), LBM_ESTATE, LBM_EDEVICE. */
int lbm_batch_get_conserved_noalloc(lbm_handle* h, int32_t box, int32_t parts, double* dst);

/* Autotuner for the stream-collide launch shape: disabled, returns
 * LBM_ESTATE (LBM_EINVAL for a null handle) and writes an empty report.  One
 * GPU run aborted inside it with a corrupted host heap and no cause has been
 * shown, so it does not run until one is.  Launch shapes are set with
 * lbm_set_stream_collide_launch (the defaults are the fastest measured). */
int lbm_autotune(lbm_handle* h, int32_t steps_per_candidate, const char* cache_path, char* report,
                 int32_t report_len);

/* ---- gradient of the swimming displacement (discrete adjoint) -------------- */
/* Set the four parameters the adjoint differentiates of swimmer `swimmer`:
 * driving amplitudes A (bead 1) and B (bead 3), their phase shift alpha
 * (Sec. 2.2) and the constant k of both springs.  Allowed at any time; the
 * next step uses them.  Errors: LBM_EINVAL (no such swimmer), LBM_EDEVICE. */
int lbm_swimmer_set_params(lbm_handle* h, int32_t swimmer, double A, double B, double alpha, double k);

typedef struct {
  int64_t steps;      /* T: steps of the forward run (>= 1) */
  int32_t checkpoint; /* K: forward state kept every K steps, the reverse
                         sweep recomputes each K-step segment (>= 1; K >= T
                         stores the whole run) */
  int32_t swimmer;    /* objective swimmer */
  int32_t rewind;     /* nonzero: restore the state held at entry on return */
} lbm_adjoint_desc;

/* Objective J = x_cm(t0 + T) - x_cm(t0), the x displacement of swimmer
 * `swimmer`'s centre (mean of its three bead centres, Eq. vel_swim) over T
 * steps from the current state t0, and its exact gradient through the
 * discrete time stepping (the transposed linearisation of every operation of
 * lbm_step: collision, streaming, spreading, interpolation, advection and the
 * membrane, spring and driving forces of Sec. 2.2) with respect to
 * (A, B, alpha, k) of that swimmer: host grad[0..3] = dJ/dA, dJ/dB,
 * dJ/dalpha, dJ/dk (k scales both springs).  The forward run is ordinary
 * stepping, so on return the handle has advanced T steps exactly as lbm_step
 * would have taken it (unless `rewind`).  Device memory: 19*4 bytes per node
 * per checkpoint; two segment buffers (the recompute of one segment runs
 * beside the reverse sweep of the next) of 28 bytes per node per segment
 * step ((rho, u) and the force density); six population sets.  The adjoint arithmetic is FP32 on the grid and FP64 on the markers
 * and parameter sums.  Single-box handles with FP32_SHIFTED storage; Guo or
 * Shan-Chen forcing (Sec. 2.1, Eq. sc).  Errors: LBM_EINVAL (bad descriptor,
 * batch, any other storage), LBM_ENOMEM, LBM_EDEVICE, LBM_EOVERFLOW. */
int lbm_adjoint(lbm_handle* h, const lbm_adjoint_desc* desc, double* J, double grad[4]);

/* ---- checkpoint ---------------------------------------------------------------- */
/* Write / restore the full dynamic state (populations, forces, tile stamps,
 * markers, step counter) to / from a file.  Restoring needs a handle created
 * with the same grid, options and swimmers, and a file of the same format
 * version (written into its header); the restart is bit-exact.
 * Errors: LBM_EIO, LBM_EINVAL (mismatched handle or format version). */
int lbm_save(lbm_handle* h, const char* path);
int lbm_load(lbm_handle* h, const char* path);

/* ---- measurement ------------------------------------------------------------ */
/* When on, lbm_step runs without graphs and brackets every stream-collide
 * launch with HIP events on the handle's stream; lbm_kernel_time returns the
 * summed kernel time (ms) and launch count since timing was switched on. */
int lbm_set_kernel_timing(lbm_handle* h, int on);
int lbm_kernel_time(lbm_handle* h, double* ms, int64_t* launches);
/* Launch shape of the stream-collide kernel: workgroup size 128, 256 or 512
 * nodes; whether workgroups are remapped so that each of the 8 XCDs streams
 * one contiguous range of the grid; and, with swimmers, `resident` > 0 makes
 * the launch that runs concurrently with the immersed-boundary kernels
 * persistent with that many workgroups per compute unit (0: one workgroup
 * per block; -1: no concurrency, the immersed-boundary kernels then one
 * full-grid launch).  With FP32 storage (either form) the persistent
 * workgroups of each XCD claim that XCD's blocks one at a time from a device
 * counter; with FP16 storage they walk them in a fixed order.  An XCD's
 * blocks are one contiguous range when remapped, every eighth block
 * otherwise.  Results are bitwise identical for every shape.  Defaults (the
 * fastest measured on MI355X): one box with FP32 storage 512 / no remap / 1;
 * FP16 storage 256 / no remap / 2; batches 512 / no remap / 0.
 * Errors: LBM_EINVAL. */
int lbm_set_stream_collide_launch(lbm_handle* h, int block, int xcd_remap, int resident);
/* Algorithmic bytes one stream-collide launch moves (19 populations read and
 * written once per node at the storage width). */
int64_t lbm_bytes_per_step(const lbm_handle* h);

/* Achievable device-memory bandwidth: times `iters` launches of a plain copy
 * kernel between two fresh device buffers of `bytes` each (allocated and freed
 * here) and writes read+write bytes per second / 1e9 to *gbs.  Errors:
 * LBM_EINVAL (bytes < 16 KiB, iters < 1), LBM_ENOMEM, LBM_EDEVICE. */
int lbm_probe_copy_bandwidth(int64_t bytes, int iters, double* gbs);

/* ---- errors ---------------------------------------------------------------- */
const char* lbm_strerror(int code);
const char* lbm_last_error(const lbm_handle* h);

#ifdef __cplusplus
}
#endif
#endif
