/*
 * The library's C calling interface (lbm_create, lbm_swimmer_add, lbm_step,
 * the observables, batches, errors) served by the FP64 oracle, so that a test
 * can drive the same call sequence through the HIP library and through the
 * oracle and compare what comes back.  TEST INFRASTRUCTURE ONLY (see orc.h):
 * the product never loads this library.  It includes no header of the
 * product: the descriptor structs below are written out here with the field
 * order and types the interface fixes.
 *
 * What the oracle serves: lifetime, swimmers (one refinement level and one
 * set of membrane moduli per swimmer, as orc_add_swimmer takes them), body
 * force, stepping, marker / bead / swimmer observables, velocity and density
 * (host memory only, rounded to float32 as the interface's float32 outputs
 * are), conserved sums, population deviations, batches of boxes.  Calls tied
 * to the GPU implementation (time averages, adjoint, parameter changes,
 * checkpoints, kernel timing, the copy probe, device-memory sizes and the
 * allocation-free reduction) return LBM_ESTATE after their argument checks;
 * a valid launch shape is accepted and has no effect (the oracle has no
 * launch).
 *
 * Arguments are checked as the interface documents, before any work, and the
 * same invalid calls fail with the same codes.
 */
#include "orc.h"

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define E_OK 0
#define E_INVAL -1
#define E_NOMEM -2
#define E_STATE -4
#define E_NONFINITE -5

/* the interface's descriptor layouts */
typedef struct { int32_t nx, ny, nz; } abi_grid;
typedef struct {
  int32_t storage, delta_width;
  float fp16_scale;
  int32_t use_graphs;
  void* stream;
  void* field_memory;
  int64_t field_bytes;
} abi_opts;
typedef struct {
  double centre[3], radius;
  int32_t level;
  double kappa_s, C, kappa_b, kappa_v;
} abi_bead;
typedef struct { double k, L0; } abi_spring;
typedef struct { double A, B, period, alpha, phi0; } abi_act;
typedef struct {
  abi_grid grid;
  double tau;
  int32_t forcing;
} abi_box;

typedef struct {
  int nboxes, width, stepped;
  orc_sim** box;
  int* nx; /* 3 per box */
  int* last_box; /* box of the last swimmer added, -1 before */
  char err[256];
} abi_handle;

static int fail(abi_handle* h, int code, const char* msg) {
  if (h) snprintf(h->err, sizeof h->err, "%s", msg);
  return code;
}

static const char* const kNames[] = {"ok", "invalid argument", "out of memory", "HIP runtime error",
                                     "call not allowed in this state", "non-finite conserved sums",
                                     "file I/O error", "bead outgrew its reserved tile region"};

const char* lbm_strerror(int code) {
  const int i = -code;
  if (i < 0 || i >= (int)(sizeof kNames / sizeof kNames[0])) return "unknown error";
  return kNames[i];
}

const char* lbm_last_error(const abi_handle* h) { return h ? h->err : "null handle"; }

static int valid_box(const abi_box* b) {
  if (!(b->tau > 0.5) || !isfinite(b->tau)) return 0;
  if (b->grid.nx < 16 || b->grid.ny < 16 || b->grid.nz < 16) return 0;
  if ((int64_t)b->grid.nx * b->grid.ny * b->grid.nz > ((int64_t)1 << 31) - ((int64_t)1 << 16)) return 0;
  return b->forcing == ORC_GUO || b->forcing == ORC_SHAN_CHEN;
}

static int valid_opts(const abi_opts* o) {
  if (o->storage < 0 || o->storage > 3) return 0;
  if (o->delta_width < 2 || o->delta_width > 4) return 0;
  if (o->fp16_scale != 0.0f) {
    int e;
    frexpf(o->fp16_scale, &e);
    if (!(o->fp16_scale > 0.0f) || ldexpf(1.0f, e - 1) != o->fp16_scale) return 0;
  }
  return o->field_memory == NULL; /* the oracle holds no device memory */
}

static int create(const abi_box* boxes, int nboxes, const abi_opts* opts, abi_handle** out) {
  if (!out || !boxes || nboxes < 1) return E_INVAL;
  *out = NULL;
  int64_t total = 0;
  for (int b = 0; b < nboxes; ++b) {
    if (!valid_box(&boxes[b])) return E_INVAL;
    total += (int64_t)boxes[b].grid.nx * boxes[b].grid.ny * boxes[b].grid.nz;
  }
  if (total >= (int64_t)1 << 31) return E_INVAL;
  abi_opts o = {0, 3, 1.0f, 1, NULL, NULL, 0};
  if (opts) o = *opts;
  if (!valid_opts(&o)) return E_INVAL;
  abi_handle* h = (abi_handle*)calloc(1, sizeof(abi_handle));
  if (!h) return E_NOMEM;
  h->nboxes = nboxes;
  h->width = o.delta_width;
  h->box = (orc_sim**)calloc(nboxes, sizeof(orc_sim*));
  h->nx = (int*)calloc(3 * (size_t)nboxes, sizeof(int));
  h->last_box = (int*)malloc(sizeof(int));
  *h->last_box = -1;
  for (int b = 0; b < nboxes; ++b) {
    h->box[b] = orc_new(boxes[b].grid.nx, boxes[b].grid.ny, boxes[b].grid.nz, boxes[b].tau, boxes[b].forcing,
                        o.delta_width);
    h->nx[3 * b] = boxes[b].grid.nx;
    h->nx[3 * b + 1] = boxes[b].grid.ny;
    h->nx[3 * b + 2] = boxes[b].grid.nz;
  }
  *out = h;
  return E_OK;
}

int lbm_create(const abi_grid* grid, double tau, int forcing, const abi_opts* opts, abi_handle** out) {
  if (!grid) return E_INVAL;
  abi_box b = {*grid, tau, forcing};
  return create(&b, 1, opts, out);
}

int lbm_batch_create(const abi_box* boxes, int32_t nboxes, const abi_opts* opts, abi_handle** out) {
  return create(boxes, nboxes, opts, out);
}

int lbm_destroy(abi_handle* h) {
  if (!h) return E_OK;
  for (int b = 0; b < h->nboxes; ++b) orc_free(h->box[b]);
  free(h->box);
  free(h->nx);
  free(h->last_box);
  free(h);
  return E_OK;
}

static long nodes(const abi_handle* h, int b) { return (long)h->nx[3 * b] * h->nx[3 * b + 1] * h->nx[3 * b + 2]; }

int lbm_batch_swimmer_add(abi_handle* h, int32_t box, const abi_bead beads[3], const abi_spring springs[2],
                          const abi_act* act, int32_t* id) {
  if (!h || !beads || !springs || !act) return E_INVAL;
  if (box < 0 || box >= h->nboxes) return fail(h, E_INVAL, "box index out of range");
  if (*h->last_box > box) return fail(h, E_INVAL, "swimmers must be added in non-decreasing box order");
  if (h->stepped) return fail(h, E_STATE, "swimmers must be added before the first step");
  if (!(act->period > 0)) return fail(h, E_INVAL, "actuation period must be positive");
  int minedge = h->nx[3 * box];
  if (h->nx[3 * box + 1] < minedge) minedge = h->nx[3 * box + 1];
  if (h->nx[3 * box + 2] < minedge) minedge = h->nx[3 * box + 2];
  for (int k = 0; k < 3; ++k) {
    if (!(beads[k].radius > 0) || beads[k].level < 0 || beads[k].level > 5)
      return fail(h, E_INVAL, "bead radius must be positive and level in 0..5");
    /* the interface's size limit for a bead in its box */
    if (2.0 * beads[k].radius * 1.25 + h->width + 2 > minedge / 1.5)
      return fail(h, E_INVAL, "bead too large for the box");
    if (beads[k].level != beads[0].level || beads[k].kappa_s != beads[0].kappa_s || beads[k].C != beads[0].C ||
        beads[k].kappa_b != beads[0].kappa_b || beads[k].kappa_v != beads[0].kappa_v)
      return fail(h, E_INVAL, "the oracle takes one level and one set of moduli per swimmer");
  }
  double centres[9], radius[3], k[2] = {springs[0].k, springs[1].k}, L0[2] = {springs[0].L0, springs[1].L0};
  for (int b = 0; b < 3; ++b) {
    radius[b] = beads[b].radius;
    for (int q = 0; q < 3; ++q) centres[3 * b + q] = beads[b].centre[q];
  }
  orc_add_swimmer(h->box[box], centres, radius, beads[0].level, beads[0].kappa_s, beads[0].C, beads[0].kappa_b,
                  beads[0].kappa_v, k, L0, act->A, act->B, act->period, act->alpha, act->phi0);
  *h->last_box = box;
  if (id) {
    int n = 0;
    for (int b = 0; b < h->nboxes; ++b) n += orc_n_swimmers(h->box[b]);
    *id = n - 1;
  }
  return E_OK;
}

int lbm_swimmer_add(abi_handle* h, const abi_bead beads[3], const abi_spring springs[2], const abi_act* act,
                    int32_t* id) {
  return lbm_batch_swimmer_add(h, 0, beads, springs, act, id);
}

int lbm_set_body_force(abi_handle* h, const double g[3]) {
  if (!h || !g) return E_INVAL;
  for (int b = 0; b < h->nboxes; ++b) orc_set_body_force(h->box[b], g);
  return E_OK;
}

int lbm_step(abi_handle* h, int64_t n) {
  if (!h || n < 0) return E_INVAL;
  for (int b = 0; b < h->nboxes; ++b) orc_step(h->box[b], (long)n);
  if (n > 0) h->stepped = 1;
  return E_OK;
}

int lbm_batch_step(abi_handle* h, int64_t n) { return lbm_step(h, n); }

int lbm_sync(abi_handle* h) { return h ? E_OK : E_INVAL; }

int64_t lbm_time(const abi_handle* h) { return h ? orc_time(h->box[0]) : -1; }

int32_t lbm_n_markers(const abi_handle* h) {
  if (!h) return -1;
  int n = 0;
  for (int b = 0; b < h->nboxes; ++b) n += orc_n_markers(h->box[b]);
  return n;
}

int32_t lbm_n_swimmers(const abi_handle* h) {
  if (!h) return -1;
  int n = 0;
  for (int b = 0; b < h->nboxes; ++b) n += orc_n_swimmers(h->box[b]);
  return n;
}

int32_t lbm_n_boxes(const abi_handle* h) { return h ? h->nboxes : -1; }

/* Per-marker or per-swimmer arrays of every box, box after box (the swimmers'
 * order, since they are added in non-decreasing box order). */
typedef void (*getter)(const orc_sim*, double*);
static int gather(abi_handle* h, double* out, getter get, int per_box_count(const orc_sim*), int width) {
  if (!h || !out) return E_INVAL;
  for (int b = 0; b < h->nboxes; ++b) {
    const int n = per_box_count(h->box[b]);
    if (n) get(h->box[b], out);
    out += (size_t)width * n;
  }
  return E_OK;
}
static int n_beads3(const orc_sim* s) { return orc_n_beads(s); }

int lbm_get_swimmer_centres(abi_handle* h, double* out) {
  return gather(h, out, orc_get_swimmer_centres, orc_n_swimmers, 3);
}
int lbm_get_bead_centres(abi_handle* h, double* out) { return gather(h, out, orc_get_bead_centres, n_beads3, 3); }
int lbm_get_markers(abi_handle* h, double* out) { return gather(h, out, orc_get_markers, orc_n_markers, 3); }
int lbm_get_marker_velocities(abi_handle* h, double* out) {
  return gather(h, out, orc_get_marker_velocities, orc_n_markers, 3);
}
int lbm_get_marker_forces(abi_handle* h, double* out) {
  return gather(h, out, orc_get_marker_forces, orc_n_markers, 3);
}

/* a field of box b, `comps` values per node, rounded to float32 */
static int field(abi_handle* h, int b, float* dst, int on_device, int comps, getter get) {
  if (!h || !dst) return E_INVAL;
  if (b < 0 || b >= h->nboxes) return fail(h, E_INVAL, "box index out of range");
  if (on_device) return fail(h, E_INVAL, "the oracle has no device memory: on_device must be 0");
  const long n = nodes(h, b) * comps;
  double* tmp = (double*)malloc(sizeof(double) * n);
  if (!tmp) return E_NOMEM;
  get(h->box[b], tmp);
  for (long i = 0; i < n; ++i) dst[i] = (float)tmp[i];
  free(tmp);
  return E_OK;
}

int lbm_get_velocity(abi_handle* h, float* dst, int on_device) {
  return field(h, 0, dst, on_device, 3, orc_get_velocity);
}
int lbm_batch_get_velocity(abi_handle* h, int32_t box, float* dst, int on_device) {
  return field(h, box, dst, on_device, 3, orc_get_velocity);
}
int lbm_get_density(abi_handle* h, float* dst, int on_device) {
  return field(h, 0, dst, on_device, 1, orc_get_density);
}

int lbm_batch_get_conserved(abi_handle* h, int32_t box, double out[4]) {
  if (!h || !out) return E_INVAL;
  if (box < -1 || box >= h->nboxes) return fail(h, E_INVAL, "box index out of range");
  double s[4] = {0, 0, 0, 0};
  for (int b = 0; b < h->nboxes; ++b) {
    if (box >= 0 && b != box) continue;
    double o[4];
    orc_conserved(h->box[b], o);
    for (int q = 0; q < 4; ++q) s[q] += o[q];
  }
  for (int q = 0; q < 4; ++q) {
    out[q] = s[q];
    if (!isfinite(s[q])) return fail(h, E_NONFINITE, "non-finite conserved sums");
  }
  return E_OK;
}
int lbm_get_conserved(abi_handle* h, double out[4]) { return lbm_batch_get_conserved(h, -1, out); }

/* deviations g = f* - w, [19][nz][ny][nx] per box, box after box */
int lbm_get_populations(abi_handle* h, double* dev) {
  if (!h || !dev) return E_INVAL;
  int cx[19], cy[19], cz[19];
  double w[19];
  orc_lattice(cx, cy, cz, w);
  for (int b = 0; b < h->nboxes; ++b) {
    const long n = nodes(h, b);
    orc_get_pops(h->box[b], dev);
    for (int q = 0; q < 19; ++q)
      for (long i = 0; i < n; ++i) dev[q * n + i] -= w[q];
    dev += 19 * n;
  }
  return E_OK;
}

int lbm_set_populations(abi_handle* h, const double* dev) {
  if (!h || !dev) return E_INVAL;
  if (h->stepped) return fail(h, E_STATE, "populations can only be set before the first step");
  for (int b = 0; b < h->nboxes; ++b) {
    orc_set_deviation(h->box[b], dev);
    dev += 19 * nodes(h, b);
  }
  return E_OK;
}

/* ---- calls the oracle does not serve ------------------------------------ */
static int not_served(abi_handle* h) {
  if (!h) return E_INVAL;
  return fail(h, E_STATE, "not provided by the oracle");
}
int lbm_average_begin(abi_handle* h, int32_t every) {
  (void)every;
  return not_served(h);
}
int lbm_get_average_velocity(abi_handle* h, int32_t box, float* dst, int on_device, int64_t* samples) {
  (void)box, (void)dst, (void)on_device, (void)samples;
  return not_served(h);
}
int lbm_save(abi_handle* h, const char* path) {
  (void)path;
  return not_served(h);
}
int lbm_load(abi_handle* h, const char* path) {
  (void)path;
  return not_served(h);
}
int lbm_set_kernel_timing(abi_handle* h, int on) {
  (void)on;
  return not_served(h);
}
int lbm_kernel_time(abi_handle* h, double* ms, int64_t* launches) {
  (void)ms, (void)launches;
  return not_served(h);
}
int64_t lbm_bytes_per_step(const abi_handle* h) {
  (void)h;
  return 0;
}
int lbm_probe_copy_bandwidth(int64_t bytes, int iters, double* gbs) {
  if (bytes < 16 * 1024 || iters < 1 || !gbs) return E_INVAL;
  return E_STATE;
}
int lbm_set_stream_collide_launch(abi_handle* h, int block, int remap, int resident) {
  (void)remap;
  if (!h || (block != 128 && block != 256 && block != 512) || resident < -1 || resident > 64) return E_INVAL;
  return E_OK;
}
int lbm_batch_get_conserved_noalloc(abi_handle* h, int32_t box, int32_t parts, double* dst) {
  (void)box, (void)parts, (void)dst;
  return not_served(h);
}
int lbm_autotune(abi_handle* h, int32_t steps, const char* cache, char* report, int32_t report_len) {
  (void)steps, (void)cache;
  if (report && report_len > 0) report[0] = '\0';
  return not_served(h);
}
int lbm_swimmer_set_params(abi_handle* h, int32_t swimmer, double A, double B, double alpha, double k) {
  (void)swimmer, (void)A, (void)B, (void)alpha, (void)k;
  return not_served(h);
}
int lbm_adjoint(abi_handle* h, const void* desc, double* J, double grad[4]) {
  (void)desc, (void)J, (void)grad;
  return not_served(h);
}
int lbm_field_bytes(const abi_box* boxes, int32_t nboxes, int32_t storage, int64_t* bytes) {
  (void)boxes, (void)nboxes, (void)storage, (void)bytes;
  return E_STATE;
}
