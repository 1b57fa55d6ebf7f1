/*
 * Oracle: lattice Boltzmann fluid, immersed-boundary coupling, swimmers and
 * the time step.  TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * One step n -> n+1 (the paper does not fix the order inside a step; this is
 * the reading used throughout):
 *   O1  bead centres R_b = mean of the bead's mesh nodes (Fig. 1 caption,
 *       Sec. 2.2 "centers of mass");
 *   O2  driving forces f1 = A sin(w t + phi0), f3 = B sin(w t + phi0 + alpha),
 *       f2 = -f1 - f3 along x, w = 2 pi / T, t = n (Sec. 2.2, Eq. ext forces);
 *   O3  spring forces between beads 1-2 and 3-2 (Sec. 2.2);
 *   O4  membrane forces f_part = -dW/dr (Sec. 2.2, virtual work);
 *   O5  total nodal force f_tot = f_part + (f_d + f_s)/N_v (Sec. 2.2);
 *   O6  spreading F(x) = sum_m f_tot,m Delta(x - r_m) over all periodic
 *       images (Sec. 2.3, Eq. spreading);
 *   O7  streaming f_i(x) = f*_i(x - c_i) on the periodic box (Eq. lbe);
 *   O8  moments rho = sum f_i, j = sum f_i c_i, physical velocity
 *       rho u = j + F/2 (Sec. 2.1);
 *   O9  BGK collision (Eq. lbe, Eq. lbm:equilibrium) with either the
 *       Shan-Chen velocity shift rho u_eq = j + tau F (Eq. sc) or the Guo
 *       source term;
 *   O10 interpolation U_m = sum_x u(x) Delta(x - r_m) (Eq. interpolation);
 *   O11 marker advection r_m += U_m (forward Euler, dt = 1; Sec. 2.3 says the
 *       markers move with the local fluid velocity);
 *   O12 n += 1.
 */
#include "orc_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D3Q19 (Sec. 2.1): weights 1/3 (rest), 1/18 (faces), 1/36 (edges) */
static const int CX[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static const double WT[19] = {1.0 / 3.0,  1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                               1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                               1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static double W(int i) { return WT[i]; }
static int OPP(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

void orc_lattice(int* cx, int* cy, int* cz, double* w) {
  for (int i = 0; i < 19; ++i) {
    cx[i] = CX[i];
    cy[i] = CY[i];
    cz[i] = CZ[i];
    w[i] = W(i);
  }
}

static int g_threads = 1;
void orc_set_threads(int n) { g_threads = n < 1 ? 1 : n; }
int orc_get_threads(void) { return g_threads; }

/* ---- discrete delta kernels (Sec. 2.3) --------------------------------- */
/* width 2: the two-point linear kernel the paper names; width 3: Roma, Peskin
 * and Berger (1999); width 4: Peskin (2002) standard four-point kernel. */
double orc_phi(int width, double r) {
  r = fabs(r);
  if (width == 2) return r < 1.0 ? 1.0 - r : 0.0;
  if (width == 3) {
    if (r <= 0.5) return (1.0 + sqrt(1.0 - 3.0 * r * r)) / 3.0;
    if (r <= 1.5) return (5.0 - 3.0 * r - sqrt(1.0 - 3.0 * (1.0 - r) * (1.0 - r))) / 6.0;
    return 0.0;
  }
  if (width == 4) {
    if (r <= 1.0) return (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r)) / 8.0;
    if (r <= 2.0) return (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) / 8.0;
    return 0.0;
  }
  return 0.0;
}

static int wrap(long i, int n) {
  if (i >= 0 && i < n) return (int)i;
  long m = i % n;
  return (int)(m < 0 ? m + n : m);
}

/* every node within distance 2 of r along each axis: floor(r)-2 .. floor(r)+3 */
void orc_spread(int nx, int ny, int nz, int width, int m, const double* r,
                const double* f, double* F) {
  long N = (long)nx * ny * nz;
  for (int p = 0; p < m; ++p) {
    const double* rp = r + 3 * p;
    long bx = (long)floor(rp[0]) - 2, by = (long)floor(rp[1]) - 2,
         bz = (long)floor(rp[2]) - 2;
    for (long k = bz; k <= bz + 5; ++k) {
      double wz = orc_phi(width, (double)k - rp[2]);
      if (wz == 0.0) continue;
      for (long j = by; j <= by + 5; ++j) {
        double wy = orc_phi(width, (double)j - rp[1]);
        if (wy == 0.0) continue;
        for (long i = bx; i <= bx + 5; ++i) {
          double wx = orc_phi(width, (double)i - rp[0]);
          if (wx == 0.0) continue;
          double d = wx * wy * wz;
          long n = ((long)wrap(k, nz) * ny + wrap(j, ny)) * nx + wrap(i, nx);
          F[n] += d * f[3 * p];
          F[N + n] += d * f[3 * p + 1];
          F[2 * N + n] += d * f[3 * p + 2];
        }
      }
    }
  }
}

void orc_interp(int nx, int ny, int nz, int width, int m, const double* r,
                const double* u, double* U) {
  long N = (long)nx * ny * nz;
#pragma omp parallel for num_threads(g_threads) schedule(static)
  for (int p = 0; p < m; ++p) {
    const double* rp = r + 3 * p;
    long bx = (long)floor(rp[0]) - 2, by = (long)floor(rp[1]) - 2,
         bz = (long)floor(rp[2]) - 2;
    double s0 = 0, s1 = 0, s2 = 0;
    for (long k = bz; k <= bz + 5; ++k) {
      double wz = orc_phi(width, (double)k - rp[2]);
      if (wz == 0.0) continue;
      for (long j = by; j <= by + 5; ++j) {
        double wy = orc_phi(width, (double)j - rp[1]);
        if (wy == 0.0) continue;
        for (long i = bx; i <= bx + 5; ++i) {
          double wx = orc_phi(width, (double)i - rp[0]);
          if (wx == 0.0) continue;
          double d = wx * wy * wz;
          long n = ((long)wrap(k, nz) * ny + wrap(j, ny)) * nx + wrap(i, nx);
          s0 += d * u[n];
          s1 += d * u[N + n];
          s2 += d * u[2 * N + n];
        }
      }
    }
    U[3 * p] = s0;
    U[3 * p + 1] = s1;
    U[3 * p + 2] = s2;
  }
}

/* ---- simulation state ----------------------------------------------------- */
typedef struct {
  orc_mesh mesh;
  int first; /* index of the bead's first marker */
  double ks, C, kb, kv;
  double fext[3]; /* constant external force on the whole bead (test mode) */
} orc_bead;

typedef struct {
  int bead[3];
  double k[2], L0[2];
  double A, B, T, alpha, phi0;
} orc_swimmer;

struct orc_sim {
  int nx, ny, nz;
  long N;
  double tau;
  int forcing, width, walls_y;
  double g[3];
  double *f, *fs, *F, *u, *rho;
  long time;
  int nm, cap;
  double *r, *fm, *U, *fpoint; /* markers: position, total force, velocity */
  int* owner;                  /* bead of a marker, or -1 for a free point */
  int nb, ns;
  orc_bead* beads;
  orc_swimmer* sw;
  double* R; /* bead centres, 3 per bead */
};

orc_sim* orc_new(int nx, int ny, int nz, double tau, int forcing, int width) {
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  s->nx = nx;
  s->ny = ny;
  s->nz = nz;
  s->N = (long)nx * ny * nz;
  s->tau = tau;
  s->forcing = forcing;
  s->width = width;
  s->f = (double*)malloc(sizeof(double) * 19 * s->N);
  s->fs = (double*)malloc(sizeof(double) * 19 * s->N);
  s->F = (double*)calloc(3 * s->N, sizeof(double));
  s->u = (double*)calloc(3 * s->N, sizeof(double));
  s->rho = (double*)malloc(sizeof(double) * s->N);
  for (int i = 0; i < 19; ++i)
    for (long n = 0; n < s->N; ++n) s->f[i * s->N + n] = W(i);
  for (long n = 0; n < s->N; ++n) s->rho[n] = 1.0;
  return s;
}

void orc_free(orc_sim* s) {
  if (!s) return;
  free(s->f);
  free(s->fs);
  free(s->F);
  free(s->u);
  free(s->rho);
  free(s->r);
  free(s->fm);
  free(s->U);
  free(s->fpoint);
  free(s->owner);
  for (int b = 0; b < s->nb; ++b) orc_mesh_free(&s->beads[b].mesh);
  free(s->beads);
  free(s->sw);
  free(s->R);
  free(s);
}

void orc_set_walls_y(orc_sim* s, int on) { s->walls_y = on; }
void orc_set_body_force(orc_sim* s, const double g[3]) {
  s->g[0] = g[0];
  s->g[1] = g[1];
  s->g[2] = g[2];
}
void orc_set_deviation(orc_sim* s, const double* dev) {
  for (int i = 0; i < 19; ++i)
    for (long n = 0; n < s->N; ++n) s->f[i * s->N + n] = W(i) + dev[i * s->N + n];
}
void orc_get_pops(const orc_sim* s, double* f) {
  memcpy(f, s->f, sizeof(double) * 19 * s->N);
}

static void grow_markers(orc_sim* s, int add) {
  int need = s->nm + add;
  if (need <= s->cap) return;
  int cap = need * 2;
  s->r = (double*)realloc(s->r, sizeof(double) * 3 * cap);
  s->fm = (double*)realloc(s->fm, sizeof(double) * 3 * cap);
  s->U = (double*)realloc(s->U, sizeof(double) * 3 * cap);
  s->fpoint = (double*)realloc(s->fpoint, sizeof(double) * 3 * cap);
  s->owner = (int*)realloc(s->owner, sizeof(int) * cap);
  s->cap = cap;
}

int orc_add_swimmer(orc_sim* s, const double centres[9], const double radius[3],
                    int level, double ks, double C, double kb, double kv,
                    const double k[2], const double L0[2], double A, double B,
                    double T, double alpha, double phi0) {
  int nv, nt;
  orc_icosphere_counts(level, &nv, &nt);
  s->beads = (orc_bead*)realloc(s->beads, sizeof(orc_bead) * (s->nb + 3));
  s->R = (double*)realloc(s->R, sizeof(double) * 3 * (s->nb + 3));
  s->sw = (orc_swimmer*)realloc(s->sw, sizeof(orc_swimmer) * (s->ns + 1));
  orc_swimmer* w = &s->sw[s->ns];
  double* v = (double*)malloc(sizeof(double) * 3 * nv);
  int* t = (int*)malloc(sizeof(int) * 3 * nt);
  for (int b = 0; b < 3; ++b) {
    orc_icosphere(level, radius[b], centres + 3 * b, v, t);
    orc_bead* bd = &s->beads[s->nb];
    orc_mesh_build(&bd->mesh, nv, nt, t, v);
    bd->ks = ks;
    bd->fext[0] = bd->fext[1] = bd->fext[2] = 0.0;
    bd->C = C;
    bd->kb = kb;
    bd->kv = kv;
    grow_markers(s, nv);
    bd->first = s->nm;
    for (int i = 0; i < nv; ++i) {
      for (int q = 0; q < 3; ++q) {
        s->r[3 * (s->nm + i) + q] = v[3 * i + q];
        s->fm[3 * (s->nm + i) + q] = 0;
        s->U[3 * (s->nm + i) + q] = 0;
        s->fpoint[3 * (s->nm + i) + q] = 0;
      }
      s->owner[s->nm + i] = s->nb;
    }
    s->nm += nv;
    w->bead[b] = s->nb;
    s->nb += 1;
  }
  free(v);
  free(t);
  w->k[0] = k[0];
  w->k[1] = k[1];
  w->L0[0] = L0[0];
  w->L0[1] = L0[1];
  w->A = A;
  w->B = B;
  w->T = T;
  w->alpha = alpha;
  w->phi0 = phi0;
  return s->ns++;
}

int orc_add_bead(orc_sim* s, const double centre[3], double radius, int level,
                 double ks, double C, double kb, double kv, const double force[3]) {
  int nv, nt;
  orc_icosphere_counts(level, &nv, &nt);
  s->beads = (orc_bead*)realloc(s->beads, sizeof(orc_bead) * (s->nb + 1));
  s->R = (double*)realloc(s->R, sizeof(double) * 3 * (s->nb + 1));
  double* v = (double*)malloc(sizeof(double) * 3 * nv);
  int* t = (int*)malloc(sizeof(int) * 3 * nt);
  orc_icosphere(level, radius, centre, v, t);
  orc_bead* bd = &s->beads[s->nb];
  orc_mesh_build(&bd->mesh, nv, nt, t, v);
  bd->ks = ks;
  bd->C = C;
  bd->kb = kb;
  bd->kv = kv;
  for (int q = 0; q < 3; ++q) bd->fext[q] = force[q];
  grow_markers(s, nv);
  bd->first = s->nm;
  for (int i = 0; i < nv; ++i) {
    for (int q = 0; q < 3; ++q) {
      s->r[3 * (s->nm + i) + q] = v[3 * i + q];
      s->fm[3 * (s->nm + i) + q] = 0;
      s->U[3 * (s->nm + i) + q] = 0;
      s->fpoint[3 * (s->nm + i) + q] = 0;
    }
    s->owner[s->nm + i] = s->nb;
  }
  s->nm += nv;
  free(v);
  free(t);
  return s->nb++;
}

int orc_add_points(orc_sim* s, int m, const double* r, const double* f) {
  grow_markers(s, m);
  for (int i = 0; i < m; ++i) {
    for (int q = 0; q < 3; ++q) {
      s->r[3 * (s->nm + i) + q] = r[3 * i + q];
      s->fpoint[3 * (s->nm + i) + q] = f[3 * i + q];
      s->fm[3 * (s->nm + i) + q] = 0;
      s->U[3 * (s->nm + i) + q] = 0;
    }
    s->owner[s->nm + i] = -1;
  }
  s->nm += m;
  return 0;
}

/* O1 */
static void bead_centres(orc_sim* s) {
  for (int b = 0; b < s->nb; ++b) {
    const orc_bead* bd = &s->beads[b];
    double c[3] = {0, 0, 0};
    for (int i = 0; i < bd->mesh.nv; ++i)
      for (int q = 0; q < 3; ++q) c[q] += s->r[3 * (bd->first + i) + q];
    for (int q = 0; q < 3; ++q) s->R[3 * b + q] = c[q] / bd->mesh.nv;
  }
}

/* O2-O5 */
static void marker_forces(orc_sim* s) {
  for (int m = 0; m < s->nm; ++m)
    for (int q = 0; q < 3; ++q) s->fm[3 * m + q] = s->fpoint[3 * m + q];
  for (int b = 0; b < s->nb; ++b) {
    const orc_bead* bd = &s->beads[b];
    orc_mesh_forces(&bd->mesh, s->r + 3 * bd->first, bd->ks, bd->C, bd->kb, bd->kv,
                    NULL, s->fm + 3 * bd->first);
    for (int i = 0; i < bd->mesh.nv; ++i)
      for (int q = 0; q < 3; ++q) s->fm[3 * (bd->first + i) + q] += bd->fext[q] / bd->mesh.nv;
  }
  for (int w = 0; w < s->ns; ++w) {
    const orc_swimmer* sw = &s->sw[w];
    double fb[3][3] = {{0}};
    double om = 2.0 * M_PI / sw->T, t = (double)s->time;
    double f1 = sw->A * sin(om * t + sw->phi0);
    double f3 = sw->B * sin(om * t + sw->phi0 + sw->alpha);
    fb[0][0] += f1;
    fb[2][0] += f3;
    fb[1][0] += -f1 - f3;
    const double* R2 = s->R + 3 * sw->bead[1];
    for (int sp = 0; sp < 2; ++sp) {
      int outer = sp == 0 ? 0 : 2;
      const double* Ro = s->R + 3 * sw->bead[outer];
      double d[3] = {Ro[0] - R2[0], Ro[1] - R2[1], Ro[2] - R2[2]};
      double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
      for (int q = 0; q < 3; ++q) {
        double fs = -sw->k[sp] * (len - sw->L0[sp]) * d[q] / len;
        fb[outer][q] += fs;
        fb[1][q] -= fs;
      }
    }
    for (int bi = 0; bi < 3; ++bi) {
      const orc_bead* bd = &s->beads[sw->bead[bi]];
      for (int i = 0; i < bd->mesh.nv; ++i)
        for (int q = 0; q < 3; ++q)
          s->fm[3 * (bd->first + i) + q] += fb[bi][q] / bd->mesh.nv;
    }
  }
}

/* O7: pull streaming on the periodic box; with walls_y the planes y=-1/2 and
 * y=ny-1/2 reflect populations (half-way bounce-back, test mode only) */
static void stream(orc_sim* s) {
  const int nx = s->nx, ny = s->ny, nz = s->nz;
  const long N = s->N;
  for (int i = 0; i < 19; ++i) {
#pragma omp parallel for num_threads(g_threads) schedule(static)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y) {
        int ys = y - CY[i];
        int zs = wrap(z - CZ[i], nz);
        for (int x = 0; x < nx; ++x) {
          long n = ((long)z * ny + y) * nx + x;
          if (s->walls_y && (ys < 0 || ys >= ny)) {
            s->fs[i * N + n] = s->f[OPP(i) * N + n];
            continue;
          }
          long src = ((long)zs * ny + wrap(ys, ny)) * nx + wrap(x - CX[i], nx);
          s->fs[i * N + n] = s->f[i * N + src];
        }
      }
  }
}

/* O8 + O9 */
static void collide(orc_sim* s) {
  const long N = s->N;
  const double tau = s->tau;
#pragma omp parallel for num_threads(g_threads) schedule(static)
  for (long n = 0; n < N; ++n) {
    double rho = 0, j[3] = {0, 0, 0};
    for (int i = 0; i < 19; ++i) {
      double fi = s->fs[i * N + n];
      rho += fi;
      j[0] += fi * CX[i];
      j[1] += fi * CY[i];
      j[2] += fi * CZ[i];
    }
    double F[3] = {s->F[n] + s->g[0], s->F[N + n] + s->g[1], s->F[2 * N + n] + s->g[2]};
    double u[3], ue[3];
    for (int q = 0; q < 3; ++q) {
      u[q] = (j[q] + 0.5 * F[q]) / rho;
      ue[q] = s->forcing == ORC_GUO ? u[q] : (j[q] + tau * F[q]) / rho;
    }
    s->rho[n] = rho;
    s->u[n] = u[0];
    s->u[N + n] = u[1];
    s->u[2 * N + n] = u[2];
    double uu = ue[0] * ue[0] + ue[1] * ue[1] + ue[2] * ue[2];
    for (int i = 0; i < 19; ++i) {
      double cu = CX[i] * ue[0] + CY[i] * ue[1] + CZ[i] * ue[2];
      double feq = W(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      double fi = s->fs[i * N + n];
      double out = fi - (fi - feq) / tau;
      if (s->forcing == ORC_GUO) {
        double cuv = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        double src = 0;
        double c[3] = {(double)CX[i], (double)CY[i], (double)CZ[i]};
        for (int q = 0; q < 3; ++q) src += (3.0 * (c[q] - u[q]) + 9.0 * cuv * c[q]) * F[q];
        out += (1.0 - 0.5 / tau) * W(i) * src;
      }
      s->f[i * N + n] = out;
    }
  }
}

void orc_step(orc_sim* s, long nsteps) {
  for (long it = 0; it < nsteps; ++it) {
    bead_centres(s);                                           /* O1 */
    marker_forces(s);                                          /* O2-O5 */
    memset(s->F, 0, sizeof(double) * 3 * s->N);
    orc_spread(s->nx, s->ny, s->nz, s->width, s->nm, s->r, s->fm, s->F); /* O6 */
    stream(s);                                                 /* O7 */
    collide(s);                                                /* O8, O9 */
    orc_interp(s->nx, s->ny, s->nz, s->width, s->nm, s->r, s->u, s->U); /* O10 */
    for (int m = 0; m < s->nm; ++m)                            /* O11 */
      for (int q = 0; q < 3; ++q) s->r[3 * m + q] += s->U[3 * m + q];
    s->time += 1;                                              /* O12 */
  }
  bead_centres(s);
}

long orc_time(const orc_sim* s) { return s->time; }
int orc_n_markers(const orc_sim* s) { return s->nm; }
int orc_n_beads(const orc_sim* s) { return s->nb; }
int orc_n_swimmers(const orc_sim* s) { return s->ns; }
void orc_get_markers(const orc_sim* s, double* r) {
  memcpy(r, s->r, sizeof(double) * 3 * s->nm);
}
void orc_get_marker_forces(const orc_sim* s, double* f) {
  memcpy(f, s->fm, sizeof(double) * 3 * s->nm);
}
void orc_get_marker_velocities(const orc_sim* s, double* U) {
  memcpy(U, s->U, sizeof(double) * 3 * s->nm);
}
void orc_get_bead_centres(const orc_sim* s, double* R) {
  for (int b = 0; b < s->nb; ++b) {
    const orc_bead* bd = &s->beads[b];
    double c[3] = {0, 0, 0};
    for (int i = 0; i < bd->mesh.nv; ++i)
      for (int q = 0; q < 3; ++q) c[q] += s->r[3 * (bd->first + i) + q];
    for (int q = 0; q < 3; ++q) R[3 * b + q] = c[q] / bd->mesh.nv;
  }
}
/* swimmer centre x_cm = 1/3 sum of its three bead centres (Eq. vel_swim) */
void orc_get_swimmer_centres(const orc_sim* s, double* X) {
  double* R = (double*)malloc(sizeof(double) * 3 * (s->nb > 0 ? s->nb : 1));
  orc_get_bead_centres(s, R);
  for (int w = 0; w < s->ns; ++w)
    for (int q = 0; q < 3; ++q)
      X[3 * w + q] = (R[3 * s->sw[w].bead[0] + q] + R[3 * s->sw[w].bead[1] + q] +
                      R[3 * s->sw[w].bead[2] + q]) / 3.0;
  free(R);
}
void orc_get_velocity(const orc_sim* s, double* u) {
  memcpy(u, s->u, sizeof(double) * 3 * s->N);
}
void orc_get_density(const orc_sim* s, double* rho) {
  memcpy(rho, s->rho, sizeof(double) * s->N);
}
void orc_get_force(const orc_sim* s, double* F) {
  memcpy(F, s->F, sizeof(double) * 3 * s->N);
}
void orc_conserved(const orc_sim* s, double out[4]) {
  double M = 0, P[3] = {0, 0, 0};
  for (int i = 0; i < 19; ++i)
    for (long n = 0; n < s->N; ++n) {
      double fi = s->f[i * s->N + n];
      M += fi;
      P[0] += fi * CX[i];
      P[1] += fi * CY[i];
      P[2] += fi * CZ[i];
    }
  out[0] = M;
  out[1] = P[0];
  out[2] = P[1];
  out[3] = P[2];
}
