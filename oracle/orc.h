/*
 * FP64 CPU oracle for the lattice Boltzmann + immersed boundary + finite
 * element bead-spring swimmer method of Geyer et al., "Lattice Boltzmann
 * Simulations of Two Linear Microswimmers Using the Immersed Boundary Method"
 * (arXiv 2202.12147).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that the tests, the smoke
 * check and the CPU-baseline leg of the benchmark have an independent,
 * obviously correct reference.  The product (the HIP library) never links,
 * loads or calls it, and it shares no code, header, table or helper with the
 * product.  Plain loops, unfused, FP64 everywhere, unshifted populations,
 * marker positions stored absolute and unwrapped.
 *
 * Conventions (readings of the paper where it is silent):
 *   - D3Q19, index 0 = rest, 1..6 = +x,-x,+y,-y,+z,-z, 7..18 = the twelve
 *     edge directions with opposite pairs adjacent (Sec. 2.1 gives only the
 *     weights 1/3, 1/18, 1/36).
 *   - Arrays of lattice fields are [component][z][y][x], x fastest.
 *   - Node (i,j,k) sits at integer coordinates (i,j,k); markers use the same
 *     units.
 */
#ifndef ORC_H
#define ORC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_GUO = 0, ORC_SHAN_CHEN = 1 };

typedef struct orc_sim orc_sim;

/* ---- pure functions (pins) ------------------------------------------- */
double orc_phi(int width, double r);                       /* 1-D delta kernel */
void orc_lattice(int* cx, int* cy, int* cz, double* w);    /* velocity set, 19 each */
int orc_icosphere(int level, double radius, const double centre[3],
                  double* verts, int* tris);               /* returns nv; arrays sized by caller */
int orc_icosphere_counts(int level, int* nv, int* ntri);
/* membrane energy and forces of one closed mesh: reference geometry from
 * xref, evaluated at x.  energy[0..2] = Skalak, bending, volume parts. */
void orc_membrane_eval(int nv, int ntri, const int* tris, const double* xref,
                       const double* x, double ks, double C, double kb,
                       double kv, double* energy, double* force);
void orc_spread(int nx, int ny, int nz, int width, int m, const double* r,
                const double* f, double* F);
void orc_interp(int nx, int ny, int nz, int width, int m, const double* r,
                const double* u, double* U);

/* ---- simulation ------------------------------------------------------- */
orc_sim* orc_new(int nx, int ny, int nz, double tau, int forcing, int width);
void orc_free(orc_sim* s);
void orc_set_walls_y(orc_sim* s, int on);
void orc_set_body_force(orc_sim* s, const double g[3]);
void orc_set_threads(int n);
int orc_get_threads(void);
/* f*_i = w_i + dev_i, dev laid out [19][z][y][x] */
void orc_set_deviation(orc_sim* s, const double* dev);
void orc_get_pops(const orc_sim* s, double* f);
int orc_add_swimmer(orc_sim* s, const double centres[9], const double radius[3],
                    int level, double ks, double C, double kb, double kv,
                    const double k[2], const double L0[2], double A, double B,
                    double T, double alpha, double phi0);
/* one bead (no swimmer) pulled by a constant total force (test mode) */
int orc_add_bead(orc_sim* s, const double centre[3], double radius, int level,
                 double ks, double C, double kb, double kv, const double force[3]);
/* free markers carrying a constant prescribed force (test mode) */
int orc_add_points(orc_sim* s, int m, const double* r, const double* f);
void orc_step(orc_sim* s, long n);
long orc_time(const orc_sim* s);
int orc_n_markers(const orc_sim* s);
int orc_n_beads(const orc_sim* s);
int orc_n_swimmers(const orc_sim* s);
void orc_get_markers(const orc_sim* s, double* r);
void orc_get_marker_forces(const orc_sim* s, double* f);
void orc_get_marker_velocities(const orc_sim* s, double* U);
void orc_get_bead_centres(const orc_sim* s, double* R);
void orc_get_swimmer_centres(const orc_sim* s, double* X);
void orc_get_velocity(const orc_sim* s, double* u);  /* u_n of the last step */
void orc_get_density(const orc_sim* s, double* rho);
void orc_get_force(const orc_sim* s, double* F);     /* F_n of the last step */
void orc_conserved(const orc_sim* s, double out[4]); /* sum f*, sum f* c */

#ifdef __cplusplus
}
#endif
#endif
