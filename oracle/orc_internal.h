/* Oracle internals.  TEST INFRASTRUCTURE ONLY (see orc.h). */
#ifndef ORC_INTERNAL_H
#define ORC_INTERNAL_H

#include "orc.h"

typedef struct {
  int nv, ntri, nh;
  int* tris;      /* 3 per triangle, counter-clockwise seen from outside */
  double* G0inv;  /* reference metric inverse (11, 12, 22) per triangle */
  double* detG0;  /* det of the reference metric */
  double* A0;     /* reference area */
  int* hinge;     /* x1, x2 (shared edge), x3, x4 (opposite vertices) */
  double* theta0; /* stress-free dihedral angle */
  double V0;      /* stress-free enclosed volume */
} orc_mesh;

void orc_mesh_build(orc_mesh* M, int nv, int ntri, const int* tris,
                    const double* xref);
void orc_mesh_free(orc_mesh* M);
double orc_mesh_volume(const orc_mesh* M, const double* x);
void orc_mesh_forces(const orc_mesh* M, const double* x, double ks, double C,
                     double kb, double kv, double* energy, double* force);

#endif
