/*
 * Oracle: bead meshes and membrane mechanics (paper Sec. 2.2).
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 *   - Icosphere: an icosahedron refined recursively (Sec. 2.2); each level
 *     splits every triangle in four at the edge midpoints and projects the new
 *     vertices onto the sphere.
 *   - Skalak strain energy with linear (constant-strain) triangles, Sec. 2.2:
 *     W_sk = ks/4 * sum_tri A0 [I1^2 + 2 I1 - 2 I2 + C I2^2], with
 *     I1 = l1^2 + l2^2 - 2 = tr(G0^-1 g) - 2 and I2 = l1^2 l2^2 - 1 =
 *     det g / det G0 - 1, where g and G0 are the current and reference metric
 *     tensors of the triangle's edge vectors (area measured on the reference
 *     triangle).
 *   - Helfrich bending discretised after Kantor and Nelson: W_b = kt * sum over
 *     edges [1 - cos(theta - theta0)] with kt = 2 kb / sqrt(3), theta the
 *     dihedral angle between the two face normals and theta0 its stress-free
 *     value.  The Gaussian-curvature term is a topological constant on a closed
 *     surface and exerts no force.
 *   - Volume penalty, Eq. (vol_cons): W_v = kv/2 (V - V0)^2 / V0.
 *   - Nodal forces by virtual work: f = -dW/dr (Sec. 2.2).
 */
#include "orc_internal.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* golden-ratio icosahedron: vertices are cyclic permutations of (0,+-1,+-phi),
 * faces listed counter-clockwise seen from outside */
static const double ICO_P = 1.6180339887498948482;
static const int ICO_F[20][3] = {
    {0, 11, 5}, {0, 5, 1},  {0, 1, 7},   {0, 7, 10}, {0, 10, 11},
    {1, 5, 9},  {5, 11, 4}, {11, 10, 2}, {10, 7, 6}, {7, 1, 8},
    {3, 9, 4},  {3, 4, 2},  {3, 2, 6},   {3, 6, 8},  {3, 8, 9},
    {4, 9, 5},  {2, 4, 11}, {6, 2, 10},  {8, 6, 7},  {9, 8, 1}};

int orc_icosphere_counts(int level, int* nv, int* ntri) {
  int p = 1;
  for (int i = 0; i < level; ++i) p *= 4;
  *nv = 10 * p + 2;
  *ntri = 20 * p;
  return 0;
}

static void normalise(double* v) {
  double len = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  v[0] = v[0] / len;
  v[1] = v[1] / len;
  v[2] = v[2] / len;
}

/* look up or create the midpoint vertex of edge (a,b) */
static int edge_mid(int a, int b, int* keys_a, int* keys_b, int* vals, int cap,
                    double* v, int* nv) {
  int lo = a < b ? a : b, hi = a < b ? b : a;
  unsigned h = ((unsigned)lo * 73856093u) ^ ((unsigned)hi * 19349663u);
  int slot = (int)(h % (unsigned)cap);
  for (;;) {
    if (keys_a[slot] < 0) break;
    if (keys_a[slot] == lo && keys_b[slot] == hi) return vals[slot];
    slot = (slot + 1) % cap;
  }
  int id = (*nv)++;
  double* m = v + 3 * id;
  for (int k = 0; k < 3; ++k) m[k] = (v[3 * a + k] + v[3 * b + k]) * 0.5;
  normalise(m);
  keys_a[slot] = lo;
  keys_b[slot] = hi;
  vals[slot] = id;
  return id;
}

int orc_icosphere(int level, double radius, const double centre[3],
                  double* verts, int* tris) {
  int nvt, ntt;
  orc_icosphere_counts(level, &nvt, &ntt);
  double* v = (double*)malloc(sizeof(double) * 3 * nvt);
  int* t = (int*)malloc(sizeof(int) * 3 * ntt);
  int* t2 = (int*)malloc(sizeof(int) * 3 * ntt);
  const double base[12][3] = {
      {-1, ICO_P, 0}, {1, ICO_P, 0}, {-1, -ICO_P, 0}, {1, -ICO_P, 0},
      {0, -1, ICO_P}, {0, 1, ICO_P}, {0, -1, -ICO_P}, {0, 1, -ICO_P},
      {ICO_P, 0, -1}, {ICO_P, 0, 1}, {-ICO_P, 0, -1}, {-ICO_P, 0, 1}};
  int nv = 12, nt = 20;
  for (int i = 0; i < 12; ++i) {
    for (int k = 0; k < 3; ++k) v[3 * i + k] = base[i][k];
    normalise(v + 3 * i);
  }
  for (int i = 0; i < 20; ++i)
    for (int k = 0; k < 3; ++k) t[3 * i + k] = ICO_F[i][k];
  for (int l = 0; l < level; ++l) {
    int cap = 4 * (3 * nt / 2) + 7;
    int* ka = (int*)malloc(sizeof(int) * cap);
    int* kb = (int*)malloc(sizeof(int) * cap);
    int* kv = (int*)malloc(sizeof(int) * cap);
    for (int i = 0; i < cap; ++i) ka[i] = -1;
    int nt2 = 0;
    for (int f = 0; f < nt; ++f) {
      int a = t[3 * f], b = t[3 * f + 1], c = t[3 * f + 2];
      int ab = edge_mid(a, b, ka, kb, kv, cap, v, &nv);
      int bc = edge_mid(b, c, ka, kb, kv, cap, v, &nv);
      int ca = edge_mid(c, a, ka, kb, kv, cap, v, &nv);
      int nf[4][3] = {{a, ab, ca}, {b, bc, ab}, {c, ca, bc}, {ab, bc, ca}};
      for (int q = 0; q < 4; ++q)
        for (int k = 0; k < 3; ++k) t2[3 * nt2 + 3 * q + k] = nf[q][k];
      nt2 += 4;
    }
    free(ka);
    free(kb);
    free(kv);
    nt = nt2;
    int* sw = t;
    t = t2;
    t2 = sw;
  }
  for (int i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) verts[3 * i + k] = centre[k] + radius * v[3 * i + k];
  memcpy(tris, t, sizeof(int) * 3 * nt);
  free(v);
  free(t);
  free(t2);
  return nv;
}

/* ---- small vector helpers ------------------------------------------------ */
static void sub3(const double* a, const double* b, double* o) {
  o[0] = a[0] - b[0];
  o[1] = a[1] - b[1];
  o[2] = a[2] - b[2];
}
static double dot3(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void cross3(const double* a, const double* b, double* o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* ---- reference geometry ---------------------------------------------------- */
/* hinge (x1,x2 shared edge; x3 opposite in the face holding the directed edge
 * x1->x2; x4 opposite in the face holding x2->x1) */
static double dihedral(const double* x1, const double* x2, const double* x3,
                       const double* x4) {
  double e[3], a[3], b[3], nA[3], nB[3], c[3];
  sub3(x2, x1, e);
  sub3(x3, x1, a);
  cross3(e, a, nA); /* (x2-x1) x (x3-x1) */
  double m[3], d[3];
  sub3(x1, x2, m);
  sub3(x4, x2, d);
  cross3(m, d, nB); /* (x1-x2) x (x4-x2) */
  double la = sqrt(dot3(nA, nA)), lb = sqrt(dot3(nB, nB)), le = sqrt(dot3(e, e));
  for (int k = 0; k < 3; ++k) {
    nA[k] /= la;
    nB[k] /= lb;
    b[k] = e[k] / le;
  }
  cross3(nA, nB, c);
  return atan2(dot3(c, b), dot3(nA, nB));
}

void orc_mesh_build(orc_mesh* M, int nv, int ntri, const int* tris,
                    const double* xref) {
  M->nv = nv;
  M->ntri = ntri;
  M->tris = (int*)malloc(sizeof(int) * 3 * ntri);
  memcpy(M->tris, tris, sizeof(int) * 3 * ntri);
  M->G0inv = (double*)malloc(sizeof(double) * 3 * ntri);
  M->detG0 = (double*)malloc(sizeof(double) * ntri);
  M->A0 = (double*)malloc(sizeof(double) * ntri);
  for (int t = 0; t < ntri; ++t) {
    const double* X0 = xref + 3 * tris[3 * t];
    const double* X1 = xref + 3 * tris[3 * t + 1];
    const double* X2 = xref + 3 * tris[3 * t + 2];
    double E1[3], E2[3];
    sub3(X1, X0, E1);
    sub3(X2, X0, E2);
    double g11 = dot3(E1, E1), g12 = dot3(E1, E2), g22 = dot3(E2, E2);
    double det = g11 * g22 - g12 * g12;
    M->detG0[t] = det;
    M->G0inv[3 * t + 0] = g22 / det;
    M->G0inv[3 * t + 1] = -g12 / det;
    M->G0inv[3 * t + 2] = g11 / det;
    M->A0[t] = 0.5 * sqrt(det);
  }
  /* hinges: one per undirected edge, taken from the face that holds it as
   * lo->hi */
  int nh = 3 * ntri / 2;
  M->nh = nh;
  M->hinge = (int*)malloc(sizeof(int) * 4 * nh);
  M->theta0 = (double*)malloc(sizeof(double) * nh);
  int h = 0;
  for (int f = 0; f < ntri; ++f) {
    for (int q = 0; q < 3; ++q) {
      int a = tris[3 * f + q], b = tris[3 * f + (q + 1) % 3];
      int c = tris[3 * f + (q + 2) % 3];
      if (a > b) continue;
      int d = -1;
      for (int g = 0; g < ntri && d < 0; ++g) {
        for (int p = 0; p < 3; ++p) {
          if (tris[3 * g + p] == b && tris[3 * g + (p + 1) % 3] == a) {
            d = tris[3 * g + (p + 2) % 3];
            break;
          }
        }
      }
      M->hinge[4 * h + 0] = a;
      M->hinge[4 * h + 1] = b;
      M->hinge[4 * h + 2] = c;
      M->hinge[4 * h + 3] = d;
      M->theta0[h] = dihedral(xref + 3 * a, xref + 3 * b, xref + 3 * c, xref + 3 * d);
      ++h;
    }
  }
  M->V0 = orc_mesh_volume(M, xref);
}

void orc_mesh_free(orc_mesh* M) {
  free(M->tris);
  free(M->G0inv);
  free(M->detG0);
  free(M->A0);
  free(M->hinge);
  free(M->theta0);
  memset(M, 0, sizeof(*M));
}

/* V = 1/6 sum over triangles of (x0-c).((x1-c) x (x2-c)), c = vertex mean */
double orc_mesh_volume(const orc_mesh* M, const double* x) {
  double c[3] = {0, 0, 0};
  for (int i = 0; i < M->nv; ++i)
    for (int k = 0; k < 3; ++k) c[k] += x[3 * i + k];
  for (int k = 0; k < 3; ++k) c[k] /= M->nv;
  double V = 0;
  for (int t = 0; t < M->ntri; ++t) {
    double a[3], b[3], d[3], cr[3];
    sub3(x + 3 * M->tris[3 * t], c, a);
    sub3(x + 3 * M->tris[3 * t + 1], c, b);
    sub3(x + 3 * M->tris[3 * t + 2], c, d);
    cross3(b, d, cr);
    V += dot3(a, cr);
  }
  return V / 6.0;
}

/* energies and nodal forces f = -dW/dx, accumulated into force[] */
void orc_mesh_forces(const orc_mesh* M, const double* x, double ks, double C,
                     double kb, double kv, double* energy, double* force) {
  double Wsk = 0, Wb = 0, Wv = 0;
  /* Skalak */
  for (int t = 0; t < M->ntri; ++t) {
    int i0 = M->tris[3 * t], i1 = M->tris[3 * t + 1], i2 = M->tris[3 * t + 2];
    double e1[3], e2[3];
    sub3(x + 3 * i1, x + 3 * i0, e1);
    sub3(x + 3 * i2, x + 3 * i0, e2);
    double g11 = dot3(e1, e1), g12 = dot3(e1, e2), g22 = dot3(e2, e2);
    const double* Gi = M->G0inv + 3 * t;
    double I1 = Gi[0] * g11 + 2.0 * Gi[1] * g12 + Gi[2] * g22 - 2.0;
    double detg = g11 * g22 - g12 * g12;
    double J = detg / M->detG0[t];
    double I2 = J - 1.0;
    double A0 = M->A0[t];
    Wsk += ks / 4.0 * A0 * (I1 * I1 + 2.0 * I1 - 2.0 * I2 + C * I2 * I2);
    double dW1 = ks / 4.0 * A0 * (2.0 * I1 + 2.0);
    double dW2 = ks / 4.0 * A0 * (-2.0 + 2.0 * C * I2);
    /* P = dW/dg = dW1 * G0^-1 + dW2 * J * g^-1, g^-1 = adj(g)/det g */
    double P11 = dW1 * Gi[0] + dW2 * g22 / M->detG0[t];
    double P12 = dW1 * Gi[1] - dW2 * g12 / M->detG0[t];
    double P22 = dW1 * Gi[2] + dW2 * g11 / M->detG0[t];
    for (int k = 0; k < 3; ++k) {
      double dWde1 = 2.0 * (P11 * e1[k] + P12 * e2[k]);
      double dWde2 = 2.0 * (P12 * e1[k] + P22 * e2[k]);
      force[3 * i1 + k] -= dWde1;
      force[3 * i2 + k] -= dWde2;
      force[3 * i0 + k] += dWde1 + dWde2;
    }
  }
  /* bending */
  double kt = 2.0 * kb / sqrt(3.0);
  for (int h = 0; h < M->nh; ++h) {
    const int* q = M->hinge + 4 * h;
    const double *x1 = x + 3 * q[0], *x2 = x + 3 * q[1], *x3 = x + 3 * q[2],
                 *x4 = x + 3 * q[3];
    double th = dihedral(x1, x2, x3, x4);
    double dth = th - M->theta0[h];
    Wb += kt * (1.0 - cos(dth));
    double dWdth = kt * sin(dth);
    double e[3], a[3], nA[3], m[3], d[3], nB[3];
    sub3(x2, x1, e);
    sub3(x3, x1, a);
    cross3(e, a, nA);
    sub3(x1, x2, m);
    sub3(x4, x2, d);
    cross3(m, d, nB);
    double E = sqrt(dot3(e, e));
    double eh[3] = {e[0] / E, e[1] / E, e[2] / E};
    double nA2 = dot3(nA, nA), nB2 = dot3(nB, nB);
    double t32[3], t13[3], t24[3], t41[3];
    sub3(x3, x2, t32);
    sub3(x1, x3, t13);
    sub3(x2, x4, t24);
    sub3(x4, x1, t41);
    double s32 = dot3(t32, eh), s13 = dot3(t13, eh), s24 = dot3(t24, eh),
           s41 = dot3(t41, eh);
    for (int k = 0; k < 3; ++k) {
      double a_k = nA[k] / nA2, b_k = nB[k] / nB2;
      double g1 = -s32 * a_k + s24 * b_k;
      double g2 = -s13 * a_k + s41 * b_k;
      double g3 = -E * a_k;
      double g4 = -E * b_k;
      force[3 * q[0] + k] -= dWdth * g1;
      force[3 * q[1] + k] -= dWdth * g2;
      force[3 * q[2] + k] -= dWdth * g3;
      force[3 * q[3] + k] -= dWdth * g4;
    }
  }
  /* volume */
  double V = orc_mesh_volume(M, x);
  Wv = 0.5 * kv * (V - M->V0) * (V - M->V0) / M->V0;
  double pref = kv * (V - M->V0) / M->V0;
  double c[3] = {0, 0, 0};
  for (int i = 0; i < M->nv; ++i)
    for (int k = 0; k < 3; ++k) c[k] += x[3 * i + k];
  for (int k = 0; k < 3; ++k) c[k] /= M->nv;
  for (int t = 0; t < M->ntri; ++t) {
    int i0 = M->tris[3 * t], i1 = M->tris[3 * t + 1], i2 = M->tris[3 * t + 2];
    double a[3], b[3], d[3], g0[3], g1[3], g2[3];
    sub3(x + 3 * i0, c, a);
    sub3(x + 3 * i1, c, b);
    sub3(x + 3 * i2, c, d);
    cross3(b, d, g0);
    cross3(d, a, g1);
    cross3(a, b, g2);
    for (int k = 0; k < 3; ++k) {
      force[3 * i0 + k] -= pref * g0[k] / 6.0;
      force[3 * i1 + k] -= pref * g1[k] / 6.0;
      force[3 * i2 + k] -= pref * g2[k] / 6.0;
    }
  }
  if (energy) {
    energy[0] = Wsk;
    energy[1] = Wb;
    energy[2] = Wv;
  }
}

void orc_membrane_eval(int nv, int ntri, const int* tris, const double* xref,
                       const double* x, double ks, double C, double kb,
                       double kv, double* energy, double* force) {
  orc_mesh M;
  orc_mesh_build(&M, nv, ntri, tris, xref);
  memset(force, 0, sizeof(double) * 3 * nv);
  orc_mesh_forces(&M, x, ks, C, kb, kv, energy, force);
  orc_mesh_free(&M);
}
