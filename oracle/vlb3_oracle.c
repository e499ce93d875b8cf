/*
 * vlb3_oracle.c -- plain FP64 CPU oracle of the three-dimensional version
 * of the volumetric lattice Boltzmann step (arXiv 2410.23802).
 *
 * TEST INFRASTRUCTURE ONLY.  Loaded by tests/, the smoke check and the CPU
 * baseline of the benchmark.  No product code includes or links it, and it
 * shares no code with the GPU library.  Built together with vlb_oracle.c,
 * whose exact disk-cell area it uses for the cross-sections of a sphere.
 * Build with -O2 -ffp-contract=off.
 *
 * The paper develops the method in two dimensions and states that the
 * extension to three is straightforward (Sec. 2).  Readings that carry it
 * over (tagged "Reading:" at the point of use):
 *   - flow: D3Q19 with the MRT collision of eq. lbe.rho.col; the moment
 *     basis is the orthogonal D3Q19 basis of d'Humieres et al. (2002),
 *     built here from its defining polynomials; as in two dimensions (where
 *     the printed m^eq and F_m are exactly the moments of the textbook
 *     equilibrium and of Guo's force term) m^eq = M f^eq and F_m = M F;
 *     rates: the conserved moments 1, the energy-like even moments (e,
 *     epsilon, pi) 1.25 as the two-dimensional e and epsilon, the shear
 *     moments s_nu = 1/tau_f, the odd moments (q, m) by the same rule as the
 *     two-dimensional q, (1/s_nu - 1/2)(1/s_q - 1/2) = 1/12;
 *   - energy: D3Q7.  The two-dimensional energy scheme with the paper's
 *     parameters (alpha_1 = -2, alpha_2 = 1, beta_1 = -4, beta_2 = 4,
 *     sigma_q = sigma_j, sigma_epsilon = sigma_e) is a two-relaxation-time
 *     collision: equilibrium g_i^eq = w_i c_ref T (i > 0), g_0^eq = epsilon
 *     - (1 - w_0) c_ref T; odd part relaxed at sigma_j = 1/tau_g, even part
 *     at sigma_e; the source q_c enters the rest population only, as
 *     (1 - sigma_e/2) q_c.  The same collision on D3Q7 (w_0 = 1/4,
 *     w_i = 1/8, c_s^2 = 1/4), with eq. lambda read as lambda/rho_f =
 *     c_s^2 c_ref (tau_g - 1/2) and the gradient of Sec. 2.2 as
 *     grad T = -sum_i e_i g_i / (c_s^2 c_ref tau_g);
 *   - particles: spheres; V = 4 pi R^3/3, I = 2 M R^2/5 (isotropic, so the
 *     gyroscopic term vanishes); u_s = U + Omega x (x - X) (eq. us); the
 *     momentum-exchange force and torque as in Sec. 2.3 with the
 *     three-dimensional cross product; f_s is the exact volume of the
 *     sphere inside the cell;
 *   - walls, repulsion, body force, initial state, the coupled T-u solve,
 *     [df_s/dt] and the per-particle outputs as in two dimensions; where a
 *     population's upstream point lies beyond two or three walls the z
 *     wall decides, then the y wall.
 */
#include "vlb3_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 19
#define QG 7
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* disk-cell area of the two-dimensional oracle (vlb_oracle.c) */
double or_disk_cell_area(double cx, double cy, double R, double x0,
                         double y0);

/* D3Q19 velocities: rest, the six axis directions, the twelve edge
 * diagonals; D3Q7 uses the first seven. */
static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1,
                          1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1,
                          0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0,
                          1, -1, -1, 1, 1, -1, -1, 1};
static const int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9,
                           12, 11, 14, 13, 16, 15, 18, 17};
/* textbook D3Q19 weights (c_s^2 = 1/3) */
static double wflow(int q) {
  return q == 0 ? 1.0 / 3.0 : q < 7 ? 1.0 / 18.0 : 1.0 / 36.0;
}
/* Reading: D3Q7 weights of the energy lattice (c_s^2 = 1/4) */
#define W0G 0.25
#define W1G 0.125
#define CS2G 0.25
static double wg(int q) { return q == 0 ? W0G : W1G; }

struct o3_state {
  o3_domain dom;
  o3_hooks hk;
  int np, kmax;
  double *X, *Y, *Z, *U, *V, *W, *Ox, *Oy, *Oz;   /* centres, velocities */
  double *Up, *Vp, *Wp, *Oxp, *Oyp, *Ozp;        /* previous velocities */
  double *R, *rhos, *Tp0;
  int *fixed;
  double *Fx, *Fy, *Fz, *Tx, *Ty, *Tz, *Fabs;
  double *Tmean, *Tmin, *E, *fssum;
  double *f, *g, *fst, *gst, *dfs, *fs, *fs_next;
  double *rho, *ux, *uy, *uz, *T;
  int *cnt, *ids, *full;
  double *fsp, *usx, *usy, *usz;
  double *dP;      /* [cell][k][4]: share of sum_i (f^eq_i - f*_i) e_i, and
                      of sum_i |f^eq_i + f*_i| */
  double M[Q][Q], Minv[Q][Q];
  int64_t step;
};

/* ------------------------------------------------------------------ */
/* the D3Q19 moment basis (d'Humieres et al. 2002), row by row          */

static void build_basis(double M[Q][Q], double Minv[Q][Q]) {
  for (int q = 0; q < Q; ++q) {
    double x = CX[q], y = CY[q], z = CZ[q];
    double c2 = x * x + y * y + z * z;
    double r[Q] = {
        1.0,
        19.0 * c2 - 30.0,                          /* e       */
        (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0, /* epsilon */
        x, (5.0 * c2 - 9.0) * x,                   /* j_x, q_x */
        y, (5.0 * c2 - 9.0) * y,
        z, (5.0 * c2 - 9.0) * z,
        3.0 * x * x - c2,                          /* 3 p_xx  */
        (3.0 * c2 - 5.0) * (3.0 * x * x - c2),     /* 3 pi_xx */
        y * y - z * z,                             /* p_ww    */
        (3.0 * c2 - 5.0) * (y * y - z * z),        /* pi_ww   */
        x * y, y * z, x * z,                       /* p_xy, p_yz, p_xz */
        (y * y - z * z) * x,                       /* m_x     */
        (z * z - x * x) * y,                       /* m_y     */
        (x * x - y * y) * z};                      /* m_z     */
    for (int k = 0; k < Q; ++k) M[k][q] = r[k];
  }
  /* the rows are mutually orthogonal: M^{-1} = M^T diag(1/|row|^2) */
  for (int k = 0; k < Q; ++k) {
    double n2 = 0.0;
    for (int q = 0; q < Q; ++q) n2 += M[k][q] * M[k][q];
    for (int q = 0; q < Q; ++q) Minv[q][k] = M[k][q] / n2;
  }
}

static void mat_vec(const double A[Q][Q], const double* x, double* y) {
  for (int i = 0; i < Q; ++i) {
    double s = 0.0;
    for (int k = 0; k < Q; ++k) s += A[i][k] * x[k];
    y[i] = s;
  }
}

/* textbook second-order D3Q19 equilibrium */
static void feq_flow(double rho, double ux, double uy, double uz,
                     double* f) {
  double u2 = ux * ux + uy * uy + uz * uz;
  for (int q = 0; q < Q; ++q) {
    double eu = CX[q] * ux + CY[q] * uy + CZ[q] * uz;
    f[q] = wflow(q) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * u2);
  }
}

/* Guo's force term in velocity space (without the relaxation factor) */
static void guo_force(double Fx, double Fy, double Fz, double ux, double uy,
                      double uz, double* F) {
  double uF = ux * Fx + uy * Fy + uz * Fz;
  for (int q = 0; q < Q; ++q) {
    double eF = CX[q] * Fx + CY[q] * Fy + CZ[q] * Fz;
    double eu = CX[q] * ux + CY[q] * uy + CZ[q] * uz;
    F[q] = wflow(q) * (3.0 * eF + 9.0 * eu * eF - 3.0 * uF);
  }
}

/* ------------------------------------------------------------------ */
/* geometry: volume of a sphere inside a unit cell                      */

/* Cross-sectional area at height z (relative to the centre): the disk of
 * radius sqrt(R^2 - z^2) inside the cell's square. */
static double section(double cx, double cy, double R, double x0, double y0,
                      double z) {
  double r2 = (R - z) * (R + z);
  if (!(r2 > 0.0)) return 0.0;
  return or_disk_cell_area(cx, cy, sqrt(r2), x0, y0);
}

/* Integral of the section over [u, v] by the tanh-sinh rule (Takahashi
 * and Mori, 1974), whose nodes crowd towards the ends, so that the
 * algebraic endpoint behaviour where the circle touches an edge or a
 * corner costs nothing; the step is halved until two levels agree to
 * 1e-15.  Points are placed by their distance from the nearer end. */
static double tanh_sinh(double cx, double cy, double R, double x0, double y0,
                        double u, double v) {
  const double half = 0.5 * (v - u), tmax = 3.6;
  double h = 0.5;
  double sum = 0.5 * M_PI * section(cx, cy, R, x0, y0, 0.5 * (u + v));
  for (int k = 1; k * h <= tmax; ++k) {
    double t = k * h, s = 0.5 * M_PI * sinh(t);
    double w = 0.5 * M_PI * cosh(t) / (cosh(s) * cosh(s));
    double dist = 2.0 * half / (1.0 + exp(2.0 * s));
    sum += w * (section(cx, cy, R, x0, y0, v - dist) +
                section(cx, cy, R, x0, y0, u + dist));
  }
  double I = half * h * sum;
  for (int level = 0; level < 6; ++level) {
    h *= 0.5;
    for (int k = 1; k * h <= tmax; k += 2) {   /* the new (odd) nodes */
      double t = k * h, s = 0.5 * M_PI * sinh(t);
      double w = 0.5 * M_PI * cosh(t) / (cosh(s) * cosh(s));
      double dist = 2.0 * half / (1.0 + exp(2.0 * s));
      sum += w * (section(cx, cy, R, x0, y0, v - dist) +
                  section(cx, cy, R, x0, y0, u + dist));
    }
    double In = half * h * sum;
    int done = level >= 1 && fabs(In - I) < 1e-15;
    I = In;
    if (done) break;
  }
  return I;
}

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return x < y ? -1 : x > y;
}

/* Solid fraction of the cell with lower corner (x0, y0, z0) covered by the
 * sphere of radius R centred at (cx, cy, cz): the volume percentage of
 * Sec. 2 in three dimensions.  Reading: the exact volume, integrated over
 * z as the exact cross-sectional area; [z0, z0+1] is split where the
 * section's circle passes a line or a corner of the cell's square, so that
 * the area is smooth inside every piece. */
double o3_sphere_cell_volume(double cx, double cy, double cz, double R,
                             double x0, double y0, double z0) {
  double a[2] = {x0 - cx, x0 + 1.0 - cx}, b[2] = {y0 - cy, y0 + 1.0 - cy};
  double lo = z0 - cz > -R ? z0 - cz : -R;
  double hi = z0 + 1.0 - cz < R ? z0 + 1.0 - cz : R;
  if (!(lo < hi)) return 0.0;
  double d2[8] = {a[0] * a[0], a[1] * a[1], b[0] * b[0], b[1] * b[1],
                  a[0] * a[0] + b[0] * b[0], a[0] * a[0] + b[1] * b[1],
                  a[1] * a[1] + b[0] * b[0], a[1] * a[1] + b[1] * b[1]};
  double bp[18];
  int n = 0;
  bp[n++] = lo;
  for (int m = 0; m < 8; ++m) {
    if (!(d2[m] < R * R)) continue;
    double zb = sqrt((R * R) - d2[m]);
    if (zb > lo && zb < hi) bp[n++] = zb;
    if (-zb > lo && -zb < hi) bp[n++] = -zb;
  }
  bp[n++] = hi;
  qsort(bp, (size_t)n, sizeof(double), cmp_double);
  double V = 0.0;
  for (int m = 0; m + 1 < n; ++m)
    if (bp[m] < bp[m + 1])
      V += tanh_sinh(cx, cy, R, x0, y0, bp[m], bp[m + 1]);
  if (V < 0.0) V = 0.0;
  if (V > 1.0) V = 1.0;
  return V;
}

/* The closed cell meets the open ball: its point nearest to the centre
 * lies strictly inside the sphere. */
int o3_cell_in_band(double X, double Y, double Z, double R, int32_t i,
                    int32_t j, int32_t k) {
  double P[3] = {X, Y, Z};
  int lo[3] = {i, j, k};
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    double d = 0.0, e = (double)lo[a] - P[a], f = P[a] - (double)(lo[a] + 1);
    if (e > d) d = e;
    if (f > d) d = f;
    s += d * d;
  }
  return s < R * R;
}

/* The whole cell lies in the closed ball: its farthest corner does. */
int o3_cell_inside(double X, double Y, double Z, double R, int32_t i,
                   int32_t j, int32_t k) {
  double P[3] = {X, Y, Z};
  int lo[3] = {i, j, k};
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    double e = P[a] - (double)lo[a], f = (double)(lo[a] + 1) - P[a];
    double d = e > f ? e : f;
    s += d * d;
  }
  return s <= R * R;
}

/* ------------------------------------------------------------------ */

static int periodic(const o3_state* s, int axis) {
  return s->dom.face_flow[2 * axis] == O3_PERIODIC;
}
static double extent(const o3_state* s, int axis) {
  return axis == 0 ? s->dom.nx : axis == 1 ? s->dom.ny : s->dom.nz;
}
/* Reading (as in two dimensions): a node sees a particle through its
 * nearest periodic copy. */
static double near_copy(double Xp, double node, double L, int per) {
  if (!per) return Xp;
  if (node - Xp > 0.5 * L) return Xp + L;
  if (Xp - node > 0.5 * L) return Xp - L;
  return Xp;
}
static double cv_solid(const o3_state* s) { return s->dom.R_cv * s->dom.cv_f; }
static double lam_solid(const o3_state* s) {
  return s->dom.R_lambda * s->dom.lambda_f;
}
/* c_v,ref: harmonic mean of the two specific heats (Sec. 2.2) */
static double c_ref(const o3_state* s) {
  double a = s->dom.cv_f, b = cv_solid(s);
  return 2.0 * a * b / (a + b);
}

static void* zalloc(size_t n) { return calloc(n ? n : 1, 1); }

void o3_destroy(o3_state* s) {
  if (!s) return;
  double** d[] = {&s->X, &s->Y, &s->Z, &s->U, &s->V, &s->W, &s->Ox, &s->Oy,
                  &s->Oz, &s->Up, &s->Vp, &s->Wp, &s->Oxp, &s->Oyp, &s->Ozp,
                  &s->R, &s->rhos, &s->Tp0, &s->Fx, &s->Fy, &s->Fz, &s->Tx,
                  &s->Ty, &s->Tz, &s->Fabs, &s->Tmean, &s->Tmin, &s->E,
                  &s->fssum, &s->f, &s->g, &s->fst, &s->gst, &s->dfs, &s->fs,
                  &s->fs_next, &s->rho, &s->ux, &s->uy, &s->uz, &s->T,
                  &s->fsp, &s->usx, &s->usy, &s->usz, &s->dP};
  for (size_t k = 0; k < sizeof d / sizeof d[0]; ++k) free(*d[k]);
  free(s->fixed);
  free(s->cnt);
  free(s->ids);
  free(s->full);
  free(s);
}

int o3_create(const o3_domain* d, int32_t np, const o3_particle* p,
              o3_state** out) {
  if (!d || !out || np < 0 || (np > 0 && !p)) return O3_EINVAL;
  if (d->nx < 1 || d->ny < 1 || d->nz < 1 || d->kmax < 1 || !(d->tau_f > 0.5))
    return O3_EINVAL;
  for (int a = 0; a < 3; ++a)
    if ((d->face_flow[2 * a] == O3_PERIODIC) !=
        (d->face_flow[2 * a + 1] == O3_PERIODIC))
      return O3_EINVAL;
  o3_state* s = (o3_state*)zalloc(sizeof(o3_state));
  if (!s) return O3_ENOMEM;
  s->dom = *d;
  s->np = np;
  s->kmax = d->kmax;
  size_t nc = (size_t)d->nx * d->ny * d->nz, K = (size_t)d->kmax;
  size_t P = (size_t)(np > 0 ? np : 1);
  double** pp[] = {&s->X, &s->Y, &s->Z, &s->U, &s->V, &s->W, &s->Ox, &s->Oy,
                   &s->Oz, &s->Up, &s->Vp, &s->Wp, &s->Oxp, &s->Oyp, &s->Ozp,
                   &s->R, &s->rhos, &s->Tp0, &s->Fx, &s->Fy, &s->Fz, &s->Tx,
                   &s->Ty, &s->Tz, &s->Fabs, &s->Tmean, &s->Tmin, &s->E,
                   &s->fssum};
  for (size_t k = 0; k < sizeof pp / sizeof pp[0]; ++k)
    *pp[k] = (double*)zalloc(sizeof(double) * P);
  s->fixed = (int*)zalloc(sizeof(int) * P);
  s->f = (double*)zalloc(sizeof(double) * nc * Q);
  s->fst = (double*)zalloc(sizeof(double) * nc * Q);
  s->g = (double*)zalloc(sizeof(double) * nc * QG);
  s->gst = (double*)zalloc(sizeof(double) * nc * QG);
  double** fl[] = {&s->dfs, &s->fs, &s->fs_next, &s->rho, &s->ux, &s->uy,
                   &s->uz, &s->T};
  for (size_t k = 0; k < sizeof fl / sizeof fl[0]; ++k)
    *fl[k] = (double*)zalloc(sizeof(double) * nc);
  s->cnt = (int*)zalloc(sizeof(int) * nc);
  s->ids = (int*)zalloc(sizeof(int) * nc * K);
  s->full = (int*)zalloc(sizeof(int) * nc * K);
  s->fsp = (double*)zalloc(sizeof(double) * nc * K);
  s->usx = (double*)zalloc(sizeof(double) * nc * K);
  s->usy = (double*)zalloc(sizeof(double) * nc * K);
  s->usz = (double*)zalloc(sizeof(double) * nc * K);
  s->dP = (double*)zalloc(sizeof(double) * nc * K * 4);
  if (!s->f || !s->g || !s->fst || !s->gst || !s->dP || !s->T || !s->fsp ||
      !s->ids) {
    o3_destroy(s);
    return O3_ENOMEM;
  }
  for (int i = 0; i < np; ++i) {
    if (!(p[i].radius > 0.0) || !(p[i].rho_s > 0.0)) {
      o3_destroy(s);
      return O3_EINVAL;
    }
    s->X[i] = p[i].x; s->Y[i] = p[i].y; s->Z[i] = p[i].z;
    s->U[i] = p[i].ux; s->V[i] = p[i].uy; s->W[i] = p[i].uz;
    s->Ox[i] = p[i].ox; s->Oy[i] = p[i].oy; s->Oz[i] = p[i].oz;
    s->R[i] = p[i].radius; s->rhos[i] = p[i].rho_s; s->Tp0[i] = p[i].T_init;
    s->fixed[i] = p[i].fixed;
  }
  build_basis(s->M, s->Minv);
  *out = s;
  return O3_OK;
}

int o3_set_hooks(o3_state* s, const o3_hooks* h) {
  if (!s || !h) return O3_EINVAL;
  s->hk = *h;
  return O3_OK;
}

double* o3_f(o3_state* s) { return s->f; }
double* o3_g(o3_state* s) { return s->g; }
double* o3_d(o3_state* s) { return s->dfs; }
double* o3_fs(o3_state* s) { return s->fs; }
double* o3_rho(o3_state* s) { return s->rho; }
double* o3_ux(o3_state* s) { return s->ux; }
double* o3_uy(o3_state* s) { return s->uy; }
double* o3_uz(o3_state* s) { return s->uz; }
double* o3_T(o3_state* s) { return s->T; }
double* o3_fs_next(o3_state* s) { return s->fs_next; }
int32_t* o3_own_count(o3_state* s) { return s->cnt; }
int32_t* o3_own_ids(o3_state* s) { return s->ids; }

/* ------------------------------------------------------------------ */
/* stage 1: particle dynamics (Sec. 2.3)                                */

/* Reading (as in two dimensions): a short-range repulsion of range zeta,
 * F = k ((R_i + R_j + zeta - d)/zeta)^2 along the line of centres, and
 * against each wall the same law for the mirror image (distance twice the
 * gap) with the wall stiffness. */
static void repulsion(const o3_state* s, int i, double F[3]) {
  const o3_domain* d = &s->dom;
  F[0] = F[1] = F[2] = 0.0;
  double zeta = d->coll_range;
  if (!(zeta > 0.0)) return;
  double Pi[3] = {s->X[i], s->Y[i], s->Z[i]};
  for (int j = 0; j < s->np; ++j) {
    if (j == i) continue;
    double Pj[3] = {s->X[j], s->Y[j], s->Z[j]}, r[3], dist2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      r[a] = Pi[a] - near_copy(Pj[a], Pi[a], extent(s, a), periodic(s, a));
      dist2 += r[a] * r[a];
    }
    double dist = sqrt(dist2), reach = s->R[i] + s->R[j] + zeta;
    if (dist < reach && dist > 0.0) {
      double w = (reach - dist) / zeta, mag = d->coll_stiff_pp * w * w;
      for (int a = 0; a < 3; ++a) F[a] += mag * r[a] / dist;
    }
  }
  for (int face = 0; face < 6; ++face) {
    if (d->face_flow[face] != O3_WALL) continue;
    int a = face / 2;
    double gap = face % 2 ? extent(s, a) - Pi[a] : Pi[a];
    double dist = 2.0 * gap, reach = 2.0 * s->R[i] + zeta;
    if (dist < reach) {
      double w = (reach - dist) / zeta;
      F[a] += (face % 2 ? -1.0 : 1.0) * d->coll_stiff_pw * w * w;
    }
  }
}

/* Newton-Euler equations (eq. particle) for a sphere with the inside
 * "numerical fluid" terms of eq. inside.fluid (backward differences of U
 * and Omega), forward Euler; the position advances with U^n. */
static void particle_update(o3_state* s) {
  const o3_domain* d = &s->dom;
  int np = s->np;
  double* rep = (double*)zalloc(sizeof(double) * 3 * (size_t)np);
  for (int i = 0; i < np; ++i) repulsion(s, i, rep + 3 * i);
  for (int i = 0; i < np; ++i) {
    double R = s->R[i], Vol = 4.0 / 3.0 * M_PI * R * R * R;
    double Mp = s->rhos[i] * Vol, Ip = 0.4 * Mp * R * R;
    double Min = d->rho_f * Vol, Iin = d->rho_f * Ip / s->rhos[i];
    double U[3] = {s->U[i], s->V[i], s->W[i]};
    double O[3] = {s->Ox[i], s->Oy[i], s->Oz[i]};
    double Upr[3] = {s->Up[i], s->Vp[i], s->Wp[i]};
    double Opr[3] = {s->Oxp[i], s->Oyp[i], s->Ozp[i]};
    double F[3] = {s->Fx[i], s->Fy[i], s->Fz[i]};
    double T[3] = {s->Tx[i], s->Ty[i], s->Tz[i]};
    double nU[3] = {U[0], U[1], U[2]}, nO[3] = {O[0], O[1], O[2]};
    if (!s->fixed[i]) {
      for (int a = 0; a < 3; ++a) {
        double Fin = -Min * (U[a] - Upr[a]), Tin = -Iin * (O[a] - Opr[a]);
        double Fc = (F[a] - Fin) + (s->rhos[i] - d->rho_f) * Vol * d->gravity[a] +
                    rep[3 * i + a];
        nU[a] = U[a] + Fc / Mp;
        nO[a] = O[a] + (T[a] - Tin) / Ip;
      }
    }
    double Pn[3] = {s->X[i] + U[0], s->Y[i] + U[1], s->Z[i] + U[2]};
    for (int a = 0; a < 3; ++a)
      if (periodic(s, a)) {
        if (Pn[a] >= extent(s, a)) Pn[a] -= extent(s, a);
        if (Pn[a] < 0.0) Pn[a] += extent(s, a);
      }
    s->Up[i] = U[0]; s->Vp[i] = U[1]; s->Wp[i] = U[2];
    s->Oxp[i] = O[0]; s->Oyp[i] = O[1]; s->Ozp[i] = O[2];
    s->U[i] = nU[0]; s->V[i] = nU[1]; s->W[i] = nU[2];
    s->Ox[i] = nO[0]; s->Oy[i] = nO[1]; s->Oz[i] = nO[2];
    s->X[i] = Pn[0]; s->Y[i] = Pn[1]; s->Z[i] = Pn[2];
  }
  free(rep);
}

/* ------------------------------------------------------------------ */
/* stage 2: ownership, per-particle solid fractions and u_s (eq. us)    */

static int geometry(o3_state* s, double* fs_out) {
  const o3_domain* d = &s->dom;
  int nx = d->nx, ny = d->ny, nz = d->nz, K = s->kmax;
  size_t nc = (size_t)nx * ny * nz;
  memset(s->cnt, 0, sizeof(int) * nc);
  for (size_t k = 0; k < nc * (size_t)K; ++k) {
    s->ids[k] = -1;
    s->full[k] = 0;
    s->fsp[k] = s->usx[k] = s->usy[k] = s->usz[k] = 0.0;
  }
  int status = O3_OK;
  for (int p = 0; p < s->np; ++p) {
    double R = s->R[p], C[3] = {s->X[p], s->Y[p], s->Z[p]};
    int lo[3], hi[3], n3[3] = {nx, ny, nz};
    for (int a = 0; a < 3; ++a) {
      lo[a] = (int)floor(C[a] - R) - 1;
      hi[a] = (int)floor(C[a] + R) + 1;
    }
    for (int kk = lo[2]; kk <= hi[2]; ++kk)
      for (int jj = lo[1]; jj <= hi[1]; ++jj)
        for (int ii = lo[0]; ii <= hi[0]; ++ii) {
          int idx[3] = {ii, jj, kk}, ok = 1;
          for (int a = 0; a < 3; ++a) {
            if (periodic(s, a)) idx[a] = ((idx[a] % n3[a]) + n3[a]) % n3[a];
            if (idx[a] < 0 || idx[a] >= n3[a]) ok = 0;
          }
          if (!ok) continue;
          double Pc[3];
          for (int a = 0; a < 3; ++a)
            Pc[a] = near_copy(C[a], idx[a] + 0.5, n3[a], periodic(s, a));
          if (!o3_cell_in_band(Pc[0], Pc[1], Pc[2], R, idx[0], idx[1],
                               idx[2]))
            continue;
          size_t c = ((size_t)idx[2] * ny + idx[1]) * nx + idx[0];
          int n = s->cnt[c];
          if (n >= K) {
            status = O3_EOVERLAP;
            continue;
          }
          size_t sl = c * K + (size_t)n;
          int inside = o3_cell_inside(Pc[0], Pc[1], Pc[2], R, idx[0], idx[1],
                                      idx[2]);
          s->ids[sl] = p;
          s->full[sl] = inside;
          s->fsp[sl] = inside ? 1.0
                              : o3_sphere_cell_volume(Pc[0], Pc[1], Pc[2], R,
                                                      idx[0], idx[1], idx[2]);
          /* u_s = U + Omega x (x - X), x the node (eq. us) */
          double r[3] = {idx[0] + 0.5 - Pc[0], idx[1] + 0.5 - Pc[1],
                         idx[2] + 0.5 - Pc[2]};
          s->usx[sl] = s->U[p] + (s->Oy[p] * r[2] - s->Oz[p] * r[1]);
          s->usy[sl] = s->V[p] + (s->Oz[p] * r[0] - s->Ox[p] * r[2]);
          s->usz[sl] = s->W[p] + (s->Ox[p] * r[1] - s->Oy[p] * r[0]);
          s->cnt[c] = n + 1;
        }
  }
  /* Reading (as in two dimensions): shares adding up to more than one
   * (overlapping spheres) are scaled to sum to one. */
  for (size_t c = 0; c < nc; ++c) {
    double S = 0.0;
    for (int k = 0; k < s->cnt[c]; ++k) S += s->fsp[c * K + k];
    if (S > 1.0) {
      for (int k = 0; k < s->cnt[c]; ++k) s->fsp[c * K + k] /= S;
      S = 1.0;
    }
    fs_out[c] = S;
  }
  return status;
}

/* ------------------------------------------------------------------ */
/* stage 4: pull streaming with the wall rules                           */

static void stream(o3_state* s) {
  const o3_domain* d = &s->dom;
  int nx = d->nx, ny = d->ny, nz = d->nz;
  size_t nc = (size_t)nx * ny * nz;
  double cref = c_ref(s);
#pragma omp parallel for schedule(static)
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        size_t c = ((size_t)k * ny + j) * nx + i;
        for (int q = 0; q < Q; ++q) {
          int src[3] = {i - CX[q], j - CY[q], k - CZ[q]};
          int n3[3] = {nx, ny, nz}, wall = -1;
          for (int a = 0; a < 3; ++a) {
            if (src[a] < 0) {
              if (periodic(s, a)) src[a] += n3[a]; else wall = 2 * a;
            } else if (src[a] >= n3[a]) {
              if (periodic(s, a)) src[a] -= n3[a]; else wall = 2 * a + 1;
            }
          }
          /* the last axis found beyond a wall decides: z, then y, then x */
          if (wall < 0) {
            size_t sc = ((size_t)src[2] * ny + src[1]) * nx + src[0];
            s->fst[q * nc + c] = s->f[q * nc + sc];
            if (q < QG) s->gst[q * nc + c] = s->g[q * nc + sc];
          } else {
            double eu = CX[q] * d->u_wall[wall][0] + CY[q] * d->u_wall[wall][1] +
                        CZ[q] * d->u_wall[wall][2];
            s->fst[q * nc + c] =
                s->f[OPP[q] * nc + c] + 6.0 * wflow(q) * d->init_rho * eu;
            if (q < QG) {
              if (d->face_thermal[wall] == O3_DIRICHLET)
                s->gst[q * nc + c] =
                    -s->g[OPP[q] * nc + c] + 2.0 * wg(q) * cref * d->T_wall[wall];
              else
                s->gst[q * nc + c] = s->g[OPP[q] * nc + c];
            }
          }
        }
      }
}

/* ------------------------------------------------------------------ */
/* stages 5-9 for one cell                                              */

static int update_cell(o3_state* s, size_t c) {
  const o3_domain* d = &s->dom;
  size_t nc = (size_t)d->nx * d->ny * d->nz;
  int K = s->kmax;
  double fst[Q], f[Q], g[QG];
  for (int q = 0; q < Q; ++q) fst[q] = s->fst[q * nc + c];
  for (int q = 0; q < QG; ++q) g[q] = s->gst[q * nc + c];
  double fs = s->fs[c], cvf = d->cv_f, cvs = cv_solid(s), cref = c_ref(s);

  /* stage 5: volumetric no-slip step (eq. fi) and each particle's share of
   * sum_i (f_i - f*_i) e_i */
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  if (!s->hk.thermal_only) {
    for (int q = 0; q < Q; ++q) rho += fst[q];
    for (int q = 0; q < Q; ++q) f[q] = (1.0 - fs) * fst[q];
    for (int k = 0; k < s->cnt[c]; ++k) {
      size_t sl = c * K + k;
      double fe[Q], P[4] = {0.0, 0.0, 0.0, 0.0};
      feq_flow(rho, s->usx[sl], s->usy[sl], s->usz[sl], fe);
      for (int q = 0; q < Q; ++q) {
        f[q] += s->fsp[sl] * fe[q];
        double df = s->fsp[sl] * (fe[q] - fst[q]);
        P[0] += df * CX[q];
        P[1] += df * CY[q];
        P[2] += df * CZ[q];
        P[3] += s->fsp[sl] * fabs(fe[q] + fst[q]);
      }
      for (int a = 0; a < 4; ++a) s->dP[sl * 4 + a] = P[a];
    }
    for (int q = 0; q < Q; ++q) {
      j[0] += CX[q] * f[q];
      j[1] += CY[q] * f[q];
      j[2] += CZ[q] * f[q];
    }
  }

  /* stage 6: per-cell properties (Sec. 2.2); eq. lambda on D3Q7 */
  double cv = (1.0 - fs) * cvf + fs * cvs;
  double lam = (1.0 - fs) * d->lambda_f + fs * lam_solid(s);
  double tau_g = 0.5 + lam / (d->rho_f * CS2G * cref);
  double sj = 1.0 / tau_g, se;
  if (d->sigma_rule == 0)
    se = 1.0 / (0.5 + 0.25 / (tau_g - 0.5));
  else
    se = 1.0;

  /* stage 7: macroscopic quantities and the coupled T-u solve */
  double G = 0.0, J[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < QG; ++q) {
    G += g[q];
    J[0] += CX[q] * g[q];
    J[1] += CY[q] * g[q];
    J[2] += CZ[q] * g[q];
  }
  double gT[3];
  for (int a = 0; a < 3; ++a) gT[a] = -J[a] / (CS2G * cref * tau_g);
  double dfs = s->dfs[c], dcv = cvs - cvf, T, u[3], F[3] = {0.0, 0.0, 0.0};
  if (s->hk.thermal_only) {
    for (int a = 0; a < 3; ++a) u[a] = s->hk.u_pres[a];
    T = (G - 0.5 * cv * (u[0] * gT[0] + u[1] * gT[1] + u[2] * gT[2])) /
        (cv - 0.5 * dcv * dfs);
  } else {
    /* F = a + b T on the fluid fraction: the external force and the
     * Boussinesq buoyancy; u = (j + F/2)/rho (eq. rho.rhou) */
    double wf = 1.0 - fs, A[3], B[3];
    for (int a = 0; a < 3; ++a) {
      A[a] = wf * (d->body_force[a] + d->rho_f * d->beta * d->T_ref * d->gravity[a]);
      B[a] = -wf * d->rho_f * d->beta * d->gravity[a];
    }
    double jg = 0.0, bg = 0.0;
    for (int a = 0; a < 3; ++a) {
      jg += (j[a] + 0.5 * A[a]) * gT[a];
      bg += B[a] * gT[a];
    }
    T = (G - 0.5 * cv * jg / rho) / (cv - 0.5 * dcv * dfs + 0.25 * cv * bg / rho);
    for (int a = 0; a < 3; ++a) {
      F[a] = A[a] + B[a] * T;
      u[a] = (j[a] + 0.5 * F[a]) / rho;
    }
  }
  double eps = cv * T;
  double qc = -cv * (u[0] * gT[0] + u[1] * gT[1] + u[2] * gT[2]) + dcv * T * dfs;
  if (!isfinite(T) || !isfinite(u[0]) || !isfinite(u[1]) || !isfinite(u[2]) ||
      (!s->hk.thermal_only && !(rho > 0.0)))
    return O3_EUNSTABLE;
  s->rho[c] = s->hk.thermal_only ? 1.0 : rho;
  s->ux[c] = u[0];
  s->uy[c] = u[1];
  s->uz[c] = u[2];
  s->T[c] = T;

  /* stage 8: flow MRT collision (eq. lbe.rho.col) */
  if (!s->hk.thermal_only) {
    double tf = d->tau_f, snu = 1.0 / tf;
    double sq = 1.0 / (0.5 + (1.0 / 12.0) / (tf - 0.5));
    double S[Q] = {1.0, 1.25, 1.25, 1.0, sq, 1.0, sq, 1.0, sq, snu, 1.25,
                   snu, 1.25, snu, snu, snu, sq, sq, sq};
    double fe[Q], Fv[Q], m[Q], meq[Q], Fm[Q], mb[Q], fb[Q];
    feq_flow(rho, u[0], u[1], u[2], fe);
    guo_force(F[0], F[1], F[2], u[0], u[1], u[2], Fv);
    mat_vec(s->M, f, m);
    mat_vec(s->M, fe, meq);
    mat_vec(s->M, Fv, Fm);
    for (int k = 0; k < Q; ++k)
      mb[k] = m[k] - S[k] * (m[k] - meq[k]) + (1.0 - 0.5 * S[k]) * Fm[k];
    mat_vec(s->Minv, mb, fb);
    for (int q = 0; q < Q; ++q) s->f[q * nc + c] = fb[q];
  }

  /* stage 9: energy collision: even part at sigma_e, odd part at sigma_j,
   * the source on the rest population */
  {
    double geq[QG];
    geq[0] = eps - (1.0 - W0G) * cref * T;
    for (int q = 1; q < QG; ++q) geq[q] = W1G * cref * T;
    for (int q = 0; q < QG; ++q) {
      double ev = 0.5 * (g[q] + g[OPP[q]]), od = 0.5 * (g[q] - g[OPP[q]]);
      double eqe = 0.5 * (geq[q] + geq[OPP[q]]);
      double gb = g[q] - se * (ev - eqe) - sj * od;
      if (q == 0) gb += (1.0 - 0.5 * se) * qc;
      s->g[q * nc + c] = gb;
    }
  }
  return O3_OK;
}

/* stage 10: per-particle outputs and the momentum-exchange sums, in a
 * fixed cell order.  F = -sum f_s,p sum_i (f^eq_i - f*_i) e_i and
 * T = -sum (x - X) x [the same], x the node. */
static void particle_sums(o3_state* s, int with_mes) {
  const o3_domain* d = &s->dom;
  int np = s->np, K = s->kmax, nx = d->nx, ny = d->ny;
  size_t nc = (size_t)nx * ny * d->nz;
  if (np == 0) return;
  double* sT = (double*)zalloc(sizeof(double) * (size_t)np);
  double* mfull = (double*)zalloc(sizeof(double) * (size_t)np);
  double* many = (double*)zalloc(sizeof(double) * (size_t)np);
  for (int p = 0; p < np; ++p) {
    mfull[p] = many[p] = INFINITY;
    s->E[p] = s->fssum[p] = 0.0;
    if (with_mes)
      s->Fx[p] = s->Fy[p] = s->Fz[p] = s->Tx[p] = s->Ty[p] = s->Tz[p] =
          s->Fabs[p] = 0.0;
  }
  double cvs = cv_solid(s);
  for (size_t c = 0; c < nc; ++c) {
    int i = (int)(c % (size_t)nx), j = (int)((c / (size_t)nx) % (size_t)ny);
    int k = (int)(c / ((size_t)nx * ny));
    for (int n = 0; n < s->cnt[c]; ++n) {
      size_t sl = c * K + n;
      int p = s->ids[sl];
      double w = s->fsp[sl], Tc = s->T[c];
      sT[p] += w * Tc;
      s->E[p] += w * cvs * Tc;
      s->fssum[p] += w;
      if (Tc < many[p]) many[p] = Tc;
      if (s->full[sl] && Tc < mfull[p]) mfull[p] = Tc;
      if (with_mes) {
        double r[3] = {i + 0.5 - near_copy(s->X[p], i + 0.5, nx, periodic(s, 0)),
                       j + 0.5 - near_copy(s->Y[p], j + 0.5, ny, periodic(s, 1)),
                       k + 0.5 - near_copy(s->Z[p], k + 0.5, d->nz, periodic(s, 2))};
        const double* P = s->dP + sl * 4;
        s->Fx[p] -= P[0];
        s->Fy[p] -= P[1];
        s->Fz[p] -= P[2];
        s->Tx[p] -= r[1] * P[2] - r[2] * P[1];
        s->Ty[p] -= r[2] * P[0] - r[0] * P[2];
        s->Tz[p] -= r[0] * P[1] - r[1] * P[0];
        s->Fabs[p] += P[3];
      }
    }
  }
  for (int p = 0; p < np; ++p) {
    s->Tmean[p] = s->fssum[p] > 0.0 ? sT[p] / s->fssum[p] : 0.0;
    s->Tmin[p] = isfinite(mfull[p]) ? mfull[p] : many[p];
  }
  free(sT);
  free(mfull);
  free(many);
}

/* ------------------------------------------------------------------ */

int o3_init(o3_state* s) {
  if (!s) return O3_EINVAL;
  const o3_domain* d = &s->dom;
  size_t nc = (size_t)d->nx * d->ny * d->nz;
  int K = s->kmax;
  s->step = 0;
  for (int p = 0; p < s->np; ++p) {
    s->Up[p] = s->U[p]; s->Vp[p] = s->V[p]; s->Wp[p] = s->W[p];
    s->Oxp[p] = s->Ox[p]; s->Oyp[p] = s->Oy[p]; s->Ozp[p] = s->Oz[p];
    s->Fx[p] = s->Fy[p] = s->Fz[p] = s->Tx[p] = s->Ty[p] = s->Tz[p] = 0.0;
  }
  if (s->hk.fs_from_array) {
    memset(s->cnt, 0, sizeof(int) * nc);
    memcpy(s->fs, s->fs_next, sizeof(double) * nc);
  } else {
    int st = geometry(s, s->fs);
    if (st != O3_OK) return st;
  }
  double cvf = d->cv_f, cvs = cv_solid(s), cref = c_ref(s);
  /* Reading (as in two dimensions): rho = rho_0; u and the internal energy
   * are the volume-weighted mixtures of the fluid and particle values;
   * f = f^eq, g = g^eq are the post-collision populations at n = 0;
   * [df_s/dt] = 0. */
  for (size_t c = 0; c < nc; ++c) {
    double fs = s->fs[c], cv = (1.0 - fs) * cvf + fs * cvs, u[3], T, eps;
    if (s->hk.fs_from_array) {
      for (int a = 0; a < 3; ++a) u[a] = s->hk.u_pres[a];
      T = s->T[c];
      eps = cv * T;
    } else {
      for (int a = 0; a < 3; ++a) u[a] = (1.0 - fs) * d->init_u[a];
      eps = (1.0 - fs) * cvf * d->init_T;
      for (int n = 0; n < s->cnt[c]; ++n) {
        size_t sl = c * K + n;
        u[0] += s->fsp[sl] * s->usx[sl];
        u[1] += s->fsp[sl] * s->usy[sl];
        u[2] += s->fsp[sl] * s->usz[sl];
        eps += s->fsp[sl] * cvs * s->Tp0[s->ids[sl]];
      }
      T = eps / cv;
      if (s->hk.thermal_only)
        for (int a = 0; a < 3; ++a) u[a] = s->hk.u_pres[a];
    }
    double fe[Q];
    feq_flow(d->init_rho, u[0], u[1], u[2], fe);
    for (int q = 0; q < Q; ++q) s->f[q * nc + c] = fe[q];
    s->g[c] = eps - (1.0 - W0G) * cref * T;
    for (int q = 1; q < QG; ++q) s->g[q * nc + c] = W1G * cref * T;
    s->dfs[c] = 0.0;
    s->rho[c] = d->init_rho;
    s->ux[c] = u[0];
    s->uy[c] = u[1];
    s->uz[c] = u[2];
    s->T[c] = T;
  }
  particle_sums(s, 0);
  return O3_OK;
}

int o3_step(o3_state* s, int64_t nsteps) {
  if (!s || nsteps < 0) return O3_EINVAL;
  const o3_domain* d = &s->dom;
  size_t nc = (size_t)d->nx * d->ny * d->nz;
  double* fs_new = (double*)zalloc(sizeof(double) * nc);
  if (!fs_new) return O3_ENOMEM;
  int status = O3_OK;
  for (int64_t it = 0; it < nsteps && status == O3_OK; ++it) {
    if (!s->hk.fs_from_array && s->np > 0) particle_update(s);   /* 1 */
    if (s->hk.fs_from_array)                                     /* 2 */
      memcpy(fs_new, s->fs_next, sizeof(double) * nc);
    else if ((status = geometry(s, fs_new)) != O3_OK)
      break;
    for (size_t c = 0; c < nc; ++c) {   /* 3: eq. dfs_dt */
      s->dfs[c] = 2.0 * (fs_new[c] - s->fs[c]) - s->dfs[c];
      s->fs[c] = fs_new[c];
    }
    stream(s);                                                   /* 4 */
    int bad = 0;                                                 /* 5-9 */
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (long c = 0; c < (long)nc; ++c)
      if (update_cell(s, (size_t)c) != O3_OK) bad |= 1;
    if (bad) status = O3_EUNSTABLE;
    particle_sums(s, !s->hk.thermal_only);                       /* 10 */
    s->step++;
  }
  free(fs_new);
  return status;
}

int o3_read_particles(o3_state* s, int32_t n, o3_particle_state* out) {
  if (!s || !out || n < 0 || n > s->np) return O3_EINVAL;
  for (int p = 0; p < n; ++p) {
    o3_particle_state* o = out + p;
    o->x = s->X[p]; o->y = s->Y[p]; o->z = s->Z[p];
    o->ux = s->U[p]; o->uy = s->V[p]; o->uz = s->W[p];
    o->ox = s->Ox[p]; o->oy = s->Oy[p]; o->oz = s->Oz[p];
    o->Fx = s->Fx[p]; o->Fy = s->Fy[p]; o->Fz = s->Fz[p];
    o->Tx = s->Tx[p]; o->Ty = s->Ty[p]; o->Tz = s->Tz[p];
    o->T_mean = s->Tmean[p];
    o->T_min = s->Tmin[p];
    o->E_solid = s->E[p];
    o->fs_sum = s->fssum[p];
    o->F_abs = s->Fabs[p];
  }
  return O3_OK;
}
