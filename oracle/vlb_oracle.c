/*
 * vlb_oracle.c -- plain FP64 CPU oracle of one time step of the volumetric
 * lattice Boltzmann method for thermal particulate flows with conjugate heat
 * transfer (arXiv 2410.23802).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by tests/, the smoke check and the CPU
 * baseline of the benchmark.  No product code includes or links it, and it
 * shares no code with the GPU library.
 *
 * It follows the paper's equations in the paper's order, with the 9x9
 * transformation matrix M written out as printed (Sec. 2.1) and no blocking
 * or fusion.  Build with -O2 -ffp-contract=off so no multiply-add is fused.
 * Where the paper leaves a choice open, the reading taken is stated at the
 * point of use (tagged "Reading:").
 *
 * Parity unpinned: the particle repulsion (or_collision_force).  The paper
 * adopts a collision model without giving its law or constants, so only
 * invariants pin it here (force at contact equals the stiffness, zero at
 * and beyond the range, equal and opposite pair forces, a wall acting as a
 * mirror-image particle); the quadratic law itself is a reading.
 *
 * One step n -> n+1 (stage numbers are used in comments below):
 *   1  particle update from the force and torque of step n   (Sec. 2.3)
 *   2  cell ownership and solid fraction at n+1               (Sec. 2, Fig. 1)
 *   3  [df_s/dt] at n+1                                        (eq. dfs_dt)
 *   4  streaming of f and g, with wall rules                   (eq. lbe.rho.str, lbe.e.str)
 *   5  volumetric no-slip step and momentum exchange           (eq. fi, Sec. 2.3)
 *   5b held particle temperatures (a reading)                  (Sec. 3.3)
 *   6  per-cell properties                                     (Sec. 2.2, eq. lambda)
 *   7  macroscopic rho, u, T, eps, q_c                         (eq. rho.rhou, eq. e)
 *   8  flow MRT collision with the discrete force term         (eq. lbe.rho.col)
 *   9  energy MRT collision with the discrete source term      (eq. lbe.e.col)
 *   10 per-particle thermal outputs
 */
#include "vlb_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q 9
#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* D2Q9 velocities e_i of Sec. 2: e_0 = 0, e_1..4 along the axes, e_5..8
 * along the diagonals, counter-clockwise from +x. */
static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
/* Standard D2Q9 weights, used only by the wall rules (Reading Q9). */
static const double WT[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

/* Orthogonal transformation matrix M, as printed in Sec. 2.1. */
static const double MM[Q][Q] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

/* Free parameters of the energy LB as fixed in Sec. 2.2. */
#define ALPHA1 (-2.0)
#define ALPHA2 (1.0)
#define BETA2 (4.0)

struct or_state {
  or_domain dom;
  or_hooks hk;
  int np;
  /* particle state at the current step; the *p arrays hold the previous
   * step's velocities for the backward differences of Sec. 2.3 */
  double *X, *Y, *th, *Ux, *Uy, *Om, *Uxp, *Uyp, *Omp;
  double *R, *rhos, *Tp0;
  double *Rb;  /* minor semi-axis: R for a disk, < R for an ellipse */
  int *fixed;
  int *hold;  /* 1: temperature held at Tp0 (stage 5b) */
  double *Fx, *Fy, *Tz; /* momentum-exchange force/torque, current step */
  double *Tmean, *Tmin, *E, *fssum, *Fabs;
  /* fields */
  double *f, *g;     /* post-collision populations [q][cell] */
  double *fst, *gst; /* post-streaming populations [q][cell] */
  double *dfs;       /* [df_s/dt] at the current step        */
  double *fs;        /* total solid fraction, current step    */
  double *fs_next;   /* caller-provided f_s (hook)            */
  double *rho, *ux, *uy, *T, *eps, *qc;
  /* per-cell particle lists at the current step, [cell][k] */
  int *cnt, *ids, *full;
  double *fsp, *usx, *usy;
  double *dPx, *dPy; /* per-cell share of sum_i (f_i - f*_i) e_i */
  double Minv[Q][Q];
  int64_t step;
  int overlaps;
  int kmax;
};

/* ------------------------------------------------------------------ */
/* small linear algebra                                                 */

/* M^{-1}: the rows of M are mutually orthogonal, so M^{-1} = M^T N^{-1}
 * with N = diag(sum_k M_ik^2). */
static void build_minv(double Minv[Q][Q]) {
  for (int i = 0; i < Q; ++i) {
    double n2 = 0.0;
    for (int k = 0; k < Q; ++k) n2 += MM[i][k] * MM[i][k];
    for (int k = 0; k < Q; ++k) Minv[k][i] = MM[i][k] / n2;
  }
}

static void mat_vec(const double A[Q][Q], const double* x, double* y) {
  for (int i = 0; i < Q; ++i) {
    double s = 0.0;
    for (int k = 0; k < Q; ++k) s += A[i][k] * x[k];
    y[i] = s;
  }
}

/* Equilibrium moments m^eq(rho, u), Sec. 2.1 (c = 1). */
static void meq_flow(double rho, double ux, double uy, double* m) {
  double u2 = ux * ux + uy * uy;
  m[0] = rho;
  m[1] = -2.0 * rho + 3.0 * rho * u2;
  m[2] = rho - 3.0 * rho * u2;
  m[3] = rho * ux;
  m[4] = -rho * ux;
  m[5] = rho * uy;
  m[6] = -rho * uy;
  m[7] = rho * (ux * ux - uy * uy);
  m[8] = rho * ux * uy;
}

/* Discrete force term F_m(F, u), Sec. 2.1 (c = 1). */
static void force_moments(double Fx, double Fy, double ux, double uy,
                          double* Fm) {
  double Fu = Fx * ux + Fy * uy;
  Fm[0] = 0.0;
  Fm[1] = 6.0 * Fu;
  Fm[2] = -6.0 * Fu;
  Fm[3] = Fx;
  Fm[4] = -Fx;
  Fm[5] = Fy;
  Fm[6] = -Fy;
  Fm[7] = 2.0 * (Fx * ux - Fy * uy);
  Fm[8] = Fx * uy + Fy * ux;
}

/* Equilibrium moments n^eq(eps, T), Sec. 2.2. */
static void neq_energy(double eps, double T, double cref, double* n) {
  n[0] = eps;
  n[1] = -4.0 * eps + (4.0 + ALPHA1) * cref * T;
  n[2] = 4.0 * eps - (4.0 - ALPHA2) * cref * T;
  for (int k = 3; k < Q; ++k) n[k] = 0.0;
}

/* f^eq(rho, u) in velocity space.  The paper defines m^eq = M f^eq, so
 * f^eq = M^{-1} m^eq. */
static void feq_velocity(const double Minv[Q][Q], double rho, double ux,
                         double uy, double* feq) {
  double m[Q];
  meq_flow(rho, ux, uy, m);
  mat_vec(Minv, m, feq);
}

/* ------------------------------------------------------------------ */
/* geometry: exact area of a disk intersected with a unit cell          */

/* Half chord h(x) = sqrt(R^2 - x^2) of the disk at abscissa x, written as
 * a product so it stays accurate near |x| = R. */
static double half_chord(double x, double R) {
  if (x <= -R || x >= R) return 0.0;
  return sqrt((R - x) * (R + x));
}

/* Integral of h(x) over [u, v], -R <= u <= v <= R:
 *   (v h(v) - u h(u))/2 + R^2 (asin(v/R) - asin(u/R))/2,
 * with the difference of the two angles taken from its sine and cosine
 * (angle subtraction), which stays accurate for short intervals. */
static double chord_integral(double u, double v, double R) {
  double hu = half_chord(u, R), hv = half_chord(v, R);
  double ang = fabs(atan2(v * hu - u * hv, hu * hv + u * v));
  return 0.5 * (v * hv - u * hu) + 0.5 * R * R * ang;
}

/* Solid fraction of the cell [x0, x0+1] x [y0, y0+1] covered by the disk of
 * radius R centred at (cx, cy): the volume percentage of the solid part of
 * the lattice cell that defines f_s in Sec. 2 (Fig. 1).  Reading: the exact
 * area.  It is integrated column by column, A = int l(x) dx with
 * l(x) = min(b1, h) - max(b0, -h) clipped at zero, splitting [a0, a1] where
 * the circle crosses the lines y = b0 and y = b1 so that on each piece the
 * upper and lower limits are either a cell edge or the circle. */
double or_disk_cell_area(double cx, double cy, double R, double x0,
                         double y0) {
  double a0 = x0 - cx, a1 = (x0 + 1.0) - cx;
  double b0 = y0 - cy, b1 = (y0 + 1.0) - cy;
  double lo = a0 > -R ? a0 : -R, hi = a1 < R ? a1 : R;
  if (!(lo < hi)) return 0.0;
  double bp[6];
  int n = 0;
  bp[n++] = lo;
  double bs[2] = {b0, b1};
  for (int k = 0; k < 2; ++k) {
    if (fabs(bs[k]) >= R) continue;
    double xb = half_chord(bs[k], R);
    if (-xb > lo && -xb < hi) bp[n++] = -xb;
    if (xb > lo && xb < hi) bp[n++] = xb;
  }
  bp[n++] = hi;
  for (int a = 1; a < n; ++a) /* insertion sort of at most six points */
    for (int b = a; b > 0 && bp[b - 1] > bp[b]; --b) {
      double t = bp[b];
      bp[b] = bp[b - 1];
      bp[b - 1] = t;
    }
  double A = 0.0;
  for (int k = 0; k + 1 < n; ++k) {
    double u = bp[k], v = bp[k + 1];
    if (!(u < v)) continue;
    double hm = half_chord(0.5 * (u + v), R);
    double top = b1 < hm ? b1 : hm, bot = b0 > -hm ? b0 : -hm;
    if (!(top > bot)) continue; /* the strip misses the disk here */
    double piece = 0.0;
    if (b1 < hm) piece += b1 * (v - u);            /* upper limit: y = b1 */
    else piece += chord_integral(u, v, R);         /* upper limit: circle */
    if (b0 > -hm) piece -= b0 * (v - u);           /* lower limit: y = b0 */
    else piece += chord_integral(u, v, R);         /* lower limit: circle */
    A += piece;
  }
  if (A < 0.0) A = 0.0;
  if (A > 1.0) A = 1.0;
  return A;
}

/* ------------------------------------------------------------------ */
/* geometry: exact area of an ellipse intersected with a unit cell      */

/* For the ellipse of semi-axes a (along (c, s) = (cos th, sin th)) and b
 * centred at the origin, the points on the vertical line x = t have
 *   y in [k t - h(t), k t + h(t)],  h(t) = g(t) / A,  g(t) = sqrt(A - m^2 t^2),
 * with A = s^2/a^2 + c^2/b^2, k = c s (1/b^2 - 1/a^2) / A and m = 1/(a b):
 * the quadratic form (x.(c,s))^2/a^2 + (x.(-s,c))^2/b^2 <= 1 solved for y.
 * The line meets the ellipse for |t| <= W = sqrt(A)/m. */
typedef struct {
  double A, k, m, sA, W;
} or_ellipse;

static or_ellipse ellipse_of(double a, double b, double th) {
  or_ellipse e;
  double c = cos(th), s = sin(th);
  e.A = s * s / (a * a) + c * c / (b * b);
  e.k = c * s * (1.0 / (b * b) - 1.0 / (a * a)) / e.A;
  e.m = 1.0 / (a * b);
  e.sA = sqrt(e.A);
  e.W = e.sA / e.m;
  return e;
}

/* g(t), as a product so it stays accurate near |t| = W. */
static double ellipse_g(const or_ellipse* e, double t) {
  double mt = e->m * t;
  if (mt <= -e->sA || mt >= e->sA) return 0.0;
  return sqrt((e->sA - mt) * (e->sA + mt));
}

/* Integral of h(t) over [u, v] within [-W, W]:
 *   [ (v g(v) - u g(u))/2 + A/(2m) (asin(v/W) - asin(u/W)) ] / A,
 * the angle difference taken from its sine and cosine. */
static double ellipse_h_integral(const or_ellipse* e, double u, double v) {
  double gu = ellipse_g(e, u), gv = ellipse_g(e, v);
  double ang = atan2(e->m * (v * gu - u * gv), gu * gv + e->m * e->m * u * v);
  return (0.5 * (v * gv - u * gu) + 0.5 * e->A / e->m * ang) / e->A;
}

/* Solid fraction of the cell [x0, x0+1] x [y0, y0+1] covered by the
 * ellipse of semi-axes a (major, at angle th to the x axis) and b centred
 * at (cx, cy): the volume percentage of Sec. 2 for an elliptical particle
 * (Sec. 3.2).  Reading: the exact area, integrated column by column as for
 * the disk: A = int l(t) dt with l(t) = min(q1, k t + h) - max(q0, k t - h)
 * clipped at zero, [t0, t1] split where k t +- h(t) crosses q0 or q1 (the
 * roots of (A^2 k^2 + m^2) t^2 - 2 A^2 k q t + A^2 q^2 - A = 0). */
double or_ellipse_cell_area(double cx, double cy, double a, double b,
                            double th, double x0, double y0) {
  or_ellipse e = ellipse_of(a, b, th);
  double t0 = x0 - cx, t1 = (x0 + 1.0) - cx;
  double q0 = y0 - cy, q1 = (y0 + 1.0) - cy;
  double lo = t0 > -e.W ? t0 : -e.W, hi = t1 < e.W ? t1 : e.W;
  if (!(lo < hi)) return 0.0;
  double bp[6];
  int n = 0;
  bp[n++] = lo;
  double qs[2] = {q0, q1};
  double qa = e.A * e.A * e.k * e.k + e.m * e.m;
  for (int r = 0; r < 2; ++r) {
    double qb = -2.0 * e.A * e.A * e.k * qs[r];
    double qc = e.A * e.A * qs[r] * qs[r] - e.A;
    double disc = qb * qb - 4.0 * qa * qc;
    if (!(disc > 0.0)) continue;
    double sd = sqrt(disc);
    double ra = (-qb - sd) / (2.0 * qa), rb = (-qb + sd) / (2.0 * qa);
    if (ra > lo && ra < hi) bp[n++] = ra;
    if (rb > lo && rb < hi) bp[n++] = rb;
  }
  bp[n++] = hi;
  for (int u = 1; u < n; ++u) /* insertion sort of at most six points */
    for (int w = u; w > 0 && bp[w - 1] > bp[w]; --w) {
      double t = bp[w];
      bp[w] = bp[w - 1];
      bp[w - 1] = t;
    }
  double S = 0.0;
  for (int r = 0; r + 1 < n; ++r) {
    double u = bp[r], v = bp[r + 1];
    if (!(u < v)) continue;
    double tm = 0.5 * (u + v);
    double hm = ellipse_g(&e, tm) / e.A;
    double up = e.k * tm + hm, dn = e.k * tm - hm;
    double top = q1 < up ? q1 : up, bot = q0 > dn ? q0 : dn;
    if (!(top > bot)) continue; /* the strip misses the ellipse here */
    double lin = 0.5 * e.k * (v * v - u * u), hint = ellipse_h_integral(&e, u, v);
    double piece = 0.0;
    if (q1 < up) piece += q1 * (v - u);      /* upper limit: y = q1 */
    else piece += lin + hint;                /* upper limit: ellipse */
    if (q0 > dn) piece -= q0 * (v - u);      /* lower limit: y = q0 */
    else piece -= lin - hint;                /* lower limit: ellipse */
    S += piece;
  }
  if (S < 0.0) S = 0.0;
  if (S > 1.0) S = 1.0;
  return S;
}

/* Ownership predicate (integer work; no fused operations): the closed cell
 * [i, i+1] x [j, j+1] meets the open disk, i.e. the point of the cell
 * nearest to the centre lies strictly inside the circle. */
int or_cell_in_band(double X, double Y, double R, int32_t i, int32_t j) {
  double a = (double)i - X, b = X - (double)(i + 1);
  double dx = 0.0;
  if (a > dx) dx = a;
  if (b > dx) dx = b;
  double c = (double)j - Y, e = Y - (double)(j + 1);
  double dy = 0.0;
  if (c > dy) dy = c;
  if (e > dy) dy = e;
  return dx * dx + dy * dy < R * R;
}

/* The whole cell lies in the closed disk: its farthest corner does. */
int or_cell_inside(double X, double Y, double R, int32_t i, int32_t j) {
  double ax = X - (double)i, bx = (double)(i + 1) - X;
  double ex = ax > bx ? ax : bx;
  double ay = Y - (double)j, by = (double)(j + 1) - Y;
  double ey = ay > by ? ay : by;
  return ex * ex + ey * ey <= R * R;
}

/* Reading: on a periodic axis of length L, the particle is seen from a node
 * through its nearest periodic copy (lever arms, u_s and ownership). */
static double min_image(double Xp, double node, double L, int periodic) {
  if (!periodic) return Xp;
  if (node - Xp > 0.5 * L) return Xp + L;
  if (Xp - node > 0.5 * L) return Xp - L;
  return Xp;
}

/* ------------------------------------------------------------------ */

static int per_x(const or_state* s) {
  return s->dom.face_flow[OR_FACE_XLO] == OR_PERIODIC;
}
static int per_y(const or_state* s) {
  return s->dom.face_flow[OR_FACE_YLO] == OR_PERIODIC;
}
static double cv_solid(const or_state* s) { return s->dom.R_cv * s->dom.cv_f; }
static double lambda_solid(const or_state* s) {
  return s->dom.R_lambda * s->dom.lambda_f;
}
/* c_{v,ref}: harmonic mean of the fluid and solid specific heats, Sec. 2.2. */
static double c_ref(const or_state* s) {
  double a = s->dom.cv_f, b = cv_solid(s);
  return 2.0 * a * b / (a + b);
}

void or_default_hooks(or_hooks* h) {
  memset(h, 0, sizeof(*h));
  h->beta1 = -4.0;
}

int or_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

static void* zalloc(size_t n) { return calloc(n ? n : 1, 1); }

void or_destroy(or_state* s) {
  if (!s) return;
  double* dp[] = {s->X,    s->Y,   s->th,  s->Ux,  s->Uy,    s->Om,
                  s->Uxp,  s->Uyp, s->Omp, s->R,   s->rhos,  s->Tp0, s->Rb,
                  s->Fx,   s->Fy,  s->Tz,  s->Tmean, s->Tmin, s->E,
                  s->fssum, s->Fabs, s->f, s->g, s->fst, s->gst, s->dfs,
                  s->fs,   s->fs_next, s->rho, s->ux, s->uy, s->T,
                  s->eps,  s->qc,  s->fsp, s->usx, s->usy,   s->dPx,
                  s->dPy};
  for (size_t k = 0; k < sizeof(dp) / sizeof(dp[0]); ++k) free(dp[k]);
  free(s->fixed);
  free(s->hold);
  free(s->cnt);
  free(s->ids);
  free(s->full);
  free(s);
}

int or_create(const or_domain* d, int32_t np, const or_particle* p,
              or_state** out) {
  if (!d || !out || d->nx < 1 || d->ny < 1 || np < 0 || (np > 0 && !p))
    return OR_EINVAL;
  for (int a = 0; a < 2; ++a)
    if ((d->face_flow[2 * a] == OR_PERIODIC) !=
        (d->face_flow[2 * a + 1] == OR_PERIODIC))
      return OR_EINVAL;
  if (!(d->tau_f > 0.5) || !(d->cv_f > 0) || !(d->lambda_f > 0) ||
      !(d->R_lambda > 0) || !(d->R_cv > 0) || !(d->rho_f > 0) || d->kmax < 1)
    return OR_EINVAL;
  for (int k = 0; k < np; ++k) {
    if (!(p[k].radius > 0.0) || !(p[k].rho_s > 0.0)) return OR_EINVAL;
    if (!(p[k].radius_minor >= 0.0) || p[k].radius_minor > p[k].radius)
      return OR_EINVAL;
    if (d->face_flow[0] == OR_PERIODIC && !(d->nx > 2.0 * p[k].radius + 4.0))
      return OR_EINVAL;
    if (d->face_flow[2] == OR_PERIODIC && !(d->ny > 2.0 * p[k].radius + 4.0))
      return OR_EINVAL;
  }
  or_state* s = (or_state*)zalloc(sizeof(or_state));
  if (!s) return OR_ENOMEM;
  s->dom = *d;
  or_default_hooks(&s->hk);
  s->np = np;
  s->kmax = d->kmax;
  size_t nc = (size_t)d->nx * d->ny, K = (size_t)d->kmax, n = (size_t)np;
  double** dp[] = {&s->X,   &s->Y,    &s->th,  &s->Ux,    &s->Uy,
                   &s->Om,  &s->Uxp,  &s->Uyp, &s->Omp,   &s->R,
                   &s->rhos, &s->Tp0, &s->Rb,  &s->Fx,    &s->Fy,  &s->Tz,
                   &s->Tmean, &s->Tmin, &s->E, &s->fssum, &s->Fabs};
  for (size_t k = 0; k < sizeof(dp) / sizeof(dp[0]); ++k)
    *dp[k] = (double*)zalloc(sizeof(double) * n);
  s->fixed = (int*)zalloc(sizeof(int) * n);
  s->hold = (int*)zalloc(sizeof(int) * n);
  s->f = (double*)zalloc(sizeof(double) * Q * nc);
  s->g = (double*)zalloc(sizeof(double) * Q * nc);
  s->fst = (double*)zalloc(sizeof(double) * Q * nc);
  s->gst = (double*)zalloc(sizeof(double) * Q * nc);
  double** fp[] = {&s->dfs, &s->fs, &s->fs_next, &s->rho, &s->ux,
                   &s->uy,  &s->T,  &s->eps,     &s->qc};
  for (size_t k = 0; k < sizeof(fp) / sizeof(fp[0]); ++k)
    *fp[k] = (double*)zalloc(sizeof(double) * nc);
  s->cnt = (int*)zalloc(sizeof(int) * nc);
  s->ids = (int*)zalloc(sizeof(int) * nc * K);
  s->full = (int*)zalloc(sizeof(int) * nc * K);
  double** kp[] = {&s->fsp, &s->usx, &s->usy, &s->dPx, &s->dPy};
  for (size_t k = 0; k < sizeof(kp) / sizeof(kp[0]); ++k)
    *kp[k] = (double*)zalloc(sizeof(double) * nc * K);
  if (!s->f || !s->g || !s->fst || !s->gst || !s->dPy || !s->ids) {
    or_destroy(s);
    return OR_ENOMEM;
  }
  build_minv(s->Minv);
  for (int k = 0; k < np; ++k) {
    s->X[k] = p[k].x;
    s->Y[k] = p[k].y;
    s->th[k] = p[k].theta;
    s->Ux[k] = p[k].ux;
    s->Uy[k] = p[k].uy;
    s->Om[k] = p[k].omega;
    s->R[k] = p[k].radius;
    s->Rb[k] = p[k].radius_minor > 0.0 ? p[k].radius_minor : p[k].radius;
    s->rhos[k] = p[k].rho_s;
    s->Tp0[k] = p[k].T_init;
    s->fixed[k] = p[k].fixed;
    s->hold[k] = p[k].hold_T;
  }
  *out = s;
  return OR_OK;
}

int or_set_hooks(or_state* s, const or_hooks* h) {
  if (!s || !h) return OR_EINVAL;
  if (h->fs_from_array && s->np > 0) return OR_EINVAL;
  s->hk = *h;
  return OR_OK;
}

int64_t or_step_count(const or_state* s) { return s->step; }
double* or_f(or_state* s) { return s->f; }
double* or_g(or_state* s) { return s->g; }
double* or_d(or_state* s) { return s->dfs; }
double* or_fs(or_state* s) { return s->fs; }
double* or_rho(or_state* s) { return s->rho; }
double* or_ux(or_state* s) { return s->ux; }
double* or_uy(or_state* s) { return s->uy; }
double* or_T(or_state* s) { return s->T; }
double* or_eps(or_state* s) { return s->eps; }
double* or_qc(or_state* s) { return s->qc; }
double* or_fs_next(or_state* s) { return s->fs_next; }
int32_t* or_own_count(or_state* s) { return s->cnt; }
int32_t* or_own_ids(or_state* s) { return s->ids; }
int32_t* or_own_full(or_state* s) { return s->full; }
int or_overlap_count(const or_state* s) { return s->overlaps; }

/* ------------------------------------------------------------------ */
/* stage 1: particle dynamics (Sec. 2.3)                                */

/* Parity unpinned (law and constants).  Reading of the collision model
 * the paper adopts without giving it:
 * a short-range repulsion of range zeta,
 *   F_ij = k_pp ((R_i + R_j + zeta - d_ij) / zeta)^2 (X_i - X_j) / d_ij
 * for d_ij < R_i + R_j + zeta, and against each wall the same law applied
 * to the particle's mirror image (distance d' = 2 x wall distance) with
 * stiffness k_pw.  Central forces exert no torque.  Summed over j in
 * ascending order, then the walls x-, x+, y-, y+. */
int or_collision_force(const or_state* s, int32_t i, double* fx,
                       double* fy) {
  const or_domain* d = &s->dom;
  double zeta = d->coll_range, sx = 0.0, sy = 0.0;
  if (!(zeta > 0.0)) {
    *fx = *fy = 0.0;
    return OR_OK;
  }
  for (int j = 0; j < s->np; ++j) {
    if (j == i) continue;
    double rx = s->X[i] - min_image(s->X[j], s->X[i], d->nx, per_x(s));
    double ry = s->Y[i] - min_image(s->Y[j], s->Y[i], d->ny, per_y(s));
    double dist = sqrt(rx * rx + ry * ry);
    double reach = s->R[i] + s->R[j] + zeta;
    if (dist < reach && dist > 0.0) {
      double w = (reach - dist) / zeta;
      double mag = d->coll_stiff_pp * w * w;
      sx += mag * rx / dist;
      sy += mag * ry / dist;
    }
  }
  /* walls: outward normal of the wall points into the domain */
  double wd[4] = {s->X[i], d->nx - s->X[i], s->Y[i], d->ny - s->Y[i]};
  double nx_[4] = {1.0, -1.0, 0.0, 0.0}, ny_[4] = {0.0, 0.0, 1.0, -1.0};
  for (int w = 0; w < 4; ++w) {
    if (d->face_flow[w] != OR_WALL) continue;
    double dist = 2.0 * wd[w];
    double reach = 2.0 * s->R[i] + zeta;
    if (dist < reach) {
      double q = (reach - dist) / zeta;
      double mag = d->coll_stiff_pw * q * q;
      sx += mag * nx_[w];
      sy += mag * ny_[w];
    }
  }
  *fx = sx;
  *fy = sy;
  return OR_OK;
}

static void wrap_position(const or_state* s, double* X, double* Y) {
  if (per_x(s)) {
    if (*X >= s->dom.nx) *X -= s->dom.nx;
    if (*X < 0.0) *X += s->dom.nx;
  }
  if (per_y(s)) {
    if (*Y >= s->dom.ny) *Y -= s->dom.ny;
    if (*Y < 0.0) *Y += s->dom.ny;
  }
}

/* Newton-Euler equations (eq. particle) for a disk in 2-D, where the
 * gyroscopic term Omega x (I Omega) vanishes.  The inside "numerical fluid"
 * force and torque (eq. inside.fluid) use backward differences of U and
 * Omega; the total force adds the net body force (rho_s - rho_f) V g and
 * the repulsion; the equations are then advanced by forward Euler (Sec. 2.3
 * end).  Reading: X^{n+1} = X^n + U^n and theta^{n+1} = theta^n + Omega^n
 * (forward Euler on the position too). */
static void particle_update(or_state* s) {
  const or_domain* d = &s->dom;
  int np = s->np;
  double* nFx = (double*)zalloc(sizeof(double) * (size_t)np);
  double* nFy = (double*)zalloc(sizeof(double) * (size_t)np);
  for (int i = 0; i < np; ++i)
    or_collision_force(s, i, &nFx[i], &nFy[i]); /* from positions at n */
  for (int i = 0; i < np; ++i) {
    double R = s->R[i], Rb = s->Rb[i];
    double V = M_PI * R * Rb;  /* disk: pi R^2; ellipse: pi a b */
    double Mp = s->rhos[i] * V;
    /* moment of inertia about the centre: M R^2/2 for a disk, M (a^2 +
     * b^2)/4 for an ellipse of semi-axes a, b */
    double Ip = Rb == R ? 0.5 * Mp * R * R : 0.25 * Mp * (R * R + Rb * Rb);
    double Min = d->rho_f * Mp / s->rhos[i]; /* M_in = rho_f M / rho_s */
    double Iin = d->rho_f * Ip / s->rhos[i];
    double Ux = s->Ux[i], Uy = s->Uy[i], Om = s->Om[i];
    double nUx = Ux, nUy = Uy, nOm = Om;
    if (!s->fixed[i]) {
      double Finx = -Min * (Ux - s->Uxp[i]);
      double Finy = -Min * (Uy - s->Uyp[i]);
      double Tin = -Iin * (Om - s->Omp[i]);
      double Foutx = s->Fx[i] - Finx, Fouty = s->Fy[i] - Finy;
      double Tout = s->Tz[i] - Tin;
      /* gravity: (rho_s - rho_f) V g (situation I of Sec. 3.2), or rho_s V
       * g when the fluid carries its own weight (situation II; the
       * buoyancy then comes through the momentum exchange) */
      double rg = d->fluid_gravity ? s->rhos[i] : s->rhos[i] - d->rho_f;
      double Fcx = Foutx + rg * V * d->gravity[0] + nFx[i];
      double Fcy = Fouty + rg * V * d->gravity[1] + nFy[i];
      nUx = Ux + Fcx / Mp;
      nUy = Uy + Fcy / Mp;
      nOm = Om + Tout / Ip;
    }
    double nX = s->X[i] + Ux, nY = s->Y[i] + Uy;
    wrap_position(s, &nX, &nY);
    s->th[i] += Om;
    s->Uxp[i] = Ux;
    s->Uyp[i] = Uy;
    s->Omp[i] = Om;
    s->Ux[i] = nUx;
    s->Uy[i] = nUy;
    s->Om[i] = nOm;
    s->X[i] = nX;
    s->Y[i] = nY;
  }
  free(nFx);
  free(nFy);
}

/* ------------------------------------------------------------------ */
/* stage 2: ownership, per-particle solid fractions and u_s (eq. us)    */

static int geometry(or_state* s, double* fs_out) {
  const or_domain* d = &s->dom;
  int nx = d->nx, ny = d->ny, K = s->kmax;
  size_t nc = (size_t)nx * ny;
  memset(s->cnt, 0, sizeof(int) * nc);
  for (size_t k = 0; k < nc * (size_t)K; ++k) {
    s->ids[k] = -1;
    s->full[k] = 0;
    s->fsp[k] = 0.0;
    s->usx[k] = 0.0;
    s->usy[k] = 0.0;
  }
  int status = OR_OK;
  for (int p = 0; p < s->np; ++p) {
    double R = s->R[p];
    int i0 = (int)floor(s->X[p] - R) - 1, i1 = (int)floor(s->X[p] + R) + 1;
    int j0 = (int)floor(s->Y[p] - R) - 1, j1 = (int)floor(s->Y[p] + R) + 1;
    for (int jj = j0; jj <= j1; ++jj) {
      int j = jj;
      if (per_y(s)) j = ((jj % ny) + ny) % ny;
      if (j < 0 || j >= ny) continue;
      for (int ii = i0; ii <= i1; ++ii) {
        int i = ii;
        if (per_x(s)) i = ((ii % nx) + nx) % nx;
        if (i < 0 || i >= nx) continue;
        double Xi = min_image(s->X[p], i + 0.5, nx, per_x(s));
        double Yi = min_image(s->Y[p], j + 0.5, ny, per_y(s));
        if (!or_cell_in_band(Xi, Yi, R, i, j)) continue;
        size_t c = (size_t)j * nx + i;
        int n = s->cnt[c];
        if (n >= K) {
          status = OR_EOVERLAP;
          continue;
        }
        size_t slot = c * K + (size_t)n;
        s->ids[slot] = p;
        /* Reading for an ellipse (semi-axes R > Rb): its band is that of
         * the circumscribed disk (radius R) and a cell is wholly inside
         * when it lies in the inscribed disk (radius Rb), which keeps both
         * integer decisions free of the orientation; the share is the
         * exact area (zero for band cells the ellipse misses). */
        double Rb = s->Rb[p];
        int inside = or_cell_inside(Xi, Yi, Rb, i, j);
        s->full[slot] = inside;
        s->fsp[slot] = inside ? 1.0
                       : Rb == R ? or_disk_cell_area(Xi, Yi, R, i, j)
                       : or_ellipse_cell_area(Xi, Yi, R, Rb, s->th[p], i, j);
        /* u_s = U_c + Omega_c x (x - X_c), x the node (eq. us) */
        double rx = (i + 0.5) - Xi, ry = (j + 0.5) - Yi;
        s->usx[slot] = s->Ux[p] - s->Om[p] * ry;
        s->usy[slot] = s->Uy[p] + s->Om[p] * rx;
        s->cnt[c] = n + 1;
      }
    }
  }
  /* Reading: several particles in one cell each bring their own share
   * f_s,p; if the shares add up to more than one (overlapping disks) they
   * are scaled down to sum to one. */
  for (size_t c = 0; c < nc; ++c) {
    double S = 0.0;
    for (int k = 0; k < s->cnt[c]; ++k) S += s->fsp[c * K + k];
    if (S > 1.0) {
      s->overlaps++;
      for (int k = 0; k < s->cnt[c]; ++k) s->fsp[c * K + k] /= S;
      S = 1.0;
    }
    fs_out[c] = S;
  }
  return status;
}

/* ------------------------------------------------------------------ */
/* stage 4: streaming (eq. lbe.rho.str and eq. lbe.e.str), pull form    */

/* Reading (the paper gives no wall scheme): walls lie on the outer cell
 * faces.  A population whose upstream cell lies beyond a wall is replaced
 * by halfway bounce-back of the opposite population of the same cell, plus
 * 6 w_i rho_0 (e_i . u_w) for a moving wall; for g, adiabatic walls bounce
 * back and Dirichlet walls use anti-bounce-back
 * g_i = -gbar_opp + 2 w_i c_ref T_w.  Where the upstream point is beyond
 * two walls (a corner), the y wall decides. */
static void stream(or_state* s) {
  const or_domain* d = &s->dom;
  int nx = d->nx, ny = d->ny;
  size_t nc = (size_t)nx * ny;
  static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  double cref = c_ref(s);
  int px = per_x(s), py = per_y(s);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    for (int i = 0; i < nx; ++i) {
      size_t c = (size_t)j * nx + i;
      for (int q = 0; q < Q; ++q) {
        int si = i - EX[q], sj = j - EY[q];
        int xw = -1, yw = -1;
        if (si < 0) {
          if (px) si += nx; else xw = OR_FACE_XLO;
        } else if (si >= nx) {
          if (px) si -= nx; else xw = OR_FACE_XHI;
        }
        if (sj < 0) {
          if (py) sj += ny; else yw = OR_FACE_YLO;
        } else if (sj >= ny) {
          if (py) sj -= ny; else yw = OR_FACE_YHI;
        }
        if (xw < 0 && yw < 0) {
          size_t src = (size_t)sj * nx + si;
          s->fst[q * nc + c] = s->f[q * nc + src];
          s->gst[q * nc + c] = s->g[q * nc + src];
        } else {
          int w = yw >= 0 ? yw : xw;
          double eu = EX[q] * d->u_wall[w][0] + EY[q] * d->u_wall[w][1];
          s->fst[q * nc + c] =
              s->f[OPP[q] * nc + c] + 6.0 * WT[q] * d->init_rho * eu;
          if (d->face_thermal[w] == OR_DIRICHLET)
            s->gst[q * nc + c] =
                -s->g[OPP[q] * nc + c] + 2.0 * WT[q] * cref * d->T_wall[w];
          else
            s->gst[q * nc + c] = s->g[OPP[q] * nc + c];
        }
      }
    }
  }
}

/* ------------------------------------------------------------------ */
/* stages 5-9 for one cell                                              */

static int update_cell(or_state* s, size_t c, int i, int j) {
  const or_domain* d = &s->dom;
  size_t nc = (size_t)d->nx * d->ny;
  int K = s->kmax;
  double fst[Q], f[Q], g[Q];
  for (int q = 0; q < Q; ++q) {
    fst[q] = s->fst[q * nc + c];
    g[q] = s->gst[q * nc + c];
  }
  double fs = s->fs[c];
  double cvf = d->cv_f, cvs = cv_solid(s), cref = c_ref(s);

  /* ---- stage 5: volumetric no-slip step, eq. fi ---- */
  double rho = 0.0, ux = 0.0, uy = 0.0;
  double jx = 0.0, jy = 0.0;
  if (!s->hk.thermal_only) {
    for (int q = 0; q < Q; ++q) rho += fst[q]; /* rho = sum_i f*_i */
    for (int q = 0; q < Q; ++q) f[q] = (1.0 - fs) * fst[q];
    for (int k = 0; k < s->cnt[c]; ++k) {
      size_t sl = c * K + k;
      double feq[Q];
      feq_velocity(s->Minv, rho, s->usx[sl], s->usy[sl], feq);
      double px = 0.0, py = 0.0;
      for (int q = 0; q < Q; ++q) {
        f[q] += s->fsp[sl] * feq[q];
        /* this particle's share of sum_i (f_i - f*_i) e_i (Sec. 2.3) */
        px += s->fsp[sl] * (feq[q] - fst[q]) * EX[q];
        py += s->fsp[sl] * (feq[q] - fst[q]) * EY[q];
      }
      s->dPx[sl] = px;
      s->dPy[sl] = py;
    }
    for (int q = 0; q < Q; ++q) {
      jx += EX[q] * f[q];
      jy += EY[q] * f[q];
    }
  }

  /* ---- stage 5b: particles whose temperature is held (Sec. 3.3's cold
   * particle of fixed temperature).  Reading (the paper does not give the
   * rule): the energy distribution gets the volumetric step that eq. fi
   * gives the flow distribution, g = (1 - sum_h f_s,p) g* + sum_h f_s,p
   * g^eq(c_v T_p, T_p), the sums over the held particles p reaching the
   * cell, c_v the cell's heat capacity of stage 6 (as eq. fi takes the
   * cell's rho); a cell wholly inside one is set to the solid's
   * equilibrium at T_p, and a uniform temperature stays uniform.  It acts
   * before the macroscopic quantities of stage 7. ---- */
  {
    double phi = 0.0, gh[Q];
    double cv_cell = (1.0 - fs) * cvf + fs * cvs;
    for (int q = 0; q < Q; ++q) gh[q] = 0.0;
    for (int k = 0; k < s->cnt[c]; ++k) {
      size_t sl = c * K + k;
      int p = s->ids[sl];
      if (!s->hold[p]) continue;
      double n[Q], geq[Q];
      neq_energy(cv_cell * s->Tp0[p], s->Tp0[p], cref, n);
      mat_vec(s->Minv, n, geq);
      phi += s->fsp[sl];
      for (int q = 0; q < Q; ++q) gh[q] += s->fsp[sl] * geq[q];
    }
    if (phi > 0.0)
      for (int q = 0; q < Q; ++q) g[q] = (1.0 - phi) * g[q] + gh[q];
  }

  /* ---- stage 6: per-cell properties (Sec. 2.2) ---- */
  double cv = (1.0 - fs) * cvf + fs * cvs;
  double lam = (1.0 - fs) * d->lambda_f + fs * lambda_solid(s);
  /* eq. lambda: lambda/rho_f = (4+alpha1)/6 c_ref (1/sigma_j - 1/2) */
  double tau_g = 0.5 + 6.0 * lam / (d->rho_f * (4.0 + ALPHA1) * cref);
  double sig_j = 1.0 / tau_g, sig_q = sig_j, sig_0 = 1.0, sig_e;
  if (d->sigma_rule == 0)  /* (1/sig_j - 1/2)(1/sig_e - 1/2) = 1/4 */
    sig_e = 1.0 / (0.5 + 0.25 / (tau_g - 0.5));
  else                     /* dense-case choice of Sec. 3.5 */
    sig_e = 1.0;
  double sig_eps = sig_e;

  /* ---- stage 7: macroscopic quantities ---- */
  double G = 0.0, Jgx = 0.0, Jgy = 0.0;
  for (int q = 0; q < Q; ++q) {
    G += g[q];
    Jgx += EX[q] * g[q];
    Jgy += EY[q] * g[q];
  }
  /* local temperature gradient at t+dt (Sec. 2.2) */
  double gTx = -6.0 / (4.0 + ALPHA1) * Jgx / (cref * tau_g);
  double gTy = -6.0 / (4.0 + ALPHA1) * Jgy / (cref * tau_g);
  double dfs = s->dfs[c];
  double dcv = cvs - cvf;
  double T, Fx = 0.0, Fy = 0.0;
  if (s->hk.thermal_only) {
    ux = s->hk.u_pres[0];
    uy = s->hk.u_pres[1];
    /* implicit T of Sec. 2.2 with the prescribed velocity */
    T = (G - 0.5 * cv * (ux * gTx + uy * gTy)) / (cv - 0.5 * dcv * dfs);
  } else {
    /* Reading: the body force acts on the fluid fraction (1 - f_s): an
     * external force plus the Boussinesq buoyancy -rho_f g beta (T - T_ref)
     * of Sec. 3.3, so F = a + b T.  Reading: T and u at t+dt are solved
     * together; eq. rho.rhou gives u = (j + F/2)/rho, and the implicit T of
     * Sec. 2.2 then is linear in T. */
    double wf = 1.0 - fs;
    /* situation II of Sec. 3.2 adds the fluid's own weight rho_f g */
    double gw = d->fluid_gravity ? d->rho_f : 0.0;
    double ax = wf * (d->body_force[0] + gw * d->gravity[0] +
                      d->rho_f * d->beta * d->T_ref * d->gravity[0]);
    double ay = wf * (d->body_force[1] + gw * d->gravity[1] +
                      d->rho_f * d->beta * d->T_ref * d->gravity[1]);
    double bx = -wf * d->rho_f * d->beta * d->gravity[0];
    double by = -wf * d->rho_f * d->beta * d->gravity[1];
    double num = G - 0.5 * cv * ((jx + 0.5 * ax) * gTx + (jy + 0.5 * ay) * gTy) / rho;
    double den = cv - 0.5 * dcv * dfs + 0.25 * cv * (bx * gTx + by * gTy) / rho;
    T = num / den;
    Fx = ax + bx * T;
    Fy = ay + by * T;
    ux = (jx + 0.5 * Fx) / rho;
    uy = (jy + 0.5 * Fy) / rho;
  }
  double eps = cv * T;
  double qc = -cv * (ux * gTx + uy * gTy) + dcv * T * dfs;
  if (!(T == T) || !isfinite(T) || !isfinite(ux) || !isfinite(uy) ||
      (!s->hk.thermal_only && !(rho > 0.0)))
    return OR_EUNSTABLE;
  s->rho[c] = s->hk.thermal_only ? 1.0 : rho;
  s->ux[c] = ux;
  s->uy[c] = uy;
  s->T[c] = T;
  s->eps[c] = eps;
  s->qc[c] = qc;

  /* ---- stage 8: flow collision, eq. lbe.rho.col ---- */
  if (!s->hk.thermal_only) {
    double tau_f = d->tau_f;
    double s_p = 1.0 / tau_f;
    double s_q = 1.0 / (0.5 + (1.0 / 12.0) / (tau_f - 0.5));
    double Sd[Q] = {1.0, 1.25, 1.25, 1.0, s_q, 1.0, s_q, s_p, s_p};
    double m[Q], meq[Q], Fm[Q], mb[Q];
    mat_vec(MM, f, m);
    meq_flow(rho, ux, uy, meq);
    force_moments(Fx, Fy, ux, uy, Fm);
    for (int k = 0; k < Q; ++k)
      mb[k] = m[k] - Sd[k] * (m[k] - meq[k]) + (1.0 - 0.5 * Sd[k]) * Fm[k];
    double fb[Q];
    mat_vec(s->Minv, mb, fb);
    for (int q = 0; q < Q; ++q) s->f[q * nc + c] = fb[q];
  }

  /* ---- stage 9: energy collision, eq. lbe.e.col ---- */
  {
    double Rd[Q] = {sig_0, sig_e, sig_eps, sig_j, sig_q,
                    sig_j, sig_q, sig_e,   sig_e};
    double n[Q], neq[Q], qm[Q], nb[Q];
    mat_vec(MM, g, n);
    neq_energy(eps, T, cref, neq);
    qm[0] = qc;
    qm[1] = s->hk.beta1 * qc;
    qm[2] = BETA2 * qc;
    for (int k = 3; k < Q; ++k) qm[k] = 0.0;
    for (int k = 0; k < Q; ++k)
      nb[k] = n[k] - Rd[k] * (n[k] - neq[k]) + (1.0 - 0.5 * Rd[k]) * qm[k];
    double gb[Q];
    mat_vec(s->Minv, nb, gb);
    for (int q = 0; q < Q; ++q) s->g[q * nc + c] = gb[q];
  }
  (void)i;
  (void)j;
  return OR_OK;
}

/* stage 10: per-particle outputs (Reading: the paper reports only the
 * minimum particle temperature; here mean T, minimum T over cells wholly
 * inside the disk, sum f_s,p c_vs T, and sum f_s,p) and the
 * momentum-exchange sums of Sec. 2.3, both in a fixed cell order. */
static void particle_sums(or_state* s, int with_mes) {
  const or_domain* d = &s->dom;
  int np = s->np, K = s->kmax;
  size_t nc = (size_t)d->nx * d->ny;
  if (np == 0) return;
  double* sT = (double*)zalloc(sizeof(double) * (size_t)np);
  double* minT_full = (double*)zalloc(sizeof(double) * (size_t)np);
  double* minT_any = (double*)zalloc(sizeof(double) * (size_t)np);
  for (int p = 0; p < np; ++p) {
    minT_full[p] = INFINITY;
    minT_any[p] = INFINITY;
    s->E[p] = 0.0;
    s->fssum[p] = 0.0;
    if (with_mes) {
      s->Fx[p] = 0.0;
      s->Fy[p] = 0.0;
      s->Tz[p] = 0.0;
      s->Fabs[p] = 0.0;
    }
  }
  double cvs = cv_solid(s);
  for (size_t c = 0; c < nc; ++c) {
    int i = (int)(c % (size_t)d->nx), j = (int)(c / (size_t)d->nx);
    for (int k = 0; k < s->cnt[c]; ++k) {
      size_t sl = c * K + k;
      int p = s->ids[sl];
      double w = s->fsp[sl];
      sT[p] += w * s->T[c];
      s->E[p] += w * cvs * s->T[c];
      s->fssum[p] += w;
      if (s->T[c] < minT_any[p]) minT_any[p] = s->T[c];
      if (s->full[sl] && s->T[c] < minT_full[p]) minT_full[p] = s->T[c];
      if (with_mes) {
        /* F_MES = -sum_x sum_i (f_i - f*_i) e_i, T_MES likewise with the
         * lever arm x - X_c (dx^D/dt = 1) */
        double Xi = min_image(s->X[p], i + 0.5, d->nx, per_x(s));
        double Yi = min_image(s->Y[p], j + 0.5, d->ny, per_y(s));
        double rx = (i + 0.5) - Xi, ry = (j + 0.5) - Yi;
        s->Fx[p] -= s->dPx[sl];
        s->Fy[p] -= s->dPy[sl];
        s->Tz[p] -= rx * s->dPy[sl] - ry * s->dPx[sl];
        s->Fabs[p] += fabs(s->dPx[sl]) + fabs(s->dPy[sl]);
      }
    }
  }
  for (int p = 0; p < np; ++p) {
    s->Tmean[p] = s->fssum[p] > 0.0 ? sT[p] / s->fssum[p] : 0.0;
    s->Tmin[p] = isfinite(minT_full[p]) ? minT_full[p] : minT_any[p];
  }
  free(sT);
  free(minT_full);
  free(minT_any);
}

/* ------------------------------------------------------------------ */

int or_init(or_state* s) {
  if (!s) return OR_EINVAL;
  const or_domain* d = &s->dom;
  size_t nc = (size_t)d->nx * d->ny;
  int K = s->kmax;
  s->step = 0;
  s->overlaps = 0;
  for (int p = 0; p < s->np; ++p) {
    s->Uxp[p] = s->Ux[p];
    s->Uyp[p] = s->Uy[p];
    s->Omp[p] = s->Om[p];
    s->Fx[p] = s->Fy[p] = s->Tz[p] = 0.0;
  }
  int st = OR_OK;
  if (s->hk.fs_from_array) {
    memset(s->cnt, 0, sizeof(int) * nc);
    memcpy(s->fs, s->fs_next, sizeof(double) * nc);
  } else {
    st = geometry(s, s->fs);
    if (st != OR_OK) return st;
  }
  double cvf = d->cv_f, cvs = cv_solid(s), cref = c_ref(s);
  /* Reading of the initial state: rho = rho_0 (situation II of Sec. 3.2:
   * the hydrostatic rho_0 + 3 rho_f g.(x - x_m), from grad p = rho_f g
   * with p = rho c_s^2, c_s^2 = 1/3, for the constant force density rho_f
   * g on the fluid, x_m the domain's centre; the paper asks only that the
   * initialisation consider the pressure gradient); u and the internal
   * energy are the volume-weighted mixtures of the fluid and particle
   * values; f = f^eq(rho, u), g = g^eq(eps, T) are taken as the
   * post-collision populations at n = 0; [df_s/dt] = q_c = 0. */
  for (size_t c = 0; c < nc; ++c) {
    double fs = s->fs[c];
    double rho0 = d->init_rho;
    if (d->fluid_gravity) {
      int ci = (int)(c % (size_t)d->nx), cj = (int)(c / (size_t)d->nx);
      double hx = (ci + 0.5) - 0.5 * d->nx, hy = (cj + 0.5) - 0.5 * d->ny;
      rho0 = d->init_rho +
             3.0 * d->rho_f * (d->gravity[0] * hx + d->gravity[1] * hy);
    }
    double ux, uy, T, eps;
    double cv = (1.0 - fs) * cvf + fs * cvs;
    if (s->hk.fs_from_array) {
      ux = s->hk.u_pres[0];
      uy = s->hk.u_pres[1];
      T = s->T[c];        /* caller-written initial temperature */
      eps = cv * T;
    } else {
      ux = (1.0 - fs) * d->init_u[0];
      uy = (1.0 - fs) * d->init_u[1];
      eps = (1.0 - fs) * cvf * d->init_T;
      for (int k = 0; k < s->cnt[c]; ++k) {
        size_t sl = c * K + k;
        int p = s->ids[sl];
        ux += s->fsp[sl] * s->usx[sl];
        uy += s->fsp[sl] * s->usy[sl];
        eps += s->fsp[sl] * cvs * s->Tp0[p];
      }
      T = eps / cv;
      if (s->hk.thermal_only) {
        ux = s->hk.u_pres[0];
        uy = s->hk.u_pres[1];
      }
    }
    double feq[Q], n[Q], geq[Q];
    feq_velocity(s->Minv, rho0, ux, uy, feq);
    neq_energy(eps, T, cref, n);
    mat_vec(s->Minv, n, geq);
    for (int q = 0; q < Q; ++q) {
      s->f[q * nc + c] = feq[q];
      s->g[q * nc + c] = geq[q];
    }
    s->dfs[c] = 0.0;
    s->rho[c] = rho0;
    s->ux[c] = ux;
    s->uy[c] = uy;
    s->T[c] = T;
    s->eps[c] = eps;
    s->qc[c] = 0.0;
  }
  particle_sums(s, 0);
  return OR_OK;
}

int or_step(or_state* s, int64_t nsteps) {
  if (!s || nsteps < 0) return OR_EINVAL;
  const or_domain* d = &s->dom;
  int nx = d->nx, ny = d->ny;
  size_t nc = (size_t)nx * ny;
  double* fs_new = (double*)zalloc(sizeof(double) * nc);
  if (!fs_new) return OR_ENOMEM;
  int status = OR_OK;
  for (int64_t it = 0; it < nsteps && status == OR_OK; ++it) {
    /* stage 1 */
    if (!s->hk.fs_from_array && s->np > 0) particle_update(s);
    /* stage 2: f_s at n+1 from the updated particle positions */
    if (s->hk.fs_from_array) {
      memcpy(fs_new, s->fs_next, sizeof(double) * nc);
    } else {
      status = geometry(s, fs_new);
      if (status != OR_OK) break;
    }
    /* stage 3: eq. dfs_dt, d^{n+1} = 2 (f_s^{n+1} - f_s^n)/dt - d^n */
    for (size_t c = 0; c < nc; ++c) {
      if (s->hk.dfs_backward)
        s->dfs[c] = fs_new[c] - s->fs[c];
      else
        s->dfs[c] = 2.0 * (fs_new[c] - s->fs[c]) - s->dfs[c];
      s->fs[c] = fs_new[c];
    }
    /* stage 4 */
    stream(s);
    /* stages 5-9 */
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i)
        if (update_cell(s, (size_t)j * nx + i, i, j) != OR_OK) bad |= 1;
    if (bad) status = OR_EUNSTABLE;
    /* stage 10 and the momentum-exchange sums */
    particle_sums(s, !s->hk.thermal_only);
    s->step++;
  }
  free(fs_new);
  return status;
}

int or_read_particles(or_state* s, int32_t n, or_particle_state* out) {
  if (!s || !out || n < 0 || n > s->np) return OR_EINVAL;
  for (int p = 0; p < n; ++p) {
    or_particle_state* o = &out[p];
    o->x = s->X[p];
    o->y = s->Y[p];
    o->theta = s->th[p];
    o->ux = s->Ux[p];
    o->uy = s->Uy[p];
    o->omega = s->Om[p];
    o->Fx = s->Fx[p];
    o->Fy = s->Fy[p];
    o->Tz = s->Tz[p];
    o->T_mean = s->Tmean[p];
    o->T_min = s->Tmin[p];
    o->E_solid = s->E[p];
    o->fs_sum = s->fssum[p];
    o->F_abs = s->Fabs[p];
  }
  return OR_OK;
}
