/*
 * vlb_oracle.h -- plain FP64 CPU oracle of the volumetric lattice Boltzmann
 * step for thermal particulate flow with conjugate heat transfer
 * (Zhang, Wang, Li, Huang, arXiv 2410.23802).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product library
 * (include/vlb.h) never includes, links or calls anything here, and this
 * file shares no code, header or table with it.
 *
 * Everything is in lattice units: dx = dt = c = 1, c_s^2 = 1/3.
 * Coordinates: cell (i, j) covers [i, i+1] x [j, j+1]; its node is the
 * cell centre (i + 1/2, j + 1/2) (volumetric interpretation, Sec. 2, Fig. 1).
 * Arrays are row-major [j][i] (x fastest); populations are [q][j][i].
 */
#ifndef VLB_ORACLE_H
#define VLB_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_FACE_XLO = 0, OR_FACE_XHI = 1, OR_FACE_YLO = 2, OR_FACE_YHI = 3 };
enum { OR_PERIODIC = 0, OR_WALL = 1 };           /* flow type of a face     */
enum { OR_ADIABATIC = 0, OR_DIRICHLET = 1 };     /* thermal type of a wall  */

enum {
  OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2, OR_EUNSTABLE = -4,
  OR_EOVERLAP = -5
};

typedef struct {
  int32_t nx, ny;
  int32_t face_flow[4];      /* OR_PERIODIC (must pair) or OR_WALL          */
  double  u_wall[4][2];      /* tangential wall velocity (moving wall)      */
  int32_t face_thermal[4];   /* OR_ADIABATIC or OR_DIRICHLET (walls only)   */
  double  T_wall[4];
  double  tau_f;             /* flow relaxation time, s_p = 1/tau_f         */
  double  rho_f;             /* fluid density (inside-fluid mass, buoyancy) */
  double  cv_f;              /* fluid specific heat                          */
  double  lambda_f;          /* fluid conductivity                           */
  double  R_lambda, R_cv;    /* solid/fluid conductivity and heat capacity   */
  double  body_force[2];     /* external force density on the fluid          */
  double  gravity[2];
  double  beta, T_ref;       /* Boussinesq buoyancy -rho_f g beta (T-T_ref)  */
  int32_t sigma_rule;        /* 0: (1/sj-1/2)(1/se-1/2)=1/4; 1: se=1         */
  int32_t fluid_gravity;     /* 1: situation II of Sec. 3.2                  */
  double  coll_range;        /* repulsion range zeta (cells)                 */
  double  coll_stiff_pp;     /* particle-particle force at contact           */
  double  coll_stiff_pw;     /* particle-wall force at contact               */
  double  init_rho, init_u[2], init_T;   /* initial fluid state              */
  int32_t kmax;              /* max particles touching one cell              */
} or_domain;

typedef struct {
  double x, y, theta, ux, uy, omega, radius, rho_s, T_init;
  double radius_minor;       /* 0 or radius: a disk; 0 < radius_minor <
                                radius: an ellipse of semi-axes radius and
                                radius_minor, its major axis at theta        */
  int32_t fixed;             /* 1: velocity prescribed (not integrated)      */
  int32_t hold_T;            /* 1: temperature held at T_init (stage 5b)     */
} or_particle;

/* Per-particle state and outputs (stage 10 of a step). */
typedef struct {
  double x, y, theta, ux, uy, omega;
  double Fx, Fy, Tz;         /* momentum-exchange force / torque (MES)       */
  double T_mean, T_min, E_solid, fs_sum;
  double F_abs;              /* sum over cells of |share of sum_i (f_i - f*_i) e_i|
                                (x and y added): the size of the terms the
                                momentum-exchange sum adds up               */
} or_particle_state;

/* Switches that exist only to plant the paper's own negative controls
 * (Appendix A) and to drive the 1-D conjugate-heat-transfer tests of
 * Sec. 3.1, in which the velocity field is prescribed. */
typedef struct {
  double  beta1;             /* source weight of moment 1; the paper: -4     */
  int32_t dfs_backward;      /* 1: backward difference for dfs/dt (wrong)    */
  int32_t thermal_only;      /* 1: skip the flow LB, u = u_pres everywhere   */
  double  u_pres[2];
  int32_t fs_from_array;     /* 1: f_s^{n+1} comes from or_fs_next()         */
} or_hooks;

typedef struct or_state or_state;

int  or_create(const or_domain* d, int32_t np, const or_particle* p,
               or_state** out);
void or_destroy(or_state* s);
void or_default_hooks(or_hooks* h);
int  or_set_hooks(or_state* s, const or_hooks* h);
int  or_init(or_state* s);
int  or_step(or_state* s, int64_t nsteps);
int  or_set_threads(int n);
int64_t or_step_count(const or_state* s);

/* Raw arrays (owned by the state, valid until or_destroy). */
double* or_f(or_state* s);        /* post-collision f, [9][ny][nx]          */
double* or_g(or_state* s);        /* post-collision g, [9][ny][nx]          */
double* or_d(or_state* s);        /* [dfs/dt] at the current step           */
double* or_fs(or_state* s);       /* total solid fraction at current step   */
double* or_rho(or_state* s);      /* macroscopic fields at current step     */
double* or_ux(or_state* s);
double* or_uy(or_state* s);
double* or_T(or_state* s);
double* or_eps(or_state* s);      /* internal energy eps = c_v T            */
double* or_qc(or_state* s);       /* source q_c                             */
double* or_fs_next(or_state* s);  /* written by the caller when hooked      */
int32_t* or_own_count(or_state* s);   /* particles touching each cell       */
int32_t* or_own_ids(or_state* s);     /* [ny][nx][kmax], sorted, -1 padded  */
int32_t* or_own_full(or_state* s);    /* [ny][nx][kmax] 1: cell inside disk */
int  or_read_particles(or_state* s, int32_t n, or_particle_state* out);
int  or_overlap_count(const or_state* s);

/* Geometry primitives, exposed for the geometry pins. */
double or_disk_cell_area(double cx, double cy, double R, double x0, double y0);
double or_ellipse_cell_area(double cx, double cy, double a, double b,
                            double th, double x0, double y0);
int    or_cell_in_band(double X, double Y, double R, int32_t i, int32_t j);
int    or_cell_inside(double X, double Y, double R, int32_t i, int32_t j);

/* Particle-pair and wall repulsion on particle i (exposed for tests). */
int  or_collision_force(const or_state* s, int32_t i, double* fx, double* fy);

#ifdef __cplusplus
}
#endif
#endif
