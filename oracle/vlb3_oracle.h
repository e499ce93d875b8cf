/*
 * vlb3_oracle.h -- plain FP64 CPU oracle of the three-dimensional version of
 * the volumetric lattice Boltzmann step for thermal particulate flow with
 * conjugate heat transfer (arXiv 2410.23802; the paper states that the
 * extension to three dimensions is straightforward, Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product library
 * never includes, links or calls anything here, and this file shares no
 * code, header or table with it.
 *
 * Lattice units: dx = dt = c = 1.  Cell (i, j, k) covers [i, i+1] x
 * [j, j+1] x [k, k+1]; its node is the cell centre.  Arrays are [k][j][i]
 * (x fastest); populations are [q][k][j][i].  Flow: D3Q19 MRT; energy:
 * D3Q7; particles: spheres.  The readings that carry the two-dimensional
 * scheme to three dimensions are stated in vlb3_oracle.c.
 */
#ifndef VLB3_ORACLE_H
#define VLB3_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  O3_XLO = 0, O3_XHI = 1, O3_YLO = 2, O3_YHI = 3, O3_ZLO = 4, O3_ZHI = 5
};
enum { O3_PERIODIC = 0, O3_WALL = 1 };
enum { O3_ADIABATIC = 0, O3_DIRICHLET = 1 };
enum {
  O3_OK = 0, O3_EINVAL = -1, O3_ENOMEM = -2, O3_EUNSTABLE = -4,
  O3_EOVERLAP = -5
};

typedef struct {
  int32_t nx, ny, nz;
  int32_t face_flow[6];      /* O3_PERIODIC (in pairs) or O3_WALL          */
  double  u_wall[6][3];      /* wall velocity (moving wall)                */
  int32_t face_thermal[6];   /* O3_ADIABATIC or O3_DIRICHLET (walls only)  */
  double  T_wall[6];
  double  tau_f;             /* flow relaxation time, s_nu = 1/tau_f       */
  double  rho_f, cv_f, lambda_f;
  double  R_lambda, R_cv;    /* solid/fluid conductivity and heat capacity */
  double  body_force[3];     /* external force density on the fluid        */
  double  gravity[3];
  double  beta, T_ref;       /* Boussinesq buoyancy -rho_f g beta (T-T_ref) */
  int32_t sigma_rule;        /* 0: (1/sj-1/2)(1/se-1/2)=1/4; 1: se = 1     */
  double  coll_range, coll_stiff_pp, coll_stiff_pw;
  double  init_rho, init_u[3], init_T;
  int32_t kmax;              /* max particles touching one cell            */
} o3_domain;

typedef struct {
  double x, y, z, ux, uy, uz, ox, oy, oz;   /* centre, velocity, spin      */
  double radius, rho_s, T_init;
  int32_t fixed;             /* 1: velocity and spin prescribed            */
} o3_particle;

typedef struct {
  double x, y, z, ux, uy, uz, ox, oy, oz;
  double Fx, Fy, Fz, Tx, Ty, Tz;            /* momentum-exchange sums      */
  double T_mean, T_min, E_solid, fs_sum;
  double F_abs;  /* sum over the particle's cells of f_s,p sum_i |f^eq_i +
                    f*_i|: the size of the populations the sums cancel     */
} o3_particle_state;

/* Switches for the conduction tests: thermal_only freezes the flow at
 * u = u_pres, fs_from_array takes f_s from a caller-written field (no
 * particles) and T from the caller-written T field at init. */
typedef struct {
  int32_t thermal_only;
  double  u_pres[3];
  int32_t fs_from_array;
} o3_hooks;

typedef struct o3_state o3_state;

int o3_create(const o3_domain* d, int32_t np, const o3_particle* p,
              o3_state** out);
int o3_set_hooks(o3_state* s, const o3_hooks* h);
int o3_init(o3_state* s);
int o3_step(o3_state* s, int64_t nsteps);
void o3_destroy(o3_state* s);
int o3_read_particles(o3_state* s, int32_t n, o3_particle_state* out);

/* Field views (owned by the state). */
double* o3_f(o3_state* s);      /* [19][nz][ny][nx] post-collision */
double* o3_g(o3_state* s);      /* [7][nz][ny][nx]                 */
double* o3_d(o3_state* s);      /* [df_s/dt]                       */
double* o3_fs(o3_state* s);
double* o3_rho(o3_state* s);
double* o3_ux(o3_state* s);
double* o3_uy(o3_state* s);
double* o3_uz(o3_state* s);
double* o3_T(o3_state* s);
double* o3_fs_next(o3_state* s);  /* caller-written f_s (hook) */
int32_t* o3_own_count(o3_state* s);
int32_t* o3_own_ids(o3_state* s);    /* [cell][kmax] */

/* Volume of the sphere (centre, radius R) inside the unit cell with lower
 * corner (x0, y0, z0). */
double o3_sphere_cell_volume(double cx, double cy, double cz, double R,
                             double x0, double y0, double z0);
/* Ownership predicates (integer work, no fused operations). */
int o3_cell_in_band(double X, double Y, double Z, double R, int32_t i,
                    int32_t j, int32_t k);
int o3_cell_inside(double X, double Y, double Z, double R, int32_t i,
                   int32_t j, int32_t k);

#ifdef __cplusplus
}
#endif
#endif
