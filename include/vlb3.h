/*
 * vlb3.h -- C ABI of the three-dimensional version of the MI355X (gfx950)
 * volumetric lattice Boltzmann solver for particle-resolved thermal
 * particulate flow with conjugate heat transfer (arXiv 2410.23802; the
 * paper develops the method in two dimensions and states that its
 * extension to three is straightforward, Sec. 2).
 *
 * One call of vlb3_step advances the same per-time-step update as vlb_step
 * (include/vlb.h) in three dimensions:
 *   - the Newton-Euler update of every sphere with the inside-fluid terms
 *     and the short-range repulsion (Sec. 2.3, eq. particle,
 *     eq. inside.fluid; I = 2 M R^2/5);
 *   - the solid fraction f_s of every cell as the exact volume of the
 *     spheres inside it, and u_s = U + Omega x (x - X) (Sec. 2, eq. us);
 *   - the flow lattice, D3Q19 with the MRT collision of eq. lbe.rho.col (the
 *     orthogonal D3Q19 moment basis; m^eq and F_m the moments of the
 *     textbook equilibrium and of Guo's force term) and the volumetric
 *     no-slip step f = (1 - f_s) f* + sum_p f_s,p f^eq(rho, u_s,p) (eq. fi);
 *   - the energy lattice, D3Q7, in the two-rate form that the paper's
 *     two-dimensional energy collision takes with its parameters (even part
 *     relaxed at sigma_e, odd part at sigma_j = 1/tau_g, the source q_c on
 *     the rest population), with the per-cell c_v, lambda, tau_g
 *     (lambda/rho_f = c_s^2 c_ref (tau_g - 1/2), c_s^2 = 1/4), the local
 *     temperature gradient, the convection-as-source term and the
 *     [df_s/dt] recursion (Sec. 2.2, eq. lbe.e, eq. e, eq. dfs_dt);
 *   - the per-sphere momentum-exchange force and torque (Sec. 2.3).
 *
 * Units: lattice units, dx = dt = c = 1.  Cell (i, j, k) covers [i, i+1] x
 * [j, j+1] x [k, k+1]; its node is the cell centre.  Fields are [k][j][i]
 * (x fastest).  D3Q19 order: e_0 = 0; e_1..6 = +x, -x, +y, -y, +z, -z;
 * e_7..18 = (1,1,0), (-1,-1,0), (1,-1,0), (-1,1,0), (1,0,1), (-1,0,-1),
 * (1,0,-1), (-1,0,1), (0,1,1), (0,-1,-1), (0,1,-1), (0,-1,1); D3Q7 takes
 * e_0..6.
 *
 * Status codes, threading and memory ownership as in vlb.h: every call
 * returns a vlb_status; vlb3_last_error() describes the last failure on a
 * context; calls on one context must not overlap; the library owns all
 * device memory of a context; descriptors are copied at the call.
 */
#ifndef VLB3_H
#define VLB3_H

#include <stddef.h>
#include <stdint.h>

#include "vlb.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { VLB3_FACE_XLO = 0, VLB3_FACE_XHI = 1, VLB3_FACE_YLO = 2,
       VLB3_FACE_YHI = 3, VLB3_FACE_ZLO = 4, VLB3_FACE_ZHI = 5 };

/* Domain descriptor.  Walls lie on the outer cell faces (halfway
 * bounce-back; a moving wall adds 6 w_i rho_0 e_i.u_wall); thermal walls
 * are adiabatic (bounce-back of g) or held at T_wall (anti-bounce-back).
 * Where a population's upstream point lies beyond two or three walls, the
 * z wall decides, then the y wall. */
typedef struct {
  int32_t nx, ny, nz;        /* cells; each >= 1; nx*ny*nz < 2^31           */
  int32_t face_flow[6];      /* VLB_PERIODIC (in pairs) or VLB_WALL          */
  double  u_wall[6][3];      /* wall velocity                                */
  int32_t face_thermal[6];   /* VLB_ADIABATIC or VLB_DIRICHLET               */
  double  T_wall[6];
  double  tau_f;             /* flow relaxation time (> 1/2); the shear rate
                                1/tau_f, nu = (tau_f - 1/2)/3                */
  double  rho_f, cv_f, lambda_f;   /* fluid density, specific heat,
                                      conductivity                          */
  double  R_lambda, R_cv;    /* solid/fluid conductivity and heat capacity   */
  double  body_force[3];     /* external force density on the fluid          */
  double  gravity[3];        /* on the spheres (net of buoyancy) and in the
                                Boussinesq buoyancy -rho_f g beta (T - T_ref)
                                of the fluid                                 */
  double  beta, T_ref;
  int32_t sigma_rule;        /* 0: (1/sigma_j - 1/2)(1/sigma_e - 1/2) = 1/4;
                                1: sigma_e = 1                               */
  double  coll_range;        /* repulsion range zeta (0: none)               */
  double  coll_stiff_pp;     /* sphere-sphere force at contact               */
  double  coll_stiff_pw;     /* sphere-wall force at contact                 */
  double  init_rho, init_u[3], init_T;   /* initial fluid state              */
  int32_t kmax;              /* max spheres touching one cell, 1..4          */
  int32_t precision;         /* storage of the populations and the carrier:
                                VLB_FP64, or VLB_FP32 (deviations from the
                                equilibria of the initial state at rest);
                                the arithmetic is FP64 in both            */
} vlb3_domain_desc;

/* A sphere.  fixed = 1: velocity and spin prescribed (not integrated). */
typedef struct {
  double  x, y, z, ux, uy, uz, ox, oy, oz;   /* centre, velocity, spin      */
  double  radius, rho_s, T_init;
  int32_t fixed;
} vlb3_sphere_desc;

/* State and outputs of a sphere after the last step: centre, velocity,
 * spin, the momentum-exchange force and torque of that step, the mean and
 * minimal temperature (over the cells wholly inside, else over all it
 * reaches), sum f_s,p c_v,s T and sum f_s,p. */
typedef struct {
  double x, y, z, ux, uy, uz, ox, oy, oz;
  double Fx, Fy, Fz, Tx, Ty, Tz;
  double T_mean, T_min, E_solid, fs_sum;
} vlb3_sphere_state;

typedef struct vlb3_ctx vlb3_ctx;

/* Create a domain with nspheres in 0..64 spheres (host memory, copied; may
 * be NULL when nspheres is 0) on the given HIP stream (NULL: the library
 * creates one of default priority).  VLB_EINVAL for a bad descriptor or
 * sphere (the message names the field), VLB_ENOMEM when device memory does
 * not suffice. */
vlb_status vlb3_create(const vlb3_domain_desc* desc, int32_t nspheres,
                       const vlb3_sphere_desc* spheres, void* hip_stream,
                       vlb3_ctx** out);

/* Initial state: equilibria of the volume-weighted mixture of the fluid
 * and sphere states in every cell, [df_s/dt] = 0. */
vlb_status vlb3_init(vlb3_ctx* ctx);

/* Advance nsteps >= 0 steps.  VLB_EUNSTABLE / VLB_EOVERLAP as in vlb.h;
 * the context must then be initialised again. */
vlb_status vlb3_step(vlb3_ctx* ctx, int64_t nsteps);

enum { VLB3_RHO = 0, VLB3_UX = 1, VLB3_UY = 2, VLB3_UZ = 3, VLB3_T = 4,
       VLB3_FS = 5, VLB3_DFS = 6 };

/* Copy a field of the last step (nx*ny*nz doubles, [k][j][i]) to dst, host
 * memory or (dst_is_device) device memory of the context's device. */
vlb_status vlb3_read_field(vlb3_ctx* ctx, int32_t field, double* dst,
                           int32_t dst_is_device);

/* Copy the post-collision populations: which = 0 the 19 flow planes,
 * 1 the 7 energy planes ([q][k][j][i], host memory, FP64; the FP32 storage
 * form's values with its reference added back). */
vlb_status vlb3_read_populations(vlb3_ctx* ctx, int32_t which, double* dst);

/* The first n spheres' states (n <= the count; host memory). */
vlb_status vlb3_read_spheres(vlb3_ctx* ctx, int32_t n, vlb3_sphere_state* dst);

/* Checkpoint, as vlb_save / vlb_load: vlb3_save writes the complete state
 * (populations and carrier in the storage form, macroscopic fields, the
 * spheres' state, the last step's momentum-exchange partial sums and tile
 * candidate masks, the step counter) into buf; with buf == NULL it only
 * stores the needed size in *inout_len.  vlb3_load restores a buffer written
 * by vlb3_save for a context created with the same descriptor and spheres;
 * stepping after a load continues bit for bit.  VLB_EINVAL for a buffer
 * that is too short or does not match the context. */
vlb_status vlb3_save(vlb3_ctx* ctx, void* buf, size_t* inout_len);
vlb_status vlb3_load(vlb3_ctx* ctx, const void* buf, size_t len);

/* Kernel timing, as vlb_timing_enable / vlb_timing_read: while enabled,
 * every launch of the step kernel is bracketed by HIP events on the context
 * stream; read returns the summed duration (ms) and the count, and resets
 * them. */
vlb_status vlb3_timing_enable(vlb3_ctx* ctx, int32_t on);
vlb_status vlb3_timing_read(vlb3_ctx* ctx, double* total_ms, int64_t* count);

int64_t vlb3_step_count(const vlb3_ctx* ctx);
size_t vlb3_device_bytes(const vlb3_ctx* ctx);

/* Message for the last failing call on ctx (or on creation when NULL). */
const char* vlb3_last_error(const vlb3_ctx* ctx);

/* Free the context (NULL is ignored). */
void vlb3_destroy(vlb3_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
