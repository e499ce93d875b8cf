/*
 * vlb.h -- C ABI of the MI355X (gfx950) volumetric lattice Boltzmann solver
 * for particle-resolved thermal particulate flow with conjugate heat
 * transfer (Zhang, Wang, Li, Huang, arXiv 2410.23802).
 *
 * One call of vlb_step advances the whole per-time-step update of the paper
 * on the GPU:
 *   - the Newton-Euler particle update with the inside-fluid correction and
 *     a short-range repulsion (Sec. 2.3, eq. particle, eq. inside.fluid);
 *   - the solid fraction f_s of every cell from the disks' exact areas and
 *     the solid velocity u_s (Sec. 2, Fig. 1; eq. us);
 *   - the flow MRT collide-and-stream with the volumetric no-slip step
 *     f = (1 - f_s) f* + f_s f^eq(rho, u_s) (Sec. 2.1, eq. lbe.rho, eq. fi);
 *   - the energy MRT lattice with the convection-as-source term q_c, the
 *     per-cell c_v, lambda and tau_g, the local temperature gradient and the
 *     [df_s/dt] recursion (Sec. 2.2, eq. lbe.e, eq. e, eq. lambda,
 *     eq. dfs_dt);
 *   - the per-particle momentum-exchange force and torque (Sec. 2.3).
 *
 * Units: lattice units, dx = dt = c = 1.  Cell (i, j) covers [i, i+1] x
 * [j, j+1]; its node is the cell centre.  Fields are row-major [j][i]
 * (x fastest), ny rows of nx values; population fields are 9 such planes
 * in the D2Q9 order e_0 = (0,0), e_1..4 = (1,0), (0,1), (-1,0), (0,-1),
 * e_5..8 = (1,1), (-1,1), (-1,-1), (1,-1).
 *
 * Errors: every call returns a vlb_status; no exception crosses the ABI.
 * vlb_last_error() gives a message for the last failing call on a context.
 * Threading: one context per HIP stream; contexts are independent; calls on
 * one context must not overlap.
 * Memory: the library owns all device memory of a context (allocated at
 * vlb_create/vlb_set_particles, freed by vlb_destroy).  Descriptors are
 * copied at the call; caller buffers are only read or written during it.
 */
#ifndef VLB_H
#define VLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VLB_OK = 0,
  VLB_EINVAL = -1,     /* bad argument or descriptor                      */
  VLB_ENOMEM = -2,     /* device or host allocation failed                */
  VLB_EHIP = -3,       /* a HIP runtime call failed                       */
  VLB_EUNSTABLE = -4,  /* a cell reached rho <= 0 or a non-finite value   */
  VLB_EOVERLAP = -5,   /* more than kmax particles in a cell, or a full
                          per-block particle list                          */
  VLB_ESTATE = -6      /* call out of order (e.g. step before init)       */
} vlb_status;

/* Storage of the populations.  FP64 stores f_i and g_i.  FP32, FP16 and
 * BF16 store the deviations f_i - w_i rho_0 and g_i - w_i c_ref T_0
 * (rho_0 = shift_rho0, T_0 = shift_T0) and compute on deviations in FP32;
 * the per-particle sums and the particle integration are FP64 in every
 * form. */
typedef enum {
  VLB_FP64 = 0,
  VLB_FP32 = 1,
  VLB_FP16_SHIFT = 2,
  VLB_BF16_SHIFT = 3
} vlb_precision;

enum { VLB_FACE_XLO = 0, VLB_FACE_XHI = 1, VLB_FACE_YLO = 2, VLB_FACE_YHI = 3 };
enum { VLB_PERIODIC = 0, VLB_WALL = 1 };         /* flow type of a face      */
enum { VLB_ADIABATIC = 0, VLB_DIRICHLET = 1 };   /* thermal type of a wall   */

/* Domain descriptor.  Walls lie on the outer cell faces (halfway
 * bounce-back; a moving wall adds 6 w_i rho_0 e_i.u_wall); thermal walls are
 * adiabatic (bounce-back of g) or held at T_wall (anti-bounce-back). */
typedef struct {
  int32_t nx, ny;            /* cells; 1 <= nx, ny; nx*ny < 2^31             */
  int32_t face_flow[4];      /* VLB_PERIODIC (in pairs) or VLB_WALL           */
  double  u_wall[4][2];      /* wall velocity (tangential component used)     */
  int32_t face_thermal[4];   /* VLB_ADIABATIC or VLB_DIRICHLET                */
  double  T_wall[4];
  double  tau_f;             /* flow relaxation time, nu = (tau_f - 1/2)/3    */
  double  rho_f;             /* fluid density: inside-fluid mass, buoyancy    */
  double  cv_f;              /* fluid specific heat                           */
  double  lambda_f;          /* fluid conductivity                            */
  double  R_lambda, R_cv;    /* solid/fluid conductivity, specific heat       */
  double  body_force[2];     /* external force density on the fluid share     */
  double  gravity[2];        /* g: particles feel (rho_s - rho_f) V g, the
                                fluid the buoyancy -rho_f g beta (T - T_ref)  */
  double  beta, T_ref;
  int32_t sigma_rule;        /* 0: (1/sigma_j - 1/2)(1/sigma_e - 1/2) = 1/4;
                                1: sigma_e = 1 (the dense case of Sec. 3.5)   */
  int32_t fluid_gravity;     /* 0: situation I of Sec. 3.2 (gravity as above);
                                1: situation II: the fluid's share also
                                carries rho_f g, the particles feel
                                rho_s V g, and the initial density is the
                                hydrostatic rho_0 + 3 rho_f g.(x - centre)  */
  double  coll_range;        /* repulsion range zeta; 0 disables collisions   */
  double  coll_stiff_pp;     /* particle-particle repulsion at contact        */
  double  coll_stiff_pw;     /* particle-wall repulsion at contact            */
  double  init_rho, init_u[2], init_T;   /* initial fluid state               */
  int32_t kmax;              /* max particles touching one cell (1..8)        */
  int32_t precision;         /* vlb_precision                                 */
  double  shift_rho0;        /* rho_0 of the deviation storage (not FP64)     */
  double  shift_T0;          /* T_0 of the deviation storage (not FP64)       */
} vlb_domain_desc;

typedef struct {
  double x, y;               /* centre                                        */
  double theta;              /* orientation: the major axis's angle to the x
                                axis (integrated; not used by a disk)        */
  double ux, uy, omega;      /* initial velocity and angular velocity         */
  double radius;             /* 0 < radius <= 28                              */
  double rho_s;              /* solid density                                 */
  double T_init;             /* initial particle temperature                  */
  double radius_minor;       /* 0 (or radius): a disk of the given radius;
                                0 < radius_minor < radius: an ellipse of
                                semi-axes radius and radius_minor whose major
                                axis makes the angle theta with the x axis
                                (Sec. 3.2).  An ellipse's band of cells is
                                that of its circumscribed disk, and a cell is
                                wholly inside when its inscribed disk holds
                                it; its share of a cell is the exact area     */
  int32_t fixed;             /* 1: velocity held (prescribed motion)          */
  int32_t hold_T;            /* 1: temperature held at T_init (a particle of
                                fixed temperature, Sec. 3.3; the rule that
                                holds it is this library's reading: the
                                energy populations of the cells it covers
                                take the volumetric step, share-weighted,
                                towards their equilibrium at T_init)          */
} vlb_particle_desc;

typedef struct {
  double x, y, theta, ux, uy, omega;
  double Fx, Fy, Tz;         /* momentum-exchange force and torque of the
                                current step (Sec. 2.3)                        */
  double T_mean;             /* sum f_s,p T / sum f_s,p                        */
  double T_min;              /* min T over cells wholly inside the disk        */
  double E_solid;            /* sum f_s,p c_vs T                               */
  double fs_sum;             /* sum f_s,p                                      */
} vlb_particle_state;

/* Fields for vlb_read_field.  Scalar fields write nx*ny doubles; the
 * population fields write 9*nx*ny doubles (post-collision, unshifted). */
enum {
  VLB_FIELD_RHO = 0, VLB_FIELD_UX = 1, VLB_FIELD_UY = 2, VLB_FIELD_T = 3,
  VLB_FIELD_FS = 4,    /* total solid fraction                              */
  VLB_FIELD_DFS = 5,   /* [df_s/dt] of eq. dfs_dt                           */
  VLB_FIELD_F = 6, VLB_FIELD_G = 7
};

typedef struct vlb_ctx vlb_ctx;

/* Create a context for one domain on the current HIP device.  hip_stream is
 * a hipStream_t (NULL: the default stream); all work of the context runs on
 * it.  Validates the descriptor (VLB_EINVAL) and allocates the populations,
 * the [df_s/dt] carrier and the per-block particle lists (VLB_ENOMEM). */
vlb_status vlb_create(const vlb_domain_desc* desc, void* hip_stream,
                      vlb_ctx** out);

/* Set the particles (n >= 0 descriptors, host memory, copied).  Must precede
 * vlb_init; replaces any previous set.  VLB_EINVAL for a bad radius/density
 * or a disk that does not fit a periodic axis. */
vlb_status vlb_set_particles(vlb_ctx* ctx, int32_t n,
                             const vlb_particle_desc* p);

/* Initial state (n = 0): rho = init_rho; u and the internal energy are the
 * volume-weighted mixtures of fluid and particle values per cell; f = f^eq,
 * g = g^eq are the post-collision populations; [df_s/dt] = 0; the
 * momentum-exchange force is zero.  Synchronous. */
vlb_status vlb_init(vlb_ctx* ctx);

/* Advance nsteps >= 0 time steps (each: particle update, solid fraction,
 * stream, volumetric step, momentum exchange, macroscopic solve, both
 * collisions).  Returns after the stream has drained; VLB_EUNSTABLE or
 * VLB_EOVERLAP if any step flagged it (the state is then not meaningful).
 * The last step also stores the macroscopic fields read by vlb_read_field. */
vlb_status vlb_step(vlb_ctx* ctx, int64_t nsteps);

/* Copy a field of the current step into dst (host memory if dst_is_device is
 * 0, else a device pointer on the context's device; the copy is ordered on
 * the context stream and complete on return). */
vlb_status vlb_read_field(vlb_ctx* ctx, int32_t field, double* dst,
                          int32_t dst_is_device);

/* Per-particle state of the current step for the first n particles (host
 * buffer of n entries).  Computes the thermal sums on the GPU. */
vlb_status vlb_read_particles(vlb_ctx* ctx, int32_t n,
                              vlb_particle_state* dst);

/* Cell ownership of the current step (integer work): count[nx*ny] particles
 * touching each cell, ids[nx*ny*kmax] their indices ascending (-1 padded),
 * full[nx*ny*kmax] 1 where the cell lies wholly inside that disk.  A cell is
 * touched when its closed square meets the open disk.  Host buffers. */
vlb_status vlb_read_ownership(vlb_ctx* ctx, int32_t* count, int32_t* ids,
                              int32_t* full);

/* vlb_read_ownership for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same outputs, bit for bit, with no hipMalloc, hipFree or other
 * allocation.  The kernels stage their results in a 16 MiB array in device
 * memory that the library holds on every GPU it runs on until the process
 * ends; the domain is read in chunks of whole 256-cell tiles that fit it
 * (at most 963 tiles per chunk at kmax = 8), so no domain size is refused.
 * The array is shared by every call on a GPU and keeps the last call's
 * contents (each call overwrites every entry it copies out): calls that
 * overlap on one GPU, from any context or thread, race and must be
 * serialised by the caller.  count, ids, full: host buffers as for
 * vlb_read_ownership.  VLB_EHIP if the array's device address cannot be
 * obtained on the context's device. */
vlb_status vlb_read_ownership_noalloc(vlb_ctx* ctx, int32_t* count,
                                      int32_t* ids, int32_t* full);

/* Checkpoint: vlb_save writes the complete state (populations, [df_s/dt]
 * carrier, particle state, step counter) into buf.  With buf == NULL it only
 * stores the needed size in *inout_len.  vlb_load restores a buffer written
 * by vlb_save for a context created with the same descriptor and particle
 * count; stepping after a load continues bit for bit. */
vlb_status vlb_save(vlb_ctx* ctx, void* buf, size_t* inout_len);
vlb_status vlb_load(vlb_ctx* ctx, const void* buf, size_t len);

/* Steps taken since vlb_init. */
int64_t vlb_step_count(const vlb_ctx* ctx);

/* Kernel timing: while enabled, every launch of the lattice step kernel
 * (all cells, particle tiles included) is bracketed by HIP events on the
 * context stream; vlb_timing_read returns the summed duration (ms) and the
 * number of launches timed since the last read, then resets. */
vlb_status vlb_timing_enable(vlb_ctx* ctx, int32_t on);
vlb_status vlb_timing_read(vlb_ctx* ctx, double* total_ms, int64_t* count);

/* Memory-pattern probe (measurement support).  Runs `reps` launches of a
 * kernel that moves exactly what one step moves -- per cell the nine f and
 * nine g populations pulled from the neighbours of the streaming step
 * (Sec. 2.1, eq. lbe.rho; Sec. 2.2, eq. lbe.e) over the context's own SoA
 * planes and tile order, plus the [df_s/dt] carrier, read once and written
 * once -- with none of the arithmetic, on the context stream, and stores
 * the average duration of one launch (microseconds) in *us_per_launch.
 * Algorithmic bytes per cell over that duration is the bandwidth the
 * access pattern itself reaches on the device: the ceiling for the step
 * kernel.  It writes only the buffers the next step overwrites in full, so
 * the state is unchanged.  Blocks until done.  VLB_EINVAL for reps <= 0 or
 * a null pointer; VLB_ESTATE before a successful vlb_init. */
vlb_status vlb_stream_probe(vlb_ctx* ctx, int32_t reps, double* us_per_launch);

/* Bytes of device memory the context holds. */
size_t vlb_device_bytes(const vlb_ctx* ctx);

/* Message for the last failing call on ctx (or on creation when ctx is NULL). */
const char* vlb_last_error(const vlb_ctx* ctx);

/* The hash of the sources the library was built from (16 hex digits, a
 * static string): a caller can check that the binary it loaded matches the
 * sources it expects. */
const char* vlb_build_hash(void);

/* Free the context and its device memory (NULL is ignored). */
void vlb_destroy(vlb_ctx* ctx);

/* ------------------------------------------------------------------------
 * Batches: many independent domains (each the problem of Sec. 2 on its own
 * grid, with its own parameters and up to 64 particles) advanced together.
 * One launch of one kernel advances every domain by a step; a fixed set of
 * persistent blocks walks a table of tiles that lists every domain's
 * particle tiles first.  Results of a domain are those the single-domain
 * calls give for it, bit for bit, whatever the batch and the tuning.
 * All domains share one precision and step in lockstep.  The batch owns a
 * HIP stream of default priority; every call is complete on return. */

typedef struct vlb_batch vlb_batch;

/* Launch shape of the batch step kernel.  grid_blocks: persistent blocks, a
 * multiple of 8 (0: one block per task).  order 0: tiles listed domain by
 * domain; 1: tiles dealt to the 8 XCDs in contiguous bands.  use_graph:
 * replay steady-state steps from a captured two-step hipGraph.
 * pair_min_tiles: the tiling of each domain -- a domain of at least this
 * many tiles streams its particle-free tiles two per block (512 cells, two
 * per lane), a smaller one one per block (256 cells); 0 pairs every
 * domain, -1 none.  waves: the occupancy the step kernel is built for, 4
 * waves per SIMD, or 5 for the 32- and 16-bit forms (0: 4 for FP64, 5 for
 * the others).
 * us_per_step: the time vlb_batch_autotune measured for the choice. */
typedef struct {
  int32_t grid_blocks;
  int32_t order;
  int32_t use_graph;
  int32_t pair_min_tiles;
  int32_t waves;
  double  us_per_step;
} vlb_batch_tuning;

/* Create ncases domains: descs[ncases] (copied), nparticles[ncases] in
 * 0..64 disks (no ellipses) and the particles of all domains back to back
 * in `particles`
 * (host memory, copied; may be NULL when every count is 0).  VLB_EINVAL for
 * a bad descriptor (the message names the domain) or mixed precisions,
 * VLB_ENOMEM when the device memory does not suffice. */
vlb_status vlb_batch_create(int32_t ncases, const vlb_domain_desc* descs,
                            const int32_t* nparticles,
                            const vlb_particle_desc* particles,
                            vlb_batch** out);

/* Initial state of every domain (as vlb_init). */
vlb_status vlb_batch_init(vlb_batch* b);

/* Advance every domain by nsteps >= 0 steps.  VLB_EUNSTABLE / VLB_EOVERLAP
 * name the first failing domain in vlb_batch_last_error; the batch must
 * then be initialised again. */
vlb_status vlb_batch_step(vlb_batch* b, int64_t nsteps);

/* Time every candidate tuning over `steps` steps -- grid_blocks 4, 8 and
 * 16 per compute unit and one block per task; both orders; pair_min_tiles
 * -1 (no pairs), the median tile count of the domains (the larger half
 * paired) and 0 (all); waves 4 and 5 (FP64: 4) -- keep the fastest (with
 * use_graph = 1) and initialise the batch again.  Only on a freshly
 * initialised batch (VLB_ESTATE otherwise).  chosen may be NULL.
 * vlb_batch_set_tuning rejects values outside the ranges above
 * (VLB_EINVAL). */
vlb_status vlb_batch_autotune(vlb_batch* b, int32_t steps,
                              vlb_batch_tuning* chosen);
vlb_status vlb_batch_set_tuning(vlb_batch* b, const vlb_batch_tuning* t);
vlb_status vlb_batch_get_tuning(const vlb_batch* b, vlb_batch_tuning* t);

/* Reads of domain i, as vlb_read_field and vlb_read_particles. */
vlb_status vlb_batch_read_field(vlb_batch* b, int32_t i, int32_t field,
                                double* dst, int32_t dst_is_device);
vlb_status vlb_batch_read_particles(vlb_batch* b, int32_t i, int32_t n,
                                    vlb_particle_state* dst);

/* Number of domains; total cells; steps since vlb_batch_init; device
 * bytes held. */
int32_t vlb_batch_size(const vlb_batch* b);
int64_t vlb_batch_cells(const vlb_batch* b);
int64_t vlb_batch_step_count(const vlb_batch* b);
size_t vlb_batch_device_bytes(const vlb_batch* b);

/* Message for the last failing call on b (or on creation when b is NULL). */
const char* vlb_batch_last_error(const vlb_batch* b);

/* Free the batch, its domains and its stream (NULL is ignored). */
void vlb_batch_destroy(vlb_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* VLB_H */
