// vlb_internal.h -- device-side data structures and kernel launchers of the
// MI355X volumetric lattice Boltzmann library (private to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vlb.h"

namespace vlb {

constexpr int kBlock = 256;       // cells per lattice block (one per thread)
constexpr int kListCap = 32;      // particle entries per block list
constexpr int kMaxRadius = 28;    // band rows of one particle fit one wave
constexpr int kRedVals = 3;       // Fx, Fy, Tz per partial slot

enum : int {
  kFlagUnstable = 1,    // rho <= 0 or non-finite value in a cell
  kFlagOverlap = 2,     // more than kmax particles in a cell
  kFlagListFull = 4     // a block list overflowed kListCap
};

// Per-domain constants derived on the host from the descriptor.
struct Params {
  int nx, ny, N, nblocks;
  int perx, pery;
  int kmax, sigma_rule;
  // flow lattice (s_0 = s_j = 1, s_e = s_eps = 1.25; Sec. 3)
  double s_e, s_q, s_p;
  // energy lattice
  double cvf, cvs, dcv, lamf, dlam, cref;
  double taug_coef;   // tau_g = 1/2 + taug_coef * lambda   (eq. lambda)
  // fluid force F = (1 - f_s)(A0 + B0 T)
  double A0x, A0y, B0x, B0y;
  double init_rho, init_ux, init_uy, init_T;
  // wall rules: per face w and direction q, f* = f_opp + fadd[w][q];
  // g = gsign[w] * g_opp + gadd[w][q]
  double fadd[4][9];
  double gadd[4][9];
  double gsign[4];
  // storage shifts of the 16-bit forms (zero otherwise)
  double fshift[9], gshift[9];
  // particles
  double rho_f, grav_x, grav_y;
  double coll_range, coll_pp, coll_pw;
  int wall_face[4];   // 1 where the face is a wall (collisions)
  int np, maxb;
};

// Structure-of-arrays particle state; two copies alternate between steps.
struct PState {
  double *X, *Y, *th, *Ux, *Uy, *Om, *Uxp, *Uyp, *Omp, *Fx, *Fy, *Tz;
  int* nslot;   // partial slots written by the last lattice pass
};

struct PConst {
  const double *R, *rhos, *Tinit;
  const int* fixed;
};

struct Lists {
  int* cnt;     // [nblocks]
  int2* ent;    // [nblocks][kListCap] (particle id, partial slot)
};

// Launchers (defined in vlb_kernels.hip).  All run on `s`.
hipError_t launch_particles(const Params& P, PState cur, PState next,
                            PConst pc, Lists L, double* partial,
                            int have_partials, int mode, int* flags,
                            hipStream_t s);
hipError_t launch_lattice(int prec, bool write_macro, const Params& P,
                          const void* f_in, void* f_out, const void* g_in,
                          void* g_out, void* h, size_t plane, PState pn,
                          PConst pc, Lists L, double* partial, double* macro,
                          int* flags, hipStream_t s);
hipError_t launch_init(int prec, const Params& P, void* f, void* g, void* h,
                       size_t plane, PState pn, PConst pc, Lists L,
                       double* macro, int* flags, hipStream_t s);
hipError_t launch_particle_sums(const Params& P, PState ps, PConst pc,
                                const double* macro, double* out4,
                                hipStream_t s);
hipError_t launch_ownership(const Params& P, PState ps, PConst pc, Lists L,
                            int* count, int* ids, int* full, int* flags,
                            hipStream_t s);
hipError_t launch_unpack(int prec, const Params& P, const void* pop,
                         size_t plane, int which_g, double* out,
                         hipStream_t s);

enum { kModeUpdate = 0, kModeReduceOnly = 1, kModeBinOnly = 2 };

}  // namespace vlb
