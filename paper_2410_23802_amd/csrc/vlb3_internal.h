// vlb3_internal.h -- the three-dimensional step's constants and launchers,
// shared by its kernels (vlb3_kernels.hip) and its host side
// (vlb3_api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vlb3 {

constexpr int kBlock = 256;      // cells per tile (one per thread)
constexpr int kMaxSpheres = 64;  // one per lane of a wave
constexpr int kMaxK = 4;         // spheres per cell
constexpr int kQ = 19, kQG = 7;

// The sphere state buffer: kFields planes of np doubles.
enum Field {
  fX, fY, fZ, fU, fV, fW, fOx, fOy, fOz,       // centre, velocity, spin
  fUp, fVp, fWp, fOxp, fOyp, fOzp,             // the previous step's
  fFx, fFy, fFz, fTx, fTy, fTz,                // momentum-exchange sums
  kFields
};
// The constants: R, rho_s, T_init, fixed (as 0/1).
enum Const { cR, cRho, cTinit, cFixed, kConsts };

// Macroscopic output planes written by the last step of a call.
enum Macro { mRho, mUx, mUy, mUz, mT, mFs, mD, kMacro };

struct Params3 {
  int nx, ny, nz, N, nblocks, np, kmax;
  int per[3];                 // periodic axes
  int wall_dirichlet[6];      // thermal type of each wall face
  double u_wall[6][3], T_wall[6];
  double rho0, rho_f, cv_f, cv_s, lam_f, lam_s, cref;
  double snu, sq;             // shear rate, odd-moment rate
  int sigma_rule;
  double body[3], grav[3], beta, T_ref;
  double zeta, k_pp, k_pw;
  double init_u[3], init_T;
  int nt_stores;              // the step stores past the caches
  // storage: FP64, or FP32 populations and carrier (f32 = 1) kept as the
  // deviations f_q - fshift[q], g_q - gshift[q] (the arithmetic stays FP64)
  int f32;
  double fshift[kQ], gshift[kQG];
};

// Per (sphere, tile) partial sums of sum f_s,p (f^eq - f*) e (3) and of its
// moment about the centre (3).
constexpr int kPartial = 6;

// f, g, h: populations and carrier in the storage type (FP64, or FP32
// where P.f32)
hipError_t launch_init(const Params3& P, void* f, void* g, void* h,
                       double* macro, const double* S, const double* C,
                       int* flags, hipStream_t s);
// the momentum-exchange sums over the tiles whose candidate masks (tmask,
// from the geometry pass of the last step) hold the sphere; update: the
// Newton-Euler step into nxt
hipError_t launch_particles(const Params3& P, double* cur, double* nxt,
                            const double* C, const double* partial,
                            const unsigned long long* tmask, int have,
                            int update, hipStream_t s);
// the spheres' shares of the cells of the tiles they may reach (gid: count
// and ids packed, gw: kMaxK shares per cell) and each tile's candidate mask
// (items, nitems: the lists of partly covered cell slots, kSegs of them,
// segment k at items + k * seg_items(P) for the tiles b with b mod kSegs =
// k, its length in nitems[k])
constexpr int kSegs = 8;
__host__ __device__ inline size_t seg_items(const Params3& P) {
  return (size_t)((P.nblocks + kSegs - 1) / kSegs) * kBlock * kMaxK;
}
hipError_t launch_geometry(const Params3& P, const double* S,
                           const double* C, int* gid, double* gw,
                           unsigned long long* tmask, int* items, int* nitems,
                           int* flags, hipStream_t s);
hipError_t launch_step(const Params3& P, bool out, const void* fin,
                       void* fout, const void* gin, void* gout,
                       const void* hin, void* hout, const double* S,
                       const double* C, const int* gid, const double* gw,
                       const unsigned long long* tmask, double* partial,
                       double* macro, int* flags, hipStream_t s);
hipError_t launch_sphere_sums(const Params3& P, const double* S,
                              const double* C, const double* macro,
                              double* out, hipStream_t s);
// Gauss-Legendre nodes and weights on [0, 1] for the volume quadrature,
// computed on the host, copied to the device's constant memory.
hipError_t upload_quadrature();

constexpr int kFlagUnstable = 1, kFlagOverlap = 2;

}  // namespace vlb3
