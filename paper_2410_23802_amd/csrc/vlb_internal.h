// vlb_internal.h -- device-side data structures and kernel launchers of the
// MI355X volumetric lattice Boltzmann library (private to the library).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vlb.h"

namespace vlb {

constexpr int kBlock = 256;       // cells per lattice block (one per thread)
constexpr int kListCap = 32;      // particle entries per block list
constexpr int kBinCap = 8;        // particle entries per centre bin
constexpr int kMaxRadius = 28;    // band rows of one particle fit one wave
constexpr int kRedVals = 3;       // Fx, Fy, Tz per partial slot
constexpr int kScanMax = 64;      // scan form up to this many particles

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
  int fluid_gravity;   // situation II of Sec. 3.2 (see vlb_domain_desc)
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
  // storage reference: populations are kept as f_i - w_i rho0s and
  // g_i - w_i c_ref T0s (both zero for FP64); fshift/gshift = the products
  double rho0s, cT0s;
  double fshift[9], gshift[9];
  // particles
  double rho_f, grav_x, grav_y;
  double rmax;        // largest particle radius
  double coll_range, coll_pp, coll_pw;
  // list form: the grid of centre bins the repulsion searches (bins at
  // least 2 rmax + coll_range + 2 wide, so that two particles within reach
  // lie in neighbouring bins; never more bins than lattice blocks)
  int nbx, nby, nbins;
  double binw_x, binw_y;
  int wall_face[4];   // 1 where the face is a wall (collisions)
  int np, maxb;
  int scan;           // 1: scan form (few particles, one launch per step)
  int maxr;           // scan form: bound on the tiles one particle reaches
  int nfirst;         // step kernel: blocks of the particle-tile group
                      // (scan form: np * maxr rounded up to 8; else 0)
  int xcd_group;      // step kernel: consecutive tiles per XCD group
  int stream_blocks;  // step kernel: blocks of the streaming group
  int tile_stride;    // step kernel, list form: block k of the streaming
                      // group takes tile k * tile_stride mod stream_blocks
                      // (0: the XCD groups)
  int pair_tiles;     // step kernel, 16-bit forms: two plain tiles per
                      // streaming block (never in the list form)
  int nt_stores;      // step kernel and probe: populations and carrier
                      // stored non-temporally
  int ellipses;       // some particle is an ellipse (its kernels carry the
                      // ellipse geometry; no paired tiles)
};

// The constants the per-cell arithmetic uses, in the compute precision C
// (built on the host so the hot path converts nothing).
template <class C>
struct Hot {
  C s_e, s_q, s_p;
  C cvf, dcv, lamf, dlam, cref, taug_coef, grad_coef;
  C A0x, A0y, B0x, B0y;
  C rho0s, cT0s;
  C fadd[4][9];
  C gadd[4][9];
  C gsign[4];
  int sigma_rule;
};

template <class C>
inline Hot<C> make_hot(const Params& P) {
  Hot<C> H;
  H.s_e = (C)P.s_e; H.s_q = (C)P.s_q; H.s_p = (C)P.s_p;
  H.cvf = (C)P.cvf; H.dcv = (C)P.dcv; H.lamf = (C)P.lamf; H.dlam = (C)P.dlam;
  H.cref = (C)P.cref; H.taug_coef = (C)P.taug_coef;
  H.grad_coef = (C)(-3.0 / P.cref);   // -6/(4+alpha1)/c_ref, alpha1 = -2
  H.A0x = (C)P.A0x; H.A0y = (C)P.A0y; H.B0x = (C)P.B0x; H.B0y = (C)P.B0y;
  H.rho0s = (C)P.rho0s; H.cT0s = (C)P.cT0s;
  for (int w = 0; w < 4; ++w) {
    for (int q = 0; q < 9; ++q) {
      H.fadd[w][q] = (C)P.fadd[w][q];
      H.gadd[w][q] = (C)P.gadd[w][q];
    }
    H.gsign[w] = (C)P.gsign[w];
  }
  H.sigma_rule = P.sigma_rule;
  return H;
}

// Structure-of-arrays particle state; two copies alternate between steps.
struct PState {
  double *X, *Y, *th, *Ux, *Uy, *Om, *Uxp, *Uyp, *Omp, *Fx, *Fy, *Tz;
  int* nslot;   // partial slots written by the last lattice pass
};

struct PConst {
  const double *R, *rhos, *Tinit;
  const double* Rb;   // minor semi-axis: R for a disk, < R for an ellipse
  const int* fixed;   // bit 0: velocity held; bit 1: temperature held at Tinit
};

// Per-tile particle lists of the list form.  The counts are double
// buffered: the particle pass fills `cnt` (all zero on entry) and clears
// `clr`, the counts of the previous step, which both lattice kernels of
// that step have finished reading.
// Scan form: whether the step kernel finds its particle tiles from the
// per-tile counts (FP64, and the paired 16-bit tiles) or tests them in its
// streaming blocks (FP32 and the unpaired 16-bit forms, 3-6 % faster that
// way on a 0.8 M-cell channel, where their particle blocks' chain is as
// long as the streaming).  The host keeps the counts for the same cases.
__host__ __device__ constexpr bool counted_tiles(int prec, bool pair) {
  return prec == VLB_FP64 || pair;
}

struct Lists {
  int* cnt;     // [nblocks]
  int2* ent;    // [nblocks][kListCap] (particle id, partial slot)
  int* clr;     // [nblocks] or null: counts to reset to zero
  // or null: the lists of the particle state the pass reads (its
  // positions' band boxes), for the neighbour search of the repulsion
  const int* ocnt;
  const int2* oent;
  // list form, a binning pass: the centre bins of the positions it writes
  // (filled), the stale ones (cleared) and those of the positions it starts
  // from (read by the repulsion), or null
  int* bcnt;     // [nbins]
  int* bent;     // [nbins][kBinCap] particle ids
  int* bclr;     // [nbins]
  const int* obcnt;
  const int* obent;
};

// The centre bin of a particle at (X, Y): the same arithmetic where the bins
// are filled and where they are searched.
__host__ __device__ inline void centre_bin(const Params& P, double X,
                                           double Y, int& bx, int& by) {
  // clamped to the grid (a NaN goes to bin 0)
  const double fx = floor(X / P.binw_x), fy = floor(Y / P.binw_y);
  bx = fx > 0.0 ? (fx < (double)P.nbx ? (int)fx : P.nbx - 1) : 0;
  by = fy > 0.0 ? (fy < (double)P.nby ? (int)fy : P.nby - 1) : 0;
}

// The buffers one lattice step of one domain reads and writes (device
// pointers; the population and carrier pointers are in the storage type of
// the domain's precision).  `cur` is the particle state of step n; `nxt`
// receives step n+1 (scan form) or already holds it (list form).  Partials
// of step n are read from `partial_in`, those of step n+1 written to
// `partial_out`.
struct StepBufs {
  const void* fi; void* fo;
  const void* gi; void* go;
  const void* hin; void* hout;   // [df_s/dt] carrier, step n / step n+1
  size_t plane;
  PState cur, nxt;
  PConst pc;
  Lists L;
  const double* partial_in;
  double* partial_out;
  double* macro;
  int* flags;
  // scan form of one domain (null otherwise): per tile, the number of
  // particles whose band box reaches it at this step's positions (read), at
  // the next step's (filled by the blocks that store the particles' new
  // state) and a stale buffer (cleared, one entry per tile)
  const int* tcount;
  int* tcount_next;
  int* tcount_clear;
};

// Arguments of one launch of the step kernel.  ev_start/ev_stop (may be
// null) are recorded by the dispatch itself.
struct StepLaunch {
  const Params* P;
  bool out;                  // also store the macroscopic fields
  int have;                  // partial_in holds a previous step
  StepBufs B;
  hipEvent_t ev_start, ev_stop;
};

// One domain of a batch as the batch step kernel sees it: its constants in
// both compute precisions and the buffers of a step taken from each of the
// two buffer parities.  All domains of a batch advance in lockstep.  In the
// device copy of the table every pointer of B holds the byte offset of its
// buffer from the batch's arena pointer (the kernel adds the arena back).
struct BatchCase {
  Params P;
  Hot<double> Hd;
  Hot<float> Hf;
  StepBufs B[2];
};

// A task of the batch step kernel: (domain, k); k < P.nfirst is the k-th
// particle-tile task of the domain, k | kPairTask the tiles k and k + 1
// streamed by one block (two cells per lane), else tile k - P.nfirst.
// Domain -1: no work (padding).
typedef int2 BatchTask;
constexpr int kPairTask = 1 << 30;

// Launchers (defined in vlb_kernels.hip).  All run on `s`.
hipError_t launch_particles(const Params& P, PState cur, PState next,
                            PConst pc, Lists L, const double* partial,
                            int have_partials, int mode, int* flags,
                            hipStream_t s);
// k_step: the lattice step over every cell (events, if given, bracket it)
hipError_t launch_step(int prec, const StepLaunch& a, hipStream_t s);
// k_batch_step: one step of every domain of a batch; `grid` persistent
// blocks walk the task table in steps of `grid`.  The variant: `waves`, the
// occupancy (waves per SIMD: 4, or 5 for the 32- and 16-bit forms), and
// `pair`, whether the table holds pair tasks.
struct BatchLaunch {
  const BatchCase* cases;
  const BatchTask* tasks;
  char* arena;
  int ntasks, grid, parity, have, waves;
  bool pair;
};
hipError_t launch_batch_step(int prec, bool out, const BatchLaunch& a,
                             hipStream_t s);
// out[i] = the error flags of domain i
hipError_t launch_gather_flags(const BatchCase* cases, char* arena, int n,
                               int* out, hipStream_t s);
hipError_t launch_init(int prec, const Params& P, void* f, void* g, void* h,
                       size_t plane, PState pn, PConst pc, Lists L,
                       double* macro, int* flags, hipStream_t s);
// Scan form: count[tile] += the particles reaching it at the next step.
hipError_t launch_tile_counts(const Params& P, PState cur, PConst pc,
                              int* count, int* flags, hipStream_t s);
hipError_t launch_particle_sums(const Params& P, PState ps, PConst pc,
                                const double* macro, double* out4,
                                hipStream_t s);
// Ownership of the cells of tiles [tile0, tile0 + ntiles); count, ids and
// full are indexed from the first cell of tile0.
hipError_t launch_ownership(const Params& P, PState ps, PConst pc, Lists L,
                            int tile0, int ntiles, int* count, int* ids,
                            int* full, int* flags, hipStream_t s);
// The step's memory pattern without its arithmetic (fi -> fo, gi -> go,
// hin -> hout of B; the state in fi, gi, hin is left as it was).
hipError_t launch_stream_probe(int prec, const Params& P, const StepBufs& B,
                              hipStream_t s);
hipError_t launch_unpack(int prec, const Params& P, const void* pop,
                         size_t plane, int which_g, double* out,
                         hipStream_t s);

enum { kModeUpdate = 0, kModeReduceOnly = 1, kModeBinOnly = 2 };

}  // namespace vlb
