// vlb_api.hip -- host implementation of the C ABI declared in include/vlb.h.
// Owns the device memory of a context, derives the kernel constants from the
// descriptor, and sequences the kernels of each time step on the context's
// stream.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "vlb_context.h"

#ifndef VLB_SOURCE_HASH
#error "build with -DVLB_SOURCE_HASH (paper_2410_23802_amd/build.py sets it)"
#endif

using namespace vlb;

static std::string g_create_error;

static const double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
static const int kEx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int kEy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};

static vlb_status fail(vlb_ctx* c, vlb_status s, const std::string& msg) {
  if (c) c->err = msg; else g_create_error = msg;
  return s;
}

static vlb_status hip_fail(vlb_ctx* c, hipError_t e, const char* where) {
  return fail(c, VLB_EHIP,
              std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                   \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr); \
  } while (0)

static bool dalloc(vlb_ctx* c, void** p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return false;
  }
  c->dev_bytes += bytes;
  return true;
}

static void free_particles(vlb_ctx* c) {
  for (int k = 0; k < 2; ++k) {
    if (c->pmem[k]) (void)hipFree(c->pmem[k]);
    if (c->pslot[k]) (void)hipFree(c->pslot[k]);
    c->pmem[k] = nullptr;
    c->pslot[k] = nullptr;
  }
  if (c->pconst) (void)hipFree(c->pconst);
  if (c->pfixed) (void)hipFree(c->pfixed);
  for (int k = 0; k < 2; ++k) {
    if (c->partial[k]) (void)hipFree(c->partial[k]);
    c->partial[k] = nullptr;
  }
  if (c->thermal4) (void)hipFree(c->thermal4);
  c->pconst = nullptr;
  c->pfixed = nullptr;
  c->thermal4 = nullptr;
}

// Scan form: the step kernel reads per-tile particle counts (and keeps
// them) for these storage forms; it tests its tiles directly for the others.
static bool tile_counts_kept(const vlb_ctx* c) {
  return c->np > 0 && c->P.scan &&
         counted_tiles(c->prec, c->P.pair_tiles != 0);
}

// Zero the block lists and the scan form's tile counts; in the scan form,
// count the tiles the particles of the stored state reach at the next step
// (the step kernel keeps the counts from then on).
static hipError_t clear_lists(vlb_ctx* c) {
  c->lpar = 0;
  c->tpar = 0;
  for (int k = 0; k < 3; ++k) {
    hipError_t e = hipMemsetAsync(c->blk_cnt[k], 0,
                                  c->P.nblocks * sizeof(int), c->stream);
    if (e == hipSuccess)
      e = hipMemsetAsync(c->tcount[k], 0, c->P.nblocks * sizeof(int),
                         c->stream);
    if (e == hipSuccess)
      e = hipMemsetAsync(c->bin_cnt[k], 0, c->P.nblocks * sizeof(int),
                         c->stream);
    if (e != hipSuccess) return e;
  }
  if (tile_counts_kept(c))
    return launch_tile_counts(c->P, c->ps[c->pcur], c->pc, c->tcount[0],
                              c->flags, c->stream);
  return hipSuccess;
}

static vlb_status validate(const vlb_domain_desc* d, std::string& why) {
  if (d->nx < 1 || d->ny < 1) return why = "nx and ny must be >= 1", VLB_EINVAL;
  if ((int64_t)d->nx * d->ny * 9 >= ((int64_t)1 << 31))
    return why = "domain too large (9 nx ny must fit in int32)", VLB_EINVAL;
  for (int a = 0; a < 2; ++a) {
    int f0 = d->face_flow[2 * a], f1 = d->face_flow[2 * a + 1];
    if ((f0 != VLB_PERIODIC && f0 != VLB_WALL) ||
        (f1 != VLB_PERIODIC && f1 != VLB_WALL))
      return why = "face_flow must be VLB_PERIODIC or VLB_WALL", VLB_EINVAL;
    if ((f0 == VLB_PERIODIC) != (f1 == VLB_PERIODIC))
      return why = "periodic faces must come in pairs", VLB_EINVAL;
  }
  for (int k = 0; k < 4; ++k)
    if (d->face_thermal[k] != VLB_ADIABATIC &&
        d->face_thermal[k] != VLB_DIRICHLET)
      return why = "face_thermal must be VLB_ADIABATIC or VLB_DIRICHLET",
             VLB_EINVAL;
  if (!(d->tau_f > 0.5)) return why = "tau_f must exceed 1/2", VLB_EINVAL;
  if (!(d->rho_f > 0) || !(d->cv_f > 0) || !(d->lambda_f > 0) ||
      !(d->R_lambda > 0) || !(d->R_cv > 0) || !(d->init_rho > 0))
    return why = "densities, heat capacities and conductivities must be > 0",
           VLB_EINVAL;
  if (d->sigma_rule != 0 && d->sigma_rule != 1)
    return why = "sigma_rule must be 0 or 1", VLB_EINVAL;
  if (d->fluid_gravity != 0 && d->fluid_gravity != 1)
    return why = "fluid_gravity must be 0 or 1", VLB_EINVAL;
  if (d->kmax < 1 || d->kmax > 8) return why = "kmax must be in 1..8", VLB_EINVAL;
  if (d->precision < VLB_FP64 || d->precision > VLB_BF16_SHIFT)
    return why = "unknown precision", VLB_EINVAL;
  if (d->coll_range < 0) return why = "coll_range must be >= 0", VLB_EINVAL;
  return VLB_OK;
}

// Tile groups of the step kernel's streaming blocks (one group after
// another to each XCD in turn).  Where every streaming tile costs the same
// (no particles, or the scan form, whose particle tiles run in a block
// group of their own) each XCD takes one contiguous band, which keeps the
// neighbour rows a tile pulls in that XCD's L2 (measured on the channel:
// HBM reads per step 1.14 -> 1.06 of the algorithmic bytes at FP32).  In
// the list form the particle tiles are updated in place, cluster where the
// particles are and dominate the time: one contiguous band per XCD made
// the dense cavity 1.5x slower (the XCD holding the particles' rows ends
// last), and tiles dealt one at a time in order (block k takes tile k)
// run the particle rows all at once, which loads the vector ALUs in bursts.
// There block k takes tile k * s mod M (M = the streaming blocks, s odd
// near 0.618 M and coprime to it): a permutation under which every XCD and
// every stretch of the launch holds its share of particle tiles (dense
// cavity FP32: 104 -> 96 us; the rows a tile pulls are then seldom in L2,
// but a line is still fetched about once, so the HBM bytes hardly change).
//
// The 16-bit forms stream two tiles per block (each lane loads its cell of
// both before computing either) where one step moves more than the 256 MB
// Infinity Cache holds: there a wave with one cell per lane has too few
// bytes in flight (16 M-cell channel: 344 -> 288 us).  Below that size, and
// in the list form (a particle tile would share its block), one tile per
// block is faster (channel of 0.8 M cells: 17.6 vs 18.1 us).
//
// The list form in FP64 and FP32 stores the populations past the caches
// (non-temporal) where one step moves more than 320 MB, 1.25 x the
// Infinity Cache: the next step cannot find them there anyway, and L2 is
// left to the rows the scattered tiles pull from their neighbours (dense
// cavity: FP64 k_step 154.7 -> 150.6 us, FP32 89.0 -> 85.8 us; its 16-bit
// forms, 189 MB a step, lost 4 %).  Where the step fits the cache such
// stores cost a third more (0.8 M-cell channel, FP64 37 -> 49 us), and on
// the 16 M-cell channel (scan form, tiles in order) they gain nothing.
static void set_stream_groups(Params& P, bool list_form, int prec) {
  int g = list_form ? 1 : (P.nblocks + 7) / 8;
  if (g < 1) g = 1;
  P.xcd_group = g;
  const int per_xcd = (P.nblocks + 8 * g - 1) / (8 * g);
  P.stream_blocks = 8 * g * per_xcd;
  P.tile_stride = 0;
  if (list_form && P.stream_blocks > 16) {
    int sd = (int)(0.6180339887 * P.stream_blocks) | 1;
    auto gcd = [](int a, int b) {
      while (b) { const int t = a % b; a = b; b = t; }
      return a;
    };
    while (gcd(sd, P.stream_blocks) != 1) sd += 2;
    P.tile_stride = sd;
  }
  const bool b16 = prec == VLB_FP16_SHIFT || prec == VLB_BF16_SHIFT;
  const size_t step_bytes = (size_t)P.N * (2 * 9 * 2 + 2 * 4);
  P.pair_tiles = b16 && !list_form && step_bytes > ((size_t)256 << 20);
  const bool wide = prec == VLB_FP64 || prec == VLB_FP32;
  const size_t elem = prec == VLB_FP64 ? 8 : 4;
  const size_t moved = (size_t)P.N * (2 * 18 * elem + 2 * elem);
  P.nt_stores = wide && list_form && moved > ((size_t)320 << 20);
}

static void derive_params(vlb_ctx* c) {
  const vlb_domain_desc& d = c->d;
  Params& P = c->P;
  memset(&P, 0, sizeof(P));
  P.nx = d.nx;
  P.ny = d.ny;
  P.N = d.nx * d.ny;
  P.nblocks = (P.N + kBlock - 1) / kBlock;
  P.nfirst = 0;
  set_stream_groups(P, false, c->prec);
  P.perx = d.face_flow[VLB_FACE_XLO] == VLB_PERIODIC;
  P.pery = d.face_flow[VLB_FACE_YLO] == VLB_PERIODIC;
  P.kmax = d.kmax;
  P.sigma_rule = d.sigma_rule;
  P.fluid_gravity = d.fluid_gravity;
  // flow relaxation (Sec. 3): s_e = s_eps = 1.25, s_p = 1/tau_f,
  // (1/s_p - 1/2)(1/s_q - 1/2) = 1/12
  P.s_e = 1.25;
  P.s_p = 1.0 / d.tau_f;
  P.s_q = 1.0 / (0.5 + (1.0 / 12.0) / (d.tau_f - 0.5));
  P.cvf = d.cv_f;
  P.cvs = d.R_cv * d.cv_f;
  P.dcv = P.cvs - P.cvf;
  P.lamf = d.lambda_f;
  P.dlam = d.R_lambda * d.lambda_f - d.lambda_f;
  P.cref = 2.0 * P.cvf * P.cvs / (P.cvf + P.cvs);
  // eq. lambda with alpha1 = -2: lambda/rho_f = c_ref (tau_g - 1/2)/3
  P.taug_coef = 3.0 / (d.rho_f * P.cref);
  // fluid force (1 - f_s)[F_ext - rho_f g beta (T - T_ref)] = (1-f_s)(A0 + B0 T)
  // situation II of Sec. 3.2: the fluid's share also carries rho_f g
  const double gw = d.fluid_gravity ? d.rho_f : 0.0;
  P.A0x = d.body_force[0] + gw * d.gravity[0] +
          d.rho_f * d.beta * d.T_ref * d.gravity[0];
  P.A0y = d.body_force[1] + gw * d.gravity[1] +
          d.rho_f * d.beta * d.T_ref * d.gravity[1];
  P.B0x = -d.rho_f * d.beta * d.gravity[0];
  P.B0y = -d.rho_f * d.beta * d.gravity[1];
  P.init_rho = d.init_rho;
  P.init_ux = d.init_u[0];
  P.init_uy = d.init_u[1];
  P.init_T = d.init_T;
  // storage reference of the deviation form (not used by FP64)
  const bool shifted = d.precision != VLB_FP64;
  P.rho0s = shifted ? d.shift_rho0 : 0.0;
  const double T0s = shifted ? d.shift_T0 : 0.0;
  P.cT0s = P.cref * T0s;
  for (int w = 0; w < 4; ++w) {
    const bool dir = d.face_thermal[w] == VLB_DIRICHLET;
    P.gsign[w] = dir ? -1.0 : 1.0;
    for (int q = 0; q < 9; ++q) {
      const double eu = kEx[q] * d.u_wall[w][0] + kEy[q] * d.u_wall[w][1];
      P.fadd[w][q] = 6.0 * kW[q] * d.init_rho * eu;
      // anti-bounce-back on deviations: g'_i = -g'_opp + 2 w_i c_ref (T_w - T0s)
      P.gadd[w][q] = dir ? 2.0 * kW[q] * P.cref * (d.T_wall[w] - T0s) : 0.0;
    }
    P.wall_face[w] = d.face_flow[w] == VLB_WALL;
  }
  for (int q = 0; q < 9; ++q) {
    P.fshift[q] = kW[q] * P.rho0s;
    P.gshift[q] = kW[q] * P.cT0s;
  }
  P.rho_f = d.rho_f;
  P.grav_x = d.gravity[0];
  P.grav_y = d.gravity[1];
  P.coll_range = d.coll_range;
  P.coll_pp = d.coll_stiff_pp;
  P.coll_pw = d.coll_stiff_pw;
  P.np = 0;
  P.maxb = 0;
}

// The current block lists (read by the lattice, init and ownership kernels).
static Lists lists(vlb_ctx* c) {
  Lists L;
  L.cnt = c->blk_cnt[c->lpar];
  L.ent = c->blk_ent[c->lpar];
  L.clr = nullptr;
  L.ocnt = nullptr;
  L.oent = nullptr;
  L.bcnt = L.bent = L.bclr = nullptr;
  L.obcnt = L.obent = nullptr;
  return L;
}

// Lists for a particle pass that bins: it reads the current lists (the
// band boxes of the positions it starts from), fills the next buffer (zero)
// and clears the one after (stale since the pass before); the filled buffer
// becomes current.
static Lists bin_lists(vlb_ctx* c) {
  const int nxt = (c->lpar + 1) % 3, stale = (c->lpar + 2) % 3;
  Lists L;
  L.cnt = c->blk_cnt[nxt];
  L.ent = c->blk_ent[nxt];
  L.clr = c->blk_cnt[stale];
  L.ocnt = c->blk_cnt[c->lpar];
  L.oent = c->blk_ent[c->lpar];
  // the centre bins turn with them (list form only)
  const bool bins = c->np > 0 && !c->P.scan;
  L.bcnt = bins ? c->bin_cnt[nxt] : nullptr;
  L.bent = bins ? c->bin_ent[nxt] : nullptr;
  L.bclr = bins ? c->bin_cnt[stale] : nullptr;
  L.obcnt = bins ? c->bin_cnt[c->lpar] : nullptr;
  L.obent = bins ? c->bin_ent[c->lpar] : nullptr;
  c->lpar = nxt;
  return L;
}

// The buffers of the next step of context c.
StepBufs vlb::context_step_bufs(vlb_ctx* c) {
  StepBufs B;
  B.fi = c->f[c->cur];
  B.fo = c->f[1 - c->cur];
  B.gi = c->g[c->cur];
  B.go = c->g[1 - c->cur];
  B.hin = c->h[c->cur];
  B.hout = c->h[1 - c->cur];
  B.plane = c->plane;
  B.cur = c->ps[c->pcur];
  B.nxt = c->ps[1 - c->pcur];
  B.pc = c->pc;
  B.L = lists(c);
  B.partial_in = c->partial[c->pp];
  B.partial_out = c->partial[1 - c->pp];
  B.macro = c->macro;
  B.flags = c->flags;
  const bool counted = tile_counts_kept(c);
  B.tcount = counted ? c->tcount[c->tpar] : nullptr;
  B.tcount_next = counted ? c->tcount[(c->tpar + 1) % 3] : nullptr;
  B.tcount_clear = counted ? c->tcount[(c->tpar + 2) % 3] : nullptr;
  return B;
}

// Bookkeeping of n steps taken (by one_step or by a batch launch).
void vlb::context_advance(vlb_ctx* c, int64_t n) {
  if (n <= 0) return;
  const int flip = (int)(n & 1);
  if (c->np > 0) {
    c->have_partials = 1;
    c->pcur ^= flip;
    c->pp ^= flip;
  }
  c->cur ^= flip;
  c->tpar = (int)((c->tpar + n) % 3);
  c->step += n;
}

extern "C" {

vlb_status vlb_create(const vlb_domain_desc* desc, void* hip_stream,
                      vlb_ctx** out) {
  if (!desc || !out) return fail(nullptr, VLB_EINVAL, "null argument");
  *out = nullptr;
  std::string why;
  vlb_status st = validate(desc, why);
  if (st != VLB_OK) return fail(nullptr, st, why);
  vlb_ctx* c = new (std::nothrow) vlb_ctx();
  if (!c) return fail(nullptr, VLB_ENOMEM, "host allocation failed");
  c->d = *desc;
  c->stream = (hipStream_t)hip_stream;
  (void)hipGetDevice(&c->device);
  c->prec = desc->precision;
  derive_params(c);
  const size_t N = (size_t)c->P.N;
  c->plane = (N + 63) / 64 * 64;  // 256/512-byte aligned planes
  c->pop_elem = c->prec == VLB_FP64 ? 8 : (c->prec == VLB_FP32 ? 4 : 2);
  c->h_elem = c->prec == VLB_FP64 ? 8 : 4;
  bool ok = true;
  for (int k = 0; k < 2; ++k) {
    ok = ok && dalloc(c, &c->f[k], 9 * c->plane * c->pop_elem);
    ok = ok && dalloc(c, &c->g[k], 9 * c->plane * c->pop_elem);
  }
  ok = ok && dalloc(c, &c->h[0], N * c->h_elem);
  ok = ok && dalloc(c, &c->h[1], N * c->h_elem);
  ok = ok && dalloc(c, (void**)&c->macro, 6 * N * sizeof(double));
  for (int k = 0; k < 3; ++k) {
    ok = ok && dalloc(c, (void**)&c->tcount[k], c->P.nblocks * sizeof(int));
    ok = ok && dalloc(c, (void**)&c->blk_cnt[k], c->P.nblocks * sizeof(int));
    ok = ok && dalloc(c, (void**)&c->blk_ent[k],
                      (size_t)c->P.nblocks * kListCap * sizeof(int2));
    // centre bins: never more than nblocks (bins at least 16 cells wide)
    ok = ok && dalloc(c, (void**)&c->bin_cnt[k], c->P.nblocks * sizeof(int));
    ok = ok && dalloc(c, (void**)&c->bin_ent[k],
                      (size_t)c->P.nblocks * kBinCap * sizeof(int));
  }
  ok = ok && dalloc(c, (void**)&c->flags, 4 * sizeof(int));
  if (ok && hipHostMalloc((void**)&c->flags_host, 4 * sizeof(int),
                          hipHostMallocDefault) != hipSuccess)
    ok = false;
  if (!ok) {
    vlb_destroy(c);
    return fail(nullptr, VLB_ENOMEM, "device allocation failed");
  }
  if (clear_lists(c) != hipSuccess ||
      hipMemsetAsync(c->flags, 0, 4 * sizeof(int), c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess) {
    vlb_destroy(c);
    return fail(nullptr, VLB_EHIP, "initial clear failed");
  }
  *out = c;
  return VLB_OK;
}

vlb_status vlb_set_particles(vlb_ctx* c, int32_t n,
                             const vlb_particle_desc* p) {
  if (!c) return VLB_EINVAL;
  if (n < 0 || (n > 0 && !p)) return fail(c, VLB_EINVAL, "bad particle array");
  double rmax = 0.0;
  for (int k = 0; k < n; ++k) {
    if (!(p[k].radius > 0.0) || p[k].radius > kMaxRadius)
      return fail(c, VLB_EINVAL, "particle radius must be in (0, 28]");
    if (!(p[k].rho_s > 0.0))
      return fail(c, VLB_EINVAL, "particle density must be > 0");
    if (!(p[k].radius_minor >= 0.0) || p[k].radius_minor > p[k].radius)
      return fail(c, VLB_EINVAL,
                  "radius_minor must be 0 (a disk) or in (0, radius]");
    if (c->P.perx && !(c->d.nx > 2.0 * p[k].radius + 4.0))
      return fail(c, VLB_EINVAL, "particle wider than the periodic x axis");
    if (c->P.pery && !(c->d.ny > 2.0 * p[k].radius + 4.0))
      return fail(c, VLB_EINVAL, "particle wider than the periodic y axis");
    if (!(p[k].x >= 0.0 && p[k].x < c->d.nx && p[k].y >= 0.0 &&
          p[k].y < c->d.ny))
      return fail(c, VLB_EINVAL, "particle centre must lie in the domain");
    rmax = fmax(rmax, p[k].radius);
  }
  free_particles(c);
  c->parts.assign(p, p + n);
  c->np = n;
  // band rows of a particle <= 2R + 4; each row touches <= 4 blocks
  c->maxb = 4 * (2 * (int)ceil(rmax) + 5);
  c->P.rmax = rmax;
  // centre bins of the repulsion's search: at least 2 rmax + zeta + 2 cells
  // wide (two particles within reach then lie in neighbouring bins) and at
  // least 16, and no more bins than lattice blocks (their buffers' size);
  // equal widths that tile each axis
  {
    const double wmin = fmax(2.0 * rmax + fmax(c->P.coll_range, 0.0) + 2.0, 16.0);
    c->P.nbx = std::max(1, (int)floor(c->d.nx / wmin));
    c->P.nby = std::max(1, (int)floor(c->d.ny / wmin));
    // a thin domain (one side under 16 cells) could still hold more
    while ((int64_t)c->P.nbx * c->P.nby > c->P.nblocks) {
      if (c->P.nbx >= c->P.nby) --c->P.nbx;
      else --c->P.nby;
    }
    c->P.nbins = c->P.nbx * c->P.nby;
    c->P.binw_x = (double)c->d.nx / c->P.nbx;
    c->P.binw_y = (double)c->d.ny / c->P.nby;
  }
  c->P.np = n;
  c->P.maxb = c->maxb;
  // scan form for few particles: partials [particle][tile] must stay small
  const size_t scan_bytes = (size_t)n * c->P.nblocks * kRedVals * sizeof(double);
  c->P.scan = (n > 0 && n <= kScanMax && scan_bytes <= ((size_t)512 << 20)) ? 1 : 0;
  // tiles one particle reaches: its band rows (<= 2R + 4) as whole rows,
  // plus the ends and a second range when the box wraps around y
  const int rows = 2 * (int)ceil(rmax) + 5;
  c->P.maxr = (int)(((int64_t)rows * c->d.nx + kBlock - 1) / kBlock) + 3;
  c->P.nfirst = c->P.scan ? (n * c->P.maxr + 7) / 8 * 8 : 0;
  set_stream_groups(c->P, n > 0 && !c->P.scan, c->prec);
  c->P.ellipses = 0;
  for (int k = 0; k < n; ++k)
    if (p[k].radius_minor > 0.0 && p[k].radius_minor < p[k].radius)
      c->P.ellipses = 1;
  if (c->P.ellipses) {
    c->P.pair_tiles = 0;
    c->P.nt_stores = 0;
  }
  const size_t part_slots =
      c->P.scan ? (size_t)n * c->P.nblocks : (size_t)n * c->maxb;
  c->initialized = false;
  if (n == 0) return VLB_OK;
  bool ok = true;
  for (int k = 0; k < 2; ++k) {
    ok = ok && dalloc(c, (void**)&c->pmem[k], 12 * (size_t)n * sizeof(double));
    ok = ok && dalloc(c, (void**)&c->pslot[k], (size_t)n * sizeof(int));
  }
  ok = ok && dalloc(c, (void**)&c->pconst, 4 * (size_t)n * sizeof(double));
  ok = ok && dalloc(c, (void**)&c->pfixed, (size_t)n * sizeof(int));
  for (int k = 0; k < 2; ++k)
    ok = ok && dalloc(c, (void**)&c->partial[k],
                      part_slots * kRedVals * sizeof(double));
  ok = ok && dalloc(c, (void**)&c->thermal4, 4 * (size_t)n * sizeof(double));
  if (!ok) {
    free_particles(c);
    c->np = 0;
    c->P.np = 0;
    c->P.scan = 0;
    c->P.nfirst = 0;
    c->P.ellipses = 0;
    set_stream_groups(c->P, false, c->prec);
    return fail(c, VLB_ENOMEM, "particle allocation failed");
  }
  for (int k = 0; k < 2; ++k) {
    double* b = c->pmem[k];
    PState& s = c->ps[k];
    s.X = b; s.Y = b + n; s.th = b + 2 * n; s.Ux = b + 3 * n; s.Uy = b + 4 * n;
    s.Om = b + 5 * n; s.Uxp = b + 6 * n; s.Uyp = b + 7 * n; s.Omp = b + 8 * n;
    s.Fx = b + 9 * n; s.Fy = b + 10 * n; s.Tz = b + 11 * n;
    s.nslot = c->pslot[k];
  }
  c->pc.R = c->pconst;
  c->pc.rhos = c->pconst + n;
  c->pc.Tinit = c->pconst + 2 * n;
  c->pc.Rb = c->pconst + 3 * n;
  c->pc.fixed = c->pfixed;
  return VLB_OK;
}

static vlb_status check_flags(vlb_ctx* c) {
  HIP_TRY(c, hipMemcpyAsync(c->flags_host, c->flags, sizeof(int),
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  const int f = c->flags_host[0];
  if (f & kFlagUnstable)
    return fail(c, VLB_EUNSTABLE, "a cell reached rho <= 0 or a non-finite value");
  if (f & kFlagListFull)
    return fail(c, VLB_EOVERLAP, "a per-block particle list overflowed");
  if (f & kFlagOverlap)
    return fail(c, VLB_EOVERLAP, "more than kmax particles touch one cell");
  return VLB_OK;
}

vlb_status vlb_init(vlb_ctx* c) {
  if (!c) return VLB_EINVAL;
  const int n = c->np;
  c->pcur = 0;
  c->cur = 0;
  c->have_partials = 0;
  c->step = 0;
  if (n > 0) {
    std::vector<double> host(12 * (size_t)n, 0.0), cst(4 * (size_t)n);
    std::vector<int> fx(n);
    for (int k = 0; k < n; ++k) {
      const vlb_particle_desc& p = c->parts[k];
      host[k] = p.x;
      host[n + k] = p.y;
      host[2 * n + k] = p.theta;
      host[3 * n + k] = p.ux;
      host[4 * n + k] = p.uy;
      host[5 * n + k] = p.omega;
      host[6 * n + k] = p.ux;   // previous-step velocity: U^{-1} = U^0
      host[7 * n + k] = p.uy;
      host[8 * n + k] = p.omega;
      cst[k] = p.radius;
      cst[n + k] = p.rho_s;
      cst[2 * n + k] = p.T_init;
      cst[3 * n + k] = p.radius_minor > 0.0 ? p.radius_minor : p.radius;
      fx[k] = (p.fixed ? 1 : 0) | (p.hold_T ? 2 : 0);
    }
    HIP_TRY(c, hipMemcpyAsync(c->pmem[0], host.data(), host.size() * 8,
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->pconst, cst.data(), cst.size() * 8,
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->pfixed, fx.data(), fx.size() * 4,
                              hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipMemsetAsync(c->pslot[0], 0, n * sizeof(int), c->stream));
    HIP_TRY(c, hipMemsetAsync(c->pslot[1], 0, n * sizeof(int), c->stream));
    // the copies read pageable host vectors: finish before they go away
    HIP_TRY(c, hipStreamSynchronize(c->stream));
  }
  HIP_TRY(c, clear_lists(c));
  HIP_TRY(c, hipMemsetAsync(c->flags, 0, 4 * sizeof(int), c->stream));
  c->pp = 0;
  if (!c->P.scan)
    HIP_TRY(c, launch_particles(c->P, c->ps[0], c->ps[1], c->pc, bin_lists(c),
                                c->partial[0], 0, kModeBinOnly, c->flags,
                                c->stream));
  HIP_TRY(c, launch_init(c->prec, c->P, c->f[0], c->g[0], c->h[0], c->plane,
                         c->ps[0], c->pc, lists(c), c->macro, c->flags,
                         c->stream));
  vlb_status st = check_flags(c);
  c->initialized = (st == VLB_OK);
  return st;
}


// One time step: (list form) the particle pass, which advances the
// particles and fills the block lists, then the lattice step.
static vlb_status one_step(vlb_ctx* c, bool last) {
  PState cur = c->ps[c->pcur], nxt = c->ps[1 - c->pcur];
  const double* pin = c->partial[c->pp];
  if (c->np > 0 && !c->P.scan)
    HIP_TRY(c, launch_particles(c->P, cur, nxt, c->pc, bin_lists(c), pin,
                                c->have_partials, kModeUpdate, c->flags,
                                c->stream));
  StepLaunch a;
  a.P = &c->P;
  a.out = last;
  a.have = c->have_partials;
  a.B = context_step_bufs(c);
  a.ev_start = a.ev_stop = nullptr;
  if (c->timing) {
    if (c->ev_used + 2 > c->ev.size()) {
      for (int k = 0; k < 64; ++k) {
        hipEvent_t e;
        HIP_TRY(c, hipEventCreate(&e));
        c->ev.push_back(e);
      }
    }
    a.ev_start = c->ev[c->ev_used];
    a.ev_stop = c->ev[c->ev_used + 1];
    c->ev_used += 2;
  }
  HIP_TRY(c, launch_step(c->prec, a, c->stream));
  context_advance(c, 1);
  return VLB_OK;
}


vlb_status vlb_step(vlb_ctx* c, int64_t nsteps) {
  if (!c) return VLB_EINVAL;
  if (nsteps < 0) return fail(c, VLB_EINVAL, "nsteps must be >= 0");
  if (!c->initialized) return fail(c, VLB_ESTATE, "vlb_init has not succeeded");
  for (int64_t k = 0; k < nsteps; ++k) {
    vlb_status st = one_step(c, k == nsteps - 1);
    if (st != VLB_OK) return st;
  }
  vlb_status st = check_flags(c);
  if (st != VLB_OK) c->initialized = false;
  return st;
}

vlb_status vlb_read_field(vlb_ctx* c, int32_t field, double* dst,
                          int32_t dst_is_device) {
  if (!c || !dst) return VLB_EINVAL;
  if (!c->initialized) return fail(c, VLB_ESTATE, "no valid state to read");
  const size_t N = (size_t)c->P.N;
  const hipMemcpyKind kind =
      dst_is_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (field >= VLB_FIELD_RHO && field <= VLB_FIELD_DFS) {
    HIP_TRY(c, hipMemcpyAsync(dst, c->macro + (size_t)field * N,
                              N * sizeof(double), kind, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return VLB_OK;
  }
  if (field == VLB_FIELD_F || field == VLB_FIELD_G) {
    const void* pop = field == VLB_FIELD_F ? c->f[c->cur] : c->g[c->cur];
    double* tmp = dst;
    if (!dst_is_device) {
      HIP_TRY(c, hipMalloc((void**)&tmp, 9 * N * sizeof(double)));
    }
    hipError_t e = launch_unpack(c->prec, c->P, pop, c->plane,
                                 field == VLB_FIELD_G, tmp, c->stream);
    if (e == hipSuccess && !dst_is_device)
      e = hipMemcpyAsync(dst, tmp, 9 * N * sizeof(double),
                         hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (!dst_is_device) (void)hipFree(tmp);
    if (e != hipSuccess) return hip_fail(c, e, "read populations");
    return VLB_OK;
  }
  return fail(c, VLB_EINVAL, "unknown field");
}

vlb_status vlb_read_particles(vlb_ctx* c, int32_t n, vlb_particle_state* dst) {
  if (!c || (n > 0 && !dst)) return VLB_EINVAL;
  if (n < 0 || n > c->np) return fail(c, VLB_EINVAL, "bad particle count");
  if (!c->initialized) return fail(c, VLB_ESTATE, "no valid state to read");
  if (n == 0) return VLB_OK;
  const int np = c->np;
  PState cur = c->ps[c->pcur];
  HIP_TRY(c, launch_particles(c->P, cur, c->ps[1 - c->pcur], c->pc, lists(c),
                              c->partial[c->pp], c->have_partials,
                              kModeReduceOnly, c->flags, c->stream));
  HIP_TRY(c, launch_particle_sums(c->P, cur, c->pc, c->macro, c->thermal4,
                                  c->stream));
  std::vector<double> st(12 * (size_t)np), th(4 * (size_t)np);
  HIP_TRY(c, hipMemcpyAsync(st.data(), c->pmem[c->pcur], st.size() * 8,
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipMemcpyAsync(th.data(), c->thermal4, th.size() * 8,
                            hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  for (int k = 0; k < n; ++k) {
    vlb_particle_state& o = dst[k];
    o.x = st[k];
    o.y = st[np + k];
    o.theta = st[2 * np + k];
    o.ux = st[3 * np + k];
    o.uy = st[4 * np + k];
    o.omega = st[5 * np + k];
    o.Fx = st[9 * np + k];
    o.Fy = st[10 * np + k];
    o.Tz = st[11 * np + k];
    o.T_mean = th[4 * k];
    o.T_min = th[4 * k + 1];
    o.E_solid = th[4 * k + 2];
    o.fs_sum = th[4 * k + 3];
  }
  return VLB_OK;
}

vlb_status vlb_read_ownership(vlb_ctx* c, int32_t* count, int32_t* ids,
                              int32_t* full) {
  if (!c || !count || !ids || !full) return VLB_EINVAL;
  if (!c->initialized) return fail(c, VLB_ESTATE, "no valid state to read");
  const size_t N = (size_t)c->P.N, K = (size_t)c->P.kmax;
  int *dc = nullptr, *di = nullptr, *df = nullptr;
  hipError_t e = hipMalloc((void**)&dc, N * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&di, N * K * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void**)&df, N * K * sizeof(int));
  PState cur = c->ps[c->pcur];
  if (e == hipSuccess && !c->P.scan)
    e = launch_particles(c->P, cur, cur, c->pc, bin_lists(c),
                         c->partial[c->pp], 0, kModeBinOnly, c->flags,
                         c->stream);
  if (e == hipSuccess)
    e = launch_ownership(c->P, cur, c->pc, lists(c), 0, c->P.nblocks, dc, di,
                         df, c->flags, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(count, dc, N * sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(ids, di, N * K * sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(full, df, N * K * sizeof(int), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (dc) (void)hipFree(dc);
  if (di) (void)hipFree(di);
  if (df) (void)hipFree(df);
  if (e != hipSuccess) return hip_fail(c, e, "read ownership");
  return VLB_OK;
}

// ---- ownership read-out that allocates nothing ---------------------------
//
// The staging buffer lives in a file-scope device array.  Its name is a
// host-side stand-in in host code; the device address comes from
// hipGetSymbolAddress, taken once per device with that device current and
// kept in g_scratch_ptr.  Only that pointer is handed to kernels and copies.
constexpr size_t kScratchInts = (size_t)4 << 20;   // 16 MiB
static __device__ __align__(256) int scratch[kScratchInts];

constexpr int kMaxDevices = 64;
static int* g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

static hipError_t scratch_for_device(int dev, int** out) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != dev) {
      const hipError_t e2 = hipSetDevice(prev);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = (int*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Checkpoint layout: header, then f and g (current copies, storage form),
// h, macro fields, particle state (12 x np doubles), slot counts (np ints),
// partials (np x maxb x 3 doubles).
struct SaveHeader {
  char magic[8];
  int32_t nx, ny, prec, np, maxb, have_partials;
  int64_t step;
};

static size_t partial_bytes(const vlb_ctx* c) {
  const size_t slots = c->P.scan ? (size_t)c->np * c->P.nblocks
                                 : (size_t)c->np * c->maxb;
  return slots * kRedVals * sizeof(double);
}

static size_t save_size(const vlb_ctx* c) {
  const size_t N = (size_t)c->P.N;
  return sizeof(SaveHeader) + 2 * 9 * c->plane * c->pop_elem + N * c->h_elem +
         6 * N * 8 + 12 * (size_t)c->np * 8 + (size_t)c->np * 4 +
         partial_bytes(c);
}

vlb_status vlb_save(vlb_ctx* c, void* buf, size_t* inout_len) {
  if (!c || !inout_len) return VLB_EINVAL;
  const size_t need = save_size(c);
  if (!buf) {
    *inout_len = need;
    return VLB_OK;
  }
  if (*inout_len < need) return fail(c, VLB_EINVAL, "checkpoint buffer too small");
  if (!c->initialized) return fail(c, VLB_ESTATE, "no valid state to save");
  SaveHeader hd;
  memset(&hd, 0, sizeof(hd));
  memcpy(hd.magic, "VLBCKPT1", 8);
  hd.nx = c->P.nx; hd.ny = c->P.ny; hd.prec = c->prec; hd.np = c->np;
  hd.maxb = c->maxb; hd.have_partials = c->have_partials; hd.step = c->step;
  char* o = (char*)buf;
  memcpy(o, &hd, sizeof(hd));
  o += sizeof(hd);
  const size_t N = (size_t)c->P.N, pb = 9 * c->plane * c->pop_elem;
  const hipMemcpyKind D2H = hipMemcpyDeviceToHost;
  HIP_TRY(c, hipMemcpyAsync(o, c->f[c->cur], pb, D2H, c->stream)); o += pb;
  HIP_TRY(c, hipMemcpyAsync(o, c->g[c->cur], pb, D2H, c->stream)); o += pb;
  HIP_TRY(c, hipMemcpyAsync(o, c->h[c->cur], N * c->h_elem, D2H, c->stream)); o += N * c->h_elem;
  HIP_TRY(c, hipMemcpyAsync(o, c->macro, 6 * N * 8, D2H, c->stream)); o += 6 * N * 8;
  if (c->np > 0) {
    const size_t n = (size_t)c->np;
    HIP_TRY(c, hipMemcpyAsync(o, c->pmem[c->pcur], 12 * n * 8, D2H, c->stream)); o += 12 * n * 8;
    HIP_TRY(c, hipMemcpyAsync(o, c->pslot[c->pcur], n * 4, D2H, c->stream)); o += n * 4;
    HIP_TRY(c, hipMemcpyAsync(o, c->partial[c->pp], partial_bytes(c), D2H, c->stream));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  *inout_len = need;
  return VLB_OK;
}

vlb_status vlb_load(vlb_ctx* c, const void* buf, size_t len) {
  if (!c || !buf) return VLB_EINVAL;
  if (len < sizeof(SaveHeader) || len < save_size(c))
    return fail(c, VLB_EINVAL, "checkpoint too short");
  SaveHeader hd;
  memcpy(&hd, buf, sizeof(hd));
  if (memcmp(hd.magic, "VLBCKPT1", 8) != 0 || hd.nx != c->P.nx ||
      hd.ny != c->P.ny || hd.prec != c->prec || hd.np != c->np ||
      hd.maxb != c->maxb)
    return fail(c, VLB_EINVAL, "checkpoint does not match this context");
  if (c->np > 0 && c->parts.empty())
    return fail(c, VLB_ESTATE, "set the particles before loading");
  const char* o = (const char*)buf + sizeof(hd);
  const size_t N = (size_t)c->P.N, pb = 9 * c->plane * c->pop_elem;
  const hipMemcpyKind H2D = hipMemcpyHostToDevice;
  c->cur = 0;
  c->pcur = 0;
  HIP_TRY(c, hipMemcpyAsync(c->f[0], o, pb, H2D, c->stream)); o += pb;
  HIP_TRY(c, hipMemcpyAsync(c->g[0], o, pb, H2D, c->stream)); o += pb;
  HIP_TRY(c, hipMemcpyAsync(c->h[0], o, N * c->h_elem, H2D, c->stream)); o += N * c->h_elem;
  HIP_TRY(c, hipMemcpyAsync(c->macro, o, 6 * N * 8, H2D, c->stream)); o += 6 * N * 8;
  if (c->np > 0) {
    const size_t n = (size_t)c->np;
    std::vector<double> cst(4 * n);
    std::vector<int> fx(n);
    for (size_t k = 0; k < n; ++k) {
      cst[k] = c->parts[k].radius;
      cst[n + k] = c->parts[k].rho_s;
      cst[2 * n + k] = c->parts[k].T_init;
      cst[3 * n + k] = c->parts[k].radius_minor > 0.0
                           ? c->parts[k].radius_minor
                           : c->parts[k].radius;
      fx[k] = (c->parts[k].fixed ? 1 : 0) | (c->parts[k].hold_T ? 2 : 0);
    }
    HIP_TRY(c, hipMemcpyAsync(c->pmem[0], o, 12 * n * 8, H2D, c->stream)); o += 12 * n * 8;
    HIP_TRY(c, hipMemcpyAsync(c->pslot[0], o, n * 4, H2D, c->stream)); o += n * 4;
    c->pp = 0;
    HIP_TRY(c, hipMemcpyAsync(c->partial[0], o, partial_bytes(c), H2D, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->pconst, cst.data(), cst.size() * 8, H2D, c->stream));
    HIP_TRY(c, hipMemcpyAsync(c->pfixed, fx.data(), fx.size() * 4, H2D, c->stream));
  }
  HIP_TRY(c, clear_lists(c));
  HIP_TRY(c, hipMemsetAsync(c->flags, 0, 4 * sizeof(int), c->stream));
  if (c->np > 0 && !c->P.scan)   // the lists of the restored positions
    HIP_TRY(c, launch_particles(c->P, c->ps[0], c->ps[0], c->pc, bin_lists(c),
                                c->partial[0], 0, kModeBinOnly, c->flags,
                                c->stream));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  c->have_partials = hd.have_partials;
  c->step = hd.step;
  c->initialized = true;
  return VLB_OK;
}

vlb_status vlb_read_ownership_noalloc(vlb_ctx* c, int32_t* count,
                                      int32_t* ids, int32_t* full) {
  if (!c || !count || !ids || !full) return VLB_EINVAL;
  if (!c->initialized) return fail(c, VLB_ESTATE, "no valid state to read");
  int* base = nullptr;
  HIP_TRY(c, scratch_for_device(c->device, &base));
  const size_t K = (size_t)c->P.kmax;
  // tiles per chunk: count, ids and full of every cell of a tile in scratch
  const size_t per_tile = (size_t)kBlock * (1 + 2 * K);
  const int chunk = (int)(kScratchInts / per_tile);
  if (chunk < 1)
    return fail(c, VLB_EINVAL, "ownership scratch too small for kmax");
  PState cur = c->ps[c->pcur];
  if (!c->P.scan)   // the lists of the current positions, as the step reads
    HIP_TRY(c, launch_particles(c->P, cur, cur, c->pc, bin_lists(c),
                                c->partial[c->pp], 0, kModeBinOnly, c->flags,
                                c->stream));
  const size_t N = (size_t)c->P.N;
  for (int t0 = 0; t0 < c->P.nblocks; t0 += chunk) {
    const int nt = c->P.nblocks - t0 < chunk ? c->P.nblocks - t0 : chunk;
    const size_t c0 = (size_t)t0 * kBlock;
    const size_t cend = c0 + (size_t)nt * kBlock < N ? c0 + (size_t)nt * kBlock : N;
    const size_t nc = cend - c0;
    int* dc = base;
    int* di = base + (size_t)nt * kBlock;
    int* df = di + (size_t)nt * kBlock * K;
    HIP_TRY(c, launch_ownership(c->P, cur, c->pc, lists(c), t0, nt, dc, di, df,
                                c->flags, c->stream));
    const hipMemcpyKind D2H = hipMemcpyDeviceToHost;
    HIP_TRY(c, hipMemcpyAsync(count + c0, dc, nc * sizeof(int), D2H, c->stream));
    HIP_TRY(c, hipMemcpyAsync(ids + c0 * K, di, nc * K * sizeof(int), D2H,
                              c->stream));
    HIP_TRY(c, hipMemcpyAsync(full + c0 * K, df, nc * K * sizeof(int), D2H,
                              c->stream));
  }
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return VLB_OK;
}

int64_t vlb_step_count(const vlb_ctx* c) { return c ? c->step : -1; }

vlb_status vlb_timing_enable(vlb_ctx* c, int32_t on) {
  if (!c) return VLB_EINVAL;
  c->timing = on != 0;
  return VLB_OK;
}

vlb_status vlb_timing_read(vlb_ctx* c, double* total_ms, int64_t* count) {
  if (!c || !total_ms || !count) return VLB_EINVAL;
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  double tot = 0.0;
  for (size_t k = 0; k + 1 < c->ev_used; k += 2) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, c->ev[k], c->ev[k + 1]));
    tot += ms;
  }
  *total_ms = tot;
  *count = (int64_t)(c->ev_used / 2);
  c->ev_used = 0;
  return VLB_OK;
}

vlb_status vlb_stream_probe(vlb_ctx* c, int32_t reps, double* us_per_launch) {
  if (!c) return VLB_EINVAL;
  if (!us_per_launch || reps <= 0)
    return fail(c, VLB_EINVAL, "stream probe: reps must be > 0 and the "
                               "output pointer non-null");
  if (!c->initialized) return fail(c, VLB_ESTATE, "vlb_init has not succeeded");
  const StepBufs B = context_step_bufs(c);
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  HIP_TRY(c, hipEventCreate(&ev.a));
  HIP_TRY(c, hipEventCreate(&ev.b));
  HIP_TRY(c, launch_stream_probe(c->prec, c->P, B, c->stream));   // warm
  HIP_TRY(c, hipEventRecord(ev.a, c->stream));
  for (int32_t k = 0; k < reps; ++k)
    HIP_TRY(c, launch_stream_probe(c->prec, c->P, B, c->stream));
  HIP_TRY(c, hipEventRecord(ev.b, c->stream));
  HIP_TRY(c, hipEventSynchronize(ev.b));
  float ms = 0.f;
  HIP_TRY(c, hipEventElapsedTime(&ms, ev.a, ev.b));
  *us_per_launch = 1e3 * (double)ms / reps;
  return VLB_OK;
}

size_t vlb_device_bytes(const vlb_ctx* c) { return c ? c->dev_bytes : 0; }

const char* vlb_last_error(const vlb_ctx* c) {
  return c ? c->err.c_str() : g_create_error.c_str();
}

const char* vlb_build_hash(void) { return VLB_SOURCE_HASH; }

void vlb_destroy(vlb_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_particles(c);
  for (int k = 0; k < 2; ++k) {
    if (c->f[k]) (void)hipFree(c->f[k]);
    if (c->g[k]) (void)hipFree(c->g[k]);
  }
  for (int k = 0; k < 2; ++k)
    if (c->h[k]) (void)hipFree(c->h[k]);
  if (c->macro) (void)hipFree(c->macro);
  for (int k = 0; k < 3; ++k) {
    if (c->tcount[k]) (void)hipFree(c->tcount[k]);
    if (c->blk_cnt[k]) (void)hipFree(c->blk_cnt[k]);
    if (c->blk_ent[k]) (void)hipFree(c->blk_ent[k]);
    if (c->bin_cnt[k]) (void)hipFree(c->bin_cnt[k]);
    if (c->bin_ent[k]) (void)hipFree(c->bin_ent[k]);
  }
  if (c->flags) (void)hipFree(c->flags);
  if (c->flags_host) (void)hipHostFree(c->flags_host);
  for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
  delete c;
}

}  // extern "C"
