// vlb3_api.hip -- host implementation of the three-dimensional C ABI
// (include/vlb3.h): device memory of a context, the kernel constants derived
// from the descriptor, and the order of the kernels of each step.
//
// One step: the sphere pass (momentum-exchange sums of the previous step,
// then the Newton-Euler update into the other sphere buffer), the geometry
// pass at the new positions (the shares of the cells of the tiles spheres
// may reach), then the lattice step (both lattices, the volumetric step,
// the per-(sphere, tile) partial sums).  The lattice populations, the carrier
// of [df_s/dt] and the sphere state are double-buffered.
#include <math.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "vlb3.h"
#include "vlb3_internal.h"

using namespace vlb3;

struct vlb3_ctx {
  Params3 P;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;
  // populations and carrier in the storage type (8 or 4 bytes, esz)
  void *f[2] = {nullptr, nullptr}, *g[2] = {nullptr, nullptr};
  void *h[2] = {nullptr, nullptr};
  size_t esz = sizeof(double);
  double *S[2] = {nullptr, nullptr};   // sphere states
  double* C = nullptr;                 // sphere constants
  double* partial = nullptr;
  double* macro = nullptr;
  double* sums = nullptr;              // per-sphere thermal outputs
  int* gid = nullptr;                  // geometry pass: ids and count
  double* gw = nullptr;                //   and shares per cell,
  unsigned long long* tmask = nullptr; //   each tile's candidate spheres,
  int* items = nullptr;                //   the partly covered cell slots
  int* nitems = nullptr;
  int* flags = nullptr;
  int cur = 0, scur = 0, have = 0;
  bool initialized = false;
  int64_t step = 0;
  size_t dev_bytes = 0;
  std::vector<double> host_spheres;    // the initial state, [field][np]
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  double timed_ms = 0.0;
  int64_t timed_n = 0;
  std::string err;
};

static std::string g_create_error3;

static vlb_status fail3(vlb3_ctx* c, vlb_status s, const std::string& m) {
  if (c) c->err = m; else g_create_error3 = m;
  return s;
}

#define HIP3(ctx, expr)                                                  \
  do {                                                                   \
    hipError_t e_ = (expr);                                              \
    if (e_ != hipSuccess)                                                \
      return fail3((ctx), VLB_EHIP,                                      \
                   std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

static bool dalloc3b(vlb3_ctx* c, void** p, size_t bytes) {
  if (hipMalloc(p, bytes ? bytes : 8) != hipSuccess) {
    *p = nullptr;
    return false;
  }
  c->dev_bytes += bytes ? bytes : 8;
  return true;
}

static bool dalloc3(vlb3_ctx* c, double** p, size_t n) {
  if (hipMalloc((void**)p, (n ? n : 1) * sizeof(double)) != hipSuccess) {
    *p = nullptr;
    return false;
  }
  c->dev_bytes += (n ? n : 1) * sizeof(double);
  return true;
}

// The Gauss-Legendre table goes to each device once.
static std::mutex g_quad_mutex;
static std::vector<int> g_quad_done;

static hipError_t ensure_quadrature(int dev) {
  std::lock_guard<std::mutex> lock(g_quad_mutex);
  for (int d : g_quad_done)
    if (d == dev) return hipSuccess;
  hipError_t e = upload_quadrature();
  if (e == hipSuccess) g_quad_done.push_back(dev);
  return e;
}

static std::string check_desc(const vlb3_domain_desc* d) {
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return "nx, ny, nz must be >= 1";
  if ((double)d->nx * d->ny * d->nz >= 2147483647.0)
    return "nx*ny*nz must be < 2^31";
  for (int a = 0; a < 3; ++a) {
    const int lo = d->face_flow[2 * a], hi = d->face_flow[2 * a + 1];
    if ((lo != VLB_PERIODIC && lo != VLB_WALL) ||
        (hi != VLB_PERIODIC && hi != VLB_WALL))
      return "face_flow must be VLB_PERIODIC or VLB_WALL";
    if ((lo == VLB_PERIODIC) != (hi == VLB_PERIODIC))
      return "periodic faces come in pairs";
  }
  for (int f = 0; f < 6; ++f)
    if (d->face_thermal[f] != VLB_ADIABATIC &&
        d->face_thermal[f] != VLB_DIRICHLET)
      return "face_thermal must be VLB_ADIABATIC or VLB_DIRICHLET";
  if (!(d->tau_f > 0.5)) return "tau_f must be > 1/2";
  if (!(d->rho_f > 0.0) || !(d->cv_f > 0.0) || !(d->lambda_f > 0.0) ||
      !(d->R_lambda > 0.0) || !(d->R_cv > 0.0))
    return "rho_f, cv_f, lambda_f, R_lambda, R_cv must be > 0";
  if (d->sigma_rule != 0 && d->sigma_rule != 1) return "sigma_rule must be 0 or 1";
  if (d->kmax < 1 || d->kmax > kMaxK) return "kmax must be in 1..4";
  if (d->precision != VLB_FP64 && d->precision != VLB_FP32)
    return "precision must be VLB_FP64 or VLB_FP32 (storage; FP64 arithmetic)";
  if (d->coll_range < 0.0) return "coll_range must be >= 0";
  if (!(d->init_rho > 0.0)) return "init_rho must be > 0";
  return "";
}

extern "C" {

vlb_status vlb3_create(const vlb3_domain_desc* desc, int32_t nspheres,
                       const vlb3_sphere_desc* spheres, void* hip_stream,
                       vlb3_ctx** out) {
  if (!desc || !out) return fail3(nullptr, VLB_EINVAL, "desc and out are required");
  *out = nullptr;
  const std::string bad = check_desc(desc);
  if (!bad.empty()) return fail3(nullptr, VLB_EINVAL, bad);
  if (nspheres < 0 || nspheres > kMaxSpheres)
    return fail3(nullptr, VLB_EINVAL, "nspheres must be in 0..64");
  if (nspheres > 0 && !spheres)
    return fail3(nullptr, VLB_EINVAL, "spheres is NULL");
  if (nspheres > 0 &&
      (double)desc->nx * desc->ny * desc->nz * kMaxK >= 2147483647.0)
    return fail3(nullptr, VLB_EINVAL,
                 "with spheres nx*ny*nz must be < 2^29 (cell slots are int)");
  const double L[3] = {(double)desc->nx, (double)desc->ny, (double)desc->nz};
  for (int p = 0; p < nspheres; ++p) {
    const vlb3_sphere_desc& s = spheres[p];
    if (!(s.radius > 0.0) || !(s.rho_s > 0.0))
      return fail3(nullptr, VLB_EINVAL, "sphere " + std::to_string(p) +
                                            ": radius and rho_s must be > 0");
    const double c[3] = {s.x, s.y, s.z};
    for (int a = 0; a < 3; ++a)
      if (!(c[a] >= 0.0 && c[a] < L[a]))
        return fail3(nullptr, VLB_EINVAL,
                     "sphere " + std::to_string(p) + ": centre outside the domain");
  }
  vlb3_ctx* c = new (std::nothrow) vlb3_ctx();
  if (!c) return fail3(nullptr, VLB_ENOMEM, "host allocation failed");
  auto give_up = [&](vlb_status st, const std::string& m) {
    vlb3_destroy(c);
    return fail3(nullptr, st, m);
  };
  (void)hipGetDevice(&c->device);
  if (ensure_quadrature(c->device) != hipSuccess)
    return give_up(VLB_EHIP, "upload of the quadrature table failed");
  if (hip_stream) {
    c->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess)
      return give_up(VLB_EHIP, "stream creation failed");
    c->own_stream = true;
  }
  Params3& P = c->P;
  memset(&P, 0, sizeof P);
  P.nx = desc->nx; P.ny = desc->ny; P.nz = desc->nz;
  P.N = desc->nx * desc->ny * desc->nz;
  P.nblocks = (P.N + kBlock - 1) / kBlock;
  P.np = nspheres;
  P.kmax = desc->kmax;
  for (int a = 0; a < 3; ++a) P.per[a] = desc->face_flow[2 * a] == VLB_PERIODIC;
  for (int f = 0; f < 6; ++f) {
    P.wall_dirichlet[f] = desc->face_thermal[f] == VLB_DIRICHLET;
    for (int a = 0; a < 3; ++a) P.u_wall[f][a] = desc->u_wall[f][a];
    P.T_wall[f] = desc->T_wall[f];
  }
  P.rho0 = desc->init_rho;
  P.rho_f = desc->rho_f;
  P.cv_f = desc->cv_f;
  P.cv_s = desc->R_cv * desc->cv_f;
  P.lam_f = desc->lambda_f;
  P.lam_s = desc->R_lambda * desc->lambda_f;
  P.cref = 2.0 * P.cv_f * P.cv_s / (P.cv_f + P.cv_s);
  P.snu = 1.0 / desc->tau_f;
  P.sq = 1.0 / (0.5 + (1.0 / 12.0) / (desc->tau_f - 0.5));
  P.sigma_rule = desc->sigma_rule;
  for (int a = 0; a < 3; ++a) {
    P.body[a] = desc->body_force[a];
    P.grav[a] = desc->gravity[a];
    P.init_u[a] = desc->init_u[a];
  }
  P.beta = desc->beta;
  P.T_ref = desc->T_ref;
  P.zeta = desc->coll_range;
  P.k_pp = desc->coll_stiff_pp;
  P.k_pw = desc->coll_stiff_pw;
  P.init_T = desc->init_T;
  // Storage: FP64, or FP32 deviations from the equilibria of the initial
  // state at rest (w_q rho_0 for f; w_q c_ref T_0 for g, the rest
  // population's c_v,f T_0 - (1 - w_0) c_ref T_0), so that FP32 holds the
  // small departures rather than values of order one.
  P.f32 = desc->precision == VLB_FP32;
  c->esz = P.f32 ? sizeof(float) : sizeof(double);
  {
    const double w19[kQ] = {1.0 / 3.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0,
                            1.0 / 18.0, 1.0 / 18.0, 1.0 / 18.0, 1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0,
                            1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
    for (int q = 0; q < kQ; ++q) P.fshift[q] = P.f32 ? w19[q] * P.rho0 : 0.0;
    const double cT0 = P.cref * P.init_T;
    P.gshift[0] = P.f32 ? P.cv_f * P.init_T - (1.0 - 0.25) * cT0 : 0.0;
    for (int q = 1; q < kQG; ++q) P.gshift[q] = P.f32 ? 0.125 * cT0 : 0.0;
  }
  // One step moves 432 B a cell in FP64, 216 B in FP32.  Above 320 MB
  // (1.25 x the Infinity Cache) the next step cannot find the populations
  // in the cache, and non-temporal stores leave it to the loads (80 x 80 x
  // 320 channel, FP64: 254 -> 245 us a step; the 382 MB of the 96^3 box:
  // unchanged).
  const size_t moved = (size_t)P.N * (2 * (kQ + kQG + 1) * c->esz);
  P.nt_stores = moved > ((size_t)320 << 20);

  const size_t N = (size_t)P.N, np = (size_t)(nspheres > 0 ? nspheres : 1);
  bool ok = true;
  for (int b = 0; b < 2 && ok; ++b)
    ok = dalloc3b(c, &c->f[b], N * kQ * c->esz) &&
         dalloc3b(c, &c->g[b], N * kQG * c->esz) &&
         dalloc3b(c, &c->h[b], N * c->esz) &&
         dalloc3(c, &c->S[b], np * kFields);
  ok = ok && dalloc3(c, &c->C, np * kConsts) && dalloc3(c, &c->macro, N * kMacro) &&
       dalloc3(c, &c->partial, np * (size_t)P.nblocks * kPartial) &&
       dalloc3(c, &c->sums, np * 5);
  if (ok && nspheres > 0)
    ok = dalloc3(c, &c->gw, N * kMaxK) &&
         hipMalloc((void**)&c->gid, N * sizeof(int)) == hipSuccess &&
         hipMalloc((void**)&c->tmask, (size_t)P.nblocks *
                                          sizeof(unsigned long long)) ==
             hipSuccess &&
         hipMalloc((void**)&c->items, kSegs * seg_items(P) * sizeof(int)) ==
             hipSuccess &&
         hipMalloc((void**)&c->nitems, kSegs * sizeof(int)) == hipSuccess;
  if (ok && hipMalloc((void**)&c->flags, sizeof(int)) != hipSuccess) ok = false;
  if (!ok) return give_up(VLB_ENOMEM, "device allocation failed");
  // sphere constants and the initial state
  std::vector<double> hc(np * kConsts, 0.0);
  c->host_spheres.assign(np * kFields, 0.0);
  for (int p = 0; p < nspheres; ++p) {
    const vlb3_sphere_desc& s = spheres[p];
    hc[cR * np + p] = s.radius;
    hc[cRho * np + p] = s.rho_s;
    hc[cTinit * np + p] = s.T_init;
    hc[cFixed * np + p] = s.fixed ? 1.0 : 0.0;
    const double v[9] = {s.x, s.y, s.z, s.ux, s.uy, s.uz, s.ox, s.oy, s.oz};
    for (int a = 0; a < 9; ++a) c->host_spheres[(fX + a) * np + p] = v[a];
  }
  if (hipMemcpy(c->C, hc.data(), hc.size() * sizeof(double),
                hipMemcpyHostToDevice) != hipSuccess)
    return give_up(VLB_EHIP, "copy of the sphere constants failed");
  *out = c;
  return VLB_OK;
}

vlb_status vlb3_init(vlb3_ctx* c) {
  if (!c) return VLB_EINVAL;
  const size_t np = (size_t)(c->P.np > 0 ? c->P.np : 1);
  // state 0: the given centres and velocities; the previous velocities
  // equal the current ones, the sums are zero
  std::vector<double> s = c->host_spheres;
  for (size_t p = 0; p < np; ++p)
    for (int a = 0; a < 3; ++a) {
      s[(fUp + a) * np + p] = s[(fU + a) * np + p];
      s[(fOxp + a) * np + p] = s[(fOx + a) * np + p];
    }
  c->cur = c->scur = 0;
  c->have = 0;
  c->step = 0;
  HIP3(c, hipMemcpyAsync(c->S[0], s.data(), s.size() * sizeof(double),
                         hipMemcpyHostToDevice, c->stream));
  HIP3(c, hipMemsetAsync(c->flags, 0, sizeof(int), c->stream));
  HIP3(c, launch_init(c->P, c->f[0], c->g[0], c->h[0], c->macro, c->S[0], c->C,
                      c->flags, c->stream));
  int fl = 0;
  HIP3(c, hipMemcpyAsync(&fl, c->flags, sizeof(int), hipMemcpyDeviceToHost,
                         c->stream));
  HIP3(c, hipStreamSynchronize(c->stream));
  if (fl & kFlagOverlap) {
    c->initialized = false;
    return fail3(c, VLB_EOVERLAP, "more than kmax spheres reach one cell");
  }
  c->initialized = true;
  return VLB_OK;
}

vlb_status vlb3_step(vlb3_ctx* c, int64_t nsteps) {
  if (!c) return VLB_EINVAL;
  if (nsteps < 0) return fail3(c, VLB_EINVAL, "nsteps must be >= 0");
  if (!c->initialized) return fail3(c, VLB_ESTATE, "vlb3_init has not succeeded");
  const Params3& P = c->P;
  for (int64_t n = 0; n < nsteps; ++n) {
    const bool last = n == nsteps - 1;
    HIP3(c, launch_particles(P, c->S[c->scur], c->S[c->scur ^ 1], c->C,
                             c->partial, c->tmask, c->have, 1, c->stream));
    if (P.np > 0) c->scur ^= 1;
    HIP3(c, launch_geometry(P, c->S[c->scur], c->C, c->gid, c->gw, c->tmask,
                            c->items, c->nitems, c->flags, c->stream));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
      HIP3(c, hipEventCreate(&e0));
      HIP3(c, hipEventCreate(&e1));
      HIP3(c, hipEventRecord(e0, c->stream));
    }
    HIP3(c, launch_step(P, last, c->f[c->cur], c->f[c->cur ^ 1], c->g[c->cur],
                        c->g[c->cur ^ 1], c->h[c->cur], c->h[c->cur ^ 1],
                        c->S[c->scur], c->C, c->gid, c->gw, c->tmask,
                        c->partial, c->macro, c->flags, c->stream));
    if (c->timing) {
      HIP3(c, hipEventRecord(e1, c->stream));
      c->events.push_back({e0, e1});
    }
    c->cur ^= 1;
    c->have = 1;
  }
  int fl = 0;
  HIP3(c, hipMemcpyAsync(&fl, c->flags, sizeof(int), hipMemcpyDeviceToHost,
                         c->stream));
  HIP3(c, hipStreamSynchronize(c->stream));
  c->step += nsteps;
  if (fl) {
    c->initialized = false;
    return fail3(c, (fl & kFlagUnstable) ? VLB_EUNSTABLE : VLB_EOVERLAP,
                 (fl & kFlagUnstable)
                     ? "a cell reached rho <= 0 or a non-finite value"
                     : "more than kmax spheres reach one cell");
  }
  return VLB_OK;
}

vlb_status vlb3_read_field(vlb3_ctx* c, int32_t field, double* dst,
                           int32_t dst_is_device) {
  if (!c || !dst) return VLB_EINVAL;
  if (field < 0 || field >= kMacro) return fail3(c, VLB_EINVAL, "unknown field");
  if (!c->initialized) return fail3(c, VLB_ESTATE, "no state to read");
  const size_t N = (size_t)c->P.N;
  HIP3(c, hipMemcpyAsync(dst, c->macro + (size_t)field * N, N * sizeof(double),
                         dst_is_device ? hipMemcpyDeviceToDevice
                                       : hipMemcpyDeviceToHost,
                         c->stream));
  HIP3(c, hipStreamSynchronize(c->stream));
  return VLB_OK;
}

vlb_status vlb3_read_populations(vlb3_ctx* c, int32_t which, double* dst) {
  if (!c || !dst || (which != 0 && which != 1)) return VLB_EINVAL;
  if (!c->initialized) return fail3(c, VLB_ESTATE, "no state to read");
  const size_t N = (size_t)c->P.N, nq = which ? kQG : kQ, n = N * nq;
  const void* src = which ? c->g[c->cur] : c->f[c->cur];
  if (!c->P.f32) {
    HIP3(c, hipMemcpyAsync(dst, src, n * sizeof(double),
                           hipMemcpyDeviceToHost, c->stream));
    HIP3(c, hipStreamSynchronize(c->stream));
    return VLB_OK;
  }
  // FP32 storage: the deviations, plus the reference, as FP64
  std::vector<float> tmp(n);
  HIP3(c, hipMemcpyAsync(tmp.data(), src, n * sizeof(float),
                         hipMemcpyDeviceToHost, c->stream));
  HIP3(c, hipStreamSynchronize(c->stream));
  const double* shift = which ? c->P.gshift : c->P.fshift;
  for (size_t q = 0; q < nq; ++q)
    for (size_t i = 0; i < N; ++i)
      dst[q * N + i] = (double)tmp[q * N + i] + shift[q];
  return VLB_OK;
}

vlb_status vlb3_read_spheres(vlb3_ctx* c, int32_t n, vlb3_sphere_state* dst) {
  if (!c || n < 0 || n > c->P.np || (n > 0 && !dst)) return VLB_EINVAL;
  if (!c->initialized) return fail3(c, VLB_ESTATE, "no state to read");
  if (n == 0) return VLB_OK;
  const int np = c->P.np;
  // the sums of the last step, and the thermal outputs at its positions
  HIP3(c, launch_particles(c->P, c->S[c->scur], nullptr, c->C, c->partial,
                           c->tmask, c->have, 0, c->stream));
  HIP3(c, launch_sphere_sums(c->P, c->S[c->scur], c->C, c->macro, c->sums,
                             c->stream));
  std::vector<double> s((size_t)np * kFields), t((size_t)np * 5);
  HIP3(c, hipMemcpyAsync(s.data(), c->S[c->scur], s.size() * sizeof(double),
                         hipMemcpyDeviceToHost, c->stream));
  HIP3(c, hipMemcpyAsync(t.data(), c->sums, t.size() * sizeof(double),
                         hipMemcpyDeviceToHost, c->stream));
  HIP3(c, hipStreamSynchronize(c->stream));
  for (int p = 0; p < n; ++p) {
    vlb3_sphere_state& o = dst[p];
    double* v[15] = {&o.x, &o.y, &o.z, &o.ux, &o.uy, &o.uz, &o.ox, &o.oy,
                     &o.oz, &o.Fx, &o.Fy, &o.Fz, &o.Tx, &o.Ty, &o.Tz};
    const int fld[15] = {fX, fY, fZ, fU, fV, fW, fOx, fOy, fOz,
                         fFx, fFy, fFz, fTx, fTy, fTz};
    for (int a = 0; a < 15; ++a) *v[a] = s[(size_t)fld[a] * np + p];
    const double* r = &t[(size_t)p * 5];
    o.T_mean = r[2] > 0.0 ? r[0] / r[2] : 0.0;
    o.E_solid = r[1];
    o.fs_sum = r[2];
    o.T_min = isfinite(r[3]) ? r[3] : r[4];
  }
  return VLB_OK;
}

// Checkpoint layout: the header, then f, g, h of the current step (in the
// storage type), the macroscopic fields, and with spheres their current
// state, the last step's partial sums and tile candidate masks.
struct Save3Header {
  char magic[8];
  int32_t nx, ny, nz, f32, np, have;
  int64_t step;
};

static size_t save3_size(const vlb3_ctx* c) {
  const size_t N = (size_t)c->P.N, np = (size_t)c->P.np;
  size_t n = sizeof(Save3Header) + N * (kQ + kQG + 1) * c->esz +
             N * kMacro * sizeof(double);
  if (np > 0)
    n += np * kFields * sizeof(double) +
         np * (size_t)c->P.nblocks * kPartial * sizeof(double) +
         (size_t)c->P.nblocks * sizeof(unsigned long long);
  return n;
}

vlb_status vlb3_save(vlb3_ctx* c, void* buf, size_t* inout_len) {
  if (!c || !inout_len) return VLB_EINVAL;
  const size_t need = save3_size(c);
  if (!buf) {
    *inout_len = need;
    return VLB_OK;
  }
  if (*inout_len < need) return fail3(c, VLB_EINVAL, "checkpoint buffer too small");
  if (!c->initialized) return fail3(c, VLB_ESTATE, "no valid state to save");
  Save3Header hd;
  memset(&hd, 0, sizeof hd);
  memcpy(hd.magic, "VLB3CKP1", 8);
  hd.nx = c->P.nx; hd.ny = c->P.ny; hd.nz = c->P.nz; hd.f32 = c->P.f32;
  hd.np = c->P.np; hd.have = c->have; hd.step = c->step;
  char* o = (char*)buf;
  memcpy(o, &hd, sizeof hd);
  o += sizeof hd;
  const size_t N = (size_t)c->P.N, np = (size_t)c->P.np;
  const hipMemcpyKind D2H = hipMemcpyDeviceToHost;
  const size_t fb = N * kQ * c->esz, gb = N * kQG * c->esz, hb = N * c->esz;
  HIP3(c, hipMemcpyAsync(o, c->f[c->cur], fb, D2H, c->stream)); o += fb;
  HIP3(c, hipMemcpyAsync(o, c->g[c->cur], gb, D2H, c->stream)); o += gb;
  HIP3(c, hipMemcpyAsync(o, c->h[c->cur], hb, D2H, c->stream)); o += hb;
  HIP3(c, hipMemcpyAsync(o, c->macro, N * kMacro * 8, D2H, c->stream));
  o += N * kMacro * 8;
  if (np > 0) {
    const size_t sb = np * kFields * 8;
    const size_t pb = np * (size_t)c->P.nblocks * kPartial * 8;
    const size_t tb = (size_t)c->P.nblocks * 8;
    HIP3(c, hipMemcpyAsync(o, c->S[c->scur], sb, D2H, c->stream)); o += sb;
    HIP3(c, hipMemcpyAsync(o, c->partial, pb, D2H, c->stream)); o += pb;
    HIP3(c, hipMemcpyAsync(o, c->tmask, tb, D2H, c->stream));
  }
  HIP3(c, hipStreamSynchronize(c->stream));
  *inout_len = need;
  return VLB_OK;
}

vlb_status vlb3_load(vlb3_ctx* c, const void* buf, size_t len) {
  if (!c || !buf) return VLB_EINVAL;
  if (len < sizeof(Save3Header) || len < save3_size(c))
    return fail3(c, VLB_EINVAL, "checkpoint too short");
  Save3Header hd;
  memcpy(&hd, buf, sizeof hd);
  if (memcmp(hd.magic, "VLB3CKP1", 8) != 0 || hd.nx != c->P.nx ||
      hd.ny != c->P.ny || hd.nz != c->P.nz || hd.f32 != c->P.f32 ||
      hd.np != c->P.np)
    return fail3(c, VLB_EINVAL, "checkpoint does not match this context");
  const char* o = (const char*)buf + sizeof hd;
  const size_t N = (size_t)c->P.N, np = (size_t)c->P.np;
  const hipMemcpyKind H2D = hipMemcpyHostToDevice;
  const size_t fb = N * kQ * c->esz, gb = N * kQG * c->esz, hb = N * c->esz;
  c->cur = 0;
  c->scur = 0;
  HIP3(c, hipMemcpyAsync(c->f[0], o, fb, H2D, c->stream)); o += fb;
  HIP3(c, hipMemcpyAsync(c->g[0], o, gb, H2D, c->stream)); o += gb;
  HIP3(c, hipMemcpyAsync(c->h[0], o, hb, H2D, c->stream)); o += hb;
  HIP3(c, hipMemcpyAsync(c->macro, o, N * kMacro * 8, H2D, c->stream));
  o += N * kMacro * 8;
  if (np > 0) {
    const size_t sb = np * kFields * 8;
    const size_t pb = np * (size_t)c->P.nblocks * kPartial * 8;
    const size_t tb = (size_t)c->P.nblocks * 8;
    HIP3(c, hipMemcpyAsync(c->S[0], o, sb, H2D, c->stream)); o += sb;
    HIP3(c, hipMemcpyAsync(c->partial, o, pb, H2D, c->stream)); o += pb;
    HIP3(c, hipMemcpyAsync(c->tmask, o, tb, H2D, c->stream));
  }
  HIP3(c, hipMemsetAsync(c->flags, 0, sizeof(int), c->stream));
  // the copies read the caller's buffer: finish before returning
  HIP3(c, hipStreamSynchronize(c->stream));
  c->have = hd.have;
  c->step = hd.step;
  c->initialized = true;
  return VLB_OK;
}

vlb_status vlb3_timing_enable(vlb3_ctx* c, int32_t on) {
  if (!c) return VLB_EINVAL;
  c->timing = on != 0;
  return VLB_OK;
}

vlb_status vlb3_timing_read(vlb3_ctx* c, double* total_ms, int64_t* count) {
  if (!c || !total_ms || !count) return VLB_EINVAL;
  HIP3(c, hipStreamSynchronize(c->stream));
  double ms = 0.0;
  for (auto& e : c->events) {
    float x = 0.f;
    if (hipEventElapsedTime(&x, e.first, e.second) == hipSuccess) ms += x;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  *total_ms = ms;
  *count = (int64_t)c->events.size();
  c->events.clear();
  return VLB_OK;
}

int64_t vlb3_step_count(const vlb3_ctx* c) { return c ? c->step : -1; }

size_t vlb3_device_bytes(const vlb3_ctx* c) { return c ? c->dev_bytes : 0; }

const char* vlb3_last_error(const vlb3_ctx* c) {
  return c ? c->err.c_str() : g_create_error3.c_str();
}

void vlb3_destroy(vlb3_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (auto& e : c->events) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  for (int b = 0; b < 2; ++b) {
    if (c->f[b]) (void)hipFree(c->f[b]);
    if (c->g[b]) (void)hipFree(c->g[b]);
    if (c->h[b]) (void)hipFree(c->h[b]);
    if (c->S[b]) (void)hipFree(c->S[b]);
  }
  double* d[] = {c->C, c->macro, c->partial, c->sums, c->gw};
  if (c->gid) (void)hipFree(c->gid);
  if (c->tmask) (void)hipFree(c->tmask);
  if (c->items) (void)hipFree(c->items);
  if (c->nitems) (void)hipFree(c->nitems);
  for (double* p : d)
    if (p) (void)hipFree(p);
  if (c->flags) (void)hipFree(c->flags);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

}  // extern "C"
