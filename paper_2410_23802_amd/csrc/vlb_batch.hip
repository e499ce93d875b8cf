// vlb_batch.hip -- many independent domains advanced by one launch per step
// (the vlb_batch_* half of the C ABI in include/vlb.h).
//
// Each domain of a batch is an ordinary context (vlb_ctx) with its own
// device memory, created, initialised and read through the single-domain
// code.  Stepping is different: one launch of k_batch_step advances every
// domain, its persistent blocks walking a task table that lists all
// domains' particle-tile tasks and then all their tiles, one or two tiles
// per task.  The launch shape (number of persistent blocks), the table
// order, which domains stream their tiles in pairs and the kernel's
// occupancy are chosen by vlb_batch_autotune from measured candidates;
// steady-state steps are replayed from a captured two-step hipGraph.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "vlb_context.h"

using namespace vlb;

struct vlb_batch {
  std::vector<vlb_ctx*> cases;
  hipStream_t stream = nullptr;
  int prec = 0;
  int device = 0;
  int cus = 256;
  BatchCase* dcases = nullptr;
  BatchTask* dtasks = nullptr;
  size_t tasks_cap = 0;
  int ntasks = 0;
  int* dflags = nullptr;
  int* hflags = nullptr;
  int parity = 0;                // buffer parity of every domain (lockstep)
  int have = 0;                  // the partials of a previous step exist
  int64_t step = 0;
  bool initialized = false;
  vlb_batch_tuning tune;
  hipGraphExec_t graph = nullptr;  // two steps from parity 0, have = 1
  int64_t cells = 0;
  std::string err;
};

static std::string g_batch_create_error;

static vlb_status bfail(vlb_batch* b, vlb_status s, const std::string& m) {
  if (b) b->err = m; else g_batch_create_error = m;
  return s;
}

#define BHIP(b, expr)                                                   \
  do {                                                                  \
    hipError_t e_ = (expr);                                             \
    if (e_ != hipSuccess)                                               \
      return bfail((b), VLB_EHIP,                                       \
                   std::string(#expr) + ": " + hipGetErrorString(e_));  \
  } while (0)

// The task table for an order.  Particle-tile tasks (long dependency
// chains, few bytes) are spread evenly among the tiles (short, streaming)
// so that every stretch of the table mixes the two.  Order 0 keeps the
// tiles domain by domain; order 1 deals them to the 8 XCDs in contiguous
// bands: the block that runs slot w sits on XCD w % 8 (blocks reach the
// XCDs in turn and the grid is a multiple of 8), so each XCD's slots take
// its band's tiles in order, with its share of the particle tasks spread
// among them.
static std::vector<BatchTask> spread(const std::vector<BatchTask>& tiles,
                                     const std::vector<BatchTask>& part) {
  std::vector<BatchTask> out;
  out.reserve(tiles.size() + part.size());
  const size_t M = tiles.size(), Q = part.size();
  size_t t = 0;
  for (size_t k = 0; k < Q; ++k) {
    // particle task k goes before tile (k * M) / Q
    const size_t upto = (k * M) / Q;
    while (t < upto) out.push_back(tiles[t++]);
    out.push_back(part[k]);
  }
  while (t < M) out.push_back(tiles[t++]);
  return out;
}

// A domain of at least pair_min_tiles tiles (>= 0) streams tiles t and
// t + 1 (t even) in one task.
static bool paired(const vlb_batch_tuning& t, const Params& P) {
  return t.pair_min_tiles >= 0 && P.nblocks >= t.pair_min_tiles;
}

static std::vector<BatchTask> build_tasks(const vlb_batch* b,
                                          const vlb_batch_tuning& tune) {
  const int order = tune.order;
  std::vector<BatchTask> part, tiles;
  for (size_t i = 0; i < b->cases.size(); ++i) {
    const Params& P = b->cases[i]->P;
    for (int k = 0; k < P.np * P.maxr; ++k)
      part.push_back(make_int2((int)i, k));
  }
  for (size_t i = 0; i < b->cases.size(); ++i) {
    const Params& P = b->cases[i]->P;
    if (paired(tune, P))
      for (int t = 0; t < P.nblocks; t += 2)
        tiles.push_back(make_int2((int)i, kPairTask | t));
    else
      for (int t = 0; t < P.nblocks; ++t)
        tiles.push_back(make_int2((int)i, P.nfirst + t));
  }
  if (order == 0) return spread(tiles, part);
  // order 1: one queue per XCD (its band of tiles and every 8th particle
  // task), read in turn slot by slot
  const size_t M = tiles.size(), band = (M + 7) / 8;
  std::vector<BatchTask> q[8];
  for (int x = 0; x < 8; ++x) {
    std::vector<BatchTask> bt, bp;
    for (size_t k = x * band; k < std::min(M, (x + 1) * band); ++k)
      bt.push_back(tiles[k]);
    for (size_t k = x; k < part.size(); k += 8) bp.push_back(part[k]);
    q[x] = spread(bt, bp);
  }
  size_t L = 0;
  for (int x = 0; x < 8; ++x) L = std::max(L, q[x].size());
  std::vector<BatchTask> out(8 * L, make_int2(-1, 0));
  for (int x = 0; x < 8; ++x)
    for (size_t j = 0; j < q[x].size(); ++j) out[8 * j + x] = q[x][j];
  return out;
}

static vlb_status upload_tasks(vlb_batch* b) {
  std::vector<BatchTask> t = build_tasks(b, b->tune);
  if (t.size() > b->tasks_cap) {
    if (b->dtasks) (void)hipFree(b->dtasks);
    b->dtasks = nullptr;
    b->tasks_cap = 0;
    BHIP(b, hipMalloc((void**)&b->dtasks, t.size() * sizeof(BatchTask)));
    b->tasks_cap = t.size();
  }
  BHIP(b, hipMemcpyAsync(b->dtasks, t.data(), t.size() * sizeof(BatchTask),
                         hipMemcpyHostToDevice, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  b->ntasks = (int)t.size();
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  return VLB_OK;
}

// The device copy of the domain table holds every buffer as its byte
// offset from the arena (the table's own address; see BatchCase).
template <class T>
static T* arena_offset(T* p, const char* arena) {
  return p ? (T*)(intptr_t)((const char*)p - arena) : nullptr;
}

static StepBufs to_offsets(StepBufs b, const char* a) {
  b.fi = arena_offset(b.fi, a); b.fo = arena_offset(b.fo, a);
  b.gi = arena_offset(b.gi, a); b.go = arena_offset(b.go, a);
  b.hin = arena_offset(b.hin, a); b.hout = arena_offset(b.hout, a);
  for (PState* s : {&b.cur, &b.nxt}) {
    double** f[] = {&s->X, &s->Y, &s->th, &s->Ux, &s->Uy, &s->Om, &s->Uxp,
                    &s->Uyp, &s->Omp, &s->Fx, &s->Fy, &s->Tz};
    for (double** q : f) *q = arena_offset(*q, a);
    s->nslot = arena_offset(s->nslot, a);
  }
  b.pc.R = arena_offset(b.pc.R, a);
  b.pc.rhos = arena_offset(b.pc.rhos, a);
  b.pc.Tinit = arena_offset(b.pc.Tinit, a);
  b.pc.Rb = arena_offset(b.pc.Rb, a);
  b.pc.fixed = arena_offset(b.pc.fixed, a);
  b.L.cnt = arena_offset(b.L.cnt, a);
  b.L.ent = arena_offset(b.L.ent, a);
  b.L.clr = arena_offset(b.L.clr, a);
  b.partial_in = arena_offset(b.partial_in, a);
  b.partial_out = arena_offset(b.partial_out, a);
  b.macro = arena_offset(b.macro, a);
  b.flags = arena_offset(b.flags, a);
  return b;
}

static int grid_of(const vlb_batch* b) {
  const int g = b->tune.grid_blocks > 0 ? b->tune.grid_blocks : b->ntasks;
  return std::max(1, std::min(g, b->ntasks));
}

// The occupancy of the kernel variant: the tuning's, else 4 waves per
// SIMD for FP64 (128 registers, no spill) and 5 for the narrower forms.
static int waves_of(const vlb_batch* b) {
  if (b->tune.waves) return b->tune.waves;
  return b->prec == VLB_FP64 ? 4 : 5;
}

static hipError_t launch_one(vlb_batch* b, bool out) {
  BatchLaunch a;
  a.cases = b->dcases;
  a.tasks = b->dtasks;
  a.arena = (char*)b->dcases;
  a.ntasks = b->ntasks;
  a.grid = grid_of(b);
  a.parity = b->parity;
  a.have = b->have;
  a.waves = waves_of(b);
  a.pair = b->tune.pair_min_tiles >= 0;
  hipError_t e = launch_batch_step(b->prec, out, a, b->stream);
  b->parity ^= 1;
  b->have = 1;
  return e;
}

static vlb_status ensure_graph(vlb_batch* b) {
  if (b->graph) return VLB_OK;
  hipGraph_t g = nullptr;
  const int parity = b->parity, have = b->have;
  b->parity = 0;
  b->have = 1;
  BHIP(b, hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = launch_one(b, false);
  if (e == hipSuccess) e = launch_one(b, false);
  hipError_t e2 = hipStreamEndCapture(b->stream, &g);
  b->parity = parity;
  b->have = have;
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return bfail(b, VLB_EHIP, std::string("graph capture: ") +
                                  hipGetErrorString(e != hipSuccess ? e : e2));
  }
  e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    b->graph = nullptr;
    return bfail(b, VLB_EHIP, std::string("graph instantiate: ") +
                                  hipGetErrorString(e));
  }
  return VLB_OK;
}

static vlb_status batch_flags(vlb_batch* b) {
  const int n = (int)b->cases.size();
  BHIP(b, launch_gather_flags(b->dcases, (char*)b->dcases, n, b->dflags,
                              b->stream));
  BHIP(b, hipMemcpyAsync(b->hflags, b->dflags, n * sizeof(int),
                         hipMemcpyDeviceToHost, b->stream));
  BHIP(b, hipStreamSynchronize(b->stream));
  for (int i = 0; i < n; ++i) {
    const int f = b->hflags[i];
    if (!f) continue;
    char m[160];
    snprintf(m, sizeof m, "domain %d: %s", i,
             (f & kFlagUnstable) ? "a cell reached rho <= 0 or a non-finite value"
             : (f & kFlagListFull) ? "a per-block particle list overflowed"
                                   : "more than kmax particles touch one cell");
    return bfail(b, (f & kFlagUnstable) ? VLB_EUNSTABLE : VLB_EOVERLAP, m);
  }
  return VLB_OK;
}

// Advance n steps: the first after an init and any step needed to reach
// parity 0 run as single launches, then pairs of steps replay the graph,
// and the last step (which also stores the macroscopic fields) is a single
// launch again.
static vlb_status run_steps(vlb_batch* b, int64_t n) {
  int64_t left = n;
  while (left > 1 && (b->have == 0 || b->parity == 1 || !b->tune.use_graph)) {
    BHIP(b, launch_one(b, false));
    --left;
  }
  if (left > 1) {
    vlb_status st = ensure_graph(b);
    if (st != VLB_OK) return st;
    for (; left > 2; left -= 2) BHIP(b, hipGraphLaunch(b->graph, b->stream));
  }
  while (left > 1) {
    BHIP(b, launch_one(b, false));
    --left;
  }
  if (left == 1) BHIP(b, launch_one(b, true));
  for (vlb_ctx* c : b->cases) context_advance(c, n);
  b->step += n;
  return VLB_OK;
}

extern "C" {

vlb_status vlb_batch_create(int32_t ncases, const vlb_domain_desc* descs,
                            const int32_t* nparticles,
                            const vlb_particle_desc* particles,
                            vlb_batch** out) {
  if (!out || ncases < 1 || !descs || !nparticles)
    return bfail(nullptr, VLB_EINVAL, "bad argument");
  *out = nullptr;
  for (int i = 0; i < ncases; ++i) {
    if (descs[i].precision != descs[0].precision)
      return bfail(nullptr, VLB_EINVAL, "all domains of a batch share one precision");
    if (nparticles[i] < 0 || nparticles[i] > kScanMax)
      return bfail(nullptr, VLB_EINVAL, "a batch domain holds 0..64 particles");
    if (nparticles[i] > 0 && !particles)
      return bfail(nullptr, VLB_EINVAL, "particles is NULL");
  }
  vlb_batch* b = new (std::nothrow) vlb_batch();
  if (!b) return bfail(nullptr, VLB_ENOMEM, "host allocation failed");
  b->prec = descs[0].precision;
  (void)hipGetDevice(&b->device);
  if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount,
                            b->device) != hipSuccess || b->cus < 1)
    b->cus = 256;
  b->tune.grid_blocks = 4 * b->cus;   // one wave of resident blocks
  b->tune.order = 1;
  b->tune.use_graph = 1;
  b->tune.pair_min_tiles = -1;
  b->tune.waves = 0;
  b->tune.us_per_step = 0.0;
  auto give_up = [&](vlb_status s, const std::string& m) {
    vlb_batch_destroy(b);
    return bfail(nullptr, s, m);
  };
  if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess)
    return give_up(VLB_EHIP, "stream creation failed");
  int64_t off = 0;
  for (int i = 0; i < ncases; ++i) {
    vlb_ctx* c = nullptr;
    vlb_status st = vlb_create(&descs[i], b->stream, &c);
    if (st != VLB_OK)
      return give_up(st, "domain " + std::to_string(i) + ": " +
                             vlb_last_error(nullptr));
    b->cases.push_back(c);
    st = vlb_set_particles(c, nparticles[i], particles ? particles + off : nullptr);
    if (st != VLB_OK)
      return give_up(st, "domain " + std::to_string(i) + ": " + c->err);
    if (nparticles[i] > 0 && !c->P.scan)
      return give_up(VLB_EINVAL, "domain " + std::to_string(i) +
                                     ": too large for the batch form");
    if (c->P.ellipses)   // the batch kernel carries the disk geometry only
      return give_up(VLB_EINVAL, "domain " + std::to_string(i) +
                                     ": batches hold disks only");
    off += nparticles[i];
    b->cells += c->P.N;
  }
  if (hipMalloc((void**)&b->dcases, ncases * sizeof(BatchCase)) != hipSuccess ||
      hipMalloc((void**)&b->dflags, ncases * sizeof(int)) != hipSuccess ||
      hipHostMalloc((void**)&b->hflags, ncases * sizeof(int),
                    hipHostMallocDefault) != hipSuccess)
    return give_up(VLB_ENOMEM, "device allocation failed");
  // the constants and both parities' buffers of every domain
  std::vector<BatchCase> hc(ncases);
  for (int i = 0; i < ncases; ++i) {
    vlb_ctx* c = b->cases[i];
    hc[i].P = c->P;
    hc[i].Hd = make_hot<double>(c->P);
    hc[i].Hf = make_hot<float>(c->P);
    for (int p = 0; p < 2; ++p) {
      c->cur = c->pcur = c->pp = p;
      StepBufs sb = context_step_bufs(c);
      // the tile counts go round three buffers, which a two-step table
      // cannot follow: batch tasks test their tiles directly
      sb.tcount = nullptr;
      sb.tcount_next = nullptr;
      sb.tcount_clear = nullptr;
      hc[i].B[p] = to_offsets(sb, (const char*)b->dcases);
    }
    c->cur = c->pcur = c->pp = 0;
  }
  if (hipMemcpy(b->dcases, hc.data(), ncases * sizeof(BatchCase),
                hipMemcpyHostToDevice) != hipSuccess)
    return give_up(VLB_EHIP, "copy of the domain table failed");
  if (upload_tasks(b) != VLB_OK) return give_up(VLB_EHIP, b->err);
  *out = b;
  return VLB_OK;
}

vlb_status vlb_batch_init(vlb_batch* b) {
  if (!b) return VLB_EINVAL;
  b->initialized = false;
  for (size_t i = 0; i < b->cases.size(); ++i) {
    vlb_status st = vlb_init(b->cases[i]);
    if (st != VLB_OK)
      return bfail(b, st, "domain " + std::to_string(i) + ": " +
                              b->cases[i]->err);
  }
  b->parity = 0;
  b->have = 0;
  b->step = 0;
  b->initialized = true;
  return VLB_OK;
}

vlb_status vlb_batch_step(vlb_batch* b, int64_t nsteps) {
  if (!b) return VLB_EINVAL;
  if (nsteps < 0) return bfail(b, VLB_EINVAL, "nsteps must be >= 0");
  if (!b->initialized)
    return bfail(b, VLB_ESTATE, "vlb_batch_init has not succeeded");
  vlb_status st = run_steps(b, nsteps);
  if (st == VLB_OK) st = batch_flags(b);
  if (st != VLB_OK) {
    b->initialized = false;
    for (vlb_ctx* c : b->cases) c->initialized = false;
  }
  return st;
}

vlb_status vlb_batch_set_tuning(vlb_batch* b, const vlb_batch_tuning* t) {
  if (!b || !t) return VLB_EINVAL;
  if (t->grid_blocks < 0 || (t->grid_blocks % 8) != 0 || t->order < 0 ||
      t->order > 1 || t->pair_min_tiles < -1 ||
      (t->waves != 0 && t->waves != 4 &&
       (t->waves != 5 || b->prec == VLB_FP64)))
    return bfail(b, VLB_EINVAL,
                 "grid_blocks must be a multiple of 8 (0: one per task), "
                 "order 0 or 1, pair_min_tiles >= -1, waves 0 or 4 (or 5 "
                 "for the 32- and 16-bit forms)");
  b->tune.grid_blocks = t->grid_blocks;
  b->tune.use_graph = t->use_graph ? 1 : 0;
  b->tune.waves = t->waves;
  if (t->order != b->tune.order ||
      t->pair_min_tiles != b->tune.pair_min_tiles) {
    b->tune.order = t->order;
    b->tune.pair_min_tiles = t->pair_min_tiles;
    return upload_tasks(b);
  }
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  return VLB_OK;
}

vlb_status vlb_batch_get_tuning(const vlb_batch* b, vlb_batch_tuning* t) {
  if (!b || !t) return VLB_EINVAL;
  *t = b->tune;
  return VLB_OK;
}

vlb_status vlb_batch_autotune(vlb_batch* b, int32_t steps,
                              vlb_batch_tuning* chosen) {
  if (!b || steps < 1) return VLB_EINVAL;
  if (!b->initialized)
    return bfail(b, VLB_ESTATE, "vlb_batch_init has not succeeded");
  if (b->step != 0)
    return bfail(b, VLB_ESTATE, "autotune a freshly initialised batch");
  const int grids[] = {4 * b->cus, 8 * b->cus, 16 * b->cus, 0};
  // pairing thresholds: none, the larger half of the domains, all
  std::vector<int> counts;
  for (const vlb_ctx* c : b->cases) counts.push_back(c->P.nblocks);
  std::nth_element(counts.begin(), counts.begin() + counts.size() / 2,
                   counts.end());
  const int pairs[] = {-1, counts[counts.size() / 2], 0};
  const int waves[] = {4, 5};
  const int nwaves = b->prec == VLB_FP64 ? 1 : 2;
  hipEvent_t e0, e1;
  BHIP(b, hipEventCreate(&e0));
  BHIP(b, hipEventCreate(&e1));
  vlb_batch_tuning best = b->tune;
  double best_us = 1e300;
  vlb_status st = VLB_OK;
  for (int pi = 0; pi < 3 && st == VLB_OK; ++pi)
  for (int order = 0; order < 2 && st == VLB_OK; ++order)
  for (int wi = 0; wi < nwaves && st == VLB_OK; ++wi)
  for (int gi = 0; gi < 4 && st == VLB_OK; ++gi) {
    vlb_batch_tuning t;
    t.grid_blocks = grids[gi];
    t.order = order;
    t.use_graph = 0;
    t.pair_min_tiles = pairs[pi];
    t.waves = waves[wi];
    t.us_per_step = 0.0;
    st = vlb_batch_set_tuning(b, &t);
    if (st != VLB_OK) break;
    hipError_t e = launch_one(b, false);              // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
    for (int k = 0; k < steps && e == hipSuccess; ++k) e = launch_one(b, false);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e != hipSuccess) {
      st = bfail(b, VLB_EHIP, std::string("autotune: ") + hipGetErrorString(e));
      break;
    }
    const double us = 1e3 * ms / steps;
    if (us < best_us) {
      best_us = us;
      best = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != VLB_OK) return st;
  best.use_graph = 1;
  best.us_per_step = best_us;
  st = vlb_batch_set_tuning(b, &best);
  if (st != VLB_OK) return st;
  b->tune.us_per_step = best_us;
  // the candidates advanced the domains: start again from the initial state
  st = vlb_batch_init(b);
  if (st != VLB_OK) return st;
  if (chosen) *chosen = b->tune;
  return VLB_OK;
}

vlb_status vlb_batch_read_field(vlb_batch* b, int32_t i, int32_t field,
                                double* dst, int32_t dst_is_device) {
  if (!b) return VLB_EINVAL;
  if (i < 0 || i >= (int32_t)b->cases.size())
    return bfail(b, VLB_EINVAL, "domain index out of range");
  vlb_status st = vlb_read_field(b->cases[i], field, dst, dst_is_device);
  if (st != VLB_OK) return bfail(b, st, b->cases[i]->err);
  return VLB_OK;
}

vlb_status vlb_batch_read_particles(vlb_batch* b, int32_t i, int32_t n,
                                    vlb_particle_state* dst) {
  if (!b) return VLB_EINVAL;
  if (i < 0 || i >= (int32_t)b->cases.size())
    return bfail(b, VLB_EINVAL, "domain index out of range");
  vlb_status st = vlb_read_particles(b->cases[i], n, dst);
  if (st != VLB_OK) return bfail(b, st, b->cases[i]->err);
  return VLB_OK;
}

int32_t vlb_batch_size(const vlb_batch* b) {
  return b ? (int32_t)b->cases.size() : 0;
}

int64_t vlb_batch_cells(const vlb_batch* b) { return b ? b->cells : 0; }

int64_t vlb_batch_step_count(const vlb_batch* b) { return b ? b->step : -1; }

size_t vlb_batch_device_bytes(const vlb_batch* b) {
  if (!b) return 0;
  size_t s = 0;
  for (const vlb_ctx* c : b->cases) s += vlb_device_bytes(c);
  return s + b->cases.size() * (sizeof(BatchCase) + sizeof(int)) +
         b->tasks_cap * sizeof(BatchTask);
}

const char* vlb_batch_last_error(const vlb_batch* b) {
  return b ? b->err.c_str() : g_batch_create_error.c_str();
}

void vlb_batch_destroy(vlb_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  for (vlb_ctx* c : b->cases) vlb_destroy(c);
  if (b->dcases) (void)hipFree(b->dcases);
  if (b->dtasks) (void)hipFree(b->dtasks);
  if (b->dflags) (void)hipFree(b->dflags);
  if (b->hflags) (void)hipHostFree(b->hflags);
  if (b->stream) (void)hipStreamDestroy(b->stream);
  delete b;
}

}  // extern "C"
