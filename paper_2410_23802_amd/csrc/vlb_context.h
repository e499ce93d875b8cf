// vlb_context.h -- host-side state of one domain (private to the library).
#pragma once

#include <string>
#include <vector>

#include "vlb_internal.h"

// One domain: its descriptor, device memory and step bookkeeping.
struct vlb_ctx {
  vlb_domain_desc d;
  hipStream_t stream = nullptr;
  int device = 0;
  vlb::Params P;
  int prec = 0;
  size_t plane = 0, pop_elem = 0, h_elem = 0;
  void* f[2] = {nullptr, nullptr};
  void* g[2] = {nullptr, nullptr};
  void* h[2] = {nullptr, nullptr};   // [df_s/dt] carrier, alternating
  int cur = 0;                       // f[cur], g[cur], h[cur]: step n
  double* macro = nullptr;
  // block lists, three in turn: the current ones, those a binning pass
  // fills, and the stale ones it clears
  int* blk_cnt[3] = {nullptr, nullptr, nullptr};
  int2* blk_ent[3] = {nullptr, nullptr, nullptr};
  // list form: centre bins of the particles (the repulsion's search), in
  // the same turn as the block lists
  int* bin_cnt[3] = {nullptr, nullptr, nullptr};
  int* bin_ent[3] = {nullptr, nullptr, nullptr};
  int lpar = 0;                          // [lpar]: the current lists
  // scan form: particles reaching each tile, three in turn (the next
  // step's, the one after, a stale one being cleared)
  int* tcount[3] = {nullptr, nullptr, nullptr};
  int tpar = 0;                          // [tpar]: the next step's counts
  // particles
  int np = 0;
  int maxb = 0;
  double* pmem[2] = {nullptr, nullptr};
  int* pslot[2] = {nullptr, nullptr};
  vlb::PState ps[2];
  int pcur = 0;
  double* pconst = nullptr;
  int* pfixed = nullptr;
  vlb::PConst pc;
  double* partial[2] = {nullptr, nullptr};  // step n / step n+1, alternating
  int pp = 0;                                // partial[pp]: the latest pass
  double* thermal4 = nullptr;
  std::vector<vlb_particle_desc> parts;
  // status
  int* flags = nullptr;
  int* flags_host = nullptr;
  int have_partials = 0;
  int64_t step = 0;
  bool initialized = false;
  size_t dev_bytes = 0;
  // timing
  bool timing = false;
  std::vector<hipEvent_t> ev;
  size_t ev_used = 0;
  std::string err;
};


namespace vlb {

// The buffers the next step of c reads and writes.
StepBufs context_step_bufs(vlb_ctx* c);

// Advance c's bookkeeping (buffer parities, step count) by n steps taken.
void context_advance(vlb_ctx* c, int64_t n);

}  // namespace vlb
