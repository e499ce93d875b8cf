// vlb_batch_kernels.hip -- the batch step kernel (many domains, one
// launch per step) and its launchers.  Built in a translation unit of its
// own: its persistent loop needs machine loop-invariant code motion off
// (see build.py), which the single-domain kernels are better without.
#include "vlb_device.h"

namespace vlb {

// -------------------------------------------------------------------------
// Batches: many independent domains advance in one launch per step.

template <class C>
__device__ __forceinline__ const Hot<C>& hot_of(const BatchCase& b);
template <>
__device__ __forceinline__ const Hot<double>& hot_of<double>(
    const BatchCase& b) {
  return b.Hd;
}
template <>
__device__ __forceinline__ const Hot<float>& hot_of<float>(
    const BatchCase& b) {
  return b.Hf;
}

// The domain table holds each buffer of a domain as its byte offset from
// the `arena` kernel argument (see BatchCase).  A pointer formed as arena +
// offset derives from a kernel argument, so the compiler knows it addresses
// global memory (and emits GLOBAL rather than FLAT accesses), and since
// both `cases` and `arena` are restrict, no store through such a pointer
// can clobber the table, whose loads can then be scalar.
template <class T>
__device__ __forceinline__ T* rebase(char* arena, T* off) {
  return (T*)(arena + (intptr_t)off);
}

__device__ __forceinline__ PState rebase_state(char* a, PState s) {
  s.X = rebase(a, s.X); s.Y = rebase(a, s.Y); s.th = rebase(a, s.th);
  s.Ux = rebase(a, s.Ux); s.Uy = rebase(a, s.Uy); s.Om = rebase(a, s.Om);
  s.Uxp = rebase(a, s.Uxp); s.Uyp = rebase(a, s.Uyp);
  s.Omp = rebase(a, s.Omp); s.Fx = rebase(a, s.Fx); s.Fy = rebase(a, s.Fy);
  s.Tz = rebase(a, s.Tz); s.nslot = rebase(a, s.nslot);
  return s;
}

// Every pointer of the two structures is rebased; a field added to either
// must be added here too (the sizes below catch one that is not).
static_assert(sizeof(PConst) == 5 * sizeof(void*), "rebase every PConst field");
static_assert(sizeof(PState) == 13 * sizeof(void*), "rebase every PState field");

__device__ __forceinline__ PConst rebase_const(char* a, PConst c) {
  c.R = rebase(a, c.R); c.rhos = rebase(a, c.rhos);
  c.Tinit = rebase(a, c.Tinit); c.fixed = rebase(a, c.fixed);
  c.Rb = rebase(a, c.Rb);
  return c;
}

__device__ __forceinline__ StepBufs rebase_bufs(char* a, const StepBufs& b) {
  StepBufs g = b;
  g.fi = rebase(a, b.fi); g.fo = rebase(a, b.fo);
  g.gi = rebase(a, b.gi); g.go = rebase(a, b.go);
  g.hin = rebase(a, b.hin); g.hout = rebase(a, b.hout);
  g.cur = rebase_state(a, b.cur);
  g.nxt = rebase_state(a, b.nxt);
  g.pc = rebase_const(a, b.pc);
  g.L.cnt = rebase(a, b.L.cnt); g.L.ent = rebase(a, b.L.ent);
  g.L.clr = rebase(a, b.L.clr);
  g.partial_in = rebase(a, b.partial_in);
  g.partial_out = rebase(a, b.partial_out);
  g.macro = rebase(a, b.macro);
  g.flags = rebase(a, b.flags);
  return g;
}

// One step of every domain of a batch (all in the scan form or without
// particles).  A fixed set of persistent blocks walks the task table: block
// b takes tasks b, b + grid, b + 2 grid, ...  The table lists every
// domain's particle-tile tasks, then its tiles, one or two per task (two
// adjacent tiles streamed by one block, each lane loading its cell in both
// before it computes either, as pair_task describes); the autotuner chooses
// which domains stream in pairs, the table order (which XCD streams which
// tiles) and the occupancy WAVES (waves per SIMD the registers are held to).
// PAIR: the table holds pair tasks -- a kernel of its own, since the pair
// path's two cells per lane raise the register peak of the whole kernel
// (FP64: from 128 registers without spills to 54 spilled).  Every tile is
// updated by the same update_cell arithmetic, alone or in a pair, so a
// domain's results do not depend on the batch around it or on the tuning.
template <int PREC, bool OUT, int WAVES, bool PAIR>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(WAVES))) void k_batch_step(
    const BatchCase* __restrict__ cases, const BatchTask* __restrict__ tasks,
    char* __restrict__ arena, int ntasks, int parity, int have) {
  typedef typename Prec<PREC>::C C;
  __shared__ TileShared<C> sh;
  for (int w = blockIdx.x; w < ntasks; w += gridDim.x) {
    const BatchTask tk = tasks[w];                      // uniform in the block
    if (tk.x >= 0) {
      const BatchCase& bc = cases[tk.x];
      const StepBufs B = rebase_bufs(arena, bc.B[parity]);
      if (PAIR && (tk.y & kPairTask)) {
        const int tA = tk.y & ~kPairTask;
        pair_task<PREC, OUT, true>(bc.P, hot_of<C>(bc), B, tA, tA + 1);
      } else {
        int tile;
        bool ptile;
        if (tk.y < bc.P.nfirst) {
          tile = scan_task_tile(bc.P, B.cur, B.pc, tk.y);
          ptile = true;
        } else {
          tile = tk.y - bc.P.nfirst;
          ptile = false;
        }
        if (tile >= 0)
          step_task<PREC, OUT, true>(bc.P, hot_of<C>(bc), B, have, tile,
                                     ptile, sh);
      }
    }
    __syncthreads();   // the LDS of this task is free for the next
  }
}

__global__ void k_gather_flags(const BatchCase* __restrict__ cases,
                               char* __restrict__ arena, int n,
                               int* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = *rebase(arena, cases[i].B[0].flags);
}


// -------------------------------------------------------------------------
// Launchers

template <int PREC, int WAVES, bool PAIR>
static hipError_t batch_w(bool out, const BatchLaunch& a, hipStream_t s) {
  if (out)
    hipLaunchKernelGGL((k_batch_step<PREC, true, WAVES, PAIR>), dim3(a.grid),
                       dim3(kBlock), 0, s, a.cases, a.tasks, a.arena,
                       a.ntasks, a.parity, a.have);
  else
    hipLaunchKernelGGL((k_batch_step<PREC, false, WAVES, PAIR>), dim3(a.grid),
                       dim3(kBlock), 0, s, a.cases, a.tasks, a.arena,
                       a.ntasks, a.parity, a.have);
  return hipGetLastError();
}

// FP64 only at 4 waves (128 registers): at 5 it spills heavily.
template <int PREC>
static hipError_t batch_p(bool out, const BatchLaunch& a, hipStream_t s) {
  if (a.waves == 4)
    return a.pair ? batch_w<PREC, 4, true>(out, a, s)
                  : batch_w<PREC, 4, false>(out, a, s);
  if constexpr (PREC != VLB_FP64)
    if (a.waves == 5)
      return a.pair ? batch_w<PREC, 5, true>(out, a, s)
                    : batch_w<PREC, 5, false>(out, a, s);
  return hipErrorInvalidValue;
}

hipError_t launch_batch_step(int prec, bool out, const BatchLaunch& a,
                             hipStream_t s) {
  if (a.ntasks <= 0 || a.grid <= 0) return hipSuccess;
  switch (prec) {
    case VLB_FP64: return batch_p<VLB_FP64>(out, a, s);
    case VLB_FP32: return batch_p<VLB_FP32>(out, a, s);
    case VLB_FP16_SHIFT: return batch_p<VLB_FP16_SHIFT>(out, a, s);
    case VLB_BF16_SHIFT: return batch_p<VLB_BF16_SHIFT>(out, a, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_gather_flags(const BatchCase* cases, char* arena, int n,
                               int* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_flags, dim3(blocks_for(n, 256)), dim3(256), 0,
                     s, cases, arena, n, out);
  return hipGetLastError();
}

}  // namespace vlb
