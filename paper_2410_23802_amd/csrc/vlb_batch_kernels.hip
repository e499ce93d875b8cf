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
// domain's particle-tile tasks first, then its tiles; its order (chosen by
// the autotuner) decides which XCD streams which tiles.  Every task is one
// call of step_task, exactly as in k_step, so a domain's results do not
// depend on the batch around it or on the table order.  Occupancy targets
// as for k_step.
template <int PREC, bool OUT>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(PREC == VLB_FP64 ? 4 : 5))) void k_batch_step(
    const BatchCase* __restrict__ cases, const BatchTask* __restrict__ tasks,
    char* __restrict__ arena, int ntasks, int parity, int have) {
  typedef typename Prec<PREC>::C C;
  __shared__ TileShared<C> sh;
  for (int w = blockIdx.x; w < ntasks; w += gridDim.x) {
    const BatchTask tk = tasks[w];                      // uniform in the block
    if (tk.x >= 0) {
      const BatchCase& bc = cases[tk.x];
      const StepBufs B = rebase_bufs(arena, bc.B[parity]);
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
        step_task<PREC, OUT, true>(bc.P, hot_of<C>(bc), B, have, tile, ptile,
                                   sh);
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

template <int PREC>
static hipError_t batch_p(bool out, const BatchCase* cases,
                          const BatchTask* tasks, char* arena, int ntasks,
                          int grid, int parity, int have, hipStream_t s) {
  if (out)
    hipLaunchKernelGGL((k_batch_step<PREC, true>), dim3(grid), dim3(kBlock),
                       0, s, cases, tasks, arena, ntasks, parity, have);
  else
    hipLaunchKernelGGL((k_batch_step<PREC, false>), dim3(grid), dim3(kBlock),
                       0, s, cases, tasks, arena, ntasks, parity, have);
  return hipGetLastError();
}

hipError_t launch_batch_step(int prec, bool out, const BatchCase* cases,
                             const BatchTask* tasks, char* arena, int ntasks,
                             int grid, int parity, int have, hipStream_t s) {
  if (ntasks <= 0 || grid <= 0) return hipSuccess;
  switch (prec) {
    case VLB_FP64: return batch_p<VLB_FP64>(out, cases, tasks, arena, ntasks, grid, parity, have, s);
    case VLB_FP32: return batch_p<VLB_FP32>(out, cases, tasks, arena, ntasks, grid, parity, have, s);
    case VLB_FP16_SHIFT: return batch_p<VLB_FP16_SHIFT>(out, cases, tasks, arena, ntasks, grid, parity, have, s);
    case VLB_BF16_SHIFT: return batch_p<VLB_BF16_SHIFT>(out, cases, tasks, arena, ntasks, grid, parity, have, s);
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
