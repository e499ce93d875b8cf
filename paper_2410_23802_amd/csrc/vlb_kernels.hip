// vlb_kernels.hip -- gfx950 kernels of one domain: the step kernel
// (k_step), the particle pass of the list form, the initial state and the
// read-outs, with their launchers.  The device code they share is in
// vlb_device.h.
#include "vlb_device.h"

namespace vlb {

// The step kernel of one domain, one launch per step: block roles as
// step_task (vlb_device.h) describes.  FP64 is held to 128 VGPRs (4 waves
// per SIMD, the occupancy of the plain update).  The 32-bit forms are held to 5
// waves (96 VGPRs, no added spill): 4-7 % faster on the channel than the
// unconstrained 4 waves; at 6 the particle role spills and loses it again
// (and the LDS of a particle tile caps a CU at 7 blocks; on the dense
// cavity the 16-bit forms gain 3 % from 6 waves, but their spills add a
// quarter to the kernel's HBM writes).  PAIR (16-bit
// forms, where the host sets pair_tiles): the streaming blocks take two
// tiles each; a kernel of its own, so that the one-tile path keeps its code.
// NT: the populations and the carrier are stored non-temporally (list form,
// where the host sets nt_stores).
template <int PREC, bool OUT, bool SCAN, bool PAIR, bool ELL, bool NT>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(PREC == VLB_FP64 ? 4 : 5))) void k_step(
    const Params P, const Hot<typename Prec<PREC>::C> H, const StepBufs B,
    int have) {
  typedef typename Prec<PREC>::C C;
  __shared__ TileShared<C> sh;
  int tile;
  bool ptile;
  if (SCAN && (int)blockIdx.x < P.nfirst) {
    tile = scan_task_tile(P, B.cur, B.pc, blockIdx.x);  // uniform in the block
    if (tile < 0) return;
    ptile = true;
  } else if (PAIR) {
    // streaming block j: tiles k and k + 8 of the XCD-ordered sequence
    // (the same XCD's band), k = 16 (j / 8) + j mod 8; never in the list
    // form with particles
    const int j = blockIdx.x - P.nfirst;
    const int k = (j >> 3) * 16 + (j & 7);
    const int tA = stream_tile(P, k), tB = stream_tile(P, k + 8);
    if (tA >= P.nblocks) return;                         // then tB too
    pair_task<PREC, OUT, SCAN, SCAN && counted_tiles(PREC, PAIR)>(P, H, B,
                                                                  tA, tB);
    return;
  } else {
    tile = stream_tile(P, blockIdx.x - P.nfirst);
    if (tile >= P.nblocks) return;
    ptile = false;
  }
  // list form: the tile's count decides its role; entry t of its list is
  // read together with it, before the count is known (kListEntryAhead)
  int lcnt = 0;
  int2 lent = make_int2(0, 0);
  if (!SCAN && P.np > 0) {
    if (kListEntryAhead<PREC> && threadIdx.x < kListCap)
      lent = B.L.ent[(size_t)tile * kListCap + threadIdx.x];
    lcnt = B.L.cnt[tile];                                // uniform
    ptile = lcnt != 0;
  }
  step_task<PREC, OUT, SCAN, SCAN && counted_tiles(PREC, PAIR), ELL, NT,
            !SCAN && !ELL>(P, H, B, have, tile, ptile, sh, lcnt, lent);
}

// -------------------------------------------------------------------------
// Initial state: equilibria of the mixed fluid/particle state per cell.

template <int PREC, bool SCAN>
__global__ __launch_bounds__(kBlock) void k_init(
    const Params P, typename Prec<PREC>::S* __restrict__ fo,
    typename Prec<PREC>::S* __restrict__ go,
    typename Prec<PREC>::H* __restrict__ hcar, size_t plane, PState ps,
    PConst pc, Lists L, double* __restrict__ macro, int* flags) {
  typedef Prec<PREC> T;
  typedef typename T::C C;
  __shared__ BlockParticles bp;
  __shared__ int tmp[kListCap];
  gather_particles<SCAN>(bp, tmp, P, blockIdx.x, ps, ps, pc, L, nullptr, 0,
                         false, flags);
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= P.N) return;
  const int y = c / P.nx, x = c - y * P.nx;
  double S0 = 0, Sx = 0, Sy = 0, Se = 0;
  int nin = 0;
  for (int s = 0; s < bp.cnt; ++s) {
    SlotGeom sg;
    if (slot_geometry(bp, s, P, x, y, sg)) {
      ++nin;
      S0 += sg.fs;
      Sx += sg.fs * sg.usx;
      Sy += sg.fs * sg.usy;
      Se += sg.fs * P.cvs * bp.Tp[s];
    }
  }
  if (nin > P.kmax) atomicOr(flags, kFlagOverlap);
  if (S0 > 1.0) {
    const double inv = 1.0 / S0;
    Sx *= inv;
    Sy *= inv;
    Se *= inv;
    S0 = 1.0;
  }
  const double fs = S0;
  const double ux = (1.0 - fs) * P.init_ux + Sx;
  const double uy = (1.0 - fs) * P.init_uy + Sy;
  const double eps = (1.0 - fs) * P.cvf * P.init_T + Se;
  const double cv = P.cvf + P.dcv * fs;
  const double Tt = eps / cv;
  // situation II of Sec. 3.2: the hydrostatic rho_0 + 3 rho_f g.(x - x_m)
  // of the constant force density rho_f g (p = rho / 3), x_m the centre
  const double rho =
      P.fluid_gravity
          ? P.init_rho + 3.0 * P.rho_f *
                             (P.grav_x * ((x + 0.5) - 0.5 * P.nx) +
                              P.grav_y * ((y + 0.5) - 0.5 * P.ny))
          : P.init_rho;
  // f^eq = w_i rho [1 + 3 e.u + 9/2 (e.u)^2 - 3/2 u^2] (= M^{-1} m^eq);
  // g^eq_i = w_i c_ref T (i >= 1), g^eq_0 = eps - 5/9 c_ref T (= M^{-1} n^eq)
  const double w[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                       1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
  const int ex[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  const int ey[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  const double u2 = ux * ux + uy * uy;
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const double eu = ex[q] * ux + ey[q] * uy;
    const double feq = w[q] * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * u2);
    const double geq = q == 0 ? eps - (5.0 / 9.0) * P.cref * Tt : w[q] * P.cref * Tt;
    T::st(fo, (size_t)q * plane + c, (C)(feq - P.fshift[q]));
    T::st(go, (size_t)q * plane + c, (C)(geq - P.gshift[q]));
  }
  hcar[c] = (typename T::H)(2.0 * fs);
  const size_t N = (size_t)P.N;
  macro[c] = rho;
  macro[N + c] = ux;
  macro[2 * N + c] = uy;
  macro[3 * N + c] = Tt;
  macro[4 * N + c] = fs;
  macro[5 * N + c] = 0.0;
}

// LDS of the particle pass's repulsion: the neighbour search (a bitmap of
// kWords x 64 particles per wave, kCand candidates gathered at a time) or
// the all-pairs staging (kStage particles at a time).
constexpr int kWords = 128;
constexpr int kCand = 128;
constexpr int kStage = 1024;
union PassShared {
  struct {
    unsigned long long marks[4][kWords];
    int cq[4][kCand];
    double X[4][kCand], Y[4][kCand], R[4][kCand];
  } nb;
  struct {
    double X[kStage], Y[kStage], R[kStage];
  } all;
};

// Orders a wave's LDS writes before its later LDS reads (other lanes'
// included); no block barrier.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sets in `marks` the bit of every particle listed in the tiles f0 ..
// f0 + n0 - 1 and f1 .. f1 + n1 - 1 (the previous positions' lists): four
// tiles at a time, whose counts and first eight entries are each loaded
// together.
__device__ __forceinline__ void mark_listed(const Lists& L, int f0, int n0,
                                            int f1, int n1,
                                            unsigned long long* marks) {
  const int nt = n0 + n1;
  for (int g = 0; g < nt; g += 4) {
    int tt[4], n[4], q[4][8];
    // the counts and the first eight entries, all issued before any is
    // used (entries past a count are stale and left out below)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = g + u;
      tt[u] = i < n0 ? f0 + i : f1 + (i - n0);
      n[u] = i < nt ? L.ocnt[tt[u]] : 0;
#pragma unroll
      for (int e = 0; e < 8; ++e)
        q[u][e] = i < nt ? L.oent[(size_t)tt[u] * kListCap + e].x : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      n[u] = min(n[u], kListCap);
#pragma unroll
      for (int e = 0; e < 8; ++e)
        if (e < n[u])
          atomicOr(&marks[q[u][e] >> 6], 1ull << (q[u][e] & 63));
      for (int e = 8; e < n[u]; ++e) {
        const int qq = L.oent[(size_t)tt[u] * kListCap + e].x;
        atomicOr(&marks[qq >> 6], 1ull << (qq & 63));
      }
    }
  }
}

// -------------------------------------------------------------------------
// Particle pass (list form, and the force read-out of both forms): one wave
// (64 lanes) per particle.  Modes: update (Newton-Euler step, then the block
// lists of the new band box), reduce only (store the momentum-exchange
// force of the last pass), bin only (block lists of the stored positions).

__global__ __launch_bounds__(256) void k_particles(
    const Params P, PState cur, PState next, PConst pc, Lists L,
    const double* __restrict__ partial, int have_partials, int mode,
    int* flags) {
  if (L.clr) {   // the previous step's block counts (the next fill's zeros)
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < P.nblocks;
         k += gridDim.x * blockDim.x)
      L.clr[k] = 0;
  }
  if (L.bclr) {  // and the previous step's centre-bin counts
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < P.nbins;
         k += gridDim.x * blockDim.x)
      L.bclr[k] = 0;
  }
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  const bool mine = p < P.np;          // uniform in the wave
  // the particle's stored state, loaded up front (the update needs it only
  // after the repulsion)
  POne own = {};
  if (mine) own = load_one(cur, pc, p);

  // The momentum-exchange sums.  List form: the slot count, then the first
  // 64 slots' partials, are loaded now and added after the repulsion, in
  // the order of reduce_partials (lane l: slots l, l + 64, ...; then
  // wave_sum).  Scan form (the force read-out only): reduce_partials.
  const bool sums = mine && mode != kModeBinOnly;
  double fx = 0.0, fy = 0.0, tz = 0.0;
  const double* src = partial + (size_t)(mine ? p : 0) * P.maxb * kRedVals;
  int ns = 0;
  double o0 = 0.0, o1 = 0.0, o2 = 0.0;
  if (sums && !P.scan && have_partials) {
    ns = cur.nslot[p];
    if (lane < ns) {
      o0 = src[lane * kRedVals + 0];
      o1 = src[lane * kRedVals + 1];
      o2 = src[lane * kRedVals + 2];
    }
  }

  // Repulsion of the update.  The candidates of particle p are the
  // particles whose centres lie in the 3 x 3 centre bins around p's, as the
  // previous pass filled them at the positions this pass starts from (a bin
  // is at least 2 rmax + zeta + 2 cells wide, so a particle within reach,
  // d < R_p + R_q + zeta, lies there); where one of those bins overflowed,
  // the particles listed in the tiles of the box of half-width R_p + rmax +
  // zeta around its centre (a particle within reach has its centre cell in
  // that box, and a particle's band box holds its centre cell).  The wave
  // marks them in a bitmap, gathers their positions into LDS, and each lane
  // then visits its own (q = lane, lane + 64, ...) in ascending order, as a
  // loop over all particles q = lane, lane + 64, ... would -- the others
  // are out of reach and add nothing, so the sums are those of that
  // all-pairs loop.
  // Without those lists (or with more particles than the bitmap holds)
  // the block stages all particles in LDS, kStage at a time.
  double cx = 0.0, cy = 0.0;
  if (mode == kModeUpdate && P.coll_range > 0.0) {   // uniform in the grid
    __shared__ PassShared psh;
    const double Xp = own.X, Yp = own.Y, Rp = own.R;
    if (L.ocnt && P.np <= 64 * kWords) {
      auto& marks = psh.nb.marks;
      auto& cq = psh.nb.cq;
      auto& cX = psh.nb.X;
      auto& cY = psh.nb.Y;
      auto& cR = psh.nb.R;
      const int w = threadIdx.x >> 6, nwords = (P.np + 63) >> 6;
      // each wave works on its own slice of the LDS (its bitmap and
      // candidates), so wave-level ordering is enough: no block barrier
      for (int k = lane; k < nwords; k += 64) marks[w][k] = 0ull;
      wave_lds_sync();
      // the candidates: the particles whose centres lie in the 3 x 3 centre
      // bins around p's (a bin is wider than any reach, so a particle within
      // reach lies there), one bin per lane; where a bin overflowed, those
      // listed in the tiles of the box below
      bool binned = false;
      if (mine && L.obcnt) {
        int bx, by, b = -1, n = 0, q[kBinCap];
        centre_bin(P, Xp, Yp, bx, by);
        if (lane < 9) {
          int ix = bx + lane % 3 - 1, iy = by + lane / 3 - 1;
          if (P.perx) ix = (ix + P.nbx) % P.nbx;
          if (P.pery) iy = (iy + P.nby) % P.nby;
          if (ix >= 0 && ix < P.nbx && iy >= 0 && iy < P.nby)
            b = iy * P.nbx + ix;
        }
        if (b >= 0) {
          // the count and every entry issued together (entries past the
          // count are stale and left out below)
          n = L.obcnt[b];
#pragma unroll
          for (int e = 0; e < kBinCap; ++e)
            q[e] = L.obent[(size_t)b * kBinCap + e];
        }
        binned = __ballot(n > kBinCap) == 0ull;   // uniform in the wave
        if (binned) {
#pragma unroll
          for (int e = 0; e < kBinCap; ++e)
            if (e < n) atomicOr(&marks[w][q[e] >> 6], 1ull << (q[e] & 63));
        }
      }
      if (mine && !binned) {
        int i0, i1, j0, j1;
        band_box(P, Xp, Yp, Rp + P.rmax + P.coll_range, i0, i1, j0, j1);
        ColSegs cs;
        if (i1 - i0 + 1 >= P.nx) {      // the box spans the periodic axis
          cs.n = 1; cs.lo[0] = 0; cs.hi[0] = P.nx - 1; cs.lo[1] = 0; cs.hi[1] = -1;
        } else {
          cs = col_segments(i0, i1, P.nx);
        }
        const int rows = min(j1 - j0 + 1, P.ny);
        for (int r = lane; r < rows; r += 64) {
          const int row = ((j0 + r) % P.ny + P.ny) % P.ny;
          int f0 = 0, n0 = 0, f1 = 0, n1 = 0;   // per segment: first tile, tiles
          if (cs.hi[0] >= cs.lo[0]) {
            f0 = (row * P.nx + cs.lo[0]) / kBlock;
            n0 = (row * P.nx + cs.hi[0]) / kBlock - f0 + 1;
          }
          if (cs.n > 1 && cs.hi[1] >= cs.lo[1]) {
            f1 = (row * P.nx + cs.lo[1]) / kBlock;
            n1 = (row * P.nx + cs.hi[1]) / kBlock - f1 + 1;
          }
          mark_listed(L, f0, n0, f1, n1, marks[w]);
        }
      }
      wave_lds_sync();
      if (mine) {
        // the marked particles but p, ascending: the m of them are
        // gathered kCand at a time.  Word k of the bitmap (k < nwords <=
        // 128) is held by lane k mod 64 (wd[k / 64]), with the count of
        // marked particles in the words before it (wb); lane l's own
        // particles (q mod 64 = l) are bit l of the words, visited over the
        // nonzero words in ascending order.
        unsigned long long wd[2];
        int wb[2];
        int m = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = lane + 64 * h;
          unsigned long long bits = k < nwords ? marks[w][k] : 0ull;
          if (k == (p >> 6)) bits &= ~(1ull << (p & 63));
          wd[h] = bits;
          int ctotal;
          wb[h] = m + wave_excl_scan<7>(__popcll(bits), lane, ctotal);
          m += ctotal;
        }
        const unsigned long long nz[2] = {__ballot(wd[0] != 0ull),
                                          __ballot(wd[1] != 0ull)};
        const unsigned long long below = (1ull << lane) - 1ull;
        for (int c0 = 0; c0 < m; c0 += kCand) {
          const int mc = min(kCand, m - c0);
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int k = lane + 64 * h;
            unsigned long long bits = wd[h];
            for (int pos = wb[h]; bits && pos < c0 + kCand;
                 bits &= bits - 1ull, ++pos)
              if (pos >= c0)
                cq[w][pos - c0] = k * 64 + __ffsll((long long)bits) - 1;
          }
          wave_lds_sync();
          for (int i = lane; i < mc; i += 64) {
            const int q = cq[w][i];
            cX[w][i] = cur.X[q];
            cY[w][i] = cur.Y[q];
            cR[w][i] = pc.R[q];
          }
          wave_lds_sync();
          // this chunk's candidates of lane l, ascending: q = 64 k + l over
          // the words k holding bit l
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            for (unsigned long long z = nz[h]; z; z &= z - 1ull) {
              const int kl = __ffsll((long long)z) - 1;   // uniform
              const unsigned lo = (unsigned)__builtin_amdgcn_readlane(
                  (int)(unsigned)wd[h], kl);
              const unsigned hi = (unsigned)__builtin_amdgcn_readlane(
                  (int)(unsigned)(wd[h] >> 32), kl);
              const unsigned long long wk =
                  ((unsigned long long)hi << 32) | lo;
              const int bk = __builtin_amdgcn_readlane(wb[h], kl);
              if ((wk >> lane) & 1ull) {
                const int i = bk + __popcll(wk & below) - c0;
                if (i >= 0 && i < kCand)
                  repulsion_pair(P, Xp, Yp, Rp, cX[w][i], cY[w][i],
                                 cR[w][i], cx, cy);
              }
            }
          }
          wave_lds_sync();
        }
      }
    } else {
      auto& sX = psh.all.X;
      auto& sY = psh.all.Y;
      auto& sR = psh.all.R;
      for (int c0 = 0; c0 < P.np; c0 += kStage) {
        const int m1 = min(kStage, P.np - c0);
        for (int m = (int)threadIdx.x; m < m1; m += (int)blockDim.x) {
          sX[m] = cur.X[c0 + m];
          sY[m] = cur.Y[c0 + m];
          sR[m] = pc.R[c0 + m];
        }
        __syncthreads();
        if (mine) {
          for (int m = lane; m < m1; m += 64) {
            if (c0 + m == p) continue;
            repulsion_pair(P, Xp, Yp, Rp, sX[m], sY[m], sR[m], cx, cy);
          }
        }
        __syncthreads();
      }
    }
    if (mine) {
      cx = wave_sum(cx);
      cy = wave_sum(cy);
      repulsion_walls(P, Xp, Yp, Rp, cx, cy);
    }
  }
  if (!mine) return;  // whole wave
  if (sums) {
    if (P.scan) {
      reduce_partials(P, cur, pc, partial, have_partials, p, lane, fx, fy, tz);
    } else {
      fx += o0;
      fy += o1;
      tz += o2;
      for (int k = lane + 64; k < ns; k += 64) {
        fx += src[k * kRedVals + 0];
        fy += src[k * kRedVals + 1];
        tz += src[k * kRedVals + 2];
      }
      fx = wave_sum(fx);
      fy = wave_sum(fy);
      tz = wave_sum(tz);
    }
  }

  if (mode == kModeReduceOnly) {
    if (lane == 0) {
      cur.Fx[p] = fx;
      cur.Fy[p] = fy;
      cur.Tz[p] = tz;
    }
    return;
  }
  double nX = own.X, nY = own.Y;
  if (mode == kModeUpdate) {
    const PUpd u = particle_update_one(P, own, fx, fy, tz, cx, cy);
    if (lane == 0) store_particle(next, p, u);
    nX = u.X;
    nY = u.Y;
  }

  // ---- block lists for the band box at the new position
  const double R = own.R;
  const bool ok = centre_ok(P, nX, nY);
  if (!ok && lane == 0) atomicOr(flags, kFlagUnstable);
  // ---- the centre bin of the new position (list form): its place is taken
  // now and its entry written after the block lists' adds are issued, so
  // that the two round trips overlap
  int bpos = kBinCap, bidx = 0;
  if (L.bcnt && ok && lane == 0) {
    int bx, by;
    centre_bin(P, nX, nY, bx, by);
    bidx = by * P.nbx + bx;
    bpos = atomicAdd(&L.bcnt[bidx], 1);
  }
  int i0 = 0, i1 = -1, j0 = 0, j1 = -1;
  if (ok) band_box(P, nX, nY, R, i0, i1, j0, j1);
  const int rows = j1 - j0 + 1;
  const ColSegs cs = col_segments(i0, i1, P.nx);
  int f0 = 0, l0 = -1, f1 = 0, l1 = -1;   // this row's blocks
  if (lane < rows) {
    row_block_ranges(sorted_row(lane, j0, j1, P.ny), cs, P.nx, f0, l0, f1,
                     l1);
    if (lane > 0 && (l0 >= f0 || l1 >= f1)) {
      int g0, m0, g1, m1;
      row_block_ranges(sorted_row(lane - 1, j0, j1, P.ny), cs, P.nx, g0, m0,
                       g1, m1);
      const bool prev = m0 >= g0 || m1 >= g1;
      const int plast = m1 >= g1 ? m1 : m0;   // the previous row's last
      if (prev && plast == (l0 >= f0 ? f0 : f1)) {  // shared: listed there
        if (l0 >= f0) ++f0;
        else ++f1;
      }
    }
  }
  const int n0 = max(l0 - f0 + 1, 0);
  const int nb = n0 + max(l1 - f1 + 1, 0);
  int total;
  const int base = wave_excl_scan<3>(nb, lane, total);
  for (int k = 0; k < nb; ++k) {
    const int blk = k < n0 ? f0 + k : f1 + (k - n0);
    const int slot = p * P.maxb + base + k;
    const int pos = atomicAdd(&L.cnt[blk], 1);
    if (pos < kListCap)
      L.ent[(size_t)blk * kListCap + pos] = make_int2(p, slot);
    else
      atomicOr(flags, kFlagListFull);
  }
  if (lane == 0) {
    PState& dst = (mode == kModeBinOnly) ? cur : next;
    dst.nslot[p] = total;
    if (bpos < kBinCap) L.bent[(size_t)bidx * kBinCap + bpos] = p;
  }
}

// Scan form: per tile, the particles whose band box reaches it at the next
// step's positions (X + U of the stored state; the arithmetic of that
// step's scan_task_tile), one wave per particle.  Afterwards the step
// kernel keeps the counts itself.
__global__ __launch_bounds__(256) void k_tile_counts(const Params P,
                                                     PState cur, PConst pc,
                                                     int* count, int* flags) {
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (p >= P.np) return;
  double X = cur.X[p], Y = cur.Y[p];
  advance_position(P, X, Y, cur.Ux[p], cur.Uy[p]);
  const BlockRanges r = block_ranges(P, X, Y, pc.R[p], kBlock);
  for (int j = lane; j < r.count(); j += 64) atomicAdd(&count[r.at(j)], 1);
  // a centre the band-box logic cannot place: no tile serves it
  if (r.n == 0 && lane == 0) atomicOr(flags, kFlagUnstable);
}

// -------------------------------------------------------------------------
// Per-particle thermal sums over the band box, one block per particle, in a
// fixed order: sum f_s,p, sum f_s,p T, sum f_s,p c_vs T, min T over cells
// wholly inside (else over touched cells).

__global__ __launch_bounds__(256) void k_particle_sums(
    const Params P, PState ps, PConst pc, const double* __restrict__ macro,
    double* __restrict__ out4) {
  const int p = blockIdx.x;
  const double X0 = ps.X[p], Y0 = ps.Y[p], R = pc.R[p], Rb = pc.Rb[p];
  double cth, sth;
  orientation(R, Rb, ps.th[p], cth, sth);
  int i0 = 0, i1 = -1, j0 = 0, j1 = -1;
  if (centre_ok(P, X0, Y0)) band_box(P, X0, Y0, R, i0, i1, j0, j1);
  const int w = max(i1 - i0 + 1, 0), h = max(j1 - j0 + 1, 0);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, tmin_full = INFINITY, tmin_any = INFINITY;
  const double* Tf = macro + 3 * (size_t)P.N;
  for (int k = threadIdx.x; k < w * h; k += blockDim.x) {
    int i = i0 + k % w, j = j0 + k / w;
    if (P.perx) i = (i % P.nx + P.nx) % P.nx;
    if (P.pery) j = (j % P.ny + P.ny) % P.ny;
    const double xn = i + 0.5, yn = j + 0.5;
    const double X = near_copy(X0, xn, (double)P.nx, P.perx);
    const double Y = near_copy(Y0, yn, (double)P.ny, P.pery);
    if (!owns_cell(X, Y, R, i, j)) continue;
    const bool full = cell_within(X, Y, Rb, i, j);
    const double a =
        full ? 1.0 : shape_share<true>(X, Y, R, Rb, cth, sth, i, j);
    const double Tc = Tf[(size_t)j * P.nx + i];
    s0 += a;
    s1 += a * Tc;
    s2 += a * P.cvs * Tc;
    tmin_any = fmin(tmin_any, Tc);
    if (full) tmin_full = fmin(tmin_full, Tc);
  }
  __shared__ double red[4][5];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  tmin_full = wave_min(tmin_full);
  tmin_any = wave_min(tmin_any);
  if (lane == 0) {
    red[wv][0] = s0; red[wv][1] = s1; red[wv][2] = s2;
    red[wv][3] = tmin_full; red[wv][4] = tmin_any;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0, b = 0, c = 0, mf = INFINITY, ma = INFINITY;
    for (int k = 0; k < 4; ++k) {
      a += red[k][0]; b += red[k][1]; c += red[k][2];
      mf = fmin(mf, red[k][3]); ma = fmin(ma, red[k][4]);
    }
    out4[4 * p + 0] = a > 0.0 ? b / a : 0.0;        // T_mean
    out4[4 * p + 1] = isfinite(mf) ? mf : ma;        // T_min
    out4[4 * p + 2] = c;                             // E_solid
    out4[4 * p + 3] = a;                             // fs_sum
  }
}

// -------------------------------------------------------------------------
// Cell ownership for inspection: the same block lists and predicates as the
// lattice pass.

template <bool SCAN>
__global__ __launch_bounds__(kBlock) void k_ownership(
    const Params P, PState ps, PConst pc, Lists L, int tile0, int* count,
    int* ids, int* full, int* flags) {
  __shared__ BlockParticles bp;
  __shared__ int tmp[kListCap];
  const int tile = tile0 + blockIdx.x;
  gather_particles<SCAN>(bp, tmp, P, tile, ps, ps, pc, L, nullptr, 0, false,
                         flags);
  const int c = tile * kBlock + threadIdx.x;
  if (c >= P.N) return;
  const int y = c / P.nx, x = c - y * P.nx;
  // outputs are indexed from the first cell of tile0
  const int o = c - tile0 * kBlock;
  count += o;
  ids += (size_t)o * P.kmax;
  full += (size_t)o * P.kmax;
  int n = 0;
  for (int k = 0; k < P.kmax; ++k) {
    ids[k] = -1;
    full[k] = 0;
  }
  for (int s = 0; s < bp.cnt; ++s) {
    const double xn = x + 0.5, yn = y + 0.5;
    const double X = near_copy(bp.X[s], xn, (double)P.nx, P.perx);
    const double Y = near_copy(bp.Y[s], yn, (double)P.ny, P.pery);
    if (!owns_cell(X, Y, bp.R[s], x, y)) continue;
    if (n < P.kmax) {
      ids[n] = bp.pid[s];
      full[n] = cell_within(X, Y, bp.Rb[s], x, y) ? 1 : 0;
    }
    ++n;
  }
  if (n > P.kmax) atomicOr(flags, kFlagOverlap);
  count[0] = n < P.kmax ? n : P.kmax;
}

// Memory-pattern probe: the step kernel's global-memory traffic without its
// arithmetic.  Per cell: the pulled loads of the nine f and nine g
// populations (periodic neighbours, the same SoA planes), the carrier load,
// and the 9 + 9 + 1 stores, over the same XCD-ordered tiles.  What it
// reaches is the bandwidth the access pattern itself allows on the device:
// the ceiling the step kernel's algorithmic bandwidth is compared with.
template <int PREC>
__global__ __launch_bounds__(kBlock) void k_stream_probe(
    const Params P, const typename Prec<PREC>::S* __restrict__ fin,
    typename Prec<PREC>::S* __restrict__ fout,
    const typename Prec<PREC>::S* __restrict__ gin,
    typename Prec<PREC>::S* __restrict__ gout,
    const typename Prec<PREC>::H* __restrict__ hin,
    typename Prec<PREC>::H* __restrict__ hout, size_t plane) {
  typedef typename Prec<PREC>::S S;
  const int tile = stream_tile(P, blockIdx.x);
  if (tile >= P.nblocks) return;
  const int c = tile * kBlock + threadIdx.x;
  if (c >= P.N) return;
  const int y = c / P.nx, x = c - y * P.nx;
  const int xm = x == 0 ? P.nx - 1 : x - 1, xp = x == P.nx - 1 ? 0 : x + 1;
  const int ym = y == 0 ? P.ny - 1 : y - 1, yp = y == P.ny - 1 ? 0 : y + 1;
  const int src[9] = {c,           y * P.nx + xm,  ym * P.nx + x,
                      y * P.nx + xp, yp * P.nx + x, ym * P.nx + xm,
                      ym * P.nx + xp, yp * P.nx + xp, yp * P.nx + xm};
  S f[9], g[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    f[q] = fin[(size_t)q * plane + src[q]];
    g[q] = gin[(size_t)q * plane + src[q]];
  }
  const typename Prec<PREC>::H h = hin[c];
  if (P.nt_stores) {     // as the step kernel stores them
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      __builtin_nontemporal_store(f[q], fout + (size_t)q * plane + c);
      __builtin_nontemporal_store(g[q], gout + (size_t)q * plane + c);
    }
    __builtin_nontemporal_store(h, hout + c);
  } else {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      fout[(size_t)q * plane + c] = f[q];
      gout[(size_t)q * plane + c] = g[q];
    }
    hout[c] = h;
  }
}

// Populations of the current state as FP64 (unshifted).
template <int PREC>
__global__ void k_unpack(const Params P, const typename Prec<PREC>::S* pop,
                         size_t plane, int which_g, double* out) {
  typedef Prec<PREC> T;
  const size_t N = (size_t)P.N;
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= 9 * N) return;
  const int q = (int)(k / N);
  const size_t c = k - (size_t)q * N;
  const double sh = which_g ? P.gshift[q] : P.fshift[q];
  out[k] = (double)T::ld(pop, (size_t)q * plane + c) + sh;
}

// -------------------------------------------------------------------------
// Launchers


hipError_t launch_particles(const Params& P, PState cur, PState next,
                            PConst pc, Lists L, const double* partial,
                            int have_partials, int mode, int* flags,
                            hipStream_t s) {
  if (P.np == 0) return hipSuccess;
  hipLaunchKernelGGL(k_particles, dim3(blocks_for(P.np, 4)), dim3(256), 0, s,
                     P, cur, next, pc, L, partial, have_partials, mode, flags);
  return hipGetLastError();
}

template <int PREC, bool OUT, bool SCAN, bool PAIR, bool ELL, bool NT>
static hipError_t step_t(const StepLaunch& a, hipStream_t s) {
  const Params& P = *a.P;
  // the host keeps the tile counts exactly where this kernel reads them
  if (SCAN && counted_tiles(PREC, PAIR) &&
      !(a.B.tcount && a.B.tcount_next && a.B.tcount_clear))
    return hipErrorInvalidValue;
  const Hot<typename Prec<PREC>::C> H = make_hot<typename Prec<PREC>::C>(P);
  const unsigned grid = (unsigned)(P.nfirst + stream_grid(P, PAIR));
  hipExtLaunchKernelGGL((k_step<PREC, OUT, SCAN, PAIR, ELL, NT>), dim3(grid),
                        dim3(kBlock), 0, s, a.ev_start, a.ev_stop, 0, P, H,
                        a.B, a.have);
  return hipGetLastError();
}

// the list form's non-temporal stores: FP64 and FP32 disk domains only
template <int PREC>
constexpr bool kNtStores = PREC == VLB_FP64 || PREC == VLB_FP32;

template <int PREC, bool PAIR, bool ELL>
static hipError_t step_q(const StepLaunch& a, hipStream_t s) {
  if (a.P->scan)
    return a.out ? step_t<PREC, true, true, PAIR, ELL, false>(a, s)
                 : step_t<PREC, false, true, PAIR, ELL, false>(a, s);
  if constexpr (kNtStores<PREC> && !PAIR && !ELL)
    if (a.P->nt_stores)
      return a.out ? step_t<PREC, true, false, false, false, true>(a, s)
                   : step_t<PREC, false, false, false, false, true>(a, s);
  if (a.P->nt_stores) return hipErrorInvalidValue;
  return a.out ? step_t<PREC, true, false, PAIR, ELL, false>(a, s)
               : step_t<PREC, false, false, PAIR, ELL, false>(a, s);
}

// A domain holding ellipses runs the step kernel built with their geometry
// (never with paired tiles, which the host turns off for it); disk domains
// run kernels without it.
template <int PREC>
static hipError_t step_p(const StepLaunch& a, hipStream_t s) {
  if (a.P->ellipses) {
    if (a.P->pair_tiles) return hipErrorInvalidValue;
    return step_q<PREC, false, true>(a, s);
  }
  if constexpr (kPairedTiles<PREC>)
    if (a.P->pair_tiles) return step_q<PREC, true, false>(a, s);
  return step_q<PREC, false, false>(a, s);
}

hipError_t launch_step(int prec, const StepLaunch& a, hipStream_t s) {
  switch (prec) {
    case VLB_FP64: return step_p<VLB_FP64>(a, s);
    case VLB_FP32: return step_p<VLB_FP32>(a, s);
    case VLB_FP16_SHIFT: return step_p<VLB_FP16_SHIFT>(a, s);
    case VLB_BF16_SHIFT: return step_p<VLB_BF16_SHIFT>(a, s);
  }
  return hipErrorInvalidValue;
}

template <int PREC, bool SCAN>
static hipError_t init_t(const Params& P, void* f, void* g, void* h,
                         size_t plane, PState ps, PConst pc, Lists L,
                         double* macro, int* flags, hipStream_t s) {
  hipLaunchKernelGGL((k_init<PREC, SCAN>), dim3(P.nblocks), dim3(kBlock), 0,
                     s, P, (typename Prec<PREC>::S*)f,
                     (typename Prec<PREC>::S*)g, (typename Prec<PREC>::H*)h,
                     plane, ps, pc, L, macro, flags);
  return hipGetLastError();
}

hipError_t launch_init(int prec, const Params& P, void* f, void* g, void* h,
                       size_t plane, PState ps, PConst pc, Lists L,
                       double* macro, int* flags, hipStream_t s) {
#define VLB_INIT(PR)                                                        \
  return P.scan ? init_t<PR, true>(P, f, g, h, plane, ps, pc, L, macro,     \
                                   flags, s)                                \
                : init_t<PR, false>(P, f, g, h, plane, ps, pc, L, macro,    \
                                    flags, s);
  switch (prec) {
    case VLB_FP64: VLB_INIT(VLB_FP64)
    case VLB_FP32: VLB_INIT(VLB_FP32)
    case VLB_FP16_SHIFT: VLB_INIT(VLB_FP16_SHIFT)
    case VLB_BF16_SHIFT: VLB_INIT(VLB_BF16_SHIFT)
  }
#undef VLB_INIT
  return hipErrorInvalidValue;
}

hipError_t launch_tile_counts(const Params& P, PState cur, PConst pc,
                              int* count, int* flags, hipStream_t s) {
  if (P.np == 0) return hipSuccess;
  hipLaunchKernelGGL(k_tile_counts, dim3(blocks_for(P.np, 4)), dim3(256), 0,
                     s, P, cur, pc, count, flags);
  return hipGetLastError();
}

hipError_t launch_particle_sums(const Params& P, PState ps, PConst pc,
                                const double* macro, double* out4,
                                hipStream_t s) {
  if (P.np == 0) return hipSuccess;
  hipLaunchKernelGGL(k_particle_sums, dim3(P.np), dim3(256), 0, s, P, ps, pc,
                     macro, out4);
  return hipGetLastError();
}

hipError_t launch_ownership(const Params& P, PState ps, PConst pc, Lists L,
                            int tile0, int ntiles, int* count, int* ids,
                            int* full, int* flags, hipStream_t s) {
  if (tile0 < 0 || ntiles <= 0 || tile0 + ntiles > P.nblocks)
    return hipErrorInvalidValue;
  if (P.scan)
    hipLaunchKernelGGL(k_ownership<true>, dim3(ntiles), dim3(kBlock), 0, s,
                       P, ps, pc, L, tile0, count, ids, full, flags);
  else
    hipLaunchKernelGGL(k_ownership<false>, dim3(ntiles), dim3(kBlock), 0, s,
                       P, ps, pc, L, tile0, count, ids, full, flags);
  return hipGetLastError();
}

hipError_t launch_stream_probe(int prec, const Params& P, const StepBufs& B,
                              hipStream_t s) {
  const unsigned nb = (unsigned)P.stream_blocks;
#define VLB_PROBE(PR)                                                        \
  hipLaunchKernelGGL(k_stream_probe<PR>, dim3(nb), dim3(kBlock), 0, s, P,     \
                     (const Prec<PR>::S*)B.fi, (Prec<PR>::S*)B.fo,            \
                     (const Prec<PR>::S*)B.gi, (Prec<PR>::S*)B.go,            \
                     (const Prec<PR>::H*)B.hin, (Prec<PR>::H*)B.hout,         \
                     B.plane);                                                \
  return hipGetLastError();
  switch (prec) {
    case VLB_FP64: VLB_PROBE(VLB_FP64)
    case VLB_FP32: VLB_PROBE(VLB_FP32)
    case VLB_FP16_SHIFT: VLB_PROBE(VLB_FP16_SHIFT)
    case VLB_BF16_SHIFT: VLB_PROBE(VLB_BF16_SHIFT)
  }
#undef VLB_PROBE
  return hipErrorInvalidValue;
}

hipError_t launch_unpack(int prec, const Params& P, const void* pop,
                         size_t plane, int which_g, double* out,
                         hipStream_t s) {
  const unsigned nb = blocks_for(9L * P.N, 256);
#define VLB_UNPACK(PR)                                                       \
  hipLaunchKernelGGL(k_unpack<PR>, dim3(nb), dim3(256), 0, s, P,              \
                     (const Prec<PR>::S*)pop, plane, which_g, out);           \
  return hipGetLastError();
  switch (prec) {
    case VLB_FP64: VLB_UNPACK(VLB_FP64)
    case VLB_FP32: VLB_UNPACK(VLB_FP32)
    case VLB_FP16_SHIFT: VLB_UNPACK(VLB_FP16_SHIFT)
    case VLB_BF16_SHIFT: VLB_UNPACK(VLB_BF16_SHIFT)
  }
#undef VLB_UNPACK
  return hipErrorInvalidValue;
}

}  // namespace vlb
