// vlb_kernels.hip -- gfx950 kernels of the volumetric lattice Boltzmann step
// for thermal particulate flow with conjugate heat transfer (arXiv
// 2410.23802).
//
// Data layout in HBM (one context):
//   populations  f, g : 9 planes each, plane stride `plane` >= N = nx*ny,
//                       cell c = j*nx + i (x fastest); two copies (A/B),
//                       pull streaming reads A and writes B.
//   h                 : 1 value per cell, the carrier h = 2 f_s + [df_s/dt]
//                       of the eq. dfs_dt recursion (updated in place).
//   macro             : rho, ux, uy, T, f_s, [df_s/dt] as FP64 planes,
//                       written only by the last step of a vlb_step call.
//   block lists       : per 256-cell block, the particles whose band box
//                       reaches it, with the partial slot to write.
//   partials          : per particle and touched block, the block's share of
//                       the momentum-exchange force and torque (FP64).
//
// One time step is two launches: k_particles (reduce the partials of the
// previous step, Newton-Euler update, fill the block lists) and k_lattice
// (everything per cell, one HBM pass).  No floating-point atomics: every sum
// runs in a fixed order, so a run is bitwise reproducible.
#include <math.h>

#include "vlb_internal.h"

namespace vlb {

// -------------------------------------------------------------------------
// Storage forms.  FP16/BF16 keep the deviation from a per-direction shift
// and compute in FP32; the [df_s/dt] carrier stays FP32 there.

template <int PREC>
struct Prec;

template <>
struct Prec<VLB_FP64> {
  typedef double S;
  typedef double C;
  typedef double H;
  static __device__ __forceinline__ C ld(const S* p, size_t i, C) { return p[i]; }
  static __device__ __forceinline__ void st(S* p, size_t i, C v, C) { p[i] = v; }
};

template <>
struct Prec<VLB_FP32> {
  typedef float S;
  typedef float C;
  typedef float H;
  static __device__ __forceinline__ C ld(const S* p, size_t i, C) { return p[i]; }
  static __device__ __forceinline__ void st(S* p, size_t i, C v, C) { p[i] = v; }
};

template <>
struct Prec<VLB_FP16_SHIFT> {
  typedef _Float16 S;
  typedef float C;
  typedef float H;
  static __device__ __forceinline__ C ld(const S* p, size_t i, C sh) {
    return (float)p[i] + sh;
  }
  static __device__ __forceinline__ void st(S* p, size_t i, C v, C sh) {
    p[i] = (_Float16)(v - sh);
  }
};

template <>
struct Prec<VLB_BF16_SHIFT> {
  typedef uint16_t S;
  typedef float C;
  typedef float H;
  static __device__ __forceinline__ C ld(const S* p, size_t i, C sh) {
    return __uint_as_float(((uint32_t)p[i]) << 16) + sh;
  }
  static __device__ __forceinline__ void st(S* p, size_t i, C v, C sh) {
    // round to nearest even on the upper 16 bits
    uint32_t b = __float_as_uint(v - sh);
    b += 0x7fffu + ((b >> 16) & 1u);
    p[i] = (uint16_t)(b >> 16);
  }
};

// -------------------------------------------------------------------------
// Geometry (FP64 in every storage form).

// Nearest periodic copy of a particle coordinate seen from a node.
__device__ __forceinline__ double near_copy(double Xp, double node, double L,
                                            int periodic) {
  if (periodic) {
    double half = 0.5 * L;
    if (node - Xp > half) return Xp + L;
    if (Xp - node > half) return Xp - L;
  }
  return Xp;
}

// Integer ownership: the point of cell (i, j) nearest to the centre lies
// strictly inside the circle.  Evaluated without fused multiply-adds so the
// decision is the same on every IEEE machine.
__device__ __noinline__ bool owns_cell(double X, double Y, double R, int i,
                                       int j) {
#pragma clang fp contract(off)
  double lo = (double)i, hi = (double)(i + 1);
  double nx_ = X < lo ? lo : (X > hi ? hi : X);
  double ddx = X - nx_;
  lo = (double)j;
  hi = (double)(j + 1);
  double ny_ = Y < lo ? lo : (Y > hi ? hi : Y);
  double ddy = Y - ny_;
  double q = ddx * ddx;
  q = q + ddy * ddy;
  return q < R * R;
}

// The cell lies in the closed disk: its corner farthest from the centre does.
__device__ __noinline__ bool cell_within(double X, double Y, double R, int i,
                                         int j) {
#pragma clang fp contract(off)
  double ex = (X < (double)i + 0.5) ? (double)(i + 1) - X : X - (double)i;
  double ey = (Y < (double)j + 0.5) ? (double)(j + 1) - Y : Y - (double)j;
  double q = ex * ex;
  q = q + ey * ey;
  return q <= R * R;
}

// Signed area of (disk of radius R at the origin) intersected with the
// triangle (origin, P, Q): the chord part of PQ inside the circle gives a
// triangle, the parts outside give circular sectors.
__device__ double tri_disk_area(double px, double py, double qx, double qy,
                                double R) {
  const double half_r2 = 0.5 * R * R;
  double dx = qx - px, dy = qy - py;
  double a = dx * dx + dy * dy;
  double b = px * dx + py * dy;
  double c = (px * px + py * py) - R * R;
  double disc = b * b - a * c;
  double s1 = 1.0, s2 = 0.0;
  if (disc > 0.0) {
    double r = sqrt(disc);
    s1 = fmin(fmax((-b - r) / a, 0.0), 1.0);
    s2 = fmin(fmax((-b + r) / a, 0.0), 1.0);
  }
  if (!(s1 < s2)) return half_r2 * atan2(px * qy - py * qx, px * qx + py * qy);
  double ax = px + s1 * dx, ay = py + s1 * dy;
  double bx = px + s2 * dx, by = py + s2 * dy;
  double area = 0.5 * (ax * by - ay * bx);
  if (s1 > 0.0) area += half_r2 * atan2(px * ay - py * ax, px * ax + py * ay);
  if (s2 < 1.0) area += half_r2 * atan2(bx * qy - by * qx, bx * qx + by * qy);
  return area;
}

// Exact share of cell (i, j) covered by the disk (centre X, Y, radius R),
// by Green's theorem over the four edges of the square taken
// counter-clockwise.
__device__ double covered_share(double X, double Y, double R, int i, int j) {
  double x0 = (double)i - X, x1 = (double)(i + 1) - X;
  double y0 = (double)j - Y, y1 = (double)(j + 1) - Y;
  double A = tri_disk_area(x0, y0, x1, y0, R) + tri_disk_area(x1, y0, x1, y1, R) +
             tri_disk_area(x1, y1, x0, y1, R) + tri_disk_area(x0, y1, x0, y0, R);
  return fmin(fmax(A, 0.0), 1.0);
}

// -------------------------------------------------------------------------
// Reductions (fixed order: xor butterfly inside a wave, waves in index order).

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Sum of three values over the 256 threads of a block, result in thread 0.
// `red` holds 4 waves x 3 values of LDS.  Contains two barriers.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c,
                                           double (*red)[3]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  if (lane == 0) {
    red[w][0] = a;
    red[w][1] = b;
    red[w][2] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = ((red[0][0] + red[1][0]) + red[2][0]) + red[3][0];
    b = ((red[0][1] + red[1][1]) + red[2][1]) + red[3][1];
    c = ((red[0][2] + red[1][2]) + red[2][2]) + red[3][2];
  }
  __syncthreads();
}

// -------------------------------------------------------------------------
// Block particle list: load, sort by particle id, stage the particle data in
// LDS, and reset the global count for the next particle pass.

struct BlockParticles {
  int cnt;
  int pid[kListCap];
  int slot[kListCap];
  double X[kListCap], Y[kListCap], R[kListCap];
  double Ux[kListCap], Uy[kListCap], Om[kListCap], Tp[kListCap];
};

__device__ __forceinline__ void load_block_list(BlockParticles& bp, int* tmp,
                                                Lists L, PState pn, PConst pc,
                                                int* flags) {
  const int b = blockIdx.x, t = threadIdx.x;
  if (t == 0) {
    int n = L.cnt[b];
    if (n > kListCap) {
      atomicOr(flags, kFlagListFull);
      n = kListCap;
    }
    bp.cnt = n;
    L.cnt[b] = 0;  // consumed
  }
  __syncthreads();
  const int n = bp.cnt;
  if (n == 0) return;
  int2 e = make_int2(0, 0);
  if (t < n) {
    e = L.ent[(size_t)b * kListCap + t];
    tmp[t] = e.x;
  }
  __syncthreads();
  if (t < n) {
    int rank = 0;
    for (int k = 0; k < n; ++k) rank += tmp[k] < e.x;
    bp.pid[rank] = e.x;
    bp.slot[rank] = e.y;
    bp.X[rank] = pn.X[e.x];
    bp.Y[rank] = pn.Y[e.x];
    bp.R[rank] = pc.R[e.x];
    bp.Ux[rank] = pn.Ux[e.x];
    bp.Uy[rank] = pn.Uy[e.x];
    bp.Om[rank] = pn.Om[e.x];
    bp.Tp[rank] = pc.Tinit[e.x];
  }
  __syncthreads();
}

// Geometry of slot s for the cell (i, j): covered share and solid velocity
// u_s = U + Omega x (x - X) at the node (eq. us).  Returns false when the
// particle does not reach the cell.
struct SlotGeom {
  double fs, usx, usy, rx, ry;
  bool full;
};

__device__ __forceinline__ bool slot_geometry(const BlockParticles& bp, int s,
                                              const Params& P, int i, int j,
                                              SlotGeom& g) {
  double xn = (double)i + 0.5, yn = (double)j + 0.5;
  double X = near_copy(bp.X[s], xn, (double)P.nx, P.perx);
  double Y = near_copy(bp.Y[s], yn, (double)P.ny, P.pery);
  double R = bp.R[s];
  if (!owns_cell(X, Y, R, i, j)) return false;
  g.full = cell_within(X, Y, R, i, j);
  g.fs = g.full ? 1.0 : covered_share(X, Y, R, i, j);
  g.rx = xn - X;
  g.ry = yn - Y;
  g.usx = bp.Ux[s] - bp.Om[s] * g.ry;
  g.usy = bp.Uy[s] + bp.Om[s] * g.rx;
  return true;
}

// -------------------------------------------------------------------------
// The fused lattice pass.

template <int PREC, bool OUT>
__global__ __launch_bounds__(kBlock) void k_lattice(
    const Params P, const typename Prec<PREC>::S* __restrict__ fin,
    typename Prec<PREC>::S* __restrict__ fout,
    const typename Prec<PREC>::S* __restrict__ gin,
    typename Prec<PREC>::S* __restrict__ gout,
    typename Prec<PREC>::H* __restrict__ hcar, size_t plane, PState pn,
    PConst pc, Lists L, double* __restrict__ partial,
    double* __restrict__ macro, int* flags) {
  typedef Prec<PREC> T;
  typedef typename T::C C;
  typedef typename T::H H;
  __shared__ BlockParticles bp;
  __shared__ int tmp[kListCap];
  __shared__ double red[4][3];

  load_block_list(bp, tmp, L, pn, pc, flags);
  const int cnt = bp.cnt;

  const int c = blockIdx.x * kBlock + threadIdx.x;
  const bool act = c < P.N;
  const int cc = act ? c : P.N - 1;
  const int y = cc / P.nx;
  const int x = cc - y * P.nx;

  // ---- pull streaming with the wall rules (eq. lbe.rho.str, lbe.e.str)
  int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
  bool oxm = false, oxp = false, oym = false, oyp = false;
  if (xm < 0) { if (P.perx) xm += P.nx; else oxm = true; }
  if (xp >= P.nx) { if (P.perx) xp -= P.nx; else oxp = true; }
  if (ym < 0) { if (P.pery) ym += P.ny; else oym = true; }
  if (yp >= P.ny) { if (P.pery) yp -= P.ny; else oyp = true; }
  const int rx_m = xm, rx_p = xp, ry_m = ym * P.nx, ry_p = yp * P.nx,
            r0 = y * P.nx;
  // upstream cell, whether it lies beyond a wall, and which wall decides
  int src[9];
  bool out[9];
  int wall[9];
  src[0] = cc;                 out[0] = false;          wall[0] = 0;
  src[1] = r0 + rx_m;          out[1] = oxm;            wall[1] = VLB_FACE_XLO;
  src[2] = ry_m + x;           out[2] = oym;            wall[2] = VLB_FACE_YLO;
  src[3] = r0 + rx_p;          out[3] = oxp;            wall[3] = VLB_FACE_XHI;
  src[4] = ry_p + x;           out[4] = oyp;            wall[4] = VLB_FACE_YHI;
  src[5] = ry_m + rx_m;        out[5] = oxm || oym;     wall[5] = oym ? VLB_FACE_YLO : VLB_FACE_XLO;
  src[6] = ry_m + rx_p;        out[6] = oxp || oym;     wall[6] = oym ? VLB_FACE_YLO : VLB_FACE_XHI;
  src[7] = ry_p + rx_p;        out[7] = oxp || oyp;     wall[7] = oyp ? VLB_FACE_YHI : VLB_FACE_XHI;
  src[8] = ry_p + rx_m;        out[8] = oxm || oyp;     wall[8] = oyp ? VLB_FACE_YHI : VLB_FACE_XLO;
  const int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

  C f[9], g[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const int sq = out[q] ? opp[q] : q;
    const size_t idx = (size_t)sq * plane + (size_t)(out[q] ? cc : src[q]);
    C fv = 0, gv = 0;
    if (act) {
      fv = T::ld(fin, idx, (C)P.fshift[sq]);
      gv = T::ld(gin, idx, (C)P.gshift[sq]);
    }
    if (out[q]) {
      const int w = wall[q];
      fv = fv + (C)P.fadd[w][q];
      gv = (C)P.gsign[w] * gv + (C)P.gadd[w][q];
    }
    f[q] = fv;
    g[q] = gv;
  }
  H hn = act ? hcar[cc] : (H)0;

  // ---- moments of f* (rows of M, Sec. 2.1)
  const C a14 = f[1] + f[2] + f[3] + f[4];
  const C a58 = f[5] + f[6] + f[7] + f[8];
  C m[9];
  m[0] = f[0] + a14 + a58;
  m[1] = -4 * f[0] - a14 + 2 * a58;
  m[2] = 4 * f[0] - 2 * a14 + a58;
  m[3] = f[1] - f[3] + f[5] - f[6] - f[7] + f[8];
  m[4] = -2 * f[1] + 2 * f[3] + f[5] - f[6] - f[7] + f[8];
  m[5] = f[2] - f[4] + f[5] + f[6] - f[7] - f[8];
  m[6] = -2 * f[2] + 2 * f[4] + f[5] + f[6] - f[7] - f[8];
  m[7] = f[1] - f[2] + f[3] - f[4];
  m[8] = f[5] - f[6] + f[7] - f[8];
  const C rho = m[0];          // rho = sum f*_i, kept by eq. fi
  const C jxs = m[3], jys = m[5];

  // ---- particles: solid fraction, u_s, momentum exchange (Sec. 2.3)
  C S0 = 0, S1x = 0, S1y = 0, S2xx = 0, S2yy = 0, S2xy = 0;
  int nin = 0;
  for (int s = 0; s < cnt; ++s) {
    double cfx = 0.0, cfy = 0.0, ctz = 0.0;
    SlotGeom sg;
    if (act && slot_geometry(bp, s, P, x, y, sg)) {
      ++nin;
      const C a = (C)sg.fs, ux = (C)sg.usx, uy = (C)sg.usy;
      S0 += a;
      S1x += a * ux;
      S1y += a * uy;
      S2xx += a * ux * ux;
      S2yy += a * uy * uy;
      S2xy += a * ux * uy;
      // this particle's share of sum_i (f_i - f*_i) e_i = f_s,p (rho u_s - j*)
      const double dpx = (double)(a * (rho * ux - jxs));
      const double dpy = (double)(a * (rho * uy - jys));
      cfx = -dpx;
      cfy = -dpy;
      ctz = -(sg.rx * dpy - sg.ry * dpx);
    }
    block_sum3(cfx, cfy, ctz, red);
    if (threadIdx.x == 0) {
      double* o = partial + (size_t)bp.slot[s] * kRedVals;
      o[0] = cfx;
      o[1] = cfy;
      o[2] = ctz;
    }
  }
  if (nin > P.kmax) atomicOr(flags, kFlagOverlap);
  // Overlapping disks: shares are scaled to sum to one (rare path; the
  // momentum-exchange partials get the matching correction).
  if (cnt > 0 && __syncthreads_or(S0 > (C)1)) {
    const bool over = S0 > (C)1;
    const C inv = over ? (C)1 / S0 : (C)1;
    for (int s = 0; s < cnt; ++s) {
      double cfx = 0.0, cfy = 0.0, ctz = 0.0;
      SlotGeom sg;
      if (act && over && slot_geometry(bp, s, P, x, y, sg)) {
        const C a = (C)sg.fs, ux = (C)sg.usx, uy = (C)sg.usy;
        const double k = (double)(inv - (C)1);
        const double dpx = (double)(a * (rho * ux - jxs));
        const double dpy = (double)(a * (rho * uy - jys));
        cfx = -dpx * k;
        cfy = -dpy * k;
        ctz = -(sg.rx * dpy - sg.ry * dpx) * k;
      }
      block_sum3(cfx, cfy, ctz, red);
      if (threadIdx.x == 0) {
        double* o = partial + (size_t)bp.slot[s] * kRedVals;
        o[0] += cfx;
        o[1] += cfy;
        o[2] += ctz;
      }
    }
    if (over) {
      S1x *= inv; S1y *= inv; S2xx *= inv; S2yy *= inv; S2xy *= inv;
      S0 = (C)1;
    }
  }

  // ---- volumetric no-slip step in moment space (eq. fi):
  // m = (1 - f_s) M f* + rho * sum_p f_s,p m^eq(1, u_s,p)
  const C fs = S0;
  const C wf = (C)1 - fs;
  {
    const C tr = S2xx + S2yy;
    m[0] = wf * m[0] + rho * S0;
    m[1] = wf * m[1] + rho * (-2 * S0 + 3 * tr);
    m[2] = wf * m[2] + rho * (S0 - 3 * tr);
    m[3] = wf * m[3] + rho * S1x;
    m[4] = wf * m[4] - rho * S1x;
    m[5] = wf * m[5] + rho * S1y;
    m[6] = wf * m[6] - rho * S1y;
    m[7] = wf * m[7] + rho * (S2xx - S2yy);
    m[8] = wf * m[8] + rho * S2xy;
  }

  // ---- [df_s/dt] by eq. dfs_dt through the carrier h = 2 f_s + d:
  // d^{n+1} = 2 f_s^{n+1} - h^n,  h^{n+1} = 2 f_s^{n+1} + d^{n+1}
  const C dfs = 2 * fs - (C)hn;
  const H hnew = (H)(2 * fs + dfs);

  // ---- per-cell properties (Sec. 2.2) and relaxation rates (Sec. 3)
  const C cv = (C)P.cvf + (C)P.dcv * fs;
  const C lam = (C)P.lamf + (C)P.dlam * fs;
  const C tau_g = (C)0.5 + (C)P.taug_coef * lam;
  const C sig_j = (C)1 / tau_g;
  // (1/sig_j - 1/2)(1/sig_e - 1/2) = 1/4 is sig_e = 2 - sig_j
  const C sig_e = P.sigma_rule == 0 ? (C)2 - sig_j : (C)1;

  // ---- energy moments and the local temperature gradient (Sec. 2.2)
  const C b14 = g[1] + g[2] + g[3] + g[4];
  const C b58 = g[5] + g[6] + g[7] + g[8];
  C n[9];
  n[0] = g[0] + b14 + b58;
  n[1] = -4 * g[0] - b14 + 2 * b58;
  n[2] = 4 * g[0] - 2 * b14 + b58;
  n[3] = g[1] - g[3] + g[5] - g[6] - g[7] + g[8];
  n[4] = -2 * g[1] + 2 * g[3] + g[5] - g[6] - g[7] + g[8];
  n[5] = g[2] - g[4] + g[5] + g[6] - g[7] - g[8];
  n[6] = -2 * g[2] + 2 * g[4] + g[5] + g[6] - g[7] - g[8];
  n[7] = g[1] - g[2] + g[3] - g[4];
  n[8] = g[5] - g[6] + g[7] - g[8];
  const C gcoef = (C)(-3.0) * sig_j / (C)P.cref;   // -6/(4+alpha1) / (c_ref tau_g)
  const C gTx = gcoef * n[3], gTy = gcoef * n[5];

  // ---- coupled macroscopic solve: u from eq. rho.rhou with F = a + b T,
  // T from the implicit relation of Sec. 2.2 (linear in T)
  const C ax = wf * (C)P.A0x, ay = wf * (C)P.A0y;
  const C bx = wf * (C)P.B0x, by = wf * (C)P.B0y;
  const C irho = (C)1 / rho;
  const C jx = m[3], jy = m[5];
  const C num = n[0] - (C)0.5 * cv * ((jx + (C)0.5 * ax) * gTx + (jy + (C)0.5 * ay) * gTy) * irho;
  const C den = cv - (C)0.5 * (C)P.dcv * dfs + (C)0.25 * cv * (bx * gTx + by * gTy) * irho;
  const C Tc = num / den;
  const C Fx = ax + bx * Tc, Fy = ay + by * Tc;
  const C ux = (jx + (C)0.5 * Fx) * irho, uy = (jy + (C)0.5 * Fy) * irho;
  const C eps = cv * Tc;
  const C qc = -cv * (ux * gTx + uy * gTy) + (C)P.dcv * Tc * dfs;

  if (act && !(rho > (C)0 && isfinite(Tc) && isfinite(ux) && isfinite(uy)))
    atomicOr(flags, kFlagUnstable);

  // ---- flow collision with the discrete force term (eq. lbe.rho.col)
  {
    const C u2 = ux * ux + uy * uy;
    const C se = (C)P.s_e, sq = (C)P.s_q, sp = (C)P.s_p;
    const C Fu = Fx * ux + Fy * uy;
    C mb[9];
    mb[0] = rho;
    mb[1] = m[1] - se * (m[1] - (-2 * rho + 3 * rho * u2)) + ((C)1 - (C)0.5 * se) * (6 * Fu);
    mb[2] = m[2] - se * (m[2] - (rho - 3 * rho * u2)) + ((C)1 - (C)0.5 * se) * (-6 * Fu);
    mb[3] = rho * ux + (C)0.5 * Fx;
    mb[4] = m[4] - sq * (m[4] + rho * ux) + ((C)1 - (C)0.5 * sq) * (-Fx);
    mb[5] = rho * uy + (C)0.5 * Fy;
    mb[6] = m[6] - sq * (m[6] + rho * uy) + ((C)1 - (C)0.5 * sq) * (-Fy);
    mb[7] = m[7] - sp * (m[7] - rho * (ux * ux - uy * uy)) + ((C)1 - (C)0.5 * sp) * (2 * (Fx * ux - Fy * uy));
    mb[8] = m[8] - sp * (m[8] - rho * ux * uy) + ((C)1 - (C)0.5 * sp) * (Fx * uy + Fy * ux);
    // M^{-1} = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4)
    const C k0 = mb[0] / 9, k1 = mb[1] / 36, k2 = mb[2] / 36, k3 = mb[3] / 6,
            k4 = mb[4] / 12, k5 = mb[5] / 6, k6 = mb[6] / 12, k7 = mb[7] / 4,
            k8 = mb[8] / 4;
    C o[9];
    o[0] = k0 - 4 * k1 + 4 * k2;
    const C ax_ = k0 - k1 - 2 * k2;
    o[1] = ax_ + k3 - 2 * k4 + k7;
    o[2] = ax_ + k5 - 2 * k6 - k7;
    o[3] = ax_ - k3 + 2 * k4 + k7;
    o[4] = ax_ - k5 + 2 * k6 - k7;
    const C dg = k0 + 2 * k1 + k2;
    o[5] = dg + k3 + k4 + k5 + k6 + k8;
    o[6] = dg - k3 - k4 + k5 + k6 - k8;
    o[7] = dg - k3 - k4 - k5 - k6 + k8;
    o[8] = dg + k3 + k4 - k5 - k6 - k8;
    if (act) {
#pragma unroll
      for (int q = 0; q < 9; ++q)
        T::st(fout, (size_t)q * plane + cc, o[q], (C)P.fshift[q]);
    }
  }

  // ---- energy collision with the discrete source term (eq. lbe.e.col):
  // n^eq = [eps, -4 eps + 2 c_ref T, 4 eps - 3 c_ref T, 0...] (alpha1 = -2,
  // alpha2 = 1), q_m = [q, -4 q, 4 q, 0...] (beta1 = -4, beta2 = 4),
  // R = diag(1, se, se, sj, sj, sj, sj, se, se)
  {
    const C cT = (C)P.cref * Tc;
    C nb[9];
    nb[0] = eps + (C)0.5 * qc;
    nb[1] = n[1] - sig_e * (n[1] - (-4 * eps + 2 * cT)) + ((C)1 - (C)0.5 * sig_e) * (-4 * qc);
    nb[2] = n[2] - sig_e * (n[2] - (4 * eps - 3 * cT)) + ((C)1 - (C)0.5 * sig_e) * (4 * qc);
    const C rj = (C)1 - sig_j, re = (C)1 - sig_e;
    nb[3] = rj * n[3];
    nb[4] = rj * n[4];
    nb[5] = rj * n[5];
    nb[6] = rj * n[6];
    nb[7] = re * n[7];
    nb[8] = re * n[8];
    const C k0 = nb[0] / 9, k1 = nb[1] / 36, k2 = nb[2] / 36, k3 = nb[3] / 6,
            k4 = nb[4] / 12, k5 = nb[5] / 6, k6 = nb[6] / 12, k7 = nb[7] / 4,
            k8 = nb[8] / 4;
    C o[9];
    o[0] = k0 - 4 * k1 + 4 * k2;
    const C ax_ = k0 - k1 - 2 * k2;
    o[1] = ax_ + k3 - 2 * k4 + k7;
    o[2] = ax_ + k5 - 2 * k6 - k7;
    o[3] = ax_ - k3 + 2 * k4 + k7;
    o[4] = ax_ - k5 + 2 * k6 - k7;
    const C dg = k0 + 2 * k1 + k2;
    o[5] = dg + k3 + k4 + k5 + k6 + k8;
    o[6] = dg - k3 - k4 + k5 + k6 - k8;
    o[7] = dg - k3 - k4 - k5 - k6 + k8;
    o[8] = dg + k3 + k4 - k5 - k6 - k8;
    if (act) {
#pragma unroll
      for (int q = 0; q < 9; ++q)
        T::st(gout, (size_t)q * plane + cc, o[q], (C)P.gshift[q]);
      hcar[cc] = hnew;
    }
  }

  if (OUT && act) {
    const size_t N = (size_t)P.N;
    macro[cc] = (double)rho;
    macro[N + cc] = (double)ux;
    macro[2 * N + cc] = (double)uy;
    macro[3 * N + cc] = (double)Tc;
    macro[4 * N + cc] = (double)fs;
    macro[5 * N + cc] = (double)dfs;
  }
}

// -------------------------------------------------------------------------
// Initial state: equilibria of the mixed fluid/particle state per cell.

template <int PREC>
__global__ __launch_bounds__(kBlock) void k_init(
    const Params P, typename Prec<PREC>::S* __restrict__ fo,
    typename Prec<PREC>::S* __restrict__ go,
    typename Prec<PREC>::H* __restrict__ hcar, size_t plane, PState pn,
    PConst pc, Lists L, double* __restrict__ macro, int* flags) {
  typedef Prec<PREC> T;
  typedef typename T::C C;
  __shared__ BlockParticles bp;
  __shared__ int tmp[kListCap];
  load_block_list(bp, tmp, L, pn, pc, flags);
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
  const double rho = P.init_rho;
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
    T::st(fo, (size_t)q * plane + c, (C)feq, (C)P.fshift[q]);
    T::st(go, (size_t)q * plane + c, (C)geq, (C)P.gshift[q]);
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

// -------------------------------------------------------------------------
// Particle pass: one wave (64 lanes) per particle.

__device__ __forceinline__ int wave_excl_scan(int v, int lane) {
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  return incl - v;
}

// Actual row handled by lane r when the band rows [j0, j1] (unwrapped) are
// visited in ascending order of their index in the domain.
__device__ __forceinline__ int sorted_row(int r, int j0, int j1, int ny) {
  if (j1 >= ny) {  // rows 0..j1-ny, then j0..ny-1
    const int w = j1 - ny + 1;
    return r < w ? r : j0 + (r - w);
  }
  if (j0 < 0) {    // rows 0..j1, then j0+ny..ny-1
    return r <= j1 ? r : (j0 + ny) + (r - j1 - 1);
  }
  return j0 + r;
}

// Column segments of the band box in ascending order (two when the box
// wraps around a periodic x axis).
struct ColSegs {
  int n, lo[2], hi[2];
};

__device__ __forceinline__ ColSegs col_segments(int i0, int i1, int nx) {
  ColSegs cs;
  if (i0 < 0) {
    cs.n = 2; cs.lo[0] = 0; cs.hi[0] = i1; cs.lo[1] = i0 + nx; cs.hi[1] = nx - 1;
  } else if (i1 >= nx) {
    cs.n = 2; cs.lo[0] = 0; cs.hi[0] = i1 - nx; cs.lo[1] = i0; cs.hi[1] = nx - 1;
  } else {
    cs.n = 1; cs.lo[0] = i0; cs.hi[0] = i1; cs.lo[1] = 0; cs.hi[1] = -1;
  }
  return cs;
}

// Band box of a particle: cells [i0, i1] x [j0, j1] (unwrapped on periodic
// axes, clipped on walled ones).
__device__ __forceinline__ void band_box(const Params& P, double X, double Y,
                                         double R, int& i0, int& i1, int& j0,
                                         int& j1) {
  i0 = (int)floor(X - R) - 1;
  i1 = (int)floor(X + R) + 1;
  j0 = (int)floor(Y - R) - 1;
  j1 = (int)floor(Y + R) + 1;
  if (!P.perx) { i0 = max(i0, 0); i1 = min(i1, P.nx - 1); }
  if (!P.pery) { j0 = max(j0, 0); j1 = min(j1, P.ny - 1); }
}

// A particle centre the band-box logic can handle: finite, inside [0, L) on
// a periodic axis (positions are wrapped after every update) and within one
// domain length of a walled axis (boxes are clipped there).
__device__ __forceinline__ bool centre_ok(const Params& P, double X,
                                          double Y) {
  if (!isfinite(X) || !isfinite(Y)) return false;
  const double Lx = (double)P.nx, Ly = (double)P.ny;
  const bool okx = P.perx ? (X >= 0.0 && X < Lx) : (X >= -Lx && X <= 2.0 * Lx);
  const bool oky = P.pery ? (Y >= 0.0 && Y < Ly) : (Y >= -Ly && Y <= 2.0 * Ly);
  return okx && oky;
}

// The 256-cell blocks that row `row` of the band box touches, ascending, at
// most four.  Returns their number.
__device__ __forceinline__ int row_blocks(int row, const ColSegs& cs, int nx,
                                          int* b) {
  int n = 0;
  for (int k = 0; k < cs.n; ++k) {
    if (cs.hi[k] < cs.lo[k]) continue;
    const int first = (row * nx + cs.lo[k]) / kBlock;
    const int last = (row * nx + cs.hi[k]) / kBlock;
    for (int q = first; q <= last; ++q)
      if (n == 0 || b[n - 1] != q) b[n++] = q;
  }
  return n;
}

// Reduce the partials written by the previous lattice pass, update the
// particle (Newton-Euler, Sec. 2.3) and append it to the lists of the blocks
// its band box touches.  Modes: update, reduce only, bin only.
__global__ __launch_bounds__(256) void k_particles(
    const Params P, PState cur, PState next, PConst pc, Lists L,
    double* __restrict__ partial, int have_partials, int mode, int* flags) {
  const int lane = threadIdx.x & 63;
  const int p = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= P.np) return;  // whole wave

  double nX = cur.X[p], nY = cur.Y[p];
  if (mode != kModeBinOnly) {
    // ---- momentum-exchange force and torque: sum over the touched blocks
    double fx = 0.0, fy = 0.0, tz = 0.0;
    if (have_partials) {
      const int ns = cur.nslot[p];
      const double* src = partial + (size_t)p * P.maxb * kRedVals;
      for (int k = lane; k < ns; k += 64) {
        fx += src[k * kRedVals + 0];
        fy += src[k * kRedVals + 1];
        tz += src[k * kRedVals + 2];
      }
    }
    fx = wave_sum(fx);
    fy = wave_sum(fy);
    tz = wave_sum(tz);
    if (lane == 0) {
      cur.Fx[p] = fx;
      cur.Fy[p] = fy;
      cur.Tz[p] = tz;
    }
    if (mode == kModeReduceOnly) return;

    // ---- repulsion (short range, from the positions at step n)
    double cx = 0.0, cy = 0.0;
    const double zeta = P.coll_range;
    const double Xp = cur.X[p], Yp = cur.Y[p], Rp = pc.R[p];
    if (zeta > 0.0) {
      for (int q = lane; q < P.np; q += 64) {
        if (q == p) continue;
        const double dx = Xp - near_copy(cur.X[q], Xp, (double)P.nx, P.perx);
        const double dy = Yp - near_copy(cur.Y[q], Yp, (double)P.ny, P.pery);
        const double d = sqrt(dx * dx + dy * dy);
        const double reach = Rp + pc.R[q] + zeta;
        if (d < reach && d > 0.0) {
          const double s = (reach - d) / zeta;
          const double mag = P.coll_pp * s * s / d;
          cx += mag * dx;
          cy += mag * dy;
        }
      }
      cx = wave_sum(cx);
      cy = wave_sum(cy);
      if (lane == 0) {
        // walls: the particle's mirror image across each wall face
        const double dist[4] = {Xp, (double)P.nx - Xp, Yp, (double)P.ny - Yp};
        const double nrmx[4] = {1.0, -1.0, 0.0, 0.0};
        const double nrmy[4] = {0.0, 0.0, 1.0, -1.0};
        for (int w = 0; w < 4; ++w) {
          if (!P.wall_face[w]) continue;
          const double d = 2.0 * dist[w], reach = 2.0 * Rp + zeta;
          if (d < reach) {
            const double s = (reach - d) / zeta;
            cx += P.coll_pw * s * s * nrmx[w];
            cy += P.coll_pw * s * s * nrmy[w];
          }
        }
      }
    }

    // ---- Newton-Euler with the inside-fluid correction, forward Euler
    if (lane == 0) {
      const double R = Rp, rs = pc.rhos[p];
      const double V = M_PI * R * R;
      const double M = rs * V, I = 0.5 * M * R * R;
      const double Min = P.rho_f * M / rs, Iin = P.rho_f * I / rs;
      const double Ux = cur.Ux[p], Uy = cur.Uy[p], Om = cur.Om[p];
      double nUx = Ux, nUy = Uy, nOm = Om;
      if (!pc.fixed[p]) {
        const double Finx = -Min * (Ux - cur.Uxp[p]);
        const double Finy = -Min * (Uy - cur.Uyp[p]);
        const double Tin = -Iin * (Om - cur.Omp[p]);
        const double Fcx = (fx - Finx) + (rs - P.rho_f) * V * P.grav_x + cx;
        const double Fcy = (fy - Finy) + (rs - P.rho_f) * V * P.grav_y + cy;
        nUx = Ux + Fcx / M;
        nUy = Uy + Fcy / M;
        nOm = Om + (tz - Tin) / I;
      }
      nX = Xp + Ux;
      nY = Yp + Uy;
      if (P.perx) {
        if (nX >= (double)P.nx) nX -= (double)P.nx;
        if (nX < 0.0) nX += (double)P.nx;
      }
      if (P.pery) {
        if (nY >= (double)P.ny) nY -= (double)P.ny;
        if (nY < 0.0) nY += (double)P.ny;
      }
      next.X[p] = nX;
      next.Y[p] = nY;
      next.th[p] = cur.th[p] + Om;
      next.Ux[p] = nUx;
      next.Uy[p] = nUy;
      next.Om[p] = nOm;
      next.Uxp[p] = Ux;
      next.Uyp[p] = Uy;
      next.Omp[p] = Om;
      next.Fx[p] = fx;
      next.Fy[p] = fy;
      next.Tz[p] = tz;
    }
    nX = __shfl(nX, 0, 64);
    nY = __shfl(nY, 0, 64);
  }

  // ---- block lists for the band box at the new position
  const double R = pc.R[p];
  const bool ok = centre_ok(P, nX, nY);
  if (!ok && lane == 0) atomicOr(flags, kFlagUnstable);
  int i0 = 0, i1 = -1, j0 = 0, j1 = -1;
  if (ok) band_box(P, nX, nY, R, i0, i1, j0, j1);
  const int rows = j1 - j0 + 1;
  const ColSegs cs = col_segments(i0, i1, P.nx);
  int b[4];
  int nb = 0;
  if (lane < rows) {
    const int row = sorted_row(lane, j0, j1, P.ny);
    nb = row_blocks(row, cs, P.nx, b);
    if (lane > 0 && nb > 0) {
      int pb[4];
      const int prow = sorted_row(lane - 1, j0, j1, P.ny);
      const int pn = row_blocks(prow, cs, P.nx, pb);
      if (pn > 0 && pb[pn - 1] == b[0]) {   // shared with the previous row
        for (int k = 1; k < nb; ++k) b[k - 1] = b[k];
        --nb;
      }
    }
  }
  const int base = wave_excl_scan(nb, lane);
  const int total = __shfl(base + nb, 63, 64);
  for (int k = 0; k < nb; ++k) {
    const int slot = p * P.maxb + base + k;
    const int pos = atomicAdd(&L.cnt[b[k]], 1);
    if (pos < kListCap)
      L.ent[(size_t)b[k] * kListCap + pos] = make_int2(p, slot);
    else
      atomicOr(flags, kFlagListFull);
  }
  if (lane == 0) {
    PState& dst = (mode == kModeBinOnly) ? cur : next;
    dst.nslot[p] = total;
  }
}

// -------------------------------------------------------------------------
// Per-particle thermal sums over the band box, one block per particle, in a
// fixed order: sum f_s,p, sum f_s,p T, sum f_s,p c_vs T, min T over cells
// wholly inside (else over touched cells).

__global__ __launch_bounds__(256) void k_particle_sums(
    const Params P, PState ps, PConst pc, const double* __restrict__ macro,
    double* __restrict__ out4) {
  const int p = blockIdx.x;
  const double X0 = ps.X[p], Y0 = ps.Y[p], R = pc.R[p];
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
    const bool full = cell_within(X, Y, R, i, j);
    const double a = full ? 1.0 : covered_share(X, Y, R, i, j);
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

__global__ __launch_bounds__(kBlock) void k_ownership(
    const Params P, PState ps, PConst pc, Lists L, int* count, int* ids,
    int* full, int* flags) {
  __shared__ BlockParticles bp;
  __shared__ int tmp[kListCap];
  load_block_list(bp, tmp, L, ps, pc, flags);
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= P.N) return;
  const int y = c / P.nx, x = c - y * P.nx;
  int n = 0;
  for (int k = 0; k < P.kmax; ++k) {
    ids[(size_t)c * P.kmax + k] = -1;
    full[(size_t)c * P.kmax + k] = 0;
  }
  for (int s = 0; s < bp.cnt; ++s) {
    const double xn = x + 0.5, yn = y + 0.5;
    const double X = near_copy(bp.X[s], xn, (double)P.nx, P.perx);
    const double Y = near_copy(bp.Y[s], yn, (double)P.ny, P.pery);
    if (!owns_cell(X, Y, bp.R[s], x, y)) continue;
    if (n < P.kmax) {
      ids[(size_t)c * P.kmax + n] = bp.pid[s];
      full[(size_t)c * P.kmax + n] = cell_within(X, Y, bp.R[s], x, y) ? 1 : 0;
    }
    ++n;
  }
  if (n > P.kmax) atomicOr(flags, kFlagOverlap);
  count[c] = n < P.kmax ? n : P.kmax;
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
  out[k] = (double)T::ld(pop, (size_t)q * plane + c, (typename T::C)sh);
}

// -------------------------------------------------------------------------
// Launchers

static inline unsigned blocks_for(long n, int per) {
  return (unsigned)((n + per - 1) / per);
}

hipError_t launch_particles(const Params& P, PState cur, PState next,
                            PConst pc, Lists L, double* partial,
                            int have_partials, int mode, int* flags,
                            hipStream_t s) {
  if (P.np == 0) return hipSuccess;
  hipLaunchKernelGGL(k_particles, dim3(blocks_for(P.np, 4)), dim3(256), 0, s,
                     P, cur, next, pc, L, partial, have_partials, mode, flags);
  return hipGetLastError();
}

template <int PREC>
static hipError_t lattice_t(bool out, const Params& P, const void* fi,
                            void* fo, const void* gi, void* go, void* h,
                            size_t plane, PState pn, PConst pc, Lists L,
                            double* partial, double* macro, int* flags,
                            hipStream_t s) {
  typedef typename Prec<PREC>::S S;
  typedef typename Prec<PREC>::H H;
  if (out)
    hipLaunchKernelGGL((k_lattice<PREC, true>), dim3(P.nblocks), dim3(kBlock),
                       0, s, P, (const S*)fi, (S*)fo, (const S*)gi, (S*)go,
                       (H*)h, plane, pn, pc, L, partial, macro, flags);
  else
    hipLaunchKernelGGL((k_lattice<PREC, false>), dim3(P.nblocks), dim3(kBlock),
                       0, s, P, (const S*)fi, (S*)fo, (const S*)gi, (S*)go,
                       (H*)h, plane, pn, pc, L, partial, macro, flags);
  return hipGetLastError();
}

hipError_t launch_lattice(int prec, bool out, const Params& P,
                          const void* fi, void* fo, const void* gi, void* go,
                          void* h, size_t plane, PState pn, PConst pc,
                          Lists L, double* partial, double* macro, int* flags,
                          hipStream_t s) {
  switch (prec) {
    case VLB_FP64:
      return lattice_t<VLB_FP64>(out, P, fi, fo, gi, go, h, plane, pn, pc, L,
                                 partial, macro, flags, s);
    case VLB_FP32:
      return lattice_t<VLB_FP32>(out, P, fi, fo, gi, go, h, plane, pn, pc, L,
                                 partial, macro, flags, s);
    case VLB_FP16_SHIFT:
      return lattice_t<VLB_FP16_SHIFT>(out, P, fi, fo, gi, go, h, plane, pn,
                                       pc, L, partial, macro, flags, s);
    case VLB_BF16_SHIFT:
      return lattice_t<VLB_BF16_SHIFT>(out, P, fi, fo, gi, go, h, plane, pn,
                                       pc, L, partial, macro, flags, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_init(int prec, const Params& P, void* f, void* g, void* h,
                       size_t plane, PState pn, PConst pc, Lists L,
                       double* macro, int* flags, hipStream_t s) {
#define VLB_INIT(PR)                                                         \
  hipLaunchKernelGGL(k_init<PR>, dim3(P.nblocks), dim3(kBlock), 0, s, P,      \
                     (Prec<PR>::S*)f, (Prec<PR>::S*)g, (Prec<PR>::H*)h, plane, \
                     pn, pc, L, macro, flags);                                 \
  return hipGetLastError();
  switch (prec) {
    case VLB_FP64: VLB_INIT(VLB_FP64)
    case VLB_FP32: VLB_INIT(VLB_FP32)
    case VLB_FP16_SHIFT: VLB_INIT(VLB_FP16_SHIFT)
    case VLB_BF16_SHIFT: VLB_INIT(VLB_BF16_SHIFT)
  }
#undef VLB_INIT
  return hipErrorInvalidValue;
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
                            int* count, int* ids, int* full, int* flags,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_ownership, dim3(P.nblocks), dim3(kBlock), 0, s, P, ps,
                     pc, L, count, ids, full, flags);
  return hipGetLastError();
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
