// vlb_device.h -- device code shared by the kernels of the volumetric
// lattice Boltzmann step for thermal particulate flow with conjugate heat
// transfer (arXiv 2410.23802): storage forms, geometry, reductions, the
// particle helpers and the per-tile step (private to the library).
//
// Data layout in HBM (one domain):
//   populations  f, g : 9 planes each, plane stride `plane` >= N = nx*ny,
//                       cell c = j*nx + i (x fastest); two copies (A/B),
//                       pull streaming reads A and writes B.
//   h                 : 1 value per cell, the carrier h = 2 f_s + [df_s/dt]
//                       of the eq. dfs_dt recursion, two copies.
//   macro             : rho, ux, uy, T, f_s, [df_s/dt] as FP64 planes,
//                       written only by the last step of a vlb_step call.
//   partials          : FP64 shares of the momentum-exchange force and
//                       torque, one slot per (particle, 256-cell tile).
//
// A step is one launch over all tiles in two roles (see step_task): the
// tiles particles reach run the volumetric step and the momentum exchange,
// the others a plain update.  The particles are handled in one of two forms:
//   scan (few particles): each particle tile finds the particles whose band
//     box reaches it at the new position X + U (forward Euler needs no force
//     for the position) and rebuilds their new velocities itself from the
//     previous step's partials -- the same inputs in the same order in every
//     tile, hence the same bits; the first tile a particle reaches stores its
//     new state.  Partials [particle][tile].
//   list (many particles): k_particles first updates every particle (one
//     wave each) and fills per-tile particle lists.  Partials [particle][k-th
//     tile reached].
// No floating-point atomics anywhere: every sum runs in a fixed order, so a
// run is bitwise reproducible.
#pragma once

#include <math.h>

#include <hip/hip_ext.h>

#include "vlb_internal.h"

namespace vlb {

// -------------------------------------------------------------------------
// Storage forms.  Populations are stored as deviations from a fixed
// per-direction reference (f_i - w_i rho_0, g_i - w_i c_ref T_0) and the
// kernel computes on deviations, so the low-Mach momentum is never formed
// by cancelling O(1) numbers.  FP64 uses a zero reference (literal values);
// FP16/BF16 compute in FP32 and keep the [df_s/dt] carrier in FP32.

template <int PREC>
struct Prec;

template <>
struct Prec<VLB_FP64> {
  typedef double S;
  typedef double C;
  typedef double H;
  static __device__ __forceinline__ C cv(S v) { return v; }
  static __device__ __forceinline__ C ld(const S* p, size_t i) { return p[i]; }
  static __device__ __forceinline__ void st(S* p, size_t i, C v) { p[i] = v; }
  static __device__ __forceinline__ void stn(S* p, size_t i, C v) {
    __builtin_nontemporal_store(v, p + i);
  }
};

template <>
struct Prec<VLB_FP32> {
  typedef float S;
  typedef float C;
  typedef float H;
  static __device__ __forceinline__ C cv(S v) { return v; }
  static __device__ __forceinline__ C ld(const S* p, size_t i) { return p[i]; }
  static __device__ __forceinline__ void st(S* p, size_t i, C v) { p[i] = v; }
  static __device__ __forceinline__ void stn(S* p, size_t i, C v) {
    __builtin_nontemporal_store(v, p + i);
  }
};

template <>
struct Prec<VLB_FP16_SHIFT> {
  typedef _Float16 S;
  typedef float C;
  typedef float H;
  static __device__ __forceinline__ C cv(S v) { return (float)v; }
  static __device__ __forceinline__ C ld(const S* p, size_t i) {
    return (float)p[i];
  }
  static __device__ __forceinline__ void st(S* p, size_t i, C v) {
    p[i] = (_Float16)v;
  }
  static __device__ __forceinline__ void stn(S* p, size_t i, C v) {
    __builtin_nontemporal_store((_Float16)v, p + i);
  }
};

template <>
struct Prec<VLB_BF16_SHIFT> {
  typedef uint16_t S;
  typedef float C;
  typedef float H;
  static __device__ __forceinline__ C cv(S v) {
    return __uint_as_float(((uint32_t)v) << 16);
  }
  static __device__ __forceinline__ C ld(const S* p, size_t i) {
    return cv(p[i]);
  }
  // round to nearest even on the upper 16 bits (gfx950 converts in one
  // instruction, the same bits for every finite value)
  static __device__ __forceinline__ S rne(C v) {
    return __builtin_bit_cast(uint16_t, (__bf16)v);
  }
  static __device__ __forceinline__ void st(S* p, size_t i, C v) {
    p[i] = rne(v);
  }
  static __device__ __forceinline__ void stn(S* p, size_t i, C v) {
    __builtin_nontemporal_store(rne(v), p + i);
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
// decision is the same on every IEEE machine.  The _in forms are inlined
// (the step kernel of one domain, list form); the out-of-line ones keep the
// register count of the other callers down.  Both do the same operations.
__device__ __forceinline__ bool owns_cell_in(double X, double Y, double R,
                                             int i, int j) {
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
__device__ __forceinline__ bool cell_within_in(double X, double Y, double R,
                                               int i, int j) {
#pragma clang fp contract(off)
  double ex = (X < (double)i + 0.5) ? (double)(i + 1) - X : X - (double)i;
  double ey = (Y < (double)j + 0.5) ? (double)(j + 1) - Y : Y - (double)j;
  double q = ex * ex;
  q = q + ey * ey;
  return q <= R * R;
}

__device__ __noinline__ bool owns_cell(double X, double Y, double R, int i,
                                       int j) {
  return owns_cell_in(X, Y, R, i, j);
}

__device__ __noinline__ bool cell_within(double X, double Y, double R, int i,
                                         int j) {
  return cell_within_in(X, Y, R, i, j);
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

// The same area as tri_disk_area, in two parts: the triangle part is added
// to `tri`, and each circular sector, of angle arg(conj(u) v) between the
// vectors u and v that bound it, is multiplied into the complex number
// (zr, zi) as u.v + i u x v -- the angles add as the factors multiply.
// The product is rescaled by a power of two after each factor (exactly),
// and vanishing factors (a degenerate sector) are left out.
__device__ __forceinline__ void sector_factor(double ux, double uy, double vx,
                                              double vy, double& zr,
                                              double& zi) {
  const double cr = ux * vx + uy * vy, ci = ux * vy - uy * vx;
  if (cr == 0.0 && ci == 0.0) return;
  const double r = zr * cr - zi * ci, im = zr * ci + zi * cr;
  int e;
  (void)frexp(fmax(fabs(r), fabs(im)), &e);
  zr = ldexp(r, -e);
  zi = ldexp(im, -e);
}

__device__ __forceinline__ void tri_disk_parts(double px, double py,
                                               double qx, double qy, double R,
                                               double& tri, double& zr,
                                               double& zi) {
  const double dx = qx - px, dy = qy - py;
  const double a = dx * dx + dy * dy;
  const double b = px * dx + py * dy;
  const double c = (px * px + py * py) - R * R;
  const double disc = b * b - a * c;
  double s1 = 1.0, s2 = 0.0;
  if (disc > 0.0) {
    const double r = sqrt(disc);
    s1 = fmin(fmax((-b - r) / a, 0.0), 1.0);
    s2 = fmin(fmax((-b + r) / a, 0.0), 1.0);
  }
  if (!(s1 < s2)) {
    sector_factor(px, py, qx, qy, zr, zi);
    return;
  }
  const double ax = px + s1 * dx, ay = py + s1 * dy;
  const double bx = px + s2 * dx, by = py + s2 * dy;
  tri += 0.5 * (ax * by - ay * bx);
  if (s1 > 0.0) sector_factor(px, py, ax, ay, zr, zi);
  if (s2 < 1.0) sector_factor(bx, by, qx, qy, zr, zi);
}

// Area of the disk of radius R centred at the origin intersected with the
// convex quadrilateral (u[k], v[k]), k = 0..3 counter-clockwise, by Green's
// theorem over its edges: triangles from the centre to the parts of the
// edges inside the circle, circular sectors for the parts outside.  When
// the centre lies outside the closed quadrilateral the latter subtends less
// than pi from it, so the sectors' net angle is in (-pi, pi) and one atan2
// of the product of their complex factors gives it; otherwise (a disk
// narrower than the cell) each sector is evaluated on its own.
__device__ __forceinline__ double quad_disk_area(const double* u,
                                                 const double* v, double R) {
  bool inside = true;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int n = (k + 1) & 3;
    inside = inside && (u[n] - u[k]) * -v[k] - (v[n] - v[k]) * -u[k] >= 0.0;
  }
  if (inside) {
    double A = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      A += tri_disk_area(u[k], v[k], u[(k + 1) & 3], v[(k + 1) & 3], R);
    return A;
  }
  double tri = 0.0, zr = 1.0, zi = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    tri_disk_parts(u[k], v[k], u[(k + 1) & 3], v[(k + 1) & 3], R, tri, zr, zi);
  return tri + 0.5 * R * R * atan2(zi, zr);
}

// The area of the disk of radius^2 r2 centred at the origin inside the
// unit square [x0, x0 + 1] x [y0, y0 + 1] (coordinates relative to the
// centre), by Green's theorem over the square's edges counter-clockwise.
// An edge runs from p along a unit axis d (b = p.d, hh = h^2 = |p|^2 -
// b^2, cr = p x d, pp = |p|^2), so the circle meets it at
// s = -b +- sqrt(r2 - hh), with no division.  A sector of angle
// arg(conj(u) v) enters as the complex factor u.v + i u x v, multiplied
// into one product whose atan2 gives the net angle when the centre lies
// outside the closed square (it is then in (-pi, pi)); in the square that
// holds the centre each sector takes its own atan2.
struct SqAcc {
  double tri, zr, zi, ang;
};

__device__ __forceinline__ void sq_sector(double cr, double ci, bool own,
                                          SqAcc& a) {
  if (cr == 0.0 && ci == 0.0) return;
  if (own) {
    a.ang += atan2(ci, cr);
    return;
  }
  const double r = a.zr * cr - a.zi * ci, im = a.zr * ci + a.zi * cr;
  a.zr = r;
  a.zi = im;
}

__device__ __forceinline__ void sq_edge(double b, double hh, double cr,
                                        double pp, double r2, bool own,
                                        SqAcc& a) {
  const double disc = r2 - hh;
  double s1 = 1.0, s2 = 0.0;
  if (disc > 0.0) {
    const double w = sqrt(disc);
    s1 = fmin(fmax(-b - w, 0.0), 1.0);
    s2 = fmin(fmax(-b + w, 0.0), 1.0);
  }
  if (!(s1 < s2)) {              // the whole edge outside: p -> p + d
    sq_sector(pp + b, cr, own, a);
    return;
  }
  a.tri += 0.5 * (s2 - s1) * cr;
  if (s1 > 0.0) sq_sector(pp + s1 * b, s1 * cr, own, a);
  if (s2 < 1.0) sq_sector(pp + (1.0 + s2) * b + s2, (1.0 - s2) * cr, own, a);
}

// Exact share of cell (i, j) covered by the disk (centre X, Y, radius R).
__device__ double covered_share(double X, double Y, double R, int i, int j) {
  const double x0 = (double)i - X, y0 = (double)j - Y;
  const double x1 = x0 + 1.0, y1 = y0 + 1.0, r2 = R * R;
  const bool own = x0 <= 0.0 && x1 >= 0.0 && y0 <= 0.0 && y1 >= 0.0;
  const double xx0 = x0 * x0, xx1 = x1 * x1, yy0 = y0 * y0, yy1 = y1 * y1;
  SqAcc a = {0.0, 1.0, 0.0, 0.0};
  sq_edge(x0, yy0, -y0, xx0 + yy0, r2, own, a);     // bottom, +x
  sq_edge(y0, xx1, x1, xx1 + yy0, r2, own, a);      // right, +y
  sq_edge(-x1, yy1, y1, xx1 + yy1, r2, own, a);     // top, -x
  sq_edge(-y1, xx0, -x0, xx0 + yy1, r2, own, a);    // left, -y
  const double ang = own ? a.ang : atan2(a.zi, a.zr);
  return fmin(fmax(a.tri + 0.5 * r2 * ang, 0.0), 1.0);
}

// Exact share of cell (i, j) covered by the ellipse of semi-axes a (the
// major one, along (c, s) = (cos theta, sin theta)) and b centred at
// (X, Y) (Sec. 3.2).  The map x -> ((c, s).x / a, (-s, c).x / b) takes the
// ellipse to the unit disk and the cell to a parallelogram, still
// counter-clockwise (the map's determinant is 1/(a b) > 0), whose
// intersection with the unit disk is quad_disk_area's; areas scale by a b.
__device__ __forceinline__ double ellipse_share(double X, double Y, double a,
                                                double b, double c, double s,
                                                int i, int j) {
  const double x0 = (double)i - X, x1 = (double)(i + 1) - X;
  const double y0 = (double)j - Y, y1 = (double)(j + 1) - Y;
  const double cx[4] = {x0, x1, x1, x0}, cy[4] = {y0, y0, y1, y1};
  const double ia = 1.0 / a, ib = 1.0 / b;
  double u[4], v[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    u[k] = (c * cx[k] + s * cy[k]) * ia;
    v[k] = (c * cy[k] - s * cx[k]) * ib;
  }
  return fmin(fmax(a * b * quad_disk_area(u, v, 1.0), 0.0), 1.0);
}

// The share of cell (i, j) covered by a particle: a disk of radius R when
// Rb == R, else the ellipse of semi-axes R and Rb at the angle whose cosine
// and sine are (c, s).  ELL = false (no ellipse in the domain): the disk
// only, so that the kernels of disk domains carry none of the ellipse's
// code or registers (the step kernel of the 32-bit forms otherwise spills).
template <bool ELL>
__device__ __forceinline__ double shape_share(double X, double Y, double R,
                                              double Rb, double c, double s,
                                              int i, int j) {
  if constexpr (ELL) {
    if (Rb != R) return ellipse_share(X, Y, R, Rb, c, s, i, j);
  }
  return covered_share(X, Y, R, i, j);
}

// cos and sin of a particle's orientation (unused for a disk).
__device__ __forceinline__ void orientation(double R, double Rb, double th,
                                            double& c, double& s) {
  if (Rb == R) {
    c = 1.0;
    s = 0.0;
  } else {
    sincos(th, &s, &c);
  }
}

// -------------------------------------------------------------------------
// Reductions (fixed order: a tree inside a wave, waves in index order).

// The value of the lane that DPP control CTRL pairs with this one (the
// quad permutations and row mirrors used here are involutions, so partners
// exchange values).
template <int CTRL>
__device__ __forceinline__ double dpp_partner(double v) {
  return __builtin_amdgcn_update_dpp(0.0, v, CTRL, 0xF, 0xF, false);
}

// Lane `lane`'s value, uniform.
__device__ __forceinline__ double lane_value(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over the wave's 64 lanes (all active), the same bits in every lane:
// inside each row of 16 lanes, partners add (lane ^ 1, lane ^ 2, the
// mirror in 8, the mirror in 16; a + b and b + a are the same bits), then
// the four row sums are added in a fixed order.  DPP moves instead of
// LDS permutes: a few cycles per step instead of an LDS round trip.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_partner<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_partner<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_partner<0x141>(v);   // row_half_mirror
  v += dpp_partner<0x140>(v);   // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) +
         (lane_value(v, 32) + lane_value(v, 48));
}

// The same sum, complete in lane 63 only (the other lanes hold partial
// sums): after the row sums, row_bcast:15 adds row r - 1's into rows 1 and
// 3, then row_bcast:31 adds row 1's into row 3, so lane 63 holds
// (r3 + r2) + (r1 + r0) -- wave_sum's bits, as a + b and b + a are the
// same -- with two DPP steps in place of eight lane reads.
__device__ __forceinline__ double wave_sum_last(double v) {
  v += dpp_partner<0xB1>(v);
  v += dpp_partner<0x4E>(v);
  v += dpp_partner<0x141>(v);
  v += dpp_partner<0x140>(v);
  v += __builtin_amdgcn_update_dpp(0.0, v, 0x142, 0xA, 0xF, false);
  v += __builtin_amdgcn_update_dpp(0.0, v, 0x143, 0xC, 0xF, false);
  return v;
}

__device__ __forceinline__ double wave_min(double v) {
  v = fmin(v, dpp_partner<0xB1>(v));
  v = fmin(v, dpp_partner<0x4E>(v));
  v = fmin(v, dpp_partner<0x141>(v));
  v = fmin(v, dpp_partner<0x140>(v));
  return fmin(fmin(lane_value(v, 0), lane_value(v, 16)),
              fmin(lane_value(v, 32), lane_value(v, 48)));
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
// Band boxes and block bookkeeping.

// Exclusive prefix sum of v over the wave's lanes in lane order (all lanes
// active), and the wave's total.  Values below 2^BITS are summed one bit
// plane at a time from ballots (no LDS traffic); a wave holding a larger
// value takes the shuffle scan.
template <int BITS>
__device__ __forceinline__ int wave_excl_scan(int v, int lane, int& total) {
  const unsigned long long below = (1ull << lane) - 1ull;
  if (__ballot(v >= (1 << BITS)) == 0ull) {
    int s = 0, all = 0;
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const unsigned long long m = __ballot((v >> b) & 1);
      s += __popcll(m & below) << b;
      all += __popcll(m) << b;
    }
    total = all;
    return s;
  }
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  total = __shfl(incl, 63, 64);
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

// The 256-cell blocks that row `row` of the band box touches, ascending and
// without repeats: the ranges [f0, l0] and [f1, l1] (empty when l < f), one
// per column segment; the second starts past the first's last block.
// Scalars rather than an indexed array, which the compiler would otherwise
// place in LDS behind a read of the dispatch packet.
__device__ __forceinline__ void row_block_ranges(int row, const ColSegs& cs,
                                                 int nx, int& f0, int& l0,
                                                 int& f1, int& l1) {
  f0 = 0; l0 = -1; f1 = 0; l1 = -1;
  if (cs.hi[0] >= cs.lo[0]) {
    f0 = (row * nx + cs.lo[0]) / kBlock;
    l0 = (row * nx + cs.hi[0]) / kBlock;
  }
  if (cs.n > 1 && cs.hi[1] >= cs.lo[1]) {
    f1 = (row * nx + cs.lo[1]) / kBlock;
    l1 = (row * nx + cs.hi[1]) / kBlock;
    if (l0 >= f0 && f1 == l0) ++f1;   // the block the first range ends in
  }
}


// -------------------------------------------------------------------------
// Particle helpers shared by both forms.

// Forward Euler of the position (Sec. 2.3): X^{n+1} = X^n + U^n, wrapped
// into [0, L) on periodic axes.
__device__ __forceinline__ void advance_position(const Params& P, double& X,
                                                 double& Y, double Ux,
                                                 double Uy) {
  X = X + Ux;
  Y = Y + Uy;
  if (P.perx) {
    if (X >= (double)P.nx) X -= (double)P.nx;
    if (X < 0.0) X += (double)P.nx;
  }
  if (P.pery) {
    if (Y >= (double)P.ny) Y -= (double)P.ny;
    if (Y < 0.0) Y += (double)P.ny;
  }
}

// The units of `unit` consecutive cells (64: a wave, 256: a block) a
// particle's band box reaches: at most two ascending, disjoint ranges (two
// when the box wraps around a periodic y axis).  Every cell of the box lies
// in a listed unit.
struct BlockRanges {
  int n;
  int lo[2], hi[2];
  __device__ __forceinline__ int count() const {
    return n == 0 ? 0
                  : (hi[0] - lo[0] + 1) + (n > 1 ? hi[1] - lo[1] + 1 : 0);
  }
  __device__ __forceinline__ int at(int k) const {
    const int l0 = hi[0] - lo[0] + 1;
    return k < l0 ? lo[0] + k : lo[1] + (k - l0);
  }
  __device__ __forceinline__ bool contains(int b) const {
    return (n > 0 && b >= lo[0] && b <= hi[0]) ||
           (n > 1 && b >= lo[1] && b <= hi[1]);
  }
};

__device__ BlockRanges block_ranges(const Params& P, double X, double Y,
                                    double R, int unit) {
  BlockRanges r;
  r.n = 0;
  r.lo[0] = r.lo[1] = 0;
  r.hi[0] = r.hi[1] = -1;
  if (!centre_ok(P, X, Y)) return r;
  int i0, i1, j0, j1;
  band_box(P, X, Y, R, i0, i1, j0, j1);
  if (i1 < i0 || j1 < j0) return r;
  // row spans: [a0, a1], and [b0, b1] when the box wraps around y
  int a0 = j0, a1 = j1, b0 = 0, b1 = -1, na = 1;
  if (P.pery && j0 < 0) {          // rows 0..j1 and j0+ny..ny-1
    na = 2; a0 = 0; a1 = j1; b0 = j0 + P.ny; b1 = P.ny - 1;
  } else if (P.pery && j1 >= P.ny) {  // rows 0..j1-ny and j0..ny-1
    na = 2; a0 = 0; a1 = j1 - P.ny; b0 = j0; b1 = P.ny - 1;
  }
  const bool xfull = P.perx && (i0 < 0 || i1 >= P.nx);
  const int ca = xfull ? 0 : i0, cb = xfull ? P.nx - 1 : i1;
  r.lo[0] = (a0 * P.nx + ca) / unit;
  r.hi[0] = (a1 * P.nx + cb) / unit;
  if (na == 2) {
    r.lo[1] = (b0 * P.nx + ca) / unit;
    r.hi[1] = (b1 * P.nx + cb) / unit;
  }
  r.n = na;
  if (na == 2 && r.hi[0] >= r.lo[1]) {  // the two ranges touch: merge
    r.hi[0] = max(r.hi[0], r.hi[1]);
    r.n = 1;
  }
  return r;
}

// Momentum-exchange force and torque of particle p: the sum of the partials
// the last lattice pass wrote, lanes striding the slots, then wave_sum
// (every lane ends with the same bits).  Scan form, with the particle's
// centre (X, Y) at the step the partials belong to and its radius R: one
// slot per (particle, 256-cell tile) of its band box.
__device__ __forceinline__ void reduce_partials_at(const Params& P, double X,
                                                   double Y, double R,
                                                   const double* partial,
                                                   int have, int p, int lane,
                                                   double& fx, double& fy,
                                                   double& tz) {
  fx = fy = tz = 0.0;
  if (have) {
    const BlockRanges r = block_ranges(P, X, Y, R, kBlock);
    const int nb = r.count();
    const double* src = partial + (size_t)p * P.nblocks * kRedVals;
    for (int k = lane; k < nb; k += 64) {
      const double* o = src + (size_t)r.at(k) * kRedVals;
      fx += o[0];
      fy += o[1];
      tz += o[2];
    }
  }
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  tz = wave_sum(tz);
}

// The same sums from the stored state: scan form as above; list form, the
// particle's nslot slots in order.
__device__ __forceinline__ void reduce_partials(const Params& P,
                                                const PState& cur,
                                                const PConst& pc,
                                                const double* partial,
                                                int have, int p, int lane,
                                                double& fx, double& fy,
                                                double& tz) {
  if (P.scan) {
    reduce_partials_at(P, cur.X[p], cur.Y[p], pc.R[p], partial, have, p,
                       lane, fx, fy, tz);
    return;
  }
  fx = fy = tz = 0.0;
  if (have) {
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
}

// Repulsion on particle p (the collision model the paper adopts): a
// short-range force of range zeta, k ((R_p + R_q + zeta - d)/zeta)^2 along
// the centre line, and against each wall the same law applied to the
// particle's mirror image.  Positions of step n.  Every lane returns the
// same bits.
__device__ __forceinline__ void repulsion_pair(const Params& P, double Xp,
                                               double Yp, double Rp,
                                               double Xq, double Yq,
                                               double Rq, double& cx,
                                               double& cy) {
  const double zeta = P.coll_range;
  const double dx = Xp - near_copy(Xq, Xp, (double)P.nx, P.perx);
  const double dy = Yp - near_copy(Yq, Yp, (double)P.ny, P.pery);
  const double d = sqrt(dx * dx + dy * dy);
  const double reach = Rp + Rq + zeta;
  if (d < reach && d > 0.0) {
    const double s = (reach - d) / zeta;
    const double mag = P.coll_pp * s * s / d;
    cx += mag * dx;
    cy += mag * dy;
  }
}

// The walls' part of the repulsion on a particle at (Xp, Yp), added to the
// wave-summed pair part.
__device__ __forceinline__ void repulsion_walls(const Params& P, double Xp,
                                                double Yp, double Rp,
                                                double& cx, double& cy) {
  const double zeta = P.coll_range;
  const double dist[4] = {Xp, (double)P.nx - Xp, Yp, (double)P.ny - Yp};
  const double nrmx[4] = {1.0, -1.0, 0.0, 0.0};
  const double nrmy[4] = {0.0, 0.0, 1.0, -1.0};
#pragma unroll
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

// The repulsion on particle p (centre Xp, Yp, radius Rp) for at most 64
// particles, lane q holding particle q (Xq, Yq, Rq; `other`: q < np and
// q != p): the pairs lane by lane, wave_sum, then the walls.
__device__ __forceinline__ void repulsion_lanes(const Params& P, double Xp,
                                                double Yp, double Rp,
                                                double Xq, double Yq,
                                                double Rq, bool other,
                                                double& cx, double& cy) {
  cx = cy = 0.0;
  if (!(P.coll_range > 0.0)) return;
  if (other) repulsion_pair(P, Xp, Yp, Rp, Xq, Yq, Rq, cx, cy);
  cx = wave_sum(cx);
  cy = wave_sum(cy);
  repulsion_walls(P, Xp, Yp, Rp, cx, cy);
}

struct PUpd {
  double X, Y, th, Ux, Uy, Om, Uxp, Uyp, Omp, Fx, Fy, Tz;
};

// One particle's stored state and constants, in registers.
struct POne {
  double X, Y, th, Ux, Uy, Om, Uxp, Uyp, Omp, R, rhos, Tinit, Rb;
  int fixed;
};

__device__ __forceinline__ POne load_one(const PState& s, const PConst& pc,
                                         int p) {
  POne o;
  o.X = s.X[p]; o.Y = s.Y[p]; o.th = s.th[p];
  o.Ux = s.Ux[p]; o.Uy = s.Uy[p]; o.Om = s.Om[p];
  o.Uxp = s.Uxp[p]; o.Uyp = s.Uyp[p]; o.Omp = s.Omp[p];
  o.R = pc.R[p]; o.rhos = pc.rhos[p]; o.Tinit = pc.Tinit[p];
  o.Rb = pc.Rb[p];
  o.fixed = pc.fixed[p];
  return o;
}

// Lane src's POne, in every lane (src uniform).
__device__ __forceinline__ POne lane_one(const POne& v, int src) {
  POne o;
  o.X = lane_value(v.X, src); o.Y = lane_value(v.Y, src);
  o.th = lane_value(v.th, src);
  o.Ux = lane_value(v.Ux, src); o.Uy = lane_value(v.Uy, src);
  o.Om = lane_value(v.Om, src);
  o.Uxp = lane_value(v.Uxp, src); o.Uyp = lane_value(v.Uyp, src);
  o.Omp = lane_value(v.Omp, src);
  o.R = lane_value(v.R, src); o.rhos = lane_value(v.rhos, src);
  o.Tinit = lane_value(v.Tinit, src);
  o.Rb = lane_value(v.Rb, src);
  o.fixed = __builtin_amdgcn_readlane(v.fixed, src);
  return o;
}

// One step of a particle (state s), wave-level (every lane returns the same
// bits): Newton-Euler (eq. particle; the gyroscopic term vanishes in 2-D)
// with the inside-fluid correction of eq. inside.fluid by backward
// differences, total force = hydrodynamic + (rho_s - rho_f) V g +
// repulsion, forward Euler (Sec. 2.3 end).  The momentum-exchange sums
// (fx, fy, tz) and the repulsion (cx, cy) are given.
__device__ PUpd particle_update_one(const Params& P, const POne& s,
                                    double fx, double fy, double tz,
                                    double cx, double cy) {
  PUpd u;
  const double R = s.R, rs = s.rhos;
  // a disk (Rb == R): V = pi R^2, I = M R^2 / 2; an ellipse of semi-axes
  // R and Rb (Sec. 3.2): V = pi R Rb, I = M (R^2 + Rb^2) / 4
  const double V = M_PI * R * s.Rb;
  const double M = rs * V;
  const double I = s.Rb == R ? 0.5 * M * R * R
                             : 0.25 * M * (R * R + s.Rb * s.Rb);
  const double Min = P.rho_f * M / rs, Iin = P.rho_f * I / rs;
  const double Ux = s.Ux, Uy = s.Uy, Om = s.Om;
  u.Ux = Ux;
  u.Uy = Uy;
  u.Om = Om;
  if (!(s.fixed & 1)) {
    const double Finx = -Min * (Ux - s.Uxp);
    const double Finy = -Min * (Uy - s.Uyp);
    const double Tin = -Iin * (Om - s.Omp);
    // gravity: (rho_s - rho_f) V g, or rho_s V g when the fluid carries
    // its own weight (situation II of Sec. 3.2)
    const double rg = P.fluid_gravity ? rs : rs - P.rho_f;
    const double Fcx = (fx - Finx) + rg * V * P.grav_x + cx;
    const double Fcy = (fy - Finy) + rg * V * P.grav_y + cy;
    u.Ux = Ux + Fcx / M;
    u.Uy = Uy + Fcy / M;
    u.Om = Om + (tz - Tin) / I;
  }
  u.X = s.X;
  u.Y = s.Y;
  advance_position(P, u.X, u.Y, Ux, Uy);
  u.th = s.th + Om;
  u.Uxp = Ux;
  u.Uyp = Uy;
  u.Omp = Om;
  u.Fx = fx;
  u.Fy = fy;
  u.Tz = tz;
  return u;
}

// The same from the stored state of particle p.
__device__ __forceinline__ PUpd particle_update_sums(
    const Params& P, const PState& cur, const PConst& pc, int p, double fx,
    double fy, double tz, double cx, double cy) {
  return particle_update_one(P, load_one(cur, pc, p), fx, fy, tz, cx, cy);
}

__device__ __forceinline__ void store_particle(PState& s, int p,
                                               const PUpd& u) {
  s.X[p] = u.X; s.Y[p] = u.Y; s.th[p] = u.th;
  s.Ux[p] = u.Ux; s.Uy[p] = u.Uy; s.Om[p] = u.Om;
  s.Uxp[p] = u.Uxp; s.Uyp[p] = u.Uyp; s.Omp[p] = u.Omp;
  s.Fx[p] = u.Fx; s.Fy[p] = u.Fy; s.Tz[p] = u.Tz;
}

// -------------------------------------------------------------------------
// Block particle list: load, sort by particle id and stage the particle
// data in LDS.

struct BlockParticles {
  int cnt;
  int nheld;            // of them, particles whose temperature is held
  int pid[kListCap];
  int slot[kListCap];
  int held[kListCap];   // 1: the particle's temperature is held (at Tp)
  double X[kListCap], Y[kListCap], R[kListCap];
  double Ux[kListCap], Uy[kListCap], Om[kListCap], Tp[kListCap];
  // the shape: minor semi-axis (R for a disk) and the orientation's cosine
  // and sine (1, 0 for a disk)
  double Rb[kListCap], cth[kListCap], sth[kListCap];
};

__device__ __forceinline__ void load_block_list(BlockParticles& bp, int* tmp,
                                                Lists L, int b, PState pn,
                                                PConst pc, int* flags) {
  const int t = threadIdx.x;
  if (t == 0) {
    int n = L.cnt[b];
    if (n > kListCap) {
      atomicOr(flags, kFlagListFull);
      n = kListCap;
    }
    bp.cnt = n;
    bp.nheld = 0;
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
    bp.Rb[rank] = pc.Rb[e.x];
    orientation(bp.R[rank], bp.Rb[rank], pn.th[e.x], bp.cth[rank],
                bp.sth[rank]);
    bp.held[rank] = (pc.fixed[e.x] >> 1) & 1;
    if (bp.held[rank]) atomicAdd(&bp.nheld, 1);
  }
  __syncthreads();
}

// Whether the list form's step kernel reads each tile's list entries with
// its count, before the count is known (load_block_list_known): measured on
// the dense cavity, FP32 92.6 -> 90.9 us per step, FP64 156.9 -> 159.6 us.
template <int PREC>
constexpr bool kListEntryAhead = PREC != VLB_FP64;

// The same for the step kernel, which has already read the tile's count
// (cnt, uniform) and, with it, entry t of the list (e, read before the
// count was known; only threads t < cnt use theirs): one barrier and one
// round trip to memory fewer than load_block_list.
__device__ __forceinline__ void load_block_list_known(BlockParticles& bp,
                                                      int* tmp, int cnt,
                                                      int2 e, PState pn,
                                                      PConst pc, int* flags) {
  const int t = threadIdx.x;
  const int n = cnt < kListCap ? cnt : kListCap;
  if (t == 0) {
    if (cnt > kListCap) atomicOr(flags, kFlagListFull);
    bp.cnt = n;
    bp.nheld = 0;
  }
  if (t < n) tmp[t] = e.x;
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
    bp.Rb[rank] = pc.Rb[e.x];
    orientation(bp.R[rank], bp.Rb[rank], pn.th[e.x], bp.cth[rank],
                bp.sth[rank]);
    bp.held[rank] = (pc.fixed[e.x] >> 1) & 1;
    if (bp.held[rank]) atomicAdd(&bp.nheld, 1);
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
  double R = bp.R[s], Rb = bp.Rb[s];
  if (!owns_cell(X, Y, R, i, j)) return false;
  g.full = cell_within(X, Y, Rb, i, j);
  g.fs = g.full ? 1.0
                : shape_share<true>(X, Y, R, Rb, bp.cth[s], bp.sth[s], i, j);
  g.rx = xn - X;
  g.ry = yn - Y;
  g.usx = bp.Ux[s] - bp.Om[s] * g.ry;
  g.usy = bp.Uy[s] + bp.Om[s] * g.rx;
  return true;
}


// Scan form: gather the particles that reach tile b.  With `advance` (a
// lattice step) their positions are X + U and their velocities are rebuilt
// from the previous step's partials, and the first tile a particle reaches
// stores its new state in `next`; without it (init, ownership) the stored
// state is used.  Needs P.np <= 64.
__device__ void scan_block(BlockParticles& bp, const Params& P, int b,
                           PState cur, PState next, PConst pc,
                           const double* partial, int have, bool advance,
                           int* flags, int* tcount_next = nullptr) {
  __shared__ int s_nwork;
  __shared__ int s_work_pid[64], s_work_rank[64], s_work_store[64];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  // every wave loads the stored state of particle `lane`: a wave that
  // advances particle p then takes p's values from lane p, with no second
  // round trip to memory
  const bool held = lane < P.np;
  POne own = {};
  if (held) own = load_one(cur, pc, lane);
  if (wave == 0) {
    bool cand = false, store = false;
    double X = 0.0, Y = 0.0;
    if (held) {
      X = own.X;
      Y = own.Y;
      if (advance) advance_position(P, X, Y, own.Ux, own.Uy);
      const BlockRanges r = block_ranges(P, X, Y, own.R, kBlock);
      cand = r.contains(b);
      if (r.n == 0 && b == 0) atomicOr(flags, kFlagUnstable);
      store = advance && (r.n > 0 ? b == r.lo[0] : b == 0);
    }
    const unsigned long long below = (1ull << lane) - 1ull;
    const unsigned long long mc = __ballot(cand);
    const int rank = __popcll(mc & below);
    if (cand) {
      bp.pid[rank] = lane;
      bp.slot[rank] = lane * P.nblocks + b;
      bp.X[rank] = X;
      bp.Y[rank] = Y;
      bp.R[rank] = own.R;
      bp.Tp[rank] = own.Tinit;
      bp.Rb[rank] = own.Rb;
      // theta^{n+1} = theta^n + Omega^n (forward Euler, Sec. 2.3)
      orientation(own.R, own.Rb, advance ? own.th + own.Om : own.th,
                  bp.cth[rank], bp.sth[rank]);
      bp.held[rank] = (own.fixed >> 1) & 1;
    }
    const unsigned long long mw = __ballot(cand || store);
    const int wrank = __popcll(mw & below);
    if (cand || store) {
      s_work_pid[wrank] = lane;
      s_work_rank[wrank] = cand ? rank : -1;
      s_work_store[wrank] = store ? 1 : 0;
    }
    const unsigned long long mh = __ballot(cand && ((own.fixed >> 1) & 1));
    if (lane == 0) {
      bp.cnt = __popcll(mc);
      bp.nheld = __popcll(mh);
      s_nwork = __popcll(mw);
    }
  }
  __syncthreads();
  const int nwork = s_nwork;
  for (int k = wave; k < nwork; k += 4) {
    const int p = s_work_pid[k], r = s_work_rank[k];
    const POne sp = lane_one(own, p);
    if (advance) {
      double cx, cy, fx, fy, tz;
      repulsion_lanes(P, sp.X, sp.Y, sp.R, own.X, own.Y, own.R,
                      held && lane != p, cx, cy);
      reduce_partials_at(P, sp.X, sp.Y, sp.R, partial, have, p, lane, fx, fy,
                         tz);
      const PUpd u = particle_update_one(P, sp, fx, fy, tz, cx, cy);
      if (lane == 0) {
        if (r >= 0) {
          bp.Ux[r] = u.Ux;
          bp.Uy[r] = u.Uy;
          bp.Om[r] = u.Om;
        }
        if (s_work_store[k]) store_particle(next, p, u);
      }
      if (tcount_next && s_work_store[k]) {
        // the tiles the particle reaches at the next step's position (the
        // same arithmetic as that step's scan_task_tile)
        double Xn = u.X, Yn = u.Y;
        advance_position(P, Xn, Yn, u.Ux, u.Uy);
        const BlockRanges rn = block_ranges(P, Xn, Yn, sp.R, kBlock);
        for (int j = lane; j < rn.count(); j += 64)
          atomicAdd(&tcount_next[rn.at(j)], 1);
        // a centre the band-box logic cannot place: no tile serves it
        if (rn.n == 0 && lane == 0) atomicOr(flags, kFlagUnstable);
      }
    } else if (lane == 0 && r >= 0) {
      bp.Ux[r] = sp.Ux;
      bp.Uy[r] = sp.Uy;
      bp.Om[r] = sp.Om;
    }
  }
  __syncthreads();
}

// Geometry of a particle (centre X, Y, radius R, velocity U, Omega) for the
// cell (i, j): covered share and solid velocity u_s = U + Omega x (x - X) at
// the node (eq. us).  False when the particle does not reach the cell.
template <bool ELL>
__device__ __forceinline__ bool particle_geometry(const Params& P, double Xp,
                                                  double Yp, double R,
                                                  double Rb, double cth,
                                                  double sth, double Ux,
                                                  double Uy, double Om, int i,
                                                  int j, SlotGeom& g) {
  const double xn = (double)i + 0.5, yn = (double)j + 0.5;
  const double X = near_copy(Xp, xn, (double)P.nx, P.perx);
  const double Y = near_copy(Yp, yn, (double)P.ny, P.pery);
  if (!owns_cell(X, Y, R, i, j)) return false;
  g.full = cell_within(X, Y, Rb, i, j);
  g.fs = g.full ? 1.0 : shape_share<ELL>(X, Y, R, Rb, cth, sth, i, j);
  g.rx = xn - X;
  g.ry = yn - Y;
  g.usx = Ux - Om * g.ry;
  g.usy = Uy + Om * g.rx;
  return true;
}

// The lever arm x - X and the solid velocity u_s of a particle at the node
// of cell (i, j): the same arithmetic as particle_geometry, without the
// area.
__device__ __forceinline__ void particle_motion(const Params& P, double Xp,
                                                double Yp, double Ux,
                                                double Uy, double Om, int i,
                                                int j, double& rx, double& ry,
                                                double& usx, double& usy) {
  const double xn = (double)i + 0.5, yn = (double)j + 0.5;
  rx = xn - near_copy(Xp, xn, (double)P.nx, P.perx);
  ry = yn - near_copy(Yp, yn, (double)P.ny, P.pery);
  usx = Ux - Om * ry;
  usy = Uy + Om * rx;
}

// The particles reaching tile b (scan or list form).
template <bool SCAN>
__device__ __forceinline__ void gather_particles(
    BlockParticles& bp, int* tmp, const Params& P, int b, PState cur,
    PState next, PConst pc, Lists L, const double* partial, int have,
    bool advance, int* flags) {
  if (SCAN)
    scan_block(bp, P, b, cur, next, pc, partial, have, advance, flags);
  else
    load_block_list(bp, tmp, L, b, advance ? next : cur, pc, flags);
}

// -------------------------------------------------------------------------
// The fused lattice pass.

// Pull of direction Q for the cell: the upstream value, or -- when the
// upstream cell lies beyond a wall -- the rule of that wall applied to the
// opposite population of the cell itself.  XS/YS name the wall met across
// the x / y side (-1: none); when both apply (a corner) the y wall decides.
// Two halves, so that a caller can issue the loads of more than one cell
// before it uses any: pull_load reads the storage value from one selected
// address, pull_fix converts it and applies the wall's rule (selects of
// compile-time-indexed wall constants).  Branch-free.
template <int Q, int OPP, int XS, int YS, class T>
__device__ __forceinline__ void pull_load(const typename T::S* __restrict__ fin,
                                          const typename T::S* __restrict__ gin,
                                          size_t plane, int cc, int src,
                                          bool ox, bool oy,
                                          typename T::S& fr,
                                          typename T::S& gr) {
  const bool out = (XS >= 0 && ox) || (YS >= 0 && oy);
  const size_t idx = out ? (size_t)OPP * plane + cc : (size_t)Q * plane + src;
  fr = fin[idx];
  gr = gin[idx];
}

template <int Q, int XS, int YS, class T>
__device__ __forceinline__ void pull_fix(typename T::S fr, typename T::S gr,
                                         bool ox, bool oy,
                                         const Hot<typename T::C>& H,
                                         typename T::C& fv,
                                         typename T::C& gv) {
  typedef typename T::C C;
  C f = T::cv(fr), g = T::cv(gr);
  if (XS >= 0 || YS >= 0) {
    const bool out = (XS >= 0 && ox) || (YS >= 0 && oy);
    constexpr int WX = XS >= 0 ? XS : YS, WY = YS >= 0 ? YS : XS;
    const bool useY = YS >= 0 && oy;
    const C fa = useY ? H.fadd[WY][Q] : H.fadd[WX][Q];
    const C ga = useY ? H.gadd[WY][Q] : H.gadd[WX][Q];
    const C gs = useY ? H.gsign[WY] : H.gsign[WX];
    f = out ? f + fa : f;
    g = out ? gs * g + ga : g;
  }
  fv = f;
  gv = g;
}

// M f for D2Q9 (rows of M, Sec. 2.1).
template <class C>
__device__ __forceinline__ void moments(const C* f, C* m) {
  const C a14 = f[1] + f[2] + f[3] + f[4];
  const C a58 = f[5] + f[6] + f[7] + f[8];
  m[0] = f[0] + a14 + a58;
  m[1] = -4 * f[0] - a14 + 2 * a58;
  m[2] = 4 * f[0] - 2 * a14 + a58;
  const C b57 = f[5] - f[7], b68 = f[6] - f[8];
  m[3] = f[1] - f[3] + b57 - b68;
  m[4] = -2 * (f[1] - f[3]) + b57 - b68;
  m[5] = f[2] - f[4] + b57 + b68;
  m[6] = -2 * (f[2] - f[4]) + b57 + b68;
  m[7] = f[1] - f[2] + f[3] - f[4];
  m[8] = f[5] - f[6] + f[7] - f[8];
}

// m / d for the moment norms d = 9, 36, 6, 12.  In FP32 the reciprocal is
// split into two floats, hi = fl(1/d) and lo = fl(1/d - hi), so that the
// product carries no systematic error: with hi alone, the momentum the
// populations rebuild is 6 fl(1/6) j = (1 + 3e-8) j and the rest moment
// 9 fl(1/9) m_0, a gain the same in every cell at every step.  At
// tau_f = 0.53 that acts as negative friction worth about 5e-4 of the
// steady speed of a body-force channel, and in the energy lattice as a
// heat source.  FP64's fl(1/d) is exact to 1e-17 and keeps one product.
template <int D, class C>
__device__ __forceinline__ C over(C m) {
  constexpr double r = 1.0 / D;
  if constexpr (sizeof(C) == sizeof(float)) {
    constexpr float hi = (float)r;
    constexpr float lo = (float)(r - (double)hi);
    return m * hi + m * lo;
  } else {
    return m * (C)r;
  }
}

// M^{-1} m = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m
// (the rows of M are orthogonal with those squared norms).
template <class C>
__device__ __forceinline__ void inverse(const C* m, C* o) {
  const C k0 = over<9>(m[0]), k1 = over<36>(m[1]), k2 = over<36>(m[2]),
          k3 = over<6>(m[3]), k4 = over<12>(m[4]), k5 = over<6>(m[5]),
          k6 = over<12>(m[6]), k7 = m[7] * (C)0.25, k8 = m[8] * (C)0.25;
  o[0] = k0 - 4 * k1 + 4 * k2;
  const C ax = k0 - k1 - 2 * k2;
  o[1] = ax + k3 - 2 * k4 + k7;
  o[2] = ax + k5 - 2 * k6 - k7;
  o[3] = ax - k3 + 2 * k4 + k7;
  o[4] = ax - k5 + 2 * k6 - k7;
  const C dg = k0 + 2 * k1 + k2;
  const C p34 = k3 + k4, p56 = k5 + k6;
  o[5] = dg + p34 + p56 + k8;
  o[6] = dg - p34 + p56 - k8;
  o[7] = dg - p34 - p56 + k8;
  o[8] = dg + p34 - p56 - k8;
}

// Particle sums of one cell: total solid fraction f_s = sum_p f_s,p and
// sum_p f_s,p (u_s, u_s u_s), the inputs of the volumetric step.
template <class C>
struct PSums {
  C S0, S1x, S1y, S2xx, S2yy, S2xy;
  C H0, H1;   // over particles whose temperature is held: sum f_s,p, sum f_s,p T_p
};

// The storage values one lane loads for its cell of a tile (the pulled
// populations and the carrier), with the cell's coordinates.
template <int PREC>
struct CellLoad {
  typename Prec<PREC>::S f[9], g[9];
  typename Prec<PREC>::H hn;
  int cc, x, y;
  bool act;
};

// Which faces a cell's upstream neighbours lie beyond (walls only).
struct Beyond {
  bool xm, xp, ym, yp;
};

__device__ __forceinline__ Beyond beyond(const Params& P, int x, int y) {
  Beyond o;
  o.xm = x == 0 && !P.perx;
  o.xp = x == P.nx - 1 && !P.perx;
  o.ym = y == 0 && !P.pery;
  o.yp = y == P.ny - 1 && !P.pery;
  return o;
}

// Issue the loads of this lane's cell of `tile` (pull streaming with the
// wall rules' addresses, eq. lbe.rho.str and lbe.e.str); inactive lanes
// read a valid cell.
template <int PREC>
__device__ __forceinline__ void load_cell(
    const Params& P, const typename Prec<PREC>::S* __restrict__ fin,
    const typename Prec<PREC>::S* __restrict__ gin,
    const typename Prec<PREC>::H* __restrict__ hin, size_t plane, int tile,
    CellLoad<PREC>& L) {
  typedef Prec<PREC> T;
  const int c = tile * kBlock + threadIdx.x;
  L.act = c < P.N;
  const int cc = L.act ? c : P.N - 1;
  const int y = cc / P.nx;
  const int x = cc - y * P.nx;
  L.cc = cc;
  L.x = x;
  L.y = y;
  const Beyond o = beyond(P, x, y);
  int xm = x - 1, xp = x + 1, ym = y - 1, yp = y + 1;
  xm = xm < 0 ? xm + P.nx : xm;
  xp = xp >= P.nx ? xp - P.nx : xp;
  ym = ym < 0 ? ym + P.ny : ym;
  yp = yp >= P.ny ? yp - P.ny : yp;
  const int r0 = y * P.nx, rm = ym * P.nx, rp = yp * P.nx;
  constexpr int XLO = VLB_FACE_XLO, XHI = VLB_FACE_XHI;
  constexpr int YLO = VLB_FACE_YLO, YHI = VLB_FACE_YHI;
  L.f[0] = fin[cc];
  L.g[0] = gin[cc];
  pull_load<1, 3, XLO, -1, T>(fin, gin, plane, cc, r0 + xm, o.xm, false, L.f[1], L.g[1]);
  pull_load<2, 4, -1, YLO, T>(fin, gin, plane, cc, rm + x, false, o.ym, L.f[2], L.g[2]);
  pull_load<3, 1, XHI, -1, T>(fin, gin, plane, cc, r0 + xp, o.xp, false, L.f[3], L.g[3]);
  pull_load<4, 2, -1, YHI, T>(fin, gin, plane, cc, rp + x, false, o.yp, L.f[4], L.g[4]);
  pull_load<5, 7, XLO, YLO, T>(fin, gin, plane, cc, rm + xm, o.xm, o.ym, L.f[5], L.g[5]);
  pull_load<6, 8, XHI, YLO, T>(fin, gin, plane, cc, rm + xp, o.xp, o.ym, L.f[6], L.g[6]);
  pull_load<7, 5, XHI, YHI, T>(fin, gin, plane, cc, rp + xp, o.xp, o.yp, L.f[7], L.g[7]);
  pull_load<8, 6, XLO, YHI, T>(fin, gin, plane, cc, rp + xm, o.xm, o.yp, L.f[8], L.g[8]);
  L.hn = hin[cc];
}

// The lattice update of one loaded cell: the wall rules on the pulled
// values, the volumetric no-slip step with the particle sums `part`
// supplies (called as part(act, x, y, rho - rho_0, jx*, jy*, S)), the
// coupled macroscopic solve and both collisions, then the stores.
//
// Conserved moments are updated in the form that rounds no quantity of
// order one: the density moment keeps rho - rho_0, the momentum after the
// collision is j + F (exactly rho u + F/2 with rho u = j + F/2), the rest
// moment of the energy is n_0 + q_c (exactly eps + q_c/2, since the
// implicit relation for T makes eps - q_c/2 the streamed sum G), and a
// product rho v is formed as rho_0 v + (rho - rho_0) v.  In FP64 these
// equal the literal forms to rounding; in the 32- and 16-bit forms they
// keep the per-step rounding from acting as a small systematic force or
// heat source.
template <int PREC, bool OUT, bool NT, class PartFn>
__device__ __forceinline__ void update_cell(
    const Params& P, const Hot<typename Prec<PREC>::C>& H,
    const CellLoad<PREC>& L, typename Prec<PREC>::S* __restrict__ fout,
    typename Prec<PREC>::S* __restrict__ gout,
    typename Prec<PREC>::H* __restrict__ hout, size_t plane,
    double* __restrict__ macro, int* flags, PartFn part) {
  typedef Prec<PREC> T;
  typedef typename T::C C;
  typedef typename T::H HT;
  const bool act = L.act;
  const int cc = L.cc, x = L.x, y = L.y;
  const Beyond o = beyond(P, x, y);
  constexpr int XLO = VLB_FACE_XLO, XHI = VLB_FACE_XHI;
  constexpr int YLO = VLB_FACE_YLO, YHI = VLB_FACE_YHI;
  C f[9], g[9];
  f[0] = T::cv(L.f[0]);
  g[0] = T::cv(L.g[0]);
  pull_fix<1, XLO, -1, T>(L.f[1], L.g[1], o.xm, false, H, f[1], g[1]);
  pull_fix<2, -1, YLO, T>(L.f[2], L.g[2], false, o.ym, H, f[2], g[2]);
  pull_fix<3, XHI, -1, T>(L.f[3], L.g[3], o.xp, false, H, f[3], g[3]);
  pull_fix<4, -1, YHI, T>(L.f[4], L.g[4], false, o.yp, H, f[4], g[4]);
  pull_fix<5, XLO, YLO, T>(L.f[5], L.g[5], o.xm, o.ym, H, f[5], g[5]);
  pull_fix<6, XHI, YLO, T>(L.f[6], L.g[6], o.xp, o.ym, H, f[6], g[6]);
  pull_fix<7, XHI, YHI, T>(L.f[7], L.g[7], o.xp, o.yp, H, f[7], g[7]);
  pull_fix<8, XLO, YHI, T>(L.f[8], L.g[8], o.xm, o.yp, H, f[8], g[8]);
  const HT hn = L.hn;

  // ---- moments of the deviations f* - w rho_0; the reference adds
  // rho_0 (1, -2, 1, 0, ..., 0) to M f*
  C m[9];
  moments(f, m);
  const C drho = m[0];                 // rho - rho_0
  const C rho = H.rho0s + drho;        // rho = sum f*_i, kept by eq. fi
  const C jxs = m[3], jys = m[5];
  // rho v without rounding rho = rho_0 + drho first
  auto rmul = [&](C v) { return H.rho0s * v + drho * v; };

  // ---- particles: solid fraction, u_s, momentum exchange (Sec. 2.3)
  PSums<C> S;
  S.S0 = S.S1x = S.S1y = S.S2xx = S.S2yy = S.S2xy = (C)0;
  S.H0 = S.H1 = (C)0;
  part(act, x, y, drho, jxs, jys, S);

  // ---- volumetric no-slip step in moment space (eq. fi):
  // M f = (1 - f_s) M f* + rho sum_p f_s,p m^eq(1, u_s,p), written for the
  // deviations (the reference moments cancel against rho_0 S0)
  const C S0 = S.S0, S1x = S.S1x, S1y = S.S1y;
  const C S2xx = S.S2xx, S2yy = S.S2yy, S2xy = S.S2xy;
  const C fs = S0;
  const C wf = (C)1 - fs;
  {
    const C tr = S2xx + S2yy;
    const C rS1x = rmul(S1x), rS1y = rmul(S1y);
    m[0] = drho;                       // eq. fi keeps rho
    m[1] = wf * m[1] + (-2 * S0 * drho + 3 * rho * tr);
    m[2] = wf * m[2] + (S0 * drho - 3 * rho * tr);
    m[3] = wf * m[3] + rS1x;
    m[4] = wf * m[4] - rS1x;
    m[5] = wf * m[5] + rS1y;
    m[6] = wf * m[6] - rS1y;
    m[7] = wf * m[7] + rho * (S2xx - S2yy);
    m[8] = wf * m[8] + rho * S2xy;
  }

  // ---- [df_s/dt] by eq. dfs_dt through the carrier h = 2 f_s + d:
  // d^{n+1} = 2 f_s^{n+1} - h^n,  h^{n+1} = 2 f_s^{n+1} + d^{n+1}
  const C dfs = 2 * fs - (C)hn;
  const HT hnew = (HT)(2 * fs + dfs);

  // ---- per-cell properties (Sec. 2.2) and relaxation rates (Sec. 3)
  const C cv = H.cvf + H.dcv * fs;
  const C lam = H.lamf + H.dlam * fs;
  const C tau_g = (C)0.5 + H.taug_coef * lam;
  const C sig_j = (C)1 / tau_g;
  // (1/sig_j - 1/2)(1/sig_e - 1/2) = 1/4 is sig_e = 2 - sig_j
  const C sig_e = H.sigma_rule == 0 ? (C)2 - sig_j : (C)1;

  // ---- energy moments (the reference w c_ref T_0 adds c_ref T_0 (1, -2,
  // 1, 0, ..., 0)) and the local temperature gradient (Sec. 2.2)
  C n[9];
  moments(g, n);
  const C cT0 = H.cT0s;
  // ---- particles whose temperature is held (a reading; the paper gives
  // no rule): the volumetric step of the energy distribution, g = (1 -
  // sum_h f_s,p) g* + sum_h f_s,p g^eq(c_v T_p, T_p), with c_v the cell's
  // heat capacity.  g^eq is linear in (eps, T), so the held particles
  // enter through H0 = sum_h f_s,p and H1 = sum_h f_s,p T_p; in moments,
  // minus the reference c_ref T_0 (1, -2, 1, 0, ..., 0)
  if (S.H0 != (C)0) {
    const C wh = (C)1 - S.H0, e1 = cv * S.H1, c1 = H.cref * S.H1;
    n[0] = wh * n[0] - S.H0 * cT0 + e1;
    n[1] = wh * n[1] + 2 * S.H0 * cT0 + (-4 * e1 + 2 * c1);
    n[2] = wh * n[2] - S.H0 * cT0 + (4 * e1 - 3 * c1);
#pragma unroll
    for (int k = 3; k < 9; ++k) n[k] = wh * n[k];
  }
  const C G = n[0] + cT0;                          // sum g_i
  const C gcoef = H.grad_coef * sig_j;             // -3 / (c_ref tau_g)
  const C gTx = gcoef * n[3], gTy = gcoef * n[5];

  // ---- coupled macroscopic solve: u from eq. rho.rhou with F = a + b T,
  // T from the implicit relation of Sec. 2.2 (linear in T)
  const C ax = wf * H.A0x, ay = wf * H.A0y;
  const C bx = wf * H.B0x, by = wf * H.B0y;
  const C irho = (C)1 / rho;
  const C jx = m[3], jy = m[5];
  const C num = G - (C)0.5 * cv * ((jx + (C)0.5 * ax) * gTx + (jy + (C)0.5 * ay) * gTy) * irho;
  const C den = cv - (C)0.5 * H.dcv * dfs + (C)0.25 * cv * (bx * gTx + by * gTy) * irho;
  const C Tc = num / den;
  const C Fx = ax + bx * Tc, Fy = ay + by * Tc;
  const C ux = (jx + (C)0.5 * Fx) * irho, uy = (jy + (C)0.5 * Fy) * irho;
  const C eps = cv * Tc;
  const C qc = -cv * (ux * gTx + uy * gTy) + H.dcv * Tc * dfs;

  if (act && !(rho > (C)0 && isfinite(Tc) && isfinite(ux) && isfinite(uy)))
    atomicOr(flags, kFlagUnstable);

  // ---- flow collision with the discrete force term (eq. lbe.rho.col);
  // m^eq minus the reference moments is (drho, -2 drho + 3 rho u^2,
  // drho - 3 rho u^2, rho ux, -rho ux, rho uy, -rho uy, rho (ux^2 - uy^2),
  // rho ux uy); s_0 = s_j = 1
  {
    const C ru2 = rho * (ux * ux + uy * uy);
    const C se = H.s_e, sq = H.s_q, sp = H.s_p;
    const C he = (C)1 - (C)0.5 * se, hq = (C)1 - (C)0.5 * sq,
            hp = (C)1 - (C)0.5 * sp;
    const C Fu = Fx * ux + Fy * uy;
    C mb[9];
    mb[0] = drho;
    mb[1] = m[1] - se * (m[1] - (-2 * drho + 3 * ru2)) + he * (6 * Fu);
    mb[2] = m[2] - se * (m[2] - (drho - 3 * ru2)) - he * (6 * Fu);
    const C rux = jx + (C)0.5 * Fx, ruy = jy + (C)0.5 * Fy;   // rho u
    mb[3] = jx + Fx;
    mb[4] = m[4] - sq * (m[4] + rux) - hq * Fx;
    mb[5] = jy + Fy;
    mb[6] = m[6] - sq * (m[6] + ruy) - hq * Fy;
    mb[7] = m[7] - sp * (m[7] - rho * (ux * ux - uy * uy)) + hp * (2 * (Fx * ux - Fy * uy));
    mb[8] = m[8] - sp * (m[8] - rho * ux * uy) + hp * (Fx * uy + Fy * ux);
    C o[9];
    inverse(mb, o);
    if (act) {
      if constexpr (NT) {
#pragma unroll
        for (int q = 0; q < 9; ++q) T::stn(fout, (size_t)q * plane + cc, o[q]);
      } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) T::st(fout, (size_t)q * plane + cc, o[q]);
      }
    }
  }

  // ---- energy collision with the discrete source term (eq. lbe.e.col):
  // n^eq = [eps, -4 eps + 2 c_ref T, 4 eps - 3 c_ref T, 0...] (alpha1 = -2,
  // alpha2 = 1), q_m = [q, -4 q, 4 q, 0...] (beta1 = -4, beta2 = 4),
  // R = diag(1, se, se, sj, sj, sj, sj, se, se); moments minus reference
  {
    const C cT = H.cref * Tc;
    const C he = (C)1 - (C)0.5 * sig_e;
    C nb[9];
    nb[0] = n[0] + qc;   // eps + q_c/2 minus the reference
    nb[1] = n[1] - sig_e * (n[1] - (-4 * eps + 2 * cT + 2 * cT0)) - he * (4 * qc);
    nb[2] = n[2] - sig_e * (n[2] - (4 * eps - 3 * cT - cT0)) + he * (4 * qc);
    const C rj = (C)1 - sig_j, re = (C)1 - sig_e;
    nb[3] = rj * n[3];
    nb[4] = rj * n[4];
    nb[5] = rj * n[5];
    nb[6] = rj * n[6];
    nb[7] = re * n[7];
    nb[8] = re * n[8];
    C o[9];
    inverse(nb, o);
    if (act) {
      if constexpr (NT) {
#pragma unroll
        for (int q = 0; q < 9; ++q) T::stn(gout, (size_t)q * plane + cc, o[q]);
        __builtin_nontemporal_store(hnew, hout + cc);
      } else {
#pragma unroll
        for (int q = 0; q < 9; ++q) T::st(gout, (size_t)q * plane + cc, o[q]);
        hout[cc] = hnew;
      }
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

// The lattice update of the 256 cells of one tile.  Every thread of the
// block calls pre() before it issues its loads, gather() right after (so
// that its work overlaps them; a true result, which must be uniform over
// the wave, abandons the tile: the return value is then false), and part()
// as update_cell describes.
template <int PREC, bool OUT, bool NT, class PreFn, class GatherFn,
          class PartFn>
__device__ __forceinline__ bool lattice_tile(
    const Params& P, const Hot<typename Prec<PREC>::C>& H,
    const typename Prec<PREC>::S* __restrict__ fin,
    typename Prec<PREC>::S* __restrict__ fout,
    const typename Prec<PREC>::S* __restrict__ gin,
    typename Prec<PREC>::S* __restrict__ gout,
    const typename Prec<PREC>::H* __restrict__ hin,
    typename Prec<PREC>::H* __restrict__ hout, size_t plane, int tile,
    double* __restrict__ macro, int* flags, PreFn pre, GatherFn gather,
    PartFn part) {
  CellLoad<PREC> L;
  pre();
  load_cell<PREC>(P, fin, gin, hin, plane, tile, L);
  if (gather()) return false;
  update_cell<PREC, OUT, NT>(P, H, L, fout, gout, hout, plane, macro, flags,
                             part);
  return true;
}

// Tile of particle-tile block k in the scan form: block k serves the
// (k / maxr)-th particle's (k % maxr)-th tile, unless a particle of lower
// index also reaches that tile (its block serves it).  -1: nothing to do.
__device__ __forceinline__ int scan_task_tile(const Params& P, PState cur,
                                              PConst pc, int k) {
  const int p = k / P.maxr, j = k - p * P.maxr;
  if (p >= P.np) return -1;
  double X = cur.X[p], Y = cur.Y[p];
  advance_position(P, X, Y, cur.Ux[p], cur.Uy[p]);
  const BlockRanges r = block_ranges(P, X, Y, pc.R[p], kBlock);
  if (j >= r.count()) return -1;
  const int tile = r.at(j);
  for (int q = 0; q < p; ++q) {
    double Xq = cur.X[q], Yq = cur.Y[q];
    advance_position(P, Xq, Yq, cur.Ux[q], cur.Uy[q]);
    if (block_ranges(P, Xq, Yq, pc.R[q], kBlock).contains(tile)) return -1;
  }
  return tile;
}

// Tile of the k-th block of the streaming group.  Workgroups are dealt to
// the 8 XCDs in turn, so block k runs on XCD x = k % 8.  Tiles come in
// groups of G consecutive tiles, dealt to the XCDs in turn, and each XCD
// walks its groups' tiles in order: the rows a tile pulls from its
// neighbours are then mostly in the XCD's own L2 already.  (The group
// starts at a multiple of 8 blocks.)  With a tile stride (list form) block
// k takes tile k * stride mod stream_blocks instead, a permutation that
// scatters the tiles over the launch.  Tiles >= nblocks: none.
__device__ __forceinline__ int stream_tile(const Params& P, int k) {
  if (P.tile_stride)
    return (int)((long long)k * P.tile_stride % P.stream_blocks);
  const int x = k & 7, j = k >> 3;
  const int gi = j / P.xcd_group, o = j - gi * P.xcd_group;
  return (gi * 8 + x) * P.xcd_group + o;
}

// The 16-bit forms can stream two tiles per block (pair_task), where the
// host has set P.pair_tiles.
template <int PREC>
constexpr bool kPairedTiles = PREC == VLB_FP16_SHIFT || PREC == VLB_BF16_SHIFT;

// Streaming blocks of one step: one per tile of the XCD-ordered sequence,
// or one per pair (k, k + 8) of it.
__host__ __device__ inline int stream_grid(const Params& P, bool pair) {
  return pair ? (P.stream_blocks + 15) / 16 * 8 : P.stream_blocks;
}

// LDS of a particle tile: the staged particles, the per-cell particle sums
// (written before the lattice update, read by it) and the per-cell rho, j*
// (written by the lattice update, read by the momentum exchange).
constexpr int kShareCache = 4;   // shares per cell kept from phase 1

template <class C>
struct TileShared {
  BlockParticles bp;
  int tmp[kListCap];
  double red[kListCap][4][3];  // per slot and wave: force x, y, torque
  C S[6][kBlock];      // f_s and sum_p f_s,p (u_s, u_s u_s), shares scaled
  C S0raw[kBlock];     // sum_p f_s,p before scaling
  C M[3][kBlock];      // rho, jx*, jy* after streaming (before the lattice
                       // update: the held sums H0, H1 of phase 1)
  // the first kShareCache particles reaching each cell (slot order): slot
  // and share, so the momentum exchange need not recompute the areas
  C share[kShareCache][kBlock];
  unsigned char slot[kShareCache][kBlock];
  unsigned char nreach[kBlock];  // particles reaching the cell (saturated)
  // phase 1: the (cell, cache entry) pairs whose exact area is pending,
  // packed as cell * kShareCache + entry, and the per-wave counts
  unsigned short work[kShareCache * kBlock];
  int wcount[kBlock / 64];
};

// Whether the cell span [a0, a1] (unwrapped on a periodic axis of n cells)
// meets [b0, b1] (within the axis).
__device__ __forceinline__ bool span_meets(int a0, int a1, int b0, int b1,
                                           int n, int periodic) {
  if (a1 - a0 + 1 >= n) return true;
  if (!periodic) return a1 >= b0 && a0 <= b1;
  for (int sh = -n; sh <= n; sh += n)
    if (a1 + sh >= b0 && a0 + sh <= b1) return true;
  return false;
}

// The particles of a tile whose band box meets the 64 cells of wave w: bit
// k for slot k (every lane gets the same mask).  A particle owns no cell
// outside its band box, so a wave may skip the others.
__device__ __forceinline__ unsigned long long wave_particle_mask(
    const Params& P, const BlockParticles& bp, int cnt, int tile, int w,
    int lane) {
  const int c0 = tile * kBlock + w * 64;
  bool hit = false;
  if (lane < cnt && c0 < P.N) {
    const int c1 = min(c0 + 63, P.N - 1);
    const int r0 = c0 / P.nx, r1 = c1 / P.nx;
    int x0 = 0, x1 = P.nx - 1;   // whole rows where the wave spans two
    if (r0 == r1) {
      x0 = c0 - r0 * P.nx;
      x1 = c1 - r0 * P.nx;
    }
    int i0, i1, j0, j1;
    band_box(P, bp.X[lane], bp.Y[lane], bp.R[lane], i0, i1, j0, j1);
    hit = span_meets(j0, j1, r0, r1, P.ny, P.pery) &&
          span_meets(i0, i1, x0, x1, P.nx, P.perx);
  }
  return __ballot(hit);
}

// One tile of one time step (a whole step is one launch of k_step, or of
// k_batch_step for many domains).  Two roles:
//
//  * particle tiles (the tiles particles reach): the particles of the tile
//    (scan form: found and advanced here, velocities rebuilt from the
//    previous step's partials; list form: the block list k_particles
//    filled), then three phases that keep the register peak at that of the
//    plain update -- (1) exact-area solid fractions and the particle sums
//    of each cell into LDS, (2) the lattice update reading them, (3) the
//    per-block momentum-exchange partials of every particle of the tile;
//  * plain tiles: the lattice update without particles.
//
// Scan form: the first np * maxr blocks (tasks) take the particle tiles (so
// their longer dependency chain starts first and overlaps the streaming of
// the rest); the following ones take every tile and leave those some
// particle reaches to the first group.  COUNTED (one domain): they know
// those tiles from per-tile counts that the previous step's particle
// blocks filled (the same advanced positions and band boxes); otherwise
// (a batch) they test them, one particle per lane.  List form: each tile
// in the role its block count gives.
template <int PREC, bool OUT, bool SCAN, bool COUNTED = false,
          bool ELL = false, bool NT = false, bool INL = false>
__device__ __forceinline__ void step_task(
    const Params& P, const Hot<typename Prec<PREC>::C>& H, const StepBufs& B,
    int have, int tile, bool ptile, TileShared<typename Prec<PREC>::C>& sh,
    int lcnt = 0, int2 lent = make_int2(0, 0)) {
  typedef typename Prec<PREC>::C C;
  typedef typename Prec<PREC>::S S;
  typedef typename Prec<PREC>::H HT;
  const S* __restrict__ fin = (const S*)B.fi;
  S* __restrict__ fout = (S*)B.fo;
  const S* __restrict__ gin = (const S*)B.gi;
  S* __restrict__ gout = (S*)B.go;
  const HT* __restrict__ hin = (const HT*)B.hin;
  HT* __restrict__ hout = (HT*)B.hout;
  const size_t plane = B.plane;
  const PState cur = B.cur, nxt = B.nxt;
  const PConst pc = B.pc;
  const Lists L = B.L;
  const double* __restrict__ partial_in = B.partial_in;
  double* __restrict__ partial = B.partial_out;
  double* __restrict__ macro = B.macro;
  int* flags = B.flags;
  const int t = threadIdx.x, lane = t & 63;

  const int c0 = tile * kBlock + t;
  const bool act0 = c0 < P.N;
  const int cy = (act0 ? c0 : P.N - 1) / P.nx;
  const int cx = (act0 ? c0 : P.N - 1) - cy * P.nx;

  unsigned long long wmask = 0ull;  // particle tiles: the wave's particles
  bool anyheld = false;             // particle tiles: a held particle among them
  // ---- phase 1 (particle tiles): particles of the tile, and per cell the
  // solid fraction f_s = sum_p f_s,p and sum_p f_s,p (u_s, u_s u_s); where
  // overlapping disks cover more than the cell the shares are scaled to
  // sum to one
  if (ptile) {
    if (SCAN)
      scan_block(sh.bp, P, tile, cur, nxt, pc, partial_in, have, true, flags,
                 B.tcount_next);
    else
      if (kListEntryAhead<PREC>)
        load_block_list_known(sh.bp, sh.tmp, lcnt, lent, nxt, pc, flags);
      else
        load_block_list(sh.bp, sh.tmp, L, tile, nxt, pc, flags);
    // (a) which particles reach the cell (slot order; only those whose
    // band box meets the wave's cells), whether they cover it wholly; the
    // first kShareCache are kept
    const int cnt = sh.bp.cnt;
    anyheld = sh.bp.nheld > 0;
    wmask = cnt > 1 ? wave_particle_mask(P, sh.bp, cnt, tile, t >> 6, lane)
                    : (unsigned long long)cnt;   // one particle: no test
    const double xn = (double)cx + 0.5, yn = (double)cy + 0.5;
    int nin = 0;
    unsigned cut = 0;                 // cache entries whose area is pending
    for (unsigned long long m = act0 ? wmask : 0ull; m; m &= m - 1) {
      const int k = __ffsll((long long)m) - 1;
      const double X = near_copy(sh.bp.X[k], xn, (double)P.nx, P.perx);
      const double Y = near_copy(sh.bp.Y[k], yn, (double)P.ny, P.pery);
      const double R = sh.bp.R[k];
      if (!(INL ? owns_cell_in(X, Y, R, cx, cy) : owns_cell(X, Y, R, cx, cy)))
        continue;
      if (nin < kShareCache) {
        sh.slot[nin][t] = (unsigned char)k;
        if (INL ? cell_within_in(X, Y, sh.bp.Rb[k], cx, cy)
                : cell_within(X, Y, sh.bp.Rb[k], cx, cy))
          sh.share[nin][t] = (C)1;
        else
          cut |= 1u << nin;
      }
      ++nin;
    }
    // (b) the exact areas of the partly covered cells.  With one particle
    // each lane computes its own (a wave evaluates one area at most);
    // with more they are compacted over the block so that every lane of a
    // wave computes one (a tile has a few dozen of them; lane by lane, a
    // wave would evaluate one area per particle it meets).
    if (cnt <= 1) {
      if (cut) {
        const int k = sh.slot[0][t];
        const double X = near_copy(sh.bp.X[k], xn, (double)P.nx, P.perx);
        const double Y = near_copy(sh.bp.Y[k], yn, (double)P.ny, P.pery);
        sh.share[0][t] = (C)shape_share<ELL>(X, Y, sh.bp.R[k], sh.bp.Rb[k],
                                             sh.bp.cth[k], sh.bp.sth[k], cx,
                                             cy);
      }
    } else {
      const int mine = __popc(cut);
      const int w = t >> 6;
      int wtotal;
      const int below = wave_excl_scan<3>(mine, lane, wtotal);
      if (lane == 0) sh.wcount[w] = wtotal;
      __syncthreads();
      int base = below, total = 0;
      for (int v = 0; v < kBlock / 64; ++v) {
        base += v < w ? sh.wcount[v] : 0;
        total += sh.wcount[v];
      }
      for (unsigned m = cut; m; m &= m - 1)
        sh.work[base++] = (unsigned short)(t * kShareCache + __ffs(m) - 1);
      __syncthreads();
      for (int q = t; q < total; q += kBlock) {
        const int item = sh.work[q];
        const int tt = item / kShareCache, e = item - tt * kShareCache;
        const int c = tile * kBlock + tt;
        const int j = c / P.nx, i = c - j * P.nx;
        const int k = sh.slot[e][tt];
        const double X =
            near_copy(sh.bp.X[k], (double)i + 0.5, (double)P.nx, P.perx);
        const double Y =
            near_copy(sh.bp.Y[k], (double)j + 0.5, (double)P.ny, P.pery);
        sh.share[e][tt] = (C)shape_share<ELL>(X, Y, sh.bp.R[k], sh.bp.Rb[k],
                                              sh.bp.cth[k], sh.bp.sth[k], i,
                                              j);
      }
      __syncthreads();
    }
    // (c) the particle sums, in slot order; past the cache (more than
    // kShareCache particles in one cell) the geometry is computed here
    PSums<C> S;
    S.S0 = S.S1x = S.S1y = S.S2xx = S.S2yy = S.S2xy = (C)0;
    S.H0 = S.H1 = (C)0;
    const int ncached = nin < kShareCache ? nin : kShareCache;
    for (int e = 0; e < ncached; ++e) {
      const int k = sh.slot[e][t];
      double rx, ry, usx, usy;
      particle_motion(P, sh.bp.X[k], sh.bp.Y[k], sh.bp.Ux[k], sh.bp.Uy[k],
                      sh.bp.Om[k], cx, cy, rx, ry, usx, usy);
      const C a = sh.share[e][t], ux = (C)usx, uy = (C)usy;
      S.S0 += a;
      S.S1x += a * ux;
      S.S1y += a * uy;
      S.S2xx += a * ux * ux;
      S.S2yy += a * uy * uy;
      S.S2xy += a * ux * uy;
      if (anyheld && sh.bp.held[k]) {
        S.H0 += a;
        S.H1 += a * (C)sh.bp.Tp[k];
      }
    }
    if (nin > kShareCache) {
      for (int k = sh.slot[kShareCache - 1][t] + 1; k < cnt; ++k) {
        if (!((wmask >> k) & 1ull)) continue;
        SlotGeom sg;
        if (particle_geometry<ELL>(P, sh.bp.X[k], sh.bp.Y[k], sh.bp.R[k],
                              sh.bp.Rb[k], sh.bp.cth[k], sh.bp.sth[k],
                              sh.bp.Ux[k], sh.bp.Uy[k], sh.bp.Om[k], cx, cy,
                              sg)) {
          const C a = (C)sg.fs, ux = (C)sg.usx, uy = (C)sg.usy;
          S.S0 += a;
          S.S1x += a * ux;
          S.S1y += a * uy;
          S.S2xx += a * ux * ux;
          S.S2yy += a * uy * uy;
          S.S2xy += a * ux * uy;
          if (anyheld && sh.bp.held[k]) {
            S.H0 += a;
            S.H1 += a * (C)sh.bp.Tp[k];
          }
        }
      }
    }
    if (act0 && nin > P.kmax) atomicOr(flags, kFlagOverlap);
    sh.nreach[t] = (unsigned char)(nin < 255 ? nin : 255);
    sh.S0raw[t] = S.S0;
    if (S.S0 > (C)1) {
      const C inv = (C)1 / S.S0;
      S.S1x *= inv; S.S1y *= inv; S.S2xx *= inv; S.S2yy *= inv;
      S.S2xy *= inv; S.H0 *= inv; S.H1 *= inv;
      S.S0 = (C)1;
    }
    sh.S[0][t] = S.S0; sh.S[1][t] = S.S1x; sh.S[2][t] = S.S1y;
    sh.S[3][t] = S.S2xx; sh.S[4][t] = S.S2yy; sh.S[5][t] = S.S2xy;
    // the held sums wait in M, which the lattice update fills only after
    // part() has read them
    if (anyheld) {
      sh.M[0][t] = S.H0;
      sh.M[1][t] = S.H1;
    }
  }

  // ---- phase 2: the lattice update
  // scan form, plain tiles: is the tile a particle tile (the first group's)?
  // COUNTED: the count the previous step left for it (and this block clears
  // the tile's stale count).  Otherwise wave 0 tests it (one particle per
  // lane) and shares the answer through LDS; the test is issued after the
  // population loads, so it hides behind them.
  const bool counted = COUNTED && SCAN && !ptile;
  const bool probe = !COUNTED && SCAN && !ptile && t < P.np;
  double X = 0.0, Y = 0.0, Ux = 0.0, Uy = 0.0, R = 0.0;
  auto pre = [&] {
    if (counted && t == 0) B.tcount_clear[tile] = 0;
    if (probe) {
      X = cur.X[lane];
      Y = cur.Y[lane];
      Ux = cur.Ux[lane];
      Uy = cur.Uy[lane];
      R = pc.R[lane];
    }
  };
  auto gather = [&]() -> bool {
    if (!SCAN || ptile) return false;
    // read after the population loads are issued (a scalar load, whose
    // wait would otherwise hold them back)
    if (counted) return B.tcount[tile] != 0;
    if (t < 64) {
      bool hit = false;
      if (probe) {
        advance_position(P, X, Y, Ux, Uy);
        const BlockRanges r = block_ranges(P, X, Y, R, kBlock);
        hit = r.contains(tile);
        // a centre the band-box logic cannot place: no tile serves it
        if (r.n == 0 && tile == 0) atomicOr(flags, kFlagUnstable);
      }
      const bool any = __ballot(hit) != 0ull;
      if (t == 0) sh.tmp[0] = any ? 1 : 0;
    }
    __syncthreads();
    return sh.tmp[0] != 0;   // a particle tile: the first group's
  };
  auto part = [&](bool, int, int, C drho, C jxs, C jys, PSums<C>& S) {
    if (ptile) {
      S.S0 = sh.S[0][t]; S.S1x = sh.S[1][t]; S.S1y = sh.S[2][t];
      S.S2xx = sh.S[3][t]; S.S2yy = sh.S[4][t]; S.S2xy = sh.S[5][t];
      if (anyheld) {
        S.H0 = sh.M[0][t];
        S.H1 = sh.M[1][t];
      }
      sh.M[0][t] = drho; sh.M[1][t] = jxs; sh.M[2][t] = jys;
    }
  };
  if (!lattice_tile<PREC, OUT, NT>(P, H, fin, fout, gin, gout, hin, hout,
                                   plane, tile, macro, flags, pre, gather,
                                   part))
    return;
  if (!ptile) return;

  // ---- phase 3 (particle tiles): momentum exchange.  Each particle's share
  // of sum_i (f_i - f*_i) e_i in a cell is f_s,p (rho u_s - j*); the block
  // sums of minus that (force) and of its moment about the centre (torque)
  // go to the particle's partial slot of this tile.  Pass 2 adds the
  // correction of the scaled shares (cells covered more than once; rare).
  // The shares come from phase 1 (recomputed only past kShareCache per
  // cell); every slot's sums are reduced per wave into LDS, then the four
  // waves in order by one thread per slot.
  const C drho = sh.M[0][t], jxs = sh.M[1][t], jys = sh.M[2][t];
  const C rho0s = H.rho0s;
  const C S0raw = sh.S0raw[t];
  const int cnt = sh.bp.cnt;
  const int nreach = act0 ? sh.nreach[t] : 0;
  const int ncached = nreach < kShareCache ? nreach : kShareCache;
  const int wv = t >> 6;
  for (int pass = 0; pass < 2; ++pass) {
    // pass 2 only where shares were scaled: never with one particle (its
    // share of a cell is at most 1), so that tile skips the barrier
    if (pass == 1 && (cnt <= 1 || !__syncthreads_or(act0 && S0raw > (C)1)))
      break;
    const bool over = pass == 1 && S0raw > (C)1;
    const C inv = over ? (C)1 / S0raw : (C)1;
    int e = 0;                       // next cached share of this cell
    // slots whose band box misses the wave: nothing to add
    if (lane < cnt && !((wmask >> lane) & 1ull)) {
      sh.red[lane][wv][0] = 0.0;
      sh.red[lane][wv][1] = 0.0;
      sh.red[lane][wv][2] = 0.0;
    }
    for (unsigned long long m = wmask; m; m &= m - 1) {
      const int k = __ffsll((long long)m) - 1;
      bool has = false;
      C a = (C)0;
      if (e < ncached && sh.slot[e][t] == k) {
        a = sh.share[e][t];
        has = true;
        ++e;
      } else if (e == kShareCache && nreach > kShareCache) {
        SlotGeom sg;                 // past the cache: recompute
        if (particle_geometry<ELL>(P, sh.bp.X[k], sh.bp.Y[k], sh.bp.R[k],
                              sh.bp.Rb[k], sh.bp.cth[k], sh.bp.sth[k],
                              sh.bp.Ux[k], sh.bp.Uy[k], sh.bp.Om[k], cx, cy,
                              sg)) {
          a = (C)sg.fs;
          has = true;
        }
      }
      const bool add = has && (pass == 0 || over);
      double cfx = 0.0, cfy = 0.0, ctz = 0.0;
      if (add) {
        double rx, ry, usx, usy;
        particle_motion(P, sh.bp.X[k], sh.bp.Y[k], sh.bp.Ux[k], sh.bp.Uy[k],
                        sh.bp.Om[k], cx, cy, rx, ry, usx, usy);
        const C ux = (C)usx, uy = (C)usy;
        const double kk = pass == 0 ? 1.0 : (double)(inv - (C)1);
        // rho u_s - j* with rho = rho_0 + drho: the O(1) parts cancel
        // before anything of order one is rounded
        const double dpx = (double)(a * ((rho0s * ux - jxs) + drho * ux));
        const double dpy = (double)(a * ((rho0s * uy - jys) + drho * uy));
        cfx = -dpx * kk;
        cfy = -dpy * kk;
        ctz = -(rx * dpy - ry * dpx) * kk;
      }
      if (__ballot(add) != 0ull) {   // uniform in the wave
        cfx = wave_sum_last(cfx);
        cfy = wave_sum_last(cfy);
        ctz = wave_sum_last(ctz);
      }
      if (lane == 63) {
        sh.red[k][wv][0] = cfx;
        sh.red[k][wv][1] = cfy;
        sh.red[k][wv][2] = ctz;
      }
    }
    __syncthreads();
    if (t < cnt) {
      const double(*r)[3] = sh.red[t];
      const double fx = ((r[0][0] + r[1][0]) + r[2][0]) + r[3][0];
      const double fy = ((r[0][1] + r[1][1]) + r[2][1]) + r[3][1];
      const double tz = ((r[0][2] + r[1][2]) + r[2][2]) + r[3][2];
      double* o = partial + (size_t)sh.bp.slot[t] * kRedVals;
      if (pass == 0) {
        o[0] = fx; o[1] = fy; o[2] = tz;
      } else {
        o[0] += fx; o[1] += fy; o[2] += tz;
      }
    }
  }
}

// Two plain tiles per block (the 16-bit forms): each lane issues the loads
// of its cell in both tiles before it computes either.  The 16-bit forms
// move half the FP32 bytes per cell with the same arithmetic; with one cell
// per lane a wave has too few bytes in flight to cover the memory latency,
// with two it has as many as an FP32 wave.  tB may lie past the last tile
// (its lanes then only load a valid cell).  Scan form: a tile a particle
// reaches is left to the particle group, as in step_task (COUNTED as
// there).
template <int PREC, bool OUT, bool SCAN, bool COUNTED = false>
__device__ __forceinline__ void pair_task(
    const Params& P, const Hot<typename Prec<PREC>::C>& H, const StepBufs& B,
    int tA, int tB) {
  typedef typename Prec<PREC>::C C;
  typedef typename Prec<PREC>::S S;
  typedef typename Prec<PREC>::H HT;
  const S* __restrict__ fin = (const S*)B.fi;
  S* __restrict__ fout = (S*)B.fo;
  const S* __restrict__ gin = (const S*)B.gi;
  S* __restrict__ gout = (S*)B.go;
  const HT* __restrict__ hin = (const HT*)B.hin;
  HT* __restrict__ hout = (HT*)B.hout;
  const size_t plane = B.plane;
  double* __restrict__ macro = B.macro;
  int* flags = B.flags;
  const int lane = threadIdx.x & 63;
  const bool counted = COUNTED && SCAN;
  const bool probe = !COUNTED && SCAN && lane < P.np;
  double X = 0.0, Y = 0.0, Ux = 0.0, Uy = 0.0, R = 0.0;
  if (counted && threadIdx.x == 0) {
    B.tcount_clear[tA] = 0;
    if (tB < P.nblocks) B.tcount_clear[tB] = 0;
  }
  if (probe) {
    X = B.cur.X[lane];
    Y = B.cur.Y[lane];
    Ux = B.cur.Ux[lane];
    Uy = B.cur.Uy[lane];
    R = B.pc.R[lane];
  }
  CellLoad<PREC> a, b;
  load_cell<PREC>(P, fin, gin, hin, plane, tA, a);
  load_cell<PREC>(P, fin, gin, hin, plane, tB, b);
  bool skipA = false, skipB = tB >= P.nblocks;
  if (counted) {   // read after the loads, as in step_task
    skipA = B.tcount[tA] != 0;
    skipB = skipB || B.tcount[tB] != 0;
  } else if (SCAN) {
    bool ha = false, hb = false;
    if (probe) {
      advance_position(P, X, Y, Ux, Uy);
      const BlockRanges r = block_ranges(P, X, Y, R, kBlock);
      ha = r.contains(tA);
      hb = r.contains(tB);
      // a centre the band-box logic cannot place: no tile serves it
      if (r.n == 0 && (tA == 0 || tB == 0)) atomicOr(flags, kFlagUnstable);
    }
    skipA = __ballot(ha) != 0ull;
    skipB = skipB || __ballot(hb) != 0ull;
  }
  auto none = [](bool, int, int, C, C, C, PSums<C>&) {};
  if (!skipA)
    update_cell<PREC, OUT, false>(P, H, a, fout, gout, hout, plane, macro,
                                  flags, none);
  if (!skipB)
    update_cell<PREC, OUT, false>(P, H, b, fout, gout, hout, plane, macro,
                                  flags, none);
}

static inline unsigned blocks_for(long n, int per) {
  return (unsigned)((n + per - 1) / per);
}

}  // namespace vlb
