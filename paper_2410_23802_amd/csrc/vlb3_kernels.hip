// vlb3_kernels.hip -- gfx950 kernels of the three-dimensional step: the
// sphere pass (momentum-exchange sums, Newton-Euler update), the lattice
// step (geometry, D3Q19 flow, D3Q7 energy, per-tile partial sums), the
// initial state and the per-sphere thermal outputs.
//
// Layout: every population is a plane of N doubles (structure of arrays,
// f[q][k][j][i]), pulled by one thread per cell; a tile is 256 consecutive
// cells.  The spheres (at most 64, one per lane) are tested against each
// tile's bounding box by every wave, which keeps the candidates of a tile
// as a wave-uniform bit mask; the per-(sphere, tile) sums are reduced over
// the block in a fixed order and summed by the sphere pass in tile order.
#include <utility>

#include "vlb3_internal.h"
#include "vlb_device.h"   // covered_share: exact disk-cell area

namespace vlb3 {

// ---------------------------------------------------------------------------
// Lattices

__host__ __device__ constexpr int ex(int q) {
  constexpr int t[kQ] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1,
                         1, -1, 1, -1, 0, 0, 0, 0};
  return t[q];
}
__host__ __device__ constexpr int ey(int q) {
  constexpr int t[kQ] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1,
                         0, 0, 0, 0, 1, -1, 1, -1};
  return t[q];
}
__host__ __device__ constexpr int ez(int q) {
  constexpr int t[kQ] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0,
                         1, -1, -1, 1, 1, -1, -1, 1};
  return t[q];
}
// opposite directions come in consecutive pairs (1, 2), (3, 4), ...
__host__ __device__ constexpr int opp(int q) {
  return q == 0 ? 0 : (q & 1) ? q + 1 : q - 1;
}
__host__ __device__ constexpr double wq(int q) {
  return q == 0 ? 1.0 / 3.0 : q < 7 ? 1.0 / 18.0 : 1.0 / 36.0;
}
// energy lattice (D3Q7): w_0 = 1/4, w_i = 1/8, c_s^2 = 1/4
constexpr double kW0G = 0.25, kW1G = 0.125, kCs2G = 0.25;

// The orthogonal D3Q19 moment basis: row k evaluated at velocity q.
__host__ __device__ constexpr double mrow(int k, int q) {
  const double x = ex(q), y = ey(q), z = ez(q), c2 = x * x + y * y + z * z;
  switch (k) {
    case 0: return 1.0;
    case 1: return 19.0 * c2 - 30.0;
    case 2: return (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    case 3: return x;
    case 4: return (5.0 * c2 - 9.0) * x;
    case 5: return y;
    case 6: return (5.0 * c2 - 9.0) * y;
    case 7: return z;
    case 8: return (5.0 * c2 - 9.0) * z;
    case 9: return 3.0 * x * x - c2;
    case 10: return (3.0 * c2 - 5.0) * (3.0 * x * x - c2);
    case 11: return y * y - z * z;
    case 12: return (3.0 * c2 - 5.0) * (y * y - z * z);
    case 13: return x * y;
    case 14: return y * z;
    case 15: return x * z;
    case 16: return (y * y - z * z) * x;
    case 17: return (z * z - x * x) * y;
    default: return (x * x - y * y) * z;
  }
}
__host__ __device__ constexpr double mnorm(int k) {
  double s = 0.0;
  for (int q = 0; q < kQ; ++q) s += mrow(k, q) * mrow(k, q);
  return s;
}

// The transforms with every entry a compile-time constant: row K of M
// dotted with a (zero entries skipped), and column Q of M^T dotted with b.
template <int K, int Q>
struct Basis {
  static constexpr double v = mrow(K, Q);
};

template <int K, int Q = 0>
__device__ __forceinline__ double row_dot(const double (&a)[kQ]) {
  if constexpr (Q == kQ) {
    return 0.0;
  } else if constexpr (Basis<K, Q>::v == 0.0) {
    return row_dot<K, Q + 1>(a);
  } else {
    return Basis<K, Q>::v * a[Q] + row_dot<K, Q + 1>(a);
  }
}

template <int Q, int K = 0>
__device__ __forceinline__ double col_dot(const double (&b)[kQ]) {
  if constexpr (K == kQ) {
    return 0.0;
  } else if constexpr (Basis<K, Q>::v == 0.0) {
    return col_dot<Q, K + 1>(b);
  } else {
    return Basis<K, Q>::v * b[K] + col_dot<Q, K + 1>(b);
  }
}

// Relaxation rate of moment K: the conserved moments (rho, j) 1; the
// energy-like even moments (e, epsilon, pi_xx, pi_ww) 1.25; the shear
// moments s_nu; the odd moments (q, m) s_q.
template <int K>
__device__ __forceinline__ double rate(double snu, double sq) {
  if constexpr (K == 0 || K == 3 || K == 5 || K == 7) return 1.0;
  else if constexpr (K == 4 || K == 6 || K == 8 || K >= 16) return sq;
  else if constexpr (K == 9 || K == 11 || (K >= 13 && K <= 15)) return snu;
  else return 1.25;
}

// dm_K = -s_K (M a)_K / |row K|^2, so that M^-1 diag(-s) M a = M^T dm
template <size_t... K>
__device__ __forceinline__ void relax_moments(const double (&a)[kQ],
                                              double (&dm)[kQ], double snu,
                                              double sq,
                                              std::index_sequence<K...>) {
  ((dm[K] = -rate<(int)K>(snu, sq) * row_dot<(int)K>(a) *
            (1.0 / mnorm((int)K))),
   ...);
}

// f'_Q = (base of Q) + (M^T dm)_Q, stored as each is formed (no array of
// 19 results held)
// (NT: stored non-temporally)
template <bool NT, class T>
__device__ __forceinline__ void put(T* p, double v) {
  if constexpr (NT)
    __builtin_nontemporal_store((T)v, p);
  else
    *p = (T)v;
}

// a population in the storage form: FP64 as it is, FP32 less its shift
template <bool NT, class T>
__device__ __forceinline__ void put_pop(T* p, double v, double shift) {
  if constexpr (sizeof(T) < sizeof(double)) v -= shift;
  put<NT>(p, v);
}

// (stored minus shift[Q]: the storage form's reference)
template <bool NT, class T, class Base, size_t... Q>
__device__ __forceinline__ void back_transform_store(
    const double (&dm)[kQ], Base base, T* __restrict__ out, size_t N,
    size_t c, const double* shift, std::index_sequence<Q...>) {
  (put_pop<NT>(out + Q * N + c, base((int)Q) + col_dot<(int)Q>(dm), shift[Q]),
   ...);
}

// ---------------------------------------------------------------------------
// Geometry (integer decisions without fused operations, as the oracle's)

__device__ __forceinline__ double near_copy(double Xp, double node, double L,
                                            int per) {
  if (!per) return Xp;
  if (node - Xp > 0.5 * L) return Xp + L;
  if (Xp - node > 0.5 * L) return Xp - L;
  return Xp;
}

// the closed cell meets the open ball
__device__ __noinline__ bool in_band(double X, double Y, double Z, double R,
                                     int i, int j, int k) {
#pragma clang fp contract(off)
  const double P[3] = {X, Y, Z};
  const int lo[3] = {i, j, k};
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    double d = 0.0;
    const double e = (double)lo[a] - P[a], f = P[a] - (double)(lo[a] + 1);
    if (e > d) d = e;
    if (f > d) d = f;
    s += d * d;
  }
  return s < R * R;
}

// the whole cell lies in the closed ball
__device__ __noinline__ bool wholly_inside(double X, double Y, double Z,
                                           double R, int i, int j, int k) {
#pragma clang fp contract(off)
  const double P[3] = {X, Y, Z};
  const int lo[3] = {i, j, k};
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double e = P[a] - (double)lo[a], f = (double)(lo[a] + 1) - P[a];
    const double d = e > f ? e : f;
    s += d * d;
  }
  return s <= R * R;
}

// Gauss-Legendre rule on [0, 1] (host-computed)
constexpr int kGL = 16;
__constant__ double gl_x[kGL], gl_w[kGL];

// Volume of the sphere (centre X, Y, Z, radius R) inside cell (i, j, k):
// the exact cross-sectional area (a disk of radius sqrt(R^2 - z^2) in the
// cell's square) integrated over z.  The area is analytic in z except
// where the section's circle passes a line or a corner of the square or
// shrinks to a point (z* = +-sqrt(R^2 - d^2), +-R), where it has
// half-integer powers.  [k, k+1] is split at the z* inside it; on a piece
// the substitution z - z* ~ t^2 at an end that is such a point makes the
// integrand smooth in t; a z* just outside a piece (closer than 0.6 of its
// length) is met by geometric grading of the sub-intervals towards it
// (ratio 3: each at least half its own length away); 16-point
// Gauss-Legendre on every sub-interval.  Deterministic: about 95 area
// evaluations per partly covered cell of a sphere of radius 3 to 10 (with
// ratio 2 up to half the piece: 125), within 1e-14 of the exact volume
// for radii 0.5 to 14 in tests.
//
// The section is the disk of radius^2 r2 centred at the origin against the
// unit square [x0, x0 + 1] x [y0, y0 + 1] (coordinates relative to the
// centre), by Green's theorem over the square's edges taken
// counter-clockwise: triangles from the centre to the parts of the edges
// inside the circle, circular sectors for the parts outside.  An edge runs
// from p along a unit axis d, so the circle meets it at
// s = -p.d +- sqrt(r2 - h^2) (h the edge line's distance from the centre)
// with no division, and the sectors' vectors follow from p, d and s.  Each
// sector of angle arg(conj(u) v) enters as the complex factor u.v + i u x v;
// with the centre outside the closed
// square the net angle lies in (-pi, pi) and one atan2 of the product
// gives it, otherwise (the square's column of cells) each edge's product
// takes its own (an edge's sectors subtend less than pi from a centre
// inside the square).  One atan2 call site serves both, so the code is
// emitted once.
// (No rescaling is needed: a factor's modulus is |u| |v| <= (R + 2)^2 and
// an edge contributes at most two, so eight factors stay far from
// overflow; a vanishing factor, a corner at the centre, is left out.  A
// form with selects instead of branches measured 5 % slower.)
__device__ __forceinline__ void cmul(double cr, double ci, double& zr,
                                     double& zi) {
  if (cr == 0.0 && ci == 0.0) return;
  const double r = zr * cr - zi * ci, im = zr * ci + zi * cr;
  zr = r;
  zi = im;
}

// edge from p (|p|^2 = pp) along the unit axis d: b = p.d, hh = h^2 =
// |p|^2 - b^2, cr = p x d; adds its triangle part to tri and its sectors'
// factors to (zr, zi)
__device__ __forceinline__ void sec_edge(double b, double hh, double cr,
                                         double pp, double r2, double& tri,
                                         double& zr, double& zi) {
  const double disc = r2 - hh;
  double s1 = 1.0, s2 = 0.0;
  if (disc > 0.0) {
    const double w = sqrt(disc);
    s1 = fmin(fmax(-b - w, 0.0), 1.0);
    s2 = fmin(fmax(-b + w, 0.0), 1.0);
  }
  if (!(s1 < s2)) {              // the whole edge outside: p -> p + d
    cmul(pp + b, cr, zr, zi);
    return;
  }
  tri += 0.5 * (s2 - s1) * cr;
  if (s1 > 0.0) cmul(pp + s1 * b, s1 * cr, zr, zi);
  if (s2 < 1.0) cmul(pp + (1.0 + s2) * b + s2, (1.0 - s2) * cr, zr, zi);
}

__device__ __forceinline__ double unit_square_section(double x0, double y0,
                                                      double r2) {
  const double x1 = x0 + 1.0, y1 = y0 + 1.0;
  const bool own = x0 <= 0.0 && x1 >= 0.0 && y0 <= 0.0 && y1 >= 0.0;
  const double xx0 = x0 * x0, xx1 = x1 * x1, yy0 = y0 * y0, yy1 = y1 * y1;
  double tri = 0.0;
  // per edge products (own) or the running product in slot 0
  double ar = 1.0, ai = 0.0, br = 1.0, bi = 0.0, cr = 1.0, ci = 0.0;
  double dr = 1.0, di = 0.0;
  double xr, xi;
  sec_edge(x0, yy0, -y0, xx0 + yy0, r2, tri, ar, ai);      // bottom, +x
  xr = own ? 1.0 : ar; xi = own ? 0.0 : ai;
  sec_edge(y0, xx1, x1, xx1 + yy0, r2, tri, xr, xi);      // right, +y
  if (own) { br = xr; bi = xi; } else { ar = xr; ai = xi; }
  xr = own ? 1.0 : ar; xi = own ? 0.0 : ai;
  sec_edge(-x1, yy1, y1, xx1 + yy1, r2, tri, xr, xi);     // top, -x
  if (own) { cr = xr; ci = xi; } else { ar = xr; ai = xi; }
  xr = own ? 1.0 : ar; xi = own ? 0.0 : ai;
  sec_edge(-y1, xx0, -x0, xx0 + yy1, r2, tri, xr, xi);    // left, -y
  if (own) { dr = xr; di = xi; } else { ar = xr; ai = xi; }
  double ang = 0.0;
  const int nang = own ? 4 : 1;
#pragma unroll 1
  for (int e = 0; e < nang; ++e) {
    ang += atan2(ai, ar);
    ar = br; ai = bi;
    br = cr; bi = ci;
    cr = dr; ci = di;
  }
  return fmin(fmax(tri + 0.5 * r2 * ang, 0.0), 1.0);
}

// (x0, y0: the cell's lower corner relative to the centre)
__device__ __forceinline__ double section_area(double x0, double y0, double R,
                                               double z) {
  const double r2 = (R - z) * (R + z);
  return r2 > 0.0 ? unit_square_section(x0, y0, r2) : 0.0;
}

// one Gauss-Legendre sub-interval [p, q] (nodes g0, g0 + gs, ... of the
// rule; ONE: the node g0 only); sp / sq: p / q is a singular end
template <bool ONE>
__device__ __forceinline__ double gl_piece(double x0, double y0, double R,
                                           double p, double q, bool sp,
                                           bool sq, int g0, int gs) {
  const double L = q - p;
  double sum = 0.0;
  for (int g = g0; g < (ONE ? g0 + 1 : kGL); g += gs) {
    const double t = gl_x[g];
    double z, dz;
    if (sp && sq) {
      z = p + L * (t * t * (3.0 - 2.0 * t));
      dz = 6.0 * t * (1.0 - t) * L;
    } else if (sp) {
      z = p + L * t * t;
      dz = 2.0 * t * L;
    } else if (sq) {
      const double s = 1.0 - t;
      z = q - L * s * s;
      dz = 2.0 * s * L;
    } else {
      z = p + L * t;
      dz = L;
    }
    sum += gl_w[g] * section_area(x0, y0, R, z) * dz;
  }
  return sum;
}

// The sub-intervals of the volume of the sphere (centre X, Y, Z, radius R)
// in cell (i, j, k), in order: emit(p, q, sp, sq) for each (z relative to
// the centre; sp / sq: p / q is a singular end), until it returns false.
// One flat loop with a single emit site.
template <class Emit>
__device__ __forceinline__ void walk_subintervals(double X, double Y,
                                                  double Z, double R, int i,
                                                  int j, int k, Emit emit) {
  constexpr double kNone = 1e300;
  const double a0 = (double)i - X, a1 = a0 + 1.0;
  const double b0 = (double)j - Y, b1 = b0 + 1.0;
  const double zlo = (double)k - Z, zhi = (double)(k + 1) - Z;
  const double lo = fmax(zlo, -R), hi = fmin(zhi, R);
  if (!(lo < hi)) return;
  // the points where the area is not analytic are +-zp[m] (absent ones:
  // zp = kNone); fixed-size and fully unrolled, so they stay in registers
  const double d2[8] = {a0 * a0, a1 * a1, b0 * b0, b1 * b1,
                        a0 * a0 + b0 * b0, a0 * a0 + b1 * b1,
                        a1 * a1 + b0 * b0, a1 * a1 + b1 * b1};
  double zp[9];
  zp[0] = R;
#pragma unroll
  for (int m = 0; m < 8; ++m)
    zp[m + 1] = d2[m] < R * R ? sqrt(R * R - d2[m]) : kNone;
  // the nearest singular point above / below x (kNone / -kNone: none)
  auto above = [&](double x) {
    double r = kNone;
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      if (zp[m] > x) r = fmin(r, zp[m]);
      if (-zp[m] > x) r = fmin(r, -zp[m]);
    }
    return r;
  };
  auto below = [&](double x) {
    double r = -kNone;
#pragma unroll
    for (int m = 0; m < 9; ++m) {
      if (zp[m] < x) r = fmax(r, zp[m]);
      if (-zp[m] < x) r = fmax(r, -zp[m]);
    }
    return r;
  };
  // Pieces [u, v] run between consecutive breakpoints (lo, hi and the
  // singular points between them).  On a piece: sub-intervals graded
  // towards u (phase 0), then towards v (phase 1), then the last one
  // (phase 2); phase 3 starts the next piece.
  constexpr double kGrade = 0.6;
  double u = lo, v = lo, L = 0.0, db = 0.0, da = 0.0, s = 0.0;
  double sk = 0.0;
  double cur = lo;
  bool cur_sing = false, sv = false;
  int ph = 3, kk = 0;
  for (;;) {
    if (ph == 3) {
      u = v;
      if (!(u < hi)) break;
      v = fmin(hi, above(u));
      L = v - u;
      db = u - below(u);
      da = above(v) - v;
      // The ends of the piece are singular where they are singular points
      // (not a face); one within 1e-9 of the piece's length from an end
      // counts as at it (the substitution then meets it; grading would
      // take ~30 halvings).
      cur_sing = u != zlo || db <= 1e-9 * L;
      sv = v != zhi || da <= 1e-9 * L;
      cur = u;
      // graded boundaries at d (3^m - 1) from the end, d the singular
      // point's distance, while below kGrade L; towards v: kk of them, the
      // farthest sk
      kk = 0;
      if (da > 1e-9 * L)
        for (double t = 2.0 * da; t < kGrade * L; t = 3.0 * t + 2.0 * da) {
          ++kk;
          sk = t;
        }
      s = 2.0 * db;
      ph = db > 1e-9 * L && s < kGrade * L ? 0 : kk > 0 ? 1 : 2;
    }
    const double q = ph == 0 ? u + s : ph == 1 ? v - sk : v;
    if (!emit(cur, q, cur_sing, ph == 2 && sv)) return;
    cur = q;
    cur_sing = false;
    if (ph == 0) {
      s = 3.0 * s + 2.0 * db;
      if (!(s < kGrade * L)) ph = kk > 0 ? 1 : 2;
    } else if (ph == 1) {
      sk = (sk - 2.0 * da) / 3.0;
      if (--kk < 1) ph = 2;
    } else {
      ph = 3;
    }
  }
}

// The whole volume on one lane (all nodes of every sub-interval).
__device__ __forceinline__ double volume_all_nodes(double X, double Y,
                                                   double Z, double R, int i,
                                                   int j, int k) {
  const double x0 = (double)i - X, y0 = (double)j - Y;
  double V = 0.0;
  walk_subintervals(X, Y, Z, R, i, j, k,
                    [&](double p, double q, bool sp, bool sq) {
                      V += gl_piece<false>(x0, y0, R, p, q, sp, sq, 0, 1);
                      return true;
                    });
  return V;
}

__device__ __forceinline__ double sphere_cell_volume(double X, double Y,
                                                     double Z, double R, int i,
                                                     int j, int k) {
  return fmin(fmax(volume_all_nodes(X, Y, Z, R, i, j, k), 0.0), 1.0);
}

// The box of a tile (cells b*256 .. b*256+255), as cell-coordinate
// intervals; a tile that wraps a row or a plane takes the whole extent of
// the axes below.
__device__ __forceinline__ void tile_box(const Params3& P, int b, int lo[3],
                                         int hi[3]) {
  const int c0 = b * kBlock, c1 = min(P.N, c0 + kBlock) - 1;
  const int nxy = P.nx * P.ny;
  const int k0 = c0 / nxy, k1 = c1 / nxy;
  const int j0 = (c0 - k0 * nxy) / P.nx, j1 = (c1 - k1 * nxy) / P.nx;
  const int i0 = c0 - k0 * nxy - j0 * P.nx, i1 = c1 - k1 * nxy - j1 * P.nx;
  lo[2] = k0; hi[2] = k1 + 1;
  if (k0 == k1) {
    lo[1] = j0; hi[1] = j1 + 1;
    if (j0 == j1) { lo[0] = i0; hi[0] = i1 + 1; }
    else { lo[0] = 0; hi[0] = P.nx; }
  } else {
    lo[1] = 0; hi[1] = P.ny; lo[0] = 0; hi[0] = P.nx;
  }
}

// Distance^2 from a centre to a box, through the nearest periodic copy.
__device__ __forceinline__ bool sphere_meets_tile(const Params3& P,
                                                  const double c[3], double R,
                                                  int b) {
#pragma clang fp contract(off)
  int lo[3], hi[3];
  tile_box(P, b, lo, hi);
  const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
  double s = 0.0;
  for (int a = 0; a < 3; ++a) {
    double best = 1e300;
    for (int sh = -1; sh <= 1; ++sh) {
      if (sh != 0 && !P.per[a]) continue;
      const double x = c[a] + sh * L[a];
      const double d = fmax(0.0, fmax((double)lo[a] - x, x - (double)hi[a]));
      best = fmin(best, d);
    }
    s += best * best;
  }
  return s < R * R;
}

// Candidate spheres of tile b: bit p set if sphere p may reach it (every
// wave computes the same mask).
__device__ __forceinline__ unsigned long long tile_candidates(
    const Params3& P, const double* __restrict__ S, const double* __restrict__ C,
    int b) {
  const int lane = threadIdx.x & 63;
  bool hit = false;
  if (lane < P.np) {
    const double c[3] = {S[fX * P.np + lane], S[fY * P.np + lane],
                         S[fZ * P.np + lane]};
    hit = sphere_meets_tile(P, c, C[cR * P.np + lane], b);
  }
  return __ballot(hit);
}

// The spheres reaching cell (i, j, k): ids and shares f_s,p in ascending
// sphere order (scaled to sum to one where they exceed it), and f_s.
struct CellGeo {
  int cnt;
  int id[kMaxK];
  double w[kMaxK];
  double fs;
};

__device__ __forceinline__ void cell_geometry(const Params3& P,
                                              const double* __restrict__ S,
                                              const double* __restrict__ C,
                                              unsigned long long mask, int i,
                                              int j, int k, CellGeo& g,
                                              int* flags) {
  g.cnt = 0;
  double sum = 0.0;
  const double node[3] = {i + 0.5, j + 0.5, k + 0.5};
  const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
  for (unsigned long long m = mask; m; m &= m - 1) {
    const int p = __ffsll((long long)m) - 1;
    const double R = C[cR * P.np + p];
    double c[3];
    for (int a = 0; a < 3; ++a)
      c[a] = near_copy(S[(fX + a) * P.np + p], node[a], L[a], P.per[a]);
    if (!in_band(c[0], c[1], c[2], R, i, j, k)) continue;
    if (g.cnt >= P.kmax) {
      if (flags) atomicOr(flags, kFlagOverlap);
      continue;
    }
    const double w = wholly_inside(c[0], c[1], c[2], R, i, j, k)
                         ? 1.0
                         : sphere_cell_volume(c[0], c[1], c[2], R, i, j, k);
    g.id[g.cnt] = p;
    g.w[g.cnt] = w;
    ++g.cnt;
  }
  for (int n = 0; n < kMaxK; ++n)
    if (n < g.cnt) sum += g.w[n];
  if (sum > 1.0) {
    for (int n = 0; n < kMaxK; ++n)
      if (n < g.cnt) g.w[n] /= sum;
    sum = 1.0;
  }
  g.fs = sum;
}

// u_s = U + Omega x (x - X) at the node, through the nearest copy
__device__ __forceinline__ void solid_velocity(const Params3& P,
                                               const double* __restrict__ S,
                                               int p, int i, int j, int k,
                                               double us[3], double r[3]) {
  const double node[3] = {i + 0.5, j + 0.5, k + 0.5};
  const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
  for (int a = 0; a < 3; ++a)
    r[a] = node[a] - near_copy(S[(fX + a) * P.np + p], node[a], L[a], P.per[a]);
  const double Ox = S[fOx * P.np + p], Oy = S[fOy * P.np + p],
               Oz = S[fOz * P.np + p];
  us[0] = S[fU * P.np + p] + (Oy * r[2] - Oz * r[1]);
  us[1] = S[fV * P.np + p] + (Oz * r[0] - Ox * r[2]);
  us[2] = S[fW * P.np + p] + (Ox * r[1] - Oy * r[0]);
}

__device__ __forceinline__ double feq_q(int q, double rho, double ux,
                                        double uy, double uz, double u2) {
  const double eu = ex(q) * ux + ey(q) * uy + ez(q) * uz;
  return wq(q) * rho * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * u2);
}

// wave sum of a double (fixed butterfly order: every lane ends with the
// same value)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Initial state

// T: the storage type of the populations and the carrier
template <class T>
__global__ __launch_bounds__(kBlock) void k3_init(
    const Params3 P, T* __restrict__ f, T* __restrict__ g,
    T* __restrict__ h, double* __restrict__ macro,
    const double* __restrict__ S, const double* __restrict__ C, int* flags) {
  const unsigned long long mask = tile_candidates(P, S, C, blockIdx.x);
  const int c = blockIdx.x * kBlock + threadIdx.x;
  if (c >= P.N) return;
  const int nxy = P.nx * P.ny, k = c / nxy, j = (c - k * nxy) / P.nx,
            i = c - k * nxy - j * P.nx;
  CellGeo geo;
  cell_geometry(P, S, C, mask, i, j, k, geo, flags);
  const double fs = geo.fs;
  double u[3] = {(1.0 - fs) * P.init_u[0], (1.0 - fs) * P.init_u[1],
                 (1.0 - fs) * P.init_u[2]};
  double eps = (1.0 - fs) * P.cv_f * P.init_T;
  for (int n = 0; n < kMaxK; ++n) {
    if (n >= geo.cnt) break;
    double us[3], r[3];
    solid_velocity(P, S, geo.id[n], i, j, k, us, r);
    for (int a = 0; a < 3; ++a) u[a] += geo.w[n] * us[a];
    eps += geo.w[n] * P.cv_s * C[cTinit * P.np + geo.id[n]];
  }
  const double cv = (1.0 - fs) * P.cv_f + fs * P.cv_s, Tc = eps / cv;
  const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
#pragma unroll
  for (int q = 0; q < kQ; ++q)
    put_pop<false>(f + (size_t)q * P.N + c,
                   feq_q(q, P.rho0, u[0], u[1], u[2], u2), P.fshift[q]);
  put_pop<false>(g + c, eps - (1.0 - kW0G) * P.cref * Tc, P.gshift[0]);
#pragma unroll
  for (int q = 1; q < kQG; ++q)
    put_pop<false>(g + (size_t)q * P.N + c, kW1G * P.cref * Tc, P.gshift[q]);
  put<false>(h + c, 2.0 * fs);
  const double mv[kMacro] = {P.rho0, u[0], u[1], u[2], Tc, fs, 0.0};
#pragma unroll
  for (int m = 0; m < kMacro; ++m) macro[(size_t)m * P.N + c] = mv[m];
}

// ---------------------------------------------------------------------------
// Sphere pass: one block per sphere.  The momentum-exchange sums of the
// last lattice step (tiles thread-strided, then fixed wave and block
// trees), then (update) the Newton-Euler step of eq. particle with the
// inside-fluid terms of eq. inside.fluid and the repulsion, into nxt.

__global__ __launch_bounds__(kBlock) void k3_particles(
    const Params3 P, double* __restrict__ cur, double* __restrict__ nxt,
    const double* __restrict__ C, const double* __restrict__ partial,
    const unsigned long long* __restrict__ tmask, int have, int update) {
  __shared__ double red[kBlock / 64][kPartial];
  __shared__ double sp[4][kMaxSpheres];   // positions and radii, step n
  const int p = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int np = P.np;
  if (t < np) {
    for (int a = 0; a < 3; ++a) sp[a][t] = cur[(fX + a) * np + t];
    sp[3][t] = C[cR * np + t];
  }
  double acc[kPartial] = {0, 0, 0, 0, 0, 0};
  if (have) {   // the tiles whose candidates included the sphere
    // the masks of kBatch tiles are loaded together, then the partials of
    // the hits (one dependent round trip per batch, not per tile)
    constexpr int kBatch = 8;
    for (int b0 = t; b0 < P.nblocks; b0 += kBatch * kBlock) {
      unsigned long long m[kBatch];
#pragma unroll
      for (int u = 0; u < kBatch; ++u) {
        const int b = b0 + u * kBlock;
        m[u] = b < P.nblocks ? tmask[b] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < kBatch; ++u)
        if ((m[u] >> p) & 1ull) {
          const int b = b0 + u * kBlock;
          for (int v = 0; v < kPartial; ++v)
            acc[v] += partial[((size_t)p * P.nblocks + b) * kPartial + v];
        }
    }
  }
  for (int v = 0; v < kPartial; ++v) {
    const double s = wave_sum(acc[v]);
    if (lane == 0) red[wv][v] = s;
  }
  __syncthreads();
  if (wv != 0) return;
  // repulsion (positions at n) from the other spheres, one per lane
  double Fr[3] = {0.0, 0.0, 0.0};
  if (update && P.zeta > 0.0) {
    const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
    const double Xp[3] = {sp[0][p], sp[1][p], sp[2][p]};
    if (lane < np && lane != p) {
      double r[3], d2 = 0.0;
      for (int a = 0; a < 3; ++a) {
        r[a] = Xp[a] - near_copy(sp[a][lane], Xp[a], L[a], P.per[a]);
        d2 += r[a] * r[a];
      }
      const double d = sqrt(d2), reach = sp[3][p] + sp[3][lane] + P.zeta;
      if (d < reach && d > 0.0) {
        const double w = (reach - d) / P.zeta, mag = P.k_pp * w * w;
        for (int a = 0; a < 3; ++a) Fr[a] = mag * r[a] / d;
      }
    }
    for (int a = 0; a < 3; ++a) Fr[a] = wave_sum(Fr[a]);
  }
  if (t != 0) return;
  for (int v = 0; v < kPartial; ++v)
    acc[v] = ((red[0][v] + red[1][v]) + red[2][v]) + red[3][v];
  // F = -sum f_s,p (f^eq - f*) e, T = -sum (x - X) x [the same]
  const double F[3] = {-acc[0], -acc[1], -acc[2]};
  const double T[3] = {-acc[3], -acc[4], -acc[5]};
  for (int a = 0; a < 3; ++a) {
    cur[(fFx + a) * np + p] = F[a];
    cur[(fTx + a) * np + p] = T[a];
  }
  if (!update) return;
  const double R = C[cR * np + p], rs = C[cRho * np + p];
  const double Vol = 4.0 / 3.0 * M_PI * R * R * R, M = rs * Vol;
  const double I = 0.4 * M * R * R, Min = P.rho_f * Vol, Iin = P.rho_f * I / rs;
  const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
  double X[3], U[3], O[3], Up[3], Op[3];
  for (int a = 0; a < 3; ++a) {
    X[a] = cur[(fX + a) * np + p];
    U[a] = cur[(fU + a) * np + p];
    O[a] = cur[(fOx + a) * np + p];
    Up[a] = cur[(fUp + a) * np + p];
    Op[a] = cur[(fOxp + a) * np + p];
  }
  // repulsion of the walls (the spheres' is in Fr already)
  if (P.zeta > 0.0) {
    for (int face = 0; face < 6; ++face) {
      const int a = face / 2;
      if (P.per[a]) continue;
      const double gap = (face & 1) ? L[a] - X[a] : X[a];
      const double d = 2.0 * gap, reach = 2.0 * R + P.zeta;
      if (d < reach) {
        const double w = (reach - d) / P.zeta;
        Fr[a] += ((face & 1) ? -1.0 : 1.0) * P.k_pw * w * w;
      }
    }
  }
  double nU[3] = {U[0], U[1], U[2]}, nO[3] = {O[0], O[1], O[2]};
  if (C[cFixed * np + p] == 0.0) {
    for (int a = 0; a < 3; ++a) {
      const double Fin = -Min * (U[a] - Up[a]), Tin = -Iin * (O[a] - Op[a]);
      const double Fc = (F[a] - Fin) + (rs - P.rho_f) * Vol * P.grav[a] + Fr[a];
      nU[a] = U[a] + Fc / M;
      nO[a] = O[a] + (T[a] - Tin) / I;
    }
  }
  for (int a = 0; a < 3; ++a) {
    double x = X[a] + U[a];
    if (P.per[a]) {
      if (x >= L[a]) x -= L[a];
      if (x < 0.0) x += L[a];
    }
    nxt[(fX + a) * np + p] = x;
    nxt[(fU + a) * np + p] = nU[a];
    nxt[(fOx + a) * np + p] = nO[a];
    nxt[(fUp + a) * np + p] = U[a];
    nxt[(fOxp + a) * np + p] = O[a];
    nxt[(fFx + a) * np + p] = 0.0;
    nxt[(fTx + a) * np + p] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Geometry: the spheres' shares of the cells of the tiles they may reach,
// written to gid (count in bits 0-2, sphere ids in the bytes above) and gw
// (kMaxK shares), and each tile's candidate mask to tmask.  Kernels of their
// own, so that the exact-volume quadrature holds no registers in the
// streaming kernel.
//   pass A (one block per tile): band tests; a cell a sphere covers wholly
//     takes share 1, a partly covered one becomes an item of a global list;
//   pass B (a fixed grid walking the list): each item is integrated by a
//     group of 16 lanes, one Gauss-Legendre node each.  A tile holds from
//     none to hundreds of items, so a global list balances the work that
//     per-tile groups would leave to the busiest tile.
// The step kernel scales shares that add up to more than one.

constexpr int kGroup = 16;
static_assert(kGroup == kGL, "one lane per quadrature node");

__global__ __launch_bounds__(kBlock) void k3_geometry_a(
    const Params3 P, const double* __restrict__ S, const double* __restrict__ C,
    int* __restrict__ gid, double* __restrict__ gw,
    unsigned long long* __restrict__ tmask, int* __restrict__ items,
    int* __restrict__ nitems, int* flags) {
  __shared__ double sp[4][kMaxSpheres];   // X, Y, Z, R of every sphere
  __shared__ int woff[kBlock / 64 + 1];   // the waves' item offsets
  const unsigned long long mask = tile_candidates(P, S, C, blockIdx.x);
  if (threadIdx.x == 0) tmask[blockIdx.x] = mask;     // for the step and
  if (!mask) return;                                  // the sphere pass
  const int t = threadIdx.x, lane = t & 63;
  if (t < P.np) {
    sp[0][t] = S[fX * P.np + t];
    sp[1][t] = S[fY * P.np + t];
    sp[2][t] = S[fZ * P.np + t];
    sp[3][t] = C[cR * P.np + t];
  }
  __syncthreads();
  const int c = blockIdx.x * kBlock + t;
  const int nxy = P.nx * P.ny;
  const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
  // the wave's candidates: spheres meeting the box of its 64 cells (one
  // sphere per lane), so that each cell tests only those
  unsigned long long wmask;
  {
    const int c0 = min(c - lane, P.N - 1), c1 = min(c - lane + 63, P.N - 1);
    const int k0 = c0 / nxy, k1 = c1 / nxy;
    const int j0 = (c0 - k0 * nxy) / P.nx, j1 = (c1 - k1 * nxy) / P.nx;
    int lo[3], hi[3];
    lo[2] = k0; hi[2] = k1 + 1;
    if (k0 == k1) {
      lo[1] = j0; hi[1] = j1 + 1;
      if (j0 == j1) { lo[0] = c0 - k0 * nxy - j0 * P.nx; hi[0] = c1 - k1 * nxy - j1 * P.nx + 1; }
      else { lo[0] = 0; hi[0] = P.nx; }
    } else {
      lo[1] = 0; hi[1] = P.ny; lo[0] = 0; hi[0] = P.nx;
    }
    bool hit = false;
    if (lane < P.np && ((mask >> lane) & 1ull)) {
      double ss = 0.0;
      for (int a = 0; a < 3; ++a) {
        double best = 1e300;
        for (int sh = -1; sh <= 1; ++sh) {
          if (sh != 0 && !P.per[a]) continue;
          const double x = sp[a][lane] + sh * L[a];
          best = fmin(best, fmax(0.0, fmax((double)lo[a] - x, x - (double)hi[a])));
        }
        ss += best * best;
      }
      hit = ss < sp[3][lane] * sp[3][lane];
    }
    wmask = __ballot(hit);
  }
  const bool act = c < P.N;
  const int cc = act ? c : P.N - 1;
  const int k = cc / nxy, j = (cc - k * nxy) / P.nx, i = cc - k * nxy - j * P.nx;
  const double node[3] = {i + 0.5, j + 0.5, k + 0.5};
  int cnt = 0, packed = 0, part = 0;   // part: bit s = slot s partly covered
  double w[kMaxK] = {0.0, 0.0, 0.0, 0.0};
  for (unsigned long long m = act ? wmask : 0ull; m; m &= m - 1) {
    const int p = __ffsll((long long)m) - 1;          // ascending spheres
    const double R = sp[3][p];
    double cp[3];
    for (int a = 0; a < 3; ++a)
      cp[a] = near_copy(sp[a][p], node[a], L[a], P.per[a]);
    if (!in_band(cp[0], cp[1], cp[2], R, i, j, k)) continue;
    if (cnt >= P.kmax) {
      atomicOr(flags, kFlagOverlap);
      continue;
    }
    packed |= p << (8 * cnt + 8);
    if (wholly_inside(cp[0], cp[1], cp[2], R, i, j, k)) {
#pragma unroll
      for (int s2 = 0; s2 < kMaxK; ++s2)
        if (s2 == cnt) w[s2] = 1.0;
    } else {
      part |= 1 << cnt;
    }
    ++cnt;
  }
  // the block's items: prefix sums of the per-lane counts over the wave and
  // the block, and one atomic per block on the counter of the block's
  // segment (kSegs of them: one counter for every block queued at a single
  // address and took longer than the rest of the pass)
  const int mine = __popc(part);
  int pre = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int v = __shfl_up(pre, o, 64);
    if (lane >= o) pre += v;
  }
  const int wv = t >> 6;
  if (lane == 63) woff[wv] = pre;
  __syncthreads();
  if (t == 0) {
    int acc = 0;
    for (int w2 = 0; w2 < kBlock / 64; ++w2) {
      const int n2 = woff[w2];
      woff[w2] = acc;
      acc += n2;
    }
    woff[kBlock / 64] =
        acc > 0 ? atomicAdd(&nitems[blockIdx.x % kSegs], acc) : 0;
  }
  __syncthreads();
  // room for every slot of the segment's tiles
  int* seg = items + (size_t)(blockIdx.x % kSegs) * seg_items(P);
  int at = woff[kBlock / 64] + woff[wv] + pre - mine;
  for (int s2 = 0; s2 < kMaxK; ++s2)
    if ((part >> s2) & 1) seg[at++] = c * kMaxK + s2;
  if (!act) return;
#pragma unroll
  for (int s2 = 0; s2 < kMaxK; ++s2) gw[(size_t)c * kMaxK + s2] = w[s2];
  gid[c] = packed | cnt;
}

// The exact volumes of the partly covered cell slots listed by the first
// pass, four slots per wave at a time, in passes: each 16-lane group walks
// its slot's sub-intervals into LDS (up to kCap a pass), then the wave
// evaluates the four lists together, sixteen lanes (one node each) per
// sub-interval, so that a wave takes the mean of its slots' sub-interval
// counts rather than the largest; each group adds its sub-intervals' sums
// in order (the volume does not depend on the other slots of the wave).
// Past kCap sub-intervals a slot takes further passes, its walk skipping
// those already done.
constexpr int kCap = 48;

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k3_geometry_b(
    const Params3 P, const double* __restrict__ S, const double* __restrict__ C,
    const int* __restrict__ gid, double* __restrict__ gw,
    const int* __restrict__ items, const int* __restrict__ nitems) {
  constexpr int kW = kBlock / 64, kG = 64 / kGroup;   // waves, groups
  __shared__ double sp_[kW][kG][kCap], sq_[kW][kG][kCap], sv_[kW][kG][kCap];
  __shared__ unsigned char sf_[kW][kG][kCap];
  __shared__ double cell_[kW][kG][3];                 // x0, y0, R
  __shared__ int sn_[kW][kG];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int grp = lane / kGroup, r = lane % kGroup;
  int first[kSegs + 1];                 // the segments, concatenated
  first[0] = 0;
#pragma unroll
  for (int k = 0; k < kSegs; ++k) first[k + 1] = first[k] + nitems[k];
  const int n = first[kSegs];
  const size_t seg = seg_items(P);
  const int nxy = P.nx * P.ny;
  const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
  const int nwaves = gridDim.x * kW;
  for (int it0 = (blockIdx.x * kW + wv) * kG; it0 < n; it0 += nwaves * kG) {
    const int it = it0 + grp;                            // uniform in a group
    const bool has = it < n;
    int c = 0, slot = 0, i = 0, j = 0, k = 0;
    double cp[3] = {0.0, 0.0, 0.0}, R = 0.0;
    if (has) {
      int sg = 0;
#pragma unroll
      for (int k2 = 1; k2 < kSegs; ++k2) sg += it >= first[k2];
      int base = first[0];
#pragma unroll
      for (int k2 = 1; k2 < kSegs; ++k2) base = sg == k2 ? first[k2] : base;
      const int item = items[(size_t)sg * seg + (it - base)];
      c = item / kMaxK;
      slot = item - c * kMaxK;
      const int p = (gid[c] >> (8 * slot + 8)) & 255;
      k = c / nxy;
      j = (c - k * nxy) / P.nx;
      i = c - k * nxy - j * P.nx;
      const double node[3] = {i + 0.5, j + 0.5, k + 0.5};
      for (int a = 0; a < 3; ++a)
        cp[a] = near_copy(S[(fX + a) * P.np + p], node[a], L[a], P.per[a]);
      R = C[cR * P.np + p];
      if (r == 0) {
        cell_[wv][grp][0] = (double)i - cp[0];
        cell_[wv][grp][1] = (double)j - cp[1];
        cell_[wv][grp][2] = R;
      }
    }
    double V = 0.0;
    for (int skip = 0;; skip += kCap) {
      // walk: this pass's sub-intervals of the group's slot into LDS
      int cnt = 0, idx = 0;
      bool more = false;
      if (has)
        walk_subintervals(cp[0], cp[1], cp[2], R, i, j, k,
                          [&](double p, double q, bool sp, bool sq) {
                            if (idx++ < skip) return true;
                            if (cnt == kCap) {
                              more = true;
                              return false;
                            }
                            if (r == 0) {
                              sp_[wv][grp][cnt] = p;
                              sq_[wv][grp][cnt] = q;
                              sf_[wv][grp][cnt] =
                                  (unsigned char)((sp ? 1 : 0) | (sq ? 2 : 0));
                            }
                            ++cnt;
                            return true;
                          });
      if (r == 0) sn_[wv][grp] = cnt;
      wave_lds_sync();
      // evaluate the four lists together: entry e of the concatenation by
      // group e mod kG in round e / kG
      int nn[kG], tot = 0;
#pragma unroll
      for (int g = 0; g < kG; ++g) {
        nn[g] = sn_[wv][g];
        tot += nn[g];
      }
      for (int e0 = 0; e0 < tot; e0 += kG) {            // uniform in the wave
        const int e = e0 + grp;
        double val = 0.0;
        int g = 0, l = e;
        if (e < tot) {
#pragma unroll
          for (int g2 = 0; g2 < kG - 1; ++g2)
            if (g == g2 && l >= nn[g2]) {
              l -= nn[g2];
              g = g2 + 1;
            }
          const unsigned f = sf_[wv][g][l];
          val = gl_piece<true>(cell_[wv][g][0], cell_[wv][g][1],
                               cell_[wv][g][2], sp_[wv][g][l], sq_[wv][g][l],
                               f & 1u, (f & 2u) != 0u, r, kGroup);
        }
#pragma unroll
        for (int o = kGroup / 2; o >= 1; o >>= 1) val += __shfl_xor(val, o, kGroup);
        if (e < tot && r == 0) sv_[wv][g][l] = val;
      }
      wave_lds_sync();
      for (int l = 0; l < cnt; ++l) V += sv_[wv][grp][l];   // in order
      const bool again = __ballot(more) != 0ull;
      wave_lds_sync();   // the lists are read before the next pass writes
      if (!again) break;
    }
    if (has && r == 0) gw[(size_t)c * kMaxK + slot] = fmin(fmax(V, 0.0), 1.0);
  }
}

// ---------------------------------------------------------------------------
// The lattice step

// NT (the host's nt_stores): populations and carrier stored
// non-temporally; St: their storage type (double, or float holding the
// deviations from P.fshift and P.gshift, the arithmetic in FP64 either way)
template <bool OUT, bool NT, class St>
__global__ __launch_bounds__(kBlock) void k3_step(
    const Params3 P, const St* __restrict__ fin, St* __restrict__ fout,
    const St* __restrict__ gin, St* __restrict__ gout,
    const St* __restrict__ hin, St* __restrict__ hout,
    const double* __restrict__ S, const double* __restrict__ C,
    const int* __restrict__ gid, const double* __restrict__ gw,
    const unsigned long long* __restrict__ tmask, double* __restrict__ partial,
    double* __restrict__ macro, int* flags) {
  __shared__ double red[kBlock / 64][kPartial];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // the candidate spheres of the tile, as the geometry pass found them
  const unsigned long long mask = P.np > 0 ? tmask[blockIdx.x] : 0ull;
  const int c = blockIdx.x * kBlock + t;
  const bool act = c < P.N;
  const int cc = act ? c : P.N - 1;
  const int nxy = P.nx * P.ny, k = cc / nxy, j = (cc - k * nxy) / P.nx,
            i = cc - k * nxy - j * P.nx;

  // pull streaming.  A population whose upstream cell lies beyond a wall
  // is read from the cell's own opposite population instead (halfway
  // bounce-back), so that all 26 loads are independent and issued at once;
  // the walls' velocity and temperature terms are added afterwards.  Where
  // the upstream point lies beyond several walls the z wall decides, then
  // the y wall.
  const bool bxl = i == 0, bxh = i == P.nx - 1, byl = j == 0,
             byh = j == P.ny - 1, bzl = k == 0, bzh = k == P.nz - 1;
  double fst[kQ], g[kQG];
  bool wz_[kQ], wy_[kQ], wx_[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    const int exq = ex(q), eyq = ey(q), ezq = ez(q);
    const bool ox = exq > 0 ? bxl : exq < 0 ? bxh : false;
    const bool oy = eyq > 0 ? byl : eyq < 0 ? byh : false;
    const bool oz = ezq > 0 ? bzl : ezq < 0 ? bzh : false;
    int off = -exq - eyq * P.nx - ezq * nxy;
    off += ox && P.per[0] ? (exq > 0 ? P.nx : -P.nx) : 0;
    off += oy && P.per[1] ? (eyq > 0 ? nxy : -nxy) : 0;
    off += oz && P.per[2] ? (ezq > 0 ? P.N : -P.N) : 0;
    wx_[q] = ox && !P.per[0];
    wy_[q] = oy && !P.per[1];
    wz_[q] = oz && !P.per[2];
    const bool wall = wx_[q] || wy_[q] || wz_[q];
    const size_t at = wall ? (size_t)opp(q) * P.N + cc
                           : (size_t)q * P.N + (size_t)(cc + off);
    fst[q] = (double)fin[at];
    if (q < kQG) g[q] = (double)gin[at];
  }
  const double hold = (double)hin[cc];
  // the storage form's reference (zero in FP64; w_q is w_opp(q), so a
  // bounced population takes its own direction's shift)
  if constexpr (sizeof(St) < sizeof(double)) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      fst[q] += P.fshift[q];
      if (q < kQG) g[q] += P.gshift[q];
    }
  }
  if (bxl || bxh || byl || byh || bzl || bzh) {
#pragma unroll
    for (int q = 1; q < kQ; ++q) {
      const int exq = ex(q), eyq = ey(q), ezq = ez(q);
      // the deciding face (its index is a constant for each branch)
      double eu = 0.0;
      if (wz_[q]) {
        const int fz = ezq > 0 ? 4 : 5;
        eu = exq * P.u_wall[fz][0] + eyq * P.u_wall[fz][1] + ezq * P.u_wall[fz][2];
      } else if (wy_[q]) {
        const int fy = eyq > 0 ? 2 : 3;
        eu = exq * P.u_wall[fy][0] + eyq * P.u_wall[fy][1] + ezq * P.u_wall[fy][2];
      } else if (wx_[q]) {
        const int fx = exq > 0 ? 0 : 1;
        eu = exq * P.u_wall[fx][0] + eyq * P.u_wall[fx][1] + ezq * P.u_wall[fx][2];
      }
      fst[q] += 6.0 * wq(q) * P.rho0 * eu;
      if (q < kQG && (wx_[q] || wy_[q] || wz_[q])) {
        // an axis direction: exactly one face
        const int fc = exq > 0 ? 0 : exq < 0 ? 1 : eyq > 0 ? 2 : eyq < 0 ? 3
                     : ezq > 0 ? 4 : 5;
        if (P.wall_dirichlet[fc])
          g[q] = -g[q] + 2.0 * kW1G * P.cref * P.T_wall[fc];
      }
    }
  }

  // the geometry pass's shares at the new positions; [df_s/dt] through the
  // carrier h = 2 f_s + d (eq. dfs_dt: d' = 2 f_s' - h, h' = 2 f_s' + d')
  int packed = 0;
  double w4[kMaxK] = {0.0, 0.0, 0.0, 0.0};
  if (mask) {
    packed = gid[cc];
#pragma unroll
    for (int n = 0; n < kMaxK; ++n) w4[n] = gw[(size_t)cc * kMaxK + n];
  }
  const int cnt = packed & 7;
  double fs = 0.0;
#pragma unroll
  for (int n = 0; n < kMaxK; ++n) fs += n < cnt ? w4[n] : 0.0;
  if (fs > 1.0) {            // overlapping spheres: shares scaled to sum to 1
#pragma unroll
    for (int n = 0; n < kMaxK; ++n) w4[n] /= fs;
    fs = 1.0;
  }
  const double dfs = 2.0 * fs - hold;

  // volumetric no-slip step (eq. fi), sphere by sphere in ascending order;
  // each sphere's momentum-exchange share is reduced over the block at once
  double rho = 0.0;
#pragma unroll
  for (int q = 0; q < kQ; ++q) rho += fst[q];
  double f[kQ];
#pragma unroll
  for (int q = 0; q < kQ; ++q) f[q] = (1.0 - fs) * fst[q];
  for (unsigned long long m = mask; m; m &= m - 1) {      // uniform
    const int p = __ffsll((long long)m) - 1;
    double part[kPartial] = {0, 0, 0, 0, 0, 0};
    double w = 0.0;
    bool mine = false;
#pragma unroll
    for (int n = 0; n < kMaxK; ++n)
      if (n < cnt && ((packed >> (8 * n + 8)) & 255) == p) {
        w = w4[n];
        mine = true;
      }
    if (act && mine) {
      double us[3], r[3];
      solid_velocity(P, S, p, i, j, k, us, r);
      const double u2 = us[0] * us[0] + us[1] * us[1] + us[2] * us[2];
      double dP[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int q = 0; q < kQ; ++q) {
        const double fe = feq_q(q, rho, us[0], us[1], us[2], u2);
        f[q] += w * fe;
        const double df = w * (fe - fst[q]);
        dP[0] += df * ex(q);
        dP[1] += df * ey(q);
        dP[2] += df * ez(q);
      }
      part[0] = dP[0];
      part[1] = dP[1];
      part[2] = dP[2];
      part[3] = r[1] * dP[2] - r[2] * dP[1];
      part[4] = r[2] * dP[0] - r[0] * dP[2];
      part[5] = r[0] * dP[1] - r[1] * dP[0];
    }
    for (int v = 0; v < kPartial; ++v) {
      const double s = wave_sum(part[v]);
      if (lane == 0) red[wv][v] = s;
    }
    __syncthreads();
    if (t < kPartial)
      partial[((size_t)p * P.nblocks + blockIdx.x) * kPartial + t] =
          ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    __syncthreads();
  }
  if (!act) return;

  double jx = 0.0, jy = 0.0, jz = 0.0;
#pragma unroll
  for (int q = 0; q < kQ; ++q) {
    jx += ex(q) * f[q];
    jy += ey(q) * f[q];
    jz += ez(q) * f[q];
  }
  // per-cell properties (Sec. 2.2); lambda/rho_f = c_s^2 c_ref (tau_g - 1/2)
  const double cv = (1.0 - fs) * P.cv_f + fs * P.cv_s;
  const double lam = (1.0 - fs) * P.lam_f + fs * P.lam_s;
  const double tau_g = 0.5 + lam / (P.rho_f * kCs2G * P.cref);
  const double sj = 1.0 / tau_g;
  const double se = P.sigma_rule ? 1.0 : 1.0 / (0.5 + 0.25 / (tau_g - 0.5));
  // macroscopic values and the coupled T-u solve (F = A + B T)
  double G = 0.0, J[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < kQG; ++q) {
    G += g[q];
    J[0] += ex(q) * g[q];
    J[1] += ey(q) * g[q];
    J[2] += ez(q) * g[q];
  }
  double gT[3];
  for (int a = 0; a < 3; ++a) gT[a] = -J[a] / (kCs2G * P.cref * tau_g);
  const double wf = 1.0 - fs, dcv = P.cv_s - P.cv_f;
  const double jv[3] = {jx, jy, jz};
  double A[3], B[3], jg = 0.0, bg = 0.0;
  for (int a = 0; a < 3; ++a) {
    A[a] = wf * (P.body[a] + P.rho_f * P.beta * P.T_ref * P.grav[a]);
    B[a] = -wf * P.rho_f * P.beta * P.grav[a];
    jg += (jv[a] + 0.5 * A[a]) * gT[a];
    bg += B[a] * gT[a];
  }
  const double T = (G - 0.5 * cv * jg / rho) /
                   (cv - 0.5 * dcv * dfs + 0.25 * cv * bg / rho);
  double F[3], u[3];
  for (int a = 0; a < 3; ++a) {
    F[a] = A[a] + B[a] * T;
    u[a] = (jv[a] + 0.5 * F[a]) / rho;
  }
  const double eps = cv * T;
  const double qc = -cv * (u[0] * gT[0] + u[1] * gT[1] + u[2] * gT[2]) +
                    dcv * T * dfs;
  if (!(rho > 0.0) || !isfinite(T) || !isfinite(u[0]) || !isfinite(u[1]) ||
      !isfinite(u[2]))
    atomicOr(flags, kFlagUnstable);

  // energy collision: even part at sigma_e, odd part at sigma_j, the
  // source on the rest population
  {
    const double geq0 = eps - (1.0 - kW0G) * P.cref * T, geqi = kW1G * P.cref * T;
    put_pop<NT>(gout + c, g[0] - se * (g[0] - geq0) + (1.0 - 0.5 * se) * qc,
                P.gshift[0]);
#pragma unroll
    for (int q = 1; q < kQG; ++q) {
      const double ev = 0.5 * (g[q] + g[opp(q)]), od = 0.5 * (g[q] - g[opp(q)]);
      put_pop<NT>(gout + (size_t)q * P.N + c,
                  g[q] - se * (ev - geqi) - sj * od, P.gshift[q]);
    }
  }
  // flow MRT collision (eq. lbe.rho.col),
  //   f' = f + M^-1 [-S M (f - f^eq) + (I - S/2) M F_G],
  // F_G Guo's term; with a = f - f^eq + F_G/2 this is
  //   f' = a + f^eq + F_G/2 - M^-1 S M a,
  // which holds one vector of 19 (a) and its 19 relaxed moments at a time
  {
    const double u2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    auto guo = [&](int q) {
      const double eF = ex(q) * F[0] + ey(q) * F[1] + ez(q) * F[2];
      const double eu = ex(q) * u[0] + ey(q) * u[1] + ez(q) * u[2];
      return wq(q) * (3.0 * eF + 9.0 * eu * eF - 3.0 * uF);
    };
    double a[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q)
      a[q] = f[q] - feq_q(q, rho, u[0], u[1], u[2], u2) + 0.5 * guo(q);
    double dm[kQ];
    relax_moments(a, dm, P.snu, P.sq, std::make_index_sequence<kQ>{});
    auto base = [&](int q) {
      return a[q] + feq_q(q, rho, u[0], u[1], u[2], u2) + 0.5 * guo(q);
    };
    back_transform_store<NT>(dm, base, fout, (size_t)P.N, (size_t)c,
                             P.fshift, std::make_index_sequence<kQ>{});
  }
  put<NT>(hout + c, 2.0 * fs + dfs);
  if (OUT) {
    const double mv[kMacro] = {rho, u[0], u[1], u[2], T, fs, dfs};
#pragma unroll
    for (int m = 0; m < kMacro; ++m) macro[(size_t)m * P.N + c] = mv[m];
  }
}

// ---------------------------------------------------------------------------
// Per-sphere thermal outputs: one block per sphere over the cells of its
// bounding box (through the nearest copies); out[p] = {sum f_s,p T,
// sum f_s,p c_vs T, sum f_s,p, min T over wholly covered cells, min T over
// all}.

__global__ __launch_bounds__(kBlock) void k3_sphere_sums(
    const Params3 P, const double* __restrict__ S, const double* __restrict__ C,
    const double* __restrict__ macro, double* __restrict__ out) {
  __shared__ double red[kBlock / 64][5];
  const int p = blockIdx.x, t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int np = P.np;
  const double R = C[cR * np + p];
  const double c0[3] = {S[fX * np + p], S[fY * np + p], S[fZ * np + p]};
  int lo[3], ext[3];
  const int n3[3] = {P.nx, P.ny, P.nz};
  for (int a = 0; a < 3; ++a) {
    lo[a] = (int)floor(c0[a] - R) - 1;
    ext[a] = (int)floor(c0[a] + R) + 1 - lo[a] + 1;
  }
  const long long total = (long long)ext[0] * ext[1] * ext[2];
  double sT = 0.0, sE = 0.0, sW = 0.0, mFull = INFINITY, mAny = INFINITY;
  const unsigned long long all = np >= 64 ? ~0ull : ((1ull << np) - 1ull);
  for (long long e = t; e < total; e += kBlock) {
    int idx[3] = {(int)(e % ext[0]), (int)((e / ext[0]) % ext[1]),
                  (int)(e / ((long long)ext[0] * ext[1]))};
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
      idx[a] += lo[a];
      if (P.per[a]) idx[a] = ((idx[a] % n3[a]) + n3[a]) % n3[a];
      if (idx[a] < 0 || idx[a] >= n3[a]) ok = false;
    }
    if (!ok) continue;
    CellGeo geo;
    cell_geometry(P, S, C, all, idx[0], idx[1], idx[2], geo, nullptr);
    for (int n = 0; n < kMaxK; ++n) {
      if (n >= geo.cnt || geo.id[n] != p) continue;
      const size_t c = ((size_t)idx[2] * P.ny + idx[1]) * P.nx + idx[0];
      const double T = macro[(size_t)mT * P.N + c], w = geo.w[n];
      sT += w * T;
      sE += w * P.cv_s * T;
      sW += w;
      mAny = fmin(mAny, T);
      double cp[3];
      const double node[3] = {idx[0] + 0.5, idx[1] + 0.5, idx[2] + 0.5};
      const double L[3] = {(double)P.nx, (double)P.ny, (double)P.nz};
      for (int a = 0; a < 3; ++a) cp[a] = near_copy(c0[a], node[a], L[a], P.per[a]);
      if (wholly_inside(cp[0], cp[1], cp[2], R, idx[0], idx[1], idx[2]))
        mFull = fmin(mFull, T);
    }
  }
  double v[5] = {wave_sum(sT), wave_sum(sE), wave_sum(sW), mFull, mAny};
  for (int o = 32; o >= 1; o >>= 1) {
    v[3] = fmin(v[3], __shfl_xor(v[3], o, 64));
    v[4] = fmin(v[4], __shfl_xor(v[4], o, 64));
  }
  if (lane == 0)
    for (int m = 0; m < 5; ++m) red[wv][m] = v[m];
  __syncthreads();
  if (t == 0) {
    double r[5] = {0.0, 0.0, 0.0, INFINITY, INFINITY};
    for (int w = 0; w < kBlock / 64; ++w) {
      for (int m = 0; m < 3; ++m) r[m] += red[w][m];
      r[3] = fmin(r[3], red[w][3]);
      r[4] = fmin(r[4], red[w][4]);
    }
    for (int m = 0; m < 5; ++m) out[p * 5 + m] = r[m];
  }
}

// ---------------------------------------------------------------------------
// Launchers

static unsigned nblocks_of(const Params3& P) { return (unsigned)P.nblocks; }

hipError_t launch_init(const Params3& P, void* f, void* g, void* h,
                       double* macro, const double* S, const double* C,
                       int* flags, hipStream_t s) {
  if (P.f32)
    hipLaunchKernelGGL(k3_init<float>, dim3(nblocks_of(P)), dim3(kBlock), 0,
                       s, P, (float*)f, (float*)g, (float*)h, macro, S, C,
                       flags);
  else
    hipLaunchKernelGGL(k3_init<double>, dim3(nblocks_of(P)), dim3(kBlock), 0,
                       s, P, (double*)f, (double*)g, (double*)h, macro, S, C,
                       flags);
  return hipGetLastError();
}

hipError_t launch_particles(const Params3& P, double* cur, double* nxt,
                            const double* C, const double* partial,
                            const unsigned long long* tmask, int have,
                            int update, hipStream_t s) {
  if (P.np == 0) return hipSuccess;
  hipLaunchKernelGGL(k3_particles, dim3(P.np), dim3(kBlock), 0, s, P, cur, nxt, C,
                     partial, tmask, have, update);
  return hipGetLastError();
}

hipError_t launch_geometry(const Params3& P, const double* S,
                           const double* C, int* gid, double* gw,
                           unsigned long long* tmask, int* items, int* nitems,
                           int* flags, hipStream_t s) {
  if (P.np == 0) return hipSuccess;
  hipError_t e = hipMemsetAsync(nitems, 0, kSegs * sizeof(int), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k3_geometry_a, dim3(nblocks_of(P)), dim3(kBlock), 0, s,
                     P, S, C, gid, gw, tmask, items, nitems, flags);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k3_geometry_b, dim3(2048), dim3(kBlock), 0, s, P, S, C,
                     gid, gw, items, nitems);
  return hipGetLastError();
}

hipError_t launch_step(const Params3& P, bool out, const void* fin,
                       void* fout, const void* gin, void* gout,
                       const void* hin, void* hout, const double* S,
                       const double* C, const int* gid, const double* gw,
                       const unsigned long long* tmask, double* partial,
                       double* macro, int* flags, hipStream_t s) {
#define VLB3_STEP(O, N, T)                                                   \
  hipLaunchKernelGGL((k3_step<O, N, T>), dim3(nblocks_of(P)), dim3(kBlock),  \
                     0, s, P, (const T*)fin, (T*)fout, (const T*)gin,        \
                     (T*)gout, (const T*)hin, (T*)hout, S, C, gid, gw, tmask, \
                     partial, macro, flags)
#define VLB3_STEP_T(T)                                                       \
  if (P.nt_stores) {                                                         \
    if (out) VLB3_STEP(true, true, T); else VLB3_STEP(false, true, T);       \
  } else {                                                                   \
    if (out) VLB3_STEP(true, false, T); else VLB3_STEP(false, false, T);     \
  }
  if (P.f32) {
    VLB3_STEP_T(float)
  } else {
    VLB3_STEP_T(double)
  }
#undef VLB3_STEP_T
#undef VLB3_STEP
  return hipGetLastError();
}

hipError_t launch_sphere_sums(const Params3& P, const double* S,
                              const double* C, const double* macro,
                              double* out, hipStream_t s) {
  if (P.np == 0) return hipSuccess;
  hipLaunchKernelGGL(k3_sphere_sums, dim3(P.np), dim3(kBlock), 0, s, P, S, C,
                     macro, out);
  return hipGetLastError();
}

// Gauss-Legendre nodes on [0, 1]: roots of P_n by Newton's method from
// Chebyshev-like starting points, weights 2/((1 - x^2) P_n'(x)^2), mapped
// from [-1, 1].
hipError_t upload_quadrature() {
  double x[kGL], w[kGL];
  for (int m = 0; m < kGL; ++m) {
    double z = cos(M_PI * (m + 0.75) / (kGL + 0.5)), dp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int l = 2; l <= kGL; ++l) {
        const double p2 = ((2.0 * l - 1.0) * z * p1 - (l - 1.0) * p0) / l;
        p0 = p1;
        p1 = p2;
      }
      dp = kGL * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-17) break;
    }
    x[m] = 0.5 * (1.0 - z);
    w[m] = 1.0 / ((1.0 - z * z) * dp * dp);   // (2/((1-z^2) P'^2)) / 2
  }
  hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(gl_x), x, sizeof x);
  if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(gl_w), w, sizeof w);
  return e;
}

}  // namespace vlb3
