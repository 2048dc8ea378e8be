// Device-side particle shapes and orbit segmentation for gfx950.
//
// Shapes: centred cardinal B-splines of degree r on nodes x_g = g H
// (eq. Ah-mesh).  A point at cell coordinate u = x / H is written against a
// base node: degree 1 uses floor(u) and the two nodes {base, base+1};
// degree 2 uses the nearest node floor(u + 1/2) and {base-1, base, base+1};
// degree 3 uses floor(u) and {base-1, ..., base+2}.  Knots sit at integer u
// (odd degrees) and half-integer u (degree 2).
//
// Orbits: x(s) = x0 + s d, 0 <= s <= 1, with unwrapped displacement d
// (eq. particle-orbit).  The breakpoints are the parameters s in (0, 1) where
// one coordinate crosses a knot (eq. breakpoint-set); the three per-axis
// crossing sequences are each monotone in s, so they are merged on the fly
// (no list is stored) and equal values from different axes collapse into one
// breakpoint.  Every piece between breakpoints is integrated with an n_q-point
// Gauss-Legendre rule against the polynomial pieces of the stencil of the
// knot interval it lies in; 2 n_q - 1 >= 3 r makes this exact (Sec. 4.7).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecpic {

// Mesh sizes are powers of two, so periodic wrapping of a node index is a
// bit mask and flat node indices are built with shifts.
struct Grid {
  int n[3];
  int mask[3];  // n - 1
  int shx, shy; // flat index = (ix << shx) | (iy << shy) | iz
  double L[3];
  double invL[3];
  double H[3];
  double invH[3];
  double dV;
  double vol;
  int64_t ncell;
};

__device__ __forceinline__ int wrapi(int i, int n) { return i & (n - 1); }

__device__ __forceinline__ int node_index(const Grid& G, int ix, int iy, int iz) {
  return ((ix & G.mask[0]) << G.shx) | ((iy & G.mask[1]) << G.shy) | (iz & G.mask[2]);
}

// Convert a floor()ed double to int without undefined behaviour for huge or
// non-finite values (clamped; such particles are flagged elsewhere).
__device__ __forceinline__ int to_int_clamped(double f) {
  f = fmin(fmax(f, -1.0e9), 1.0e9);
  return (int)f;
}

// x wrapped into [0, L); invL = 1/L
__device__ __forceinline__ double wrap_pos(double x, double L, double invL) {
  double w = x - L * floor(x * invL);
  if (w < 0.0) w += L;
  if (w >= L) w -= L;
  return w;
}

template <int R>
struct Spline;

template <>
struct Spline<1> {
  static constexpr int W = 2;
  static constexpr double knot_off = 0.0;  // knots at u = k
  static constexpr double base_off = 0.0;  // base = floor(u)
  static constexpr int first_off = 0;      // stencil = {base, base + 1}
  __device__ __forceinline__ static void w(double t, double* o) {
    o[0] = 1.0 - t;
    o[1] = t;
  }
  __device__ __forceinline__ static void wd(double t, double* o, double* d) {
    o[0] = 1.0 - t;
    o[1] = t;
    d[0] = -1.0;
    d[1] = 1.0;
  }
  // weight and derivative of stencil node k alone (k a constant after unrolling)
  __device__ __forceinline__ static void wk(int k, double t, double& w, double& dw) {
    if (k == 0) {
      w = 1.0 - t;
      dw = -1.0;
    } else {
      w = t;
      dw = 1.0;
    }
  }
};

template <>
struct Spline<2> {
  static constexpr int W = 3;
  static constexpr double knot_off = 0.5;  // knots at u = k + 1/2
  static constexpr double base_off = 0.5;  // base = floor(u + 1/2)
  static constexpr int first_off = -1;     // stencil = {base - 1, base, base + 1}
  __device__ __forceinline__ static void w(double t, double* o) {
    const double a = 0.5 - t, b = 0.5 + t;
    o[0] = 0.5 * a * a;
    o[1] = 0.75 - t * t;
    o[2] = 0.5 * b * b;
  }
  __device__ __forceinline__ static void wd(double t, double* o, double* d) {
    const double a = 0.5 - t, b = 0.5 + t;
    o[0] = 0.5 * a * a;
    o[1] = 0.75 - t * t;
    o[2] = 0.5 * b * b;
    d[0] = -a;
    d[1] = -2.0 * t;
    d[2] = b;
  }
  __device__ __forceinline__ static void wk(int k, double t, double& w, double& dw) {
    if (k == 0) {
      const double a = 0.5 - t;
      w = 0.5 * a * a;
      dw = -a;
    } else if (k == 1) {
      w = 0.75 - t * t;
      dw = -2.0 * t;
    } else {
      const double b = 0.5 + t;
      w = 0.5 * b * b;
      dw = b;
    }
  }
};

template <>
struct Spline<3> {
  static constexpr int W = 4;
  static constexpr double knot_off = 0.0;  // knots at u = k
  static constexpr double base_off = 0.0;  // base = floor(u)
  static constexpr int first_off = -1;     // stencil = {base - 1, ..., base + 2}
  // M3(xi) = 2/3 - xi^2 + |xi|^3 / 2 (|xi| <= 1), (2 - |xi|)^3 / 6 (1 <= |xi| <= 2);
  // node base - 1 + k sits at xi = t + 1 - k
  __device__ __forceinline__ static void w(double t, double* o) {
    const double u = 1.0 - t, t2 = t * t, u2 = u * u;
    o[0] = (1.0 / 6.0) * u2 * u;
    o[1] = (2.0 / 3.0) - t2 + 0.5 * t2 * t;
    o[2] = (2.0 / 3.0) - u2 + 0.5 * u2 * u;
    o[3] = (1.0 / 6.0) * t2 * t;
  }
  __device__ __forceinline__ static void wd(double t, double* o, double* d) {
    const double u = 1.0 - t, t2 = t * t, u2 = u * u;
    o[0] = (1.0 / 6.0) * u2 * u;
    o[1] = (2.0 / 3.0) - t2 + 0.5 * t2 * t;
    o[2] = (2.0 / 3.0) - u2 + 0.5 * u2 * u;
    o[3] = (1.0 / 6.0) * t2 * t;
    d[0] = -0.5 * u2;
    d[1] = -2.0 * t + 1.5 * t2;
    d[2] = 2.0 * u - 1.5 * u2;
    d[3] = 0.5 * t2;
  }
  __device__ __forceinline__ static void wk(int k, double t, double& w, double& dw) {
    const double u = 1.0 - t;
    if (k == 0) {
      w = (1.0 / 6.0) * u * u * u;
      dw = -0.5 * u * u;
    } else if (k == 1) {
      w = (2.0 / 3.0) - t * t + 0.5 * t * t * t;
      dw = -2.0 * t + 1.5 * t * t;
    } else if (k == 2) {
      w = (2.0 / 3.0) - u * u + 0.5 * u * u * u;
      dw = 2.0 * u - 1.5 * u * u;
    } else {
      w = (1.0 / 6.0) * t * t * t;
      dw = 0.5 * t * t;
    }
  }
};

// Gauss-Legendre nodes and weights on [-1, 1] (Abramowitz & Stegun, Table 25.4).
template <int NQ>
struct Gauss;

template <>
struct Gauss<2> {
  __device__ __forceinline__ static double x(int q) {
    return q == 0 ? -0.57735026918962576451 : 0.57735026918962576451;
  }
  __device__ __forceinline__ static double w(int) { return 1.0; }
};

template <>
struct Gauss<4> {
  __device__ __forceinline__ static double x(int q) {
    const double a = 0.86113631159405257522, b = 0.33998104358485626480;
    return q == 0 ? -a : (q == 1 ? -b : (q == 2 ? b : a));
  }
  __device__ __forceinline__ static double w(int q) {
    const double wa = 0.34785484513745385737, wb = 0.65214515486254614263;
    return (q == 0 || q == 3) ? wa : wb;
  }
};

template <>
struct Gauss<5> {
  __device__ __forceinline__ static double x(int q) {
    const double a = 0.90617984593866399280, b = 0.53846931010568309104;
    return q == 0 ? -a : (q == 1 ? -b : (q == 2 ? 0.0 : (q == 3 ? b : a)));
  }
  __device__ __forceinline__ static double w(int q) {
    const double wa = 0.23692688505618908751, wb = 0.47862867049936646804;
    return (q == 0 || q == 4) ? wa : ((q == 1 || q == 3) ? wb : 0.56888888888888888889);
  }
};

// Streaming merge of the three per-axis knot-crossing sequences of an orbit.
// Along axis a the crossings are equally spaced in s, H_a / |d_a| apart.  The
// first one is the breakpoint of its knot as defined, (xi_k - x0) / d with
// xi_k = (k + knot_off) H_a, taken over the knots ahead of x0 until it is
// positive, so that an orbit starting exactly on a knot (a quiet start at cell
// centres for r = 2) has no crossing there whatever the size of d; the later
// ones follow by adding the spacing (a few ulp from the quotient of each knot;
// pieces only need to be told apart by their knot intervals, so the ends may
// move by that much).
//
// The stencil of a piece is the one of the knot interval its interior lies in
// (Sec. 4.7).  Per axis that is the interval behind the first knot ahead, then
// one interval further along the motion at every crossing of that axis, so
// the choice never rests on a rounded midpoint: an orbit that leaves a knot
// by less than the rounding of x0 still takes the interval on the side it
// moves to.  An axis along which the orbit does not move takes the interval
// holding x0, closed below.  (Keeping the next crossing and the spacing per axis costs
// fewer registers in the gather kernel than recomputing each crossing from
// its knot and 1 / d_a.)
template <int R>
struct Crossings {
  double sn[3];    // next crossing parameter per axis (>= 2 when exhausted)
  double step[3];  // spacing of the crossings of that axis, with the sign of d_a
  int base[3];     // base node of the current piece's stencil per axis

  __device__ __forceinline__ void init(const double* x0, const double* d, const Grid& G) {
    // xi_k - x0 rounded once from the rounded xi_k: a contracted multiply-add
    // would leave the rounding error of k H_a for an orbit that starts on a
    // knot, and a random-signed sliver piece with it
#pragma clang fp contract(off)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      // a still axis is searched as if it moved up: its interval is the one
      // behind the first knot above x0 (closed below)
      const bool moves = d[a] != 0.0;
      const bool up = !(d[a] < 0.0);
      const double inv = 1.0 / (moves ? d[a] : 1.0);
      const double dir = up ? 1.0 : -1.0;
      // the knot at or below the rounded u0; the first knot ahead of x0 along
      // the motion is at most two knots further (x0 differs from u0 H_a by a
      // few ulp), decided by the sign of (xi_k - x0) / d
      double knot = floor(x0[a] * G.invH[a] - Spline<R>::knot_off) + Spline<R>::knot_off;
      double s = (knot * G.H[a] - x0[a]) * inv;
#pragma unroll
      for (int it = 0; it < 2; ++it) {
        const bool behind = !(s > 0.0);
        knot = behind ? knot + dir : knot;
        s = behind ? (knot * G.H[a] - x0[a]) * inv : s;
      }
      sn[a] = (moves && s < 1.0) ? s : 2.0;
      step[a] = moves ? G.H[a] * inv : 2.0;
      base[a] = to_int_clamped(knot + Spline<R>::base_off - (up ? 1.0 : 0.0));
    }
  }

  __device__ __forceinline__ double next() const {
    return fmin(fmin(sn[0], sn[1]), fmin(sn[2], 1.0));
  }

  // advance every axis that crosses at s1 (selects, no branches: the piece
  // loop is the inner loop of the particle kernels)
  __device__ __forceinline__ void consume(double s1) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const bool hit = sn[a] == s1;
      const double s = sn[a] + fabs(step[a]);
      const double adv = (s > sn[a] && s < 1.0) ? s : 2.0;
      sn[a] = hit ? adv : sn[a];
      base[a] += hit ? (step[a] > 0.0 ? 1 : -1) : 0;
    }
  }
};

constexpr int kMaxPieces = 64;

// Calls f(s0, s1, base) for every piece [s0, s1] of positive length, in
// order, with the base node of the piece's stencil per axis.  Returns false
// if the orbit had more than kMaxPieces pieces (the rest is skipped; the
// caller flags the particle).
template <int R, class F>
__device__ __forceinline__ bool for_each_piece(const double* x0, const double* d, const Grid& G,
                                               F&& f) {
  Crossings<R> c;
  c.init(x0, d, G);
  double s0 = 0.0;
  for (int k = 0; k < kMaxPieces; ++k) {
    const double s1 = c.next();
    if (s1 > s0) {
      const double base[3] = {(double)c.base[0], (double)c.base[1], (double)c.base[2]};
      f(s0, s1, base);
    }
    if (s1 >= 1.0) return true;
    c.consume(s1);
    s0 = s1;
  }
  return false;
}

// Base node of the stencil of the point at s (the rule over the whole orbit
// without splitting, where every point takes the stencil of its own cell).
template <int R>
__device__ __forceinline__ void point_base(const double* x0, const double* d, double s,
                                           const Grid& G, double* base) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
    base[a] = floor((x0[a] + s * d[a]) * G.invH[a] + Spline<R>::base_off);
}

}  // namespace ecpic
