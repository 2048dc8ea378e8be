// Particle-side kernels for gfx950: orbit current scatter, orbit gather with
// the orbit-discrete gradient and canonical-momentum push, the consistency
// sweep, and the end-of-step update.
//
// One lane per particle; particle arrays are structure-of-arrays doubles
// (component a of particle i at a*np + i).  The mesh fields a particle reads
// during the gather are interleaved per node (kGbufStride doubles per node:
// grad_h phi^{n+1/2}, A^n, A^{n+1}) so that one stencil node costs one short
// run of contiguous loads.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "internal.hpp"
#include "orbit.hpp"
#include "reduce.hpp"

namespace ecpic {

namespace {

template <int R>
struct Quad;
template <>
struct Quad<1> {
  static constexpr int NQ = 2;  // 2 n_q - 1 >= 3 r  ->  n_q = 2 for r = 1
};
template <>
struct Quad<2> {
  static constexpr int NQ = 4;  // n_q = 4 for r = 2
};
template <>
struct Quad<3> {
  static constexpr int NQ = 5;  // n_q = 5 for r = 3
};

// ---- field accessors ------------------------------------------------------
struct AosFields {
  const double* __restrict__ g;
  __device__ __forceinline__ void load9(int64_t node, double* f) const {
    const double* p = g + node * kGbufStride;
#pragma unroll
    for (int k = 0; k < 9; ++k) f[k] = p[k];
  }
  __device__ __forceinline__ double A0(int64_t node, int l) const { return g[node * kGbufStride + 3 + l]; }
  __device__ __forceinline__ double A1(int64_t node, int l) const { return g[node * kGbufStride + 6 + l]; }
};

// Accessors of the push path.  A stencil node is addressed by its unwrapped
// integer coordinates in the particle's frame; row() folds (ix, iy), node()
// adds iz and returns the node's kGbufStride doubles
// [grad_h phi (3) | A^n (3) | A^{n+1} (3) | pad].
struct GlobalGather {  // the interleaved gather buffer in global memory
  const double* __restrict__ g;
  int mask0, mask1, mask2, shx, shy;
  __device__ __forceinline__ int row(int ix, int iy) const {
    return ((ix & mask0) << shx) | ((iy & mask1) << shy);
  }
  __device__ __forceinline__ const double* node(int row, int iz) const {
    return g + (int64_t)(row | (iz & mask2)) * kGbufStride;
  }
};

typedef __attribute__((address_space(3))) const double lds_cdouble;

struct TileGather {  // a block's LDS copy of the nodes its orbits touch
  lds_cdouble* t;
  int ox, oy, oz;    // particle frame -> tile coordinates
  int dy, dz;        // tile extents along y and z
  __device__ __forceinline__ int row(int ix, int iy) const { return ((ix + ox) * dy + (iy + oy)) * dz + oz; }
  __device__ __forceinline__ lds_cdouble* node(int row, int iz) const {
    return t + (row + iz) * kGbufStride;
  }
};

struct SoaFields {
  const double* __restrict__ gphi;
  const double* __restrict__ a0;
  const double* __restrict__ a1;
  int64_t nc;
  __device__ __forceinline__ void load9(int64_t node, double* f) const {
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      f[l] = gphi[l * nc + node];
      f[3 + l] = a0[l * nc + node];
      f[6 + l] = a1[l * nc + node];
    }
  }
  __device__ __forceinline__ double A0(int64_t node, int l) const { return a0[l * nc + node]; }
  __device__ __forceinline__ double A1(int64_t node, int l) const { return a1[l * nc + node]; }
};

__device__ __forceinline__ int64_t node_of(const Grid& G, int ix, int iy, int iz) {
  return node_index(G, ix, iy, iz);
}

// ---- one orbit piece: current scatter -------------------------------------
// Iw[a][b][c] = int_{s0}^{s1} S_g(x(s)) ds for the stencil node first + (a, b, c)
// (eq. split-Sbar); first is the unwrapped index of the piece's first stencil node.
// NP quadrature points sq[] with weights wq[] against the stencil of base
template <int R, int NP>
__device__ __forceinline__ void sbar_points(const Grid& G, const double* x0, const double* d,
                                            const double* base, const double* sq,
                                            const double* wq,
                                            double (&Iw)[R + 1][R + 1][R + 1], int* first) {
  constexpr int W = R + 1;
#pragma unroll
  for (int a = 0; a < W; ++a)
#pragma unroll
    for (int b = 0; b < W; ++b)
#pragma unroll
      for (int c = 0; c < W; ++c) Iw[a][b][c] = 0.0;
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const double s = sq[q];
    const double wt = wq[q];
    double wx[W], wy[W], wz[W];
    Spline<R>::w((x0[0] + s * d[0]) * G.invH[0] - base[0], wx);
    Spline<R>::w((x0[1] + s * d[1]) * G.invH[1] - base[1], wy);
    Spline<R>::w((x0[2] + s * d[2]) * G.invH[2] - base[2], wz);
#pragma unroll
    for (int a = 0; a < W; ++a) {
      const double xa = wt * wx[a];
#pragma unroll
      for (int b = 0; b < W; ++b) {
        const double xy = xa * wy[b];
#pragma unroll
        for (int c = 0; c < W; ++c) Iw[a][b][c] += xy * wz[c];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) first[a] = to_int_clamped(base[a]) + Spline<R>::first_off;
}

// the n_q-point rule of a piece [s0, s1] (its stencil comes with the piece)
template <int R>
__device__ __forceinline__ void piece_rule(double s0, double s1, double* sq, double* wq) {
  constexpr int NQ = Quad<R>::NQ;
  const double h = s1 - s0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    sq[q] = s0 + 0.5 * h * (1.0 + Gauss<NQ>::x(q));
    wq[q] = 0.5 * h * Gauss<NQ>::w(q);
  }
}

// point q of the rule over the whole orbit (no splitting): the stencil is
// the one of x(s_q) itself (comparison runs)
template <int R>
__device__ __forceinline__ void unsplit_point(const Grid& G, const QuadRule& rule, int q,
                                              const double* x0, const double* d, double* base,
                                              double& s, double& w) {
  s = rule.s[q];
  w = rule.w[q];
  point_base<R>(x0, d, s, G, base);
}

template <int R>
__device__ __forceinline__ void piece_sbar(const Grid& G, const double* x0, const double* d,
                                           double s0, double s1, const double* base,
                                           double (&Iw)[R + 1][R + 1][R + 1], int* first) {
  constexpr int NQ = Quad<R>::NQ;
  double sq[NQ], wq[NQ];
  piece_rule<R>(s0, s1, sq, wq);
  sbar_points<R, NQ>(G, x0, d, base, sq, wq, Iw, first);
}

// J_g += (q vbar / dV) int_{s0}^{s1} S_g(x(s)) ds straight into global memory
// (eq. orbit-current, split form)
template <int R>
__device__ __forceinline__ void scatter_piece(const Grid& G, const double* x0, const double* d,
                                              double s0, double s1, const double* base,
                                              const double* c3, double* __restrict__ J) {
  constexpr int W = R + 1;
  double Iw[W][W][W];
  int f[3];
  piece_sbar<R>(G, x0, d, s0, s1, base, Iw, f);
  const int64_t nc = G.ncell;
#pragma unroll
  for (int a = 0; a < W; ++a) {
    const int ix = wrapi(f[0] + a, G.n[0]);
#pragma unroll
    for (int b = 0; b < W; ++b) {
      const int iy = wrapi(f[1] + b, G.n[1]);
#pragma unroll
      for (int c = 0; c < W; ++c) {
        const int64_t g = node_of(G, ix, iy, wrapi(f[2] + c, G.n[2]));
        const double w = Iw[a][b][c];
        unsafeAtomicAdd(J + g, w * c3[0]);
        unsafeAtomicAdd(J + nc + g, w * c3[1]);
        unsafeAtomicAdd(J + 2 * nc + g, w * c3[2]);
      }
    }
  }
}

// ---- one orbit piece: gather --------------------------------------------
// gp_l  += sum_g (grad_h phi)_lg int S_g ds                 (eq. gphibar-definition)
// D_lj  += sum_g int A_lg(s) d_j S_g(x(s)) ds, A_g(s) = (1-s) A^n + s A^{n+1}  (eq. split-DA)
// with WITH_U also Ub_l += sum_g U_lg int S_g ds and pou += int sum_g S_g ds.
// The n_q-point rule is evaluated once per piece; each stencil node then
// accumulates its weight integrals over the quadrature points and is
// contracted with the node's field values.
template <int R, int NQ, bool WITH_U, class Acc>
__device__ __forceinline__ void gather_points(const Grid& G, const double* x0, const double* d,
                                              const double* base, const double* sqs,
                                              const double* wqs, const Acc& acc,
                                              const double* __restrict__ Uh, double* gp,
                                              double (*D)[3], double* Ub, double& pou) {
  constexpr int W = R + 1;
  double X[NQ][W], dX[NQ][W], Y[NQ][W], dY[NQ][W];
  double Zw[NQ][W], Z0[NQ][W], Z1[NQ][W], dZ0[NQ][W], dZ1[NQ][W];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double s = sqs[q];
    const double wt = wqs[q];
    const double w0 = wt * (1.0 - s), w1 = wt * s;
    double wz[W], dz[W];
    Spline<R>::wd((x0[0] + s * d[0]) * G.invH[0] - base[0], X[q], dX[q]);
    Spline<R>::wd((x0[1] + s * d[1]) * G.invH[1] - base[1], Y[q], dY[q]);
    Spline<R>::wd((x0[2] + s * d[2]) * G.invH[2] - base[2], wz, dz);
#pragma unroll
    for (int k = 0; k < W; ++k) {
      dX[q][k] *= G.invH[0];
      dY[q][k] *= G.invH[1];
      const double dzk = dz[k] * G.invH[2];
      Zw[q][k] = wt * wz[k];
      Z0[q][k] = w0 * wz[k];
      Z1[q][k] = w1 * wz[k];
      dZ0[q][k] = w0 * dzk;
      dZ1[q][k] = w1 * dzk;
    }
  }
  const int fx = to_int_clamped(base[0]) + Spline<R>::first_off;
  const int fy = to_int_clamped(base[1]) + Spline<R>::first_off;
  const int fz = to_int_clamped(base[2]) + Spline<R>::first_off;
#pragma unroll
  for (int a = 0; a < W; ++a) {
    const int ix = wrapi(fx + a, G.n[0]);
#pragma unroll
    for (int b = 0; b < W; ++b) {
      const int iy = wrapi(fy + b, G.n[1]);
      double xy[NQ], dxy[NQ], xdy[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        xy[q] = X[q][a] * Y[q][b];
        dxy[q] = dX[q][a] * Y[q][b];
        xdy[q] = X[q][a] * dY[q][b];
      }
#pragma unroll
      for (int c = 0; c < W; ++c) {
        const int64_t g = node_of(G, ix, iy, wrapi(fz + c, G.n[2]));
        double f[9];
        acc.load9(g, f);
        double I = 0.0, K0x = 0.0, K1x = 0.0, K0y = 0.0, K1y = 0.0, K0z = 0.0, K1z = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          I += xy[q] * Zw[q][c];
          K0x += dxy[q] * Z0[q][c];
          K1x += dxy[q] * Z1[q][c];
          K0y += xdy[q] * Z0[q][c];
          K1y += xdy[q] * Z1[q][c];
          K0z += xy[q] * dZ0[q][c];
          K1z += xy[q] * dZ1[q][c];
        }
#pragma unroll
        for (int l = 0; l < 3; ++l) {
          gp[l] += f[l] * I;
          D[l][0] += f[3 + l] * K0x + f[6 + l] * K1x;
          D[l][1] += f[3 + l] * K0y + f[6 + l] * K1y;
          D[l][2] += f[3 + l] * K0z + f[6 + l] * K1z;
        }
        if constexpr (WITH_U) {
#pragma unroll
          for (int l = 0; l < 3; ++l) Ub[l] += Uh[l * G.ncell + g] * I;
          pou += I;
        }
      }
    }
  }
}

template <int R, bool WITH_U, class Acc>
__device__ __forceinline__ void gather_piece(const Grid& G, const double* x0, const double* d,
                                             double s0, double s1, const double* base,
                                             const Acc& acc, const double* __restrict__ Uh,
                                             double* gp, double (*D)[3], double* Ub, double& pou) {
  constexpr int NQ = Quad<R>::NQ;
  double sq[NQ], wq[NQ];
  piece_rule<R>(s0, s1, sq, wq);
  gather_points<R, NQ, WITH_U>(G, x0, d, base, sq, wq, acc, Uh, gp, D, Ub, pou);
}

// ---- one orbit piece: gather for the push ----------------------------------
// The push needs grad phi-bar and (D A)^T vbar only.  With b_g(s) = vbar . A_g(s),
//   ((D A)^T vbar)_j = sum_g int b_g(s) d_j S_g(x(s)) ds,
// so each node first contracts its A^n, A^{n+1} with vbar and the quadrature
// then carries one scalar per node instead of the 3x3 matrix D.  The tensor
// product S_g = X_a Y_b Z_c is used once more: along each z column of the
// stencil the quadrature-point sums B_q = sum_c b_c(s_q) Z_c(q) and
// B'_q = sum_c b_c(s_q) Z'_c(q) are formed first, and the x and y factors
// multiply those column sums, not every node.  Derivatives are taken per unit
// of cell coordinate: dtv accumulates H_j ((D A)^T vbar)_j, and the caller
// multiplies by 1/H_j once per particle.
template <int R, int NQ, class Acc>
__device__ __forceinline__ void push_points(const Grid& G, const double* x0, const double* d,
                                            const double* base, const double* sq,
                                            const double* wq, const double* vb, const Acc& acc,
                                            double* gp, double* dtv) {
  constexpr int W = R + 1;
  double tx[NQ], ty[NQ], Z[NQ][W], dZ[NQ][W];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double s = sq[q];
    tx[q] = (x0[0] + s * d[0]) * G.invH[0] - base[0];
    ty[q] = (x0[1] + s * d[1]) * G.invH[1] - base[1];
    Spline<R>::wd((x0[2] + s * d[2]) * G.invH[2] - base[2], Z[q], dZ[q]);
  }
  const int fx = to_int_clamped(base[0]) + Spline<R>::first_off;
  const int fy = to_int_clamped(base[1]) + Spline<R>::first_off;
  const int fz = to_int_clamped(base[2]) + Spline<R>::first_off;
#pragma unroll
  for (int a = 0; a < W; ++a) {
    double Xw[NQ], dXw[NQ];  // quadrature weight x X_a, x dX_a/dx
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double Xq, dXq;
      Spline<R>::wk(a, tx[q], Xq, dXq);
      Xw[q] = wq[q] * Xq;
      dXw[q] = wq[q] * dXq;
    }
#pragma unroll
    for (int b = 0; b < W; ++b) {
      double xyw[NQ], dxyw[NQ], xdyw[NQ];
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        double Yq, dYq;
        Spline<R>::wk(b, ty[q], Yq, dYq);
        xyw[q] = Xw[q] * Yq;
        dxyw[q] = dXw[q] * Yq;
        xdyw[q] = Xw[q] * dYq;
      }
      const int row = acc.row(fx + a, fy + b);
      double B[NQ], dB[NQ];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        const auto p = acc.node(row, fz + c);
        double f[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) f[k] = p[k];
        const double a0 = vb[0] * f[3] + vb[1] * f[4] + vb[2] * f[5];  // vbar . A^n_g
        const double da = vb[0] * f[6] + vb[1] * f[7] + vb[2] * f[8] - a0;
        double I = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          I += xyw[q] * Z[q][c];
          const double bq = a0 + sq[q] * da;  // vbar . A_g(s_q)
          B[q] = c == 0 ? bq * Z[q][c] : B[q] + bq * Z[q][c];
          dB[q] = c == 0 ? bq * dZ[q][c] : dB[q] + bq * dZ[q][c];
        }
        gp[0] += f[0] * I;
        gp[1] += f[1] * I;
        gp[2] += f[2] * I;
      }
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        dtv[0] += dxyw[q] * B[q];
        dtv[1] += xdyw[q] * B[q];
        dtv[2] += xyw[q] * dB[q];
      }
    }
  }
}

template <int R, class Acc>
__device__ __forceinline__ void push_piece(const Grid& G, const double* x0, const double* d,
                                           double s0, double s1, const double* base,
                                           const double* vb, const Acc& acc, double* gp,
                                           double* dtv) {
  constexpr int NQ = Quad<R>::NQ;
  double sq[NQ], wq[NQ];
  piece_rule<R>(s0, s1, sq, wq);
  push_points<R, NQ>(G, x0, d, base, sq, wq, vb, acc, gp, dtv);
}

// point interpolant of A^n (which = 0) or A^{n+1} (which = 1) at x, whose
// stencil nodes are moved into the particle frame by +shift[a] (a multiple
// of n[a]; zero unless x is a wrapped end point)
template <int R, class Acc>
__device__ __forceinline__ void point_A_acc(const Grid& G, const double* x, const int* shift,
                                            const Acc& acc, int which, double* out) {
  constexpr int W = R + 1;
  double w[3][W];
  int f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = x[a] * G.invH[a];
    const double base = floor(u + Spline<R>::base_off);
    Spline<R>::w(u - base, w[a]);
    f[a] = to_int_clamped(base) + Spline<R>::first_off + shift[a];
  }
  out[0] = out[1] = out[2] = 0.0;
  const int off = which ? 6 : 3;
#pragma unroll
  for (int a = 0; a < W; ++a) {
#pragma unroll
    for (int b = 0; b < W; ++b) {
      const int row = acc.row(f[0] + a, f[1] + b);
      const double wxy = w[0][a] * w[1][b];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        const auto p = acc.node(row, f[2] + c);
        const double wt = wxy * w[2][c];
#pragma unroll
        for (int l = 0; l < 3; ++l) out[l] += p[off + l] * wt;
      }
    }
  }
}

// point interpolant F_h(x) = sum_g F_g S_g(x) of A^n (which = 0) or A^{n+1} (which = 1)
template <int R, class Acc>
__device__ __forceinline__ void point_A(const Grid& G, const double* x, const Acc& acc, int which,
                                        double* out) {
  constexpr int W = R + 1;
  double w[3][W];
  int f[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = x[a] * G.invH[a];
    const double base = floor(u + Spline<R>::base_off);
    Spline<R>::w(u - base, w[a]);
    f[a] = to_int_clamped(base) + Spline<R>::first_off;
  }
  out[0] = out[1] = out[2] = 0.0;
#pragma unroll
  for (int a = 0; a < W; ++a) {
    const int ix = wrapi(f[0] + a, G.n[0]);
#pragma unroll
    for (int b = 0; b < W; ++b) {
      const int iy = wrapi(f[1] + b, G.n[1]);
      const double wxy = w[0][a] * w[1][b];
#pragma unroll
      for (int c = 0; c < W; ++c) {
        const int64_t g = node_of(G, ix, iy, wrapi(f[2] + c, G.n[2]));
        const double wt = wxy * w[2][c];
#pragma unroll
        for (int l = 0; l < 3; ++l) out[l] += (which ? acc.A1(g, l) : acc.A0(g, l)) * wt;
      }
    }
  }
}

__device__ __forceinline__ void load3(const double* __restrict__ p, int64_t np, int64_t i,
                                      double* o) {
  o[0] = p[i];
  o[1] = p[np + i];
  o[2] = p[2 * np + i];
}

// ---- kernels ---------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(kBlock) void k_extrapolate(int64_t n3, const T* __restrict__ v,
                                                       const T* __restrict__ vprev,
                                                       double* __restrict__ vit,
                                                       double* __restrict__ vbar) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n3) return;
  const double w = 2.0 * (double)v[i] - (double)vprev[i];  // v^{n+1,0} = 2 v^n - v^{n-1}
  vit[i] = w;
  if (vbar) vbar[i] = 0.5 * (w + (double)v[i]);
}

// Orbit current of a chunk of kChunk particles per block.  Lanes take
// particles with a stride of kChunk / 64 inside the chunk, so that for
// cell-sorted particles the 64 lanes of a wavefront sit in up to
// kChunk / (particles per cell) different cells and their LDS atomics rarely
// hit the same address.
// Pass 1 finds the box of nodes the chunk's orbits touch (unwrapped indices
// relative to the chunk's first particle, one node of margin per side);
// pass 2 accumulates the current in an LDS tile over that box; the tile is
// then flushed with one global atomic per non-zero node value.  A chunk whose
// box exceeds the tile adds straight to global memory.  A 4096-particle chunk
// spans 64 cells at 64 particles per cell, so the 64 lanes of a wavefront sit
// in 64 different cells and their atomics never meet on one address (2048
// particles put two lanes in every cell: scatter 0.287 -> 0.245 ms at 32^3);
// the 3072-node tile (72 KB) still leaves room for two blocks per CU.  Where
// the box of such a chunk does not fit (more particles per cell, longer
// orbits: the 64^3 thermal workload) blocks count the miss and the host
// switches to 2048-particle chunks; cubic stencils use those from the start.
// Quadratic and linear 2048-particle chunks fit a 2048-node tile (48 KB),
// which lets three blocks share a CU (three waves per SIMD at 168 registers:
// 64^3 mixed scatter 5.04 -> 4.79 ms per pass); the cubic ones need 3072.
template <int R, int CH>
struct ScatterChunk {
  static constexpr int kChunk = CH;
  static constexpr int kPerThread = kChunk / kBlock;  // particles per thread
  static constexpr int kTileNodes = (CH == 2048 && R < 3) ? 2048 : 3072;
  static constexpr int kWavesPerSimd = (CH == 2048 && R < 3) ? 3 : 1;  // minimum asked for
};

// t / d for 0 <= t < 2^22 and d >= 1, with inv_d = 1.0f / d: (t + 1/2) / d
// lies at least 1/(2d) away from an integer, further than the float rounding
// error (t + 1/2) 2^-23 / d, so the truncation is exact (no integer division)
__device__ __forceinline__ int div_small(int t, float inv_d) {
  return (int)(((float)t + 0.5f) * inv_d);
}

template <int CH>
__device__ __forceinline__ int64_t chunk_particle(int64_t base, int k) {
  return base + (int64_t)(threadIdx.x % kWave) * (CH / kWave) + threadIdx.x / kWave +
         (int64_t)(kBlock / kWave) * k;
}

// x^n, vbar^p = (v^{n+1,p} + v^n) / 2 and the unwrapped displacement
// d = dt vbar^p of particle i; vbar^p read from vbar when the previous pass
// (or the step's set-up) wrote it, else formed from v^n and the iterate
template <class PS>
__device__ __forceinline__ void orbit_of(const StepParams& P, const PS& st,
                                         const double* __restrict__ vit,
                                         const double* __restrict__ vbar, int64_t i, double* x0,
                                         double* d, double* vb) {
  st.x_of(P.G, P.np, i, x0);
  if (vbar) {
    load3(vbar, P.np, i, vb);
  } else {
    double va[3], vi[3];
    st.v_of(P.np, i, va);
    load3(vit, P.np, i, vi);
#pragma unroll
    for (int a = 0; a < 3; ++a) vb[a] = 0.5 * (vi[a] + va[a]);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) d[a] = P.dt * vb[a];
}

// Fixed-point quantum count of a current contribution w: the product
// w x scale rounded once to the nearest integer (ties to even), as the
// two's-complement bit pattern that 64-bit integer atomics add.  Adding
// 1.5 x 2^52 in the same fused operation leaves that integer in the low
// mantissa bits of the sum while the sum stays in (2^52, 2^53), which holds
// for |w scale| < 2^50: one FMA and one 64-bit subtraction in place of a
// rounding and a software FP64 -> int64 conversion.  The caller guarantees
// the range (the scatter checks it once per particle and flags a particle
// outside it).
__device__ __forceinline__ unsigned long long quantize_in_range(double w, double scale) {
  constexpr double kMagic = 0x1.8p52;
  const double t = fma(w, scale, kMagic);
  return (unsigned long long)(__double_as_longlong(t) - __double_as_longlong(kMagic));
}

// Bound on |w scale| for quantize_in_range.  The orbit weights of a piece
// are at most 1, so a particle whose |c_l| scale stays below it has every
// contribution in range.
constexpr double kFixedRange = 0x1p50;

// The same rounding for any w (a conversion outside the range).
__device__ __forceinline__ unsigned long long quantize(double w, double scale) {
  if (fabs(w) * scale < kFixedRange) return quantize_in_range(w, scale);
  return (unsigned long long)(long long)rint(w * scale);
}

// MULTI: the particles carry species (one byte each); otherwise every
// particle has the coefficients of species 0, kept in scalar registers
template <int R, class PS, bool SPLIT, bool MULTI, int CH>
__global__ __launch_bounds__(kBlock) __attribute__((
    amdgpu_waves_per_eu(ScatterChunk<R, CH>::kWavesPerSimd))) void k_scatter(StepParams P, PS st,
                                                   const double* __restrict__ vit,
                                                   const double* __restrict__ vbar,
                                                   CurrentOut out, Scratch sc,
                                                   ChunkBoxes bx) {
  constexpr int W = R + 1;
  constexpr bool FIX = PS::kMixed;  // int64 fixed-point deposit
  constexpr int kTileNodes = ScatterChunk<R, CH>::kTileNodes;
  __shared__ double tile[3 * kTileNodes];  // FIX: int64 quanta in the same bytes
  __shared__ int s_ref[3];
  unsigned long long* tile_q = reinterpret_cast<unsigned long long*>(tile);
  constexpr int kChunk = ScatterChunk<R, CH>::kChunk, kPerThread = ScatterChunk<R, CH>::kPerThread;
  const int64_t base = (int64_t)blockIdx.x * kChunk;
  double js[1] = {0.0};
  double bad = 0.0;
  late_reduce_init<2>();
  // the chunk's node box: reference cell sref (that of the chunk's first
  // particle), origin tlo relative to it and extents dim, per axis
  int sref[3], tlo[3], dim[3];
  if (bx.reuse) {  // found by this chunk in the step's first pass
    const int* b = bx.box + (int64_t)blockIdx.x * kBoxInts;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      sref[a] = b[a];
      tlo[a] = b[3 + a];
      dim[a] = b[6 + a];
    }
  } else {
    if (threadIdx.x == 0) {
      double x0[3];
      st.x_of(P.G, P.np, base, x0);
#pragma unroll
      for (int a = 0; a < 3; ++a)
        s_ref[a] = to_int_clamped(floor(x0[a] * P.G.invH[a] + Spline<R>::base_off));
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; ++a) sref[a] = s_ref[a];
    // pass 1: the box of the nodes the chunk's orbits touch
    int rmin[3] = {0x3fffffff, 0x3fffffff, 0x3fffffff};
    int rmax[3] = {-0x3fffffff, -0x3fffffff, -0x3fffffff};
    for (int k = 0; k < kPerThread; ++k) {
      const int64_t i = chunk_particle<CH>(base, k);
      if (i >= P.np) continue;
      double x0[3], d[3], vb[3];
      orbit_of(P, st, vit, vbar, i, x0, d, vb);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double u0 = x0[a] * P.G.invH[a], u1 = (x0[a] + d[a]) * P.G.invH[a];
        const int lo = to_int_clamped(floor(fmin(u0, u1) + Spline<R>::base_off)) + Spline<R>::first_off - 1;
        const int hi = to_int_clamped(floor(fmax(u0, u1) + Spline<R>::base_off)) + Spline<R>::first_off + W;
        const int rel = min_image(lo - sref[a], P.G.n[a]);
        rmin[a] = min(rmin[a], rel);
        rmax[a] = max(rmax[a], rel + (hi - lo));
      }
    }
    int mv[6] = {rmin[0], rmin[1], rmin[2], -rmax[0], -rmax[1], -rmax[2]};
    block_min_ints<6>(mv);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      tlo[a] = mv[a];
      dim[a] = -mv[3 + a] - tlo[a] + 1;
    }
    if (bx.box && threadIdx.x == 0) {
      int* b = bx.box + (int64_t)blockIdx.x * kBoxInts;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        b[a] = sref[a];
        b[3 + a] = tlo[a];
        b[6 + a] = dim[a];
      }
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {  // block-uniform
    sref[a] = __builtin_amdgcn_readfirstlane(sref[a]);
    tlo[a] = __builtin_amdgcn_readfirstlane(tlo[a]);
    dim[a] = __builtin_amdgcn_readfirstlane(dim[a]);
  }
  // block-uniform; each extent is bounded first so that the product cannot overflow
  const bool use_tile = dim[0] > 0 && dim[0] <= kTileNodes && dim[1] <= kTileNodes &&
                        dim[2] <= kTileNodes && (int64_t)dim[0] * dim[1] * dim[2] <= kTileNodes;
  const int nt = use_tile ? dim[0] * dim[1] * dim[2] : 0;
  if (!use_tile && threadIdx.x == 0) unsafeAtomicAdd(sc.spread_copy(S_SMISS), 1.0);
  for (int t = threadIdx.x; t < 3 * nt; t += kBlock) tile[t] = 0.0;  // also integer zero
  __syncthreads();
  // pass 2: accumulate.  Pieces whose stencil lies outside the tile are
  // skipped and their particles marked; a third pass adds those pieces to
  // global memory.  Keeping the global path out of the main loop keeps the
  // loop's register count (and so the kernel's occupancy) that of the tile path.
  const int64_t nc = P.G.ncell;
  unsigned outside_mask = 0u;
  auto process = [&](int k, auto global_phase) -> bool {
    constexpr bool GLOBAL = decltype(global_phase)::value;
    bool outside = false;
    const int64_t i = chunk_particle<CH>(base, k);
    if (i >= P.np) return false;
    double x0[3], d[3], vb[3], c3[3];
    orbit_of(P, st, vit, vbar, i, x0, d, vb);
    if (!GLOBAL) {  // J_s: q_i max_a |vbar_a|, once per particle
      const double vmax = fmax(fabs(vb[0]), fmax(fabs(vb[1]), fabs(vb[2])));
      js[0] += (MULTI ? species_value(P.aq, st.species(i)) : P.aq[0]) * vmax;
    }
    // FP64: q_i vbar / dV; fixed point: (q_i / q_0) vbar in units of the quantum
    const double cq = MULTI ? species_value(P.cq, st.species(i)) : P.cq[0];
    int shift[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c3[a] = cq * vb[a];
      const double u0 = x0[a] * P.G.invH[a], u1 = (x0[a] + d[a]) * P.G.invH[a];
      const int lo = to_int_clamped(floor(fmin(u0, u1) + Spline<R>::base_off)) + Spline<R>::first_off - 1;
      const int raw = lo - sref[a];
      shift[a] = min_image(raw, P.G.n[a]) - raw;  // particle frame -> chunk frame
    }
    auto deposit = [&](const double (&Iw)[W][W][W], const int* f) {
      const int ox = f[0] - sref[0] + shift[0] - tlo[0];
      const int oy = f[1] - sref[1] + shift[1] - tlo[1];
      const int oz = f[2] - sref[2] + shift[2] - tlo[2];
      const bool inside = use_tile && ox >= 0 && oy >= 0 && oz >= 0 && ox + W <= dim[0] &&
                          oy + W <= dim[1] && oz + W <= dim[2];
      outside = outside || !inside;
      if (!GLOBAL && inside) {
#pragma unroll
        for (int a = 0; a < W; ++a)
#pragma unroll
          for (int b = 0; b < W; ++b)
#pragma unroll
            for (int c = 0; c < W; ++c) {
              const int t = ((ox + a) * dim[1] + (oy + b)) * dim[2] + (oz + c);
              const double w = Iw[a][b][c];
#pragma unroll
              for (int l = 0; l < 3; ++l) {
                if constexpr (FIX)
                  atomicAdd(&tile_q[3 * t + l], quantize_in_range(w * c3[l], out.fix_scale));
                else
                  atomicAdd(&tile[3 * t + l], w * c3[l]);
              }
            }
      } else if (GLOBAL && !inside) {
#pragma unroll
        for (int a = 0; a < W; ++a)
#pragma unroll
          for (int b = 0; b < W; ++b)
#pragma unroll
            for (int c = 0; c < W; ++c) {
              const int64_t g = node_index(P.G, f[0] + a, f[1] + b, f[2] + c);
              const double w = Iw[a][b][c];
#pragma unroll
              for (int l = 0; l < 3; ++l) {
                if constexpr (FIX)
                  atomicAdd(out.Jfix + l * nc + g, quantize_in_range(w * c3[l], out.fix_scale));
                else
                  unsafeAtomicAdd(out.J + l * nc + g, w * c3[l]);
              }
            }
      }
    };
    // Cubic stencils (64 nodes): the weights are never held all at once.
    // Per quadrature point the three 1-D factors are kept (wq folded into the
    // x factor); each node's weight is summed over the points when it is
    // deposited.  Same integrals, a quarter of the registers.
    auto deposit_factored = [&](const double (&X)[Quad<R>::NQ][W],
                                const double (&Y)[Quad<R>::NQ][W],
                                const double (&Z)[Quad<R>::NQ][W], const int* f) {
      constexpr int NQ = Quad<R>::NQ;
      const int ox = f[0] - sref[0] + shift[0] - tlo[0];
      const int oy = f[1] - sref[1] + shift[1] - tlo[1];
      const int oz = f[2] - sref[2] + shift[2] - tlo[2];
      const bool inside = use_tile && ox >= 0 && oy >= 0 && oz >= 0 && ox + W <= dim[0] &&
                          oy + W <= dim[1] && oz + W <= dim[2];
      outside = outside || !inside;
      if (GLOBAL == inside) return;
#pragma unroll
      for (int a = 0; a < W; ++a)
#pragma unroll
        for (int b = 0; b < W; ++b) {
          double xy[NQ];
#pragma unroll
          for (int q = 0; q < NQ; ++q) xy[q] = X[q][a] * Y[q][b];
#pragma unroll
          for (int c = 0; c < W; ++c) {
            double w = 0.0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) w += xy[q] * Z[q][c];
            if (!GLOBAL) {
              const int t = ((ox + a) * dim[1] + (oy + b)) * dim[2] + (oz + c);
#pragma unroll
              for (int l = 0; l < 3; ++l) {
                if constexpr (FIX)
                  atomicAdd(&tile_q[3 * t + l], quantize_in_range(w * c3[l], out.fix_scale));
                else
                  atomicAdd(&tile[3 * t + l], w * c3[l]);
              }
            } else {
              const int64_t g = node_index(P.G, f[0] + a, f[1] + b, f[2] + c);
#pragma unroll
              for (int l = 0; l < 3; ++l) {
                if constexpr (FIX)
                  atomicAdd(out.Jfix + l * nc + g, quantize_in_range(w * c3[l], out.fix_scale));
                else
                  unsafeAtomicAdd(out.J + l * nc + g, w * c3[l]);
              }
            }
          }
        }
    };
    bool ok = true;
    if constexpr (SPLIT && R >= 3) {
      ok = for_each_piece<R>(x0, d, P.G, [&](double s0, double s1, const double* base) {
        constexpr int NQ = Quad<R>::NQ;
        double sq[NQ], wq[NQ], X[NQ][W], Y[NQ][W], Z[NQ][W];
        int f[3];
        piece_rule<R>(s0, s1, sq, wq);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const double sv = sq[q];
          Spline<R>::w((x0[0] + sv * d[0]) * P.G.invH[0] - base[0], X[q]);
          Spline<R>::w((x0[1] + sv * d[1]) * P.G.invH[1] - base[1], Y[q]);
          Spline<R>::w((x0[2] + sv * d[2]) * P.G.invH[2] - base[2], Z[q]);
#pragma unroll
          for (int a = 0; a < W; ++a) X[q][a] *= wq[q];
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) f[a] = to_int_clamped(base[a]) + Spline<R>::first_off;
        deposit_factored(X, Y, Z, f);
      });
    } else if constexpr (SPLIT) {
      // One x slice of the stencil at a time: the point sums of its 3 x 3 nodes
      // are deposited before the next slice's are formed, so only 9 weights
      // are live (the same sums, in the same order, as the whole stencil's;
      // 161 instead of 179 registers, no spills in the 2048-particle form).
      ok = for_each_piece<R>(x0, d, P.G, [&](double s0, double s1, const double* base) {
        constexpr int NQ = Quad<R>::NQ;
        double sq[NQ], wq[NQ], tx[NQ], Y[NQ][W], Z[NQ][W];
        piece_rule<R>(s0, s1, sq, wq);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          tx[q] = (x0[0] + sq[q] * d[0]) * P.G.invH[0] - base[0];
          Spline<R>::w((x0[1] + sq[q] * d[1]) * P.G.invH[1] - base[1], Y[q]);
          Spline<R>::w((x0[2] + sq[q] * d[2]) * P.G.invH[2] - base[2], Z[q]);
        }
        int f[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) f[a] = to_int_clamped(base[a]) + Spline<R>::first_off;
        const int ox = f[0] - sref[0] + shift[0] - tlo[0];
        const int oy = f[1] - sref[1] + shift[1] - tlo[1];
        const int oz = f[2] - sref[2] + shift[2] - tlo[2];
        const bool inside = use_tile && ox >= 0 && oy >= 0 && oz >= 0 && ox + W <= dim[0] &&
                            oy + W <= dim[1] && oz + W <= dim[2];
        outside = outside || !inside;
        if (GLOBAL == inside) return;
#pragma unroll
        for (int a = 0; a < W; ++a) {
          double Ia[W][W];
#pragma unroll
          for (int b = 0; b < W; ++b)
#pragma unroll
            for (int c = 0; c < W; ++c) Ia[b][c] = 0.0;
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            double Xq, dXq;
            Spline<R>::wk(a, tx[q], Xq, dXq);
            const double xa = wq[q] * Xq;
#pragma unroll
            for (int b = 0; b < W; ++b) {
              const double xy = xa * Y[q][b];
#pragma unroll
              for (int c = 0; c < W; ++c) Ia[b][c] += xy * Z[q][c];
            }
          }
#pragma unroll
          for (int b = 0; b < W; ++b)
#pragma unroll
            for (int c = 0; c < W; ++c) {
              const double w = Ia[b][c];
              if (!GLOBAL) {
                const int t = ((ox + a) * dim[1] + (oy + b)) * dim[2] + (oz + c);
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                  if constexpr (FIX)
                    atomicAdd(&tile_q[3 * t + l], quantize_in_range(w * c3[l], out.fix_scale));
                  else
                    atomicAdd(&tile[3 * t + l], w * c3[l]);
                }
              } else {
                const int64_t g = node_index(P.G, f[0] + a, f[1] + b, f[2] + c);
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                  if constexpr (FIX)
                    atomicAdd(out.Jfix + l * nc + g, quantize_in_range(w * c3[l], out.fix_scale));
                  else
                    unsafeAtomicAdd(out.J + l * nc + g, w * c3[l]);
                }
              }
            }
        }
      });
    } else {
      for (int q = 0; q < P.rule.n; ++q) {
        double base[3], sq, wq, Iw[W][W][W];
        int f[3];
        unsplit_point<R>(P.G, P.rule, q, x0, d, base, sq, wq);
        sbar_points<R, 1>(P.G, x0, d, base, &sq, &wq, Iw, f);
        deposit(Iw, f);
      }
    }
    if (!ok && !GLOBAL) bad = 1.0;
    if constexpr (FIX) {  // contributions beyond the fixed-point range
      const double cmax = fmax(fabs(c3[0]), fmax(fabs(c3[1]), fabs(c3[2])));
      if (!GLOBAL && !(cmax * out.fix_scale < kFixedRange)) bad = fmax(bad, 1.5);
    }
    return outside;
  };
  for (int k = 0; k < kPerThread; ++k)
    if (process(k, std::false_type{})) outside_mask |= 1u << k;
  for (int k = 0; k < kPerThread; ++k)
    if ((outside_mask >> k) & 1u) process(k, std::true_type{});
  __syncthreads();
  const float inv_d1 = 1.0f / (float)max(dim[1], 1), inv_d2 = 1.0f / (float)max(dim[2], 1);
  for (int t = threadIdx.x; t < nt; t += kBlock) {
    const int q = div_small(t, inv_d2), cx = div_small(q, inv_d1);
    const int cz = t - q * dim[2], cy = q - cx * dim[1];
    const int64_t g = node_index(P.G, sref[0] + tlo[0] + cx, sref[1] + tlo[1] + cy,
                                 sref[2] + tlo[2] + cz);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      if constexpr (FIX) {
        const unsigned long long val = tile_q[3 * t + l];
        if (val != 0ull) atomicAdd(out.Jfix + l * nc + g, val);
      } else {
        const double val = tile[3 * t + l];
        if (val != 0.0) unsafeAtomicAdd(out.J + l * nc + g, val);
      }
    }
  }
  const double part[2] = {js[0], bad};
  const bool ismax[2] = {false, true};
  double blk[2];
  if (late_reduce<2>(part, ismax, blk)) {
    sc.region(P_JS)[blockIdx.x] = blk[0];  // J_s partials, summed in order by k_finish
    atomic_max_nonneg(sc.spread_copy(S_BAD), blk[1]);
  }
}

// Gather + push of one particle (index i of store st) through accessor acc:
// grad phi-bar and (D A)^T vbar over the orbit pieces, then P^{n+1,p} and
// v^{n+1,p+1}.  v^n is read again after the orbit loop rather than kept in
// registers through it (the loop sets the kernel's register count).
template <int R, bool SPLIT, class Acc, class PS>
__device__ __forceinline__ void gather_push_one(const StepParams& P, const Acc& acc, const PS& st,
                                                int64_t i, const double* x0, const double* d,
                                                const double* vb, double qi, double mi,
                                                double* vn, double& npieces, double& bad) {
  double gp[3] = {0.0, 0.0, 0.0};
  double dtv[3] = {0.0, 0.0, 0.0};  // H_j ((D A)^T vbar)_j until the pieces are summed
  if constexpr (SPLIT) {
    const bool ok = for_each_piece<R>(x0, d, P.G, [&](double s0, double s1, const double* base) {
      push_piece<R>(P.G, x0, d, s0, s1, base, vb, acc, gp, dtv);
      npieces += 1.0;
    });
    if (!ok) bad = 1.0;
  } else {
    for (int q = 0; q < P.rule.n; ++q) {
      double base[3], sq, wq;
      unsplit_point<R>(P.G, P.rule, q, x0, d, base, sq, wq);
      push_points<R, 1>(P.G, x0, d, base, &sq, &wq, vb, acc, gp, dtv);
    }
    npieces += 1.0;
  }
  // A_h^n(x^n) rebuilds P^n = m v^n + q A_h^n(x^n) (eq. discrete-canonical-relation);
  // A_h^{n+1}(x^{n+1}) at the wrapped end point closes the velocity (eq. orbit-v-update).
  double va[3];
  asm volatile("" ::: "memory");  // a fresh load, not the value from before the loop
  st.v_of(P.np, i, va);
  double x1[3], A0s[3], A1e[3];
  int zero[3] = {0, 0, 0}, sh1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    x1[a] = wrap_pos(x0[a] + d[a], P.G.L[a], P.G.invL[a]);
    sh1[a] = (int)rint((x0[a] + d[a] - x1[a]) * P.G.invL[a]) * P.G.n[a];
  }
  point_A_acc<R>(P.G, x0, zero, acc, 0, A0s);
  point_A_acc<R>(P.G, x1, sh1, acc, 1, A1e);
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const double Pn = mi * va[j] + qi * A0s[j];
    const double DAv = dtv[j] * P.G.invH[j];                  // ((D A)^T vbar)_j
    const double P1 = Pn + P.dt * (-qi * gp[j] + qi * DAv);   // eq. orbit-P-update
    vn[j] = (P1 - qi * A1e[j]) / mi;                          // eq. orbit-v-update
  }
}

// One block = 256 cell-sorted particles.  TILED = true: the block finds the
// box of nodes its orbits touch from the rounded u0 and u1 of each orbit, with
// one node of margin per side (a piece's knot interval, decided against the
// knot positions, differs from the interval of a rounded end point only
// within rounding of a knot, and then by one), copies the gather fields of
// that box into LDS, and
// every stencil read of the node loop then comes from LDS; a block whose box
// does not fit the tile appends its index to a work list (work[0] = count,
// work[1..] = block indices).  After the first Picard pass of a step the
// block takes the box it stored in an earlier pass and starts copying at
// once; if one of its orbits has moved out of that box (by the margin test
// above) it finds and stores the box again, and copies again.  TILED = false: the blocks on that list (all
// blocks when work is null) read the gather buffer in global memory, a small
// grid looping over the list.  Two kernels keep each one's register budget.
constexpr int kGatherTileNodes = 512;
constexpr int kGatherListGrid = 512;  // blocks of the global-memory kernel with a list

// Block bid of 256 particles; thread 0 must have run late_reduce_init<4>()
// and late_reduce_init<2>() before a barrier that precedes the call.
template <int R, bool TILED, class PS, bool SPLIT>
__device__ __forceinline__ void gather_block(const StepParams& P, const PS& st,
                                             const double* __restrict__ vit,
                                             double* __restrict__ vnew,
                                             double* __restrict__ vbar_out, const AosFields& F,
                                             int* __restrict__ work, const Scratch& sc,
                                             const AndersonPrev& prev, int bid,
                                             const ChunkBoxes& bx) {
  constexpr int W = R + 1;
  const int64_t i = (int64_t)bid * kBlock + threadIdx.x;
  const bool active = i < P.np;
  double dvm = 0.0, vm = 0.0, bad = 0.0;
  double npieces[1] = {0.0};
  double x0[3] = {0.0, 0.0, 0.0}, va[3] = {0.0, 0.0, 0.0}, vi[3] = {0.0, 0.0, 0.0};
  double vb[3] = {0.0, 0.0, 0.0}, d[3] = {0.0, 0.0, 0.0};
  double qi = P.q, mi = P.m;
  if (active) {
    const int spc = st.species(i);
    qi = species_value(P.qs, spc);
    mi = species_value(P.ms, spc);
    st.x_of(P.G, P.np, i, x0);
    st.v_of(P.np, i, va);
    load3(vit, P.np, i, vi);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vb[a] = 0.5 * (vi[a] + va[a]);
      d[a] = P.dt * vb[a];
    }
  }
  double vn[3] = {0.0, 0.0, 0.0};
  if constexpr (TILED) {
    __shared__ double2 tile2[kGatherTileNodes * kGbufStride / 2];
    __shared__ int s_ref[3];
    __shared__ int s_out[kBlock / kWave];
    int lo[3] = {0, 0, 0}, span[3] = {0, 0, 0};
    if (active) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double u0 = x0[a] * P.G.invH[a], u1 = (x0[a] + d[a]) * P.G.invH[a];
        lo[a] = to_int_clamped(floor(fmin(u0, u1) + Spline<R>::base_off)) + Spline<R>::first_off - 1;
        span[a] = to_int_clamped(floor(fmax(u0, u1) + Spline<R>::base_off)) +
                  Spline<R>::first_off + W - lo[a];
      }
    }
    // the block's node box: reference node sref, origin tlo relative to it and
    // extents dim, per axis (dim[0] < 0: the box overflows the tile)
    int sref[3], shift[3], tlo[3], dim[3];
    auto uniform = [&]() {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sref[a] = __builtin_amdgcn_readfirstlane(sref[a]);
        tlo[a] = __builtin_amdgcn_readfirstlane(tlo[a]);
        dim[a] = __builtin_amdgcn_readfirstlane(dim[a]);
      }
    };
    auto to_global_kernel = [&]() {
      if (threadIdx.x == 0) work[1 + atomicAdd(work, 1)] = bid;
    };
    auto fill_tile = [&]() {
      const int nt2 = dim[0] * dim[1] * dim[2] * (kGbufStride / 2);
      const double2* g2 = reinterpret_cast<const double2*>(F.g);
      const float inv_d1 = 1.0f / (float)dim[1], inv_d2 = 1.0f / (float)dim[2];
      for (int t = threadIdx.x; t < nt2; t += kBlock) {
        const int nd = t / (kGbufStride / 2), part = t % (kGbufStride / 2);
        const int q = div_small(nd, inv_d2), cx = div_small(q, inv_d1);
        const int cz = nd - q * dim[2], cy = q - cx * dim[1];
        const int64_t g = node_index(P.G, sref[0] + tlo[0] + cx, sref[1] + tlo[1] + cy,
                                     sref[2] + tlo[2] + cz);
        tile2[t] = g2[g * (kGbufStride / 2) + part];
      }
    };
    bool find_box = true;
    if (bx.reuse) {  // the box this block found in an earlier pass of the step
      const int* b = bx.box + (int64_t)bid * kBoxInts;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sref[a] = b[a];
        tlo[a] = b[3 + a];
        dim[a] = b[6 + a];
      }
      uniform();
      if (dim[0] < 0) {
        to_global_kernel();
        return;
      }
      bool outside = false;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int raw = lo[a] - sref[a];
        const int rel = min_image(raw, P.G.n[a]);
        shift[a] = rel - raw;
        outside = outside || (active && (rel < tlo[a] || rel + span[a] > tlo[a] + dim[a] - 1));
      }
      fill_tile();  // the loads start before the vote below is known
      const bool wave_out = __ballot(outside) != 0ull;  // all lanes take part
      if (threadIdx.x % kWave == 0) s_out[threadIdx.x / kWave] = wave_out;
      __syncthreads();
      find_box = false;
#pragma unroll
      for (int w = 0; w < kBlock / kWave; ++w) find_box = find_box || s_out[w] != 0;
    }
    if (find_box) {  // first pass of the step, or an orbit left the stored box
      if (threadIdx.x == 0)
#pragma unroll
        for (int a = 0; a < 3; ++a) s_ref[a] = lo[a];
      __syncthreads();
      int mv[6];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sref[a] = s_ref[a];
        const int raw = lo[a] - sref[a];
        const int rel = min_image(raw, P.G.n[a]);
        shift[a] = rel - raw;
        mv[a] = active ? rel : 0x3fffffff;
        mv[3 + a] = active ? -(rel + span[a]) : 0x3fffffff;
      }
      block_min_ints<6>(mv);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        tlo[a] = mv[a];
        dim[a] = -mv[3 + a] - tlo[a] + 1;
      }
      // each extent is bounded first so that the product cannot overflow
      const bool fits = dim[0] <= kGatherTileNodes && dim[1] <= kGatherTileNodes &&
                        dim[2] <= kGatherTileNodes &&
                        (int64_t)dim[0] * dim[1] * dim[2] <= kGatherTileNodes;
      if (!fits) dim[0] = -1;
      uniform();
      if (bx.box && threadIdx.x == 0) {
        int* b = bx.box + (int64_t)bid * kBoxInts;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          b[a] = sref[a];
          b[3 + a] = tlo[a];
          b[6 + a] = dim[a];
        }
      }
      if (dim[0] < 0) {
        to_global_kernel();
        return;
      }
      fill_tile();
      __syncthreads();
    }
    if (active) {
      TileGather acc;
      acc.t = (lds_cdouble*)(reinterpret_cast<double*>(tile2));
      acc.ox = shift[0] - sref[0] - tlo[0];
      acc.oy = shift[1] - sref[1] - tlo[1];
      acc.oz = shift[2] - sref[2] - tlo[2];
      acc.dy = dim[1];
      acc.dz = dim[2];
      gather_push_one<R, SPLIT>(P, acc, st, i, x0, d, vb, qi, mi, vn, npieces[0], bad);
    }
  } else {
    if (active) {
      GlobalGather acc{F.g, P.G.mask[0], P.G.mask[1], P.G.mask[2], P.G.shx, P.G.shy};
      gather_push_one<R, SPLIT>(P, acc, st, i, x0, d, vb, qi, mi, vn, npieces[0], bad);
    }
  }
  if (active) {
    // v^n and v^{n+1,p} again (see gather_push_one)
    asm volatile("" ::: "memory");
    st.v_of(P.np, i, va);
    load3(vit, P.np, i, vi);
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      vnew[j * P.np + i] = vn[j];
      if (vbar_out) vbar_out[j * P.np + i] = 0.5 * (vn[j] + va[j]);  // the next pass's vbar
      dvm = fmax(dvm, fabs(vn[j] - vi[j]));
      vm = fmax(vm, fabs(vn[j]));
      if (!isfinite(vn[j])) bad = 2.0;  // max-reductions drop NaN: flag it explicitly
    }
  }
  // no block barrier after the orbit loops: a wavefront with fewer pieces
  // does not wait for the block's slowest one
  const double part[4] = {dvm, vm, bad, npieces[0]};
  const bool ismax[4] = {true, true, true, false};
  double blk[4];
  if (late_reduce<4>(part, ismax, blk)) {
    atomic_max_nonneg(sc.spread_copy(S_DVMAX), blk[0]);
    atomic_max_nonneg(sc.spread_copy(S_VMAX), blk[1]);
    atomic_max_nonneg(sc.spread_copy(S_BAD), blk[2]);
    // integer counts: the atomic sum is exact and order-free
    if (blk[3] > 0.0) unsafeAtomicAdd(sc.spread_copy(S_PIECES), blk[3]);
  }
  if (prev.w) {  // Anderson mixing over one difference: dF . dF and dF . f_p
    double aa[2] = {0.0, 0.0};
    if (active) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int64_t e = j * P.np + i;
        const double f0 = vn[j] - vi[j], df = f0 - (prev.g[e] - prev.w[e]);
        aa[0] += df * df;
        aa[1] += df * f0;
      }
    }
    const bool sums[2] = {false, false};
    double ab[2];
    if (late_reduce<2>(aa, sums, ab)) {
      const int64_t nb = (P.np + kBlock - 1) / kBlock;
      sc.region(P_AA)[bid] = ab[0];
      sc.region(P_AA)[nb + bid] = ab[1];
    }
  }
}

// Two waves per SIMD for the tiled quadratic gather: its orbit loop fits 256
// registers, and asking for the occupancy makes the compiler keep it (it would
// otherwise go to one wave and twice the registers for a few more values).
// The global-memory kernel, which only takes blocks whose box overflows the
// tile, is left to the compiler's choice.
template <int R, bool TILED>
constexpr int kGatherWavesPerSimd = (R == 2 && TILED) ? 2 : 1;

template <int R, bool TILED, class PS, bool SPLIT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    kGatherWavesPerSimd<R, TILED>))) void k_gather_push(StepParams P, PS st,
                                                       const double* __restrict__ vit,
                                                       double* __restrict__ vnew,
                                                       double* __restrict__ vbar_out, AosFields F,
                                                       int* __restrict__ work, Scratch sc,
                                                       AndersonPrev prev, ChunkBoxes bx) {
  if (TILED || !work) {
    late_reduce_init<4>();
    late_reduce_init<2>();
    if (!TILED) __syncthreads();  // the tiled path has a barrier before its first use
    gather_block<R, TILED, PS, SPLIT>(P, st, vit, vnew, vbar_out, F, work, sc, prev, blockIdx.x,
                                      bx);
    return;
  }
  const int count = work[0];  // written by the tiled kernel (previous launch)
  for (int j = blockIdx.x; j < count; j += gridDim.x) {
    __syncthreads();  // the previous block's LDS reductions are complete
    late_reduce_init<4>();
    late_reduce_init<2>();
    __syncthreads();
    gather_block<R, TILED, PS, SPLIT>(P, st, vit, vnew, vbar_out, F, work, sc, prev, work[1 + j],
                                      ChunkBoxes{});
  }
}

// Consistency sweep of the accepted iterate: Ubar, Ebar = -gphibar - Ubar,
// sum_i q vbar . Ebar, R_A = A_h^{n+1}(x^{n+1}) - A_h^n(x^n) - dt (Ubar + D vbar)
// (eq. RA-test) and the partition of unity sum_g Sbar_g.
template <int R, class PS, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_sweep(StepParams P, PS st,
                                                 const double* __restrict__ vit, AosFields F,
                                                 const double* __restrict__ Uh, Scratch sc) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double sums[2] = {0.0, 0.0};  // work, |R_A|^2
  double ramax = 0.0, poudev = 0.0;
  if (i < P.np) {
    const double qi = species_value(P.qs, st.species(i));
    double x0[3], va[3], vi[3], vb[3], d[3];
    st.x_of(P.G, P.np, i, x0);
    st.v_of(P.np, i, va);
    load3(vit, P.np, i, vi);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      vb[a] = 0.5 * (vi[a] + va[a]);
      d[a] = P.dt * vb[a];
    }
    double gp[3] = {0.0, 0.0, 0.0}, Ub[3] = {0.0, 0.0, 0.0};
    double D[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    double pou = 0.0;
    if constexpr (SPLIT) {
      for_each_piece<R>(x0, d, P.G, [&](double s0, double s1, const double* base) {
        gather_piece<R, true>(P.G, x0, d, s0, s1, base, F, Uh, gp, D, Ub, pou);
      });
    } else {
      for (int q = 0; q < P.rule.n; ++q) {
        double base[3], sq, wq;
        unsplit_point<R>(P.G, P.rule, q, x0, d, base, sq, wq);
        gather_points<R, 1, true>(P.G, x0, d, base, &sq, &wq, F, Uh, gp, D, Ub, pou);
      }
    }
    double x1[3], A0s[3], A1e[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) x1[a] = wrap_pos(x0[a] + d[a], P.G.L[a], P.G.invL[a]);
    point_A<R>(P.G, x0, F, 0, A0s);
    point_A<R>(P.G, x1, F, 1, A1e);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const double Dv = D[l][0] * vb[0] + D[l][1] * vb[1] + D[l][2] * vb[2];
      const double ra = A1e[l] - A0s[l] - P.dt * (Ub[l] + Dv);
      sums[1] += ra * ra;
      ramax = fmax(ramax, fabs(ra));
      sums[0] += qi * vb[l] * (-gp[l] - Ub[l]);
    }
    poudev = fabs(pou - 1.0);
  }
  block_max_to(ramax, sc.red + S_RAMAX);
  block_max_to(poudev, sc.red + S_POU);
  double s2[2] = {sums[0], sums[1]};
  block_partials<2>(s2, sc.region(P_SWEEP));  // -> S_WORK, S_RA2
}

// Accept the step: x^{n+1} = x^n + dt vbar^p (wrapped), v^{n-1} <- v^n,
// v^n <- v^{n+1,p+1} (with the store's rounding, keyed by the particle's
// stored state and the step).  The kinetic energies are those of the stored
// values.
template <class PS>
__global__ __launch_bounds__(kBlock) void k_finalize(StepParams P, PS st,
                                                    const double* __restrict__ vit,
                                                    const double* __restrict__ vnew, uint64_t step,
                                                    Scratch sc) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double s[2] = {0.0, 0.0};  // K^{n+1}, K^{n+1} - K^n
  if (i < P.np) {
    double x0[3], vo[3], vi[3], vn[3], x1[3], w[3];
    const double mi = species_value(P.ms, st.species(i));
    st.x_of(P.G, P.np, i, x0);
    st.v_of(P.np, i, vo);
    load3(vit, P.np, i, vi);
    load3(vnew, P.np, i, vn);
#pragma unroll
    for (int a = 0; a < 3; ++a)
      x1[a] = wrap_pos(x0[a] + P.dt * 0.5 * (vi[a] + vo[a]), P.G.L[a], P.G.invL[a]);
    const uint64_t key = splitmix64(st.state_key(P.np, i) ^ (step * 0xd1b54a32d192ed03ull));
    st.set_x(P.G, P.np, i, x1);
    st.set_vp(P.np, i, vo);
    st.accept_v(P.np, i, vn, key, w);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      s[0] += 0.5 * mi * w[a] * w[a];
      s[1] += 0.5 * mi * (w[a] - vo[a]) * (w[a] + vo[a]);
    }
  }
  block_partials<2>(s, sc.region(P_K));  // -> S_K, S_DK
}

template <class PS>
__global__ __launch_bounds__(kBlock) void k_kinetic(StepParams P, PS st, Scratch sc) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double s[2] = {0.0, 0.0};
  if (i < P.np) {
    double va[3];
    st.v_of(P.np, i, va);
    const double mi = species_value(P.ms, st.species(i));
#pragma unroll
    for (int a = 0; a < 3; ++a) s[0] += 0.5 * mi * va[a] * va[a];
  }
  block_partials<2>(s, sc.region(P_K));
}

// which = 0: x (wrapped into [0, L)), 1: v^n, 2: v^{n-1}
template <class PS>
__global__ __launch_bounds__(kBlock) void k_import(StepParams P, PS st, int which,
                                                  const double* __restrict__ src) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= P.np) return;
  double w[3];
  load3(src, P.np, i, w);
  if (which == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a) w[a] = wrap_pos(w[a], P.G.L[a], P.G.invL[a]);
    st.set_x(P.G, P.np, i, w);
  } else if (which == 1) {
    st.set_v(P.np, i, w);
  } else {
    st.set_vp(P.np, i, w);
  }
}

template <class PS>
__global__ __launch_bounds__(kBlock) void k_export(StepParams P, PS st, int which,
                                                  double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= P.np) return;
  double w[3];
  if (which == 0)
    st.x_of(P.G, P.np, i, w);
  else if (which == 1)
    st.v_of(P.np, i, w);
  else
    st.vp_of(P.np, i, w);
#pragma unroll
  for (int a = 0; a < 3; ++a) dst[a * P.np + i] = w[a];
}

__global__ __launch_bounds__(kBlock) void k_fixed_current(int64_t n,
                                                         unsigned long long* __restrict__ Jfix,
                                                         double* __restrict__ J, double unit) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  J[i] = unit * (double)(long long)Jfix[i];
  Jfix[i] = 0ull;
}

// rho_g += q S_g(x_i) / dV (eq. source-moments), point shape.  Mixed state:
// S_g as fixed-point quanta into out.Jfix (rho = q / dV / scale x quanta).
template <int R, class PS>
__global__ __launch_bounds__(kBlock) void k_deposit_rho(StepParams P, PS st, CurrentOut out) {
  constexpr int W = R + 1;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= P.np) return;
  double w[3][W], x0[3];
  int f[3];
  st.x_of(P.G, P.np, i, x0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double u = x0[a] * P.G.invH[a];
    const double base = floor(u + Spline<R>::base_off);
    Spline<R>::w(u - base, w[a]);
    f[a] = to_int_clamped(base) + Spline<R>::first_off;
  }
  const double cq = species_value(P.cq, st.species(i));  // q_i / dV; fixed point: q_i / q_0
#pragma unroll
  for (int a = 0; a < W; ++a)
#pragma unroll
    for (int b = 0; b < W; ++b)
#pragma unroll
      for (int cc = 0; cc < W; ++cc) {
        const int64_t g = node_of(P.G, wrapi(f[0] + a, P.G.n[0]), wrapi(f[1] + b, P.G.n[1]),
                                  wrapi(f[2] + cc, P.G.n[2]));
        const double s = w[0][a] * w[1][b] * w[2][cc];
        if constexpr (PS::kMixed)
          atomicAdd(out.Jfix + g, quantize(cq * s, out.fix_scale));
        else
          unsafeAtomicAdd(out.J + g, cq * s);
      }
}

// Orbit integrals of independent particles against SoA fields (kernel-level check).
template <int R, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_orbit_gather_soa(QuadRule rule, Grid G, int64_t n,
                                                            const double* __restrict__ x0s,
                                                            const double* __restrict__ ds,
                                                            SoaFields F,
                                                            const double* __restrict__ Uh,
                                                            double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double x0[3], d[3];
  load3(x0s, n, i, x0);
  load3(ds, n, i, d);
  double gp[3] = {0.0, 0.0, 0.0}, Ub[3] = {0.0, 0.0, 0.0};
  double D[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
  double pou = 0.0;
  int pieces = 0;
  bool ok = true;
  if constexpr (SPLIT) {
    ok = for_each_piece<R>(x0, d, G, [&](double s0, double s1, const double* base) {
      gather_piece<R, true>(G, x0, d, s0, s1, base, F, Uh, gp, D, Ub, pou);
      ++pieces;
    });
  } else {
    for (int q = 0; q < rule.n; ++q) {
      double base[3], sq, wq;
      unsplit_point<R>(G, rule, q, x0, d, base, sq, wq);
      gather_points<R, 1, true>(G, x0, d, base, &sq, &wq, F, Uh, gp, D, Ub, pou);
    }
    pieces = rule.n;
  }
  double x1[3], A0s[3], A1e[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) x1[a] = wrap_pos(x0[a] + d[a], G.L[a], G.invL[a]);
  point_A<R>(G, x0, F, 0, A0s);
  point_A<R>(G, x1, F, 1, A1e);
  double* o = out + 24 * i;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    o[l] = gp[l];
    o[3 + l] = Ub[l];
#pragma unroll
    for (int j = 0; j < 3; ++j) o[6 + 3 * l + j] = D[l][j];
    o[15 + l] = A1e[l];
    o[18 + l] = A0s[l];
  }
  o[21] = pou;
  o[22] = ok ? (double)pieces : -1.0;
  o[23] = 0.0;
}

template <int R, bool SPLIT>
__global__ __launch_bounds__(kBlock) void k_orbit_deposit_soa(QuadRule rule, Grid G, int64_t n,
                                                             const double* __restrict__ x0s,
                                                             const double* __restrict__ ds,
                                                             const double* __restrict__ qv,
                                                             double* __restrict__ J) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double x0[3], d[3], c3[3];
  load3(x0s, n, i, x0);
  load3(ds, n, i, d);
  load3(qv, n, i, c3);
#pragma unroll
  for (int a = 0; a < 3; ++a) c3[a] /= G.dV;
  if constexpr (SPLIT) {
    for_each_piece<R>(x0, d, G, [&](double s0, double s1, const double* base) {
      scatter_piece<R>(G, x0, d, s0, s1, base, c3, J);
    });
  } else {
    constexpr int W = R + 1;
    for (int q = 0; q < rule.n; ++q) {
      double base[3], sq, wq, Iw[W][W][W];
      int f[3];
      unsplit_point<R>(G, rule, q, x0, d, base, sq, wq);
      sbar_points<R, 1>(G, x0, d, base, &sq, &wq, Iw, f);
      for (int a = 0; a < W; ++a)
        for (int b = 0; b < W; ++b)
          for (int c = 0; c < W; ++c) {
            const int64_t g = node_index(G, f[0] + a, f[1] + b, f[2] + c);
#pragma unroll
            for (int l = 0; l < 3; ++l) unsafeAtomicAdd(J + l * G.ncell + g, Iw[a][b][c] * c3[l]);
          }
    }
  }
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int64_t scatter_blocks(int64_t np, int chunk) { return (np + chunk - 1) / chunk; }
int64_t particle_blocks(int64_t np) { return (np + kBlock - 1) / kBlock; }

// ---- launchers ---------------------------------------------------------------

// f(std::integral_constant<int, r>{}) for the spline degree r = 1, 2, 3
template <class F>
void by_degree(int r, F&& f) {
  if (r == 1)
    f(std::integral_constant<int, 1>{});
  else if (r == 2)
    f(std::integral_constant<int, 2>{});
  else
    f(std::integral_constant<int, 3>{});
}

template <class PS>
void launch_extrapolate(hipStream_t s, int64_t np, const PS& st, double* vit, double* vbar) {
  if (np <= 0) return;
  k_extrapolate<<<blocks_for(3 * np), kBlock, 0, s>>>(3 * np, st.v, st.vp, vit, vbar);
}

template <class PS>
void launch_scatter(hipStream_t s, int r, const StepParams& P, const PS& st, const double* vit,
                    const double* vbar, CurrentOut out, Scratch sc, ChunkBoxes bx) {
  if (P.np <= 0) return;
  const bool multi = P.nsp > 1;
  // degree x (split) x species x chunk length (4096 for r <= 2 only; the
  // host validates P.chunk, whose block count the reductions also use)
  auto go = [&](auto R, auto SPLIT) {
    auto launch = [&](auto MULTI, auto CH) {
      const unsigned nblk = (unsigned)scatter_blocks(P.np, CH.value);
      k_scatter<R.value, PS, SPLIT.value, MULTI.value, CH.value>
          <<<nblk, kBlock, 0, s>>>(P, st, vit, vbar, out, sc, bx);
    };
    auto by_multi = [&](auto CH) {
      if (multi)
        launch(std::true_type{}, CH);
      else
        launch(std::false_type{}, CH);
    };
    if (R.value < 3 && P.chunk == 4096)
      by_multi(std::integral_constant<int, 4096>{});
    else
      by_multi(std::integral_constant<int, 2048>{});
  };
  if constexpr (!PS::kMixed) {
    if (!P.split) {
      by_degree(r, [&](auto R) { go(R, std::false_type{}); });
      return;
    }
  }
  by_degree(r, [&](auto R) { go(R, std::true_type{}); });
}

template <class PS>
void launch_gather_push(hipStream_t s, int r, const StepParams& P, const PS& st,
                        const double* vit, double* vnew, double* vbar_out, const double* gbuf,
                        int* work, Scratch sc, AndersonPrev prev, ChunkBoxes bx) {
  if (P.np <= 0) return;
  AosFields F{gbuf};
  const unsigned nb = blocks_for(P.np);
  const unsigned ng = work ? std::min<unsigned>(nb, kGatherListGrid) : nb;
#define ECPIC_GATHER_PAIR(R_, SPLIT_)                                                          \
  k_gather_push<R_, true, PS, SPLIT_><<<nb, kBlock, 0, s>>>(P, st, vit, vnew, vbar_out, F,    \
                                                             work, sc, prev, bx);              \
  k_gather_push<R_, false, PS, SPLIT_><<<ng, kBlock, 0, s>>>(P, st, vit, vnew, vbar_out, F,   \
                                                              work, sc, prev, ChunkBoxes{})
  if constexpr (!PS::kMixed) {
    if (!P.split) {
      by_degree(r, [&](auto R) { ECPIC_GATHER_PAIR(R.value, false); });
      return;
    }
  }
  by_degree(r, [&](auto R) { ECPIC_GATHER_PAIR(R.value, true); });
#undef ECPIC_GATHER_PAIR
}

template <class PS>
void launch_sweep(hipStream_t s, int r, const StepParams& P, const PS& st, const double* vit,
                  const double* gbuf, const double* Uhalf, Scratch sc) {
  if (P.np <= 0) return;
  AosFields F{gbuf};
  if constexpr (!PS::kMixed) {
    if (!P.split) {
      by_degree(r, [&](auto R) {
        k_sweep<R.value, PS, false><<<blocks_for(P.np), kBlock, 0, s>>>(P, st, vit, F, Uhalf, sc);
      });
      return;
    }
  }
  by_degree(r, [&](auto R) {
    k_sweep<R.value, PS, true><<<blocks_for(P.np), kBlock, 0, s>>>(P, st, vit, F, Uhalf, sc);
  });
}

template <class PS>
void launch_finalize(hipStream_t s, const StepParams& P, const PS& st, const double* vit,
                     const double* vnew, uint64_t step, Scratch sc) {
  if (P.np <= 0) return;
  k_finalize<PS><<<blocks_for(P.np), kBlock, 0, s>>>(P, st, vit, vnew, step, sc);
}

template <class PS>
void launch_kinetic(hipStream_t s, const StepParams& P, const PS& st, Scratch sc) {
  if (P.np <= 0) return;
  k_kinetic<PS><<<blocks_for(P.np), kBlock, 0, s>>>(P, st, sc);
}

template <class PS>
void launch_deposit_rho(hipStream_t s, int r, const StepParams& P, const PS& st, CurrentOut out) {
  if (P.np <= 0) return;
  by_degree(r, [&](auto R) {
    k_deposit_rho<R.value, PS><<<blocks_for(P.np), kBlock, 0, s>>>(P, st, out);
  });
}

template <class PS>
void launch_import(hipStream_t s, const StepParams& P, const PS& st, int which, const double* src) {
  if (P.np <= 0) return;
  k_import<PS><<<blocks_for(P.np), kBlock, 0, s>>>(P, st, which, src);
}

template <class PS>
void launch_export(hipStream_t s, const StepParams& P, const PS& st, int which, double* dst) {
  if (P.np <= 0) return;
  k_export<PS><<<blocks_for(P.np), kBlock, 0, s>>>(P, st, which, dst);
}

void launch_fixed_current(hipStream_t s, int64_t n, unsigned long long* Jfix, double* J,
                          double unit) {
  if (n <= 0) return;
  k_fixed_current<<<blocks_for(n), kBlock, 0, s>>>(n, Jfix, J, unit);
}

#define ECPIC_INSTANTIATE_STORE(PS)                                                              \
  template void launch_extrapolate<PS>(hipStream_t, int64_t, const PS&, double*, double*);                \
  template void launch_scatter<PS>(hipStream_t, int, const StepParams&, const PS&, const double*, \
                                   const double*, CurrentOut, Scratch, ChunkBoxes);              \
  template void launch_gather_push<PS>(hipStream_t, int, const StepParams&, const PS&,           \
                                       const double*, double*, double*, const double*, int*,     \
                                       Scratch, AndersonPrev, ChunkBoxes);                       \
  template void launch_sweep<PS>(hipStream_t, int, const StepParams&, const PS&, const double*,  \
                                 const double*, const double*, Scratch);                         \
  template void launch_finalize<PS>(hipStream_t, const StepParams&, const PS&, const double*,     \
                                    const double*, uint64_t, Scratch);                           \
  template void launch_kinetic<PS>(hipStream_t, const StepParams&, const PS&, Scratch);          \
  template void launch_deposit_rho<PS>(hipStream_t, int, const StepParams&, const PS&,          \
                                       CurrentOut);                                              \
  template void launch_import<PS>(hipStream_t, const StepParams&, const PS&, int, const double*); \
  template void launch_export<PS>(hipStream_t, const StepParams&, const PS&, int, double*);

ECPIC_INSTANTIATE_STORE(Fp64Store)
ECPIC_INSTANTIATE_STORE(MixedStore)
#undef ECPIC_INSTANTIATE_STORE

void launch_orbit_gather_soa(hipStream_t s, int r, const QuadRule* rule, const Grid& G,
                             int64_t n, const double* x0, const double* d, const double* gphi,
                             const double* U, const double* A0, const double* A1, double* out) {
  if (n <= 0) return;
  SoaFields F{gphi, A0, A1, G.ncell};
  const QuadRule ru = rule ? *rule : QuadRule{};
  const unsigned nb = blocks_for(n);
  by_degree(r, [&](auto R) {
    if (rule)
      k_orbit_gather_soa<R.value, false><<<nb, kBlock, 0, s>>>(ru, G, n, x0, d, F, U, out);
    else
      k_orbit_gather_soa<R.value, true><<<nb, kBlock, 0, s>>>(ru, G, n, x0, d, F, U, out);
  });
}

void launch_orbit_deposit_soa(hipStream_t s, int r, const QuadRule* rule, const Grid& G,
                              int64_t n, const double* x0, const double* d, const double* qv,
                              double* J) {
  if (n <= 0) return;
  const QuadRule ru = rule ? *rule : QuadRule{};
  const unsigned nb = blocks_for(n);
  by_degree(r, [&](auto R) {
    if (rule)
      k_orbit_deposit_soa<R.value, false><<<nb, kBlock, 0, s>>>(ru, G, n, x0, d, qv, J);
    else
      k_orbit_deposit_soa<R.value, true><<<nb, kBlock, 0, s>>>(ru, G, n, x0, d, qv, J);
  });
}

}  // namespace ecpic
