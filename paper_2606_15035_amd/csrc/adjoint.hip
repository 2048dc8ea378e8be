// Particle side of the adjoint of a converged step (degree 2, split orbits).
//
// The converged step solves w = G(w; x, v, F) with vbar = (w + v)/2,
// d = dt vbar and (P^n rebuilt from eq. discrete-canonical-relation)
//   G = v + (q/m) [A0_h(x) - A1_h(x + d)] + (q dt/m) [-gphibar + (D A)^T vbar],
//   gphibar = sum_g gphi_g Sbar_g,
//   ((D A)^T vbar)_j = sum_g int b_g(s) d_j S_g(x(s)) ds,  b_g(s) = vbar.((1-s) A0_g + s A1_g),
// (eqs. orbit-push, split-Sbar, split-DA), and the current
//   J_g = (q/dV) sum_i vbar_i Sbar_ig   (eq. orbit-current).
// For a particle with push adjoint eta = (q/m) xi and current adjoint
// mu = (q/dV) lambda_J, the kernels below add the derivatives with respect
// to x, d and vbar, and scatter the push's mesh adjoints of gphi, A0 and A1.
// Inside each split piece the integrands are polynomials of degree <= 6 in s
// (4-point Gauss-Legendre is exact); the piece ends move with x and d, but
// the integrands b_g d_j S_g and S_g are continuous across knots for degree
// 2, so no end-point terms arise.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.hpp"
#include "orbit.hpp"
#include "reduce.hpp"

namespace ecpic {

namespace {

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// weights and first derivatives (physical units) of the three degree-2
// stencil nodes along one axis
struct Axis2 {
  double w[3], dw[3];
  __device__ __forceinline__ void at(double t, double invH) {
    Spline<2>::wd(t, w, dw);
#pragma unroll
    for (int o = 0; o < 3; ++o) dw[o] *= invH;
  }
};

// Where the push's mesh adjoints go (nine values per node: component l of
// grad phi, A^n and A^{n+1} as 0 + l, 3 + l and 6 + l).  add() takes the node
// in the particle's unwrapped frame (ix, iy, iz) and its flat index g.
struct GlobalAdjSink {
  const AdjParticleArgs* P;
  __device__ __forceinline__ double* target(int comp) const {
    double* base = comp < 3 ? P->lgphi : (comp < 6 ? P->lA0 : P->lA1);
    return base + (int64_t)(comp % 3) * P->G.ncell;
  }
  __device__ __forceinline__ void add(int comp, int, int, int, int64_t g, double v) const {
    unsafeAtomicAdd(target(comp) + g, v);
  }
};

// The block's LDS tile over its chunk's node box (nine doubles per node);
// o[] takes the particle's frame to the tile's.  A node outside the box
// (not expected: the box has a node of margin per side) goes to global
// memory.  The tile pointer carries the LDS address space, so the additions
// are LDS atomics (through a plain pointer they compiled to flat atomics,
// the slower path that serves either memory).
typedef __attribute__((address_space(3))) double lds_double;
struct TileAdjSink {
  GlobalAdjSink glob;
  lds_double* tile;
  int o[3], dim[3];
  bool use;
  __device__ __forceinline__ void add(int comp, int ix, int iy, int iz, int64_t g,
                                      double v) const {
    const int tx = ix + o[0], ty = iy + o[1], tz = iz + o[2];
    if (use && tx >= 0 && ty >= 0 && tz >= 0 && tx < dim[0] && ty < dim[1] && tz < dim[2])
      __hip_atomic_fetch_add(&tile[9 * ((tx * dim[1] + ty) * dim[2] + tz) + comp], v,
                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
      glob.add(comp, ix, iy, iz, g, v);
  }
};

// The push terms of particle i (eta = (q/m) xi) in tensor-product form.
// With eta'_j = eta_j / H_j and derivatives per unit of cell coordinate
// (S_g = X_a Y_b Z_c; the degree-2 second derivatives are 1, -2, 1):
//  - per node, three point sums feed the mesh adjoints and the vbar adjoint:
//      Sbar = sum_q w S,  T0 = sum_q w (1 - s) eta'.grad S,  T1 = sum_q w s eta'.grad S
//    (dL/dgphi_l = -dt eta_l Sbar, dL/dA0_l = dt vbar_l T0, dL/dA1_l = dt vbar_l T1;
//    lvbar += dt (A0_g T0 + A1_g T1));
//  - the x and d adjoints, dt / H_k sum_g sum_q w_q (1, s) [b_g(s_q) (eta'.grad)(d_k S_g)
//    - (eta.gphi_g) d_k S_g] with b_g(s) = (1 - s) vbar.A0_g + s vbar.A1_g, need
//    per stencil row only the z-column sums of b0 = vbar.A0, b1 = vbar.A1 and
//    eg = eta.gphi against Z and Z' at each point (and against Z'', the same at
//    every point); the row's x and y factors then give the Hessian terms.
// The same sums as a node-by-node evaluation, with about a quarter of its
// arithmetic.
template <class Sink>
__device__ __forceinline__ void push_adjoint(const AdjParticleArgs& P, int64_t i,
                                             const Sink& sink) {
  const Grid& G = P.G;
  const int64_t np = P.np, nc = G.ncell;
  double x0[3], vb[3], d[3], eta[3], ep[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    x0[a] = P.x[a * np + i];
    vb[a] = P.vb[a * np + i];
    d[a] = P.dt * vb[a];
    eta[a] = P.qm * P.xi[a * np + i];
    ep[a] = eta[a] * G.invH[a];
  }
  // piece terms of lx and ld per unit of cell coordinate (times dt / H_k below)
  double lx[3] = {0.0, 0.0, 0.0}, ld[3] = {0.0, 0.0, 0.0}, lvb[3] = {0.0, 0.0, 0.0};
  const bool ok = for_each_piece<2>(x0, d, G, [&](double s0, double s1, const double* base) {
    const double h = s1 - s0;
    double sq[4], wq[4], tx[4], ty[4], Z[4][3], dZ[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sq[q] = s0 + 0.5 * h * (1.0 + Gauss<4>::x(q));
      wq[q] = 0.5 * h * Gauss<4>::w(q);
      tx[q] = (x0[0] + sq[q] * d[0]) * G.invH[0] - base[0];
      ty[q] = (x0[1] + sq[q] * d[1]) * G.invH[1] - base[1];
      Spline<2>::wd((x0[2] + sq[q] * d[2]) * G.invH[2] - base[2], Z[q], dZ[q]);
    }
    const int fx = to_int_clamped(base[0]) + Spline<2>::first_off;
    const int fy = to_int_clamped(base[1]) + Spline<2>::first_off;
    const int fz = to_int_clamped(base[2]) + Spline<2>::first_off;
#pragma unroll 1
    for (int a = 0; a < 3; ++a) {
      const double ddX = a == 1 ? -2.0 : 1.0;
      double Xq[4], dXq[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) Spline<2>::wk(a, tx[q], Xq[q], dXq[q]);
#pragma unroll 1
      for (int b = 0; b < 3; ++b) {
        const double ddY = b == 1 ? -2.0 : 1.0;
        double Yq[4], dYq[4], xy[4], dxy[4], xdy[4], pe[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          Spline<2>::wk(b, ty[q], Yq[q], dYq[q]);
          xy[q] = Xq[q] * Yq[q];
          dxy[q] = dXq[q] * Yq[q];
          xdy[q] = Xq[q] * dYq[q];
          pe[q] = ep[0] * dxy[q] + ep[1] * xdy[q];  // (eta'_x d_x + eta'_y d_y)(X Y)
        }
        double C0[4], C0d[4], C1[4], C1d[4], Eg[4], Egd[4], C0dd = 0.0, C1dd = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double ddZ = c == 1 ? -2.0 : 1.0;
          const int ix = fx + a, iy = fy + b, iz = fz + c;
          const int64_t g = node_index(G, ix, iy, iz);
          double A0g[3], A1g[3];
          double b0 = 0.0, b1 = 0.0, eg = 0.0;
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            A0g[l] = P.A0[l * nc + g];
            A1g[l] = P.A1[l * nc + g];
            b0 += vb[l] * A0g[l];
            b1 += vb[l] * A1g[l];
            eg += eta[l] * P.gphi[l * nc + g];
          }
          double Sbar = 0.0, T0 = 0.0, T1 = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double z = Z[q][c], dz = dZ[q][c];
            C0[q] = c == 0 ? b0 * z : C0[q] + b0 * z;
            C0d[q] = c == 0 ? b0 * dz : C0d[q] + b0 * dz;
            C1[q] = c == 0 ? b1 * z : C1[q] + b1 * z;
            C1d[q] = c == 0 ? b1 * dz : C1d[q] + b1 * dz;
            Eg[q] = c == 0 ? eg * z : Eg[q] + eg * z;
            Egd[q] = c == 0 ? eg * dz : Egd[q] + eg * dz;
            const double edS = pe[q] * z + ep[2] * xy[q] * dz;  // eta'.grad S
            Sbar += wq[q] * xy[q] * z;
            T0 += wq[q] * (1.0 - sq[q]) * edS;
            T1 += wq[q] * sq[q] * edS;
          }
          C0dd += b0 * ddZ;
          C1dd += b1 * ddZ;
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            lvb[l] += P.dt * (A0g[l] * T0 + A1g[l] * T1);
            sink.add(l, ix, iy, iz, g, -P.dt * eta[l] * Sbar);
            sink.add(3 + l, ix, iy, iz, g, P.dt * vb[l] * T0);
            sink.add(6 + l, ix, iy, iz, g, P.dt * vb[l] * T1);
          }
        }
        // the row's share of sum_g b (eta'.grad)(d_k S_g) (with b0 and b1) and
        // of sum_g eg d_k S_g, per point
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double dxdy = dXq[q] * dYq[q];
          // (eta'.grad)(d_k S) summed over the row against b0 and b1
          const double hx = ep[0] * ddX * Yq[q] + ep[1] * dxdy;     // with Z
          const double hy = ep[0] * dxdy + ep[1] * Xq[q] * ddY;     // with Z
          const double u0x = hx * C0[q] + ep[2] * dxy[q] * C0d[q];
          const double u0y = hy * C0[q] + ep[2] * xdy[q] * C0d[q];
          const double u0z = pe[q] * C0d[q] + ep[2] * xy[q] * C0dd;
          const double u1x = hx * C1[q] + ep[2] * dxy[q] * C1d[q];
          const double u1y = hy * C1[q] + ep[2] * xdy[q] * C1d[q];
          const double u1z = pe[q] * C1d[q] + ep[2] * xy[q] * C1dd;
          // d_k S summed over the row against eg
          const double vx = dxy[q] * Eg[q], vy = xdy[q] * Eg[q], vz = xy[q] * Egd[q];
          const double q0 = wq[q] * (1.0 - sq[q]), q1 = wq[q] * sq[q];
          lx[0] += q0 * u0x + q1 * u1x - wq[q] * vx;
          lx[1] += q0 * u0y + q1 * u1y - wq[q] * vy;
          lx[2] += q0 * u0z + q1 * u1z - wq[q] * vz;
          ld[0] += sq[q] * (q0 * u0x + q1 * u1x - wq[q] * vx);
          ld[1] += sq[q] * (q0 * u0y + q1 * u1y - wq[q] * vy);
          ld[2] += sq[q] * (q0 * u0z + q1 * u1z - wq[q] * vz);
        }
      }
    }
  });
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    lx[k] *= P.dt * G.invH[k];
    ld[k] *= P.dt * G.invH[k];
  }
  // + A0_h(x0) - A1_h(x0 + d), end point wrapped
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const double sgn = e == 0 ? 1.0 : -1.0;
    const double* F = e == 0 ? P.A0 : P.A1;
    double base[3];
    int first[3], sh[3];
    Axis2 ax[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double xp = e == 0 ? x0[a] : wrap_pos(x0[a] + d[a], G.L[a], G.invL[a]);
      const double u = xp * G.invH[a];
      base[a] = floor(u + Spline<2>::base_off);
      first[a] = to_int_clamped(base[a]) + Spline<2>::first_off;
      ax[a].at(u - base[a], G.invH[a]);
      // periods between the wrapped end point and the unwrapped orbit end
      sh[a] = e == 0 ? 0 : (int)rint((x0[a] + d[a] - xp) * G.invL[a]) * G.n[a];
    }
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c) {
          const int64_t g = node_index(G, first[0] + a, first[1] + b, first[2] + c);
          const double S = ax[0].w[a] * ax[1].w[b] * ax[2].w[c];
          const double dS[3] = {ax[0].dw[a] * ax[1].w[b] * ax[2].w[c],
                                ax[0].w[a] * ax[1].dw[b] * ax[2].w[c],
                                ax[0].w[a] * ax[1].w[b] * ax[2].dw[c]};
          double eF = 0.0;
#pragma unroll
          for (int l = 0; l < 3; ++l) {
            eF += eta[l] * F[l * nc + g];
            sink.add((e == 0 ? 3 : 6) + l, first[0] + a + sh[0], first[1] + b + sh[1],
                     first[2] + c + sh[2], g, sgn * eta[l] * S);
          }
#pragma unroll
          for (int kk = 0; kk < 3; ++kk) {
            lx[kk] += sgn * eF * dS[kk];
            if (e == 1) ld[kk] += sgn * eF * dS[kk];
          }
        }
  }
  if (!ok) P.bad[0] = 1.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    P.lx[a * np + i] += lx[a];
    P.ld[a * np + i] += ld[a];
    P.lvb[a * np + i] += lvb[a];
  }
}

// The current terms alone (eta = 0: the current's adjoint mu seen by one
// particle), in the tensor-product form of the forward gather: per stencil
// row (a, b) the x and y factors of every quadrature point are formed once,
// and per node only the seven point sums
//   I = sum_q w_q X Y Z,  I_k = sum_q w_q d_k(X Y Z),  I_k^s = sum_q w_q s_q d_k(X Y Z)
// (derivatives per unit of cell coordinate, scaled by 1/H once per particle)
// meet the node's mu:  lvbar += mu_g I,  lx += (vbar . mu_g) I_k,
// ld += (vbar . mu_g) I_k^s.  The same sums as the node-by-node form above,
// with about a third of its arithmetic.
__global__ __launch_bounds__(kBlock) void k_current_adjoint(AdjParticleArgs P) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= P.np) return;
  const Grid& G = P.G;
  const int64_t np = P.np, nc = G.ncell;
  double x0[3], vb[3], d[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    x0[a] = P.x[a * np + i];
    vb[a] = P.vb[a * np + i];
    d[a] = P.dt * vb[a];
  }
  double lx[3] = {0.0, 0.0, 0.0}, ld[3] = {0.0, 0.0, 0.0}, lvb[3] = {0.0, 0.0, 0.0};
  const bool ok = for_each_piece<2>(x0, d, G, [&](double s0, double s1, const double* base) {
    const double h = s1 - s0;
    double sq[4], wq[4], tx[4], ty[4], Z[4][3], dZ[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      sq[q] = s0 + 0.5 * h * (1.0 + Gauss<4>::x(q));
      wq[q] = 0.5 * h * Gauss<4>::w(q);
      tx[q] = (x0[0] + sq[q] * d[0]) * G.invH[0] - base[0];
      ty[q] = (x0[1] + sq[q] * d[1]) * G.invH[1] - base[1];
      Spline<2>::wd((x0[2] + sq[q] * d[2]) * G.invH[2] - base[2], Z[q], dZ[q]);
    }
    const int fx = to_int_clamped(base[0]) + Spline<2>::first_off;
    const int fy = to_int_clamped(base[1]) + Spline<2>::first_off;
    const int fz = to_int_clamped(base[2]) + Spline<2>::first_off;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double Xw[4], dXw[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double Xq, dXq;
        Spline<2>::wk(a, tx[q], Xq, dXq);
        Xw[q] = wq[q] * Xq;
        dXw[q] = wq[q] * dXq;
      }
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        double xyw[4], dxyw[4], xdyw[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double Yq, dYq;
          Spline<2>::wk(b, ty[q], Yq, dYq);
          xyw[q] = Xw[q] * Yq;
          dxyw[q] = dXw[q] * Yq;
          xdyw[q] = Xw[q] * dYq;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int64_t g = node_index(G, fx + a, fy + b, fz + c);
          const double m0 = P.mu[g], m1 = P.mu[nc + g], m2 = P.mu[2 * nc + g];
          const double vm = vb[0] * m0 + vb[1] * m1 + vb[2] * m2;
          double I = 0.0, Ix = 0.0, Iy = 0.0, Iz = 0.0, Ixs = 0.0, Iys = 0.0, Izs = 0.0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const double zx = dxyw[q] * Z[q][c], zy = xdyw[q] * Z[q][c], zz = xyw[q] * dZ[q][c];
            I += xyw[q] * Z[q][c];
            Ix += zx;
            Iy += zy;
            Iz += zz;
            Ixs += sq[q] * zx;
            Iys += sq[q] * zy;
            Izs += sq[q] * zz;
          }
          lvb[0] += m0 * I;
          lvb[1] += m1 * I;
          lvb[2] += m2 * I;
          lx[0] += vm * Ix;
          lx[1] += vm * Iy;
          lx[2] += vm * Iz;
          ld[0] += vm * Ixs;
          ld[1] += vm * Iys;
          ld[2] += vm * Izs;
        }
      }
    }
  });
  if (!ok) P.bad[0] = 1.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    P.lx[a * np + i] += lx[a] * G.invH[a];
    P.ld[a * np + i] += ld[a] * G.invH[a];
    P.lvb[a * np + i] += lvb[a];
  }
}

// The push terms over cell-sorted particles, one block per chunk of kAdjChunk
// particles whose wavefronts' lanes sit kAdjChunk / 64 particles apart (one
// cell apart at 64 particles per cell), as in the current scatter: the block
// finds the node box of its chunk's orbits and end points (one node of
// margin per side), sums the nine mesh adjoints of its particles in an LDS
// tile over that box, and adds the tile to global memory once.  A chunk
// whose box exceeds the tile adds straight to global memory.  The kernel
// runs at one wavefront per SIMD (its registers), so one block per CU loses
// nothing to the 144 KB tile.
constexpr int kAdjChunk = 4096;
constexpr int kAdjTileNodes = 2048;

__device__ __forceinline__ int64_t adj_chunk_particle(int64_t base, int k) {
  return base + (int64_t)(threadIdx.x % kWave) * (kAdjChunk / kWave) + threadIdx.x / kWave +
         (int64_t)(kBlock / kWave) * k;
}

__global__ __launch_bounds__(kBlock) void k_push_adjoint_tiled(AdjParticleArgs P) {
  constexpr int kPerThread = kAdjChunk / kBlock;
  __shared__ double tile[9 * kAdjTileNodes];
  __shared__ int s_ref[3];
  const Grid& G = P.G;
  const int64_t base = (int64_t)blockIdx.x * kAdjChunk;
  if (threadIdx.x == 0)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      s_ref[a] = to_int_clamped(floor(P.x[a * P.np + base] * G.invH[a] + Spline<2>::base_off));
  __syncthreads();
  // node box of the chunk: the orbits from x0 to x0 + d (unwrapped), which
  // also hold both end points' stencils
  int rmin[3] = {0x3fffffff, 0x3fffffff, 0x3fffffff};
  int rmax[3] = {-0x3fffffff, -0x3fffffff, -0x3fffffff};
  for (int k = 0; k < kPerThread; ++k) {
    const int64_t i = adj_chunk_particle(base, k);
    if (i >= P.np) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double x0 = P.x[a * P.np + i], d = P.dt * P.vb[a * P.np + i];
      const double u0 = x0 * G.invH[a], u1 = (x0 + d) * G.invH[a];
      const int lo = to_int_clamped(floor(fmin(u0, u1) + Spline<2>::base_off)) +
                     Spline<2>::first_off - 1;
      const int hi = to_int_clamped(floor(fmax(u0, u1) + Spline<2>::base_off)) +
                     Spline<2>::first_off + 3;
      const int rel = min_image(lo - s_ref[a], G.n[a]);
      rmin[a] = min(rmin[a], rel);
      rmax[a] = max(rmax[a], rel + (hi - lo));
    }
  }
  int tlo[3], dim[3];
  {
    int mv[6] = {rmin[0], rmin[1], rmin[2], -rmax[0], -rmax[1], -rmax[2]};
    block_min_ints<6>(mv);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      tlo[a] = mv[a];
      dim[a] = -mv[3 + a] - tlo[a] + 1;
    }
  }
  // block-uniform; each extent is bounded first so that the product cannot overflow
  const bool use_tile = dim[0] > 0 && dim[0] <= kAdjTileNodes && dim[1] <= kAdjTileNodes &&
                        dim[2] <= kAdjTileNodes &&
                        (int64_t)dim[0] * dim[1] * dim[2] <= kAdjTileNodes;
  const int nt = use_tile ? dim[0] * dim[1] * dim[2] : 0;
  for (int t = threadIdx.x; t < 9 * nt; t += kBlock) tile[t] = 0.0;
  __syncthreads();
  for (int k = 0; k < kPerThread; ++k) {
    const int64_t i = adj_chunk_particle(base, k);
    if (i >= P.np) break;
    TileAdjSink sink{GlobalAdjSink{&P}, (lds_double*)tile, {0, 0, 0}, {dim[0], dim[1], dim[2]},
                     use_tile};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double x0 = P.x[a * P.np + i], d = P.dt * P.vb[a * P.np + i];
      const double u0 = x0 * G.invH[a], u1 = (x0 + d) * G.invH[a];
      const int lo = to_int_clamped(floor(fmin(u0, u1) + Spline<2>::base_off)) +
                     Spline<2>::first_off - 1;
      const int raw = lo - s_ref[a];
      // particle frame -> chunk frame -> tile
      sink.o[a] = min_image(raw, G.n[a]) - raw - s_ref[a] - tlo[a];
    }
    push_adjoint(P, i, sink);
  }
  __syncthreads();
  if (!use_tile) return;
  const GlobalAdjSink glob{&P};
  for (int t = threadIdx.x; t < nt; t += kBlock) {
    const int cz = t % dim[2], cy = (t / dim[2]) % dim[1], cx = t / (dim[1] * dim[2]);
    const int64_t g = node_index(G, s_ref[0] + tlo[0] + cx, s_ref[1] + tlo[1] + cy,
                                 s_ref[2] + tlo[2] + cz);
#pragma unroll
    for (int comp = 0; comp < 9; ++comp) {
      const double val = tile[9 * t + comp];
      if (val != 0.0) unsafeAtomicAdd(glob.target(comp) + g, val);
    }
  }
}

// vbar = (w + v)/2
__global__ __launch_bounds__(kBlock) void k_vbar(int64_t n3, const double* __restrict__ w,
                                                const double* __restrict__ v,
                                                double* __restrict__ vb) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n3) vb[i] = 0.5 * (w[i] + v[i]);
}

// b = lv1 + (lvb + dt (ld + lx1)) / 2, lxacc = lx1 + lx
__global__ __launch_bounds__(kBlock) void k_adjoint_rhs(int64_t n3, double dt,
                                                       const double* __restrict__ lx1,
                                                       const double* __restrict__ lv1,
                                                       const double* __restrict__ lx,
                                                       const double* __restrict__ ld,
                                                       const double* __restrict__ lvb,
                                                       double* __restrict__ b,
                                                       double* __restrict__ lxacc) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n3) return;
  const double x1 = lx1 ? lx1[i] : 0.0;
  b[i] = (lv1 ? lv1[i] : 0.0) + 0.5 * (lvb[i] + dt * (ld[i] + x1));
  lxacc[i] = x1 + lx[i];
}

// xn = b + (lvb + dt ld)/2; max|xn - xi| and max|xn| into red[0], red[1]
__global__ __launch_bounds__(kBlock) void k_adjoint_update(int64_t n3, double dt,
                                                          const double* __restrict__ b,
                                                          const double* __restrict__ lvb,
                                                          const double* __restrict__ ld,
                                                          const double* __restrict__ xi,
                                                          double* __restrict__ xn,
                                                          double* __restrict__ red) {
  double dm = 0.0, xm = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n3;
       i += (int64_t)gridDim.x * kBlock) {
    const double x = b[i] + 0.5 * (lvb[i] + dt * ld[i]);
    xn[i] = x;
    dm = fmax(dm, fabs(x - xi[i]));
    xm = fmax(xm, fabs(x));
    if (!isfinite(x)) dm = INFINITY;
  }
  block_max_to(dm, red);
  block_max_to(xm, red + 1);
}

// lx0 = lxacc + lx, lv0 = 2 xi - lv1
__global__ __launch_bounds__(kBlock) void k_adjoint_out(int64_t n3, const double* __restrict__ lxacc,
                                                       const double* __restrict__ lx,
                                                       const double* __restrict__ xi,
                                                       const double* __restrict__ lv1,
                                                       double* __restrict__ lx0,
                                                       double* __restrict__ lv0) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n3) return;
  lx0[i] = lxacc[i] + lx[i];
  lv0[i] = 2.0 * xi[i] - (lv1 ? lv1[i] : 0.0);
}

}  // namespace

void launch_particle_adjoint(hipStream_t s, const AdjParticleArgs& P, bool eta, bool mu) {
  if (P.np <= 0) return;
  if (eta)
    k_push_adjoint_tiled<<<(unsigned)((P.np + kAdjChunk - 1) / kAdjChunk), kBlock, 0, s>>>(P);
  if (mu) k_current_adjoint<<<blocks_for(P.np), kBlock, 0, s>>>(P);
}

void launch_vbar(hipStream_t s, int64_t n3, const double* w, const double* v, double* vb) {
  if (n3 > 0) k_vbar<<<blocks_for(n3), kBlock, 0, s>>>(n3, w, v, vb);
}

void launch_adjoint_rhs(hipStream_t s, int64_t n3, double dt, const double* lx1, const double* lv1,
                        const double* lx, const double* ld, const double* lvb, double* b,
                        double* lxacc) {
  if (n3 > 0) k_adjoint_rhs<<<blocks_for(n3), kBlock, 0, s>>>(n3, dt, lx1, lv1, lx, ld, lvb, b, lxacc);
}

void launch_adjoint_update(hipStream_t s, int64_t n3, double dt, const double* b,
                           const double* lvb, const double* ld, const double* xi, double* xn,
                           double* red) {
  // a grid of at most 1024 blocks: every block adds its two maxima to the
  // same two words, so fewer blocks mean fewer contended atomics
  if (n3 > 0)
    k_adjoint_update<<<std::min(blocks_for(n3), 1024u), kBlock, 0, s>>>(n3, dt, b, lvb, ld, xi, xn,
                                                                        red);
}

void launch_adjoint_out(hipStream_t s, int64_t n3, const double* lxacc, const double* lx,
                        const double* xi, const double* lv1, double* lx0, double* lv0) {
  if (n3 > 0) k_adjoint_out<<<blocks_for(n3), kBlock, 0, s>>>(n3, lxacc, lx, xi, lv1, lx0, lv0);
}

}  // namespace ecpic
