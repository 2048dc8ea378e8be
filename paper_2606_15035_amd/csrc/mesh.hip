// Mesh-side kernels for gfx950: batched radix-2 FFT passes in LDS, the
// per-mode continuity + Crank-Nicolson update, the initial Poisson solve and
// the Parseval / constraint reductions.
//
// Spectral fields are full complex spectra data[b*ncell + g] with the node /
// mode index g = (ix*Ny + iy)*Nz + iz.  The Fourier symbol of d/dx_a at mode
// index m is i k~ with k~ = 2 pi m_s / L_a, m_s the signed index, and
// k~ = 0 on the Nyquist index; Delta_h -> -|k~|^2 (Sec. 3.3).  Forward
// transforms are unnormalised; the 1/ncell of the inverse is folded into the
// kernel that prepares its input.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.hpp"
#include "reduce.hpp"

namespace ecpic {

namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// i * k * a
__device__ __forceinline__ double2 ik(double k, double2 a) { return make_double2(-k * a.y, k * a.x); }

struct FftPass {
  double2* data;
  const double2* tw;  // exp(-2 pi i t / N), t < N/2
  int64_t ncell;
  int64_t stride;     // distance between consecutive elements of a pencil
  int64_t npb;        // pencils per batch field = ncell / N
  int64_t npencils;   // nb * npb
  int N, logN;
  double sgn;         // -1 forward, +1 inverse (sign of the exponent)
  RealIO io;          // real input (forward first pass) or output (inverse last pass)
  const double* prev; // optional: max |in - prev| -> S_DJMAX (a spread slot)
  double* clear;      // optional: real buffer (same layout as prev) zeroed by the pass
  Scratch sc;
};

// MODE 0: complex in place; 1: real input -> complex; 2: complex -> real output.
// Each block transforms 256 / (N/2) pencils held in LDS; one thread per
// butterfly; input in bit-reversed order, decimation in time.
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_fft(FftPass A) {
  __shared__ double2 buf[2 * kBlock];
  const int N = A.N, half = N >> 1, P = kBlock / half;
  const int t = threadIdx.x;
  int pl, j;
  if (A.stride == 1) {
    pl = t / half;
    j = t % half;
  } else {
    pl = t % P;
    j = t / P;
  }
  const int64_t pencil = (int64_t)blockIdx.x * P + pl;
  const bool active = pencil < A.npencils;
  int64_t b = 0, off = 0;
  if (active) {
    b = pencil / A.npb;
    const int64_t pin = pencil % A.npb;
    const int64_t outer = pin / A.stride, inner = pin % A.stride;
    off = outer * N * A.stride + inner;
  }
  double2* lds = buf + pl * N;
  double dmax = 0.0;
  if (active) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = j + h * half;
      const int64_t g = off + e * A.stride;
      double2 val;
      if constexpr (MODE == 1) {
        const double re = A.io.p[b][g * A.io.stride[b]];
        if (A.prev) dmax = fmax(dmax, fabs(re - A.prev[b * A.ncell + g]));
        if (A.clear) A.clear[b * A.ncell + g] = 0.0;  // after prev was read (same element)
        val = make_double2(re, 0.0);
      } else {
        val = A.data[b * A.ncell + g];
      }
      lds[__brev((unsigned)e) >> (32 - A.logN)] = val;
    }
  }
  __syncthreads();
  for (int hs = 1; hs < N; hs <<= 1) {
    if (active) {
      const int pos = j % hs;
      const int i0 = (j / hs) * 2 * hs + pos, i1 = i0 + hs;
      double2 w = A.tw[pos * (half / hs)];  // exp(-2 pi i pos / (2 hs))
      if (A.sgn > 0.0) w.y = -w.y;           // inverse: conjugate twiddle
      const double2 a = lds[i0];
      const double2 bb = cmul(lds[i1], w);
      lds[i0] = cadd(a, bb);
      lds[i1] = csub(a, bb);
    }
    __syncthreads();
  }
  if (active) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = j + h * half;
      const int64_t g = off + e * A.stride;
      if constexpr (MODE == 2)
        A.io.p[b][g * A.io.stride[b]] = lds[e].x;
      else
        A.data[b * A.ncell + g] = lds[e];
    }
  }
  if constexpr (MODE == 1) {
    if (A.prev) {
      const double r = block_max(dmax);
      if (threadIdx.x == 0) atomic_max_nonneg(A.sc.spread_copy(S_DJMAX), r);
    }
  }
}

__device__ __forceinline__ double ktil(int m, int N, double L) {
  if (2 * m == N) return 0.0;
  const int ms = (2 * m < N) ? m : m - N;
  return 6.283185307179586476925286766559 * (double)ms / L;
}

__device__ __forceinline__ void mode_k(const Grid& G, int64_t g, double* k) {
  const int iz = (int)(g % G.n[2]);
  const int iy = (int)((g / G.n[2]) % G.n[1]);
  const int ix = (int)(g / ((int64_t)G.n[2] * G.n[1]));
  k[0] = ktil(ix, G.n[0], G.L[0]);
  k[1] = ktil(iy, G.n[1], G.L[1]);
  k[2] = ktil(iz, G.n[2], G.L[2]);
}

// field order in a spectral level: phi, psi, Ax, Ay, Az, Ux, Uy, Uz, rho
enum { F_PHI = 0, F_PSI = 1, F_A = 2, F_U = 5, F_RHO = 8 };

__device__ __forceinline__ double2 ld(const double2* p, int f, int64_t nc, int64_t g) {
  return p[f * nc + g];
}

// |E|^2 / (2 sigma1) + |B|^2 / (2 sigma2) of one mode (E = -i k phi - U, B = i k x A)
__device__ __forceinline__ double mode_energy(const double* k, double2 phi, const double2* A,
                                              const double2* U, double h1, double h2) {
  double e = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const double2 E = csub(make_double2(k[l] * phi.y, -k[l] * phi.x), U[l]);
    e += h1 * (E.x * E.x + E.y * E.y);
  }
  const double2 B0 = csub(ik(k[1], A[2]), ik(k[2], A[1]));
  const double2 B1 = csub(ik(k[2], A[0]), ik(k[0], A[2]));
  const double2 B2 = csub(ik(k[0], A[1]), ik(k[1], A[0]));
  e += h2 * (B0.x * B0.x + B0.y * B0.y + B1.x * B1.x + B1.y * B1.y + B2.x * B2.x + B2.y * B2.y);
  return e;
}

// Continuity (eq. cn-continuity) and CN (eq. cn-field-update) for every mode:
//   rho1 = rho0 - dt i k.J,  rho_h = (rho0 + rho1)/2,
//   psi1 = [(1 - a^2 w^2) psi0 - 2 a w^2 phi0 + dt kappa^2 sigma1 rho_h] / (1 + a^2 w^2),
//   phi1 = phi0 + a (psi0 + psi1),  a = dt/2, w^2 = kappa^2 |k|^2,
// and (A_l, U_l) likewise with sigma2 J_l.  The closed form is the exact
// inverse of the 2x2 CN system of each (value, rate) pair.
struct CNArgs {
  FieldParams F;
  const double2* cur;
  const double2* Jh;
  double2* next;
  double2* inv;
  Scratch sc;
};

// One mode: c = the 9 level-n spectra (field order of a level), J = the 3
// current spectra; out = the 9 level-(n+1) spectra, inv = the inverse-transform
// inputs [i k phi^{n+1/2} (3), A^{n+1} (3)] / ncell, sums = JE, W^{n+1} and
// W^{n+1} - W^n of this mode (times dV / ncell, Parseval).
__device__ __forceinline__ void cn_mode(const FieldParams& F, const double* k, const double2* J,
                                        const double2* c, double2* out, double2* inv,
                                        double* sums) {
  const Grid& G = F.G;
  const double dt = F.dt, a = 0.5 * dt, kap2 = F.kappa * F.kappa;
  const double w2 = kap2 * (k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  const double inv_den = 1.0 / (1.0 + a * a * w2);
  const double c_old = 1.0 - a * a * w2, c_x = 2.0 * a * w2;
  double2 A0[3], U0[3], A1[3], U1[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    A0[l] = c[F_A + l];
    U0[l] = c[F_U + l];
  }
  const double2 phi0 = c[F_PHI], psi0 = c[F_PSI], rho0 = c[F_RHO];
  const double2 divJ = cadd(cadd(ik(k[0], J[0]), ik(k[1], J[1])), ik(k[2], J[2]));
  const double2 rho1 = csub(rho0, cscale(divJ, dt));
  const double2 rhoh = cscale(cadd(rho0, rho1), 0.5);
  const double src1 = dt * kap2 * F.sigma1, src2 = dt * kap2 * F.sigma2;
  double2 psi1, phi1;
  psi1.x = (c_old * psi0.x - c_x * phi0.x + src1 * rhoh.x) * inv_den;
  psi1.y = (c_old * psi0.y - c_x * phi0.y + src1 * rhoh.y) * inv_den;
  phi1 = cadd(phi0, cscale(cadd(psi0, psi1), a));
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    U1[l].x = (c_old * U0[l].x - c_x * A0[l].x + src2 * J[l].x) * inv_den;
    U1[l].y = (c_old * U0[l].y - c_x * A0[l].y + src2 * J[l].y) * inv_den;
    A1[l] = cadd(A0[l], cscale(cadd(U0[l], U1[l]), a));
  }
  out[F_PHI] = phi1;
  out[F_PSI] = psi1;
  out[F_RHO] = rho1;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    out[F_A + l] = A1[l];
    out[F_U + l] = U1[l];
  }
  // inverse-transform inputs: grad_h phi^{n+1/2} and A^{n+1}, scaled by 1/ncell
  const double sc = 1.0 / (double)G.ncell;
  const double2 phih = cscale(cadd(phi0, phi1), 0.5);
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    inv[l] = cscale(ik(k[l], phih), sc);
    inv[3 + l] = cscale(A1[l], sc);
  }
  // Parseval: sum_g f_g h_g = (1/ncell) sum_k Re(conj(f^_k) h^_k)
  const double h1 = 0.5 / F.sigma1, h2 = 0.5 / F.sigma2;
  double je = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const double2 Uh = cscale(cadd(U0[l], U1[l]), 0.5);
    const double2 Eh = csub(make_double2(k[l] * phih.y, -k[l] * phih.x), Uh);  // -i k phi - U
    je += J[l].x * Eh.x + J[l].y * Eh.y;
  }
  const double e1 = mode_energy(k, phi1, A1, U1, h1, h2);
  // W^{n+1} - W^n per mode as (f1 - f0).(f1 + f0) to keep the difference accurate
  double de = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const double2 E1 = csub(make_double2(k[l] * phi1.y, -k[l] * phi1.x), U1[l]);
    const double2 E0 = csub(make_double2(k[l] * phi0.y, -k[l] * phi0.x), U0[l]);
    const double2 dE = csub(E1, E0), sE = cadd(E1, E0);
    de += h1 * (dE.x * sE.x + dE.y * sE.y);
  }
  double2 dA[3], sA[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    dA[l] = csub(A1[l], A0[l]);
    sA[l] = cadd(A1[l], A0[l]);
  }
  const double2 dB[3] = {csub(ik(k[1], dA[2]), ik(k[2], dA[1])),
                         csub(ik(k[2], dA[0]), ik(k[0], dA[2])),
                         csub(ik(k[0], dA[1]), ik(k[1], dA[0]))};
  const double2 sB[3] = {csub(ik(k[1], sA[2]), ik(k[2], sA[1])),
                         csub(ik(k[2], sA[0]), ik(k[0], sA[2])),
                         csub(ik(k[0], sA[1]), ik(k[1], sA[0]))};
#pragma unroll
  for (int l = 0; l < 3; ++l) de += h2 * (dB[l].x * sB[l].x + dB[l].y * sB[l].y);
  const double f = G.dV / (double)G.ncell;
  sums[0] = je * f;
  sums[1] = e1 * f;
  sums[2] = de * f;
}

__global__ __launch_bounds__(kBlock) void k_cn(CNArgs C) {
  const Grid& G = C.F.G;
  const int64_t nc = G.ncell;
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double sums[3] = {0.0, 0.0, 0.0};  // JE, W^{n+1}, W^{n+1} - W^n
  if (g < nc) {
    double k[3];
    mode_k(G, g, k);
    double2 J[3], c[9], out[9], inv[6];
#pragma unroll
    for (int l = 0; l < 3; ++l) J[l] = C.Jh[l * nc + g];
#pragma unroll
    for (int f = 0; f < 9; ++f) c[f] = ld(C.cur, f, nc, g);
    cn_mode(C.F, k, J, c, out, inv, sums);
#pragma unroll
    for (int f = 0; f < 9; ++f) C.next[f * nc + g] = out[f];
#pragma unroll
    for (int f = 0; f < 6; ++f) C.inv[f * nc + g] = inv[f];
  }
  block_partials<3>(sums, C.sc.region(P_CN));  // -> S_JE, S_WNEXT, S_DW
}

__global__ __launch_bounds__(kBlock) void k_half_U(Grid G, const double2* cur, const double2* next,
                                                  double2* inv) {
  const int64_t nc = G.ncell;
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= nc) return;
  const double sc = 0.5 / (double)nc;
#pragma unroll
  for (int l = 0; l < 3; ++l)
    inv[l * nc + g] = cscale(cadd(cur[(F_U + l) * nc + g], next[(F_U + l) * nc + g]), sc);
}

// phi^0 from -Delta_h phi = sigma1 rho on modes with k~ != 0; rho and phi zero
// on every mode where k~ = 0 (this removes the mean and the uniform
// background); psi = A = U = 0.
__global__ __launch_bounds__(kBlock) void k_poisson_init(FieldParams F, double2* cur) {
  const Grid& G = F.G;
  const int64_t nc = G.ncell;
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= nc) return;
  double k[3];
  mode_k(G, g, k);
  const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  double2 rho = cur[F_RHO * nc + g];
  double2 phi = make_double2(0.0, 0.0);
  if (k2 == 0.0)
    rho = make_double2(0.0, 0.0);
  else
    phi = cscale(rho, F.sigma1 / k2);
  cur[F_RHO * nc + g] = rho;
  cur[F_PHI * nc + g] = phi;
  cur[F_PSI * nc + g] = make_double2(0.0, 0.0);
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    cur[(F_A + l) * nc + g] = make_double2(0.0, 0.0);
    cur[(F_U + l) * nc + g] = make_double2(0.0, 0.0);
  }
}

// G_h = psi/kappa^2 + i k.A and R_h = i k.E - sigma1 rho (E = -i k phi - U),
// scaled by 1/ncell, and W of the level.
__global__ __launch_bounds__(kBlock) void k_constraints(FieldParams F, const double2* cur,
                                                       double2* inv, Scratch sc) {
  const Grid& G = F.G;
  const int64_t nc = G.ncell;
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double w[1] = {0.0};
  if (g < nc) {
    double k[3];
    mode_k(G, g, k);
    const double2 phi = cur[F_PHI * nc + g], psi = cur[F_PSI * nc + g], rho = cur[F_RHO * nc + g];
    double2 A[3], U[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      A[l] = cur[(F_A + l) * nc + g];
      U[l] = cur[(F_U + l) * nc + g];
    }
    const double kap2 = F.kappa * F.kappa;
    double2 gh = cscale(psi, 1.0 / kap2);
    double2 divE = make_double2(0.0, 0.0);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      gh = cadd(gh, ik(k[l], A[l]));
      const double2 E = csub(make_double2(k[l] * phi.y, -k[l] * phi.x), U[l]);
      divE = cadd(divE, ik(k[l], E));
    }
    const double2 rh = csub(divE, cscale(rho, F.sigma1));
    const double s = 1.0 / (double)nc;
    inv[g] = cscale(gh, s);
    inv[nc + g] = cscale(rh, s);
    w[0] = mode_energy(k, phi, A, U, 0.5 / F.sigma1, 0.5 / F.sigma2) * G.dV / (double)nc;
  }
  block_partials<1>(w, sc.region(P_W));  // -> S_WCUR
}

__global__ __launch_bounds__(kBlock) void k_field_energy(FieldParams F, const double2* cur,
                                                        Scratch sc) {
  const Grid& G = F.G;
  const int64_t nc = G.ncell;
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double w[1] = {0.0};
  if (g < nc) {
    double k[3];
    mode_k(G, g, k);
    double2 A[3], U[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      A[l] = cur[(F_A + l) * nc + g];
      U[l] = cur[(F_U + l) * nc + g];
    }
    w[0] = mode_energy(k, cur[F_PHI * nc + g], A, U, 0.5 / F.sigma1, 0.5 / F.sigma2) * G.dV /
           (double)nc;
  }
  block_partials<1>(w, sc.region(P_W));  // -> S_WCUR
}

__global__ __launch_bounds__(kBlock) void k_norms(int64_t nc, const double* gf, const double* rf,
                                                 Scratch sc) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  double gv = 0.0, rv = 0.0;
  if (g < nc) {
    gv = gf[g];
    rv = rf[g];
  }
  block_max_to(fabs(gv), sc.red + S_GMAX);
  block_max_to(fabs(rv), sc.red + S_RMAX);
  double s[2] = {gv * gv, rv * rv};
  block_partials<2>(s, sc.region(P_NORM));  // -> S_GL2, S_RL2
}

struct FinishArgs {
  Scratch sc;
  FinishJob job[kMaxFinishJobs];
  int njobs;
  int* clear_int;  // optional: set to zero once every job is done (a work-list count)
};

constexpr int kFinishThreads = 1024;  // one wavefront per row, 16 rows at a time
static_assert(kSpread == kWave, "the finishing kernel folds one copy per lane");

// One block; every requested row is reduced by one wavefront in a fixed
// order (lanes stride the row, then a fixed butterfly): a row of block
// partials is summed into its slot, a spread slot's copies are folded by max
// (slot = max) or sum (slot += sum) and then cleared for the next pass.
__global__ __launch_bounds__(kFinishThreads) void k_finish(FinishArgs F) {
  constexpr int NW = kFinishThreads / kWave;
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  int row = 0;
  for (int j = 0; j < F.njobs; ++j) {
    const FinishJob jb = F.job[j];
    for (int m = 0; m < jb.M; ++m, ++row) {
      if (row % NW != wid) continue;
      double* slot = F.sc.red + jb.slot + m;
      if (jb.op == F_SUM) {
        const double* r = F.sc.region(jb.site) + (size_t)(jb.row0 + m) * jb.nb;
        double acc = 0.0;
#pragma unroll 8
        for (int b = lane; b < jb.nb; b += kWave) acc += r[b];
        acc = wave_sum(acc);
        if (lane == 0) *slot = acc;
      } else {
        double* cp = F.sc.spread + ((size_t)(jb.slot + m) * kSpread + lane) * kSpreadStride;
        const double c = *cp;  // kSpread == kWave: one copy per lane
        *cp = 0.0;
        if (jb.op == F_SPREAD_MAX) {
          const double r = wave_max(c);
          if (lane == 0) *slot = r;
        } else {
          const double r = wave_sum(c);
          if (lane == 0) *slot += r;
        }
      }
    }
  }
  if (F.clear_int && threadIdx.x == 0) *F.clear_int = 0;
}

__global__ __launch_bounds__(kBlock) void k_reset_slots(Scratch sc, int first, int count) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= count * (kSpread + 1)) return;
  const int j = i / (kSpread + 1), c = i % (kSpread + 1);
  if (c == kSpread)
    sc.red[first + j] = 0.0;
  else
    sc.spread[((size_t)(first + j) * kSpread + c) * kSpreadStride] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_spec_copy(int64_t n, const double2* src, double2* dst,
                                                     double scale) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) dst[i] = cscale(src[i], scale);
}

__global__ __launch_bounds__(kBlock) void k_accept_A(int64_t nc, double* gbuf) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= nc) return;
#pragma unroll
  for (int l = 0; l < 3; ++l) gbuf[g * kGbufStride + 3 + l] = gbuf[g * kGbufStride + 6 + l];
}

__global__ __launch_bounds__(kBlock) void k_set_A0(int64_t nc, const double* A, double* gbuf) {
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= nc) return;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    gbuf[g * kGbufStride + 3 + l] = A[l * nc + g];
    gbuf[g * kGbufStride + 6 + l] = A[l * nc + g];
  }
}

__global__ __launch_bounds__(kBlock) void k_fill(int64_t n, double* p, double v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// One pass along `axis` over nb batch fields.
template <int MODE>
void fft_pass(hipStream_t s, const Grid& G, int nb, double2* data, int axis, double sgn,
              const double2* tw, const RealIO* io, const double* prev, double* clear,
              const Scratch& sc) {
  FftPass A;
  A.data = data;
  A.tw = tw;
  A.ncell = G.ncell;
  A.N = G.n[axis];
  A.logN = ilog2(A.N);
  int64_t stride = 1;
  for (int a = axis + 1; a < 3; ++a) stride *= G.n[a];
  A.stride = stride;
  A.npb = G.ncell / A.N;
  A.npencils = (int64_t)nb * A.npb;
  A.sgn = sgn;
  if (io) A.io = *io;
  else
    for (int b = 0; b < kMaxBatch; ++b) {
      A.io.p[b] = nullptr;
      A.io.stride[b] = 1;
    }
  A.prev = prev;
  A.clear = clear;
  A.sc = sc;
  const int P = kBlock / (A.N / 2);
  const unsigned nblk = (unsigned)((A.npencils + P - 1) / P);
  k_fft<MODE><<<nblk, kBlock, 0, s>>>(A);
}

// ---- fused field solve of a Picard pass -----------------------------------
// Three kernels instead of seven: (1) per field and x-plane, the forward
// transform along z and y of the real current in LDS (with max|J - J_prev|
// and the clearing of J_prev); (2) per block of x-pencils, the forward
// transform along x, the continuity + CN update of every mode of those
// pencils, and the inverse transform along x of the six gather fields;
// (3) per field and x-plane, the inverse transform along y and z with the real
// part written to the gather buffer.  Four x-pencils per block: at 32^3
// that is 256 blocks (16 pencils per block: 64 blocks, 23 us for the pencil
// kernel alone; 4: 0.035 ms for the whole solve against 0.047 for seven
// kernels).  Every 1-D transform is the radix-2
// decimation in time of k_fft with bit-reversed LDS input; in a plane both
// indices are bit-reversed at load, so the z and y stages run back to back.
constexpr int kPlaneMax = 4096;  // ny nz limit of the plane kernels (64 KB of LDS)

__device__ __forceinline__ int brev(int e, int logn) {
  return (int)(__brev((unsigned)e) >> (32 - logn));
}

__device__ __forceinline__ void butterfly(double2* lds, int i0, int i1, double2 w) {
  const double2 a = lds[i0];
  const double2 b = cmul(lds[i1], w);
  lds[i0] = cadd(a, b);
  lds[i1] = csub(a, b);
}

struct PlaneArgs {
  Grid G;
  const double2* tw_y;  // exp(-2 pi i t / ny), t < ny/2
  const double2* tw_z;
  int logy, logz;
  // forward: real SoA input (nb fields), optional prev / clear, complex output
  const double* in;
  const double* prev;
  double* clear;
  double2* cout;
  // inverse: complex input, real output through io
  const double2* cin;
  RealIO io;
  Scratch sc;
};

// INVERSE = false: block = (field, x-plane) of the forward transform;
// true: of the inverse transform (conjugate twiddles, real output).
template <bool INVERSE>
__global__ __launch_bounds__(kBlock) void k_fft_plane(PlaneArgs A) {
  __shared__ double2 buf[kPlaneMax];
  const Grid& G = A.G;
  const int ny = G.n[1], nz = G.n[2], plane = ny * nz, nx = G.n[0];
  const int b = blockIdx.x / nx, ix = blockIdx.x % nx;
  const int64_t base = (int64_t)ix * plane, fo = (int64_t)b * G.ncell;
  double dmax = 0.0;
  for (int e = threadIdx.x; e < plane; e += kBlock) {
    const int iy = e >> A.logz, iz = e & (nz - 1);
    const int64_t g = base + e;
    double2 v;
    if constexpr (INVERSE) {
      v = A.cin[fo + g];
    } else {
      const double re = A.in[fo + g];
      if (A.prev) dmax = fmax(dmax, fabs(re - A.prev[fo + g]));
      if (A.clear) A.clear[fo + g] = 0.0;  // after prev was read (same element)
      v = make_double2(re, 0.0);
    }
    buf[(brev(iy, A.logy) << A.logz) | brev(iz, A.logz)] = v;
  }
  __syncthreads();
  const int hz = nz >> 1, hy = ny >> 1;
  for (int hs = 1; hs < nz; hs <<= 1) {  // along z: rows of nz
    for (int u = threadIdx.x; u < ny * hz; u += kBlock) {
      const int row = u / hz, j = u - row * hz, pos = j % hs;
      const int i0 = (j / hs) * 2 * hs + pos;
      double2 w = A.tw_z[pos * (hz / hs)];
      if (INVERSE) w.y = -w.y;
      butterfly(buf + row * nz, i0, i0 + hs, w);
    }
    __syncthreads();
  }
  for (int hs = 1; hs < ny; hs <<= 1) {  // along y: columns of ny, stride nz
    for (int u = threadIdx.x; u < hy * nz; u += kBlock) {
      const int col = u & (nz - 1), j = u >> A.logz, pos = j % hs;
      const int i0 = (j / hs) * 2 * hs + pos;
      double2 w = A.tw_y[pos * (hy / hs)];
      if (INVERSE) w.y = -w.y;
      butterfly(buf, i0 * nz + col, (i0 + hs) * nz + col, w);
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < plane; e += kBlock) {
    const int64_t g = base + e;
    if constexpr (INVERSE)
      A.io.p[b][g * A.io.stride[b]] = buf[e].x;
    else
      A.cout[fo + g] = buf[e];
  }
  if constexpr (!INVERSE) {
    if (A.prev) {
      const double r = block_max(dmax);
      if (threadIdx.x == 0) atomic_max_nonneg(A.sc.spread_copy(S_DJMAX), r);
    }
  }
}

struct PencilArgs {
  FieldParams F;
  const double2* tw_x;
  int logx, npl;       // pencils per block
  const double2* Jh;   // 3 fields after the z and y transforms
  const double2* cur;  // level n (9 fields)
  double2* next;       // level n+1 (9 fields)
  double2* inv;        // 6 gather fields after the inverse x transform
  Scratch sc;
};

constexpr int kPencilLds = 2 * kBlock + 16;  // npl * (nx + 1) <= 2 kBlock + npl, npl <= 16

__global__ __launch_bounds__(kBlock) void k_cn_pencils(PencilArgs A) {
  __shared__ double2 jb[3 * kPencilLds];
  __shared__ double2 ib[6 * kPencilLds];
  const Grid& G = A.F.G;
  const int nx = G.n[0], hx = nx >> 1, npl = A.npl, ld = nx + 1;  // padded pencil stride
  const int64_t S = (int64_t)G.n[1] * G.n[2], nc = G.ncell;
  const int64_t q0 = (int64_t)blockIdx.x * npl;  // first pencil (iy nz + iz) of the block
  const int span = npl * nx;
  // the three current spectra, pencil by pencil, bit-reversed along x
  for (int f = 0; f < 3; ++f)
    for (int e = threadIdx.x; e < span; e += kBlock) {
      const int kx = e / npl, pl = e - kx * npl;
      jb[f * kPencilLds + pl * ld + brev(kx, A.logx)] = A.Jh[f * nc + kx * S + q0 + pl];
    }
  __syncthreads();
  for (int hs = 1; hs < nx; hs <<= 1) {
    for (int u = threadIdx.x; u < 3 * npl * hx; u += kBlock) {
      const int f = u / (npl * hx), r = u - f * npl * hx, pl = r / hx, j = r - pl * hx;
      const int pos = j % hs, i0 = (j / hs) * 2 * hs + pos;
      butterfly(jb + f * kPencilLds + pl * ld, i0, i0 + hs, A.tw_x[pos * (hx / hs)]);
    }
    __syncthreads();
  }
  // continuity + CN of every mode of the block's pencils
  double sums[3] = {0.0, 0.0, 0.0};
  for (int e = threadIdx.x; e < span; e += kBlock) {
    const int kx = e / npl, pl = e - kx * npl;
    const int64_t g = kx * S + q0 + pl;
    double k[3];
    mode_k(G, g, k);
    double2 J[3], c[9], out[9], iv[6];
    double s3[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) J[l] = jb[l * kPencilLds + pl * ld + kx];
#pragma unroll
    for (int f = 0; f < 9; ++f) c[f] = A.cur[f * nc + g];
    cn_mode(A.F, k, J, c, out, iv, s3);
#pragma unroll
    for (int f = 0; f < 9; ++f) A.next[f * nc + g] = out[f];
#pragma unroll
    for (int f = 0; f < 6; ++f) ib[f * kPencilLds + pl * ld + brev(kx, A.logx)] = iv[f];
    sums[0] += s3[0];
    sums[1] += s3[1];
    sums[2] += s3[2];
  }
  __syncthreads();
  for (int hs = 1; hs < nx; hs <<= 1) {
    for (int u = threadIdx.x; u < 6 * npl * hx; u += kBlock) {
      const int f = u / (npl * hx), r = u - f * npl * hx, pl = r / hx, j = r - pl * hx;
      const int pos = j % hs, i0 = (j / hs) * 2 * hs + pos;
      double2 w = A.tw_x[pos * (hx / hs)];
      w.y = -w.y;
      butterfly(ib + f * kPencilLds + pl * ld, i0, i0 + hs, w);
    }
    __syncthreads();
  }
  for (int f = 0; f < 6; ++f)
    for (int e = threadIdx.x; e < span; e += kBlock) {
      const int kx = e / npl, pl = e - kx * npl;
      A.inv[f * nc + kx * S + q0 + pl] = ib[f * kPencilLds + pl * ld + kx];
    }
  block_partials<3>(sums, A.sc.region(P_CN));  // -> S_JE, S_WNEXT, S_DW
}

// ---- adjoint of the field update ----------------------------------------
// Complex spectra carry adjoints in the convention dL = Re sum conj(lambda) dz;
// every coefficient of k_cn is real except -dt i k of the continuity update,
// whose adjoint is +dt i k.  Given the adjoints l1 of the next level (9
// fields, may be null) and the gather-side adjoints lg = [grad phi^{n+1/2}
// (3), A^{n+1} (3), A^n (3)] as spectra (may be null; A^n only when lcur is
// set), writes the adjoint of J^ to lJh and adds the current level's share to
// lcur (may be null).  Transposes k_cn's arithmetic step by step.
__global__ __launch_bounds__(kBlock) void k_cn_adjoint(FieldParams F, const double2* l1,
                                                      const double2* lg, double2* lcur,
                                                      double2* lJh) {
  const Grid& G = F.G;
  const int64_t nc = G.ncell;
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= nc) return;
  double k[3];
  mode_k(G, g, k);
  const double dt = F.dt, a = 0.5 * dt, kap2 = F.kappa * F.kappa;
  const double w2 = kap2 * (k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  const double inv_den = 1.0 / (1.0 + a * a * w2);
  const double c_old = 1.0 - a * a * w2, c_x = 2.0 * a * w2;
  const double src1 = dt * kap2 * F.sigma1, src2 = dt * kap2 * F.sigma2;
  const double2 z = make_double2(0.0, 0.0);
  auto at = [&](const double2* p, int f) { return p ? p[f * nc + g] : z; };
  // gather side: grad phi^{n+1/2} = i k (phi0 + phi1)/2 -> (-i k / 2) per component
  double2 lphi_g = z;
  if (lg)
#pragma unroll
    for (int l = 0; l < 3; ++l) lphi_g = cadd(lphi_g, ik(-0.5 * k[l], lg[l * nc + g]));
  const double2 lphi1 = cadd(at(l1, F_PHI), lphi_g);
  // phi1 = phi0 + a psi0 + a psi1; psi1 = (c_old psi0 - c_x phi0 + src1 rho_h) inv_den
  const double2 lpsi1 = cadd(at(l1, F_PSI), cscale(lphi1, a));
  const double2 lphi0 = csub(cadd(lphi1, lphi_g), cscale(lpsi1, c_x * inv_den));
  const double2 lpsi0 = cadd(cscale(lphi1, a), cscale(lpsi1, c_old * inv_den));
  const double2 lrhoh = cscale(lpsi1, src1 * inv_den);
  // rho_h = (rho0 + rho1)/2, rho1 = rho0 - dt i k.J
  const double2 lrho1 = cadd(at(l1, F_RHO), cscale(lrhoh, 0.5));
  const double2 lrho0 = cadd(lrho1, cscale(lrhoh, 0.5));
  double2 lJ[3], lA0[3], lU0[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    const double2 lA1 = cadd(at(l1, F_A + l), lg ? lg[(3 + l) * nc + g] : z);
    const double2 lU1 = cadd(at(l1, F_U + l), cscale(lA1, a));
    lA0[l] = csub(lA1, cscale(lU1, c_x * inv_den));
    if (lg && lcur) lA0[l] = cadd(lA0[l], lg[(6 + l) * nc + g]);
    lU0[l] = cadd(cscale(lA1, a), cscale(lU1, c_old * inv_den));
    lJ[l] = cadd(cscale(lU1, src2 * inv_den), ik(dt * k[l], lrho1));
    lJh[l * nc + g] = lJ[l];
  }
  if (lcur) {
    lcur[F_PHI * nc + g] = cadd(lcur[F_PHI * nc + g], lphi0);
    lcur[F_PSI * nc + g] = cadd(lcur[F_PSI * nc + g], lpsi0);
    lcur[F_RHO * nc + g] = cadd(lcur[F_RHO * nc + g], lrho0);
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      lcur[(F_A + l) * nc + g] = cadd(lcur[(F_A + l) * nc + g], lA0[l]);
      lcur[(F_U + l) * nc + g] = cadd(lcur[(F_U + l) * nc + g], lU0[l]);
    }
  }
}

// Adjoint of W (eq. field-energy) with respect to the spectra of the
// present level, before the inverse transforms: with E = -i k phi - U and
// B = i k x A evaluated as real fields and scaled by dV/sigma, lE and lB are
// their forward transforms / ncell; writes the 9-field adjoint spectrum (lF
// may be the same buffer as lEB).
__global__ __launch_bounds__(kBlock) void k_energy_adjoint(Grid G, const double2* lEB,
                                                          double2* lF) {
  const int64_t nc = G.ncell;
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= nc) return;
  double k[3];
  mode_k(G, g, k);
  const double2 z = make_double2(0.0, 0.0);
  double2 lE[3], lB[3];  // all inputs first: lF may alias lEB (same mode, other rows)
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    lE[l] = lEB[l * nc + g];
    lB[l] = lEB[(3 + l) * nc + g];
  }
  double2 lphi = z, lA[3] = {z, z, z};
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    lphi = cadd(lphi, ik(k[l], lE[l]));          // E_l = -i k_l phi - U_l
    const int p = (l + 1) % 3, q = (l + 2) % 3;  // B_l = i (k_p A_q - k_q A_p)
    lA[q] = cadd(lA[q], ik(-k[p], lB[l]));
    lA[p] = cadd(lA[p], ik(k[q], lB[l]));
  }
#pragma unroll
  for (int l = 0; l < 3; ++l) lF[(F_U + l) * nc + g] = cscale(lE[l], -1.0);
  lF[F_PHI * nc + g] = lphi;
  lF[F_PSI * nc + g] = z;
  lF[F_RHO * nc + g] = z;
#pragma unroll
  for (int l = 0; l < 3; ++l) lF[(F_A + l) * nc + g] = lA[l];
}

// E = -i k phi - U and B = i k x A of the present level, / ncell (inverse
// transform inputs of the energy adjoint)
__global__ __launch_bounds__(kBlock) void k_fields_EB(Grid G, const double2* cur, double2* EB) {
  const int64_t nc = G.ncell;
  const int64_t g = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (g >= nc) return;
  double k[3];
  mode_k(G, g, k);
  const double sc = 1.0 / (double)nc;
  const double2 phi = cur[F_PHI * nc + g];
  double2 A[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    A[l] = cur[(F_A + l) * nc + g];
    EB[l * nc + g] = cscale(csub(ik(-k[l], phi), cur[(F_U + l) * nc + g]), sc);
  }
  EB[3 * nc + g] = cscale(csub(ik(k[1], A[2]), ik(k[2], A[1])), sc);
  EB[4 * nc + g] = cscale(csub(ik(k[2], A[0]), ik(k[0], A[2])), sc);
  EB[5 * nc + g] = cscale(csub(ik(k[0], A[1]), ik(k[1], A[0])), sc);
}

}  // namespace

void fft3_forward(hipStream_t s, const Grid& G, int nb, double2* data, const RealIO* in,
                  const double* prev, const double2* const* tw, Scratch sc, double* clear) {
  // z (contiguous) first, reading the real input; then y and x in place
  if (in)
    fft_pass<1>(s, G, nb, data, 2, -1.0, tw[2], in, prev, clear, sc);
  else
    fft_pass<0>(s, G, nb, data, 2, -1.0, tw[2], nullptr, nullptr, nullptr, sc);
  fft_pass<0>(s, G, nb, data, 1, -1.0, tw[1], nullptr, nullptr, nullptr, sc);
  fft_pass<0>(s, G, nb, data, 0, -1.0, tw[0], nullptr, nullptr, nullptr, sc);
}

void fft3_inverse(hipStream_t s, const Grid& G, int nb, double2* data, const RealIO* out,
                  const double2* const* tw) {
  const Scratch none{};
  fft_pass<0>(s, G, nb, data, 0, +1.0, tw[0], nullptr, nullptr, nullptr, none);
  fft_pass<0>(s, G, nb, data, 1, +1.0, tw[1], nullptr, nullptr, nullptr, none);
  if (out)
    fft_pass<2>(s, G, nb, data, 2, +1.0, tw[2], out, nullptr, nullptr, none);
  else
    fft_pass<0>(s, G, nb, data, 2, +1.0, tw[2], nullptr, nullptr, nullptr, none);
}

bool fused_field_solve_fits(const Grid& G) {
  return G.n[1] * G.n[2] <= kPlaneMax && G.n[0] <= 2 * kBlock;
}

int cn_pencil_blocks(const Grid& G) {
  const int npl = std::min(4, kBlock / (G.n[0] / 2));
  return (int)((int64_t)G.n[1] * G.n[2] / npl);
}

void field_solve_fused(hipStream_t s, const FieldParams& F, const double* J, const double* prev,
                       double* clear, const double2* cur, double2* next, double2* Jh,
                       double2* batch, const RealIO& out, const double2* const* tw, Scratch sc) {
  const Grid& G = F.G;
  PlaneArgs A{};
  A.G = G;
  A.tw_y = tw[1];
  A.tw_z = tw[2];
  A.logy = ilog2(G.n[1]);
  A.logz = ilog2(G.n[2]);
  A.in = J;
  A.prev = prev;
  A.clear = clear;
  A.cout = Jh;
  A.sc = sc;
  k_fft_plane<false><<<3 * G.n[0], kBlock, 0, s>>>(A);
  PencilArgs C{};
  C.F = F;
  C.tw_x = tw[0];
  C.logx = ilog2(G.n[0]);
  C.npl = std::min(4, kBlock / (G.n[0] / 2));
  C.Jh = Jh;
  C.cur = cur;
  C.next = next;
  C.inv = batch;
  C.sc = sc;
  k_cn_pencils<<<cn_pencil_blocks(G), kBlock, 0, s>>>(C);
  PlaneArgs B{};
  B.G = G;
  B.tw_y = tw[1];
  B.tw_z = tw[2];
  B.logy = A.logy;
  B.logz = A.logz;
  B.cin = batch;
  B.io = out;
  k_fft_plane<true><<<6 * G.n[0], kBlock, 0, s>>>(B);
}

void launch_cn_update(hipStream_t s, const FieldParams& F, const double2* cur, const double2* Jh,
                      double2* next, double2* inv, Scratch sc) {
  CNArgs C{F, cur, Jh, next, inv, sc};
  k_cn<<<blocks_for(F.G.ncell), kBlock, 0, s>>>(C);
}

void launch_half_U(hipStream_t s, const Grid& G, const double2* cur, const double2* next,
                   double2* inv) {
  k_half_U<<<blocks_for(G.ncell), kBlock, 0, s>>>(G, cur, next, inv);
}

void launch_poisson_init(hipStream_t s, const FieldParams& F, double2* cur) {
  k_poisson_init<<<blocks_for(F.G.ncell), kBlock, 0, s>>>(F, cur);
}

void launch_constraint_spectra(hipStream_t s, const FieldParams& F, const double2* cur,
                               double2* inv, Scratch sc) {
  k_constraints<<<blocks_for(F.G.ncell), kBlock, 0, s>>>(F, cur, inv, sc);
}

void launch_field_energy(hipStream_t s, const FieldParams& F, const double2* cur, Scratch sc) {
  k_field_energy<<<blocks_for(F.G.ncell), kBlock, 0, s>>>(F, cur, sc);
}

void launch_constraint_norms(hipStream_t s, int64_t ncell, const double* g, const double* r,
                             Scratch sc) {
  k_norms<<<blocks_for(ncell), kBlock, 0, s>>>(ncell, g, r, sc);
}

void launch_spec_copy(hipStream_t s, int64_t count, const double2* src, double2* dst,
                      double scale) {
  if (count <= 0) return;
  k_spec_copy<<<blocks_for(count), kBlock, 0, s>>>(count, src, dst, scale);
}

void launch_accept_A(hipStream_t s, int64_t ncell, double* gbuf) {
  k_accept_A<<<blocks_for(ncell), kBlock, 0, s>>>(ncell, gbuf);
}

void launch_set_A0(hipStream_t s, int64_t ncell, const double* A, double* gbuf) {
  k_set_A0<<<blocks_for(ncell), kBlock, 0, s>>>(ncell, A, gbuf);
}

void launch_finish(hipStream_t s, Scratch sc, const FinishJob* jobs, int njobs, int* clear_int) {
  FinishArgs F;
  F.sc = sc;
  F.njobs = njobs < kMaxFinishJobs ? njobs : kMaxFinishJobs;
  for (int j = 0; j < F.njobs; ++j) F.job[j] = jobs[j];
  F.clear_int = clear_int;
  if (F.njobs > 0 || clear_int) k_finish<<<1, kFinishThreads, 0, s>>>(F);
}

int64_t mesh_blocks(int64_t ncell) { return (ncell + kBlock - 1) / kBlock; }

void launch_fill(hipStream_t s, int64_t count, double* p, double value) {
  if (count <= 0) return;
  k_fill<<<blocks_for(count), kBlock, 0, s>>>(count, p, value);
}

void launch_reset_slots(hipStream_t s, const Scratch& sc, int first, int count) {
  if (count <= 0) return;
  k_reset_slots<<<blocks_for((int64_t)count * (kSpread + 1)), kBlock, 0, s>>>(sc, first, count);
}

}  // namespace ecpic

namespace ecpic {

void launch_cn_adjoint(hipStream_t s, const FieldParams& F, const double2* l1, const double2* lg,
                       double2* lcur, double2* lJh) {
  k_cn_adjoint<<<blocks_for(F.G.ncell), kBlock, 0, s>>>(F, l1, lg, lcur, lJh);
}

void launch_energy_adjoint(hipStream_t s, const Grid& G, const double2* lEB, double2* lF) {
  k_energy_adjoint<<<blocks_for(G.ncell), kBlock, 0, s>>>(G, lEB, lF);
}

void launch_fields_EB(hipStream_t s, const Grid& G, const double2* cur, double2* EB) {
  k_fields_EB<<<blocks_for(G.ncell), kBlock, 0, s>>>(G, cur, EB);
}

}  // namespace ecpic
