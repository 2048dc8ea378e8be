// Anderson mixing of the Picard iterates on the GPU (an extension of the
// nonlinear solve of Algorithm 1; the conservation statement concerns the
// converged discrete equations, not the solver that reaches them, and the
// paper names Anderson acceleration as future work, Sec. 6).
//
// Pass p has the iterate w_p = v^{n+1,p} and its image g_p = v^{n+1,p+1};
// f = g - w.  With mk = min(m, p) differences
//   dF_j = f_{p-j+1} - f_{p-j},  dG_j = g_{p-j+1} - g_{p-j},  j = 1..mk,
// the next iterate is w_{p+1} = g_p - sum_j gamma_j dG_j with gamma the
// least-squares solution of dF gamma ~ f_p (Walker and Ni 2011, mixing
// parameter 1).  k_aa_dots forms the normal equations (Gram matrix and right
// side) as deterministic block partial sums, the host solves the mk x mk
// system (anderson_gamma), and k_aa_update applies the update.  Both
// kernels stream 3 np doubles per array: the bound is HBM bandwidth.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"
#include "reduce.hpp"

namespace ecpic {

namespace {

template <int MK>
__global__ __launch_bounds__(kBlock) void k_aa_dots(int64_t n, AndersonVecs V, Scratch sc) {
  constexpr int NV = anderson_sums(MK);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += stride) {
    double f[MK + 1], df[MK];
#pragma unroll
    for (int j = 0; j <= MK; ++j) f[j] = V.g[j][e] - V.w[j][e];
#pragma unroll
    for (int j = 1; j <= MK; ++j) df[j - 1] = f[j - 1] - f[j];
    int k = 0;
#pragma unroll
    for (int i = 0; i < MK; ++i)
#pragma unroll
      for (int j = i; j < MK; ++j) acc[k++] += df[i] * df[j];
#pragma unroll
    for (int i = 0; i < MK; ++i) acc[k++] += df[i] * f[0];
  }
  block_partials<NV>(acc, sc.region(P_AA));
}

template <int MK>
__global__ __launch_bounds__(kBlock) void k_aa_update(int64_t n, AndersonVecs V,
                                                     AndersonCoef c, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  double g[MK + 1];
#pragma unroll
  for (int j = 0; j <= MK; ++j) g[j] = V.g[j][e];
  double u = g[0];
#pragma unroll
  for (int j = 1; j <= MK; ++j) u -= c.gamma[j - 1] * (g[j - 1] - g[j]);
  out[e] = u;
}

unsigned blocks_of(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int anderson_dot_blocks(int64_t n) {
  const int64_t b = (n + kBlock - 1) / kBlock;
  return (int)(b < 1 ? 1 : (b > kAndersonBlocks ? kAndersonBlocks : b));
}

void launch_anderson_dots(hipStream_t s, int mk, int64_t n, const AndersonVecs& V,
                          const Scratch& sc) {
  const int nb = anderson_dot_blocks(n);
  switch (mk) {
    case 1: k_aa_dots<1><<<nb, kBlock, 0, s>>>(n, V, sc); break;
    case 2: k_aa_dots<2><<<nb, kBlock, 0, s>>>(n, V, sc); break;
    case 3: k_aa_dots<3><<<nb, kBlock, 0, s>>>(n, V, sc); break;
    case 4: k_aa_dots<4><<<nb, kBlock, 0, s>>>(n, V, sc); break;
    default: break;
  }
}

void launch_anderson_update(hipStream_t s, int mk, int64_t n, const AndersonVecs& V,
                            const AndersonCoef& c, double* out) {
  if (n <= 0) return;
  switch (mk) {
    case 0: k_aa_update<0><<<blocks_of(n), kBlock, 0, s>>>(n, V, c, out); break;
    case 1: k_aa_update<1><<<blocks_of(n), kBlock, 0, s>>>(n, V, c, out); break;
    case 2: k_aa_update<2><<<blocks_of(n), kBlock, 0, s>>>(n, V, c, out); break;
    case 3: k_aa_update<3><<<blocks_of(n), kBlock, 0, s>>>(n, V, c, out); break;
    case 4: k_aa_update<4><<<blocks_of(n), kBlock, 0, s>>>(n, V, c, out); break;
    default: break;
  }
}

// gamma from the normal equations A gamma = b, A = dF^T dF (sums[] holds the
// upper triangle row by row, then b = dF^T f_p).  The Cholesky factor is
// built one difference at a time, newest first; a difference whose pivot is
// at most 1e-12 of its diagonal (the part of dF_j outside the span of the
// kept ones is at most 1e-6 of |dF_j|), or whose diagonal is zero, is
// dropped with gamma_j = 0.
void anderson_gamma(int mk, const double* sums, double* gamma) {
  double A[kMaxAnderson][kMaxAnderson];
  int k = 0;
  for (int i = 0; i < mk; ++i)
    for (int j = i; j < mk; ++j) A[i][j] = A[j][i] = sums[k++];
  const double* b = sums + k;
  double L[kMaxAnderson][kMaxAnderson] = {};
  int kept[kMaxAnderson];
  int nk = 0;
  for (int j = 0; j < mk; ++j) {
    gamma[j] = 0.0;
    if (!(A[j][j] > 0.0)) continue;
    double row[kMaxAnderson];
    double d = A[j][j];
    for (int c = 0; c < nk; ++c) {
      double t = A[j][kept[c]];
      for (int l = 0; l < c; ++l) t -= row[l] * L[c][l];
      row[c] = t / L[c][c];
      d -= row[c] * row[c];
    }
    if (!(d > 1e-12 * A[j][j])) continue;
    for (int c = 0; c < nk; ++c) L[nk][c] = row[c];
    L[nk][nk] = std::sqrt(d);
    kept[nk++] = j;
  }
  double y[kMaxAnderson], x[kMaxAnderson];
  for (int c = 0; c < nk; ++c) {
    double t = b[kept[c]];
    for (int l = 0; l < c; ++l) t -= L[c][l] * y[l];
    y[c] = t / L[c][c];
  }
  for (int c = nk - 1; c >= 0; --c) {
    double t = y[c];
    for (int l = c + 1; l < nk; ++l) t -= L[l][c] * x[l];
    x[c] = t / L[c][c];
  }
  for (int c = 0; c < nk; ++c) gamma[kept[c]] = x[c];
}

}  // namespace ecpic
