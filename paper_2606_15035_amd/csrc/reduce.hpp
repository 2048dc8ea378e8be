// Wavefront and block reductions for gfx950 (wave64).
//
// Sums are deterministic: every block writes its partial sums and a
// one-block kernel adds them in a fixed order.  Maxima of non-negative doubles use atomicMax
// on the IEEE bit pattern, which orders like the values and is
// order-independent.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ecpic {

constexpr int kBlock = 256;
constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, kWave));
  return v;
}

// Sum of M values over the block; the totals are valid in every thread of
// wave 0 (thread 0 uses them).  Must be called by all threads of the block.
template <int M>
__device__ __forceinline__ void block_sum(double (&v)[M]) {
  __shared__ double red_lds[kBlock / kWave][M > 0 ? M : 1];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int m = 0; m < M; ++m) v[m] = wave_sum(v[m]);
  if (lane == 0)
#pragma unroll
    for (int m = 0; m < M; ++m) red_lds[wid][m] = v[m];
  __syncthreads();
  if (wid == 0) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
      double s = lane < kBlock / kWave ? red_lds[lane][m] : 0.0;
      v[m] = wave_sum(s);
    }
  }
  __syncthreads();
}

__device__ __forceinline__ double block_max(double v) {
  __shared__ double max_lds[kBlock / kWave];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  v = wave_max(v);
  if (lane == 0) max_lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (wid == 0) r = wave_max(lane < kBlock / kWave ? max_lds[lane] : 0.0);
  __syncthreads();
  return r;
}

// Block reductions without a barrier after the producing loops, so that a
// wavefront that finishes early does not wait for its block's slowest one:
// every wavefront reduces its lanes (sum, or max where ismax[m]) and leaves
// its M values in LDS; the last wavefront of the block to arrive (an LDS
// counter) combines the block's wavefronts in a fixed order.  Returns true
// in exactly one thread of the block (lane 0 of that wavefront), with the
// block's values in out.  Thread 0 must run late_reduce_init<M>() before a
// barrier that precedes the call.
template <int M>
__device__ __forceinline__ unsigned int* late_counter() {
  __shared__ unsigned int c;
  return &c;
}
template <int M>
__device__ __forceinline__ double* late_values() {
  __shared__ double v[M * (kBlock / kWave)];
  return v;
}
template <int M>
__device__ __forceinline__ void late_reduce_init() {
  if (threadIdx.x == 0) *late_counter<M>() = 0u;
}
template <int M>
__device__ __forceinline__ bool late_reduce(const double (&v)[M], const bool (&ismax)[M],
                                            double (&out)[M]) {
  constexpr int NW = kBlock / kWave;
  const int wid = threadIdx.x / kWave;
  double r[M];
#pragma unroll
  for (int m = 0; m < M; ++m) r[m] = ismax[m] ? wave_max(v[m]) : wave_sum(v[m]);
  if (threadIdx.x % kWave != 0) return false;
  double* vals = late_values<M>();
#pragma unroll
  for (int m = 0; m < M; ++m) vals[m * NW + wid] = r[m];
  __threadfence_block();  // the values before the arrival count
  if (atomicAdd(late_counter<M>(), 1u) != NW - 1) return false;
  __threadfence_block();
#pragma unroll
  for (int m = 0; m < M; ++m) {
    double a = vals[m * NW];
    for (int w = 1; w < NW; ++w) a = ismax[m] ? fmax(a, vals[m * NW + w]) : a + vals[m * NW + w];
    out[m] = a;
  }
  return true;
}

// bit-pattern atomicMax of a non-negative double (order-independent)
__device__ __forceinline__ void atomic_max_nonneg(double* slot, double v) {
  if (v > 0.0)
    atomicMax(reinterpret_cast<unsigned long long*>(slot), (unsigned long long)__double_as_longlong(v));
}

// Block max of a non-negative value, folded into *slot (bit-pattern atomicMax).
// fmax drops NaN operands, so callers flag non-finite values separately.
__device__ __forceinline__ void block_max_to(double v, double* slot) {
  const double r = block_max(v);
  if (threadIdx.x == 0 && r > 0.0)
    atomicMax(reinterpret_cast<unsigned long long*>(slot), (unsigned long long)__double_as_longlong(r));
}

// Grid-wide sums, deterministic: every block writes its M block sums to
// region[m * gridDim.x + blockIdx.x]; a one-block finishing kernel (launched
// by the host after the producing kernels) adds each row in a fixed order.
// The kernel boundary in between makes the partials visible; no device-scope
// fences are needed inside the producing kernels.
template <int M>
__device__ __forceinline__ void block_partials(double (&v)[M], double* region) {
  block_sum<M>(v);
  if (threadIdx.x == 0)
#pragma unroll
    for (int m = 0; m < M; ++m) region[(size_t)m * gridDim.x + blockIdx.x] = v[m];
}

// Periodic minimum image of a node-index difference: raw mod n in
// [-n/2, n/2].
__device__ __forceinline__ int min_image(int raw, int n) {
  int r = raw % n;
  if (2 * r > n) r -= n;
  if (2 * r < -n) r += n;
  return r;
}

// block-wide minimum of M ints at once (one barrier pair for all of them)
template <int M>
__device__ __forceinline__ void block_min_ints(int (&v)[M]) {
  __shared__ int lds_i[M][kBlock / kWave];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
#pragma unroll
  for (int m = 0; m < M; ++m) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v[m] = min(v[m], __shfl_xor(v[m], o, kWave));
    if (lane == 0) lds_i[m][wid] = v[m];
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m) {
    int r = lds_i[m][0];
#pragma unroll
    for (int w = 1; w < kBlock / kWave; ++w) r = min(r, lds_i[m][w]);
    v[m] = r;
  }
  __syncthreads();
}

}  // namespace ecpic
