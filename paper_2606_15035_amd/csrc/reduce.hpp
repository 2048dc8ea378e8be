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

}  // namespace ecpic
