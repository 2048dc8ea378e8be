// Microbenchmarks of the device: its FP64 vector throughput and its HBM
// streaming bandwidth, the measured rates that the particle kernels'
// roofline is stated against beside the published peaks.
#include "internal.hpp"
#include "reduce.hpp"

namespace ecpic {
namespace {

constexpr int kFmaChains = 8;    // independent FMA chains per lane
constexpr int kFmaIters = 2048;  // FMAs per chain

// Every lane runs kFmaChains independent chains acc = acc b + c on registers
// (b, c and `never` are launch arguments, so nothing folds); with b in (0, 1)
// and c > 0 the chains stay positive and finite.  Their sum is stored only if
// it equals `never` (negative), which keeps the work without a store.
__global__ __launch_bounds__(kBlock) void k_fma_peak(double b, double c, double never,
                                                     double* out) {
  double acc[kFmaChains];
#pragma unroll
  for (int k = 0; k < kFmaChains; ++k) acc[k] = (double)(threadIdx.x + k);
#pragma unroll 4
  for (int it = 0; it < kFmaIters; ++it)
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) acc[k] = fma(acc[k], b, c);
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < kFmaChains; ++k) s += acc[k];
  if (s == never) out[blockIdx.x] = s;
}

// dst[i] = src[i] for n 16-byte elements, a grid-stride loop (with 256
// workgroups per compute unit the many resident waves keep enough loads in
// flight; unrolled forms with 4 or 8 loads per lane, or 32-byte elements,
// were no faster)
__global__ __launch_bounds__(kBlock) void k_stream_copy(const double2* __restrict__ src,
                                                        double2* __restrict__ dst, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
    dst[i] = src[i];
}

}  // namespace

double fma_peak_flops(int blocks) {
  return 2.0 * kFmaChains * (double)kFmaIters * kBlock * (double)blocks;
}

void launch_fma_peak(hipStream_t s, int blocks, double* out) {
  k_fma_peak<<<blocks, kBlock, 0, s>>>(1.0 - 0x1p-20, 0x1p-20, -1.0, out);
}

void launch_stream_copy(hipStream_t s, int blocks, const void* src, void* dst, int64_t n16) {
  k_stream_copy<<<blocks, kBlock, 0, s>>>(static_cast<const double2*>(src),
                                          static_cast<double2*>(dst), n16);
}

}  // namespace ecpic
