// Counting sort of the particles by the mesh cell of x^n, run at the start of
// a time step.  Keeping each cell's particles contiguous keeps the stencil
// reads of a wavefront in a few cache lines (gather) and the node box of a
// scatter chunk small enough for its LDS tile.  The two beams of a
// two-stream problem drift apart by 2 v0 dt per step, so without re-sorting
// a chunk's box grows linearly in time.
//
// Cells are numbered like nodes (z fastest); inside a cell the particles are
// grouped by the octant of their velocity.  The order inside a group is the
// order in which the atomic cursor hands out slots, so it is not
// reproducible; every result of the method is invariant under particle
// permutation up to rounding.  A particle id array travels with the
// particles so that state read-back and upload use the caller's order.
#include <hip/hip_runtime.h>

#include "internal.hpp"
#include "reduce.hpp"

namespace ecpic {

namespace {

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Wavefront-aggregated atomicAdd(counter + key, 1): the lanes of a wavefront
// that share a key take one atomic for the whole group and consecutive
// slots in lane order.  With sorted keys a wavefront has only a few distinct
// keys, so this replaces tens of same-address atomics by one.  Returns the
// lane's slot (old value + rank among the group's lanes).
__device__ __forceinline__ int wave_aggregated_inc(int* counter, int key, bool active) {
  const int lane = threadIdx.x % kWave;
  unsigned long long todo = __ballot(active);
  int slot = 0;
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int lkey = __shfl(key, leader, kWave);
    const unsigned long long group = __ballot(active && key == lkey) & todo;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter + lkey, __popcll(group));
    base = __shfl(base, leader, kWave);
    if ((group >> lane) & 1ull) slot = base + __popcll(group & ((1ull << lane) - 1ull));
    todo &= ~group;
  }
  return slot;
}

__global__ __launch_bounds__(kBlock) void k_fill_int(int64_t n, int* p, int v) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_iota(int64_t n, int* p) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) p[i] = (int)i;
}

// key = 8 * cell + octant of v^n: inside a cell, particles moving the same
// way stay together, which keeps the orbit-piece structure of a wavefront's
// lanes alike (less divergence in the gather).
template <class PS>
__global__ __launch_bounds__(kBlock) void k_cell_keys(Grid G, int64_t np, PS st,
                                                     int* __restrict__ key,
                                                     int* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < np;
  int k = 0;
  if (active) {
    int c[3];
    double va[3];
    st.cell_of(G, np, i, c);
    st.v_of(np, i, va);
    int oct = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) oct |= (va[a] > 0.0 ? 1 : 0) << a;
    k = (node_index(G, c[0], c[1], c[2]) << 3) | oct;
    key[i] = k;
  }
  wave_aggregated_inc(count, k, active);
}

// Exclusive scan of count[0..n) into offset[0..n] and cursor[0..n):
// (1) per-block totals of kScanTile elements, (2) one block scans the
// totals, (3) every block scans its tile starting from its total's prefix.
constexpr int kScanPer = 4;
constexpr int kScanTile = kBlock * kScanPer;

__device__ __forceinline__ int block_exclusive_scan(int v, int* total) {
  __shared__ int sh[kBlock / kWave];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  int incl = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const int t = __shfl_up(incl, o, kWave);
    if (lane >= o) incl += t;
  }
  if (lane == kWave - 1) sh[wid] = incl;
  __syncthreads();
  int woff = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kBlock / kWave; ++w) {
    if (w < wid) woff += sh[w];
    tot += sh[w];
  }
  __syncthreads();
  *total = tot;
  return woff + incl - v;
}

__global__ __launch_bounds__(kBlock) void k_scan_totals(int64_t n, const int* __restrict__ count,
                                                       int* __restrict__ totals) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < n) s += count[base + k];
  double v[1] = {(double)s};  // counts stay far below 2^53: the double sum is exact
  block_sum<1>(v);
  if (threadIdx.x == 0) totals[blockIdx.x] = (int)v[0];
}

__global__ __launch_bounds__(kBlock) void k_scan_block_totals(int64_t nb, int* __restrict__ totals,
                                                             int* __restrict__ offset_end,
                                                             int64_t n) {
  // one block, nb totals, scanned in chunks of kBlock
  int carry = 0;
  for (int64_t c = 0; c < nb; c += kBlock) {
    const int64_t i = c + threadIdx.x;
    const int v = i < nb ? totals[i] : 0;
    int tot;
    const int ex = block_exclusive_scan(v, &tot);
    if (i < nb) totals[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) offset_end[n] = carry;
}

__global__ __launch_bounds__(kBlock) void k_scan_apply(int64_t n, const int* __restrict__ count,
                                                      const int* __restrict__ totals,
                                                      int* __restrict__ offset,
                                                      int* __restrict__ cursor) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  int c[kScanPer];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    c[k] = base + k < n ? count[base + k] : 0;
    s += c[k];
  }
  int tot;
  int acc = totals[blockIdx.x] + block_exclusive_scan(s, &tot);
#pragma unroll
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) {
      offset[base + k] = acc;
      cursor[base + k] = acc;
    }
    acc += c[k];
  }
}

template <class PS>
__global__ __launch_bounds__(kBlock) void k_permute(int64_t np, const int* __restrict__ key,
                                                   int* __restrict__ cursor, PS src, PS dst,
                                                   const int* __restrict__ id,
                                                   int* __restrict__ id2,
                                                   double* __restrict__ vit,
                                                   double* __restrict__ vbar) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const bool active = i < np;
  const int k = active ? key[i] : 0;
  const int64_t j = wave_aggregated_inc(cursor, k, active);
  if (!active) return;
  src.move_to(dst, np, i, j);
  id2[j] = id[i];
  if (vit) {  // v^{n+1,0} = 2 v^n - v^{n-1}
    double v[3], vp[3];
    src.v_of(np, i, v);
    src.vp_of(np, i, vp);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double w = 2.0 * v[a] - vp[a];
      vit[a * np + j] = w;
      if (vbar) vbar[a * np + j] = 0.5 * (w + v[a]);
    }
  }
}

// dst[a*np + id[i]] = src[a*np + i]   (stored order -> caller order)
__global__ __launch_bounds__(kBlock) void k_to_caller(int64_t np, const int* __restrict__ id,
                                                     const double* __restrict__ src,
                                                     double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= np) return;
  const int64_t k = id[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) dst[a * np + k] = src[a * np + i];
}

// dst[a*np + i] = src[a*np + id[i]]   (caller order -> stored order)
__global__ __launch_bounds__(kBlock) void k_from_caller(int64_t np, const int* __restrict__ id,
                                                       const double* __restrict__ src,
                                                       double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= np) return;
  const int64_t k = id[i];
#pragma unroll
  for (int a = 0; a < 3; ++a) dst[a * np + i] = src[a * np + k];
}

}  // namespace

int64_t sort_scan_blocks(int64_t ncell) { return (8 * ncell + kScanTile - 1) / kScanTile; }

void launch_iota(hipStream_t s, int64_t n, int* p) {
  if (n > 0) k_iota<<<blocks_for(n), kBlock, 0, s>>>(n, p);
}

template <class PS>
void launch_sort(hipStream_t s, const Grid& G, int64_t np, PS& cur, PS& alt, int*& id, int*& id2,
                 const SortScratch& b, double* vit, double* vbar) {
  if (np <= 0) return;
  const int64_t nkeys = 8 * G.ncell;
  k_fill_int<<<blocks_for(nkeys), kBlock, 0, s>>>(nkeys, b.count, 0);
  k_cell_keys<PS><<<blocks_for(np), kBlock, 0, s>>>(G, np, cur, b.key, b.count);
  const int64_t nb = (nkeys + kScanTile - 1) / kScanTile;
  k_scan_totals<<<(unsigned)nb, kBlock, 0, s>>>(nkeys, b.count, b.scan_totals);
  k_scan_block_totals<<<1, kBlock, 0, s>>>(nb, b.scan_totals, b.offset, nkeys);
  k_scan_apply<<<(unsigned)nb, kBlock, 0, s>>>(nkeys, b.count, b.scan_totals, b.offset, b.cursor);
  k_permute<PS><<<blocks_for(np), kBlock, 0, s>>>(np, b.key, b.cursor, cur, alt, id, id2, vit,
                                                   vbar);
  // the sorted copies become the particle arrays
  const PS t = cur;
  cur = alt;
  alt = t;
  int* ti = id;
  id = id2;
  id2 = ti;
}

template void launch_sort<Fp64Store>(hipStream_t, const Grid&, int64_t, Fp64Store&, Fp64Store&,
                                     int*&, int*&, const SortScratch&, double*,
                                     double*);
template void launch_sort<MixedStore>(hipStream_t, const Grid&, int64_t, MixedStore&,
                                      MixedStore&, int*&, int*&, const SortScratch&, double*,
                                     double*);

void launch_to_caller(hipStream_t s, int64_t np, const int* id, const double* src, double* dst) {
  if (np > 0) k_to_caller<<<blocks_for(np), kBlock, 0, s>>>(np, id, src, dst);
}

void launch_from_caller(hipStream_t s, int64_t np, const int* id, const double* src, double* dst) {
  if (np > 0) k_from_caller<<<blocks_for(np), kBlock, 0, s>>>(np, id, src, dst);
}

}  // namespace ecpic
