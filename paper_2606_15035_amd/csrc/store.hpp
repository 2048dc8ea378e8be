// Particle state storage on the device: x^n, v^n and v^{n-1}.
//
// Fp64Store:  3 x np doubles each (component a of particle i at a * np + i).
// MixedStore: the cell that holds x^n as one int32 (flat node index of its
//             lower corner), the offset inside that cell in cell units as
//             3 x np floats, and v^n, v^{n-1} as 3 x np floats.  A position
//             is decoded to FP64 as (cell + offset) H, the same value every
//             time, and every orbit, weight, field and energy operation runs
//             in FP64 on the decoded values; only the stored state is FP32.
// The Picard iterates v^{n+1,p} are FP64 arrays outside the store in both
// forms.  With several species each store also holds one byte per particle,
// its species (null with one species).  Kernels take the store as a template
// parameter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "orbit.hpp"

namespace ecpic {

constexpr int kMaxSpecies = 4;

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", OOPSLA 2014): a counter-based 64-bit generator, here keyed by
// (particle id, step, component) so that the numbers depend on neither the
// order of the particles nor the launch configuration.
__device__ __forceinline__ uint64_t splitmix64(uint64_t z) {
  z += 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
// uniform in [0, 1) from the top 53 bits
__device__ __forceinline__ double uniform01(uint64_t z) {
  return (double)(splitmix64(z) >> 11) * 0x1p-53;
}

struct Fp64Store {
  static constexpr bool kMixed = false;
  double* x;
  double* v;
  double* vp;
  uint8_t* sp = nullptr;

  __device__ __forceinline__ int species(int64_t i) const { return sp ? (int)sp[i] : 0; }

  __device__ __forceinline__ void x_of(const Grid&, int64_t np, int64_t i, double* o) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a] = x[a * np + i];
  }
  __device__ __forceinline__ void v_of(int64_t np, int64_t i, double* o) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a] = v[a * np + i];
  }
  __device__ __forceinline__ void vp_of(int64_t np, int64_t i, double* o) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a] = vp[a * np + i];
  }
  // xw wrapped into [0, L)
  __device__ __forceinline__ void set_x(const Grid&, int64_t np, int64_t i, const double* xw) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a * np + i] = xw[a];
  }
  __device__ __forceinline__ void set_v(int64_t np, int64_t i, const double* w) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a * np + i] = w[a];
  }
  __device__ __forceinline__ void set_vp(int64_t np, int64_t i, const double* w) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) vp[a * np + i] = w[a];
  }
  // the value a velocity component has once stored
  __device__ __forceinline__ static double stored(double w) { return w; }
  // key of the accepted velocity's rounding (FP64 does not round)
  __device__ __forceinline__ uint64_t state_key(int64_t, int64_t) const { return 0; }
  // the accepted velocity v^{n+1} into v^n (FP64: exact); returns the stored values
  __device__ __forceinline__ void accept_v(int64_t np, int64_t i, const double* w, uint64_t,
                                           double* out) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      v[a * np + i] = w[a];
      out[a] = w[a];
    }
  }
  // cell of x^n (lower-corner node per axis)
  __device__ __forceinline__ void cell_of(const Grid& G, int64_t np, int64_t i, int* c) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) c[a] = to_int_clamped(floor(x[a * np + i] * G.invH[a]));
  }
  // particle i of this store -> particle j of dst
  __device__ __forceinline__ void move_to(const Fp64Store& dst, int64_t np, int64_t i,
                                          int64_t j) const {
    if (sp) dst.sp[j] = sp[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      dst.x[a * np + j] = x[a * np + i];
      dst.v[a * np + j] = v[a * np + i];
      dst.vp[a * np + j] = vp[a * np + i];
    }
  }
};

struct MixedStore {
  static constexpr bool kMixed = true;
  int* cell;
  float* off;
  float* v;
  float* vp;
  uint8_t* sp = nullptr;

  __device__ __forceinline__ int species(int64_t i) const { return sp ? (int)sp[i] : 0; }

  __device__ __forceinline__ void x_of(const Grid& G, int64_t np, int64_t i, double* o) const {
    const int c = cell[i];
    const int ci[3] = {c >> G.shx, (c >> G.shy) & G.mask[1], c & G.mask[2]};
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a] = ((double)ci[a] + (double)off[a * np + i]) * G.H[a];
  }
  __device__ __forceinline__ void v_of(int64_t np, int64_t i, double* o) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a] = (double)v[a * np + i];
  }
  __device__ __forceinline__ void vp_of(int64_t np, int64_t i, double* o) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) o[a] = (double)vp[a * np + i];
  }
  // xw wrapped into [0, L): cell = floor(xw / H), offset = xw / H - cell
  // rounded to FP32 (an offset that rounds up to 1 moves to the next cell)
  __device__ __forceinline__ void set_x(const Grid& G, int64_t np, int64_t i, const double* xw) const {
    int ci[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double u = xw[a] * G.invH[a];
      const double fl = floor(u);
      float f = (float)(u - fl);
      int k = to_int_clamped(fl);
      if (f >= 1.0f) {
        f = 0.0f;
        k += 1;
      }
      ci[a] = k & G.mask[a];
      off[a * np + i] = f;
    }
    cell[i] = (ci[0] << G.shx) | (ci[1] << G.shy) | ci[2];
  }
  __device__ __forceinline__ void set_v(int64_t np, int64_t i, const double* w) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) v[a * np + i] = (float)w[a];
  }
  __device__ __forceinline__ void set_vp(int64_t np, int64_t i, const double* w) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) vp[a * np + i] = (float)w[a];
  }
  __device__ __forceinline__ static double stored(double w) { return (double)(float)w; }
  // A hash of the particle's stored state (cell, offsets, v^n): the same for
  // the same particle whatever its index, so that a step does not depend on
  // the order of the particles.
  __device__ __forceinline__ uint64_t state_key(int64_t np, int64_t i) const {
    uint64_t h = splitmix64((uint64_t)(uint32_t)cell[i]);
#pragma unroll
    for (int a = 0; a < 3; ++a) h = splitmix64(h ^ (uint64_t)__float_as_uint(off[a * np + i]));
#pragma unroll
    for (int a = 0; a < 3; ++a)
      h = splitmix64(h ^ ((uint64_t)__float_as_uint(v[a * np + i]) << 32));
    return h;
  }
  // The accepted velocity v^{n+1} into v^n, each component rounded to one of
  // its two neighbouring FP32 values, up with probability (w - lo) / (hi - lo)
  // (stochastic rounding; key: the state_key of the particle before the
  // update, mixed with the step).
  // Rounded to nearest, the velocities of a cold lattice beam, which are
  // nearly equal, round alike and their kinetic-energy errors add up
  // (1.7e-9 of the energy per step on the 32^3 two-stream workload); rounded
  // without bias they add like independent errors, ~2^-24 / sqrt(N_p).
  // Returns the stored values.
  __device__ __forceinline__ void accept_v(int64_t np, int64_t i, const double* w, uint64_t key,
                                           double* out) const {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float f = (float)w[a];
      if ((double)f != w[a] && isfinite(f)) {
        float lo = f, hi = f;
        if ((double)f > w[a])
          lo = nextafterf(f, -INFINITY);
        else
          hi = nextafterf(f, INFINITY);
        const double pu = (w[a] - (double)lo) / ((double)hi - (double)lo);
        f = uniform01(key * 3ull + (uint64_t)a) < pu ? hi : lo;
      }
      v[a * np + i] = f;
      out[a] = (double)f;
    }
  }
  __device__ __forceinline__ void cell_of(const Grid& G, int64_t, int64_t i, int* c) const {
    const int k = cell[i];
    c[0] = k >> G.shx;
    c[1] = (k >> G.shy) & G.mask[1];
    c[2] = k & G.mask[2];
  }
  __device__ __forceinline__ void move_to(const MixedStore& dst, int64_t np, int64_t i,
                                          int64_t j) const {
    dst.cell[j] = cell[i];
    if (sp) dst.sp[j] = sp[i];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      dst.off[a * np + j] = off[a * np + i];
      dst.v[a * np + j] = v[a * np + i];
      dst.vp[a * np + j] = vp[a * np + i];
    }
  }
};

}  // namespace ecpic
