// Host-side declarations shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "orbit.hpp"
#include "store.hpp"

namespace ecpic {

// Anderson mixing: at most this many differences, and the sums its
// least-squares step needs (upper triangle of the Gram matrix + right side).
constexpr int kMaxAnderson = 4;
constexpr int anderson_sums(int mk) { return mk * (mk + 1) / 2 + mk; }
constexpr int kAndersonSums = anderson_sums(kMaxAnderson);

// Reduction slots (doubles) in the device scratch array.
enum Slot : int {
  S_DVMAX = 0,  // max_i |v^{p+1} - v^p|_inf            (bit-pattern max)
  S_VMAX,       // max_i |v^{p+1}|_inf                  (bit-pattern max)
  S_DJMAX,      // max_g |J^p - J^{p-1}|                (bit-pattern max)
  S_JS,         // J_s = sum_i |q| |vbar_i|_inf / |Omega| (sum)
  S_BAD,        // 1: an orbit had too many pieces, 1.5: a current contribution beyond the
                // fixed-point range, 2: a non-finite velocity (max)
  S_AA,         // Anderson sums dF_i . dF_j (i <= j), then dF_i . f_p   (sums)
  S_AA_END = S_AA + kAndersonSums - 1,
  S_JE,         // sum_g J . E^{n+1/2} dV               (sum)
  S_WNEXT,      // W of the new field level             (sum)
  S_DW,         // W^{n+1} - W^n, per-mode differences  (sum)
  S_K,          // K of the new particle level          (sum)
  S_DK,         // K^{n+1} - K^n, per-particle differences (sum)
  S_WORK,       // sum_i q vbar . Ebar                  (sum)
  S_RA2,        // sum_i |R_A,i|^2                      (sum)
  S_RAMAX,      // max |R_A|                            (bit-pattern max)
  S_POU,        // max_i |sum_g Sbar_ig - 1|            (bit-pattern max)
  S_GMAX,       // max |G_h|                            (bit-pattern max)
  S_RMAX,       // max |R_h|                            (bit-pattern max)
  S_GL2,        // sum G_h^2                            (sum)
  S_RL2,        // sum R_h^2                            (sum)
  S_WCUR,       // W of the current field level         (sum)
  S_PIECES,     // orbit pieces summed over particles    (sum of integers)
  S_SMISS,      // scatter chunks whose node box missed the LDS tile (sum of integers)
  S_NSLOTS
};
// Producer sites of block partial sums (each has its own region).
enum Site : int { P_JS = 0, P_CN, P_SWEEP, P_K, P_W, P_NORM, P_AA, P_NSITES };
constexpr int kMaxSumValues = 4;

// Gauss-Legendre rule on [0, 1] for orbits integrated without splitting at
// knots (comparison runs): n points s[q] with weights w[q] (sum 1).
constexpr int kMaxRule = 16;
struct QuadRule {
  int n;
  double s[kMaxRule];
  double w[kMaxRule];
};

struct StepParams {
  Grid G;
  double dt, q, m;  // q, m: species 0, the reference charge of the fixed-point current
  int64_t np;
  int split;      // 1: split orbit integrals at knots; 0: one rule over the orbit
  QuadRule rule;  // the rule of split = 0
  // particle species (each particle carries its own charge and mass, Sec. 2):
  // a particle of species s has qs[s], ms[s]; one species: the store holds no
  // species array and every particle has (q, m) = (qs[0], ms[0])
  int chunk;  // particles per scatter block: 4096 or 2048 (always 2048 for degree 3)
  int nsp;
  double qs[kMaxSpecies];
  double ms[kMaxSpecies];
  double cq[kMaxSpecies];  // current coefficient: q_s / dV (FP64), q_s / q_0 (fixed point)
  double aq[kMaxSpecies];  // |q_s| / |Omega| (beam-current scale J_s)
};

// the entry of a species table for species s (a select chain: the tables stay
// in kernel arguments, no per-lane indexing)
__device__ __forceinline__ double species_value(const double (&t)[kMaxSpecies], int s) {
  double r = t[0];
#pragma unroll
  for (int k = 1; k < kMaxSpecies; ++k) r = s == k ? t[k] : r;
  return r;
}

// Slots that many blocks of a kernel update with atomics (maxima, exact
// integer counts) get kSpread copies, one 128-byte line apart, so that the
// atomics of different blocks rarely meet on one address; a block uses copy
// blockIdx.x % kSpread and k_finish folds the copies into the slot.
constexpr int kSpread = 64;
constexpr int kSpreadStride = 16;

struct Scratch {
  double* red;          // S_NSLOTS
  double* part;         // P_NSITES regions of part_stride doubles
  int64_t part_stride;  // kMaxSumValues * (largest grid of a producing kernel)
  double* spread;       // S_NSLOTS x kSpread copies, kSpreadStride doubles apart
  __host__ __device__ double* region(int site) const { return part + site * part_stride; }
  __device__ double* spread_copy(int slot) const {
    return spread + ((size_t)slot * kSpread + blockIdx.x % kSpread) * kSpreadStride;
  }
};

// One row reduction for the finishing kernel: rows row0 .. row0 + M - 1 of
// site `site`, each over nb partials, into red[slot .. slot + M).
// F_SUM: set the slot to the sum of the partial row; F_SPREAD_MAX: set the slot
// to the max of its kSpread copies; F_SPREAD_SUM: add the sum of the copies to
// the slot.  Spread copies are cleared once folded (site, nb, row0 unused).
enum FinishOp : int { F_SUM = 0, F_SPREAD_MAX = 1, F_SPREAD_SUM = 2 };
struct FinishJob {
  int site, nb, M, slot;
  int op = F_SUM;
  int row0 = 0;
};
constexpr int kMaxFinishJobs = 8;
// clear_int (optional): an int set to zero after the jobs (the gather's work-list count)
void launch_finish(hipStream_t s, Scratch sc, const FinishJob* jobs, int njobs,
                   int* clear_int = nullptr);

// Anderson mixing (anderson.hip): iterates w[j] and images g[j] of passes
// p - j, j = 0..mk, each 3 x np doubles.
struct AndersonVecs {
  const double* w[kMaxAnderson + 1];
  const double* g[kMaxAnderson + 1];
};
struct AndersonCoef {
  double gamma[kMaxAnderson];
};
constexpr int kAndersonBlocks = 2048;  // grid of the dot-product kernel (at most)
int anderson_dot_blocks(int64_t n);
// block partial sums of anderson_sums(mk) values into site P_AA (mk = 1..4)
void launch_anderson_dots(hipStream_t s, int mk, int64_t n, const AndersonVecs& V,
                          const Scratch& sc);
// out = g[0] - sum_j gamma_j (g[j-1] - g[j]), j = 1..mk (mk = 0: a copy of g[0])
void launch_anderson_update(hipStream_t s, int mk, int64_t n, const AndersonVecs& V,
                            const AndersonCoef& c, double* out);
// host: gamma (mk values) from the anderson_sums(mk) sums of k_aa_dots
void anderson_gamma(int mk, const double* sums, double* gamma);
// grid sizes of the producing kernels
int64_t scatter_blocks(int64_t np, int chunk);
int64_t particle_blocks(int64_t np);
int64_t mesh_blocks(int64_t ncell);

// ---- particle kernels (particles.hip) ----
// PS = Fp64Store or MixedStore (store.hpp); explicit instantiations of both
// live in particles.hip and sort.hip.
//
// Orbit current output: FP64 state adds into J (3 x ncell doubles); mixed
// state adds int64 fixed-point quanta into Jfix (3 x ncell), turned into J
// by launch_fixed_current.
struct CurrentOut {
  double* J;
  unsigned long long* Jfix;
  double fix_scale;  // quanta per unit of vbar Sbar (2^40 by default)
};
// v^{n+1,0} = 2 v^n - v^{n-1} into vit and, with vbar, its vbar^0 there
template <class PS>
void launch_extrapolate(hipStream_t s, int64_t np, const PS& st, double* vit,
                        double* vbar = nullptr);
// Node boxes of the scatter's chunks, kBoxInts ints per chunk (reference
// cell, box origin and extents, each per axis).  With box non-null and reuse
// zero the scatter finds each chunk's box from its orbits and stores it; with
// reuse non-zero it takes the stored box (x^n, and with it the chunk's
// cells, is the same in every pass of a step; an orbit whose stencil leaves
// the stored box goes through the scatter's global-memory path).
constexpr int kBoxInts = 12;
struct ChunkBoxes {
  int* box = nullptr;
  int reuse = 0;
};
// Orbit current of iterate vit; with vbar non-null, vbar^p (3 x np) is read
// from there instead of being formed from v^n and vit
template <class PS>
void launch_scatter(hipStream_t s, int r, const StepParams& P, const PS& st, const double* vit,
                    const double* vbar, CurrentOut out, Scratch sc, ChunkBoxes bx = {});
// Iterate and image of the previous Picard pass: with w non-null the gather
// also writes the block partial sums dF . dF and dF . f_p of Anderson mixing
// over one difference (dF = f_p - f_{p-1}, f = image - iterate) to site P_AA.
struct AndersonPrev {
  const double* w = nullptr;
  const double* g = nullptr;
};
// work: 1 + (blocks of 256 particles) ints, work[0] = 0 on entry; the tiled
// kernel lists the blocks whose node box missed the LDS tile, the second
// kernel runs them from global memory; the per-pass finishing kernel resets
// work[0].  vbar_out (nullable): (vnew + v^n) / 2, the vbar of a next pass
// whose iterate is vnew.  bx: node boxes of the blocks of 256 particles, as
// for the scatter's chunks; with reuse, a block one of whose orbits leaves
// its stored box finds its box again and stores it.
template <class PS>
void launch_gather_push(hipStream_t s, int r, const StepParams& P, const PS& st,
                        const double* vit, double* vnew, double* vbar_out, const double* gbuf,
                        int* work, Scratch sc, AndersonPrev prev = AndersonPrev{},
                        ChunkBoxes bx = {});
template <class PS>
void launch_sweep(hipStream_t s, int r, const StepParams& P, const PS& st, const double* vit,
                  const double* gbuf, const double* Uhalf, Scratch sc);
// step: the step being accepted (part of the key of the store's rounding of
// the accepted velocity)
template <class PS>
void launch_finalize(hipStream_t s, const StepParams& P, const PS& st, const double* vit,
                     const double* vnew, uint64_t step, Scratch sc);
template <class PS>
void launch_kinetic(hipStream_t s, const StepParams& P, const PS& st, Scratch sc);
// rho^0 of the point shapes: FP64 adds into out.J (ncell); mixed adds
// fixed-point quanta into out.Jfix (then launch_fixed_current)
template <class PS>
void launch_deposit_rho(hipStream_t s, int r, const StepParams& P, const PS& st, CurrentOut out);
// which: 0 = x (wrapped into [0, L) on import), 1 = v^n, 2 = v^{n-1};
// src/dst are 3 x np doubles in stored order
template <class PS>
void launch_import(hipStream_t s, const StepParams& P, const PS& st, int which, const double* src);
template <class PS>
void launch_export(hipStream_t s, const StepParams& P, const PS& st, int which, double* dst);
// J = unit * Jfix (as signed integers), then Jfix = 0
void launch_fixed_current(hipStream_t s, int64_t n, unsigned long long* Jfix, double* J,
                          double unit);
// kernel-level checks; rule = nullptr: split orbits, else that rule over [0, 1]
void launch_orbit_gather_soa(hipStream_t s, int r, const QuadRule* rule, const Grid& G,
                             int64_t n, const double* x0, const double* d, const double* gphi,
                             const double* U, const double* A0, const double* A1, double* out);
void launch_orbit_deposit_soa(hipStream_t s, int r, const QuadRule* rule, const Grid& G,
                              int64_t n, const double* x0, const double* d, const double* qv,
                              double* J);

// ---- particle sort (sort.hip) ----
struct SortScratch {
  int* key;     // np
  int* count;   // 8 * ncell (cell x velocity octant)
  int* offset;  // 8 * ncell + 1
  int* cursor;  // 8 * ncell
  int* scan_totals;  // sort_scan_blocks(ncell)
};
int64_t sort_scan_blocks(int64_t ncell);
void launch_iota(hipStream_t s, int64_t n, int* p);
// Sorts the particles of cur (with their ids) into alt, then swaps cur/alt
// and id/id2, so that cur and id hold the sorted particles.  With vit, the
// permutation also writes the first Picard guess 2 v^n - v^{n-1} of every
// particle there, in the sorted order (3 x np FP64, component-major), and
// with vbar its vbar^0.
template <class PS>
void launch_sort(hipStream_t s, const Grid& G, int64_t np, PS& cur, PS& alt, int*& id, int*& id2,
                 const SortScratch& b, double* vit = nullptr, double* vbar = nullptr);
void launch_to_caller(hipStream_t s, int64_t np, const int* id, const double* src, double* dst);
void launch_from_caller(hipStream_t s, int64_t np, const int* id, const double* src, double* dst);

// ---- mesh kernels (mesh.hip) ----
constexpr int kMaxBatch = 9;
struct RealIO {
  double* p[kMaxBatch];
  int64_t stride[kMaxBatch];
};

// 3D FFT of nb fields held as complex arrays data[b*ncell + g], z fastest.
// forward: real input from `in` (may be nullptr for complex in-place), and
// optionally max|in - prev| folded into S_DJMAX.  inverse: real part of the
// result to `out` (nullptr keeps the complex result in place).
// clear (optional): a real buffer laid out like prev, zeroed by the first pass
void fft3_forward(hipStream_t s, const Grid& G, int nb, double2* data, const RealIO* in,
                  const double* prev, const double2* const* tw, Scratch sc,
                  double* clear = nullptr);
void fft3_inverse(hipStream_t s, const Grid& G, int nb, double2* data, const RealIO* out,
                  const double2* const* tw);

struct FieldParams {
  Grid G;
  double dt, kappa, sigma1, sigma2;
};

// Continuity + CN update of every mode; writes the next spectral level, the
// inverse-transform inputs [i k (phi0+phi1)/2, A1] / ncell, and S_JE, S_WNEXT,
// S_DW.
// The field solve of a Picard pass in three kernels (transforms along z and y
// per x-plane, then x with the continuity + CN update per block of x-pencils,
// then the inverse along y and z into the gather buffer); same results as
// fft3_forward + launch_cn_update + fft3_inverse up to rounding.  Needs
// ny nz <= 4096; the P_CN partial rows have cn_pencil_blocks(G) blocks.
bool fused_field_solve_fits(const Grid& G);
int cn_pencil_blocks(const Grid& G);
void field_solve_fused(hipStream_t s, const FieldParams& F, const double* J, const double* prev,
                       double* clear, const double2* cur, double2* next, double2* Jh,
                       double2* batch, const RealIO& out, const double2* const* tw, Scratch sc);
void launch_cn_update(hipStream_t s, const FieldParams& F, const double2* cur, const double2* Jh,
                      double2* next, double2* inv, Scratch sc);
// (U0 + U1)/2 / ncell into inv[0..2]
void launch_half_U(hipStream_t s, const Grid& G, const double2* cur, const double2* next,
                   double2* inv);
// Initial potentials from a forward-transformed charge in cur[8*ncell..].
void launch_poisson_init(hipStream_t s, const FieldParams& F, double2* cur);
// G_h and R_h spectra / ncell into inv[0..1]; W of cur into S_WCUR.
void launch_constraint_spectra(hipStream_t s, const FieldParams& F, const double2* cur,
                               double2* inv, Scratch sc);
void launch_field_energy(hipStream_t s, const FieldParams& F, const double2* cur, Scratch sc);
// max|f| and sum f^2 of two real arrays into (S_GMAX, S_GL2), (S_RMAX, S_RL2)
void launch_constraint_norms(hipStream_t s, int64_t ncell, const double* g, const double* r,
                             Scratch sc);
// scale-copy nb spectral fields: dst[b] = src[b] * scale
void launch_spec_copy(hipStream_t s, int64_t count, const double2* src, double2* dst, double scale);
// gbuf A0 slots <- A1 slots
void launch_accept_A(hipStream_t s, int64_t ncell, double* gbuf);
// gbuf A0 slots <- real A (3 x ncell)
void launch_set_A0(hipStream_t s, int64_t ncell, const double* A, double* gbuf);
void launch_fill(hipStream_t s, int64_t count, double* p, double value);
// zero slots first .. first + count - 1 and their spread copies
void launch_reset_slots(hipStream_t s, const Scratch& sc, int first, int count);

// ---- adjoint (adjoint.hip, mesh.hip) ----
struct AdjParticleArgs {
  Grid G;
  double dt, qm;       // time step, q/m
  int64_t np;
  const double* x;     // x^n, 3 x np
  const double* vb;    // vbar of the converged iterate, 3 x np
  const double* xi;    // adjoint of the push output (eta = qm xi), 3 x np
  const double* mu;    // (q/dV) x adjoint of J, 3 x ncell
  const double* gphi;  // grad_h phi^{n+1/2}, A^n, A^{n+1}: 3 x ncell each
  const double* A0;
  const double* A1;
  double* lx;          // accumulated per-particle adjoints of x, d, vbar (3 x np)
  double* ld;
  double* lvb;
  double* lgphi;       // push-side mesh adjoints (3 x ncell each), atomics
  double* lA0;
  double* lA1;
  double* bad;         // set to 1 if an orbit had too many pieces
};
// eta: push terms with xi (fast for cell-ordered particles: local chunks fit
// an LDS tile); mu: current terms
void launch_particle_adjoint(hipStream_t s, const AdjParticleArgs& P, bool eta, bool mu);
void launch_vbar(hipStream_t s, int64_t n3, const double* w, const double* v, double* vb);
void launch_adjoint_rhs(hipStream_t s, int64_t n3, double dt, const double* lx1, const double* lv1,
                        const double* lx, const double* ld, const double* lvb, double* b,
                        double* lxacc);
void launch_adjoint_update(hipStream_t s, int64_t n3, double dt, const double* b,
                           const double* lvb, const double* ld, const double* xi, double* xn,
                           double* red);
void launch_adjoint_out(hipStream_t s, int64_t n3, const double* lxacc, const double* lx,
                        const double* xi, const double* lv1, double* lx0, double* lv0);
// adjoint of k_cn; l1: next level's adjoint spectra (9, nullable); lg: gather
// fields' adjoint spectra [grad phi (3), A^{n+1} (3), A^n (3)] (nullable);
// lcur: current level's adjoint spectra, accumulated (nullable); lJh written
void launch_cn_adjoint(hipStream_t s, const FieldParams& F, const double2* l1, const double2* lg,
                       double2* lcur, double2* lJh);
// E, B spectra / ncell of a level (6 fields) and the energy adjoint from
// their scaled transforms (9 fields)
void launch_fields_EB(hipStream_t s, const Grid& G, const double2* cur, double2* EB);
void launch_energy_adjoint(hipStream_t s, const Grid& G, const double2* lEB, double2* lF);

constexpr int kGbufStride = 10;  // [gphi x,y,z | A^n x,y,z | A^{n+1} x,y,z | pad]

// ---- device microbenchmarks (measure.hip) ----
// FP64 flops of one launch of launch_fma_peak with `blocks` workgroups;
// out: one double per workgroup, never written in practice
double fma_peak_flops(int blocks);
void launch_fma_peak(hipStream_t s, int blocks, double* out);
// copy of n16 16-byte elements from src to dst (16-byte aligned, disjoint)
void launch_stream_copy(hipStream_t s, int blocks, const void* src, void* dst, int64_t n16);

}  // namespace ecpic
