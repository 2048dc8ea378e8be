/*
 * ecpic.h -- C ABI of the MI355X (gfx950) implementation of the
 * energy-conserving, unstaggered, Lorenz-gauge potential particle-in-cell step
 * of Christlieb, Chacon and Gong, "An Energy-Conserving Unstaggered
 * Electromagnetic-Potential Particle-in-Cell Method, Part I: Non-relativistic
 * Generalized-Momentum Formulation".
 *
 * Model (Sec. 2-3): periodic box, collocated nodes x_g = g H, potentials
 * (phi, psi = d_t phi, A, U = d_t A) advanced by Crank-Nicolson
 * (eq. cn-field-update) with Fourier derivatives (Sec. 3.3), charge advanced
 * from the orbit current by continuity (eq. cn-continuity), particles pushed in
 * canonical momentum with the orbit-discrete gradient (eq. orbit-push) inside
 * the Picard iteration of Algorithm 1.
 *
 * General rules of the ABI
 *   - Every function returns an ecpic_status.  Nothing aborts, nothing throws.
 *     ecpic_last_error() gives a thread-local message for the last non-OK status.
 *   - Device memory belongs to the caller.  ecpic_state_bytes() tells how much
 *     "state" (persistent between steps) and "workspace" (scratch) memory a
 *     simulation needs; the caller allocates both on the device (256-byte
 *     aligned) and hands them to ecpic_create().  The library never allocates or
 *     frees device memory; the one device array it holds is the fixed
 *     workspace of ecpic_adjoint_step_noalloc(), loaded with its code.  It
 *     allocates a small pinned host buffer for the per-iteration convergence
 *     read-back, and each simulation keeps up to two HIP graph executables
 *     of its cell sort (runtime objects, released by ecpic_destroy()).
 *   - All device work is enqueued on the HIP stream given to ecpic_create()
 *     (NULL = default stream).  Calls that return host data synchronise that
 *     stream; ecpic_picard_step() waits once per Picard iteration for the
 *     read-back of the two fixed-point errors (the next iteration's current
 *     may already be running behind it) and synchronises the stream before it
 *     returns.
 *   - Host arrays passed in are copied before the call returns; the library
 *     keeps no host pointer.
 *   - Array layouts.  Particle arrays are component-major (SoA): x[a*np + i].
 *     Mesh arrays are node arrays with node (ix, iy, iz) at flat index
 *     (ix*Ny + iy)*Nz + iz; vector fields store their 3 components one after
 *     the other (component-major).
 *   - Units are the nondimensional ones of Sec. 2; q and m are per macro-particle.
 */
#ifndef ECPIC_H
#define ECPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ECPIC_OK = 0,
  ECPIC_ENOCONV = 1,     /* warning: the step completed but Picard reached picard_max;
                            the last iterate is accepted (end of Algorithm 1) */
  ECPIC_EINVAL = -1,     /* invalid argument or configuration */
  ECPIC_ENOMEM = -2,     /* state/workspace too small, or pinned host allocation failed */
  ECPIC_EDEVICE = -3,    /* a HIP call failed */
  ECPIC_ENONFINITE = -4, /* a non-finite particle velocity or field appeared */
  ECPIC_ESTATE = -5      /* call out of order (e.g. a step before init) */
} ecpic_status;

typedef enum { ECPIC_FP64 = 0, ECPIC_MIXED = 1 } ecpic_precision;

typedef struct {
  int32_t n[3];                 /* mesh points per axis: powers of two, 4 <= n <= 256 */
  int32_t spline_degree;        /* r = 1 (linear B-spline, App. A/B), 2 (quadratic) or 3
                                   (cubic; Table 2's degrees) */
  double L[3];                  /* periodic box lengths; H_a = L_a / n_a */
  double kappa;                 /* nondimensional speed of light (Sec. 2.1) */
  double sigma1, sigma2;        /* source coefficients; must satisfy sigma1 = kappa^2 sigma2
                                   (eq. Maxwell_scaling), checked to 1e-13 relative */
  double dt;                    /* time step */
  double picard_tol;            /* tau: stop when both fixed-point errors are below it (p >= 1) */
  int32_t picard_max;           /* p_max: iterations p = 0..p_max (at most p_max+1 passes) */
  int32_t split_orbit_at_knots; /* 1: split orbit integrals at every crossed knot (Sec. 4.7);
                                   0: one Gauss rule over the whole orbit, each point with the
                                   stencil of its own cell (the paper's unsplit comparison
                                   runs; FP64 only, no adjoint) */
  int32_t quad_points;          /* Gauss-Legendre points, 0..16; 0 = smallest exact rule
                                   (2 n_q - 1 >= 3 r): 2, 4, 5 for r = 1, 2, 3.  Split pieces
                                   are polynomial, so every rule with at least that many
                                   points gives the same integrals and the smallest one is
                                   used; without splitting the given rule is used as is */
  int32_t precision;            /* ecpic_precision.  ECPIC_MIXED stores the particle state in
                                   FP32 (the cell of x^n and the FP32 offset inside it, v^n,
                                   v^{n-1}); iterates, orbit, field and energy arithmetic stay
                                   FP64, and the current is summed as int64 quanta.  The
                                   accepted velocity is rounded to one of its two neighbouring
                                   FP32 values without bias (up with probability equal to its
                                   distance from the lower one), from a counter-based generator
                                   keyed by the particle's stored state and the step, so a run
                                   is deterministic and independent of the particle order */
  double fixed_point_scale;     /* mixed precision: current quantum is 1/fixed_point_scale of
                                   the per-particle charge unit (0 = 2^40) */
  int32_t diagnostics;          /* 1: after each accepted step run the consistency sweep
                                   (R_particle, R_A, partition of unity) */
  int32_t sort_interval;        /* particles are re-sorted by mesh cell at the start of every
                                   k-th step: 0 or 1 = every step, k > 1 = every k steps,
                                   -1 = never (results are the same up to rounding) */
  int32_t anderson_depth;       /* 0: the Picard iteration of Algorithm 1.  m = 1..4: Anderson
                                   mixing of the iterates over the last m passes (Walker and
                                   Ni 2011, mixing parameter 1): with w_p the iterate
                                   v^{n+1,p}, g_p = G(w_p) the velocity the pass returns and
                                   f = g - w, the next iterate is g_p - sum_j gamma_j
                                   (g_{p-j+1} - g_{p-j}), gamma minimising
                                   |f_p - sum_j gamma_j (f_{p-j+1} - f_{p-j})|_2 over
                                   j = 1..min(m, p).  The stopping test, the accepted
                                   iterate and the converged equations are those of
                                   Algorithm 1; energy conservation holds at convergence
                                   whatever the solver (Sec. 4, Picard iteration of the
                                   experiments; Anderson acceleration is the paper's future
                                   work, Sec. 6).  Costs 2 m more 3 x np FP64 arrays of state.
                                   In mixed precision the mixing coefficients are FP64 sums
                                   over the particles, so with m > 0 the step is no longer
                                   bitwise independent of the particle order. */
  int32_t scatter_chunk;        /* cell-sorted particles per block of the current scatter:
                                   0 = automatic (4096, switched to 2048 for good once more
                                   than 1% of a step's chunks overflow the LDS tile; 2048 for
                                   r = 3), or 2048, or 4096 for r <= 2.  Results are the same
                                   up to the order of the FP64 atomic additions. */
} ecpic_config;

typedef struct {
  int32_t iters;     /* Picard passes executed (p + 1) */
  int32_t converged; /* 1 if both errors fell below picard_tol */
  double err_v;      /* max_i |v^{p+1} - v^p|_inf / max_i |v^{p+1}|_inf */
  double err_J;      /* max_g |J^p - J^{p-1}|_inf / J_s, J_s = sum_i |q| |vbar_i|_inf / |Omega| */
} ecpic_step_info;

typedef struct {
  double K, W, E_total;              /* eqs. particle-energy, field-energy, total-discrete-energy */
  double R_field, R_particle, R_total; /* eqs. R-field, R-particle, R-total of the last step */
  double gauge_max, gauge_l2;        /* G_h = psi/kappa^2 + div_h A (eq. gauge-diagnostic) */
  double gauss_max, gauss_l2;        /* R_h = div_h E - sigma1 rho (eq. gauss-diagnostic) */
  double RA_rms, RA_max;             /* chain-rule residual R_A (eq. RA-test), last step */
  double pou_max;                    /* max_i |sum_g Sbar_ig - 1| (App. A), last step */
  double JE_mesh;                    /* sum_g J^{n+1/2} . E^{n+1/2} dV of the last step */
  double work_particle;              /* sum_i q vbar_i . Ebar_i of the last step */
  int64_t step;                      /* number of accepted steps */
} ecpic_energy;

typedef struct ecpic_sim ecpic_sim;

/* Bytes of device state and workspace for this configuration and particle
   count (0 <= n_particles <= 2^31 - 1: particle ids and cell offsets are
   32-bit).  Returns ECPIC_EINVAL for an invalid configuration or count. */
ecpic_status ecpic_state_bytes(const ecpic_config* cfg, int64_t n_particles, size_t* state_bytes,
                               size_t* workspace_bytes);

/* Create a simulation over caller-owned device buffers (sizes from
   ecpic_state_bytes, 256-byte aligned).  hip_stream is a hipStream_t or NULL.
   The buffers must stay valid until ecpic_destroy(). */
ecpic_status ecpic_create(const ecpic_config* cfg, int64_t n_particles, void* state_dev,
                          size_t state_bytes, void* workspace_dev, size_t workspace_bytes,
                          void* hip_stream, ecpic_sim** out);

void ecpic_destroy(ecpic_sim* sim);

/* Initial state of Sec. 5.4: host positions x and velocities v (3*np each,
   component-major); positions are wrapped into the box.  rho^0 is the
   point-shape charge deposit (eq. source-moments) plus a uniform background
   n0, mean removed and zeroed on every mode whose Fourier symbol vanishes;
   phi^0 solves -Delta_h phi = sigma1 rho; psi = A = U = 0; P = m v;
   v^{-1} = v^0. */
ecpic_status ecpic_init_particles(ecpic_sim* sim, const double* x, const double* v, double q,
                                  double m, double n0);

/* As ecpic_init_particles with several particle species (the model gives
   every particle its own charge q_i and mass m_i, Sec. 2): particle i (host
   arrays in the caller's order) has charge q[species[i]] and mass
   m[species[i]].  nspecies in [1, 4]; q[s] finite and non-zero, m[s] > 0;
   every species[i] in [0, nspecies), else ECPIC_EINVAL and nothing changes.
   rho^0 = sum_i q_i S_g(x_i) / dV, P_i = m_i v_i.  With more than one species
   the state holds one byte per particle for it; the adjoint takes one species
   only.  In mixed precision the current quanta are those of q[0]: a
   contribution of species s is quantised as (q[s] / q[0]) vbar Sbar. */
ecpic_status ecpic_init_species(ecpic_sim* sim, const double* x, const double* v,
                                const int32_t* species, int32_t nspecies, const double* q,
                                const double* m, double n0);

/* One time step by Algorithm 1: extrapolated guess, then per Picard pass the
   orbit current (eq. orbit-current), continuity and CN solve, orbit gather and
   orbit-discrete-gradient push (eq. orbit-push); stop when both fixed-point
   errors are below tau (p >= 1) or at p_max.  Returns ECPIC_OK, or
   ECPIC_ENOCONV when p_max was reached (the step is still taken).  Errors
   (the step is not taken): ECPIC_ENONFINITE for a non-finite velocity or
   current; ECPIC_EINVAL for an orbit crossing more than 63 knots in one step
   or, in mixed precision, a particle whose |q_s / q_0| |vbar_l|
   fixed_point_scale reaches 2^50 (the range of the rounding to quanta). */
ecpic_status ecpic_picard_step(ecpic_sim* sim, ecpic_step_info* info);

/* Continuity + CN field update alone (eqs. cn-continuity, cn-field-update)
   with a caller current J^{n+1/2} (device, 3*ncell, component-major), or the
   current of the last accepted step when J_dev is NULL.  Advances the mesh
   state one level; particles are not touched. */
ecpic_status ecpic_field_solve(ecpic_sim* sim, const double* J_dev);

/* Energies and constraint residuals of the current state, and the balance
   terms of the last step (Sec. 5.1-5.3).  R_particle, RA_* and pou_max need
   diagnostics = 1 in the configuration (they are zero otherwise). */
ecpic_status ecpic_energy_diagnostics(ecpic_sim* sim, ecpic_energy* out);

/* Copy state to caller buffers (any may be NULL): x, v, v^{n-1} (3*np each) and
   real-space mesh fields (9*ncell: phi, psi, Ax, Ay, Az, Ux, Uy, Uz, rho).
   Host or device memory: the copy direction follows from the pointers
   (unified addressing).  Returns after the copies are complete. */
ecpic_status ecpic_get_state(ecpic_sim* sim, double* x, double* v, double* vprev,
                             double* fields);

/* Replace the state from caller buffers, host or device (same layout as
   ecpic_get_state; any may be NULL to keep the current value).  m > 0: every particle gets charge q and
   mass m (one species); m = 0: every particle keeps its species (q ignored;
   ECPIC_ESTATE before the first initialisation).  The fields pass through
   real space, so a state read and written back differs from the original at
   rounding level.  The balance terms of the last step (R_*, JE_mesh,
   work_particle, RA_*, pou_max) are cleared; the step counter, which sets the
   sort schedule, is kept. */
ecpic_status ecpic_set_state(ecpic_sim* sim, const double* x, const double* v,
                             const double* vprev, const double* fields, double q, double m);

/* Checkpoint and restart: a byte-exact copy of the simulation's state (the
   caller's state buffer, the live arrangement of its particle stores, the
   step counter and energy bookkeeping) in a host buffer of
   ecpic_checkpoint_bytes() bytes, owned by the caller.  A simulation created
   with the same configuration and particle count (and this library version)
   and restored from it continues exactly as the saved one would: bitwise in
   the mixed form, whose current is an exact integer sum, and up to the order
   of the FP64 atomic additions in the FP64 form.  Restore: ECPIC_EINVAL for a
   buffer that is not a checkpoint of this configuration and version. */
ecpic_status ecpic_checkpoint_bytes(ecpic_sim* sim, size_t* bytes);
ecpic_status ecpic_checkpoint_save(ecpic_sim* sim, void* host_dst);
ecpic_status ecpic_checkpoint_restore(ecpic_sim* sim, const void* host_src);

/* Orbit current J^{n+1/2} (3*ncell) of the last accepted step, to host. */
ecpic_status ecpic_get_current(ecpic_sim* sim, double* J);

/* Kernel-level entry points (device pointers, no simulation object): the
   orbit integrals of n independent particles against given mesh fields, for
   checking the particle kernels in isolation.
     x0, d      3*n component-major: start positions (inside the box) and
                unwrapped displacements of straight orbits x(s) = x0 + s d
     gphi, U, A0, A1   3*ncell each (real-space node fields)
     out        24*n, particle-major: [0:3] sum_g gphi_g Sbar_g, [3:6] sum_g U_g Sbar_g,
                [6:15] D (row l = component of A, column j = derivative) per
                eq. DA-def with A_g(s) = (1-s) A0 + s A1, [15:18] A1_h(x0+d),
                [18:21] A0_h(x0), [21] sum_g Sbar_g, [22] number of orbit pieces
   and the orbit current of n particles, accumulated into J (3*ncell):
     J_g += qv_i Sbar_ig / dV   (qv: 3*n component-major, q_i vbar_i)   */
ecpic_status ecpic_orbit_gather(const ecpic_config* cfg, int64_t n, const double* x0,
                                const double* d, const double* gphi, const double* U,
                                const double* A0, const double* A1, double* out,
                                void* hip_stream);
ecpic_status ecpic_orbit_deposit(const ecpic_config* cfg, int64_t n, const double* x0,
                                 const double* d, const double* qv, double* J, void* hip_stream);

/* Kernel timing.  level 1: ecpic_picard_step() records HIP events on the
   simulation's stream around each phase of every Picard pass and accumulates
   the elapsed times (milliseconds) and launch counts per phase:
     0 orbit current scatter, 1 field solve (forward FFT, continuity + CN,
     inverse FFT), 2 orbit gather + push, 3 consistency sweep, 4 end-of-step
     update, 5 whole steps (host wall clock from entry to return).
   level 2: phases 2 and 5 only (two events per pass instead of four; each
   event between two kernels costs a few microseconds of idle GPU).
   level 0 turns timing off; other levels are ECPIC_EINVAL.
   pieces: total orbit pieces summed over particles and gather launches, so
   that pieces / (np * launches[2]) is the mean number of pieces per orbit.
   scatter_chunk: particles per block the current scatter uses now (set at
   every level, 0 included; see ecpic_config.scatter_chunk).
   Setting a level resets the counters. */
typedef struct {
  double ms[8];
  int64_t launches[8];
  double pieces;
  int32_t scatter_chunk;
  int32_t reserved;
} ecpic_profile;

ecpic_status ecpic_set_profiling(ecpic_sim* sim, int32_t level);
ecpic_status ecpic_get_profile(ecpic_sim* sim, ecpic_profile* out);

/* ---- Differentiation: adjoint of one converged step --------------------
   The converged step of Algorithm 1 maps the level-n state (x, v, fields) to
   the level-(n+1) state through the solution w = v^{n+1} of the implicit
   push (eq. orbit-push with P^n rebuilt by eq. discrete-canonical-relation,
   the orbit current of eq. orbit-current, and eqs. cn-continuity and
   cn-field-update).  ecpic_adjoint_step() applies the transpose of that
   map's Jacobian (implicit-function form, solved by the transposed Picard
   iteration xi = b + (dG/dw)^T xi, which contracts like the forward one):
   given the adjoints of x^{n+1}, v^{n+1} and the level-(n+1) fields it
   returns those of x^n, v^n and the level-n fields.  v^{n-1} only sets the
   first guess of the iteration, so the converged step does not depend on it.
   Requirements: precision ECPIC_FP64, spline_degree 2 (with degree 1 the
   derivative of the piecewise-constant shape gradient jumps at knots),
   split_orbit_at_knots 1.

   Device pointers, FP64, particles in the caller's order, on the simulation's
   stream (the call returns after the stream is synchronised):
     x, v, w      3*np component-major: x^n (inside the box), v^n, and the
                  converged v^{n+1} of the step from this state
     fields       9*ncell: level-n fields (layout of ecpic_get_state)
     lx1, lv1     3*np adjoints of x^{n+1} and v^{n+1}; NULL = zero
     lF1          9*ncell adjoint of the level-(n+1) fields; NULL = zero
     lx0, lv0     3*np outputs: adjoints of x^n and v^n
     lF0          9*ncell output: adjoint of the level-n fields
     tol          stop when max|xi^{k+1} - xi^k| <= tol max|xi^{k+1}|
     max_iters    iteration bound (ECPIC_ENOCONV if reached; outputs still set)
   workspace: caller-owned device buffer of ecpic_adjoint_workspace_bytes()
   bytes (256-byte aligned; 372 B per particle plus the mesh arrays).
   Inside the call the particles are sorted by cell (the kernels work on
   local chunks); the outputs come back in the caller's order.  The
   simulation's own state is not changed; its scratch is reused. */
typedef struct {
  int32_t iters;     /* transposed Picard iterations */
  int32_t converged; /* 1 if tol was reached */
  double err;        /* last max|xi^{k+1} - xi^k| / max|xi^{k+1}| */
} ecpic_adjoint_info;

ecpic_status ecpic_adjoint_workspace_bytes(const ecpic_config* cfg, int64_t n_particles,
                                           size_t* bytes);
ecpic_status ecpic_adjoint_step(ecpic_sim* sim, void* workspace, size_t workspace_bytes,
                                const double* x, const double* v, const double* w,
                                const double* fields, const double* lx1, const double* lv1,
                                const double* lF1, double* lx0, double* lv0, double* lF0,
                                double tol, int32_t max_iters, ecpic_adjoint_info* info);

/* Allocation-free variant of ecpic_adjoint_step, for callers that cannot
   allocate device memory or take a caller workspace (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc).  Same
   arguments, requirements, results and status codes as ecpic_adjoint_step
   without the workspace pair: the workspace is a device array inside the
   library, ECPIC_STATIC_SCRATCH_BYTES (64 MiB) on every GPU the library runs
   on, held from the first ecpic_create() on that GPU until the process ends.
   The call allocates nothing (no hipMalloc, hipFree or allocating library
   routine).
     - ECPIC_ENOMEM if ecpic_adjoint_workspace_bytes() of this simulation
       exceeds ECPIC_STATIC_SCRATCH_BYTES (about 76,000 particles on a 32^3
       mesh, 167,000 on 16^3); nothing is run.
     - ECPIC_EINVAL if the device current at ecpic_create() is not current.
   Every call on one GPU uses that GPU's one array and leaves its contents
   behind (each call writes every part it reads before reading it): calls
   that overlap in time on one GPU, from other threads or on other streams,
   race on it, and the caller must serialise them. */
#define ECPIC_STATIC_SCRATCH_BYTES ((size_t)64 << 20)
ecpic_status ecpic_adjoint_step_noalloc(ecpic_sim* sim, const double* x, const double* v,
                                        const double* w, const double* fields, const double* lx1,
                                        const double* lv1, const double* lF1, double* lx0,
                                        double* lv0, double* lF0, double tol, int32_t max_iters,
                                        ecpic_adjoint_info* info);

/* Gradient of the field energy W (eq. field-energy) of the present state with
   respect to its real-space fields: device output, 9*ncell (layout of
   ecpic_get_state; the psi and rho rows are zero). */
ecpic_status ecpic_field_energy_grad(ecpic_sim* sim, double* lF);

/* Measured peaks of the current device, the rates that the particle kernels'
   roofline is stated against beside the published ones (not a step of the
   method).  No simulation object.
     buffer, bytes  caller-owned device memory of at least 64 MiB, contents
                    overwritten (its first half is copied into its second;
                    give several GiB so that the copy exceeds the caches)
     repeats        timed launches per figure (>= 1), after one untimed
     hip_stream     a hipStream_t or NULL; synchronised
     fp64_tflops    out: FP64 TFLOP/s (2 per FMA) of a kernel whose every lane
                    runs 8 independent FMA chains on registers, 32 workgroups
                    of 256 lanes per compute unit; the best launch
     hbm_gbs        out: bytes read plus bytes written per second (1e9 B/s)
                    of a 16-byte-per-lane streaming copy; the best launch
   Errors: ECPIC_EINVAL for a null pointer, bytes below 64 MiB or repeats
   below 1; ECPIC_EDEVICE on a HIP failure. */
ecpic_status ecpic_measure_peaks(void* buffer, size_t bytes, int32_t repeats, void* hip_stream,
                                 double* fp64_tflops, double* hbm_gbs);

/* Message for the last non-OK status of this thread ("" if none). */
const char* ecpic_last_error(void);

/* Library version string. */
const char* ecpic_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ECPIC_H */
