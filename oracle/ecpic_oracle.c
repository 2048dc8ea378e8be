/*
 * ecpic_oracle.c -- plain serial FP64 CPU oracle.  TEST INFRASTRUCTURE ONLY.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark load this file.  The product path (the HIP library) never calls
 * it, includes it, or shares any code, table or constant with it.
 *
 * What it computes is the time step of the energy-conserving, unstaggered,
 * Lorenz-gauge potential PIC method of Christlieb, Chacon and Gong,
 * "An Energy-Conserving Unstaggered Electromagnetic-Potential Particle-in-Cell
 * Method, Part I":
 *
 *   shapes      B-spline particle shapes S_g on a collocated periodic mesh
 *               (Sec. 2.3, eq. Ah-mesh)
 *   orbit       straight unwrapped orbit and knot-crossing breakpoints
 *               (Sec. 4.2 eq. particle-orbit; Sec. 4.7 eq. breakpoint-set)
 *   weights     split orbit integrals S-bar and D (eqs. split-Sbar, split-DA):
 *               closed forms of App. A / App. B for degree 1, Gauss-Legendre
 *               per segment otherwise (Sec. 4.7, 2 n_q - 1 >= 3 r)
 *   deposit     orbit current (eq. orbit-current)
 *   fields      continuity update (eq. cn-continuity) and Crank-Nicolson
 *               potential update (eq. cn-field-update) with Fourier symbols
 *               (Sec. 3.3), evaluated with a plain separable DFT
 *   push        orbit-discrete-gradient canonical-momentum push (eq. orbit-push)
 *   step        Picard iteration of Algorithm 1, optionally with Anderson
 *               mixing of the iterates (an extension: the conservation
 *               statement concerns the converged discrete equations, not the
 *               nonlinear solver, Sec. 4 "Picard iteration used in the
 *               numerical experiments"; Anderson acceleration is the paper's
 *               named future work, Sec. 6)
 *   diagnostics K, W (eqs. particle-energy, field-energy), R_field, R_particle,
 *               R_total (Sec. 5.3), gauge/Gauss residuals (Sec. 5.1),
 *               chain-rule residual R_A (Sec. 5.2)
 *
 * Everything is double precision, no blocking or fusion: one particle at a
 * time, one segment at a time, one stencil node at a time.
 *
 * Readings where the paper leaves a choice open (each listed in the design
 * notes of the repository):
 *   - every field and every spline degree live on nodes x_g = g H; degrees 1
 *     and 3 use the cell floor(x/H), degree 2 the nearest node floor(x/H + 1/2);
 *   - the first-derivative Fourier symbol is zero on the Nyquist index and the
 *     Laplacian symbol is -|k~|^2 with that same k~ (keeps curl curl =
 *     grad div - Laplacian exact);
 *   - the stencil of a split segment is the one of the knot interval it lies
 *     in, found from x0's side of the knots along the motion and the knots
 *     crossed so far (not from a rounded midpoint); along a still axis, the
 *     interval holding x0, closed below;
 *   - the initial charge is also zeroed on every mode where k~ = 0;
 *   - v^{n-1} := v^0 at the first step;
 *   - Picard errors: e_v = max|v^{p+1}-v^p| / max|v^{p+1}|,
 *     e_J = max|J^p - J^{p-1}| / J_s with J_s = sum_i |q_i| max_a|vbar_ia| / |Omega|;
 *     at most p_max + 1 iterations, stop only for p >= 1;
 *   - diagnostics of a step use the accepted iterate's orbit, current and fields.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

#define ORC_MAX_ANDERSON 4

/* ------------------------------------------------------------------------- */
/* configuration and state                                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
  int32_t n[3];      /* mesh points per axis */
  double L[3];       /* periodic box lengths */
  double kappa;      /* nondimensional speed of light */
  double sigma1;     /* source coefficient of the phi equation */
  double sigma2;     /* source coefficient of the A equation */
  double dt;
  int32_t r;         /* spline degree: 1, 2 or 3 */
  int32_t split;     /* 1: split every orbit integral at crossed knots; 0: one rule over [0,1] */
  int32_t nq;        /* Gauss points per segment, 0: smallest exact rule (2 nq - 1 >= 3 r) */
  int32_t analytic;  /* degree 1 with splitting: 1 = App. A/B closed forms, 0 = Gauss */
  double tol;        /* Picard tolerance */
  int32_t pmax;      /* Picard iterations p = 0..pmax */
  int32_t anderson;  /* Anderson depth m (0: the plain Picard iteration of Algorithm 1) */
} orc_cfg;

typedef struct {
  int32_t iters;
  int32_t converged;
  double err_v, err_J;
} orc_step_info;

typedef struct {
  double K, W, E_total;
  double R_field, R_particle, R_total;
  double gauge_max, gauge_l2, gauss_max, gauss_l2;
  double RA_rms, RA_max, pou_max;
  double JE_mesh;       /* sum_g J.E^{n+1/2} dV of the accepted iterate */
  double work_particle; /* sum_i q vbar.Ebar of the accepted iterate */
  int64_t step;
} orc_energy;

typedef struct {
  int n[3];
  double L[3], H[3], dV, vol;
  int64_t ncell;
} grid;

typedef struct {
  orc_cfg c;
  grid G;
  int nq;
  double gx[64], gw[64];     /* Gauss-Legendre nodes/weights on [-1, 1] */
  int64_t np;
  double q, m;               /* the species of a one-species run (and of the adjoint) */
  double *qi, *mi;           /* charge and mass of every particle (np each) */
  int one_species;           /* 1 when every particle carries (q, m) */
  double *x, *v, *vprev, *P; /* 3*np each, component-major: x[a*np + i] */
  cplx *phi, *psi, *A, *U, *rho; /* Fourier state, A and U hold 3 components */
  double *J;                 /* real-space current of the accepted iterate (3*ncell) */
  orc_energy en;
  double K0, W0;
  int have_energy;
  /* optional record of the Picard passes of the next steps (tests): iterate
     w_p and image G(w_p) of pass p at trace_w/g + 3 np p, passes < trace_max */
  double *trace_w, *trace_g;
  int trace_max;
} orc_sim;

/* ------------------------------------------------------------------------- */
/* small helpers                                                             */
/* ------------------------------------------------------------------------- */

static void make_grid(const orc_cfg* c, grid* G) {
  G->ncell = 1;
  for (int a = 0; a < 3; ++a) {
    G->n[a] = c->n[a];
    G->L[a] = c->L[a];
    G->H[a] = c->L[a] / c->n[a];
    G->ncell *= c->n[a];
  }
  G->dV = G->H[0] * G->H[1] * G->H[2];
  G->vol = G->L[0] * G->L[1] * G->L[2];
}

static long wrap_index(long i, int n) {
  long r = i % n;
  return r < 0 ? r + n : r;
}

static int64_t node_id(const grid* G, long ix, long iy, long iz) {
  return ((int64_t)wrap_index(ix, G->n[0]) * G->n[1] + wrap_index(iy, G->n[1])) * G->n[2] +
         wrap_index(iz, G->n[2]);
}

/* position wrapped into the periodic box (used only where a point shape is
   evaluated at the end of an orbit, and when a step is accepted) */
static double wrap_pos(double x, double L) {
  double w = x - L * floor(x / L);
  if (w < 0) w += L;
  if (w >= L) w -= L;
  return w;
}

/* Gauss-Legendre rule on [-1,1]: Newton iteration on the Legendre polynomial
   P_n, evaluated by the three-term recurrence (k+1)P_{k+1} = (2k+1) x P_k - k P_{k-1}. */
static void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-17) break;
    }
    /* recompute the derivative at the converged node */
    {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < n; ++k) {
        double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1.0; }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = -z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

/* ------------------------------------------------------------------------- */
/* B-spline shapes (Sec. 2.3; degree r centred B-spline per axis)            */
/* ------------------------------------------------------------------------- */

/* index of the node the local polynomial pieces are written against:
   odd degree (knots on the nodes) -> the cell's left node floor(u);
   degree 2 (knots between nodes) -> the nearest node */
static long spline_base(int r, double u) { return r == 2 ? (long)floor(u + 0.5) : (long)floor(u); }

/* first stencil node relative to the base */
static long spline_first(int r, long base) { return r == 1 ? base : base - 1; }

/* weights w[o] and derivatives dw[o] (per unit of u) of the stencil nodes
   first+o, for local coordinate t = u - base.  Degree 1: M1(xi) = 1 - |xi|.
   Degree 2: M2(xi) = 3/4 - xi^2 (|xi| <= 1/2), (3/2 - |xi|)^2 / 2 (1/2 <= |xi| <= 3/2).
   Degree 3: M3(xi) = 2/3 - xi^2 + |xi|^3 / 2 (|xi| <= 1), (2 - |xi|)^3 / 6 (1 <= |xi| <= 2). */
static void spline_pieces(int r, double t, double* w, double* dw) {
  if (r == 3) {
    double u = 1.0 - t;
    w[0] = u * u * u / 6.0;                    /* node base-1, xi = t + 1 */
    w[1] = 2.0 / 3.0 - t * t + 0.5 * t * t * t; /* node base,   xi = t     */
    w[2] = 2.0 / 3.0 - u * u + 0.5 * u * u * u; /* node base+1, |xi| = 1 - t */
    w[3] = t * t * t / 6.0;                    /* node base+2, |xi| = 2 - t */
    dw[0] = -0.5 * u * u;
    dw[1] = -2.0 * t + 1.5 * t * t;
    dw[2] = 2.0 * u - 1.5 * u * u;
    dw[3] = 0.5 * t * t;
    return;
  }
  if (r == 1) {
    w[0] = 1.0 - t;  /* node base,   xi = t     */
    w[1] = t;        /* node base+1, xi = t - 1 */
    dw[0] = -1.0;
    dw[1] = 1.0;
  } else {
    w[0] = 0.5 * (0.5 - t) * (0.5 - t); /* node base-1, xi = t + 1 */
    w[1] = 0.75 - t * t;                /* node base,   xi = t     */
    w[2] = 0.5 * (0.5 + t) * (0.5 + t); /* node base+1, xi = t - 1 */
    dw[0] = -(0.5 - t);
    dw[1] = -2.0 * t;
    dw[2] = 0.5 + t;
  }
}

/* ------------------------------------------------------------------------- */
/* orbit segments (Sec. 4.7, eq. breakpoint-set)                             */
/* ------------------------------------------------------------------------- */

static int cmp_double(const void* a, const void* b) {
  double x = *(const double*)a, y = *(const double*)b;
  return (x > y) - (x < y);
}

#define MAX_BREAKS 512

/* sorted, de-duplicated breakpoints 0 = s_0 < ... < s_M = 1 of the orbit
   x(s) = x0 + s d.  Knots sit at k H (degrees 1, 3) and (k + 1/2) H (degree 2).
   Returns the number of breakpoints, or -1 if the orbit is absurdly long. */
static int orbit_breakpoints(const grid* G, int r, const double x0[3], const double d[3],
                             double* s) {
  int ns = 0;
  s[ns++] = 0.0;
  s[ns++] = 1.0;
  double off = (r == 2) ? 0.5 : 0.0;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) continue; /* no breakpoints from a coordinate that does not move */
    double H = G->H[a];
    double u0 = x0[a] / H, u1 = (x0[a] + d[a]) / H;
    long klo = (long)floor(fmin(u0, u1) - off) - 1;
    long khi = (long)floor(fmax(u0, u1) - off) + 1;
    for (long k = klo; k <= khi; ++k) {
      double xi = ((double)k + off) * H;
      double sk = (xi - x0[a]) / d[a];
      if (sk > 0.0 && sk < 1.0) {
        if (ns >= MAX_BREAKS) return -1;
        s[ns++] = sk;
      }
    }
  }
  qsort(s, ns, sizeof(double), cmp_double);
  int m = 1;
  for (int i = 1; i < ns; ++i)
    if (s[i] != s[m - 1]) s[m++] = s[i];
  return m;
}

/* Base node per axis of the stencil of the piece of x(s) = x0 + s d that
   starts at the breakpoint s0 (Sec. 4.7): the piece lies inside one knot
   interval per axis, and the stencil is that interval's.  Along a moving axis
   the orbit enters, from x0 and in its direction of motion, the interval
   behind the first knot xi_k = (k + off) H with xi_k ahead of x0 (decided by
   comparing the two positions, so an orbit that starts on a knot takes the
   side it moves to however short its step), then one interval further for
   every knot of that axis crossed at a breakpoint (xi_k - x0) / d <= s0 (the
   values orbit_breakpoints produces).  A still axis takes the interval holding
   x0, closed below: the one behind the first knot above x0. */
static void piece_bases(const grid* G, int r, const double x0[3], const double d[3], double s0,
                        long base[3]) {
  double off = (r == 2) ? 0.5 : 0.0;
  for (int a = 0; a < 3; ++a) {
    double H = G->H[a];
    long k = (long)floor(x0[a] / H - off);
    long b;
    int dir;
    if (d[a] >= 0.0) { /* first knot above x0; the interval below it */
      k -= 2;
      while (((double)k + off) * H <= x0[a]) ++k;
      b = spline_base(r, (double)k - 0.5 + off);
      dir = 1;
    } else { /* first knot below x0; the interval above it */
      k += 3;
      while (((double)k + off) * H >= x0[a]) --k;
      b = spline_base(r, (double)k + 0.5 + off);
      dir = -1;
    }
    for (long j = k; d[a] != 0.0; j += dir) {
      double sk = (((double)j + off) * H - x0[a]) / d[a];
      if (!(sk <= s0)) break;
      b += dir;
    }
    base[a] = b;
  }
}

/* Integrals of one orbit piece against its stencil (at most 4x4x4 nodes):
     Iw[nu]   = int S_nu(x(s)) ds
     X[j][nu] = int d_j S_nu(x(s)) ds
     Y[j][nu] = int (s - s0) d_j S_nu(x(s)) ds
   so that, with A_g(s) = A^(m) + C (s - s0) (App. B),
     int A_g(s) d_j S_g ds = A^(m) X + C Y. */
typedef struct {
  long first[3];
  int w; /* stencil width r + 1 */
  double s0;
  double Iw[64];
  double X[3][64];
  double Y[3][64];
} piece;

static int pidx(int w, int i, int j, int k) { return (i * w + j) * w + k; }

/* App. A and App. B closed forms for degree 1 on the segment [s0, s1] */
static void piece_r1_analytic(const grid* G, const double x0[3], const double d[3], double s0,
                              double s1, const long pb[3], piece* o) {
  double h = s1 - s0;
  double lam[3][2], mu[3][2];
  o->w = 2;
  o->s0 = s0;
  for (int a = 0; a < 3; ++a) {
    double H = G->H[a];
    long base = pb[a];
    o->first[a] = spline_first(1, base);
    double rm = (x0[a] + s0 * d[a]) / H - (double)base; /* r_{alpha,m} */
    double beta = d[a] / H;                             /* beta_alpha  */
    lam[a][0] = 1.0 - rm;
    mu[a][0] = -beta;
    lam[a][1] = rm;
    mu[a][1] = beta;
  }
  double h2 = h * h, h3 = h2 * h, h4 = h3 * h;
  for (int nx = 0; nx < 2; ++nx)
    for (int ny = 0; ny < 2; ++ny)
      for (int nz = 0; nz < 2; ++nz) {
        int nu[3] = {nx, ny, nz};
        double Lc[3], Mc[3];
        for (int a = 0; a < 3; ++a) {
          Lc[a] = lam[a][nu[a]];
          Mc[a] = mu[a][nu[a]];
        }
        int id = pidx(2, nx, ny, nz);
        double c0 = Lc[0] * Lc[1] * Lc[2];
        double c1 = Mc[0] * Lc[1] * Lc[2] + Lc[0] * Mc[1] * Lc[2] + Lc[0] * Lc[1] * Mc[2];
        double c2 = Mc[0] * Mc[1] * Lc[2] + Mc[0] * Lc[1] * Mc[2] + Lc[0] * Mc[1] * Mc[2];
        double c3 = Mc[0] * Mc[1] * Mc[2];
        o->Iw[id] = c0 * h + c1 / 2.0 * h2 + c2 / 3.0 * h3 + c3 / 4.0 * h4;
        for (int j = 0; j < 3; ++j) {
          int p = (j + 1) % 3, q = (j + 2) % 3;
          double sig = nu[j] ? 1.0 : -1.0;
          double d0 = Lc[p] * Lc[q];
          double d1 = Mc[p] * Lc[q] + Lc[p] * Mc[q];
          double d2 = Mc[p] * Mc[q];
          o->X[j][id] = sig / G->H[j] * (d0 * h + d1 / 2.0 * h2 + d2 / 3.0 * h3);
          o->Y[j][id] = sig / G->H[j] * (d0 / 2.0 * h2 + d1 / 3.0 * h3 + d2 / 4.0 * h4);
        }
      }
}

/* Empty piece against the polynomial pieces of the given base nodes,
   with A_g(s) written relative to s0. */
static void piece_init(int r, const long base[3], double s0, piece* o) {
  o->w = r + 1;
  o->s0 = s0;
  for (int a = 0; a < 3; ++a) o->first[a] = spline_first(r, base[a]);
  memset(o->Iw, 0, sizeof(o->Iw));
  memset(o->X, 0, sizeof(o->X));
  memset(o->Y, 0, sizeof(o->Y));
}

/* add one quadrature point s with weight wt to a piece */
static void piece_add_point(const grid* G, int r, const double x0[3], const double d[3], double s,
                            double wt, const long base[3], piece* o) {
  int w = r + 1;
  double eta = s - o->s0;
  double wv[3][4], dwv[3][4];
  for (int a = 0; a < 3; ++a) {
    double u = (x0[a] + s * d[a]) / G->H[a];
    spline_pieces(r, u - (double)base[a], wv[a], dwv[a]);
    for (int o2 = 0; o2 < w; ++o2) dwv[a][o2] /= G->H[a];
  }
  for (int i = 0; i < w; ++i)
    for (int j = 0; j < w; ++j)
      for (int k = 0; k < w; ++k) {
        int id = pidx(w, i, j, k);
        double S = wv[0][i] * wv[1][j] * wv[2][k];
        double dS[3] = {dwv[0][i] * wv[1][j] * wv[2][k], wv[0][i] * dwv[1][j] * wv[2][k],
                        wv[0][i] * wv[1][j] * dwv[2][k]};
        o->Iw[id] += wt * S;
        for (int jj = 0; jj < 3; ++jj) {
          o->X[jj][id] += wt * dS[jj];
          o->Y[jj][id] += wt * eta * dS[jj];
        }
      }
}

/* Gauss-Legendre rule (nodes gx, weights gw on [-1,1]) mapped to [s0, s1]
   and evaluated against the polynomial pieces of the given base nodes. */
static void piece_gauss(const grid* G, int r, const double x0[3], const double d[3], double s0,
                        double s1, const long base[3], int nq, const double* gx,
                        const double* gw, piece* o) {
  double h = s1 - s0;
  piece_init(r, base, s0, o);
  for (int iq = 0; iq < nq; ++iq)
    piece_add_point(G, r, x0, d, s0 + 0.5 * h * (1.0 + gx[iq]), 0.5 * h * gw[iq], base, o);
}

/* All pieces of one orbit.  With splitting: one piece per segment, its stencil
   that of the knot interval the segment lies in (piece_bases).  Without splitting: the n_q-point rule over
   [0,1], each quadrature point with the stencil of its own cell (one piece per
   point, written relative to s = 0).  Returns the number of pieces (or -1). */
static int orbit_pieces(const orc_sim* S, const double x0[3], const double d[3], piece* out,
                        int cap) {
  const grid* G = &S->G;
  int r = S->c.r;
  if (!S->c.split) {
    if (S->nq > cap) return -1;
    for (int iq = 0; iq < S->nq; ++iq) {
      double sq = 0.5 * (1.0 + S->gx[iq]);
      long base[3];
      for (int a = 0; a < 3; ++a) base[a] = spline_base(r, (x0[a] + sq * d[a]) / G->H[a]);
      piece_init(r, base, 0.0, &out[iq]);
      piece_add_point(G, r, x0, d, sq, 0.5 * S->gw[iq], base, &out[iq]);
    }
    return S->nq;
  }
  double s[MAX_BREAKS];
  int nb = orbit_breakpoints(G, r, x0, d, s);
  if (nb < 0) return -1;
  int n = 0;
  for (int m = 0; m + 1 < nb; ++m) {
    double s0 = s[m], s1 = s[m + 1];
    if (!(s1 > s0)) continue; /* zero-length pieces contribute nothing */
    if (n >= cap) return -1;
    long base[3];
    piece_bases(G, r, x0, d, s0, base);
    if (r == 1 && S->c.analytic)
      piece_r1_analytic(G, x0, d, s0, s1, base, &out[n]);
    else
      piece_gauss(G, r, x0, d, s0, s1, base, S->nq, S->gx, S->gw, &out[n]);
    ++n;
  }
  return n;
}

/* ------------------------------------------------------------------------- */
/* particle <-> mesh maps                                                    */
/* ------------------------------------------------------------------------- */

/* point interpolant F_h(x) = sum_g F_g S_g(x) (eq. Ah-mesh), x wrapped first */
static void interp_point(const grid* G, int r, const double xin[3], const double* F, int ncomp,
                         double* out) {
  int w = r + 1;
  double wv[3][4], dwv[3][4];
  long first[3];
  for (int a = 0; a < 3; ++a) {
    double x = wrap_pos(xin[a], G->L[a]);
    double u = x / G->H[a];
    long base = spline_base(r, u);
    first[a] = spline_first(r, base);
    spline_pieces(r, u - (double)base, wv[a], dwv[a]);
  }
  for (int l = 0; l < ncomp; ++l) out[l] = 0.0;
  for (int i = 0; i < w; ++i)
    for (int j = 0; j < w; ++j)
      for (int k = 0; k < w; ++k) {
        int64_t g = node_id(G, first[0] + i, first[1] + j, first[2] + k);
        double Sv = wv[0][i] * wv[1][j] * wv[2][k];
        for (int l = 0; l < ncomp; ++l) out[l] += F[(int64_t)l * G->ncell + g] * Sv;
      }
}

#define MAX_PIECES 600

/* orbit current of one particle: J_g += q vbar Sbar_g / dV (eq. orbit-current) */
static int deposit_one(const orc_sim* S, const double x0[3], const double d[3], const double qv[3],
                       double* J, piece* buf) {
  const grid* G = &S->G;
  int np = orbit_pieces(S, x0, d, buf, MAX_PIECES);
  if (np < 0) return -1;
  for (int m = 0; m < np; ++m) {
    const piece* o = &buf[m];
    int w = o->w;
    for (int i = 0; i < w; ++i)
      for (int j = 0; j < w; ++j)
        for (int k = 0; k < w; ++k) {
          int64_t g = node_id(G, o->first[0] + i, o->first[1] + j, o->first[2] + k);
          double Ig = o->Iw[pidx(w, i, j, k)];
          for (int l = 0; l < 3; ++l) J[(int64_t)l * G->ncell + g] += qv[l] * Ig / G->dV;
        }
  }
  return 0;
}

/* orbit gather of one particle (eqs. orbit-gather-general, Ubar-def, DA-def):
   gphibar_l = sum_g (grad_h phi)_lg Sbar_g, Ubar_l = sum_g U_lg Sbar_g,
   D_lj = sum_g int A_lg(s) d_j S_g(x(s)) ds with A_g(s) = (1-s) A^n + s A^{n+1},
   pou = sum_g Sbar_g. */
static int gather_one(const orc_sim* S, const double x0[3], const double d[3], const double* gphi,
                      const double* Uh, const double* A0, const double* A1, double gphibar[3],
                      double Ubar[3], double D[3][3], double* pou, piece* buf) {
  const grid* G = &S->G;
  int np = orbit_pieces(S, x0, d, buf, MAX_PIECES);
  if (np < 0) return -1;
  for (int l = 0; l < 3; ++l) {
    gphibar[l] = 0.0;
    Ubar[l] = 0.0;
    for (int j = 0; j < 3; ++j) D[l][j] = 0.0;
  }
  *pou = 0.0;
  for (int m = 0; m < np; ++m) {
    const piece* o = &buf[m];
    int w = o->w;
    double sm = o->s0;
    for (int i = 0; i < w; ++i)
      for (int j = 0; j < w; ++j)
        for (int k = 0; k < w; ++k) {
          int64_t g = node_id(G, o->first[0] + i, o->first[1] + j, o->first[2] + k);
          int id = pidx(w, i, j, k);
          double Ig = o->Iw[id];
          *pou += Ig;
          for (int l = 0; l < 3; ++l) {
            int64_t lg = (int64_t)l * G->ncell + g;
            gphibar[l] += gphi[lg] * Ig;
            Ubar[l] += Uh[lg] * Ig;
            double Am = (1.0 - sm) * A0[lg] + sm * A1[lg]; /* A^(m): global s_m (App. B) */
            double C = A1[lg] - A0[lg];
            for (int jj = 0; jj < 3; ++jj) D[l][jj] += Am * o->X[jj][id] + C * o->Y[jj][id];
          }
        }
  }
  return 0;
}

/* point-shape charge deposit rho_g = sum_i q_i S_g(x_i) / dV (eq. source-moments) */
static void deposit_point_charge(const grid* G, int r, int64_t np, const double* x,
                                 const double* qi, double* rho) {
  int w = r + 1;
  for (int64_t i = 0; i < np; ++i) {
    double wv[3][4], dwv[3][4];
    long first[3];
    for (int a = 0; a < 3; ++a) {
      double xa = wrap_pos(x[(int64_t)a * np + i], G->L[a]);
      double u = xa / G->H[a];
      long base = spline_base(r, u);
      first[a] = spline_first(r, base);
      spline_pieces(r, u - (double)base, wv[a], dwv[a]);
    }
    for (int ii = 0; ii < w; ++ii)
      for (int jj = 0; jj < w; ++jj)
        for (int kk = 0; kk < w; ++kk) {
          int64_t g = node_id(G, first[0] + ii, first[1] + jj, first[2] + kk);
          rho[g] += qi[i] * wv[0][ii] * wv[1][jj] * wv[2][kk] / G->dV;
        }
  }
}

/* ------------------------------------------------------------------------- */
/* Fourier operators (Sec. 3.3): plain separable DFT                         */
/* ------------------------------------------------------------------------- */

/* f^_k = sum_j f_j exp(sign 2 pi i j k / N) along one axis of the 3D array */
static void dft_axis(const grid* G, cplx* f, int axis, int sign) {
  int N = G->n[axis];
  int64_t stride = 1;
  for (int a = axis + 1; a < 3; ++a) stride *= G->n[a];
  int64_t outer = 1;
  for (int a = 0; a < axis; ++a) outer *= G->n[a];
  cplx* tw = (cplx*)malloc(sizeof(cplx) * N);
  cplx* tmp = (cplx*)malloc(sizeof(cplx) * N);
  for (int t = 0; t < N; ++t) {
    double ang = 2.0 * M_PI * (double)t / (double)N;
    tw[t] = cos(ang) + (double)sign * sin(ang) * I;
  }
  for (int64_t o = 0; o < outer; ++o)
    for (int64_t in = 0; in < stride; ++in) {
      int64_t b = o * N * stride + in;
      for (int k = 0; k < N; ++k) {
        cplx acc = 0.0;
        for (int j = 0; j < N; ++j) acc += f[b + (int64_t)j * stride] * tw[((int64_t)j * k) % N];
        tmp[k] = acc;
      }
      for (int k = 0; k < N; ++k) f[b + (int64_t)k * stride] = tmp[k];
    }
  free(tw);
  free(tmp);
}

/* sign = -1: forward (unnormalised); sign = +1: inverse (scaled by 1/ncell) */
static void dft3(const grid* G, cplx* f, int sign) {
  for (int a = 0; a < 3; ++a) dft_axis(G, f, a, sign);
  if (sign > 0)
    for (int64_t g = 0; g < G->ncell; ++g) f[g] /= (double)G->ncell;
}

/* Fourier symbol k~ of the first derivative along one axis, mode index m:
   2 pi m_signed / L, and zero on the Nyquist index of an even axis */
static double ktilde(const grid* G, int a, long m) {
  int N = G->n[a];
  if (2 * m == N) return 0.0;
  long ms = (2 * m < N) ? m : m - N;
  return 2.0 * M_PI * (double)ms / G->L[a];
}

static void mode_k(const grid* G, int64_t g, double k[3]) {
  long iz = g % G->n[2];
  long iy = (g / G->n[2]) % G->n[1];
  long ix = g / ((int64_t)G->n[2] * G->n[1]);
  k[0] = ktilde(G, 0, ix);
  k[1] = ktilde(G, 1, iy);
  k[2] = ktilde(G, 2, iz);
}

static void to_real(const grid* G, const cplx* fh, double* out) {
  cplx* t = (cplx*)malloc(sizeof(cplx) * G->ncell);
  memcpy(t, fh, sizeof(cplx) * G->ncell);
  dft3(G, t, +1);
  for (int64_t g = 0; g < G->ncell; ++g) out[g] = creal(t[g]);
  free(t);
}

static void to_fourier(const grid* G, const double* f, cplx* out) {
  for (int64_t g = 0; g < G->ncell; ++g) out[g] = f[g];
  dft3(G, out, -1);
}

/* continuity (eq. cn-continuity) and Crank-Nicolson update (eq. cn-field-update)
   of one step, mode by mode.  Inputs are the level-n spectra and J^{n+1/2};
   outputs the level-(n+1) spectra.  The CN pair (phi, psi) solves the 2x2 system
     phi1 - a psi1                 = phi0 + a psi0
     a w2 phi1 + psi1              = psi0 - a w2 phi0 + dt kappa^2 sigma1 rho^{n+1/2}
   with a = dt/2, w2 = kappa^2 |k~|^2 (Delta_h -> -|k~|^2); (A_l, U_l) likewise with
   sigma2 J_l. */
static void field_update(const orc_sim* S, const cplx* Jh, const cplx* phi0, const cplx* psi0,
                         const cplx* A0, const cplx* U0, const cplx* rho0, cplx* phi1, cplx* psi1,
                         cplx* A1, cplx* U1, cplx* rho1) {
  const grid* G = &S->G;
  double dt = S->c.dt, kap2 = S->c.kappa * S->c.kappa;
  double a = 0.5 * dt;
  int64_t nc = G->ncell;
  for (int64_t g = 0; g < nc; ++g) {
    double k[3];
    mode_k(G, g, k);
    double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    double w2 = kap2 * k2;
    cplx divJ = I * (k[0] * Jh[g] + k[1] * Jh[nc + g] + k[2] * Jh[2 * nc + g]);
    rho1[g] = rho0[g] - dt * divJ;
    cplx rhoh = 0.5 * (rho1[g] + rho0[g]);
    double det = 1.0 + a * a * w2;
    {
      cplx b1 = phi0[g] + a * psi0[g];
      cplx b2 = psi0[g] - a * w2 * phi0[g] + dt * kap2 * S->c.sigma1 * rhoh;
      phi1[g] = (b1 + a * b2) / det;
      psi1[g] = (b2 - a * w2 * b1) / det;
    }
    for (int l = 0; l < 3; ++l) {
      int64_t lg = (int64_t)l * nc + g;
      cplx b1 = A0[lg] + a * U0[lg];
      cplx b2 = U0[lg] - a * w2 * A0[lg] + dt * kap2 * S->c.sigma2 * Jh[lg];
      A1[lg] = (b1 + a * b2) / det;
      U1[lg] = (b2 - a * w2 * b1) / det;
    }
  }
}

/* ------------------------------------------------------------------------- */
/* energies and constraint residuals                                         */
/* ------------------------------------------------------------------------- */

/* W = sum_g (|E_g|^2 / (2 sigma1) + |B_g|^2 / (2 sigma2)) dV with
   E = -grad_h phi - U, B = curl_h A (eqs. field-energy, fields-from-potentials-discrete) */
static double field_energy(const orc_sim* S, const cplx* phi, const cplx* A, const cplx* U) {
  const grid* G = &S->G;
  int64_t nc = G->ncell;
  cplx* Eh = (cplx*)malloc(sizeof(cplx) * 3 * nc);
  cplx* Bh = (cplx*)malloc(sizeof(cplx) * 3 * nc);
  for (int64_t g = 0; g < nc; ++g) {
    double k[3];
    mode_k(G, g, k);
    for (int l = 0; l < 3; ++l) Eh[l * nc + g] = -I * k[l] * phi[g] - U[l * nc + g];
    Bh[0 * nc + g] = I * (k[1] * A[2 * nc + g] - k[2] * A[1 * nc + g]);
    Bh[1 * nc + g] = I * (k[2] * A[0 * nc + g] - k[0] * A[2 * nc + g]);
    Bh[2 * nc + g] = I * (k[0] * A[1 * nc + g] - k[1] * A[0 * nc + g]);
  }
  double* f = (double*)malloc(sizeof(double) * nc);
  double W = 0.0;
  for (int l = 0; l < 3; ++l) {
    to_real(G, Eh + l * nc, f);
    for (int64_t g = 0; g < nc; ++g) W += f[g] * f[g] / (2.0 * S->c.sigma1) * G->dV;
    to_real(G, Bh + l * nc, f);
    for (int64_t g = 0; g < nc; ++g) W += f[g] * f[g] / (2.0 * S->c.sigma2) * G->dV;
  }
  free(Eh);
  free(Bh);
  free(f);
  return W;
}

static double kinetic_energy(const orc_sim* S) {
  double K = 0.0;
  for (int64_t i = 0; i < S->np; ++i)
    for (int a = 0; a < 3; ++a) {
      double va = S->v[(int64_t)a * S->np + i];
      K += 0.5 * S->mi[i] * va * va;
    }
  return K;
}

/* G_h = psi / kappa^2 + div_h A (eq. gauge-diagnostic),
   R_h = div_h E - sigma1 rho (eq. gauss-diagnostic), max and rms over nodes */
static void constraints(const orc_sim* S, double* gmax, double* gl2, double* rmax, double* rl2) {
  const grid* G = &S->G;
  int64_t nc = G->ncell;
  double kap2 = S->c.kappa * S->c.kappa;
  cplx* gh = (cplx*)malloc(sizeof(cplx) * nc);
  cplx* rh = (cplx*)malloc(sizeof(cplx) * nc);
  for (int64_t g = 0; g < nc; ++g) {
    double k[3];
    mode_k(G, g, k);
    cplx divA = I * (k[0] * S->A[g] + k[1] * S->A[nc + g] + k[2] * S->A[2 * nc + g]);
    gh[g] = S->psi[g] / kap2 + divA;
    cplx divE = 0.0;
    for (int l = 0; l < 3; ++l) {
      cplx El = -I * k[l] * S->phi[g] - S->U[l * nc + g];
      divE += I * k[l] * El;
    }
    rh[g] = divE - S->c.sigma1 * S->rho[g];
  }
  double* f = (double*)malloc(sizeof(double) * nc);
  to_real(G, gh, f);
  *gmax = 0.0;
  *gl2 = 0.0;
  for (int64_t g = 0; g < nc; ++g) {
    *gmax = fmax(*gmax, fabs(f[g]));
    *gl2 += f[g] * f[g];
  }
  *gl2 = sqrt(*gl2 / nc);
  to_real(G, rh, f);
  *rmax = 0.0;
  *rl2 = 0.0;
  for (int64_t g = 0; g < nc; ++g) {
    *rmax = fmax(*rmax, fabs(f[g]));
    *rl2 += f[g] * f[g];
  }
  *rl2 = sqrt(*rl2 / nc);
  free(gh);
  free(rh);
  free(f);
}

/* ------------------------------------------------------------------------- */
/* public API                                                                */
/* ------------------------------------------------------------------------- */

/* ------------------------------------------------------------------------- */
/* Anderson mixing of a fixed-point iteration w = G(w)                       */
/* ------------------------------------------------------------------------- */
/*
 * Anderson acceleration (D. G. Anderson, J. ACM 12, 1965; the form of
 * H. F. Walker and P. Ni, SIAM J. Numer. Anal. 49, 2011, with mixing
 * parameter 1).  Given the last mk + 1 iterates w_{p-j} and their images
 * g_{p-j} = G(w_{p-j}), j = 0..mk (index 0 the newest), with residuals
 * f = g - w:
 *   dF_j = f_{p-j+1} - f_{p-j},  dG_j = g_{p-j+1} - g_{p-j},  j = 1..mk
 *   gamma = argmin_gamma || f_p - sum_j gamma_j dF_j ||_2
 *   w_{p+1} = g_p - sum_j gamma_j dG_j
 * The least-squares problem is solved by modified Gram-Schmidt QR of the
 * columns dF_1..dF_mk (newest first, each orthogonalised twice); a column
 * whose norm after orthogonalisation is at most 1e-6 of its own norm, or is
 * zero, is dropped (gamma_j = 0), so that nearly dependent differences do
 * not amplify rounding.  mk = 0 gives the Picard step w_{p+1} = g_p.
 *
 * w[j], g[j]: n doubles each; out: n doubles (may alias none of the inputs);
 * gamma: mk doubles.  Returns 0, or -1 on a bad argument.
 */
int orc_anderson_mix(int mk, int64_t n, const double* const* w, const double* const* g,
                     double* out, double* gamma) {
  if (mk < 0 || mk > ORC_MAX_ANDERSON || n < 0) return -1;
  double* q[ORC_MAX_ANDERSON];
  double R[ORC_MAX_ANDERSON][ORC_MAX_ANDERSON];
  int kept[ORC_MAX_ANDERSON];
  int nk = 0;
  for (int j = 0; j < mk; ++j) gamma[j] = 0.0;
  for (int j = 1; j <= mk; ++j) {
    double* v = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double norm0 = 0.0;
    for (int64_t e = 0; e < n; ++e) {
      v[e] = (g[j - 1][e] - w[j - 1][e]) - (g[j][e] - w[j][e]);
      norm0 += v[e] * v[e];
    }
    norm0 = sqrt(norm0);
    double rcol[ORC_MAX_ANDERSON] = {0.0};
    for (int pass = 0; pass < 2; ++pass)
      for (int k = 0; k < nk; ++k) {
        double r = 0.0;
        for (int64_t e = 0; e < n; ++e) r += q[k][e] * v[e];
        for (int64_t e = 0; e < n; ++e) v[e] -= r * q[k][e];
        rcol[k] += r;
      }
    double norm = 0.0;
    for (int64_t e = 0; e < n; ++e) norm += v[e] * v[e];
    norm = sqrt(norm);
    if (norm0 == 0.0 || norm <= 1e-6 * norm0) {
      free(v);
      continue;
    }
    for (int64_t e = 0; e < n; ++e) v[e] /= norm;
    for (int k = 0; k < nk; ++k) R[k][nk] = rcol[k];
    R[nk][nk] = norm;
    q[nk] = v;
    kept[nk] = j;
    ++nk;
  }
  /* gamma_kept = R^{-1} Q^T f_p */
  double c[ORC_MAX_ANDERSON], gk[ORC_MAX_ANDERSON];
  for (int k = 0; k < nk; ++k) {
    c[k] = 0.0;
    for (int64_t e = 0; e < n; ++e) c[k] += q[k][e] * (g[0][e] - w[0][e]);
  }
  for (int k = nk - 1; k >= 0; --k) {
    double t = c[k];
    for (int l = k + 1; l < nk; ++l) t -= R[k][l] * gk[l];
    gk[k] = t / R[k][k];
  }
  for (int k = 0; k < nk; ++k) gamma[kept[k] - 1] = gk[k];
  for (int64_t e = 0; e < n; ++e) {
    double u = g[0][e];
    for (int j = 1; j <= mk; ++j) u -= gamma[j - 1] * (g[j - 1][e] - g[j][e]);
    out[e] = u;
  }
  for (int k = 0; k < nk; ++k) free(q[k]);
  return 0;
}

/* Record the passes of later steps into caller buffers of 3 np max_passes
   doubles each (NULL stops recording). */
void orc_set_trace(orc_sim* S, double* w, double* g, int max_passes) {
  S->trace_w = w;
  S->trace_g = g;
  S->trace_max = w && g ? max_passes : 0;
}

int orc_check_config(const orc_cfg* c) {
  for (int a = 0; a < 3; ++a)
    if (c->n[a] < 2 || !(c->L[a] > 0.0)) return -1;
  if (c->r < 1 || c->r > 3) return -1;
  if (!(c->dt > 0.0) || !(c->kappa > 0.0) || !(c->sigma1 > 0.0) || !(c->sigma2 > 0.0)) return -1;
  /* Maxwell scaling sigma1 = kappa^2 sigma2 (eq. Maxwell_scaling), to roundoff */
  double lhs = c->sigma1, rhs = c->kappa * c->kappa * c->sigma2;
  if (fabs(lhs - rhs) > 1e-13 * fmax(fabs(lhs), fabs(rhs))) return -1;
  if (c->nq < 0 || c->nq > 64 || c->pmax < 0) return -1;
  if (c->anderson < 0 || c->anderson > ORC_MAX_ANDERSON) return -1;
  return 0;
}

/* every particle of species (q, m) */
static void set_one_species(orc_sim* S, double q, double m) {
  S->q = q;
  S->m = m;
  S->one_species = 1;
  for (int64_t i = 0; i < S->np; ++i) {
    S->qi[i] = q;
    S->mi[i] = m;
  }
}

orc_sim* orc_create(const orc_cfg* c, int64_t np) {
  if (orc_check_config(c) != 0 || np < 0) return NULL;
  orc_sim* S = (orc_sim*)calloc(1, sizeof(orc_sim));
  S->c = *c;
  make_grid(c, &S->G);
  int nq = c->nq;
  if (nq == 0) nq = (3 * c->r + 2) / 2; /* smallest n with 2n - 1 >= 3r */
  S->nq = nq;
  gauss_legendre(nq, S->gx, S->gw);
  S->np = np;
  int64_t n3 = 3 * (np > 0 ? np : 1);
  S->x = (double*)calloc(n3, sizeof(double));
  S->v = (double*)calloc(n3, sizeof(double));
  S->vprev = (double*)calloc(n3, sizeof(double));
  S->P = (double*)calloc(n3, sizeof(double));
  int64_t nc = S->G.ncell;
  S->phi = (cplx*)calloc(nc, sizeof(cplx));
  S->psi = (cplx*)calloc(nc, sizeof(cplx));
  S->rho = (cplx*)calloc(nc, sizeof(cplx));
  S->A = (cplx*)calloc(3 * nc, sizeof(cplx));
  S->U = (cplx*)calloc(3 * nc, sizeof(cplx));
  S->J = (double*)calloc(3 * nc, sizeof(double));
  S->qi = (double*)calloc(np > 0 ? np : 1, sizeof(double));
  S->mi = (double*)calloc(np > 0 ? np : 1, sizeof(double));
  set_one_species(S, -1.0, 1.0);
  return S;
}

void orc_destroy(orc_sim* S) {
  if (!S) return;
  free(S->x);
  free(S->v);
  free(S->vprev);
  free(S->P);
  free(S->qi);
  free(S->mi);
  free(S->phi);
  free(S->psi);
  free(S->rho);
  free(S->A);
  free(S->U);
  free(S->J);
  free(S);
}

/* Gauss rule in use (for tests) */
int orc_gauss_rule(const orc_sim* S, double* x, double* w) {
  for (int i = 0; i < S->nq; ++i) {
    x[i] = S->gx[i];
    w[i] = S->gw[i];
  }
  return S->nq;
}

int orc_gauss_legendre(int n, double* x, double* w) {
  if (n < 1 || n > 64) return -1;
  gauss_legendre(n, x, w);
  return 0;
}

static void update_energy_start(orc_sim* S) {
  S->en.K = kinetic_energy(S);
  S->en.W = field_energy(S, S->phi, S->A, S->U);
  S->en.E_total = S->en.K + S->en.W;
  constraints(S, &S->en.gauge_max, &S->en.gauge_l2, &S->en.gauss_max, &S->en.gauss_l2);
}

/* Initial state of the two-stream setup (Sec. 5.4): point-shape charge deposit
   plus uniform background n0, mean removed (and zeroed on every k~ = 0 mode),
   phi^0 from -Delta_h phi = sigma1 rho, psi = A = U = 0, P = m v, v^{-1} = v^0. */
static int init_state(orc_sim* S, const double* x, const double* v, double n0);

int orc_init_particles(orc_sim* S, const double* x, const double* v, double q, double m,
                       double n0) {
  set_one_species(S, q, m);
  return init_state(S, x, v, n0);
}

/* Several species (each particle carries its own q_i and m_i, Sec. 2):
   particle i has charge q[species[i]] and mass m[species[i]]. */
int orc_init_species(orc_sim* S, const double* x, const double* v, const int32_t* species,
                     int nspecies, const double* q, const double* m, double n0) {
  if (nspecies < 1) return -1;
  for (int64_t i = 0; i < S->np; ++i)
    if (species[i] < 0 || species[i] >= nspecies) return -1;
  S->q = q[0];
  S->m = m[0];
  S->one_species = 1;
  for (int64_t i = 0; i < S->np; ++i) {
    S->qi[i] = q[species[i]];
    S->mi[i] = m[species[i]];
    if (S->qi[i] != q[0] || S->mi[i] != m[0]) S->one_species = 0;
  }
  return init_state(S, x, v, n0);
}

static int init_state(orc_sim* S, const double* x, const double* v, double n0) {
  const grid* G = &S->G;
  int64_t np = S->np, nc = G->ncell;
  for (int a = 0; a < 3; ++a)
    for (int64_t i = 0; i < np; ++i) {
      int64_t id = a * np + i;
      S->v[id] = v[id];
      S->vprev[id] = v[id];
      S->P[id] = S->mi[i] * v[id];
    }
  for (int a = 0; a < 3; ++a)
    for (int64_t i = 0; i < np; ++i) S->x[a * np + i] = wrap_pos(x[a * np + i], G->L[a]);
  double* rho = (double*)calloc(nc, sizeof(double));
  deposit_point_charge(G, S->c.r, np, S->x, S->qi, rho);
  double mean = 0.0;
  for (int64_t g = 0; g < nc; ++g) {
    rho[g] += n0;
    mean += rho[g];
  }
  mean /= (double)nc;
  for (int64_t g = 0; g < nc; ++g) rho[g] -= mean;
  to_fourier(G, rho, S->rho);
  free(rho);
  for (int64_t g = 0; g < nc; ++g) {
    double k[3];
    mode_k(G, g, k);
    double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (k2 == 0.0) {
      S->rho[g] = 0.0;
      S->phi[g] = 0.0;
    } else {
      S->phi[g] = S->c.sigma1 * S->rho[g] / k2;
    }
    S->psi[g] = 0.0;
    for (int l = 0; l < 3; ++l) {
      S->A[l * nc + g] = 0.0;
      S->U[l * nc + g] = 0.0;
    }
  }
  memset(S->J, 0, sizeof(double) * 3 * nc);
  memset(&S->en, 0, sizeof(S->en));
  update_energy_start(S);
  S->K0 = S->en.K;
  S->W0 = S->en.W;
  S->have_energy = 1;
  return 0;
}

/* One time step: Algorithm 1 (Picard iteration of the coupled orbit /
   continuity / CN / push system).  Returns 0 when converged, 1 when the
   iteration reached p_max (the last iterate is accepted), -1 on error. */
int orc_picard_step(orc_sim* S, orc_step_info* info) {
  const grid* G = &S->G;
  int64_t np = S->np, nc = G->ncell;
  double dt = S->c.dt;

  double K_n = kinetic_energy(S);
  double W_n = field_energy(S, S->phi, S->A, S->U);

  /* level-n mesh quantities in real space */
  double* A0r = (double*)malloc(sizeof(double) * 3 * nc);
  for (int l = 0; l < 3; ++l) to_real(G, S->A + l * nc, A0r + l * nc);

  double* vit = (double*)malloc(sizeof(double) * 3 * np + 8);
  double* vnew = (double*)malloc(sizeof(double) * 3 * np + 8);
  double* Pnew = (double*)malloc(sizeof(double) * 3 * np + 8);
  double* J = (double*)malloc(sizeof(double) * 3 * nc);
  double* Jprev = (double*)malloc(sizeof(double) * 3 * nc);
  cplx* Jh = (cplx*)malloc(sizeof(cplx) * 3 * nc);
  cplx *phi1 = (cplx*)malloc(sizeof(cplx) * nc), *psi1 = (cplx*)malloc(sizeof(cplx) * nc);
  cplx* rho1 = (cplx*)malloc(sizeof(cplx) * nc);
  cplx *A1 = (cplx*)malloc(sizeof(cplx) * 3 * nc), *U1 = (cplx*)malloc(sizeof(cplx) * 3 * nc);
  cplx* tmp = (cplx*)malloc(sizeof(cplx) * nc);
  double* gphi = (double*)malloc(sizeof(double) * 3 * nc);
  double* Uhalf = (double*)malloc(sizeof(double) * 3 * nc);
  double* A1r = (double*)malloc(sizeof(double) * 3 * nc);
  piece* buf = (piece*)malloc(sizeof(piece) * MAX_PIECES);
  int status = 1;
  double err_v = 0.0, err_J = 0.0;
  int p = 0;
  double work = 0.0, JE = 0.0, RA2 = 0.0, RAmax = 0.0, poumax = 0.0;
  /* Anderson history: iterates and images of the last m + 1 passes (pass k in slot k % (m + 1)) */
  const int M = S->c.anderson;
  double* hist_w[ORC_MAX_ANDERSON + 1] = {NULL};
  double* hist_g[ORC_MAX_ANDERSON + 1] = {NULL};
  for (int k = 0; M > 0 && k <= M; ++k) {
    hist_w[k] = (double*)malloc(sizeof(double) * 3 * np + 8);
    hist_g[k] = (double*)malloc(sizeof(double) * 3 * np + 8);
  }

  /* extrapolated initial guess v^{n+1,0} = 2 v^n - v^{n-1} */
  for (int64_t i = 0; i < 3 * np; ++i) vit[i] = 2.0 * S->v[i] - S->vprev[i];

  for (p = 0; p <= S->c.pmax; ++p) {
    /* orbit of the current iterate and its current J^{n+1/2,p} */
    memset(J, 0, sizeof(double) * 3 * nc);
    double Js = 0.0;
    for (int64_t i = 0; i < np; ++i) {
      double x0[3], vb[3], d[3], qv[3];
      double vmax = 0.0;
      for (int a = 0; a < 3; ++a) {
        x0[a] = S->x[a * np + i];
        vb[a] = 0.5 * (vit[a * np + i] + S->v[a * np + i]);
        d[a] = dt * vb[a];
        qv[a] = S->qi[i] * vb[a];
        vmax = fmax(vmax, fabs(vb[a]));
      }
      Js += fabs(S->qi[i]) * vmax;
      if (deposit_one(S, x0, d, qv, J, buf) != 0) { status = -1; goto done; }
    }
    Js /= G->vol;

    /* continuity + CN */
    for (int l = 0; l < 3; ++l) to_fourier(G, J + l * nc, Jh + l * nc);
    field_update(S, Jh, S->phi, S->psi, S->A, S->U, S->rho, phi1, psi1, A1, U1, rho1);

    /* midpoint and end-of-step mesh fields in real space */
    for (int l = 0; l < 3; ++l) {
      for (int64_t g = 0; g < nc; ++g) {
        double k[3];
        mode_k(G, g, k);
        tmp[g] = I * k[l] * 0.5 * (phi1[g] + S->phi[g]);
      }
      to_real(G, tmp, gphi + l * nc);
      for (int64_t g = 0; g < nc; ++g) tmp[g] = 0.5 * (U1[l * nc + g] + S->U[l * nc + g]);
      to_real(G, tmp, Uhalf + l * nc);
      to_real(G, A1 + l * nc, A1r + l * nc);
    }

    /* gather + orbit-discrete-gradient push + velocity closure */
    double dvmax = 0.0, vmaxall = 0.0;
    work = 0.0;
    RA2 = 0.0;
    RAmax = 0.0;
    poumax = 0.0;
    for (int64_t i = 0; i < np; ++i) {
      double x0[3], vb[3], d[3], x1[3];
      for (int a = 0; a < 3; ++a) {
        x0[a] = S->x[a * np + i];
        vb[a] = 0.5 * (vit[a * np + i] + S->v[a * np + i]);
        d[a] = dt * vb[a];
        x1[a] = x0[a] + d[a];
      }
      double gpb[3], Ub[3], D[3][3], pou;
      if (gather_one(S, x0, d, gphi, Uhalf, A0r, A1r, gpb, Ub, D, &pou, buf) != 0) {
        status = -1;
        goto done;
      }
      double Aend[3], Astart[3];
      interp_point(G, S->c.r, x1, A1r, 3, Aend);
      interp_point(G, S->c.r, x0, A0r, 3, Astart);
      for (int j = 0; j < 3; ++j) {
        double DTv = 0.0; /* ((D A)^T vbar)_j = sum_l D_lj vbar_l */
        for (int l = 0; l < 3; ++l) DTv += D[l][j] * vb[l];
        double Pj = S->P[j * np + i] + dt * (-S->qi[i] * gpb[j] + S->qi[i] * DTv);
        Pnew[j * np + i] = Pj;
        double vj = (Pj - S->qi[i] * Aend[j]) / S->mi[i];
        vnew[j * np + i] = vj;
        dvmax = fmax(dvmax, fabs(vj - vit[j * np + i]));
        vmaxall = fmax(vmaxall, fabs(vj));
      }
      for (int l = 0; l < 3; ++l) {
        double Dv = 0.0;
        for (int j = 0; j < 3; ++j) Dv += D[l][j] * vb[j];
        double RA = Aend[l] - Astart[l] - dt * (Ub[l] + Dv);
        RA2 += RA * RA;
        RAmax = fmax(RAmax, fabs(RA));
        work += S->qi[i] * vb[l] * (-gpb[l] - Ub[l]);
      }
      poumax = fmax(poumax, fabs(pou - 1.0));
    }

    /* mesh work sum_g J.E^{n+1/2} dV of this iterate */
    JE = 0.0;
    for (int l = 0; l < 3; ++l)
      for (int64_t g = 0; g < nc; ++g)
        JE += J[l * nc + g] * (-gphi[l * nc + g] - Uhalf[l * nc + g]) * G->dV;

    if (S->trace_w && p < S->trace_max) {
      memcpy(S->trace_w + (size_t)3 * np * p, vit, sizeof(double) * 3 * np);
      memcpy(S->trace_g + (size_t)3 * np * p, vnew, sizeof(double) * 3 * np);
    }

    /* fixed-point errors */
    err_v = vmaxall > 0.0 ? dvmax / vmaxall : dvmax;
    if (p >= 1) {
      double dJ = 0.0;
      for (int64_t g = 0; g < 3 * nc; ++g) dJ = fmax(dJ, fabs(J[g] - Jprev[g]));
      err_J = Js > 0.0 ? dJ / Js : dJ;
    } else {
      err_J = INFINITY;
    }
    memcpy(Jprev, J, sizeof(double) * 3 * nc);

    if (p >= 1 && err_v < S->c.tol && err_J < S->c.tol) {
      status = 0;
      break;
    }
    if (p == S->c.pmax) break;
    if (M == 0) {
      memcpy(vit, vnew, sizeof(double) * 3 * np); /* Picard: v^{n+1,p+1} is the next iterate */
    } else {
      memcpy(hist_w[p % (M + 1)], vit, sizeof(double) * 3 * np);
      memcpy(hist_g[p % (M + 1)], vnew, sizeof(double) * 3 * np);
      const int mk = p < M ? p : M;
      const double* wv[ORC_MAX_ANDERSON + 1];
      const double* gv[ORC_MAX_ANDERSON + 1];
      for (int j = 0; j <= mk; ++j) {
        wv[j] = hist_w[(p - j) % (M + 1)];
        gv[j] = hist_g[(p - j) % (M + 1)];
      }
      double gamma[ORC_MAX_ANDERSON];
      orc_anderson_mix(mk, 3 * np, wv, gv, vit, gamma);
    }
  }
  if (p > S->c.pmax) p = S->c.pmax;

  /* accept iterate p: x^{n+1} = x^n + dt vbar^p (wrapped), v^{n+1} = v^{n+1,p+1},
     P^{n+1} = P^{n+1,p}, mesh fields of iterate p */
  for (int a = 0; a < 3; ++a)
    for (int64_t i = 0; i < np; ++i) {
      int64_t id = a * np + i;
      double vb = 0.5 * (vit[id] + S->v[id]);
      S->x[id] = wrap_pos(S->x[id] + dt * vb, G->L[a]);
      S->vprev[id] = S->v[id];
      S->v[id] = vnew[id];
      S->P[id] = Pnew[id];
    }
  memcpy(S->phi, phi1, sizeof(cplx) * nc);
  memcpy(S->psi, psi1, sizeof(cplx) * nc);
  memcpy(S->rho, rho1, sizeof(cplx) * nc);
  memcpy(S->A, A1, sizeof(cplx) * 3 * nc);
  memcpy(S->U, U1, sizeof(cplx) * 3 * nc);
  memcpy(S->J, J, sizeof(double) * 3 * nc);

  /* diagnostics of the accepted iterate (its orbit, current and fields) */
  update_energy_start(S);
  S->en.R_field = S->en.W - W_n + dt * JE;
  S->en.R_particle = S->en.K - K_n - dt * work;
  S->en.R_total = (S->en.K + S->en.W) - (K_n + W_n);
  S->en.JE_mesh = JE;
  S->en.work_particle = work;
  S->en.RA_rms = np > 0 ? sqrt(RA2 / (3.0 * np)) : 0.0;
  S->en.RA_max = RAmax;
  S->en.pou_max = poumax;
  S->en.step += 1;

done:
  if (info) {
    info->iters = p + 1;
    info->converged = status == 0;
    info->err_v = err_v;
    info->err_J = err_J;
  }
  for (int k = 0; k <= ORC_MAX_ANDERSON; ++k) {
    free(hist_w[k]);
    free(hist_g[k]);
  }
  free(A0r);
  free(vit);
  free(vnew);
  free(Pnew);
  free(J);
  free(Jprev);
  free(Jh);
  free(phi1);
  free(psi1);
  free(rho1);
  free(A1);
  free(U1);
  free(tmp);
  free(gphi);
  free(Uhalf);
  free(A1r);
  free(buf);
  return status;
}

int orc_energy_diagnostics(const orc_sim* S, orc_energy* out) {
  *out = S->en;
  return 0;
}

/* fields layout: [phi, psi, Ax, Ay, Az, Ux, Uy, Uz, rho] real-space, ncell each */
int orc_get_state(const orc_sim* S, double* x, double* v, double* vprev, double* P,
                  double* fields) {
  int64_t n3 = 3 * S->np, nc = S->G.ncell;
  if (x) memcpy(x, S->x, sizeof(double) * n3);
  if (v) memcpy(v, S->v, sizeof(double) * n3);
  if (vprev) memcpy(vprev, S->vprev, sizeof(double) * n3);
  if (P) memcpy(P, S->P, sizeof(double) * n3);
  if (fields) {
    to_real(&S->G, S->phi, fields + 0 * nc);
    to_real(&S->G, S->psi, fields + 1 * nc);
    for (int l = 0; l < 3; ++l) to_real(&S->G, S->A + l * nc, fields + (2 + l) * nc);
    for (int l = 0; l < 3; ++l) to_real(&S->G, S->U + l * nc, fields + (5 + l) * nc);
    to_real(&S->G, S->rho, fields + 8 * nc);
  }
  return 0;
}

int orc_set_state(orc_sim* S, const double* x, const double* v, const double* vprev,
                  const double* P, const double* fields, double q, double m) {
  int64_t n3 = 3 * S->np, nc = S->G.ncell;
  if (m > 0.0) set_one_species(S, q, m); /* m = 0: keep every particle's species */
  if (x) memcpy(S->x, x, sizeof(double) * n3);
  if (v) memcpy(S->v, v, sizeof(double) * n3);
  if (vprev) memcpy(S->vprev, vprev, sizeof(double) * n3);
  if (P) memcpy(S->P, P, sizeof(double) * n3);
  if (fields) {
    to_fourier(&S->G, fields + 0 * nc, S->phi);
    to_fourier(&S->G, fields + 1 * nc, S->psi);
    for (int l = 0; l < 3; ++l) to_fourier(&S->G, fields + (2 + l) * nc, S->A + l * nc);
    for (int l = 0; l < 3; ++l) to_fourier(&S->G, fields + (5 + l) * nc, S->U + l * nc);
    to_fourier(&S->G, fields + 8 * nc, S->rho);
  }
  update_energy_start(S);
  return 0;
}

/* real-space orbit current of the accepted iterate of the last step */
int orc_get_current(const orc_sim* S, double* J) {
  memcpy(J, S->J, sizeof(double) * 3 * S->G.ncell);
  return 0;
}

/* Field update alone (continuity + CN) for a given real-space J^{n+1/2}, from the
   current state; the state advances to level n+1 (particles untouched). */
int orc_field_solve(orc_sim* S, const double* J) {
  const grid* G = &S->G;
  int64_t nc = G->ncell;
  cplx* Jh = (cplx*)malloc(sizeof(cplx) * 3 * nc);
  cplx *phi1 = (cplx*)malloc(sizeof(cplx) * nc), *psi1 = (cplx*)malloc(sizeof(cplx) * nc);
  cplx* rho1 = (cplx*)malloc(sizeof(cplx) * nc);
  cplx *A1 = (cplx*)malloc(sizeof(cplx) * 3 * nc), *U1 = (cplx*)malloc(sizeof(cplx) * 3 * nc);
  for (int l = 0; l < 3; ++l) to_fourier(G, J + l * nc, Jh + l * nc);
  field_update(S, Jh, S->phi, S->psi, S->A, S->U, S->rho, phi1, psi1, A1, U1, rho1);
  memcpy(S->phi, phi1, sizeof(cplx) * nc);
  memcpy(S->psi, psi1, sizeof(cplx) * nc);
  memcpy(S->rho, rho1, sizeof(cplx) * nc);
  memcpy(S->A, A1, sizeof(cplx) * 3 * nc);
  memcpy(S->U, U1, sizeof(cplx) * 3 * nc);
  memcpy(S->J, J, sizeof(double) * 3 * nc);
  update_energy_start(S);
  free(Jh);
  free(phi1);
  free(psi1);
  free(rho1);
  free(A1);
  free(U1);
  return 0;
}

/* W of arbitrary real-space potentials (phi, A[3], U[3]) -- used by tests */
double orc_field_energy_of(const orc_sim* S, const double* phi, const double* A, const double* U) {
  int64_t nc = S->G.ncell;
  cplx* ph = (cplx*)malloc(sizeof(cplx) * nc);
  cplx* Ah = (cplx*)malloc(sizeof(cplx) * 3 * nc);
  cplx* Uh = (cplx*)malloc(sizeof(cplx) * 3 * nc);
  to_fourier(&S->G, phi, ph);
  for (int l = 0; l < 3; ++l) {
    to_fourier(&S->G, A + l * nc, Ah + l * nc);
    to_fourier(&S->G, U + l * nc, Uh + l * nc);
  }
  double W = field_energy(S, ph, Ah, Uh);
  free(ph);
  free(Ah);
  free(Uh);
  return W;
}

/* ---- single-particle and kernel-level entry points for tests ------------ */

/* Orbit integrals of n particles against given real-space mesh fields
   gphi (3 x ncell), Uh (3 x ncell), A0, A1 (3 x ncell).
   out per particle (stride 24):
     [0:3] gphibar, [3:6] Ubar, [6:15] D (row l, column j), [15:18] A1_h(x1),
     [18:21] A0_h(x0), [21] sum_g Sbar_g, [22] number of pieces, [23] unused */
int orc_orbit_gather(const orc_sim* S, int64_t n, const double* x0, const double* d,
                     const double* gphi, const double* Uh, const double* A0, const double* A1,
                     double* out) {
  piece* buf = (piece*)malloc(sizeof(piece) * MAX_PIECES);
  for (int64_t i = 0; i < n; ++i) {
    double xa[3], da[3], x1[3];
    for (int a = 0; a < 3; ++a) {
      xa[a] = x0[3 * i + a];
      da[a] = d[3 * i + a];
      x1[a] = xa[a] + da[a];
    }
    double gpb[3], Ub[3], D[3][3], pou;
    if (gather_one(S, xa, da, gphi, Uh, A0, A1, gpb, Ub, D, &pou, buf) != 0) {
      free(buf);
      return -1;
    }
    double* o = out + 24 * i;
    for (int l = 0; l < 3; ++l) {
      o[l] = gpb[l];
      o[3 + l] = Ub[l];
      for (int j = 0; j < 3; ++j) o[6 + 3 * l + j] = D[l][j];
    }
    interp_point(&S->G, S->c.r, x1, A1, 3, o + 15);
    interp_point(&S->G, S->c.r, xa, A0, 3, o + 18);
    o[21] = pou;
    o[22] = (double)orbit_pieces(S, xa, da, buf, MAX_PIECES);
    o[23] = 0.0;
  }
  free(buf);
  return 0;
}

/* Orbit current of n particles (positions x0, displacements d, per-particle
   q vbar in qv), all 3*n row-major per particle; J is 3 x ncell, accumulated. */
int orc_orbit_deposit(const orc_sim* S, int64_t n, const double* x0, const double* d,
                      const double* qv, double* J) {
  piece* buf = (piece*)malloc(sizeof(piece) * MAX_PIECES);
  for (int64_t i = 0; i < n; ++i) {
    if (deposit_one(S, x0 + 3 * i, d + 3 * i, qv + 3 * i, J, buf) != 0) {
      free(buf);
      return -1;
    }
  }
  free(buf);
  return 0;
}

/* point interpolation of ncomp real-space fields at n points (3*n row-major) */
int orc_interp(const orc_sim* S, int64_t n, const double* x, const double* F, int ncomp,
               double* out) {
  for (int64_t i = 0; i < n; ++i) interp_point(&S->G, S->c.r, x + 3 * i, F, ncomp, out + ncomp * i);
  return 0;
}

/* breakpoints of one orbit (returns count) */
int orc_breakpoints(const orc_sim* S, const double* x0, const double* d, double* s) {
  return orbit_breakpoints(&S->G, S->c.r, x0, d, s);
}

/* 3D DFT of interleaved complex data (sign -1 forward, +1 inverse scaled) */
int orc_dft3(const orc_sim* S, double* data, int sign) {
  dft3(&S->G, (cplx*)data, sign);
  return 0;
}

/* Fourier symbols k~ of the three axes at every mode (3 x ncell) */
int orc_ktilde(const orc_sim* S, double* k) {
  int64_t nc = S->G.ncell;
  for (int64_t g = 0; g < nc; ++g) {
    double kk[3];
    mode_k(&S->G, g, kk);
    for (int a = 0; a < 3; ++a) k[a * nc + g] = kk[a];
  }
  return 0;
}

/* ------------------------------------------------------------------------- */
/* adjoint of one converged step (degree 2, split orbits)                    */
/* ------------------------------------------------------------------------- */
/*
 * The converged step is the solution w = v^{n+1} of w = G(w; x, v, F) with
 * (rebuilding P^n = m v + q A_h^n(x), eq. discrete-canonical-relation)
 *
 *   G = v + (q/m) [A0_h(x) - A1_h(x + d)] + (q dt/m) [-gphibar + (D A)^T vbar],
 *   vbar = (w + v)/2, d = dt vbar,
 *   gphibar = sum_g gphi_g Sbar_g,  ((D A)^T vbar)_j = sum_g int b_g(s) d_j S_g(x(s)) ds,
 *   b_g(s) = vbar . ((1-s) A0_g + s A1_g),
 *
 * where gphi = grad_h (phi^n + phi^{n+1})/2, A0 = A^n, A1 = A^{n+1} come from
 * the continuity + CN update driven by J = (q/dV) sum_i vbar_i Sbar_i
 * (eqs. orbit-current, cn-continuity, cn-field-update, orbit-push).  The
 * outputs are x' = x + d, v' = w and the level-(n+1) fields.
 *
 * Given the adjoints (lx1, lv1, lF1) of the outputs, the adjoint xi of w
 * solves xi = b + (dG/dw)^T xi (the transposed Picard iteration), and
 *   lv0 = 2 xi - lv1   (w and v enter every term through vbar alike, and v
 *                       once more directly),
 *   lx0 = lx1 + x-derivatives of J and G,  lF0 = fields' share.
 * Complex spectra follow dL = Re sum conj(lambda) dz.  Only degree 2: with
 * degree 1 the derivative of the piecewise-constant grad S jumps at knots.
 */

/* degree-2 weights, first and second derivatives (per unit of u) */
static void spline2_all(double t, double w[3], double dw[3], double ddw[3]) {
  w[0] = 0.5 * (0.5 - t) * (0.5 - t);
  w[1] = 0.75 - t * t;
  w[2] = 0.5 * (0.5 + t) * (0.5 + t);
  dw[0] = -(0.5 - t);
  dw[1] = -2.0 * t;
  dw[2] = 0.5 + t;
  ddw[0] = 1.0;
  ddw[1] = -2.0;
  ddw[2] = 1.0;
}

/* S, grad S and the Hessian of S for the 27 nodes first + (i, j, k), at
   position xp written against the given base nodes */
static void node_derivs(const grid* G, const double xp[3], const long base[3], double S[27],
                        double dS[27][3], double ddS[27][3][3]) {
  double w[3][3], dw[3][3], ddw[3][3];
  for (int a = 0; a < 3; ++a) {
    spline2_all(xp[a] / G->H[a] - (double)base[a], w[a], dw[a], ddw[a]);
    for (int o = 0; o < 3; ++o) {
      dw[a][o] /= G->H[a];
      ddw[a][o] /= G->H[a] * G->H[a];
    }
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) {
        int id = pidx(3, i, j, k);
        int o[3] = {i, j, k};
        S[id] = w[0][i] * w[1][j] * w[2][k];
        for (int p = 0; p < 3; ++p) {
          double f = 1.0;
          for (int a = 0; a < 3; ++a) f *= (a == p) ? dw[a][o[a]] : w[a][o[a]];
          dS[id][p] = f;
          for (int r2 = 0; r2 < 3; ++r2) {
            double h = 1.0;
            for (int a = 0; a < 3; ++a) {
              if (a == p && a == r2)
                h *= ddw[a][o[a]];
              else if (a == p || a == r2)
                h *= dw[a][o[a]];
              else
                h *= w[a][o[a]];
            }
            ddS[id][p][r2] = h;
          }
        }
      }
}

/* Per-particle adjoint contributions.  eta = (q/m) xi (push terms, may be
   NULL), mu = (q/dV) lambda_J (deposit terms, may be NULL).  Accumulates
   lx, ld, lvb (3 each) and, for eta, the mesh adjoints of gphi, A0, A1. */
static int particle_adjoint(const orc_sim* S, const double x0[3], const double vb[3],
                            const double* eta, const double* mu, const double* gphi,
                            const double* A0, const double* A1, double lx[3], double ld[3],
                            double lvb[3], double* lgphi, double* lA0, double* lA1) {
  const grid* G = &S->G;
  int64_t nc = G->ncell;
  double dt = S->c.dt;
  double d[3];
  for (int a = 0; a < 3; ++a) d[a] = dt * vb[a];
  double sb[MAX_BREAKS];
  int nb = orbit_breakpoints(G, 2, x0, d, sb);
  if (nb < 0) return -1;
  double Sv[27], dS[27][3], ddS[27][3][3];
  for (int m = 0; m + 1 < nb; ++m) {
    double s0 = sb[m], s1 = sb[m + 1];
    if (!(s1 > s0)) continue;
    double h = s1 - s0;
    long base[3], first[3];
    piece_bases(G, 2, x0, d, s0, base);
    for (int a = 0; a < 3; ++a) first[a] = spline_first(2, base[a]);
    for (int iq = 0; iq < S->nq; ++iq) {
      double s = s0 + 0.5 * h * (1.0 + S->gx[iq]);
      double wt = 0.5 * h * S->gw[iq];
      double xp[3];
      for (int a = 0; a < 3; ++a) xp[a] = x0[a] + s * d[a];
      node_derivs(G, xp, base, Sv, dS, ddS);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k) {
            int id = pidx(3, i, j, k);
            int64_t g = node_id(G, first[0] + i, first[1] + j, first[2] + k);
            if (eta) {
              double Ag[3], bg = 0.0, edS = 0.0;
              for (int l = 0; l < 3; ++l) {
                Ag[l] = (1.0 - s) * A0[l * nc + g] + s * A1[l * nc + g];
                bg += vb[l] * Ag[l];
                edS += eta[l] * dS[id][l];
              }
              /* -dt gphibar */
              double eg = 0.0;
              for (int l = 0; l < 3; ++l) eg += eta[l] * gphi[l * nc + g];
              for (int kk = 0; kk < 3; ++kk) {
                lx[kk] -= dt * wt * eg * dS[id][kk];
                ld[kk] -= dt * wt * s * eg * dS[id][kk];
              }
              for (int l = 0; l < 3; ++l) lgphi[l * nc + g] -= dt * wt * eta[l] * Sv[id];
              /* dt (D A)^T vbar */
              for (int l = 0; l < 3; ++l) lvb[l] += dt * wt * Ag[l] * edS;
              for (int kk = 0; kk < 3; ++kk) {
                double eH = 0.0;
                for (int jj = 0; jj < 3; ++jj) eH += eta[jj] * ddS[id][jj][kk];
                lx[kk] += dt * wt * bg * eH;
                ld[kk] += dt * wt * s * bg * eH;
              }
              for (int l = 0; l < 3; ++l) {
                lA0[l * nc + g] += dt * wt * (1.0 - s) * vb[l] * edS;
                lA1[l * nc + g] += dt * wt * s * vb[l] * edS;
              }
            }
            if (mu) {
              double vm = 0.0;
              for (int l = 0; l < 3; ++l) {
                lvb[l] += wt * mu[l * nc + g] * Sv[id];
                vm += vb[l] * mu[l * nc + g];
              }
              for (int kk = 0; kk < 3; ++kk) {
                lx[kk] += wt * vm * dS[id][kk];
                ld[kk] += wt * s * vm * dS[id][kk];
              }
            }
          }
    }
  }
  if (eta) { /* point terms: + A0_h(x0) - A1_h(x0 + d) */
    for (int e = 0; e < 2; ++e) {
      double sgn = e == 0 ? 1.0 : -1.0;
      const double* F = e == 0 ? A0 : A1;
      double* lF = e == 0 ? lA0 : lA1;
      double xp[3];
      long base[3], first[3];
      for (int a = 0; a < 3; ++a) {
        xp[a] = wrap_pos(x0[a] + (e == 0 ? 0.0 : d[a]), G->L[a]);
        base[a] = spline_base(2, xp[a] / G->H[a]);
        first[a] = spline_first(2, base[a]);
      }
      node_derivs(G, xp, base, Sv, dS, ddS);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          for (int k = 0; k < 3; ++k) {
            int id = pidx(3, i, j, k);
            int64_t g = node_id(G, first[0] + i, first[1] + j, first[2] + k);
            double eF = 0.0;
            for (int l = 0; l < 3; ++l) {
              eF += eta[l] * F[l * nc + g];
              lF[l * nc + g] += sgn * eta[l] * Sv[id];
            }
            for (int kk = 0; kk < 3; ++kk) {
              lx[kk] += sgn * eF * dS[id][kk];
              if (e == 1) ld[kk] += sgn * eF * dS[id][kk];
            }
          }
    }
  }
  return 0;
}

/* adjoint of the continuity + CN update of one mode set: given the adjoints
   of the new level (any may be NULL = zero), accumulate those of the old
   level (9 spectra: phi, psi, A0..2, U0..2, rho; may be NULL) and of J^ */
static void cn_adjoint(const orc_sim* S, const cplx* lphi1, const cplx* lpsi1, const cplx* lA1,
                       const cplx* lU1, const cplx* lrho1, cplx* lF0, cplx* lJh) {
  const grid* G = &S->G;
  double dt = S->c.dt, kap2 = S->c.kappa * S->c.kappa, a = 0.5 * dt;
  int64_t nc = G->ncell;
  for (int64_t g = 0; g < nc; ++g) {
    double k[3];
    mode_k(G, g, k);
    double w2 = kap2 * (k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    double det = 1.0 + a * a * w2;
    cplx lp1 = lphi1 ? lphi1[g] : 0.0, ls1 = lpsi1 ? lpsi1[g] : 0.0;
    cplx lb1 = (lp1 - a * w2 * ls1) / det;
    cplx lb2 = (a * lp1 + ls1) / det;
    cplx lrhoh = dt * kap2 * S->c.sigma1 * lb2;
    cplx lr1 = (lrho1 ? lrho1[g] : 0.0) + 0.5 * lrhoh;
    if (lF0) {
      lF0[g] += lb1 - a * w2 * lb2;
      lF0[nc + g] += a * lb1 + lb2;
      lF0[8 * nc + g] += lr1 + 0.5 * lrhoh;
    }
    for (int l = 0; l < 3; ++l) {
      int64_t lg = (int64_t)l * nc + g;
      cplx la = lA1 ? lA1[lg] : 0.0, lu = lU1 ? lU1[lg] : 0.0;
      cplx lc1 = (la - a * w2 * lu) / det;
      cplx lc2 = (a * la + lu) / det;
      if (lF0) {
        lF0[(2 + l) * nc + g] += lc1 - a * w2 * lc2;
        lF0[(5 + l) * nc + g] += a * lc1 + lc2;
      }
      lJh[lg] += dt * kap2 * S->c.sigma2 * lc2 + dt * I * k[l] * lr1;
    }
  }
}

/* lambda of a spectrum from lambda of its real-space inverse transform */
static void adj_of_to_real(const grid* G, const double* ly, cplx* lz) {
  to_fourier(G, ly, lz);
  for (int64_t g = 0; g < G->ncell; ++g) lz[g] /= (double)G->ncell;
}

/* lambda of a real array from lambda of its forward transform */
static void adj_of_to_fourier(const grid* G, const cplx* lz, double* lx) {
  cplx* t = (cplx*)malloc(sizeof(cplx) * G->ncell);
  memcpy(t, lz, sizeof(cplx) * G->ncell);
  dft3(G, t, +1);
  for (int64_t g = 0; g < G->ncell; ++g) lx[g] = creal(t[g]) * (double)G->ncell;
  free(t);
}

/* Mesh half of (dG/dw)^T: push-side mesh adjoints (gphi, A0, A1) -> adjoint
   of J (real, 3 x nc) times q/dV, and the old level's share (lF0h, spectral,
   accumulated when not NULL). */
static void mesh_adjoint(const orc_sim* S, const double* lgphi, const double* lA0r,
                         const double* lA1r, double* mu, cplx* lF0h) {
  const grid* G = &S->G;
  int64_t nc = G->ncell;
  cplx* lphi1 = (cplx*)calloc(nc, sizeof(cplx));
  cplx* lA1h = (cplx*)calloc(3 * nc, sizeof(cplx));
  cplx* lJh = (cplx*)calloc(3 * nc, sizeof(cplx));
  cplx* t = (cplx*)malloc(sizeof(cplx) * nc);
  for (int l = 0; l < 3; ++l) {
    adj_of_to_real(G, lgphi + l * nc, t);  /* gphi_l = Re IDFT(i k_l (phi + phi')/2) */
    for (int64_t g = 0; g < nc; ++g) {
      double k[3];
      mode_k(G, g, k);
      cplx c = -0.5 * I * k[l] * t[g];
      lphi1[g] += c;
      if (lF0h) lF0h[g] += c;
    }
    adj_of_to_real(G, lA1r + l * nc, lA1h + l * nc);
    if (lF0h) {
      adj_of_to_real(G, lA0r + l * nc, t);
      for (int64_t g = 0; g < nc; ++g) lF0h[(2 + l) * nc + g] += t[g];
    }
  }
  cn_adjoint(S, lphi1, NULL, lA1h, NULL, NULL, lF0h, lJh);
  for (int l = 0; l < 3; ++l) {
    adj_of_to_fourier(G, lJh + l * nc, mu + l * nc);
    for (int64_t g = 0; g < nc; ++g) mu[l * nc + g] *= S->q / G->dV;
  }
  free(lphi1);
  free(lA1h);
  free(lJh);
  free(t);
}

/* One step's adjoint.  x, v (3 x np, component-major), w = the converged
   v^{n+1}, F = level-n fields (9 x nc real: phi, psi, A, U, rho); lx1, lv1,
   lF1 = adjoints of x^{n+1}, v^{n+1}, F^{n+1} (any may be NULL = zero).
   Outputs lx0, lv0, lF0.  Returns 0, 1 if the transposed iteration did not
   reach tol within maxit, -1 on a configuration it does not cover. */
int orc_adjoint_step(const orc_sim* S, const double* x, const double* v, const double* w,
                     const double* F, const double* lx1, const double* lv1, const double* lF1,
                     double* lx0, double* lv0, double* lF0, double tol, int maxit,
                     int* iters_out) {
  const grid* G = &S->G;
  if (S->c.r != 2 || !S->c.split || !S->one_species) return -1;
  int64_t np = S->np, nc = G->ncell;
  double dt = S->c.dt, q = S->q, m = S->m;
  double* vb = (double*)malloc(sizeof(double) * 3 * np + 8);
  double* J = (double*)calloc(3 * nc, sizeof(double));
  cplx* Fh = (cplx*)malloc(sizeof(cplx) * 9 * nc);
  cplx* F1h = (cplx*)malloc(sizeof(cplx) * 9 * nc);
  cplx* Jh = (cplx*)malloc(sizeof(cplx) * 3 * nc);
  cplx* t = (cplx*)malloc(sizeof(cplx) * nc);
  double *gphi = (double*)malloc(sizeof(double) * 3 * nc), *A0r = (double*)malloc(sizeof(double) * 3 * nc),
         *A1r = (double*)malloc(sizeof(double) * 3 * nc);
  double *lgphi = (double*)malloc(sizeof(double) * 3 * nc), *lA0 = (double*)malloc(sizeof(double) * 3 * nc),
         *lA1 = (double*)malloc(sizeof(double) * 3 * nc), *mu = (double*)malloc(sizeof(double) * 3 * nc);
  cplx* lF0h = (cplx*)calloc(9 * nc, sizeof(cplx));
  cplx* lJh = (cplx*)calloc(3 * nc, sizeof(cplx));
  double *bw = (double*)malloc(sizeof(double) * 3 * np + 8), *xi = (double*)malloc(sizeof(double) * 3 * np + 8),
         *xn = (double*)malloc(sizeof(double) * 3 * np + 8);
  double* lxacc = (double*)malloc(sizeof(double) * 3 * np + 8);
  piece* buf = (piece*)malloc(sizeof(piece) * MAX_PIECES);
  int status = 0, it = 0;

  /* forward quantities at the converged w */
  for (int64_t i = 0; i < np; ++i) {
    double x0[3], b[3], d[3], qv[3];
    for (int a = 0; a < 3; ++a) {
      x0[a] = x[a * np + i];
      b[a] = 0.5 * (w[a * np + i] + v[a * np + i]);
      vb[a * np + i] = b[a];
      d[a] = dt * b[a];
      qv[a] = q * b[a];
    }
    if (deposit_one(S, x0, d, qv, J, buf) != 0) { status = -1; goto done; }
  }
  for (int f = 0; f < 9; ++f) to_fourier(G, F + f * nc, Fh + f * nc);
  for (int l = 0; l < 3; ++l) to_fourier(G, J + l * nc, Jh + l * nc);
  field_update(S, Jh, Fh, Fh + nc, Fh + 2 * nc, Fh + 5 * nc, Fh + 8 * nc, F1h, F1h + nc,
               F1h + 2 * nc, F1h + 5 * nc, F1h + 8 * nc);
  for (int l = 0; l < 3; ++l) {
    for (int64_t g = 0; g < nc; ++g) {
      double k[3];
      mode_k(G, g, k);
      t[g] = I * k[l] * 0.5 * (F1h[g] + Fh[g]);
    }
    to_real(G, t, gphi + l * nc);
    to_real(G, Fh + (2 + l) * nc, A0r + l * nc);
    to_real(G, F1h + (2 + l) * nc, A1r + l * nc);
  }

  /* adjoints reaching w directly from the outputs */
  if (lF1) {
    cplx* lF1h = (cplx*)malloc(sizeof(cplx) * 9 * nc);
    for (int f = 0; f < 9; ++f) adj_of_to_real(G, lF1 + f * nc, lF1h + f * nc);
    cn_adjoint(S, lF1h, lF1h + nc, lF1h + 2 * nc, lF1h + 5 * nc, lF1h + 8 * nc, lF0h, lJh);
    free(lF1h);
  }
  for (int l = 0; l < 3; ++l) {
    adj_of_to_fourier(G, lJh + l * nc, mu + l * nc);
    for (int64_t g = 0; g < nc; ++g) mu[l * nc + g] *= q / G->dV;
  }
  for (int64_t i = 0; i < np; ++i) {
    double x0[3], b[3], lx[3] = {0, 0, 0}, ld[3] = {0, 0, 0}, lvb[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
      x0[a] = x[a * np + i];
      b[a] = vb[a * np + i];
    }
    if (particle_adjoint(S, x0, b, NULL, mu, NULL, NULL, NULL, lx, ld, lvb, NULL, NULL, NULL)) {
      status = -1;
      goto done;
    }
    for (int a = 0; a < 3; ++a) {
      int64_t id = a * np + i;
      double lxo = lx1 ? lx1[id] : 0.0;
      ld[a] += lxo; /* x' = x + d */
      bw[id] = (lv1 ? lv1[id] : 0.0) + 0.5 * (lvb[a] + dt * ld[a]);
      lxacc[id] = lxo + lx[a];
    }
  }

  /* transposed Picard iteration xi = bw + (dG/dw)^T xi */
  memcpy(xi, bw, sizeof(double) * 3 * np);
  for (it = 1; it <= maxit + 1; ++it) {
    int last = it == maxit + 1;
    memset(lgphi, 0, sizeof(double) * 3 * nc);
    memset(lA0, 0, sizeof(double) * 3 * nc);
    memset(lA1, 0, sizeof(double) * 3 * nc);
    double* lxs = (double*)calloc(3 * np + 1, sizeof(double));
    double* lds = (double*)calloc(3 * np + 1, sizeof(double));
    double* lvbs = (double*)calloc(3 * np + 1, sizeof(double));
    for (int64_t i = 0; i < np; ++i) {
      double x0[3], b[3], eta[3], lx[3] = {0, 0, 0}, ld[3] = {0, 0, 0}, lvb[3] = {0, 0, 0};
      for (int a = 0; a < 3; ++a) {
        x0[a] = x[a * np + i];
        b[a] = vb[a * np + i];
        eta[a] = q / m * xi[a * np + i];
      }
      particle_adjoint(S, x0, b, eta, NULL, gphi, A0r, A1r, lx, ld, lvb, lgphi, lA0, lA1);
      for (int a = 0; a < 3; ++a) {
        lxs[a * np + i] = lx[a];
        lds[a * np + i] = ld[a];
        lvbs[a * np + i] = lvb[a];
      }
    }
    mesh_adjoint(S, lgphi, lA0, lA1, mu, NULL);
    for (int64_t i = 0; i < np; ++i) {
      double x0[3], b[3], lx[3] = {0, 0, 0}, ld[3] = {0, 0, 0}, lvb[3] = {0, 0, 0};
      for (int a = 0; a < 3; ++a) {
        x0[a] = x[a * np + i];
        b[a] = vb[a * np + i];
      }
      particle_adjoint(S, x0, b, NULL, mu, NULL, NULL, NULL, lx, ld, lvb, NULL, NULL, NULL);
      for (int a = 0; a < 3; ++a) {
        lxs[a * np + i] += lx[a];
        lds[a * np + i] += ld[a];
        lvbs[a * np + i] += lvb[a];
      }
    }
    double dmax = 0.0, xmax = 0.0;
    for (int64_t id = 0; id < 3 * np; ++id) {
      xn[id] = bw[id] + 0.5 * (lvbs[id] + dt * lds[id]);
      dmax = fmax(dmax, fabs(xn[id] - xi[id]));
      xmax = fmax(xmax, fabs(xn[id]));
    }
    int conv = dmax <= tol * xmax;
    if (conv || last) {
      /* xi is the fixed point (to tol): collect the inputs' adjoints with it */
      for (int64_t id = 0; id < 3 * np; ++id) lxacc[id] += lxs[id];
      mesh_adjoint(S, lgphi, lA0, lA1, mu, lF0h);
      if (!conv) status = 1;
      free(lxs);
      free(lds);
      free(lvbs);
      break;
    }
    memcpy(xi, xn, sizeof(double) * 3 * np);
    free(lxs);
    free(lds);
    free(lvbs);
  }
  if (lx0) memcpy(lx0, lxacc, sizeof(double) * 3 * np);
  if (lv0)
    for (int64_t id = 0; id < 3 * np; ++id) lv0[id] = 2.0 * xi[id] - (lv1 ? lv1[id] : 0.0);
  if (lF0)
    for (int f = 0; f < 9; ++f) adj_of_to_fourier(G, lF0h + f * nc, lF0 + f * nc);

done:
  if (iters_out) *iters_out = it;
  free(vb); free(J); free(Fh); free(F1h); free(Jh); free(t);
  free(gphi); free(A0r); free(A1r); free(lgphi); free(lA0); free(lA1); free(mu);
  free(lF0h); free(lJh); free(bw); free(xi); free(xn); free(lxacc); free(buf);
  return status;
}

/* P^n = m v^n + q A_h^n(x^n) from the present state (eq. discrete-canonical-relation) */
int orc_rebuild_P(orc_sim* S) {
  const grid* G = &S->G;
  int64_t np = S->np, nc = G->ncell;
  double* A0r = (double*)malloc(sizeof(double) * 3 * nc);
  for (int l = 0; l < 3; ++l) to_real(G, S->A + l * nc, A0r + l * nc);
  for (int64_t i = 0; i < np; ++i) {
    double x0[3], Ax[3];
    for (int a = 0; a < 3; ++a) x0[a] = S->x[a * np + i];
    interp_point(G, S->c.r, x0, A0r, 3, Ax);
    for (int a = 0; a < 3; ++a) S->P[a * np + i] = S->mi[i] * S->v[a * np + i] + S->qi[i] * Ax[a];
  }
  free(A0r);
  return 0;
}

/* gradient of W (eq. field-energy) with respect to the real-space fields
   (9 x nc: phi, psi, A, U, rho) of the present state */
int orc_field_energy_grad(const orc_sim* S, double* lF) {
  const grid* G = &S->G;
  int64_t nc = G->ncell;
  cplx* Eh = (cplx*)malloc(sizeof(cplx) * 3 * nc);
  cplx* Bh = (cplx*)malloc(sizeof(cplx) * 3 * nc);
  cplx* lFh = (cplx*)calloc(9 * nc, sizeof(cplx));
  double* f = (double*)malloc(sizeof(double) * nc);
  cplx* t = (cplx*)malloc(sizeof(cplx) * nc);
  for (int64_t g = 0; g < nc; ++g) {
    double k[3];
    mode_k(G, g, k);
    for (int l = 0; l < 3; ++l) Eh[l * nc + g] = -I * k[l] * S->phi[g] - S->U[l * nc + g];
    Bh[0 * nc + g] = I * (k[1] * S->A[2 * nc + g] - k[2] * S->A[1 * nc + g]);
    Bh[1 * nc + g] = I * (k[2] * S->A[0 * nc + g] - k[0] * S->A[2 * nc + g]);
    Bh[2 * nc + g] = I * (k[0] * S->A[1 * nc + g] - k[1] * S->A[0 * nc + g]);
  }
  for (int l = 0; l < 3; ++l) {
    /* E_l: dW/dE = dV E / sigma1 */
    to_real(G, Eh + l * nc, f);
    for (int64_t g = 0; g < nc; ++g) f[g] *= G->dV / S->c.sigma1;
    adj_of_to_real(G, f, t);
    for (int64_t g = 0; g < nc; ++g) {
      double k[3];
      mode_k(G, g, k);
      lFh[g] += I * k[l] * t[g];         /* E = -i k phi - U */
      lFh[(5 + l) * nc + g] -= t[g];
    }
    /* B_l: dW/dB = dV B / sigma2; B_l = i (k_p A_q - k_q A_p), (l, p, q) cyclic */
    to_real(G, Bh + l * nc, f);
    for (int64_t g = 0; g < nc; ++g) f[g] *= G->dV / S->c.sigma2;
    adj_of_to_real(G, f, t);
    int p = (l + 1) % 3, qq = (l + 2) % 3;
    for (int64_t g = 0; g < nc; ++g) {
      double k[3];
      mode_k(G, g, k);
      lFh[(2 + qq) * nc + g] += -I * k[p] * t[g];
      lFh[(2 + p) * nc + g] += I * k[qq] * t[g];
    }
  }
  for (int fi = 0; fi < 9; ++fi) adj_of_to_fourier(G, lFh + fi * nc, lF + fi * nc);
  free(Eh); free(Bh); free(lFh); free(f); free(t);
  return 0;
}
