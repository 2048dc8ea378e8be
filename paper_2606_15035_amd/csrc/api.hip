// C ABI of the library (declared in include/ecpic.h): configuration checks,
// carving of the caller's device buffers, and the host side of Algorithm 1
// (one Picard pass = scatter, forward FFT, continuity + CN, inverse FFT,
// gather + push, then a read-back of the two fixed-point errors).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "ecpic.h"
#include "internal.hpp"
#include "reduce.hpp"

using namespace ecpic;

namespace {

thread_local std::string g_err;

ecpic_status fail(ecpic_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
ecpic_status fail(ecpic_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ECPIC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));         \
  } while (0)

bool is_pow2(int n) { return n > 0 && (n & (n - 1)) == 0; }

ecpic_status check_config(const ecpic_config* c, int64_t np) {
  if (!c) return fail(ECPIC_EINVAL, "null configuration");
  if (np < 0) return fail(ECPIC_EINVAL, "negative particle count");
  if (np > INT32_MAX)  // particle ids and cell offsets are 32-bit
    return fail(ECPIC_EINVAL, "particle count %lld exceeds 2^31 - 1", (long long)np);
  for (int a = 0; a < 3; ++a) {
    if (!is_pow2(c->n[a]) || c->n[a] < 4 || c->n[a] > 256)
      return fail(ECPIC_EINVAL, "n[%d] = %d must be a power of two in [4, 256]", a, c->n[a]);
    if (!(c->L[a] > 0.0) || !std::isfinite(c->L[a]))
      return fail(ECPIC_EINVAL, "L[%d] must be positive", a);
  }
  if (c->spline_degree < 1 || c->spline_degree > 3)
    return fail(ECPIC_EINVAL, "spline_degree must be 1, 2 or 3");
  if (!(c->dt > 0.0) || !(c->kappa > 0.0) || !(c->sigma1 > 0.0) || !(c->sigma2 > 0.0))
    return fail(ECPIC_EINVAL, "dt, kappa, sigma1, sigma2 must be positive");
  const double lhs = c->sigma1, rhs = c->kappa * c->kappa * c->sigma2;
  if (std::fabs(lhs - rhs) > 1e-13 * std::fmax(std::fabs(lhs), std::fabs(rhs)))
    return fail(ECPIC_EINVAL, "Maxwell scaling sigma1 = kappa^2 sigma2 violated (%g vs %g)", lhs,
                rhs);
  if (c->picard_max < 0 || c->picard_max > 1000) return fail(ECPIC_EINVAL, "picard_max out of range");
  if (!(c->picard_tol >= 0.0)) return fail(ECPIC_EINVAL, "picard_tol must be >= 0");
  const int nq_min = (3 * c->spline_degree + 2) / 2;  // smallest n_q with 2 n_q - 1 >= 3 r
  if (c->split_orbit_at_knots != 0 && c->split_orbit_at_knots != 1)
    return fail(ECPIC_EINVAL, "split_orbit_at_knots must be 0 or 1");
  if (c->quad_points < 0 || c->quad_points > kMaxRule)
    return fail(ECPIC_EINVAL, "quad_points must be in [0, %d]", kMaxRule);
  if (c->split_orbit_at_knots == 1 && c->quad_points != 0 && c->quad_points < nq_min)
    return fail(ECPIC_EINVAL, "quad_points: split pieces need at least %d points (2 n_q - 1 >= 3 r)",
                nq_min);
  if (c->split_orbit_at_knots == 0 && c->precision != ECPIC_FP64)
    return fail(ECPIC_EINVAL, "unsplit orbit integrals are built for FP64 precision only");
  if (c->precision != ECPIC_FP64 && c->precision != ECPIC_MIXED)
    return fail(ECPIC_EINVAL, "precision must be ECPIC_FP64 or ECPIC_MIXED");
  if (!(c->fixed_point_scale >= 0.0) || c->fixed_point_scale > 0x1p52)
    return fail(ECPIC_EINVAL, "fixed_point_scale must be in [0, 2^52] (0 = 2^40)");
  if (c->anderson_depth < 0 || c->anderson_depth > kMaxAnderson)
    return fail(ECPIC_EINVAL, "anderson_depth must be in [0, %d]", kMaxAnderson);
  if (c->scatter_chunk != 0 && c->scatter_chunk != 2048 && c->scatter_chunk != 4096)
    return fail(ECPIC_EINVAL, "scatter_chunk must be 0, 2048 or 4096");
  if (c->spline_degree >= 3 && c->scatter_chunk == 4096)
    return fail(ECPIC_EINVAL, "cubic stencils take 2048-particle scatter chunks");
  return ECPIC_OK;
}

// Gauss-Legendre nodes and weights on [0, 1]: Newton iteration on the
// Legendre polynomial P_n (three-term recurrence) from the Chebyshev-like
// starting guesses cos(pi (i + 3/4) / (n + 1/2)).
QuadRule gauss_rule01(int n) {
  QuadRule R{};
  R.n = n;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) p1 = z, p0 = 1.0;
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // node z on [-1, 1] with weight 2 / ((1 - z^2) P_n'(z)^2), mapped to [0, 1]
    R.s[n - 1 - i] = 0.5 * (1.0 + z);
    R.w[n - 1 - i] = 0.5 * 2.0 / ((1.0 - z * z) * dp * dp);
  }
  return R;
}

int quad_rule_points(const ecpic_config* c) {
  return c->quad_points > 0 ? c->quad_points : (3 * c->spline_degree + 2) / 2;
}

int ilog2i(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

Grid make_grid(const ecpic_config* c) {
  Grid G;
  G.ncell = 1;
  for (int a = 0; a < 3; ++a) {
    G.n[a] = c->n[a];
    G.mask[a] = c->n[a] - 1;
    G.L[a] = c->L[a];
    G.invL[a] = 1.0 / c->L[a];
    G.H[a] = c->L[a] / c->n[a];
    G.invH[a] = 1.0 / G.H[a];
    G.ncell *= c->n[a];
  }
  G.shy = ilog2i(c->n[2]);
  G.shx = G.shy + ilog2i(c->n[1]);
  G.dV = G.H[0] * G.H[1] * G.H[2];
  G.vol = G.L[0] * G.L[1] * G.L[2];
  return G;
}

// Bump allocator over a caller buffer (base may be null when only sizing).
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    return p;
  }
};

// Device workspace of ecpic_adjoint_step_noalloc, for callers that cannot
// allocate: one copy of this array on every GPU the library runs on, held
// until the process ends.  In host code `scratch` is a host-side stand-in;
// its device address on each GPU comes from hipGetSymbolAddress (per device,
// with that device current) and only that address is handed to kernels.
constexpr size_t kStaticScratchBytes = ECPIC_STATIC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved once per device).
ecpic_status static_scratch_address(int* device, void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(ECPIC_EDEVICE, "no usable current device for the static scratch array");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ECPIC_EDEVICE, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                  hipGetErrorString(e));
    g_scratch_addr[dev] = p;
  }
  *device = dev;
  *out = g_scratch_addr[dev];
  return ECPIC_OK;
}

}  // namespace

struct ecpic_sim {
  ecpic_config cfg;
  Grid G;
  int64_t np;
  hipStream_t stream;
  int device = -1;                 // the device current at ecpic_create
  void* static_scratch = nullptr;  // address of `scratch` on that device
  char* state_base = nullptr;      // the caller's state buffer and its carved size
  size_t state_size = 0;
  double q = -1.0, m = 1.0;  // species 0
  int nsp = 1;               // species; > 1: the stores hold one byte per particle
  double qs[kMaxSpecies] = {-1.0}, ms[kMaxSpecies] = {1.0};
  uint8_t* spb[2] = {nullptr, nullptr};  // species bytes of the two stores
  bool initialized = false;
  // particles (state), stored in cell-sorted order; id[i] = caller index.
  // One of the two stores is live (cfg.precision); [1] is the sort's alternate.
  Fp64Store f64[2];
  MixedStore mx[2];
  double *vit, *vnew;  // Picard iterate w_p and image g_p of the current pass (FP64)
  double* vbar = nullptr;  // vbar of the next scatter, written ahead (plain Picard only)
  // 2 (m + 1) buffers of 3 np doubles for the iterates and images that the
  // Anderson mixing of depth m still needs (m = 0: the two of the plain iteration)
  double* apool[2 * (kMaxAnderson + 1)] = {};
  int npool = 0;
  int *id, *id2;
  SortScratch sb;
  unsigned long long* Jfix = nullptr;  // mixed: fixed-point current quanta
  double fix_scale = 0.0;             // quanta per unit of vbar Sbar
  bool mixed() const { return cfg.precision == ECPIC_MIXED; }
  // mesh (state)
  double2* spec[2];  // spectral levels (9 fields each); spec[cur] is level n
  int cur = 0;
  double* gbuf;      // interleaved gather fields
  double* Jb[2];     // orbit current, double-buffered across Picard passes
  int jlast = 0;     // index of the current of the last accepted pass
  bool jclean = true;  // Jb[1 - jlast] is zero (each pass's transform clears the other buffer)
  int chunk = 4096;    // scatter chunk; 2048 once chunks stop fitting the LDS tile
  // workspace
  double2* Jh;
  double2* batch;
  double* realbuf;
  double* Uhalf;
  int* gwork;  // gather work list: [count, indices of blocks whose box missed the LDS tile]
  int* sboxes;  // node boxes of the scatter's chunks, found in a step's first pass
  int* gboxes;  // node boxes of the gather's blocks, likewise
  double2* tw[3];
  Scratch sc;
  double* host = nullptr;  // pinned read-back
  // kernel timing
  int profiling = 0;  // 0 off, 1 every phase, 2 the gather phase only
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  hipEvent_t ev_read = nullptr;  // after each pass's read-back of its errors
  // the step's cell sort as a graph, one per arrangement of the two particle
  // stores and id arrays (they swap at every sort): pointers it was captured
  // with (cur, alt, id, id2, first guess, its vbar) and the executable
  struct SortGraph {
    const void* key[6] = {};
    hipGraphExec_t exec = nullptr;
  } sort_graph[2];
  int next_sort_graph = 0;
  ecpic_profile prof{};
  // Picard passes of the last steps (a ring): the passes every one of them
  // ran are queued ahead of the previous pass's errors
  int pass_hist[8] = {};
  int npass_hist = 0;
  // energy bookkeeping
  double K = 0.0, W = 0.0;
  ecpic_energy en{};
  FieldParams fp() const { return FieldParams{G, cfg.dt, cfg.kappa, cfg.sigma1, cfg.sigma2}; }
  QuadRule rule{};  // rule of the unsplit comparison path
  StepParams pp() const {
    StepParams P{};
    P.G = G;
    P.dt = cfg.dt;
    P.q = q;
    P.m = m;
    P.np = np;
    P.split = cfg.split_orbit_at_knots;
    P.rule = rule;
    // long chunks pay off for the LDS atomics (32^3 two-stream: FP64
    // 0.287 -> 0.245 ms per pass, mixed 0.247 -> 0.239 ms); the wider cubic
    // stencil takes the short ones
    P.chunk = cfg.scatter_chunk > 0 ? cfg.scatter_chunk
                                    : (cfg.spline_degree >= 3 ? 2048 : chunk);
    P.nsp = nsp;
    for (int k = 0; k < kMaxSpecies; ++k) {
      P.qs[k] = qs[k];
      P.ms[k] = ms[k];
      P.cq[k] = mixed() ? qs[k] / q : qs[k] / G.dV;
      P.aq[k] = std::fabs(qs[k]) / G.vol;
    }
    return P;
  }
  // every particle of species (q, m) (the stores hold no species bytes)
  void set_one_species(double q_, double m_) {
    q = q_;
    m = m_;
    nsp = 1;
    for (int k = 0; k < kMaxSpecies; ++k) {
      qs[k] = q_;
      ms[k] = m_;
    }
    for (int k = 0; k < 2; ++k) f64[k].sp = mx[k].sp = nullptr;
  }
};

namespace {

// fn(live store, sort alternate) for the store the configuration selects
template <class Fn>
auto on_store(ecpic_sim* S, Fn&& fn) {
  if (S->mixed()) return fn(S->mx[0], S->mx[1]);
  return fn(S->f64[0], S->f64[1]);
}

void carve(ecpic_sim* S, char* state, char* ws, size_t* state_bytes, size_t* ws_bytes) {
  const int64_t np = S->np, nc = S->G.ncell;
  const size_t n3 = (size_t)3 * (np > 0 ? np : 1);
  const size_t n1 = (size_t)(np > 0 ? np : 1);
  Carver st{state};
  for (int k = 0; k < 2; ++k) {
    if (S->mixed()) {
      S->mx[k].cell = st.take<int>(n1);
      S->mx[k].off = st.take<float>(n3);
      S->mx[k].v = st.take<float>(n3);
      S->mx[k].vp = st.take<float>(n3);
    } else {
      S->f64[k].x = st.take<double>(n3);
      S->f64[k].v = st.take<double>(n3);
      S->f64[k].vp = st.take<double>(n3);
    }
  }
  S->npool = 2 * (S->cfg.anderson_depth + 1);
  for (int k = 0; k < S->npool; ++k) S->apool[k] = st.take<double>(n3);
  S->vit = S->apool[0];
  S->vnew = S->apool[1];
  for (int k = 0; k < 2; ++k) S->spb[k] = st.take<uint8_t>(n1);
  S->id = st.take<int>(n1);
  S->id2 = st.take<int>(n1);
  S->sb.key = st.take<int>(n1);
  S->sb.count = st.take<int>(8 * nc);
  S->sb.offset = st.take<int>(8 * nc + 1);
  S->sb.cursor = st.take<int>(8 * nc);
  S->sb.scan_totals = st.take<int>(sort_scan_blocks(nc));
  S->spec[0] = st.take<double2>(9 * nc);
  S->spec[1] = st.take<double2>(9 * nc);
  S->gbuf = st.take<double>(kGbufStride * nc);
  S->Jb[0] = st.take<double>(3 * nc);
  S->Jb[1] = st.take<double>(3 * nc);
  Carver w{ws};
  S->Jh = w.take<double2>(3 * nc);
  S->batch = w.take<double2>(9 * nc);
  S->realbuf = w.take<double>(9 * nc);
  S->Uhalf = w.take<double>(3 * nc);
  for (int a = 0; a < 3; ++a) S->tw[a] = w.take<double2>(S->G.n[a] / 2);
  S->gwork = w.take<int>(particle_blocks(np) + 1);
  S->sboxes = w.take<int>((size_t)kBoxInts * std::max<int64_t>(scatter_blocks(np, 2048), 1));
  S->gboxes = w.take<int>((size_t)kBoxInts * std::max<int64_t>(particle_blocks(np), 1));
  // the plain iteration's next iterate is the gather's output, so the gather
  // (and the step's set-up) can hand the scatter vbar^p directly
  S->vbar = S->cfg.anderson_depth == 0 ? w.take<double>(n3) : nullptr;
  if (S->mixed()) S->Jfix = w.take<unsigned long long>(3 * nc);
  S->sc.red = w.take<double>(S_NSLOTS);
  S->sc.spread = w.take<double>((size_t)S_NSLOTS * kSpread * kSpreadStride);
  const int64_t maxblk = std::max<int64_t>(
      std::max<int64_t>(particle_blocks(np), scatter_blocks(np, 2048)),
      std::max<int64_t>(mesh_blocks(nc), cn_pencil_blocks(S->G)));
  S->sc.part_stride = std::max<int64_t>((int64_t)kMaxSumValues * (maxblk > 0 ? maxblk : 1),
                                        (int64_t)kAndersonSums * anderson_dot_blocks(3 * np));
  S->sc.part = w.take<double>((size_t)P_NSITES * S->sc.part_stride);
  if (state_bytes) *state_bytes = st.off + 256;
  if (ws_bytes) *ws_bytes = w.off + 256;
}

// Real output descriptors for the inverse transform of the step.
RealIO gather_fields_out(ecpic_sim* S) {
  RealIO io{};
  for (int l = 0; l < 3; ++l) {
    io.p[l] = S->gbuf + l;          // grad_h phi^{n+1/2}
    io.stride[l] = kGbufStride;
    io.p[3 + l] = S->gbuf + 6 + l;  // A^{n+1}
    io.stride[3 + l] = kGbufStride;
  }
  return io;
}

RealIO soa_io(double* base, int64_t nc, int nb) {
  RealIO io{};
  for (int b = 0; b < nb; ++b) {
    io.p[b] = base + b * nc;
    io.stride[b] = 1;
  }
  return io;
}

const double2* const* twp(ecpic_sim* S) { return S->tw; }

// the read-back of red[first .. first + count) into the pinned host buffer,
// queued with an event after it; wait_read() waits for that event only, so
// work queued behind it keeps the GPU busy while the host looks at the values
ecpic_status queue_read(ecpic_sim* S, int first, int count) {
  if (!S->ev_read) HIPCHK(hipEventCreateWithFlags(&S->ev_read, hipEventDisableTiming));
  HIPCHK(hipMemcpyAsync(S->host, S->sc.red + first, sizeof(double) * count, hipMemcpyDeviceToHost,
                        S->stream));
  HIPCHK(hipEventRecord(S->ev_read, S->stream));
  return ECPIC_OK;
}

ecpic_status wait_read(ecpic_sim* S) {
  HIPCHK(hipEventSynchronize(S->ev_read));
  return ECPIC_OK;
}

const void* store_key(const Fp64Store& s) { return s.x; }
const void* store_key(const MixedStore& s) { return s.cell; }

// The step's cell sort (six small kernels, which would otherwise each wait
// for the host's launch on an idle GPU) as one graph launch.  A graph keeps
// the pointers it was captured with, so it is captured once per arrangement
// of the stores, id arrays and first-guess buffers (two alternate), on a
// private stream, and replayed on the simulation's stream; the host then
// swaps the stores and ids as the sort itself does.
template <class PS>
ecpic_status sort_by_graph(ecpic_sim* S, PS& cur, PS& alt) {
  const void* key[6] = {store_key(cur), store_key(alt), S->id, S->id2, S->vit, S->vbar};
  ecpic_sim::SortGraph* g = nullptr;
  for (auto& c : S->sort_graph)
    if (c.exec && std::equal(key, key + 6, c.key)) g = &c;
  if (!g) {
    g = &S->sort_graph[S->next_sort_graph];
    S->next_sort_graph ^= 1;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    g->exec = nullptr;
    hipStream_t cs = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    PS c = cur, a = alt;
    int *i1 = S->id, *i2 = S->id2;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
      launch_sort(cs, S->G, S->np, c, a, i1, i2, S->sb, S->vit, S->vbar);
      e = hipStreamEndCapture(cs, &graph);
    }
    (void)hipStreamDestroy(cs);
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g->exec = nullptr;
      return fail(ECPIC_EDEVICE, "capturing the cell sort as a graph: %s", hipGetErrorString(e));
    }
    std::copy(key, key + 6, g->key);
  }
  HIPCHK(hipGraphLaunch(g->exec, S->stream));
  std::swap(cur, alt);
  std::swap(S->id, S->id2);
  return ECPIC_OK;
}

// Number of Picard passes that every one of the last (up to 8) steps ran;
// 2 without history (a step runs at least passes 0 and 1 unless p_max = 0)
int sure_passes(const ecpic_sim* S) {
  int m = 2;
  if (S->npass_hist > 0) {
    m = S->pass_hist[0];
    for (int k = 1; k < std::min(S->npass_hist, 8); ++k) m = std::min(m, S->pass_hist[k]);
  }
  return std::max(m, 2);
}

ecpic_status sync_read(ecpic_sim* S, int first, int count) {
  HIPCHK(hipMemcpyAsync(S->host, S->sc.red + first, sizeof(double) * count, hipMemcpyDeviceToHost,
                        S->stream));
  HIPCHK(hipStreamSynchronize(S->stream));
  return ECPIC_OK;
}

// forward transform of the 9 real fields in realbuf into spec[cur]; A^n into gbuf
ecpic_status load_fields_from_realbuf(ecpic_sim* S) {
  const int64_t nc = S->G.ncell;
  RealIO in = soa_io(S->realbuf, nc, 9);
  fft3_forward(S->stream, S->G, 9, S->spec[S->cur], &in, nullptr, twp(S), S->sc);
  launch_set_A0(S->stream, nc, S->realbuf + 2 * nc, S->gbuf);
  HIPCHK(hipGetLastError());
  return ECPIC_OK;
}

ecpic_status update_level_energies(ecpic_sim* S) {
  on_store(S, [&](auto& st, auto&) { launch_kinetic(S->stream, S->pp(), st, S->sc); });
  launch_field_energy(S->stream, S->fp(), S->spec[S->cur], S->sc);
  const FinishJob jobs[2] = {{P_K, (int)particle_blocks(S->np), 2, S_K},
                             {P_W, (int)mesh_blocks(S->G.ncell), 1, S_WCUR}};
  launch_finish(S->stream, S->sc, S->np > 0 ? jobs : jobs + 1, S->np > 0 ? 2 : 1);
  HIPCHK(hipGetLastError());
  if (S->np <= 0) launch_fill(S->stream, 2, S->sc.red + S_K, 0.0);
  ecpic_status st = sync_read(S, 0, S_NSLOTS);
  if (st != ECPIC_OK) return st;
  S->K = S->host[S_K];
  S->W = S->host[S_WCUR];
  return ECPIC_OK;
}

}  // namespace

namespace {

// Device workspace of the adjoint step (caller-owned).
struct AdjWs {
  double *vb, *xi, *xn, *b, *lxacc, *lx, *ld, *lvb;  // 3 x np each
  // the step's particles in cell order (x, v, w, and the adjoints lx1, lv1
  // in and lx0, lv0 out; 3 x np each); id: cell order -> caller order
  double *xs, *vs, *ws, *lx1s, *lv1s, *lx0s, *lv0s;
  int *id, *id2;
  SortScratch sb;
  double *J, *gfield, *lg_r, *mu;                     // 3, 6, 9, 3 x ncell (real)
  double2 *Fh, *F1h, *Jh, *inv, *l1, *lg, *lcur, *lJh;  // 9, 9, 3, 6, 9, 9, 9, 3 x ncell
  double* red;                                        // [max|dxi|, max|xi|, bad]
};

size_t carve_adjoint(const Grid& G, int64_t np, char* base, AdjWs* A) {
  const size_t n3 = (size_t)3 * (np > 0 ? np : 1);
  const int64_t nc = G.ncell;
  Carver c{base};
  double** pv[15] = {&A->vb,  &A->xi, &A->xn, &A->b,    &A->lxacc, &A->lx,   &A->ld,  &A->lvb,
                     &A->xs,  &A->vs, &A->ws, &A->lx1s, &A->lv1s,  &A->lx0s, &A->lv0s};
  for (double** q : pv) *q = c.take<double>(n3);
  const size_t n1 = (size_t)(np > 0 ? np : 1);
  A->id = c.take<int>(n1);
  A->id2 = c.take<int>(n1);
  A->sb.key = c.take<int>(n1);
  A->sb.count = c.take<int>(8 * nc);
  A->sb.offset = c.take<int>(8 * nc + 1);
  A->sb.cursor = c.take<int>(8 * nc);
  A->sb.scan_totals = c.take<int>(sort_scan_blocks(nc));
  A->J = c.take<double>(3 * nc);
  A->gfield = c.take<double>(6 * nc);
  A->lg_r = c.take<double>(9 * nc);
  A->mu = c.take<double>(3 * nc);
  A->Fh = c.take<double2>(9 * nc);
  A->F1h = c.take<double2>(9 * nc);
  A->Jh = c.take<double2>(3 * nc);
  A->inv = c.take<double2>(6 * nc);
  A->l1 = c.take<double2>(9 * nc);
  A->lg = c.take<double2>(9 * nc);
  A->lcur = c.take<double2>(9 * nc);
  A->lJh = c.take<double2>(3 * nc);
  A->red = c.take<double>(4);
  return c.off + 256;
}

ecpic_status check_adjoint_config(const ecpic_config* cfg) {
  if (cfg->precision != ECPIC_FP64) return fail(ECPIC_EINVAL, "adjoint: FP64 precision only");
  if (cfg->spline_degree != 2) return fail(ECPIC_EINVAL, "adjoint: spline_degree 2 only");
  if (cfg->split_orbit_at_knots != 1) return fail(ECPIC_EINVAL, "adjoint: split orbits only");
  return ECPIC_OK;
}

// mu = (q/dV) x real part of the unnormalised inverse transform of lJh
// (the adjoint of J given the adjoint of its forward transform); lJh is used up
void current_adjoint(ecpic_sim* S, const AdjWs& A) {
  const int64_t nc = S->G.ncell;
  launch_spec_copy(S->stream, 3 * nc, A.lJh, A.lJh, S->q / S->G.dV);
  RealIO o = soa_io(A.mu, nc, 3);
  fft3_inverse(S->stream, S->G, 3, A.lJh, &o, twp(S));
}

}  // namespace

extern "C" {

ecpic_status ecpic_state_bytes(const ecpic_config* cfg, int64_t n_particles, size_t* state_bytes,
                               size_t* workspace_bytes) {
  ecpic_status st = check_config(cfg, n_particles);
  if (st != ECPIC_OK) return st;
  ecpic_sim S;
  S.cfg = *cfg;
  S.G = make_grid(cfg);
  S.np = n_particles;
  carve(&S, nullptr, nullptr, state_bytes, workspace_bytes);
  return ECPIC_OK;
}

ecpic_status ecpic_create(const ecpic_config* cfg, int64_t n_particles, void* state_dev,
                          size_t state_bytes, void* workspace_dev, size_t workspace_bytes,
                          void* hip_stream, ecpic_sim** out) {
  if (!out) return fail(ECPIC_EINVAL, "null output pointer");
  *out = nullptr;
  ecpic_status st = check_config(cfg, n_particles);
  if (st != ECPIC_OK) return st;
  size_t need_s = 0, need_w = 0;
  ecpic_state_bytes(cfg, n_particles, &need_s, &need_w);
  if (!state_dev || !workspace_dev) return fail(ECPIC_EINVAL, "null device buffer");
  if (state_bytes < need_s || workspace_bytes < need_w)
    return fail(ECPIC_ENOMEM, "buffers too small: need state %zu, workspace %zu", need_s, need_w);
  if ((reinterpret_cast<uintptr_t>(state_dev) & 255) || (reinterpret_cast<uintptr_t>(workspace_dev) & 255))
    return fail(ECPIC_EINVAL, "device buffers must be 256-byte aligned");
  int device = -1;
  void* static_ws = nullptr;
  st = static_scratch_address(&device, &static_ws);
  if (st != ECPIC_OK) return st;
  ecpic_sim* S = new ecpic_sim();
  S->cfg = *cfg;
  S->G = make_grid(cfg);
  S->np = n_particles;
  S->stream = reinterpret_cast<hipStream_t>(hip_stream);
  S->device = device;
  S->static_scratch = static_ws;
  S->fix_scale = cfg->fixed_point_scale > 0.0 ? cfg->fixed_point_scale : 0x1p40;
  S->rule = gauss_rule01(quad_rule_points(cfg));
  carve(S, static_cast<char*>(state_dev), static_cast<char*>(workspace_dev), nullptr, nullptr);
  S->state_base = static_cast<char*>(state_dev);
  S->state_size = need_s;
  if (hipHostMalloc(reinterpret_cast<void**>(&S->host), sizeof(double) * S_NSLOTS,
                    hipHostMallocDefault) != hipSuccess) {
    delete S;
    return fail(ECPIC_ENOMEM, "pinned host allocation failed");
  }
  // twiddles exp(-2 pi i t / N), t < N/2, computed on the host in double
  for (int a = 0; a < 3; ++a) {
    const int N = S->G.n[a];
    std::vector<double2> t(N / 2);
    for (int k = 0; k < N / 2; ++k) {
      const double ang = 2.0 * M_PI * (double)k / (double)N;
      t[k] = make_double2(std::cos(ang), -std::sin(ang));
    }
    if (hipMemcpyAsync(S->tw[a], t.data(), sizeof(double2) * t.size(), hipMemcpyHostToDevice,
                       S->stream) != hipSuccess ||
        hipStreamSynchronize(S->stream) != hipSuccess) {
      (void)hipHostFree(S->host);
      delete S;
      return fail(ECPIC_EDEVICE, "twiddle upload failed");
    }
  }
  if (hipMemsetAsync(S->sc.red, 0, sizeof(double) * S_NSLOTS, S->stream) != hipSuccess ||
      hipMemsetAsync(S->sc.spread, 0, sizeof(double) * S_NSLOTS * kSpread * kSpreadStride,
                     S->stream) != hipSuccess ||
      hipMemsetAsync(S->gwork, 0, sizeof(int) * (particle_blocks(n_particles) + 1), S->stream) !=
          hipSuccess ||
      (S->Jfix && hipMemsetAsync(S->Jfix, 0, sizeof(unsigned long long) * 3 * S->G.ncell,
                                 S->stream) != hipSuccess) ||
      hipStreamSynchronize(S->stream) != hipSuccess) {
    (void)hipHostFree(S->host);
    delete S;
    return fail(ECPIC_EDEVICE, "scratch initialisation failed");
  }
  *out = S;
  return ECPIC_OK;
}

void ecpic_destroy(ecpic_sim* S) {
  if (!S) return;
  for (auto& e : S->ev)
    if (e) (void)hipEventDestroy(e);
  if (S->ev_read) (void)hipEventDestroy(S->ev_read);
  for (auto& g : S->sort_graph)
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (S->host) (void)hipHostFree(S->host);
  delete S;
}

namespace {

// x, v into the store (x wrapped; v^{-1} = v^0), rho^0 and phi^0 (species set)
ecpic_status init_state(ecpic_sim* S, const double* x, const double* v) {
  const int64_t np = S->np, nc = S->G.ncell;
  if (np > 0) {  // through the iterate buffers into the store (x wrapped; v^{-1} = v^0)
    HIPCHK(hipMemcpyAsync(S->vit, x, sizeof(double) * 3 * np, hipMemcpyHostToDevice, S->stream));
    HIPCHK(hipMemcpyAsync(S->vnew, v, sizeof(double) * 3 * np, hipMemcpyHostToDevice, S->stream));
    on_store(S, [&](auto& st, auto&) {
      launch_import(S->stream, S->pp(), st, 0, S->vit);
      launch_import(S->stream, S->pp(), st, 1, S->vnew);
      launch_import(S->stream, S->pp(), st, 2, S->vnew);
    });
  }
  launch_iota(S->stream, np, S->id);
  // rho^0: point-shape deposit, transformed; then the Poisson solve
  launch_fill(S->stream, nc, S->realbuf, 0.0);
  on_store(S, [&](auto& st, auto&) {
    launch_deposit_rho(S->stream, S->cfg.spline_degree, S->pp(), st,
                       CurrentOut{S->realbuf, S->Jfix, S->fix_scale});
  });
  if (S->mixed())
    launch_fixed_current(S->stream, nc, S->Jfix, S->realbuf, S->q / S->G.dV / S->fix_scale);
  RealIO in{};
  in.p[0] = S->realbuf;
  in.stride[0] = 1;
  S->cur = 0;
  fft3_forward(S->stream, S->G, 1, S->spec[0] + 8 * nc, &in, nullptr, twp(S), S->sc);
  launch_poisson_init(S->stream, S->fp(), S->spec[0]);
  launch_fill(S->stream, kGbufStride * nc, S->gbuf, 0.0);
  launch_fill(S->stream, 3 * nc, S->Jb[0], 0.0);
  launch_fill(S->stream, 3 * nc, S->Jb[1], 0.0);
  HIPCHK(hipGetLastError());
  ecpic_status st = update_level_energies(S);
  if (st != ECPIC_OK) return st;
  S->en = ecpic_energy{};
  S->initialized = true;
  return ECPIC_OK;
}

}  // namespace

ecpic_status ecpic_init_particles(ecpic_sim* S, const double* x, const double* v, double q,
                                  double m, double n0) {
  (void)n0;  // a uniform background only changes the k = 0 mode, which is zeroed
  if (!S) return fail(ECPIC_EINVAL, "null simulation");
  if (S->np > 0 && (!x || !v)) return fail(ECPIC_EINVAL, "null particle arrays");
  if (!(m > 0.0) || !std::isfinite(q)) return fail(ECPIC_EINVAL, "invalid q or m");
  S->set_one_species(q, m);
  return init_state(S, x, v);
}

ecpic_status ecpic_init_species(ecpic_sim* S, const double* x, const double* v,
                                const int32_t* species, int32_t nspecies, const double* q,
                                const double* m, double n0) {
  (void)n0;
  if (!S) return fail(ECPIC_EINVAL, "null simulation");
  if (nspecies < 1 || nspecies > kMaxSpecies)
    return fail(ECPIC_EINVAL, "nspecies must be in [1, %d]", kMaxSpecies);
  if (!q || !m) return fail(ECPIC_EINVAL, "null species tables");
  if (S->np > 0 && (!x || !v || !species)) return fail(ECPIC_EINVAL, "null particle arrays");
  for (int k = 0; k < nspecies; ++k)
    if (!(m[k] > 0.0) || !std::isfinite(m[k]) || !std::isfinite(q[k]) || q[k] == 0.0)
      return fail(ECPIC_EINVAL, "species %d: q must be finite and non-zero, m positive", k);
  std::vector<uint8_t> sp(S->np > 0 ? (size_t)S->np : 1, 0);
  for (int64_t i = 0; i < S->np; ++i) {
    if (species[i] < 0 || species[i] >= nspecies)
      return fail(ECPIC_EINVAL, "species[%lld] = %d outside [0, %d)", (long long)i, species[i],
                  nspecies);
    sp[i] = (uint8_t)species[i];
  }
  S->set_one_species(q[0], m[0]);
  if (nspecies > 1) {
    S->nsp = nspecies;
    for (int k = 0; k < nspecies; ++k) {
      S->qs[k] = q[k];
      S->ms[k] = m[k];
    }
    // caller order is the stored order until the first sort
    if (S->np > 0)
      HIPCHK(hipMemcpyAsync(S->spb[0], sp.data(), (size_t)S->np, hipMemcpyHostToDevice,
                            S->stream));
    HIPCHK(hipStreamSynchronize(S->stream));
    S->f64[0].sp = S->mx[0].sp = S->spb[0];
    S->f64[1].sp = S->mx[1].sp = S->spb[1];
  }
  return init_state(S, x, v);
}

namespace {

// a pool buffer that none of a[0..na) and b[0..nb) refers to
double* pool_free(const ecpic_sim* S, double* const* a, int na, double* const* b, int nb) {
  for (int k = 0; k < S->npool; ++k) {
    double* c = S->apool[k];
    bool used = false;
    for (int i = 0; i < na; ++i) used = used || a[i] == c;
    for (int i = 0; i < nb; ++i) used = used || b[i] == c;
    if (!used) return c;
  }
  return nullptr;
}

// put v in front of list (n entries), keeping at most cap of them
void push_front(double** list, int& n, int cap, double* v) {
  n = std::min(n + 1, cap);
  for (int j = n - 1; j > 0; --j) list[j] = list[j - 1];
  list[0] = v;
}

}  // namespace

ecpic_status ecpic_picard_step(ecpic_sim* S, ecpic_step_info* info) {
  if (!S) return fail(ECPIC_EINVAL, "null simulation");
  if (!S->initialized) return fail(ECPIC_ESTATE, "step before init_particles/set_state");
  const int r = S->cfg.spline_degree;
  const int64_t nc = S->G.ncell;
  const StepParams P = S->pp();
  const FieldParams F = S->fp();
  hipStream_t s = S->stream;
  RealIO gout = gather_fields_out(S);
  double2* cur = S->spec[S->cur];
  double2* nxt = S->spec[1 - S->cur];

  const auto t_start = std::chrono::steady_clock::now();
  const bool prof = S->profiling == 1;         // events around every phase
  const bool prof_g = S->profiling != 0;       // events around the gather
  // Iterates w_{p-j} (wl[j]) and images g_{p-j} (gl[j]) of the passes the
  // Anderson mixing still needs, newest first (the plain iteration keeps one
  // of each and takes w_{p+1} = g_p without a copy).
  const int am = S->cfg.anderson_depth;
  const int64_t n3 = 3 * S->np;
  double* wl[kMaxAnderson + 1] = {};
  double* gl[kMaxAnderson + 1] = {};
  int nw = 0, ng = 0;
  push_front(wl, nw, am + 1, S->apool[0]);
  S->vit = wl[0];
  // cell order of x^n, and v^{n+1,0} = 2 v^n - v^{n-1} (written by the sort's
  // permutation when the step sorts)
  const int sort_every = S->cfg.sort_interval <= 0 ? 1 : S->cfg.sort_interval;
  if (S->cfg.sort_interval >= 0 && (S->en.step % sort_every) == 0 && S->np > 0) {
    const ecpic_status st_sort =
        on_store(S, [&](auto& st, auto& alt) { return sort_by_graph(S, st, alt); });
    if (st_sort != ECPIC_OK) return st_sort;
  } else
    on_store(S, [&](auto& st, auto&) { launch_extrapolate(s, S->np, st, S->vit, S->vbar); });
  const CurrentOut cout{nullptr, S->Jfix, S->fix_scale};
  const double fix_unit = S->q / S->G.dV / S->fix_scale;
  const bool fused = fused_field_solve_fits(S->G);
  launch_reset_slots(s, S->sc, S_PIECES, 2);  // pieces, scatter tile misses
  int p = 0, jcur = 1 - S->jlast;
  if (!S->jclean && !S->mixed()) launch_fill(s, 3 * nc, S->Jb[jcur], 0.0);  // after a failed step
  S->jclean = false;
  bool converged = false;
  double err_v = 0.0, err_J = INFINITY;
  // J^{n+1/2,q} of iterate vit_q into Jq (the mixed form through the
  // fixed-point sums)
  auto launch_current = [&](const double* vit_q, double* Jq, int q) {
    on_store(S, [&](auto& st, auto&) {
      CurrentOut o = cout;
      o.J = Jq;
      launch_scatter(s, r, P, st, vit_q, S->vbar, o, S->sc, ChunkBoxes{S->sboxes, q >= 1});
    });
    if (S->mixed()) launch_fixed_current(s, 3 * nc, S->Jfix, Jq, fix_unit);
  };
  // In the plain iteration the next pass's iterate is this pass's output and
  // its vbar has been written by this pass's gather, so the next pass's
  // scatter can be queued before this pass's errors are read (the GPU then
  // does not wait for the host's round trip).  Only passes the step is
  // expected to run are queued so: pass 1, which every step runs, and the
  // passes every one of the last eight steps ran.  If the step stops before
  // such a pass, its current stays in the buffer that the next step clears.
  const int sure = sure_passes(S);
  bool ahead = false;  // this pass's current was queued by the previous pass
  for (p = 0; p <= S->cfg.picard_max; ++p) {
    S->vit = wl[0];
    S->vnew = pool_free(S, wl, nw, gl, std::min(ng, am));
    if (!S->vnew) return fail(ECPIC_EDEVICE, "internal: no free iterate buffer");
    push_front(gl, ng, am + 1, S->vnew);
    // Anderson: differences over mk = min(m, p) passes; one difference is
    // summed by the gather itself, more by a streaming kernel after it
    const int mk = am > 0 && S->np > 0 ? std::min(am, p) : 0;
    AndersonPrev prev{};
    if (mk == 1) {
      prev.w = wl[1];
      prev.g = gl[1];
    }
    double* J = S->Jb[jcur];
    double* Jprev = S->Jb[1 - jcur];
    // J is zero here: the previous pass's transform cleared it (FP64), or the
    // fixed-point conversion overwrites it (mixed); the atomic slots of the
    // pass were cleared when the previous pass's finishing kernel folded them
    if (prof) HIPCHK(hipEventRecord(S->ev[0], s));
    if (!ahead) launch_current(S->vit, J, p);  // J^{n+1/2,p}
    ahead = false;
    if (prof) HIPCHK(hipEventRecord(S->ev[1], s));
    // transform of J (max|J - J_prev| folded into S_DJMAX; J_prev, the next
    // pass's J, cleared in FP64), continuity + CN, inverse transform of
    // grad phi^{n+1/2} and A^{n+1} into the gather buffer
    double* jclear = S->mixed() ? nullptr : Jprev;
    if (fused) {
      field_solve_fused(s, F, J, p >= 1 ? Jprev : nullptr, jclear, cur, nxt, S->Jh, S->batch, gout,
                        twp(S), S->sc);
    } else {
      RealIO jin = soa_io(J, nc, 3);
      fft3_forward(s, S->G, 3, S->Jh, &jin, p >= 1 ? Jprev : nullptr, twp(S), S->sc, jclear);
      launch_cn_update(s, F, cur, S->Jh, nxt, S->batch, S->sc);
      fft3_inverse(s, S->G, 6, S->batch, &gout, twp(S));
    }
    if (prof_g) HIPCHK(hipEventRecord(S->ev[2], s));
    on_store(S, [&](auto& st, auto&) {  // v^{n+1,p+1}
      launch_gather_push(s, r, P, st, S->vit, S->vnew, S->vbar, S->gbuf, S->gwork, S->sc, prev,
                         ChunkBoxes{S->gboxes, p >= 1});
    });
    if (prof_g) HIPCHK(hipEventRecord(S->ev[3], s));
    AndersonVecs av{};
    for (int j = 0; j <= mk; ++j) {
      av.w[j] = wl[j];
      av.g[j] = gl[j];
    }
    if (mk >= 2) launch_anderson_dots(s, mk, n3, av, S->sc);
    {
      const FinishJob jobs[7] = {{P_CN, fused ? cn_pencil_blocks(S->G) : (int)mesh_blocks(nc), 3,
                                  S_JE},
                                 {0, 0, 1, S_DJMAX, F_SPREAD_MAX},
                                 {P_JS, (int)scatter_blocks(S->np, P.chunk), 1, S_JS},
                                 {0, 0, 2, S_DVMAX, F_SPREAD_MAX},
                                 {0, 0, 1, S_BAD, F_SPREAD_MAX},
                                 {0, 0, 2, S_PIECES, F_SPREAD_SUM},
                                 {P_AA,
                                  mk == 1 ? (int)particle_blocks(S->np) : anderson_dot_blocks(n3),
                                  anderson_sums(mk), S_AA}};
      launch_finish(s, S->sc, jobs, S->np > 0 ? (mk > 0 ? 7 : 6) : 2, S->gwork);
    }
    HIPCHK(hipGetLastError());
    ecpic_status st = queue_read(S, S_DVMAX, (S_AA - S_DVMAX) + anderson_sums(mk));
    if (st != ECPIC_OK) return st;
    if (am == 0 && !prof && p + 1 <= S->cfg.picard_max && p + 1 < sure) {
      // w_{p+1} = g_p; Jprev, read by this pass's transform, is the next
      // pass's J (cleared by that transform in FP64, overwritten in mixed)
      launch_current(gl[0], Jprev, p + 1);
      ahead = true;
    }
    st = wait_read(S);
    if (st != ECPIC_OK) return st;
    if (prof) {
      float t01 = 0.f, t12 = 0.f;
      HIPCHK(hipEventElapsedTime(&t01, S->ev[0], S->ev[1]));
      HIPCHK(hipEventElapsedTime(&t12, S->ev[1], S->ev[2]));
      S->prof.ms[0] += t01;
      S->prof.ms[1] += t12;
      S->prof.launches[0] += 1;
      S->prof.launches[1] += 1;
    }
    if (prof_g) {
      float t23 = 0.f;
      HIPCHK(hipEventElapsedTime(&t23, S->ev[2], S->ev[3]));
      S->prof.ms[2] += t23;
      S->prof.launches[2] += 1;
    }
    const double dv = S->host[0], vm = S->host[1], dj = S->host[2], js = S->host[3];
    if (S->host[4] >= 2.0 || S->host[4] != S->host[4])
      return fail(ECPIC_ENONFINITE, "non-finite velocity in Picard pass %d", p);
    if (S->host[4] == 1.5)
      return fail(ECPIC_EINVAL,
                  "a current contribution exceeds 2^50 fixed-point quanta; lower fixed_point_scale");
    if (S->host[4] != 0.0)
      return fail(ECPIC_EINVAL, "an orbit crossed more than %d knots in one step", kMaxPieces - 1);
    if (!std::isfinite(dv) || !std::isfinite(vm) || !std::isfinite(dj) || !std::isfinite(js))
      return fail(ECPIC_ENONFINITE, "non-finite velocity or current in Picard pass %d", p);
    err_v = vm > 0.0 ? dv / vm : dv;
    err_J = p >= 1 ? (js > 0.0 ? dj / js : dj) : INFINITY;
    S->jlast = jcur;
    jcur = 1 - jcur;
    if (p >= 1 && err_v < S->cfg.picard_tol && err_J < S->cfg.picard_tol) {
      converged = true;
      break;
    }
    if (p == S->cfg.picard_max) break;
    double* wnext = gl[0];  // w_{p+1} = g_p
    if (mk > 0) {           // w_{p+1} = g_p - sum_j gamma_j (g_{p-j+1} - g_{p-j})
      AndersonCoef c{};
      anderson_gamma(mk, S->host + (S_AA - S_DVMAX), c.gamma);
      wnext = pool_free(S, wl, am, gl, am + 1);
      if (!wnext) return fail(ECPIC_EDEVICE, "internal: no free iterate buffer");
      launch_anderson_update(s, mk, n3, av, c, wnext);
    }
    push_front(wl, nw, am + 1, wnext);
  }
  if (p > S->cfg.picard_max) p = S->cfg.picard_max;
  // a current queued ahead for a pass the step did not run is left in the
  // buffer the next step deposits into; that step clears it first
  S->jclean = !ahead;
  S->pass_hist[S->npass_hist % 8] = p + 1;
  S->npass_hist += 1;

  // consistency sweep of the accepted iterate (its orbit, current and fields)
  if (prof) HIPCHK(hipEventRecord(S->ev[0], s));
  if (S->cfg.diagnostics) {
    launch_reset_slots(s, S->sc, S_RAMAX, 2);
    launch_half_U(s, S->G, cur, nxt, S->batch);
    RealIO uo = soa_io(S->Uhalf, nc, 3);
    fft3_inverse(s, S->G, 3, S->batch, &uo, twp(S));
    on_store(S, [&](auto& st, auto&) {
      launch_sweep(s, r, P, st, S->vit, S->gbuf, S->Uhalf, S->sc);
    });
  }
  if (prof) HIPCHK(hipEventRecord(S->ev[1], s));
  // accept: x^{n+1} = x^n + dt vbar^p, v^{n-1} <- v^n, v^n <- v^{n+1,p+1}; fields of pass p
  on_store(S, [&](auto& st, auto&) {
    launch_finalize(s, P, st, S->vit, S->vnew, (uint64_t)S->en.step, S->sc);
  });
  if (S->np <= 0) {
    launch_reset_slots(s, S->sc, S_K, 2);
    launch_reset_slots(s, S->sc, S_WORK, 2);
  }
  launch_accept_A(s, nc, S->gbuf);
  if (S->np > 0) {
    const FinishJob jobs[2] = {{P_K, (int)particle_blocks(S->np), 2, S_K},
                               {P_SWEEP, (int)particle_blocks(S->np), 2, S_WORK}};
    launch_finish(s, S->sc, jobs, S->cfg.diagnostics ? 2 : 1);
  }
  if (prof) HIPCHK(hipEventRecord(S->ev[2], s));
  S->cur = 1 - S->cur;
  HIPCHK(hipGetLastError());
  ecpic_status st = sync_read(S, 0, S_NSLOTS);
  if (st != ECPIC_OK) return st;
  const double* h = S->host;
  // long chunks whose node boxes overflow the LDS tile fall back to global
  // atomics; past 1% of the chunks of a step, use the short ones from now on
  if (P.chunk == 4096 && h[S_SMISS] > 0.01 * (p + 1) * (double)scatter_blocks(S->np, 4096))
    S->chunk = 2048;
  if (prof) {
    float ta = 0.f, tb = 0.f;
    HIPCHK(hipEventElapsedTime(&ta, S->ev[0], S->ev[1]));
    HIPCHK(hipEventElapsedTime(&tb, S->ev[1], S->ev[2]));
    if (S->cfg.diagnostics) {
      S->prof.ms[3] += ta;
      S->prof.launches[3] += 1;
    }
    S->prof.ms[4] += tb;
    S->prof.launches[4] += 1;
  }
  if (prof_g) {
    S->prof.pieces += h[S_PIECES];
    S->prof.ms[5] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    S->prof.launches[5] += 1;
  }
  const double K1 = h[S_K], dK = h[S_DK], W1 = h[S_WNEXT], dW = h[S_DW], JE = h[S_JE];
  if (!std::isfinite(K1) || !std::isfinite(W1))
    return fail(ECPIC_ENONFINITE, "non-finite energy after the step");
  S->en.R_field = dW + S->cfg.dt * JE;
  S->en.R_total = dK + dW;
  S->en.JE_mesh = JE;
  if (S->cfg.diagnostics) {
    S->en.work_particle = h[S_WORK];
    S->en.R_particle = dK - S->cfg.dt * h[S_WORK];
    S->en.RA_rms = S->np > 0 ? std::sqrt(h[S_RA2] / (3.0 * S->np)) : 0.0;
    S->en.RA_max = h[S_RAMAX];
    S->en.pou_max = h[S_POU];
  }
  S->en.step += 1;
  S->K = K1;
  S->W = W1;
  if (info) {
    info->iters = p + 1;
    info->converged = converged ? 1 : 0;
    info->err_v = err_v;
    info->err_J = err_J;
  }
  return converged ? ECPIC_OK : ECPIC_ENOCONV;
}

ecpic_status ecpic_field_solve(ecpic_sim* S, const double* J_dev) {
  if (!S) return fail(ECPIC_EINVAL, "null simulation");
  if (!S->initialized) return fail(ECPIC_ESTATE, "field solve before init_particles/set_state");
  const int64_t nc = S->G.ncell;
  hipStream_t s = S->stream;
  const double* J = J_dev ? J_dev : S->Jb[S->jlast];
  if (J_dev) {
    HIPCHK(hipMemcpyAsync(S->Jb[S->jlast], J_dev, sizeof(double) * 3 * nc,
                          hipMemcpyDeviceToDevice, s));
    J = S->Jb[S->jlast];
  }
  RealIO jin = soa_io(const_cast<double*>(J), nc, 3);
  double2* cur = S->spec[S->cur];
  double2* nxt = S->spec[1 - S->cur];
  fft3_forward(s, S->G, 3, S->Jh, &jin, nullptr, twp(S), S->sc);
  launch_cn_update(s, S->fp(), cur, S->Jh, nxt, S->batch, S->sc);
  RealIO gout = gather_fields_out(S);
  fft3_inverse(s, S->G, 6, S->batch, &gout, twp(S));
  launch_accept_A(s, nc, S->gbuf);
  {
    const FinishJob job = {P_CN, (int)mesh_blocks(nc), 3, S_JE};
    launch_finish(s, S->sc, &job, 1);
  }
  S->cur = 1 - S->cur;
  HIPCHK(hipGetLastError());
  ecpic_status st = sync_read(S, 0, S_NSLOTS);
  if (st != ECPIC_OK) return st;
  S->en.R_field = S->host[S_DW] + S->cfg.dt * S->host[S_JE];
  S->en.JE_mesh = S->host[S_JE];
  S->W = S->host[S_WNEXT];
  return ECPIC_OK;
}

ecpic_status ecpic_energy_diagnostics(ecpic_sim* S, ecpic_energy* out) {
  if (!S || !out) return fail(ECPIC_EINVAL, "null argument");
  if (!S->initialized) return fail(ECPIC_ESTATE, "diagnostics before init_particles/set_state");
  const int64_t nc = S->G.ncell;
  hipStream_t s = S->stream;
  launch_reset_slots(s, S->sc, S_GMAX, 2);
  launch_constraint_spectra(s, S->fp(), S->spec[S->cur], S->batch, S->sc);
  RealIO o = soa_io(S->realbuf, nc, 2);
  fft3_inverse(s, S->G, 2, S->batch, &o, twp(S));
  launch_constraint_norms(s, nc, S->realbuf, S->realbuf + nc, S->sc);
  {
    const FinishJob jobs[2] = {{P_W, (int)mesh_blocks(nc), 1, S_WCUR},
                               {P_NORM, (int)mesh_blocks(nc), 2, S_GL2}};
    launch_finish(s, S->sc, jobs, 2);
  }
  HIPCHK(hipGetLastError());
  ecpic_status st = sync_read(S, 0, S_NSLOTS);
  if (st != ECPIC_OK) return st;
  const double* h = S->host;
  S->en.K = S->K;
  S->en.W = h[S_WCUR];
  S->en.E_total = S->en.K + S->en.W;
  S->en.gauge_max = h[S_GMAX];
  S->en.gauss_max = h[S_RMAX];
  S->en.gauge_l2 = std::sqrt(h[S_GL2] / (double)nc);
  S->en.gauss_l2 = std::sqrt(h[S_RL2] / (double)nc);
  *out = S->en;
  return ECPIC_OK;
}

ecpic_status ecpic_get_state(ecpic_sim* S, double* x, double* v, double* vprev, double* fields) {
  if (!S) return fail(ECPIC_EINVAL, "null simulation");
  const int64_t np = S->np, nc = S->G.ncell;
  hipStream_t s = S->stream;
  if (np > 0) {  // store -> FP64 (stored order) -> caller order, through the iterate buffers
    double* dst[3] = {x, v, vprev};
    for (int k = 0; k < 3; ++k) {
      if (!dst[k]) continue;
      on_store(S, [&](auto& st, auto&) { launch_export(s, S->pp(), st, k, S->vnew); });
      launch_to_caller(s, np, S->id, S->vnew, S->vit);
      HIPCHK(hipGetLastError());
      HIPCHK(hipMemcpyAsync(dst[k], S->vit, sizeof(double) * 3 * np, hipMemcpyDefault, s));
      HIPCHK(hipStreamSynchronize(s));
    }
  }
  if (fields) {
    launch_spec_copy(s, 9 * nc, S->spec[S->cur], S->batch, 1.0 / (double)nc);
    RealIO o = soa_io(S->realbuf, nc, 9);
    fft3_inverse(s, S->G, 9, S->batch, &o, twp(S));
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(fields, S->realbuf, sizeof(double) * 9 * nc, hipMemcpyDefault, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  return ECPIC_OK;
}

ecpic_status ecpic_set_state(ecpic_sim* S, const double* x, const double* v, const double* vprev,
                             const double* fields, double q, double m) {
  if (!S) return fail(ECPIC_EINVAL, "null simulation");
  if (m != 0.0 && (!(m > 0.0) || !std::isfinite(q))) return fail(ECPIC_EINVAL, "invalid q or m");
  if (m == 0.0 && !S->initialized)
    return fail(ECPIC_ESTATE, "m = 0 keeps the species, but none were set");
  const int64_t np = S->np, nc = S->G.ncell;
  hipStream_t s = S->stream;
  if (m != 0.0) S->set_one_species(q, m);
  if (np > 0) {  // caller order -> stored order
    if (!S->initialized) launch_iota(s, np, S->id);
    const double* src[3] = {x, v, vprev};
    for (int k = 0; k < 3; ++k) {
      if (!src[k]) continue;
      HIPCHK(hipMemcpyAsync(S->vit, src[k], sizeof(double) * 3 * np, hipMemcpyDefault, s));
      launch_from_caller(s, np, S->id, S->vit, S->vnew);
      on_store(S, [&](auto& st, auto&) { launch_import(s, S->pp(), st, k, S->vnew); });
      HIPCHK(hipGetLastError());
    }
  }
  if (fields) {
    HIPCHK(hipMemcpyAsync(S->realbuf, fields, sizeof(double) * 9 * nc, hipMemcpyDefault, s));
    ecpic_status st = load_fields_from_realbuf(S);
    if (st != ECPIC_OK) return st;
  } else if (!S->initialized) {
    for (int b = 0; b < 2; ++b) launch_spec_copy(s, 9 * nc, S->spec[b], S->spec[b], 0.0);
    launch_fill(s, kGbufStride * nc, S->gbuf, 0.0);
  }
  if (!S->initialized) {
    launch_fill(s, 3 * nc, S->Jb[0], 0.0);
    launch_fill(s, 3 * nc, S->Jb[1], 0.0);
  }
  HIPCHK(hipGetLastError());
  S->initialized = true;
  // the balance terms of the last step no longer describe the state; the step
  // counter (and with it the sort schedule) is kept
  const int64_t step = S->en.step;
  S->en = ecpic_energy{};
  S->en.step = step;
  ecpic_status st = update_level_energies(S);
  if (st != ECPIC_OK) return st;
  return ECPIC_OK;
}

ecpic_status ecpic_get_current(ecpic_sim* S, double* J) {
  if (!S || !J) return fail(ECPIC_EINVAL, "null argument");
  HIPCHK(hipMemcpyAsync(J, S->Jb[S->jlast], sizeof(double) * 3 * S->G.ncell,
                        hipMemcpyDeviceToHost, S->stream));
  HIPCHK(hipStreamSynchronize(S->stream));
  return ECPIC_OK;
}

ecpic_status ecpic_orbit_gather(const ecpic_config* cfg, int64_t n, const double* x0,
                                const double* d, const double* gphi, const double* U,
                                const double* A0, const double* A1, double* out,
                                void* hip_stream) {
  ecpic_status st = check_config(cfg, n);
  if (st != ECPIC_OK) return st;
  if (n > 0 && (!x0 || !d || !gphi || !U || !A0 || !A1 || !out))
    return fail(ECPIC_EINVAL, "null device pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const QuadRule rule = gauss_rule01(quad_rule_points(cfg));
  launch_orbit_gather_soa(s, cfg->spline_degree, cfg->split_orbit_at_knots ? nullptr : &rule,
                          make_grid(cfg), n, x0, d, gphi, U, A0, A1, out);
  HIPCHK(hipGetLastError());
  return ECPIC_OK;
}

ecpic_status ecpic_orbit_deposit(const ecpic_config* cfg, int64_t n, const double* x0,
                                 const double* d, const double* qv, double* J, void* hip_stream) {
  ecpic_status st = check_config(cfg, n);
  if (st != ECPIC_OK) return st;
  if (n > 0 && (!x0 || !d || !qv || !J)) return fail(ECPIC_EINVAL, "null device pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(hip_stream);
  const QuadRule rule = gauss_rule01(quad_rule_points(cfg));
  launch_orbit_deposit_soa(s, cfg->spline_degree, cfg->split_orbit_at_knots ? nullptr : &rule,
                           make_grid(cfg), n, x0, d, qv, J);
  HIPCHK(hipGetLastError());
  return ECPIC_OK;
}

ecpic_status ecpic_set_profiling(ecpic_sim* S, int32_t enable) {
  if (!S) return fail(ECPIC_EINVAL, "null simulation");
  if (enable < 0 || enable > 2) return fail(ECPIC_EINVAL, "profiling level must be 0, 1 or 2");
  if (enable)
    for (auto& e : S->ev)
      if (!e) HIPCHK(hipEventCreate(&e));
  S->profiling = enable;
  S->prof = ecpic_profile{};
  return ECPIC_OK;
}

ecpic_status ecpic_get_profile(ecpic_sim* S, ecpic_profile* out) {
  if (!S || !out) return fail(ECPIC_EINVAL, "null argument");
  *out = S->prof;
  out->scatter_chunk = S->pp().chunk;
  return ECPIC_OK;
}

}  // extern "C"

namespace {

// Header of a checkpoint: what identifies the simulation, where the live
// buffers of the state sit (the sort swaps the two particle stores and id
// arrays), and the host-side bookkeeping; the state buffer follows.
struct CheckpointHeader {
  uint64_t magic;
  char version[32];
  ecpic_config cfg;
  int64_t np;
  size_t state_size;
  int64_t off_f64[2][4];  // x, v, vp, sp of each FP64 store (byte offsets, -1 = none)
  int64_t off_mx[2][5];   // cell, off, v, vp, sp of each mixed store
  int64_t off_id, off_id2;
  int32_t cur, jlast, jclean, chunk, nsp, initialized;
  double q, m, qs[kMaxSpecies], ms[kMaxSpecies], K, W;
  ecpic_energy en;
};
constexpr uint64_t kCheckpointMagic = 0x3143505443504345ull;  // "ECPCTPC1"
constexpr size_t kCheckpointHeaderBytes = (sizeof(CheckpointHeader) + 255) & ~size_t(255);

int64_t offset_in(const ecpic_sim* S, const void* p) {
  return p ? (int64_t)(static_cast<const char*>(p) - S->state_base) : -1;
}
template <class T>
T* at_offset(ecpic_sim* S, int64_t off) {
  return off < 0 ? nullptr : reinterpret_cast<T*>(S->state_base + off);
}

}  // namespace

extern "C" {

ecpic_status ecpic_checkpoint_bytes(ecpic_sim* S, size_t* bytes) {
  if (!S || !bytes) return fail(ECPIC_EINVAL, "null argument");
  *bytes = kCheckpointHeaderBytes + S->state_size;
  return ECPIC_OK;
}

ecpic_status ecpic_checkpoint_save(ecpic_sim* S, void* dst) {
  if (!S || !dst) return fail(ECPIC_EINVAL, "null argument");
  if (!S->initialized) return fail(ECPIC_ESTATE, "checkpoint before init_particles/set_state");
  CheckpointHeader h{};
  h.magic = kCheckpointMagic;
  std::snprintf(h.version, sizeof(h.version), "%s", ecpic_version());
  h.cfg = S->cfg;
  h.np = S->np;
  h.state_size = S->state_size;
  for (int k = 0; k < 2; ++k) {
    const Fp64Store& f = S->f64[k];
    const MixedStore& m = S->mx[k];
    const void* fp[4] = {f.x, f.v, f.vp, f.sp};
    const void* mp[5] = {m.cell, m.off, m.v, m.vp, m.sp};
    for (int j = 0; j < 4; ++j) h.off_f64[k][j] = offset_in(S, fp[j]);
    for (int j = 0; j < 5; ++j) h.off_mx[k][j] = offset_in(S, mp[j]);
  }
  h.off_id = offset_in(S, S->id);
  h.off_id2 = offset_in(S, S->id2);
  h.cur = S->cur;
  h.jlast = S->jlast;
  h.jclean = S->jclean ? 1 : 0;
  h.chunk = S->chunk;
  h.nsp = S->nsp;
  h.initialized = 1;
  h.q = S->q;
  h.m = S->m;
  for (int k = 0; k < kMaxSpecies; ++k) {
    h.qs[k] = S->qs[k];
    h.ms[k] = S->ms[k];
  }
  h.K = S->K;
  h.W = S->W;
  h.en = S->en;
  std::memcpy(dst, &h, sizeof(h));
  HIPCHK(hipMemcpyAsync(static_cast<char*>(dst) + kCheckpointHeaderBytes, S->state_base,
                        S->state_size, hipMemcpyDeviceToHost, S->stream));
  HIPCHK(hipStreamSynchronize(S->stream));
  return ECPIC_OK;
}

ecpic_status ecpic_checkpoint_restore(ecpic_sim* S, const void* src) {
  if (!S || !src) return fail(ECPIC_EINVAL, "null argument");
  CheckpointHeader h;
  std::memcpy(&h, src, sizeof(h));
  if (h.magic != kCheckpointMagic) return fail(ECPIC_EINVAL, "not an ecpic checkpoint");
  if (std::strncmp(h.version, ecpic_version(), sizeof(h.version)) != 0)
    return fail(ECPIC_EINVAL, "checkpoint of library %.32s, this is %s", h.version, ecpic_version());
  if (std::memcmp(&h.cfg, &S->cfg, sizeof(ecpic_config)) != 0 || h.np != S->np ||
      h.state_size != S->state_size)
    return fail(ECPIC_EINVAL, "checkpoint of another configuration or particle count");
  HIPCHK(hipMemcpyAsync(S->state_base, static_cast<const char*>(src) + kCheckpointHeaderBytes,
                        S->state_size, hipMemcpyHostToDevice, S->stream));
  HIPCHK(hipStreamSynchronize(S->stream));
  for (int k = 0; k < 2; ++k) {
    Fp64Store& f = S->f64[k];
    MixedStore& m = S->mx[k];
    f.x = at_offset<double>(S, h.off_f64[k][0]);
    f.v = at_offset<double>(S, h.off_f64[k][1]);
    f.vp = at_offset<double>(S, h.off_f64[k][2]);
    f.sp = at_offset<uint8_t>(S, h.off_f64[k][3]);
    m.cell = at_offset<int>(S, h.off_mx[k][0]);
    m.off = at_offset<float>(S, h.off_mx[k][1]);
    m.v = at_offset<float>(S, h.off_mx[k][2]);
    m.vp = at_offset<float>(S, h.off_mx[k][3]);
    m.sp = at_offset<uint8_t>(S, h.off_mx[k][4]);
  }
  S->id = at_offset<int>(S, h.off_id);
  S->id2 = at_offset<int>(S, h.off_id2);
  S->cur = h.cur;
  S->jlast = h.jlast;
  S->jclean = h.jclean != 0;
  S->chunk = h.chunk;
  S->nsp = h.nsp;
  S->q = h.q;
  S->m = h.m;
  for (int k = 0; k < kMaxSpecies; ++k) {
    S->qs[k] = h.qs[k];
    S->ms[k] = h.ms[k];
  }
  S->K = h.K;
  S->W = h.W;
  S->en = h.en;
  S->initialized = true;
  return ECPIC_OK;
}

const char* ecpic_last_error(void) { return g_err.c_str(); }

ecpic_status ecpic_adjoint_workspace_bytes(const ecpic_config* cfg, int64_t n_particles,
                                           size_t* bytes) {
  if (!bytes) return fail(ECPIC_EINVAL, "null output");
  ecpic_status st = check_config(cfg, n_particles);
  if (st != ECPIC_OK) return st;
  st = check_adjoint_config(cfg);
  if (st != ECPIC_OK) return st;
  AdjWs A;
  *bytes = carve_adjoint(make_grid(cfg), n_particles, nullptr, &A);
  return ECPIC_OK;
}

}  // extern "C"

namespace {

// The adjoint step over a workspace of at least carve_adjoint() bytes
// (checked by the callers); every workspace array is written before it is read.
ecpic_status adjoint_step_impl(ecpic_sim* S, char* workspace, const double* x, const double* v,
                               const double* w, const double* fields, const double* lx1,
                               const double* lv1, const double* lF1, double* lx0, double* lv0,
                               double* lF0, double tol, int32_t max_iters,
                               ecpic_adjoint_info* info) {
  const int64_t np = S->np, nc = S->G.ncell, n3 = 3 * np;
  AdjWs A;
  if (!fields || !lx0 || !lv0 || !lF0 || (np > 0 && (!x || !v || !w)))
    return fail(ECPIC_EINVAL, "null state or output pointer");
  if (!(tol >= 0.0) || max_iters < 0) return fail(ECPIC_EINVAL, "tol >= 0 and max_iters >= 0");
  carve_adjoint(S->G, np, workspace, &A);
  hipStream_t s = S->stream;
  const Grid& G = S->G;
  const FieldParams FP = S->fp();
  StepParams P = S->pp();
  const double dt = S->cfg.dt;

  // The step's particles in cell order for the whole adjoint (x, v and w move
  // together; the particle kernels then work on local chunks), the caller's
  // order restored for lx0 and lv0 at the end.
  if (np > 0) {
    launch_iota(s, np, A.id);
    int* id = A.id;
    int* id2 = A.id2;
    Fp64Store cur{const_cast<double*>(x), const_cast<double*>(v), const_cast<double*>(w)};
    Fp64Store alt{A.xs, A.vs, A.ws};
    launch_sort(s, G, np, cur, alt, id, id2, A.sb);
    A.id = id;  // the ids of the sorted copies (cur now views A.xs, A.vs, A.ws)
    x = cur.x;
    v = cur.v;
    w = cur.vp;
    if (lx1) {
      launch_from_caller(s, np, A.id, lx1, A.lx1s);
      lx1 = A.lx1s;
    }
    if (lv1) {
      launch_from_caller(s, np, A.id, lv1, A.lv1s);
      lv1 = A.lv1s;
    }
  }

  // forward quantities of the converged iterate: J, the level n+1 spectra,
  // grad_h phi^{n+1/2} and A^{n+1} (A^n is the fields' A rows)
  launch_vbar(s, n3, w, v, A.vb);
  launch_fill(s, 3 * nc, A.J, 0.0);
  launch_reset_slots(s, S->sc, S_BAD, 1);
  {
    Fp64Store view{const_cast<double*>(x), const_cast<double*>(v), nullptr};
    launch_scatter(s, 2, P, view, w, nullptr, CurrentOut{A.J, nullptr, 0.0}, S->sc);
  }
  RealIO jin = soa_io(A.J, nc, 3);
  fft3_forward(s, G, 3, A.Jh, &jin, nullptr, twp(S), S->sc);
  RealIO fin = soa_io(const_cast<double*>(fields), nc, 9);
  fft3_forward(s, G, 9, A.Fh, &fin, nullptr, twp(S), S->sc);
  launch_cn_update(s, FP, A.Fh, A.Jh, A.F1h, A.inv, S->sc);
  RealIO gout = soa_io(A.gfield, nc, 6);
  fft3_inverse(s, G, 6, A.inv, &gout, twp(S));
  const double* gphi = A.gfield;
  const double* A1r = A.gfield + 3 * nc;
  const double* A0r = fields + 2 * nc;

  AdjParticleArgs PA{G, dt, S->q / S->m, np, x, A.vb, A.xi, A.mu, gphi, A0r, A1r,
                     A.lx, A.ld, A.lvb, A.lg_r, A.lg_r + 6 * nc, A.lg_r + 3 * nc, A.red + 2};
  launch_fill(s, 4, A.red, 0.0);

  // adjoints reaching w straight from the outputs
  launch_fill(s, 2 * 9 * nc, reinterpret_cast<double*>(A.lcur), 0.0);
  if (lF1) {
    RealIO l1in = soa_io(const_cast<double*>(lF1), nc, 9);
    fft3_forward(s, G, 9, A.l1, &l1in, nullptr, twp(S), S->sc);
    launch_spec_copy(s, 9 * nc, A.l1, A.l1, 1.0 / (double)nc);
  }
  launch_cn_adjoint(s, FP, lF1 ? A.l1 : nullptr, nullptr, A.lcur, A.lJh);
  current_adjoint(S, A);
  for (double* p : {A.lx, A.ld, A.lvb}) launch_fill(s, n3, p, 0.0);
  launch_particle_adjoint(s, PA, false, true);
  launch_adjoint_rhs(s, n3, dt, lx1, lv1, A.lx, A.ld, A.lvb, A.b, A.lxacc);
  if (n3 > 0)
    HIPCHK(hipMemcpyAsync(A.xi, A.b, sizeof(double) * n3, hipMemcpyDeviceToDevice, s));

  // transposed Picard iteration
  int it = 0;
  bool conv = false;
  double err = 0.0;
  for (it = 1; it <= max_iters + 1; ++it) {
    for (double* p : {A.lx, A.ld, A.lvb}) launch_fill(s, n3, p, 0.0);
    launch_fill(s, 9 * nc, A.lg_r, 0.0);
    PA.xi = A.xi;
    launch_particle_adjoint(s, PA, true, false);
    RealIO lgin = soa_io(A.lg_r, nc, 9);  // [grad phi, A^{n+1}, A^n]
    fft3_forward(s, G, 9, A.lg, &lgin, nullptr, twp(S), S->sc);
    launch_spec_copy(s, 9 * nc, A.lg, A.lg, 1.0 / (double)nc);
    launch_cn_adjoint(s, FP, nullptr, A.lg, nullptr, A.lJh);
    current_adjoint(S, A);
    launch_particle_adjoint(s, PA, false, true);
    launch_fill(s, 2, A.red, 0.0);
    launch_adjoint_update(s, n3, dt, A.b, A.lvb, A.ld, A.xi, A.xn, A.red);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(S->host, A.red, sizeof(double) * 3, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double dm = S->host[0], xm = S->host[1];
    if (S->host[2] != 0.0)
      return fail(ECPIC_EINVAL, "adjoint: an orbit crossed more than %d knots", kMaxPieces - 1);
    if (!std::isfinite(dm) || !std::isfinite(xm))
      return fail(ECPIC_ENONFINITE, "adjoint: non-finite iterate at iteration %d", it);
    err = xm > 0.0 ? dm / xm : dm;
    conv = dm <= tol * xm;
    if (conv || it == max_iters + 1) {
      // the inputs' adjoints from this xi: the push's mesh share of level n
      launch_cn_adjoint(s, FP, nullptr, A.lg, A.lcur, A.lJh);
      launch_adjoint_out(s, n3, A.lxacc, A.lx, A.xi, lv1, A.lx0s, A.lv0s);
      launch_to_caller(s, np, A.id, A.lx0s, lx0);
      launch_to_caller(s, np, A.id, A.lv0s, lv0);
      RealIO fo = soa_io(lF0, nc, 9);
      fft3_inverse(s, G, 9, A.lcur, &fo, twp(S));
      break;
    }
    std::swap(A.xi, A.xn);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  if (info) {
    info->iters = it;
    info->converged = conv ? 1 : 0;
    info->err = err;
  }
  return conv ? ECPIC_OK : ECPIC_ENOCONV;
}

ecpic_status check_adjoint_call(ecpic_sim* S) {
  if (!S) return fail(ECPIC_EINVAL, "null simulation");
  ecpic_status st = check_adjoint_config(&S->cfg);
  if (st != ECPIC_OK) return st;
  if (S->nsp != 1) return fail(ECPIC_EINVAL, "adjoint: one particle species only");
  return ECPIC_OK;
}

}  // namespace

extern "C" {

ecpic_status ecpic_adjoint_step(ecpic_sim* S, void* workspace, size_t workspace_bytes,
                                const double* x, const double* v, const double* w,
                                const double* fields, const double* lx1, const double* lv1,
                                const double* lF1, double* lx0, double* lv0, double* lF0,
                                double tol, int32_t max_iters, ecpic_adjoint_info* info) {
  ecpic_status st = check_adjoint_call(S);
  if (st != ECPIC_OK) return st;
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return fail(ECPIC_EINVAL, "adjoint workspace must be non-null and 256-byte aligned");
  AdjWs A;
  if (carve_adjoint(S->G, S->np, nullptr, &A) > workspace_bytes)
    return fail(ECPIC_ENOMEM, "adjoint workspace too small");
  return adjoint_step_impl(S, static_cast<char*>(workspace), x, v, w, fields, lx1, lv1, lF1, lx0,
                           lv0, lF0, tol, max_iters, info);
}

ecpic_status ecpic_adjoint_step_noalloc(ecpic_sim* S, const double* x, const double* v,
                                        const double* w, const double* fields, const double* lx1,
                                        const double* lv1, const double* lF1, double* lx0,
                                        double* lv0, double* lF0, double tol, int32_t max_iters,
                                        ecpic_adjoint_info* info) {
  ecpic_status st = check_adjoint_call(S);
  if (st != ECPIC_OK) return st;
  AdjWs A;
  const size_t need = carve_adjoint(S->G, S->np, nullptr, &A);
  if (need > kStaticScratchBytes)
    return fail(ECPIC_ENOMEM,
                "adjoint workspace of %zu bytes exceeds the %zu-byte static scratch array; "
                "use ecpic_adjoint_step with a caller workspace",
                need, kStaticScratchBytes);
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != S->device)
    return fail(ECPIC_EINVAL, "the device of ecpic_create (%d) must be current (is %d)", S->device,
                dev);
  return adjoint_step_impl(S, static_cast<char*>(S->static_scratch), x, v, w, fields, lx1, lv1,
                           lF1, lx0, lv0, lF0, tol, max_iters, info);
}

ecpic_status ecpic_field_energy_grad(ecpic_sim* S, double* lF) {
  if (!S || !lF) return fail(ECPIC_EINVAL, "null argument");
  if (!S->initialized) return fail(ECPIC_ESTATE, "field energy gradient before a state is set");
  const int64_t nc = S->G.ncell;
  hipStream_t s = S->stream;
  // E, B as real fields scaled by dV / sigma (dW/dE, dW/dB), via the batch buffers
  launch_fields_EB(s, S->G, S->spec[S->cur], S->batch);
  launch_spec_copy(s, 3 * nc, S->batch, S->batch, S->G.dV / S->cfg.sigma1);
  launch_spec_copy(s, 3 * nc, S->batch + 3 * nc, S->batch + 3 * nc, S->G.dV / S->cfg.sigma2);
  RealIO eb = soa_io(S->realbuf, nc, 6);
  fft3_inverse(s, S->G, 6, S->batch, &eb, twp(S));
  fft3_forward(s, S->G, 6, S->batch, &eb, nullptr, twp(S), S->sc);
  launch_spec_copy(s, 6 * nc, S->batch, S->batch, 1.0 / (double)nc);
  launch_energy_adjoint(s, S->G, S->batch, S->batch);  // 6 -> 9 spectra in place
  RealIO out = soa_io(S->realbuf, nc, 9);
  fft3_inverse(s, S->G, 9, S->batch, &out, twp(S));
  HIPCHK(hipMemcpyAsync(lF, S->realbuf, sizeof(double) * 9 * nc, hipMemcpyDeviceToDevice, s));
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return ECPIC_OK;
}

const char* ecpic_version(void) { return "ecpic-gfx950 0.24"; }

}  // extern "C"

namespace {

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

// smallest elapsed time (ms) of `repeats` launches of f on s, after one
// untimed launch
template <class F>
ecpic_status best_launch_ms(hipStream_t s, const EventPair& ev, int repeats, F&& f,
                            float* best) {
  f();
  HIPCHK(hipGetLastError());
  *best = INFINITY;
  for (int k = 0; k < repeats; ++k) {
    HIPCHK(hipEventRecord(ev.a, s));
    f();
    HIPCHK(hipEventRecord(ev.b, s));
    HIPCHK(hipEventSynchronize(ev.b));
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, ev.a, ev.b));
    *best = std::min(*best, ms);
  }
  HIPCHK(hipGetLastError());
  return ECPIC_OK;
}

}  // namespace

extern "C" {

ecpic_status ecpic_measure_peaks(void* buffer, size_t bytes, int32_t repeats, void* hip_stream,
                                 double* fp64_tflops, double* hbm_gbs) {
  if (!buffer || !fp64_tflops || !hbm_gbs) return fail(ECPIC_EINVAL, "null argument");
  if (bytes < ((size_t)64 << 20))
    return fail(ECPIC_EINVAL, "the copy needs a buffer of at least 64 MiB (%zu bytes given)",
                bytes);
  if (repeats < 1) return fail(ECPIC_EINVAL, "repeats must be at least 1");
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  int dev = 0, cus = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  EventPair ev;
  HIPCHK(hipEventCreate(&ev.a));
  HIPCHK(hipEventCreate(&ev.b));
  // 32 workgroups of 256 lanes per compute unit, several rounds of resident
  // waves (with one round, 8 per SIMD, uneven placement cost a fifth)
  const int fma_blocks = 32 * std::max(cus, 1);
  float ms = 0.f;
  ecpic_status st = best_launch_ms(
      s, ev, repeats, [&] { launch_fma_peak(s, fma_blocks, static_cast<double*>(buffer)); }, &ms);
  if (st != ECPIC_OK) return st;
  *fp64_tflops = fma_peak_flops(fma_blocks) / (ms * 1e-3) / 1e12;
  // the first half of the buffer copied into the second, both 256-byte aligned
  const size_t half = (bytes / 2) & ~(size_t)255;
  const char* src = static_cast<const char*>(buffer);
  char* dst = static_cast<char*>(buffer) + half;
  const int copy_blocks = 256 * std::max(cus, 1);
  st = best_launch_ms(
      s, ev, repeats,
      [&] { launch_stream_copy(s, copy_blocks, src, dst, (int64_t)(half / 16)); }, &ms);
  if (st != ECPIC_OK) return st;
  *hbm_gbs = 2.0 * (double)half / (ms * 1e-3) / 1e9;
  return ECPIC_OK;
}

}  // extern "C"
