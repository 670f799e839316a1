// wp_capi.cpp -- C ABI of libwavepacket: argument checking, per-axis tables,
// the pass schedule of a step, and observables.  See include/wavepacket.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <new>
#include <string>
#include <vector>

#include "../../include/wavepacket.h"
#include "wp_internal.hpp"
#include "wp_stage.hpp"

using wp::cx;

struct wp_sim {
  wp_grid_desc g{};
  wp_potential_desc p{};
  hipStream_t stream = nullptr;
  int device = 0;
  int lg[3] = {0, 0, 0};
  // Axes the line passes see: lg, except on a split 1D grid (more than
  // kMaxLine1D points), which is transformed as [n1][n2] = [2^vlg[0]][2^vlg[1]].
  bool split = false;
  // Some axis length is not a power of two: every pass runs the mixed-radix
  // kernels with the per-axis stage plans below.
  bool mixed = false;
  wp::GPlan plan[3] = {};
  // 3D power-of-two grids: the middle passes of a step (y forward, z
  // kinetic, y inverse) run on 2^slab_lg slabs of consecutive x planes, so
  // that a slab stays in the memory-side cache between the three passes.
  // Even slabs run on `stream`, odd ones on `side` (created on first use),
  // forked after the first-axis pass and joined before the next one by the
  // two events, so that one slab's passes fill the gaps and tails of the
  // other's.
  int slab_lg = 0;
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // Moment partials of the closing pass (wp_propagate_observe): set for the
  // duration of one schedule, one 8-slot row per workgroup of that pass.
  double *moments = nullptr;
  double *d_mpart = nullptr;
  int64_t mpart_rows = 0;
  int vdim = 1;
  int vlg[3] = {0, 0, 0};
  int64_t total = 0;
  int64_t pitch = 0;  // points between first-axis planes in storage
  int prec = 2;
  void *psi = nullptr;
  bool psi_owned = false;
  uint64_t psi_bytes = 0;
  void *scratch = nullptr;  // momentum-space copy for the energy
  void *ref = nullptr;      // reference state of the autocorrelation
  cx<double> *d_kfull = nullptr, *d_khalf = nullptr;  // n0+n1+n2 entries each
  double *d_k2 = nullptr;                              // k^2 per axis, n0+n1+n2
  cx<double> *d_tw[3] = {nullptr, nullptr, nullptr};
  double *d_partials = nullptr, *d_out8 = nullptr;
  double *d_coef = nullptr;  // waveform values for up to kCoefChunk steps
  cx<double> *d_gauss = nullptr;  // per-axis factors of the last Gaussian state
  hipEvent_t ev_gauss = nullptr;   // recorded after the kernel that reads d_gauss
  cx<double> *d_wsplit = nullptr;  // split 1D: exp(-2 pi i e/n) as [n2] high and [n1] low factors
  int obs_blocks = 1;
  double t0 = 0.0;
  uint64_t step = 0;
  int32_t order = WP_ORDER_VKV;
  wp::GridDev gd{};
  wp::PotDev pd{};
  std::string err;
};

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

bool is_pow2(uint64_t n) { return n >= 1 && (n & (n - 1)) == 0; }
int ilog2(uint64_t n) {
  int l = 0;
  while ((uint64_t(1) << l) < n) ++l;
  return l;
}

wp_status fail(wp_sim *s, wp_status code, const std::string &msg) {
  if (s) s->err = msg;
  return code;
}

wp_status hip_fail(wp_sim *s, hipError_t e, const char *what) {
  return fail(s, WP_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool wave_ok(const wp_waveform &w) {
  if (w.kind < WP_WAVE_CONST || w.kind > WP_WAVE_SIN2_COS) return false;
  const double v[] = {w.A0, w.A1, w.omega, w.phase, w.tc, w.tau, w.ti, w.tf};
  for (double x : v)
    if (!std::isfinite(x)) return false;
  if (w.kind == WP_WAVE_GAUSS_COS && w.tau == 0.0) return false;
  if (w.kind == WP_WAVE_SIN2_COS && !(w.tf > w.ti)) return false;
  return true;
}

// Returns an empty string when the descriptor is valid.
std::string check_grid(const wp_grid_desc *g) {
  if (!g) return "grid descriptor is NULL";
  if (g->ndim < 1 || g->ndim > 3) return "ndim must be 1, 2 or 3";
  if (g->prec != WP_C64 && g->prec != WP_C128 && g->prec != WP_C64X) return "prec must be WP_C64, WP_C64X or WP_C128";
  for (int d = 0; d < 3; ++d) {
    if (d < g->ndim) {
      if (g->n[d] < 2) return "n on a used axis must be >= 2";
      if (!std::isfinite(g->lo[d]) || !std::isfinite(g->hi[d]) || !(g->hi[d] > g->lo[d]))
        return "each used axis needs finite lo < hi";
    } else if (g->n[d] != 1) {
      return "unused axes must have n = 1";
    }
  }
  if (!(g->mass > 0) || !std::isfinite(g->mass)) return "mass must be finite and > 0";
  if (!(g->hbar > 0) || !std::isfinite(g->hbar)) return "hbar must be finite and > 0";
  if (!(g->dt != 0) || !std::isfinite(g->dt)) return "dt must be finite and nonzero";
  return "";
}

std::string check_pot(const wp_potential_desc *p) {
  if (!p) return "potential descriptor is NULL";
  for (int d = 0; d < 3; ++d)
    if (!wave_ok(p->a[d]) || !wave_ok(p->b[d])) return "invalid waveform in a[] or b[]";
  if (!wave_ok(p->c) || !wave_ok(p->s)) return "invalid waveform c or s";
  if (p->v0_kind < WP_V0_NONE || p->v0_kind > WP_V0_MORSE) return "unknown v0_kind";
  for (double x : p->v0_par)
    if (!std::isfinite(x)) return "v0_par must be finite";
  return "";
}

// Prime factors 2, 3, 5, 7 only.
bool smooth7(uint64_t n) {
  for (uint64_t p : {2u, 3u, 5u, 7u})
    while (n % p == 0) n /= p;
  return n == 1;
}

std::string check_supported(const wp_grid_desc *g) {
  bool mixed = false;
  for (int d = 0; d < g->ndim; ++d) mixed = mixed || !is_pow2(g->n[d]);
  if (mixed) {
    for (int d = 0; d < g->ndim; ++d)
      if (!smooth7(g->n[d]) || g->n[d] > (uint64_t)wp::kMaxMixed)
        return "axis lengths that are not powers of two must have prime factors 2, 3, 5, 7 only and at most 4096 points";
    return "";
  }
  if (g->ndim == 1) {
    if (g->n[0] > (uint64_t)wp::kMaxSplit1D) return "1D grids are limited to 2^20 points in this build";
  } else {
    for (int d = 0; d < g->ndim; ++d)
      if (g->n[d] > (uint64_t)wp::kMaxLinePass) return "2D/3D axes are limited to 4096 points in this build";
  }
  return "";
}

double spacing(const wp_grid_desc &g, int d) { return (g.hi[d] - g.lo[d]) / (double)g.n[d]; }

// Wavenumber of DFT bin m (Section 2.1 momentum grid, k = p/hbar): m for
// m < n/2, m - n otherwise.
double wavenumber(const wp_grid_desc &g, int d, uint64_t m) {
  const int64_t n = (int64_t)g.n[d];
  const int64_t mm = (2 * (int64_t)m < n) ? (int64_t)m : (int64_t)m - n;
  return 2.0 * kPi * (double)mm / ((double)n * spacing(g, d));
}

// Twiddles of an n-point line transform in stage order: after a first
// stage of radix r0 (2, 4 or 8) come radix-8 stages with Ls = r0, 8 r0, ...;
// stage Ls holds exp(-2 pi i r k/(8 Ls)) at (r-1)*Ls + k, 1 <= r < 8, k < Ls.
std::vector<cx<double>> stage_twiddles(uint64_t n) {
  std::vector<cx<double>> tw;
  if (n > 8) {
    const int lg = ilog2(n);
    const uint64_t r0 = (lg % 3 == 0) ? 8 : (uint64_t(1) << (lg % 3));
    for (uint64_t ls = r0; ls < n; ls *= 8)
      for (uint64_t r = 1; r < 8; ++r)
        for (uint64_t k = 0; k < ls; ++k) {
          const double ang = 2.0 * kPi * (double)(r * k) / (double)(8 * ls);
          tw.push_back({std::cos(ang), -std::sin(ang)});
        }
  }
  if (tw.empty()) tw.push_back({1.0, 0.0});
  return tw;
}

// Stage plan and stage-ordered twiddles of a mixed-radix line transform of
// n points (radix 8 first while 8 divides, then 4 or 2, then 3, 5, 7); stage
// s with product LS of the earlier radices owns (radix - 1) LS entries
// exp(-2 pi i r k/(radix LS)) at twoff + (r - 1) LS + k.
std::vector<cx<double>> mixed_plan(uint64_t n, wp::GPlan *plan) {
  std::vector<int> rad;
  uint64_t m = n;
  while (m % 8 == 0 && m > 1) rad.push_back(8), m /= 8;
  while (m % 4 == 0) rad.push_back(4), m /= 4;
  while (m % 2 == 0) rad.push_back(2), m /= 2;
  for (int p : {3, 5, 7})
    while (m % p == 0) rad.push_back(p), m /= p;
  std::vector<cx<double>> tw;
  *plan = wp::GPlan{};
  plan->nst = (int32_t)rad.size();
  uint64_t ls = 1;
  for (size_t st = 0; st < rad.size(); ++st) {
    const uint64_t R = (uint64_t)rad[st];
    plan->radix[st] = (int32_t)R;
    plan->ls[st] = (int32_t)ls;
    plan->twoff[st] = (int32_t)tw.size();
    for (uint64_t r = 1; r < R; ++r)
      for (uint64_t k = 0; k < ls; ++k) {
        const double ang = 2.0 * kPi * (double)((r * k) % (R * ls)) / (double)(R * ls);
        tw.push_back({std::cos(ang), -std::sin(ang)});
      }
    ls *= R;
  }
  if (tw.empty()) tw.push_back({1.0, 0.0});
  return tw;
}

wp::WaveDev to_dev(const wp_waveform &w) {
  wp::WaveDev d;
  d.kind = w.kind;
  d.A0 = w.A0; d.A1 = w.A1; d.omega = w.omega; d.phase = w.phase;
  d.tc = w.tc; d.tau = w.tau; d.ti = w.ti; d.tf = w.tf;
  return d;
}

// Tables are copied to the device on a stream of the library's own (one per
// device, created on first use, kept for the life of the process).  A copy
// from pageable host memory completes before the call returns; on the
// caller's stream it would first wait for every kernel queued there, which
// would stall a caller that creates handles while others compute.
hipError_t upload_stream(hipStream_t *out) {
  static std::mutex mu;
  static std::map<int, hipStream_t> streams;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  auto it = streams.find(dev);
  if (it == streams.end()) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    it = streams.emplace(dev, st).first;
  }
  *out = it->second;
  return hipSuccess;
}

// Copy host data into a device array; complete when this returns.
hipError_t copy_in(void *dst, const void *src, size_t bytes) {
  hipStream_t us = nullptr;
  hipError_t e = upload_stream(&us);
  if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, us);
  if (e == hipSuccess) e = hipStreamSynchronize(us);
  return e;
}

// Allocations whose failure the caller reports through its status: a
// failed call also leaves its error in the runtime's per-thread last-error
// slot, which a later successful launch (checked with hipGetLastError)
// would otherwise report as its own.
hipError_t dev_alloc(void **p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
  }
  return e;
}

hipError_t host_alloc(void **p, size_t bytes) {
  hipError_t e = hipHostMalloc(p, bytes, hipHostMallocDefault);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
  }
  return e;
}

// Allocate and fill a device array (complete when this returns).
template <class T>
hipError_t upload(T **dst, const std::vector<T> &src) {
  hipError_t e = dev_alloc((void **)dst, sizeof(T) * src.size());
  if (e != hipSuccess) return e;
  return copy_in(*dst, src.data(), sizeof(T) * src.size());
}

uint64_t table_bytes(const wp_grid_desc &g) {
  uint64_t axes = g.n[0] + g.n[1] + g.n[2];
  return axes * (16 + 16 + 8 + 16) + 1024 * 8 * 8 + 64 + 8 * wp::CO_COUNT * wp::kCoefChunk;
}

void release(wp_sim *s) {
  if (s->psi_owned && s->psi) (void)hipFree(s->psi);
  if (s->scratch) (void)hipFree(s->scratch);
  if (s->ref) (void)hipFree(s->ref);
  if (s->d_kfull) (void)hipFree(s->d_kfull);
  if (s->d_khalf) (void)hipFree(s->d_khalf);
  if (s->d_k2) (void)hipFree(s->d_k2);
  for (auto &p : s->d_tw)
    if (p) (void)hipFree(p);
  if (s->d_partials) (void)hipFree(s->d_partials);
  if (s->d_out8) (void)hipFree(s->d_out8);
  if (s->d_coef) (void)hipFree(s->d_coef);
  if (s->d_gauss) (void)hipFree(s->d_gauss);
  if (s->ev_gauss) (void)hipEventDestroy(s->ev_gauss);
  if (s->d_wsplit) (void)hipFree(s->d_wsplit);
  if (s->d_mpart) (void)hipFree(s->d_mpart);
  if (s->side) (void)hipStreamDestroy(s->side);
  if (s->ev_fork) (void)hipEventDestroy(s->ev_fork);
  if (s->ev_join) (void)hipEventDestroy(s->ev_join);
}

// The second stream of the slab schedule and its fork/join events (default
// priority, like every stream of the library).
hipError_t ensure_side(wp_sim *s) {
  if (s->side) return hipSuccess;
  hipError_t e = hipEventCreateWithFlags(&s->ev_fork, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_join, hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->side, hipStreamNonBlocking);
  if (e != hipSuccess) s->side = nullptr;
  return e;
}

// Precision of the stored state (WP_C64X keeps an FP32 state).
int storage_prec(const wp_sim *s) { return s->prec == WP_C128 ? WP_C128 : WP_C64; }

// The state buffer is allocated on first use unless the caller bound one.
hipError_t ensure_state(wp_sim *s) {
  if (s->psi) return hipSuccess;
  hipError_t e = dev_alloc(&s->psi, s->psi_bytes);
  if (e != hipSuccess) return e;
  s->psi_owned = true;
  return hipMemsetAsync(s->psi, 0, s->psi_bytes, s->stream);
}

wp_status state_fail(wp_sim *s, hipError_t e, const char *what) {
  return e == hipErrorOutOfMemory ? fail(s, WP_ENOMEM, std::string(what) + ": out of device memory")
                                  : hip_fail(s, e, what);
}

// Tuning table: the kernel variant chosen per (batched, precision, line
// length, layout, pass kind), filled by the autotuner or by wp_tune_set;
// absent entries run variant 0.  Shared by every handle in the process.
struct TuneKey {
  int batched, prec, lgN, strided, kind;
  bool operator<(const TuneKey &o) const {
    return std::tie(batched, prec, lgN, strided, kind) < std::tie(o.batched, o.prec, o.lgN, o.strided, o.kind);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;

int tune_for(int batched, int prec, int lgN, bool strided, int kind) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune.find({batched, prec, lgN, strided ? 1 : 0, kind});
  return it == g_tune.end() ? 0 : it->second;
}

void tune_store(int batched, int prec, int lgN, bool strided, int kind, int tune) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune[{batched, prec, lgN, strided ? 1 : 0, kind}] = tune;
}

// Pass kind (wp::PK_*) of a set of operations on an axis of a handle.
int kind_of(const wp_sim *s, int axis, uint32_t ops) {
  if (s->split && (axis == 0 || (ops & wp::OP_K))) return axis == 0 ? 3 : 4;
  if (ops & wp::OP_V) return 1;
  if (ops & wp::OP_K) return 2;
  return 0;
}

wp::PassArgs pass_args(const wp_sim *s, int axis, uint32_t ops) {
  wp::PassArgs a{};
  a.psi = s->psi;
  a.g = s->gd;
  a.axis = axis;
  int lgi = 0;
  for (int d = axis + 1; d < 3; ++d) lgi += s->vlg[d];
  a.lg_inner = lgi;
  a.n_lines = s->total >> s->vlg[axis];
  // A split grid's potential and kinetic passes are its own kinds; a plain
  // forward transform along axis 1 (for the energy) is an ordinary line FFT.
  const bool split_kind = s->split && (axis == 0 || (ops & wp::OP_K));
  a.ops = ops | (split_kind ? wp::OP_SPLIT : 0u);
  a.wsplit[0] = s->d_wsplit;
  a.wsplit[1] = s->split ? s->d_wsplit + ((size_t)1 << s->vlg[1]) : nullptr;
  a.split_h = s->split ? s->vlg[0] : 0;
  a.coef = nullptr;
  a.vtau = 0.0;
  a.pot = s->pd;
  int off = 0;
  for (int d = 0; d < 3; ++d) {
    a.ktab[d] = s->d_kfull + off;
    off += (int)s->g.n[d];
  }
  a.tw = s->d_tw[axis];
  a.tune = tune_for(0, s->prec, s->vlg[axis], lgi > 0, kind_of(s, axis, ops));
  return a;
}

// The part of a middle-axis pass (axis >= 1) that covers x slab `slab` of
// 2^slab_lg: the slab is a grid of its own with n0 >> slab_lg planes.
wp::PassArgs slab_args(const wp_sim *s, wp::PassArgs a, int slab) {
  if (s->slab_lg == 0) return a;
  const int64_t planes = (int64_t)s->g.n[0] >> s->slab_lg;
  const size_t elem = storage_prec(s) == WP_C128 ? 16 : 8;
  a.psi = (char *)a.psi + (size_t)slab * (size_t)planes * (size_t)s->pitch * elem;
  a.n_lines >>= s->slab_lg;
  a.g.lg[0] -= s->slab_lg;
  a.g.lo[0] += (double)(slab * planes) * a.g.dx[0];
  a.ktab[0] += slab * planes;
  return a;
}

// Cache hints: an FP32 state larger than the memory-side cache (256 MB) is
// streamed through each pass once, so its reads and writes bypass the
// caches (non-temporal), except where a slab is read again by the next
// pass of its group (see slab_args): the group's first pass reads
// non-temporally and keeps its writes, the later ones keep their reads and
// writes.  (Measured on MI355X at 512^3: 1-3 % faster steps in FP32, 3-4 %
// slower in FP64, where the hints are therefore not used; with slabs,
// non-temporal writes in the group's last pass cost 0.7 % of a step.)
constexpr uint64_t kCacheBytes = (uint64_t)256 << 20;
bool streams_state(const wp_sim *s) {
  return s->psi_bytes > kCacheBytes && !s->mixed && storage_prec(s) == WP_C64;
}
constexpr uint32_t kNT = wp::OP_LOAD_NT | wp::OP_STORE_NT;

// Default slab count: slabs of at most 256 MiB (the size the autotuner
// picks on MI355X for 512^3 in FP32 and FP64).
// Default slab count: two slabs in flight (one per stream) fit the 256 MB
// memory-side cache.
int default_slab_lg(const wp_sim *s) {
  if (s->vdim != 3 || s->mixed || s->split) return 0;
  int lg = 0;
  const uint64_t bytes = (uint64_t)s->total * (storage_prec(s) == WP_C128 ? 16 : 8);
  while ((bytes >> lg) > ((uint64_t)128 << 20) && lg < s->lg[0]) ++lg;
  return lg;
}

// Launch a line pass of the handle: the power-of-two kernels, or the
// mixed-radix kernel with the axis's stage plan.
hipError_t launch_any(const wp_sim *s, const wp::PassArgs &a, hipStream_t st) {
  if (!s->mixed) return wp::launch_pass(s->prec, a, st);
  wp::GPassArgs ga{};
  ga.p = a;
  ga.inner = 1;
  for (int d = a.axis + 1; d < 3; ++d) ga.inner *= (int64_t)s->g.n[d];
  ga.p.n_lines = s->total / (int64_t)s->g.n[a.axis];
  ga.plan = s->plan[a.axis];
  return wp::launch_gpass(s->prec, ga, st);
}

void use_half_kinetic(const wp_sim *s, wp::PassArgs &a) {
  int off = 0;
  for (int d = 0; d < 3; ++d) {
    a.ktab[d] = s->d_khalf + off;
    off += (int)s->g.n[d];
  }
}

}  // namespace

extern "C" {

const char *wp_version(void) { return "wavepacket-gfx950 0.1"; }

const char *wp_last_error(const wp_sim *sim) { return sim ? sim->err.c_str() : "NULL handle"; }

// Points between the starts of consecutive first-axis planes.  On 3D
// power-of-two grids every plane is followed by kPlanePad unused points: with
// planes a power of two apart, the 128-byte row segments that a first-axis
// pass reads from all planes at once fall on few memory channels (measured
// on MI355X at 512^3: a tile copy along x at 3.3-4.7 TB/s unpadded, 5.2 TB/s
// with 16 points; 8 points, which split row segments over two cache lines,
// were slower).
constexpr uint64_t kPlanePad = 16;
uint64_t plane_pitch(const wp_grid_desc &g) {
  const uint64_t plane = g.n[1] * g.n[2];
  const bool pow2 = is_pow2(g.n[0]) && is_pow2(g.n[1]) && is_pow2(g.n[2]);
  return g.ndim == 3 && pow2 ? plane + kPlanePad : plane;
}

wp_status wp_state_bytes(const wp_grid_desc *grid, uint64_t *bytes) {
  if (!bytes || !check_grid(grid).empty()) return WP_EINVAL;
  const uint64_t elem = grid->prec == WP_C128 ? 16 : 8;
  *bytes = grid->n[0] * plane_pitch(*grid) * elem;
  return WP_OK;
}

wp_status wp_state_pitch(const wp_grid_desc *grid, uint64_t *pitch) {
  if (!pitch || !check_grid(grid).empty()) return WP_EINVAL;
  *pitch = plane_pitch(*grid);
  return WP_OK;
}

wp_status wp_workspace_bytes(const wp_grid_desc *grid, uint64_t *bytes) {
  uint64_t st = 0;
  if (wp_state_bytes(grid, &st) != WP_OK) return WP_EINVAL;
  *bytes = st + table_bytes(*grid);
  return WP_OK;
}

wp_status wp_create(const wp_grid_desc *grid, const wp_potential_desc *pot, void *stream, wp_sim **out) {
  if (!out) return WP_EINVAL;
  *out = nullptr;
  if (!check_grid(grid).empty() || !check_pot(pot).empty()) return WP_EINVAL;
  if (!check_supported(grid).empty()) return WP_EUNSUPPORTED;
  wp_sim *s = new (std::nothrow) wp_sim();
  if (!s) return WP_ENOMEM;
  s->g = *grid;
  s->p = *pot;
  s->stream = (hipStream_t)stream;
  s->prec = grid->prec;
  hipError_t e = hipGetDevice(&s->device);
  if (e != hipSuccess) {
    delete s;
    return WP_EDEVICE;
  }
  s->total = 1;
  for (int d = 0; d < 3; ++d) {
    s->lg[d] = ilog2(grid->n[d]);
    s->total *= (int64_t)grid->n[d];
    s->gd.lg[d] = s->lg[d];
    s->gd.lo[d] = d < grid->ndim ? grid->lo[d] : 0.0;
    s->gd.dx[d] = d < grid->ndim ? spacing(*grid, d) : 0.0;
  }
  s->gd.ndim = grid->ndim;
  for (int d = 0; d < 3; ++d) {
    s->gd.n[d] = (int32_t)grid->n[d];
    s->mixed = s->mixed || (d < grid->ndim && !is_pow2(grid->n[d]));
  }
  s->gd.pow2 = s->mixed ? 0 : 1;
  s->pitch = (int64_t)plane_pitch(*grid);
  s->gd.lg_plane = s->lg[1] + s->lg[2];
  s->gd.pad = (int32_t)(s->pitch - (int64_t)(grid->n[1] * grid->n[2]));
  s->vdim = grid->ndim;
  for (int d = 0; d < 3; ++d) s->vlg[d] = s->lg[d];
  if (grid->ndim == 1 && grid->n[0] > (uint64_t)wp::kMaxLine1D) {
    s->split = true;
    s->vdim = 2;
    s->vlg[0] = (s->lg[0] + 1) / 2;
    s->vlg[1] = s->lg[0] / 2;
  }
  for (int d = 0; d < 3; ++d) {
    s->pd.w[wp::CO_A + d] = to_dev(pot->a[d]);
    s->pd.w[wp::CO_B + d] = to_dev(pot->b[d]);
  }
  s->pd.w[wp::CO_C] = to_dev(pot->c);
  s->pd.w[wp::CO_S] = to_dev(pot->s);
  s->pd.v0_kind = pot->v0_kind;
  for (int i = 0; i < 4; ++i) s->pd.v0_par[i] = pot->v0_par[i];

  // Kinetic factors exp(-i hbar k^2 tau/2m) per axis, the 1/N of the inverse
  // transform folded into the last used axis; k^2 per axis for the energy.
  std::vector<cx<double>> kf, kh;
  std::vector<double> k2;
  const double invN = 1.0 / (double)s->total;
  for (int d = 0; d < 3; ++d) {
    for (uint64_t m = 0; m < grid->n[d]; ++m) {
      const double k = d < grid->ndim ? wavenumber(*grid, d, m) : 0.0;
      const double ksq = k * k;
      const double scale = (d == grid->ndim - 1) ? invN : 1.0;
      const double thf = grid->hbar * ksq * grid->dt / (2.0 * grid->mass);
      const double thh = grid->hbar * ksq * (0.5 * grid->dt) / (2.0 * grid->mass);
      kf.push_back({scale * std::cos(thf), -scale * std::sin(thf)});
      kh.push_back({scale * std::cos(thh), -scale * std::sin(thh)});
      k2.push_back(ksq);
    }
  }
  e = upload(&s->d_kfull, kf);
  if (e == hipSuccess) e = upload(&s->d_khalf, kh);
  if (e == hipSuccess) e = upload(&s->d_k2, k2);
  // Line-FFT twiddles per axis, in the stage order the kernels read them.
  for (int d = 0; d < 3 && e == hipSuccess; ++d)
    e = upload(&s->d_tw[d], s->mixed ? mixed_plan(grid->n[d], &s->plan[d]) : stage_twiddles(uint64_t(1) << s->vlg[d]));
  if (e == hipSuccess && s->split) {
    // exp(-2 pi i e/n), e = q*n1 + r: [n2] factors of q*n1 then [n1] of r.
    const uint64_t n = grid->n[0], n1 = uint64_t(1) << s->vlg[0], n2 = uint64_t(1) << s->vlg[1];
    std::vector<cx<double>> w;
    for (uint64_t q = 0; q < n2; ++q) {
      const double a = -2.0 * kPi * (double)(q * n1) / (double)n;
      w.push_back({std::cos(a), std::sin(a)});
    }
    for (uint64_t r = 0; r < n1; ++r) {
      const double a = -2.0 * kPi * (double)r / (double)n;
      w.push_back({std::cos(a), std::sin(a)});
    }
    e = upload(&s->d_wsplit, w);
  }
  if (e == hipSuccess) {
    int64_t b = (s->total + wp::kObsThreads - 1) / wp::kObsThreads;
    s->obs_blocks = (int)(b > 1024 ? 1024 : b);
    e = dev_alloc((void **)&s->d_partials, sizeof(double) * 8 * (size_t)s->obs_blocks);
  }
  if (e == hipSuccess) e = dev_alloc((void **)&s->d_out8, sizeof(double) * 8);
  if (e == hipSuccess) e = dev_alloc((void **)&s->d_coef, sizeof(double) * wp::CO_COUNT * wp::kCoefChunk);
  if (e == hipSuccess) wp_state_bytes(grid, &s->psi_bytes);
  s->slab_lg = default_slab_lg(s);
  if (e != hipSuccess) {
    release(s);
    delete s;
    return e == hipErrorOutOfMemory ? WP_ENOMEM : WP_EDEVICE;
  }
  *out = s;
  return WP_OK;
}

wp_status wp_destroy(wp_sim *sim) {
  if (!sim) return WP_EINVAL;
  (void)hipSetDevice(sim->device);
  (void)hipStreamSynchronize(sim->stream);
  release(sim);
  delete sim;
  return WP_OK;
}

wp_status wp_bind_state(wp_sim *s, void *dev_psi, uint64_t bytes) {
  if (!s) return WP_EINVAL;
  if (!dev_psi) return fail(s, WP_EINVAL, "bind_state: NULL pointer");
  if (bytes < s->psi_bytes) return fail(s, WP_EINVAL, "bind_state: buffer smaller than the state");
  if (((uintptr_t)dev_psi & 15) != 0) return fail(s, WP_EINVAL, "bind_state: buffer not 16-byte aligned");
  (void)hipSetDevice(s->device);
  if (s->psi_owned && s->psi) {
    // the library's own buffer is freed once no queued work can use it
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(s, e, "bind_state");
    (void)hipFree(s->psi);
  }
  s->psi = dev_psi;
  s->psi_owned = false;
  s->err.clear();
  return WP_OK;
}

void *wp_state_ptr(wp_sim *s) { return s ? s->psi : nullptr; }

// Copy a state between contiguous host memory (`elem` bytes per point) and
// the handle's storage, whose first-axis planes lie s->pitch points apart.
hipError_t copy_state(const wp_sim *s, void *dst, const void *src, size_t elem, bool to_device) {
  const size_t rows = (size_t)s->g.n[0];
  const size_t row = (size_t)(s->total / (int64_t)rows) * elem, pitch = (size_t)s->pitch * elem;
  const hipMemcpyKind kind = to_device ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
  if (row == pitch) return hipMemcpyAsync(dst, src, rows * row, kind, s->stream);
  // One copy per plane, contiguous on both sides.  (A pitched 2D copy from
  // pageable host memory returned zeros under rocprofv3 at 512^3.)
  const size_t dstep = to_device ? pitch : row, sstep = to_device ? row : pitch;
  for (size_t r = 0; r < rows; ++r) {
    hipError_t e = hipMemcpyAsync((char *)dst + r * dstep, (const char *)src + r * sstep, row, kind, s->stream);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Host <-> state copy that changes the precision: runs of up to 2^22 points
// (64 MiB of complex128) go through a device staging buffer and are
// converted there, so PCIe carries each point once in the host's precision
// and the host does no per-point work.  The host side is contiguous, in
// logical order.  Synchronises.
hipError_t convert_copy(wp_sim *s, void *host, int host_prec, bool to_device) {
  const size_t he = host_prec == WP_C128 ? 16 : 8;
  const int64_t chunk = std::min<int64_t>(s->total, (int64_t)1 << 22);
  void *stage = nullptr;
  hipError_t e = dev_alloc(&stage, (size_t)chunk * he);
  for (int64_t first = 0; e == hipSuccess && first < s->total; first += chunk) {
    const int64_t n = std::min<int64_t>(chunk, s->total - first);
    char *h = (char *)host + (size_t)first * he;
    if (to_device) {
      e = hipMemcpyAsync(stage, h, (size_t)n * he, hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess) e = wp::launch_stage_in(storage_prec(s), s->psi, s->gd, host_prec, stage, first, n, s->stream);
    } else {
      e = wp::launch_stage_out(storage_prec(s), s->psi, s->gd, host_prec, stage, first, n, s->stream);
      if (e == hipSuccess) e = hipMemcpyAsync(h, stage, (size_t)n * he, hipMemcpyDeviceToHost, s->stream);
    }
  }
  // The staging buffer is released only once nothing queued uses it.
  const hipError_t es = hipStreamSynchronize(s->stream);
  if (stage) (void)hipFree(stage);
  return e != hipSuccess ? e : es;
}

wp_status wp_set_state(wp_sim *s, const double *host, double t0) {
  if (!s) return WP_EINVAL;
  if (!host) return fail(s, WP_EINVAL, "set_state: NULL host buffer");
  if (!std::isfinite(t0)) return fail(s, WP_EINVAL, "set_state: t0 must be finite");
  (void)hipSetDevice(s->device);
  hipError_t e = ensure_state(s);
  if (e != hipSuccess) return state_fail(s, e, "set_state");
  if (s->prec == WP_C128) {
    e = copy_state(s, s->psi, host, 16, true);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  } else {
    e = convert_copy(s, const_cast<double *>(host), WP_C128, true);
  }
  if (e != hipSuccess) return state_fail(s, e, "set_state");
  s->t0 = t0;
  s->step = 0;
  s->err.clear();
  return WP_OK;
}

wp_status wp_set_state_gaussian(wp_sim *s, const double center[3], const double sigma[3], const double k[3],
                                double t0) {
  if (!s) return WP_EINVAL;
  if (!center || !sigma || !k) return fail(s, WP_EINVAL, "set_state_gaussian: NULL array");
  if (!std::isfinite(t0)) return fail(s, WP_EINVAL, "set_state_gaussian: t0 must be finite");
  for (int d = 0; d < s->g.ndim; ++d)
    if (!(sigma[d] > 0) || !std::isfinite(sigma[d]) || !std::isfinite(center[d]) || !std::isfinite(k[d]))
      return fail(s, WP_EINVAL, "set_state_gaussian: sigma must be > 0 and all values finite");
  (void)hipSetDevice(s->device);
  // The Gaussian is a product over axes, so its discrete norm is the product
  // of the per-axis norms: each axis factor is normalised on its own.
  std::vector<cx<double>> f[3];
  for (int d = 0; d < 3; ++d) {
    const uint64_t n = s->g.n[d];
    f[d].resize(n);
    if (d >= s->g.ndim) {
      f[d][0] = {1.0, 0.0};
      continue;
    }
    const double dx = spacing(s->g, d);
    double nrm = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
      const double u = (s->g.lo[d] + (double)i * dx) - center[d];
      const double amp = std::pow(2.0 / kPi, 0.25) / std::sqrt(sigma[d]) * std::exp(-u * u / (sigma[d] * sigma[d]));
      f[d][i] = {amp * std::cos(k[d] * u), amp * std::sin(k[d] * u)};
      nrm += (f[d][i].x * f[d][i].x + f[d][i].y * f[d][i].y) * dx;
    }
    const double sc = 1.0 / std::sqrt(nrm);
    for (auto &v : f[d]) v = {v.x * sc, v.y * sc};
  }
  hipError_t e = ensure_state(s);
  if (e != hipSuccess) return state_fail(s, e, "set_state_gaussian");
  if (!s->d_gauss) {
    e = dev_alloc((void **)&s->d_gauss, sizeof(cx<double>) * (s->g.n[0] + s->g.n[1] + s->g.n[2]));
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s->ev_gauss, hipEventDisableTiming);
    if (e != hipSuccess) return state_fail(s, e, "set_state_gaussian");
  } else {
    // the previous Gaussian kernel must have read the old factors
    e = hipEventSynchronize(s->ev_gauss);
  }
  cx<double> *d[3] = {s->d_gauss, s->d_gauss + s->g.n[0], s->d_gauss + s->g.n[0] + s->g.n[1]};
  for (int i = 0; i < 3 && e == hipSuccess; ++i) e = copy_in(d[i], f[i].data(), sizeof(cx<double>) * f[i].size());
  if (e == hipSuccess) e = wp::launch_gaussian(storage_prec(s), s->psi, s->gd, d[0], d[1], d[2], s->stream);
  if (e == hipSuccess) e = hipEventRecord(s->ev_gauss, s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "set_state_gaussian");
  s->t0 = t0;
  s->step = 0;
  s->err.clear();
  return WP_OK;
}

wp_status wp_set_slabs(wp_sim *s, uint32_t count) {
  if (!s) return WP_EINVAL;
  if (count == 0 || (count & (count - 1)) != 0) return fail(s, WP_EINVAL, "set_slabs: count must be a power of two");
  int lg = 0;
  while ((1u << lg) < count) ++lg;
  if (lg > 0 && (s->vdim != 3 || s->mixed || s->split || lg > s->lg[0]))
    return fail(s, WP_EINVAL, "set_slabs: slabs need a 3D power-of-two grid with at least `count` x planes");
  s->slab_lg = lg;
  s->err.clear();
  return WP_OK;
}

uint32_t wp_get_slabs(const wp_sim *s) { return s ? (1u << s->slab_lg) : 0u; }

wp_status wp_set_order(wp_sim *s, int32_t order) {
  if (!s) return WP_EINVAL;
  if (order != WP_ORDER_VKV && order != WP_ORDER_KVK) return fail(s, WP_EINVAL, "unknown order");
  s->order = order;
  return WP_OK;
}

}  // extern "C"

namespace {

// Walk the launch sequence of `nsteps` steps, calling launch(kind, fn) for
// each kernel, where fn() enqueues it.  Kinds are the WP_PASS_* values.
// Events that only time device work: no system-scope fence at record time,
// so that no cache write-back or invalidation lands inside the timed interval.
inline hipError_t timing_event(hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableSystemFence); }

// With no_alloc the walk creates nothing: while the handle's second stream
// does not exist yet, the slabs of a step all run on the handle's stream
// (the same kernels in the same order per slab, so the same bits).
template <class Launch>
hipError_t run_schedule(wp_sim *s, uint64_t nsteps, Launch &&launch, bool no_alloc = false) {
  const double tau_half = 0.5 * s->g.dt / s->g.hbar;
  const double tau_full = s->g.dt / s->g.hbar;
  const int prec = s->prec;
  hipStream_t st = s->stream;
  auto pass = [&](int kind, const wp::PassArgs &a, hipStream_t q) {
    return launch(kind, [&]() { return launch_any(s, a, q); });
  };
  // The potential's waveform values come from a table filled for up to
  // kCoefChunk consecutive step times at once; the stream orders each refill
  // after the passes that read the previous contents.
  int64_t cbase = -1;
  double chalf = 0.0;
  auto coef_at = [&](int64_t n, double half, const double **out) -> hipError_t {
    if (cbase < 0 || half != chalf || n < cbase || n >= cbase + wp::kCoefChunk) {
      wp::TimeDev T{};
      T.t0 = s->t0;
      T.dt = s->g.dt;
      T.step = n;
      T.step_dev = nullptr;
      T.half = half;
      hipError_t r = launch(WP_PASS_COEF, [&]() {
        return wp::launch_coefficients(s->pd, T, wp::kCoefChunk, s->d_coef, st);
      });
      if (r != hipSuccess) return r;
      cbase = n;
      chalf = half;
    }
    *out = s->d_coef + (n - cbase) * wp::CO_COUNT;
    return hipSuccess;
  };
  if (s->g.ndim == 1 && !s->split) {
    wp::Solve1DArgs a{};
    a.psi = s->psi;
    a.g = s->gd;
    a.nsteps = (int64_t)nsteps;
    a.time.t0 = s->t0;
    a.time.dt = s->g.dt;
    a.time.step = (int64_t)s->step;
    a.time.step_dev = nullptr;
    a.time.half = 0.0;
    a.vtau_half = tau_half;
    a.vtau_full = tau_full;
    a.order = s->order;
    a.pot = s->pd;
    a.kfull = s->d_kfull;
    a.khalf = s->d_khalf;
    a.tw = s->d_tw[0];
    if (s->mixed)
      return launch(WP_PASS_SOLVE1D, [&]() { return wp::launch_gsolve1d(prec == WP_C128 ? 2 : 1, a, s->plan[0], st); });
    return launch(WP_PASS_SOLVE1D, [&]() { return wp::launch_solve1d(prec, a, st); });
  }
  const int last = s->vdim - 1;
  // Middle of a step (all axes but the first): forward over axes 1..last-1,
  // forward + kinetic + inverse along the last axis, inverse back.
  // On a 3D grid with slabs, slab by slab.
  const bool stream = streams_state(s);
  const uint32_t nt_v = stream ? kNT : 0u;                                          // first-axis passes
  const uint32_t nt_first = stream ? (s->slab_lg ? wp::OP_LOAD_NT : kNT) : 0u;      // first middle pass
  const uint32_t nt_mid = stream && s->slab_lg == 0 ? kNT : 0u;                     // the kinetic pass of 3D
  const uint32_t nt_last = stream && s->slab_lg == 0 ? kNT : 0u;                    // last middle pass
  // Slabs alternate between the handle's stream and the second one.
  const int nslab = 1 << s->slab_lg;
  const bool two = nslab > 1 && !(no_alloc && !s->side);
  if (two) {
    if (hipError_t r = ensure_side(s); r != hipSuccess) return r;
  }
  auto middle = [&](bool half_k) -> hipError_t {
    hipError_t r = hipSuccess;
    if (two) {
      r = hipEventRecord(s->ev_fork, st);
      if (r == hipSuccess) r = hipStreamWaitEvent(s->side, s->ev_fork, 0);
    }
    for (int sl = 0; sl < nslab && r == hipSuccess; ++sl) {
      const hipStream_t q = (two && (sl & 1)) ? s->side : st;
      for (int d = 1; d < last && r == hipSuccess; ++d)
        r = pass(WP_PASS_MID_FWD, slab_args(s, pass_args(s, d, wp::OP_FWD | nt_first), sl), q);
      if (r != hipSuccess) return r;
      wp::PassArgs k = pass_args(s, last, wp::OP_FWD | wp::OP_K | wp::OP_POST_INV | (last == 1 ? kNT & nt_v : nt_mid));
      if (half_k) use_half_kinetic(s, k);
      r = pass(WP_PASS_LAST, slab_args(s, k, sl), q);
      for (int d = last - 1; d >= 1 && r == hipSuccess; --d)
        r = pass(WP_PASS_MID_INV, slab_args(s, pass_args(s, d, wp::OP_PRE_INV | nt_last), sl), q);
    }
    if (two && r == hipSuccess) {
      r = hipEventRecord(s->ev_join, s->side);
      if (r == hipSuccess) r = hipStreamWaitEvent(st, s->ev_join, 0);
    }
    return r;
  };
  hipError_t e = hipSuccess;
  if (s->order == WP_ORDER_VKV) {
    // [V/2(t_n) F_0] ([middle] [F_0^-1 V(t_n+1) F_0])* ... [F_0^-1 V/2(t_N)]:
    // equal-time potential halves of consecutive steps are merged.
    wp::PassArgs a0 = pass_args(s, 0, wp::OP_V | wp::OP_FWD | nt_v);
    e = coef_at((int64_t)s->step, 0.0, &a0.coef);
    a0.vtau = tau_half;
    if (e == hipSuccess) e = pass(WP_PASS_EDGE, a0, st);
    for (uint64_t j = 0; j < nsteps && e == hipSuccess; ++j) {
      e = middle(false);
      if (e != hipSuccess) break;
      const bool lastj = (j + 1 == nsteps);
      wp::PassArgs a = pass_args(s, 0, wp::OP_PRE_INV | wp::OP_V | (lastj ? 0u : wp::OP_FWD) | nt_v);
      e = coef_at((int64_t)(s->step + j + 1), 0.0, &a.coef);
      a.vtau = lastj ? tau_half : tau_full;
      if (lastj) a.moments = s->moments;
      if (e == hipSuccess) e = pass(lastj ? WP_PASS_EDGE : WP_PASS_AXIS0, a, st);
    }
  } else {
    // K/2 V(t_n + dt/2) K/2 with consecutive kinetic halves merged.
    e = pass(WP_PASS_EDGE, pass_args(s, 0, wp::OP_FWD | nt_v), st);
    if (e == hipSuccess) e = middle(true);
    for (uint64_t j = 0; j < nsteps && e == hipSuccess; ++j) {
      wp::PassArgs a = pass_args(s, 0, wp::OP_PRE_INV | wp::OP_V | wp::OP_FWD | nt_v);
      e = coef_at((int64_t)(s->step + j), 0.5, &a.coef);
      a.vtau = tau_full;
      if (e == hipSuccess) e = pass(WP_PASS_AXIS0, a, st);
      if (e == hipSuccess) e = middle(j + 1 == nsteps);
    }
    if (e == hipSuccess) e = pass(WP_PASS_EDGE, pass_args(s, 0, wp::OP_PRE_INV | nt_v), st);
  }
  return e;
}

}  // namespace

extern "C" {

wp_status wp_propagate(wp_sim *s, uint64_t nsteps) {
  if (!s) return WP_EINVAL;
  if (nsteps == 0) return WP_OK;
  if (nsteps > (uint64_t)1 << 40) return fail(s, WP_EINVAL, "propagate: nsteps too large");
  (void)hipSetDevice(s->device);
  if (hipError_t e0 = ensure_state(s); e0 != hipSuccess) return state_fail(s, e0, "propagate");
  hipError_t e = run_schedule(s, nsteps, [](int, auto &&fn) { return fn(); });
  if (e != hipSuccess) return hip_fail(s, e, "propagate");
  s->step += nsteps;
  s->err.clear();
  return WP_OK;
}

wp_status wp_profile_propagate(wp_sim *s, uint64_t nsteps, uint32_t kinds, double *ms, uint64_t *count) {
  if (!s) return WP_EINVAL;
  if (!ms || !count) return fail(s, WP_EINVAL, "profile_propagate: NULL output");
  if (nsteps == 0 || nsteps > 100000) return fail(s, WP_EINVAL, "profile_propagate: nsteps must be in 1..100000");
  (void)hipSetDevice(s->device);
  if (hipError_t e0 = ensure_state(s); e0 != hipSuccess) return state_fail(s, e0, "profile_propagate");
  for (int k = 0; k < WP_PASS_KINDS; ++k) {
    ms[k] = 0.0;
    count[k] = 0;
  }
  // One event pair per launch, attached to the dispatch itself, so that the
  // pair spans exactly that kernel and nothing is enqueued between kernels;
  // durations are read after the whole sequence, so that the host never
  // waits between launches.
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;
  hipError_t e = run_schedule(s, nsteps, [&](int kind, auto &&fn) {
    if (!((kinds >> kind) & 1u)) return fn();
    hipEvent_t a, b;
    hipError_t r = timing_event(&a);
    if (r != hipSuccess) return r;
    r = timing_event(&b);
    if (r != hipSuccess) {
      (void)hipEventDestroy(a);
      return r;
    }
    ev.push_back({kind, {a, b}});
    wp::DispatchEvents &d = wp::tl_dispatch_events;
    d = {a, b, false};
    r = fn();
    const bool used = d.used;
    d = {};
    // every launcher of the schedule attaches the events
    if (r == hipSuccess && !used) r = hipErrorNotSupported;
    return r;
  });
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  for (auto &x : ev) {
    float m = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&m, x.second.first, x.second.second);
    if (e == hipSuccess) {
      ms[x.first] += m;
      count[x.first] += 1;
    }
    (void)hipEventDestroy(x.second.first);
    (void)hipEventDestroy(x.second.second);
  }
  if (e != hipSuccess) return hip_fail(s, e, "profile_propagate");
  s->step += nsteps;
  s->err.clear();
  return WP_OK;
}

// Average device time of `reps` back-to-back launches of one pass (after one
// warm-up launch), between one event pair on the handle's stream.
static hipError_t time_launches(wp_sim *s, const wp::PassArgs &a, uint32_t reps, double *ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = timing_event(&e0);
  if (e == hipSuccess) e = timing_event(&e1);
  if (e == hipSuccess) e = launch_any(s, a, s->stream);
  if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
  for (uint32_t r = 0; r < reps && e == hipSuccess; ++r) e = launch_any(s, a, s->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float m = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&m, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e == hipSuccess) *ms = (double)m / reps;
  return e;
}

// Coefficient row for the current step, for timing potential passes.
static hipError_t current_coef(wp_sim *s, wp::PassArgs &a) {
  wp::TimeDev T{};
  T.t0 = s->t0;
  T.dt = s->g.dt;
  T.step = (int64_t)s->step;
  a.coef = s->d_coef;
  return wp::launch_coefficients(s->pd, T, 1, s->d_coef, s->stream);
}

wp_status wp_time_pass(wp_sim *s, int32_t kind, uint32_t reps, double *ms) {
  if (!s) return WP_EINVAL;
  if (!ms) return fail(s, WP_EINVAL, "time_pass: NULL output");
  if (reps < 1 || reps > 10000) return fail(s, WP_EINVAL, "time_pass: reps must be in 1..10000");
  if (s->g.ndim == 1 && !s->split) return fail(s, WP_EINVAL, "time_pass: 1D grids up to 8192 points have no line passes");
  const int last = s->vdim - 1;
  if ((kind == WP_PASS_MID_FWD || kind == WP_PASS_MID_INV) && s->vdim != 3)
    return fail(s, WP_EINVAL, "time_pass: middle-axis passes exist only in 3D");
  wp::PassArgs a{};
  switch (kind) {
    case WP_PASS_AXIS0:
      a = pass_args(s, 0, wp::OP_PRE_INV | wp::OP_V | wp::OP_FWD);
      a.vtau = s->g.dt / s->g.hbar;
      break;
    case WP_PASS_EDGE:
      a = pass_args(s, 0, wp::OP_V | wp::OP_FWD);
      a.vtau = 0.5 * s->g.dt / s->g.hbar;
      break;
    case WP_PASS_MID_FWD: a = pass_args(s, 1, wp::OP_FWD); break;
    case WP_PASS_MID_INV: a = pass_args(s, 1, wp::OP_PRE_INV); break;
    case WP_PASS_LAST: a = pass_args(s, last, wp::OP_FWD | wp::OP_K | wp::OP_POST_INV); break;
    default: return fail(s, WP_EINVAL, "time_pass: unknown pass kind");
  }
  if (streams_state(s)) a.ops |= kNT;  // as a pass over the whole grid in wp_propagate
  (void)hipSetDevice(s->device);
  hipError_t e = ensure_state(s);
  a.psi = s->psi;
  if (e == hipSuccess && (a.ops & wp::OP_V)) e = current_coef(s, a);
  if (e == hipSuccess) e = time_launches(s, a, reps, ms);
  if (e != hipSuccess) return hip_fail(s, e, "time_pass");
  s->err.clear();
  return WP_OK;
}

wp_status wp_autotune(wp_sim *s, uint32_t reps, double *ms) {
  if (!s) return WP_EINVAL;
  if (reps < 1 || reps > 10000) return fail(s, WP_EINVAL, "autotune: reps must be in 1..10000");
  if (ms)
    for (int i = 0; i < 3 * wp::kTuneSlots + WP_TUNE_SLAB_CHOICES; ++i) ms[i] = NAN;
  if ((s->g.ndim == 1 && !s->split) || s->mixed) {
    s->err.clear();
    return WP_OK;  // a 1D grid solved in one workgroup, or mixed lengths: nothing to tune
  }
  (void)hipSetDevice(s->device);
  hipError_t e = ensure_state(s);
  // The candidates run on a copy of the state, which they transform.
  if (e == hipSuccess && !s->scratch) e = dev_alloc(&s->scratch, s->psi_bytes);
  if (e == hipSuccess) e = hipMemcpyAsync(s->scratch, s->psi, s->psi_bytes, hipMemcpyDeviceToDevice, s->stream);
  const int last = s->vdim - 1;
  struct Cls {
    int axis;
    uint32_t ops;
  } cls[3] = {{0, wp::OP_PRE_INV | wp::OP_V | wp::OP_FWD}, {1, wp::OP_FWD}, {last, wp::OP_FWD | wp::OP_K | wp::OP_POST_INV}};
  // Table key and candidates of each class.
  int ckind[3] = {}, clg[3] = {}, cnc[3] = {}, ccand[3][4] = {};
  bool cstrided[3] = {};
  for (int c = 0; c < 3 && e == hipSuccess; ++c) {
    if (c == 1 && s->vdim != 3) continue;
    wp::PassArgs a = pass_args(s, cls[c].axis, cls[c].ops);
    a.psi = s->scratch;
    a.vtau = s->g.dt / s->g.hbar;
    if (a.ops & wp::OP_V) e = current_coef(s, a);
    const int kind = kind_of(s, cls[c].axis, cls[c].ops);
    const int lgN = s->vlg[cls[c].axis];
    int *cand = ccand[c];
    const int nc = wp::tune_candidates(s->prec, lgN, kind, cand);
    ckind[c] = kind;
    clg[c] = lgN;
    cnc[c] = nc;
    cstrided[c] = a.lg_inner > 0;
    // Two rounds over the candidates, the best of each kept: the first
    // launches after an idle spell run slower than later ones.  Each
    // candidate starts from a fresh copy of the state (repeated forward
    // transforms grow the values without bound).
    double tbest[4] = {0, 0, 0, 0};
    for (int round = 0; round < 2 && e == hipSuccess; ++round)
      for (int i = 0; i < nc && e == hipSuccess; ++i) {
        a.tune = cand[i];
        double m = 0.0;
        e = hipMemcpyAsync(s->scratch, s->psi, s->psi_bytes, hipMemcpyDeviceToDevice, s->stream);
        if (e == hipSuccess) e = time_launches(s, a, reps, &m);
        if (e == hipSuccess && (round == 0 || m < tbest[i])) tbest[i] = m;
      }
    int best = 0;
    double best_ms = 0.0;
    for (int i = 0; i < nc && e == hipSuccess; ++i) {
      if (i == 0 || tbest[i] < best_ms) {
        best = cand[i];
        best_ms = tbest[i];
      }
    }
    if (e == hipSuccess) tune_store(0, s->prec, lgN, a.lg_inner > 0, kind, best);
  }
  // The back-to-back launches above leave the scratch copy far from a
  // solution (repeated unnormalised transforms overflow it), and whole steps
  // over such data run measurably faster than over a real state: the rounds
  // below start from a fresh copy of the state.
  if (e == hipSuccess) e = hipMemcpyAsync(s->scratch, s->psi, s->psi_bytes, hipMemcpyDeviceToDevice, s->stream);
  // Slab count of the middle passes (3D): whole steps on the scratch copy
  // for 1, 2, 4, ... slabs; the state and the step counter are untouched.
  if (e == hipSuccess && s->vdim == 3 && !s->mixed) {
    void *keep = s->psi;
    const int keep_lg = s->slab_lg;
    s->psi = s->scratch;
    int best = keep_lg;
    double best_ms = 0.0;
    bool first = true;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = timing_event(&e0);
    if (e == hipSuccess) e = timing_event(&e1);
    const int top = s->lg[0] < WP_TUNE_SLAB_CHOICES - 1 ? s->lg[0] : WP_TUNE_SLAB_CHOICES - 1;
    const uint64_t steps = 1 + reps / 4;
    double sbest[WP_TUNE_SLAB_CHOICES] = {};
    auto direct = [](int, auto &&fn) { return fn(); };
    for (int round = 0; round < 2 && e == hipSuccess; ++round)
      for (int lg = 0; lg <= top && e == hipSuccess; ++lg) {
        s->slab_lg = lg;
        e = run_schedule(s, 1, direct);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
        if (e == hipSuccess) e = run_schedule(s, steps, direct);
        if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float m = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&m, e0, e1);
        const double per = (double)m / (double)steps;
        if (e == hipSuccess && (round == 0 || per < sbest[lg])) sbest[lg] = per;
      }
    for (int lg = 0; lg <= top && e == hipSuccess; ++lg) {
      if (ms) ms[3 * wp::kTuneSlots + lg] = sbest[lg];
      if (first || sbest[lg] < best_ms) {
        best = lg;
        best_ms = sbest[lg];
        first = false;
      }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    s->psi = keep;
    s->slab_lg = e == hipSuccess ? best : keep_lg;
  }
  // Whole steps per variant: each class in turn runs every candidate inside
  // real steps (the chosen slab count, the other classes at their chosen
  // variants) and keeps the fastest.  Launches over the whole grid, timed
  // above, only give the starting point: the slab launches and cache hints
  // of a step differ from them.
  if (e == hipSuccess) {
    void *keep = s->psi;
    s->psi = s->scratch;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    e = timing_event(&e0);
    if (e == hipSuccess) e = timing_event(&e1);
    const uint64_t steps = 2 + reps / 2;
    auto direct = [](int, auto &&fn) { return fn(); };
    for (int c = 0; c < 3 && e == hipSuccess; ++c) {
      if (c == 1 && s->vdim != 3) continue;
      const int nc = cnc[c];
      double tbest[4] = {0, 0, 0, 0};
      for (int round = 0; round < 2 && e == hipSuccess; ++round)
        for (int i = 0; i < nc && e == hipSuccess; ++i) {
          tune_store(0, s->prec, clg[c], cstrided[c], ckind[c], ccand[c][i]);
          e = run_schedule(s, 1, direct);  // warm-up
          if (e == hipSuccess) e = hipEventRecord(e0, s->stream);
          if (e == hipSuccess) e = run_schedule(s, steps, direct);
          if (e == hipSuccess) e = hipEventRecord(e1, s->stream);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float m = 0.f;
          if (e == hipSuccess) e = hipEventElapsedTime(&m, e0, e1);
          const double per = (double)m / (double)steps;
          if (e == hipSuccess && (round == 0 || per < tbest[i])) tbest[i] = per;
        }
      int best = ccand[c][0];
      double best_ms = 0.0;
      for (int i = 0; i < nc && e == hipSuccess; ++i) {
        if (ms) ms[c * wp::kTuneSlots + ccand[c][i]] = tbest[i];
        if (i == 0 || tbest[i] < best_ms) {
          best = ccand[c][i];
          best_ms = tbest[i];
        }
      }
      if (e == hipSuccess) tune_store(0, s->prec, clg[c], cstrided[c], ckind[c], best);
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    s->psi = keep;
  }
  if (e != hipSuccess) return hip_fail(s, e, "autotune");
  s->err.clear();
  return WP_OK;
}

wp_status wp_get_state(wp_sim *s, void *host_out, int32_t as_prec) {
  if (!s) return WP_EINVAL;
  if (!host_out) return fail(s, WP_EINVAL, "get_state: NULL host buffer");
  if (as_prec != WP_C64 && as_prec != WP_C128) return fail(s, WP_EINVAL, "get_state: bad precision");
  (void)hipSetDevice(s->device);
  hipError_t e = ensure_state(s);
  if (e != hipSuccess) return state_fail(s, e, "get_state");
  if (as_prec == storage_prec(s)) {
    e = copy_state(s, host_out, s->psi, as_prec == WP_C128 ? 16 : 8, false);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  } else {
    e = convert_copy(s, host_out, as_prec, false);
  }
  if (e != hipSuccess) return state_fail(s, e, "get_state");
  s->err.clear();
  return WP_OK;
}

// <phi|psi> of the current state without the volume element.
// phi_stored: phi has the state's storage layout (else it is contiguous).
static hipError_t inner_sum(wp_sim *s, const void *phi, int phi_prec, bool phi_stored, double out2[2]) {
  double o[8];
  hipError_t e = wp::launch_inner(phi_prec, phi, storage_prec(s), s->psi, s->total, s->gd.lg_plane,
                                  phi_stored ? s->gd.pad : 0, s->gd.pad, s->obs_blocks, s->d_partials, s->d_out8,
                                  s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(o, s->d_out8, sizeof(o), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  out2[0] = o[0];
  out2[1] = o[1];
  return e;
}

wp_status wp_store_reference(wp_sim *s) {
  if (!s) return WP_EINVAL;
  (void)hipSetDevice(s->device);
  hipError_t e = ensure_state(s);
  if (e == hipSuccess && !s->ref) e = dev_alloc(&s->ref, s->psi_bytes);
  if (e == hipSuccess) e = hipMemcpyAsync(s->ref, s->psi, s->psi_bytes, hipMemcpyDeviceToDevice, s->stream);
  if (e != hipSuccess) return state_fail(s, e, "store_reference");
  s->err.clear();
  return WP_OK;
}

wp_status wp_inner(wp_sim *s, const void *dev_phi, int32_t phi_prec, double *out) {
  if (!s) return WP_EINVAL;
  if (!dev_phi || !out) return fail(s, WP_EINVAL, "inner: NULL pointer");
  if (phi_prec != WP_C64 && phi_prec != WP_C128) return fail(s, WP_EINVAL, "inner: phi_prec must be WP_C64 or WP_C128");
  (void)hipSetDevice(s->device);
  hipError_t e = ensure_state(s);
  double o[2] = {0, 0};
  if (e == hipSuccess) e = inner_sum(s, dev_phi, phi_prec, false, o);
  if (e != hipSuccess) return state_fail(s, e, "inner");
  double dV = 1.0;
  for (int d = 0; d < s->g.ndim; ++d) dV *= spacing(s->g, d);
  out[0] = o[0] * dV;
  out[1] = o[1] * dV;
  s->err.clear();
  return WP_OK;
}

wp_status wp_observables(wp_sim *s, uint32_t mask, double *out) {
  if (!s) return WP_EINVAL;
  if (!out) return fail(s, WP_EINVAL, "observables: NULL output");
  if ((mask & WP_OBS_AUTOCORR) && !s->ref) return fail(s, WP_ESTATE, "observables: no reference state stored");
  (void)hipSetDevice(s->device);
  if (hipError_t e0 = ensure_state(s); e0 != hipSuccess) return state_fail(s, e0, "observables");
  const double t = s->t0 + (double)s->step * s->g.dt;
  double dV = 1.0;
  for (int d = 0; d < s->g.ndim; ++d) dV *= spacing(s->g, d);
  const bool energy = (mask & WP_OBS_ENERGY) != 0;
  wp::ObsArgs a{};
  a.psi = s->psi;
  a.g = s->gd;
  a.total = s->total;
  a.with_v = energy ? 1 : 0;
  a.kinetic = 0;
  a.t = t;
  a.pot = s->pd;
  a.partials = s->d_partials;
  double sums[8], ksum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  hipError_t e = wp::launch_observables(storage_prec(s), a, s->obs_blocks, s->d_out8, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(sums, s->d_out8, sizeof(sums), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e == hipSuccess && energy) {
    if (!s->scratch) e = dev_alloc(&s->scratch, s->psi_bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(s->scratch, s->psi, s->psi_bytes, hipMemcpyDeviceToDevice, s->stream);
    for (int d = 0; d < s->vdim && e == hipSuccess; ++d) {
      wp::PassArgs p = pass_args(s, d, wp::OP_FWD);
      p.psi = s->scratch;
      if (!s->mixed && !wp::pass_supported(s->prec, s->vlg[d])) {
        e = hipErrorNotSupported;
        break;
      }
      e = launch_any(s, p, s->stream);
    }
    if (e == hipSuccess) {
      wp::ObsArgs k = a;
      k.psi = s->scratch;
      k.kinetic = 1;
      k.with_v = 0;
      k.split_h = s->split ? s->vlg[0] : 0;
      int off = 0;
      for (int d = 0; d < 3; ++d) {
        k.k2tab[d] = s->d_k2 + off;
        off += (int)s->g.n[d];
      }
      e = wp::launch_observables(storage_prec(s), k, s->obs_blocks, s->d_out8, s->stream);
    }
    if (e == hipSuccess) e = hipMemcpyAsync(ksum, s->d_out8, sizeof(ksum), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  }
  if (e == hipErrorNotSupported) return fail(s, WP_EUNSUPPORTED, "observables: energy needs an axis <= 4096 points");
  if (e != hipSuccess) return hip_fail(s, e, "observables");
  double all[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  all[0] = std::sqrt(sums[0] * dV);
  for (int d = 0; d < 3; ++d) {
    all[1 + d] = d < s->g.ndim ? sums[1 + d] * dV : 0.0;
    all[4 + d] = d < s->g.ndim ? sums[4 + d] * dV : 0.0;
  }
  all[7] = energy ? (s->g.hbar * s->g.hbar / (2.0 * s->g.mass)) * ksum[0] * dV / (double)s->total + sums[7] * dV
                  : 0.0;
  // widths <x^2> - <x>^2 of Table 3 (from the unnormalised moments)
  for (int d = 0; d < 3; ++d) all[8 + d] = all[4 + d] - all[1 + d] * all[1 + d];
  if (mask & WP_OBS_AUTOCORR) {
    double o[2] = {0, 0};
    hipError_t e2 = inner_sum(s, s->ref, storage_prec(s), true, o);
    if (e2 != hipSuccess) return hip_fail(s, e2, "observables");
    all[11] = (o[0] * o[0] + o[1] * o[1]) * dV * dV;
  }
  int top = 0;
  for (int i = 0; i < 12; ++i)
    if (mask & (1u << i)) top = i;
  for (int i = 0; i <= top; ++i) out[i] = (mask & (1u << i)) ? all[i] : 0.0;
  s->err.clear();
  return WP_OK;
}

}  // extern "C"

namespace {

constexpr uint32_t kMomentMask = WP_OBS_NORM | WP_OBS_X | WP_OBS_Y | WP_OBS_Z | WP_OBS_X2 | WP_OBS_Y2 | WP_OBS_Z2 |
                                 WP_OBS_SX | WP_OBS_SY | WP_OBS_SZ;

// The closing pass carries the moments on power-of-two 2D/3D grids in the
// default order (a first-axis potential pass ends the propagation there).
bool observe_fusable(const wp_sim *s, uint32_t mask) {
  return (mask & ~kMomentMask) == 0 && s->order == WP_ORDER_VKV && s->g.ndim >= 2 && !s->mixed && !s->split;
}

// Workgroups of the closing pass, i.e. 8-slot moment rows it writes.
wp_status closing_rows(wp_sim *s, int64_t *rows) {
  const wp::PassArgs probe = pass_args(s, 0, wp::OP_PRE_INV | wp::OP_V);
  const int tile = wp::pass_tile(s->prec, s->vlg[0], true, kind_of(s, 0, probe.ops), probe.tune);
  if (tile < 1) return fail(s, WP_EUNSUPPORTED, "propagate_observe: no pass for this line length");
  *rows = (probe.n_lines + tile - 1) / tile;
  if (*rows > 0x7fffffff) return fail(s, WP_EUNSUPPORTED, "propagate_observe: too many workgroups");
  return WP_OK;
}

// Propagate with the closing pass writing its moment rows to `mrows` (rows
// entries of 8 doubles, every one written by this propagation), reduce them
// in row order and return the observables of `mask`.  Synchronises.
wp_status observe_fused(wp_sim *s, uint64_t nsteps, uint32_t mask, double *out, double *mrows, int64_t rows,
                        bool no_alloc, const char *what) {
  s->moments = mrows;
  hipError_t e = run_schedule(s, nsteps, [](int, auto &&fn) { return fn(); }, no_alloc);
  s->moments = nullptr;
  double sums[8];
  if (e == hipSuccess) e = wp::launch_reduce8(mrows, (int)rows, s->d_out8, s->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(sums, s->d_out8, sizeof(sums), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, what);
  s->step += nsteps;
  double dV = 1.0;
  for (int d = 0; d < s->g.ndim; ++d) dV *= spacing(s->g, d);
  double all[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  all[0] = std::sqrt(sums[0] * dV);
  for (int d = 0; d < s->g.ndim; ++d) {
    all[1 + d] = sums[1 + d] * dV;
    all[4 + d] = sums[4 + d] * dV;
  }
  for (int d = 0; d < 3; ++d) all[8 + d] = all[4 + d] - all[1 + d] * all[1 + d];
  int top = 0;
  for (int i = 0; i < 12; ++i)
    if (mask & (1u << i)) top = i;
  for (int i = 0; i <= top; ++i) out[i] = (mask & (1u << i)) ? all[i] : 0.0;
  s->err.clear();
  return WP_OK;
}

// Moment rows of wp_propagate_observe_noalloc: one fixed array per device,
// loaded with the library's code object, so that the call allocates
// nothing.  Host code never uses the array's name as an address (on the
// host it only names the symbol): its device address comes from
// hipGetSymbolAddress, once per device with that device current, and is
// kept in scratch_dev[].  Every call on a device shares that device's
// array; a call writes every row it later reads, so nothing needs clearing.
constexpr int64_t kNoAllocRows = WP_NOALLOC_MOMENT_ROWS;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[8 * kNoAllocRows];
std::mutex scratch_mu;
double *scratch_dev[kMaxDevices] = {};

hipError_t scratch_on(int device, double **ptr) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[device]) {
    double *p = nullptr;
    hipError_t e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_dev[device] = p;
  }
  *ptr = scratch_dev[device];
  return hipSuccess;
}

}  // namespace

extern "C" {

wp_status wp_propagate_observe(wp_sim *s, uint64_t nsteps, uint32_t mask, double *out) {
  if (!s) return WP_EINVAL;
  if (!out) return fail(s, WP_EINVAL, "propagate_observe: NULL output");
  if (nsteps == 0 || nsteps > (uint64_t)1 << 40) return fail(s, WP_EINVAL, "propagate_observe: nsteps must be in 1..2^40");
  // Everything the closing pass cannot carry is a propagation followed by
  // wp_observables.
  if (!observe_fusable(s, mask)) {
    wp_status st = wp_propagate(s, nsteps);
    return st != WP_OK ? st : wp_observables(s, mask, out);
  }
  (void)hipSetDevice(s->device);
  if (hipError_t e0 = ensure_state(s); e0 != hipSuccess) return state_fail(s, e0, "propagate_observe");
  int64_t rows = 0;
  if (wp_status st = closing_rows(s, &rows); st != WP_OK) return st;
  hipError_t e = hipSuccess;
  if (rows > s->mpart_rows) {
    if (s->d_mpart) {
      e = hipStreamSynchronize(s->stream);  // earlier reductions may still read it
      (void)hipFree(s->d_mpart);
      s->d_mpart = nullptr;
      s->mpart_rows = 0;
    }
    if (e == hipSuccess) e = dev_alloc((void **)&s->d_mpart, sizeof(double) * 8 * (size_t)rows);
    if (e != hipSuccess) return hip_fail(s, e, "propagate_observe");
    s->mpart_rows = rows;
  }
  return observe_fused(s, nsteps, mask, out, s->d_mpart, rows, false, "propagate_observe");
}

wp_status wp_propagate_observe_noalloc(wp_sim *s, uint64_t nsteps, uint32_t mask, double *out) {
  if (!s) return WP_EINVAL;
  if (!out) return fail(s, WP_EINVAL, "propagate_observe_noalloc: NULL output");
  if (nsteps == 0 || nsteps > (uint64_t)1 << 40)
    return fail(s, WP_EINVAL, "propagate_observe_noalloc: nsteps must be in 1..2^40");
  if (!observe_fusable(s, mask))
    return fail(s, WP_EUNSUPPORTED,
                "propagate_observe_noalloc: needs a power-of-two 2D or 3D grid, the default order and a mask of "
                "norm, moments and widths only");
  (void)hipSetDevice(s->device);
  int64_t rows = 0;
  if (wp_status st = closing_rows(s, &rows); st != WP_OK) return st;
  if (rows > kNoAllocRows)
    return fail(s, WP_EUNSUPPORTED,
                "propagate_observe_noalloc: the closing pass has " + std::to_string(rows) +
                    " workgroups, more than the " + std::to_string(kNoAllocRows) + " rows of the fixed scratch");
  if (!s->psi) return fail(s, WP_ESTATE, "propagate_observe_noalloc: no state yet (set or bind one first)");
  double *mrows = nullptr;
  if (hipError_t e = scratch_on(s->device, &mrows); e != hipSuccess)
    return hip_fail(s, e, "propagate_observe_noalloc: scratch address");
  return observe_fused(s, nsteps, mask, out, mrows, rows, true, "propagate_observe_noalloc");
}

wp_status wp_get_time(wp_sim *s, double *t, uint64_t *step) {
  if (!s) return WP_EINVAL;
  if (t) *t = s->t0 + (double)s->step * s->g.dt;
  if (step) *step = s->step;
  return WP_OK;
}

wp_status wp_synchronize(wp_sim *s) {
  if (!s) return WP_EINVAL;
  (void)hipSetDevice(s->device);
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(s, e, "synchronize");
  return WP_OK;
}

}  // extern "C"

// ===========================================================================
// batches
// ===========================================================================

namespace {

// Argument-block variants per solve (index = solve * kVariants + variant).
enum : int { V_FIRST = 0, V_STEADY = 1, V_LAST = 2, K_LAST = 3, F_FWD = 4, F_INV = 5, kVariants = 6 };
// Position of a pass group within a step.
enum : int { SLOT_FFWD = 0, SLOT_K = 1, SLOT_FINV = 2, SLOT_V = 3 };
constexpr int kMaxSeqSteps = 64;  // steps per launch sequence (graph or direct)

struct PassGroup {
  int slot, prec, lgN, kind;
  bool strided;
  uint32_t item_off, nblocks;
  int tune;
  int lane;
};
// The solves of one pass group and their line counts (the block map is
// rebuilt from this when the group's kernel variant changes).
struct GroupSpec {
  int slot, prec, lgN, kind;
  bool strided;
  std::vector<std::pair<int, int64_t>> members;  // (solve, lines)
  int lane = 0;
};
// Pass groups that share no solve form independent chains across the slots
// of a step; the steady steps run them on up to kLanes streams (lane 0 is
// the launching stream), so that small groups fill the gaps and tails of
// large ones instead of running after them.
constexpr int kLanes = 3;
struct Group1D {
  int prec, lgN;
  uint32_t off, count;
};

}  // namespace

struct wp_batch {
  std::vector<wp_sim *> sims;
  hipStream_t stream = nullptr;
  int device = 0;
  int rows = kMaxSeqSteps + 1;
  uint32_t graph_steps = 0;
  wp::PassArgs *d_args = nullptr;
  wp::BatchItem *d_items = nullptr;
  wp::Solve1DArgs *d_args1d = nullptr;
  wp::PotDev *d_pots = nullptr;
  double *d_t0 = nullptr, *d_dt = nullptr, *d_coef = nullptr;
  // Step counters: [0, count) for the pass schedule (advanced on the device),
  // [count, 2 count) read by the 1D solvers.
  int64_t *d_step = nullptr;
  // Pinned host mirror of the counters, so that the per-call refresh is an
  // asynchronous copy; ev_step is recorded after that copy and guards the
  // mirror against being rewritten before the copy has run.
  int64_t *h_step = nullptr;
  hipEvent_t ev_step = nullptr;
  bool step_pending = false;
  std::vector<PassGroup> groups;
  std::vector<GroupSpec> specs;
  std::vector<Group1D> groups1d;
  // Members on mixed-length grids: advanced by their own schedule (the
  // launches wp_propagate makes), ordered within the batch's work.
  std::vector<int> solo;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint32_t exec_steps = 0;
  // Graphs are captured and replayed on a stream of the batch's own (the
  // caller's may be the legacy default stream, which cannot be captured),
  // ordered after and before the caller's work by events.
  hipStream_t cap_stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  // With both 1D and multi-axis members, the 1D solvers (a few workgroups
  // each, running all steps) go to a stream of their own so that they run
  // beside the pass launches instead of before them.
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // Lanes of the steady steps (see kLanes): streams and events of lanes
  // 1 .. lanes-1.
  int lanes = 1;
  hipStream_t lane_st[kLanes] = {};
  hipEvent_t ev_lfork = nullptr, ev_ljoin[kLanes] = {};
  std::string err;
};

namespace {

void batch_release(wp_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
  if (b->ev_join) (void)hipEventDestroy(b->ev_join);
  if (b->side) (void)hipStreamDestroy(b->side);
  for (int l = 1; l < kLanes; ++l) {
    if (b->lane_st[l]) (void)hipStreamDestroy(b->lane_st[l]);
    if (b->ev_ljoin[l]) (void)hipEventDestroy(b->ev_ljoin[l]);
  }
  if (b->ev_lfork) (void)hipEventDestroy(b->ev_lfork);
  if (b->ev_step) (void)hipEventDestroy(b->ev_step);
  if (b->h_step) (void)hipHostFree(b->h_step);
  for (void *p : {(void *)b->d_args, (void *)b->d_items, (void *)b->d_args1d, (void *)b->d_pots, (void *)b->d_t0,
                  (void *)b->d_dt, (void *)b->d_coef, (void *)b->d_step})
    if (p) (void)hipFree(p);
}

wp_status bfail(wp_batch *b, wp_status code, const std::string &msg) {
  if (b) b->err = msg;
  return code;
}

// Launch the pass groups of one slot of a step (of one lane, or of all for
// lane < 0).
hipError_t run_slot(wp_batch *b, hipStream_t st, int slot, int var, int row, int lane = -1) {
  for (const PassGroup &g : b->groups) {
    if (g.slot != slot || (lane >= 0 && g.lane != lane)) continue;
    wp::BatchLaunch L{};
    L.args = b->d_args;
    L.items = b->d_items + g.item_off;
    L.nblocks = (int)g.nblocks;
    L.nvar = kVariants;
    L.var = var;
    L.row = row;
    L.lgN = g.lgN;
    L.strided = g.strided;
    L.kind = g.kind;
    L.tune = g.tune;
    hipError_t r = wp::launch_batch_pass(g.prec, L, st);
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

// Block maps of all pass groups from the group specs and the tuning table:
// one item per (solve, tile), tiles sized for each group's variant.
std::vector<wp::BatchItem> build_items(wp_batch *b) {
  std::vector<wp::BatchItem> items;
  b->groups.clear();
  for (const GroupSpec &sp : b->specs) {
    const int tune = wp::effective_tune(sp.prec, sp.lgN, sp.kind, tune_for(1, sp.prec, sp.lgN, sp.strided, sp.kind));
    const int tile = wp::pass_tile(sp.prec, sp.lgN, sp.strided, sp.kind, tune);
    PassGroup g{sp.slot, sp.prec, sp.lgN, sp.kind, sp.strided, (uint32_t)items.size(), 0, tune, sp.lane};
    for (auto &m : sp.members) {
      const int64_t tiles = (m.second + tile - 1) / tile;
      for (int64_t t = 0; t < tiles; ++t) items.push_back({m.first, (int32_t)t});
    }
    g.nblocks = (uint32_t)(items.size() - g.item_off);
    b->groups.push_back(g);
  }
  return items;
}

hipError_t refresh_coef(wp_batch *b, hipStream_t st, int rows) {
  return wp::launch_coefficients_batch(b->d_pots, b->d_t0, b->d_dt, b->d_step, 0.0, (int)b->sims.size(), rows,
                                       b->rows, b->d_coef, st);
}

// k steady steps of the 2D/3D members (the middle passes of the step, then
// the merged full potential step and the forward transform of the first
// axis), then the device step counters advance by k.  Only kernel launches:
// this is what a graph captures.
// Lane l > 0 runs on its own stream, forked from `st` after the waveform
// table is filled and joined back before the counters advance.
hipError_t steady_steps(wp_batch *b, hipStream_t st, int k) {
  hipError_t e = refresh_coef(b, st, k + 1);
  if (b->lanes > 1 && e == hipSuccess) {
    e = hipEventRecord(b->ev_lfork, st);
    for (int l = 1; l < b->lanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(b->lane_st[l], b->ev_lfork, 0);
  }
  for (int l = 0; l < b->lanes && e == hipSuccess; ++l) {
    const hipStream_t q = l ? b->lane_st[l] : st;
    const int lane = b->lanes > 1 ? l : -1;
    for (int j = 0; j < k && e == hipSuccess; ++j) {
      e = run_slot(b, q, SLOT_FFWD, F_FWD, 0, lane);
      if (e == hipSuccess) e = run_slot(b, q, SLOT_K, K_LAST, 0, lane);
      if (e == hipSuccess) e = run_slot(b, q, SLOT_FINV, F_INV, 0, lane);
      if (e == hipSuccess) e = run_slot(b, q, SLOT_V, V_STEADY, j + 1, lane);
    }
  }
  for (int l = 1; l < b->lanes && e == hipSuccess; ++l) {
    e = hipEventRecord(b->ev_ljoin[l], b->lane_st[l]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, b->ev_ljoin[l], 0);
  }
  if (e == hipSuccess) e = wp::launch_step_advance(b->d_step, (int)b->sims.size(), k, st);
  return e;
}

// Lanes of the pass groups: groups sharing a solve are joined (union-find),
// and the resulting chains, largest first, go to the lane with the least
// work so far (work = lines x line length summed over the chain's groups).
int assign_lanes(std::vector<GroupSpec> &specs, int nsolves) {
  const int n = (int)specs.size();
  std::vector<int> parent(n);
  for (int i = 0; i < n; ++i) parent[i] = i;
  auto find = [&](int x) {
    while (parent[x] != x) x = parent[x] = parent[parent[x]];
    return x;
  };
  std::vector<int> first(nsolves, -1);
  for (int i = 0; i < n; ++i)
    for (auto &m : specs[i].members) {
      if (first[m.first] < 0) first[m.first] = i;
      else parent[find(i)] = find(first[m.first]);
    }
  std::vector<double> work(n, 0.0);
  for (int i = 0; i < n; ++i)
    for (auto &m : specs[i].members) work[find(i)] += (double)m.second * (double)(1 << specs[i].lgN);
  std::vector<int> roots;
  for (int i = 0; i < n; ++i)
    if (find(i) == i) roots.push_back(i);
  std::sort(roots.begin(), roots.end(), [&](int a, int c) { return work[a] > work[c] || (work[a] == work[c] && a < c); });
  const int lanes = (int)roots.size() < kLanes ? (int)roots.size() : kLanes;
  std::vector<double> load(kLanes, 0.0);
  std::vector<int> lane_of(n, 0);
  for (int r : roots) {
    int best = 0;
    for (int l = 1; l < lanes; ++l)
      if (load[l] < load[best]) best = l;
    lane_of[r] = best;
    load[best] += work[r];
  }
  for (int i = 0; i < n; ++i) specs[i].lane = lane_of[find(i)];
  return lanes < 1 ? 1 : lanes;
}

}  // namespace

extern "C" {

const char *wp_batch_last_error(const wp_batch *b) { return b ? b->err.c_str() : "NULL batch"; }

wp_status wp_batch_create(wp_sim *const *sims, uint32_t count, void *stream, wp_batch **out) {
  if (!out) return WP_EINVAL;
  *out = nullptr;
  if (!sims || count == 0) return WP_EINVAL;
  for (uint32_t i = 0; i < count; ++i)
    if (!sims[i] || sims[i]->order != WP_ORDER_VKV) return WP_EINVAL;
  wp_batch *b = new (std::nothrow) wp_batch();
  if (!b) return WP_ENOMEM;
  b->sims.assign(sims, sims + count);
  b->stream = (hipStream_t)stream;
  hipError_t e = hipGetDevice(&b->device);
  for (uint32_t i = 0; i < count && e == hipSuccess; ++i) e = ensure_state(b->sims[i]);
  // Per-solve host descriptors.
  std::vector<wp::PassArgs> args((size_t)count * kVariants);
  std::vector<wp::PotDev> pots(count);
  std::vector<double> t0(count), dt(count);
  std::vector<int64_t> steps(count);
  std::vector<wp::BatchItem> items;
  std::vector<wp::Solve1DArgs> a1d;
  // group key -> members
  struct Key {
    int slot, prec, lgN, kind;
    bool strided;
    bool operator<(const Key &o) const {
      return std::tie(slot, prec, lgN, kind, strided) < std::tie(o.slot, o.prec, o.lgN, o.kind, o.strided);
    }
  };
  std::map<Key, std::vector<std::pair<int, int64_t>>> members;  // (solve, lines)
  std::map<std::pair<int, int>, std::vector<int>> members1d;    // (prec, lgN) -> solves
  if (e == hipSuccess) {
    e = dev_alloc((void **)&b->d_coef, sizeof(double) * wp::CO_COUNT * (size_t)b->rows * count);
  }
  for (uint32_t i = 0; i < count && e == hipSuccess; ++i) {
    wp_sim *s = b->sims[i];
    pots[i] = s->pd;
    t0[i] = s->t0;
    dt[i] = s->g.dt;
    steps[i] = (int64_t)s->step;
    if (s->mixed) {
      b->solo.push_back((int)i);
      continue;
    }
    if (s->g.ndim == 1 && !s->split) {
      members1d[{s->prec, s->lg[0]}].push_back((int)i);
      continue;
    }
    const double tau_half = 0.5 * s->g.dt / s->g.hbar, tau_full = s->g.dt / s->g.hbar;
    const double *coef = b->d_coef + (size_t)i * b->rows * wp::CO_COUNT;
    const int last = s->vdim - 1;
    wp::PassArgs *A = &args[(size_t)i * kVariants];
    A[V_FIRST] = pass_args(s, 0, wp::OP_V | wp::OP_FWD);
    A[V_FIRST].vtau = tau_half;
    A[V_STEADY] = pass_args(s, 0, wp::OP_PRE_INV | wp::OP_V | wp::OP_FWD);
    A[V_STEADY].vtau = tau_full;
    A[V_LAST] = pass_args(s, 0, wp::OP_PRE_INV | wp::OP_V);
    A[V_LAST].vtau = tau_half;
    for (int v : {V_FIRST, V_STEADY, V_LAST}) A[v].coef = coef;
    A[K_LAST] = pass_args(s, last, wp::OP_FWD | wp::OP_K | wp::OP_POST_INV);
    if (s->vdim == 3) {
      A[F_FWD] = pass_args(s, 1, wp::OP_FWD);
      A[F_INV] = pass_args(s, 1, wp::OP_PRE_INV);
    }
    auto add = [&](int slot, int axis, int kind) {
      const wp::PassArgs &pa = A[slot == SLOT_V ? V_FIRST : slot == SLOT_K ? K_LAST : slot == SLOT_FFWD ? F_FWD : F_INV];
      const bool strided = pa.lg_inner > 0;
      members[{slot, s->prec, s->vlg[axis], kind, strided}].push_back({(int)i, pa.n_lines});
    };
    add(SLOT_V, 0, s->split ? 3 : 1);
    add(SLOT_K, last, s->split ? 4 : 2);
    if (s->vdim == 3) {
      add(SLOT_FFWD, 1, 0);
      add(SLOT_FINV, 1, 0);
    }
  }
  if (e == hipSuccess) {
    for (auto &kv : members)
      b->specs.push_back({kv.first.slot, kv.first.prec, kv.first.lgN, kv.first.kind, kv.first.strided, kv.second});
    b->lanes = assign_lanes(b->specs, (int)count);
    items = build_items(b);
    for (auto &kv : members1d) {
      Group1D g{kv.first.first, kv.first.second, (uint32_t)a1d.size(), (uint32_t)kv.second.size()};
      for (int i : kv.second) {
        wp_sim *s = b->sims[i];
        wp::Solve1DArgs a{};
        a.psi = s->psi;
        a.g = s->gd;
        a.nsteps = 0;
        a.time.t0 = s->t0;
        a.time.dt = s->g.dt;
        a.time.step = 0;
        a.time.half = 0.0;
        a.vtau_half = 0.5 * s->g.dt / s->g.hbar;
        a.vtau_full = s->g.dt / s->g.hbar;
        a.order = WP_ORDER_VKV;
        a.pot = s->pd;
        a.kfull = s->d_kfull;
        a.khalf = s->d_khalf;
        a.tw = s->d_tw[0];
        a1d.push_back(a);
      }
      b->groups1d.push_back(g);
    }
  }
  if (e == hipSuccess) e = dev_alloc((void **)&b->d_step, sizeof(int64_t) * 2 * count);
  if (e == hipSuccess) e = host_alloc((void **)&b->h_step, sizeof(int64_t) * 2 * count);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_step, hipEventDisableTiming);
  // The 1D argument blocks read their step from the second set of counters.
  for (size_t j = 0, gi = 0; e == hipSuccess && gi < b->groups1d.size(); ++gi)
    for (int i : members1d[{b->groups1d[gi].prec, b->groups1d[gi].lgN}])
      a1d[j++].time.step_dev = b->d_step + count + i;
  if (e == hipSuccess && (!b->groups1d.empty() || !b->solo.empty()) && !b->groups.empty()) {
    e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming);
  }
  if (e == hipSuccess && b->lanes > 1) {
    e = hipEventCreateWithFlags(&b->ev_lfork, hipEventDisableTiming);
    for (int l = 1; l < b->lanes && e == hipSuccess; ++l) {
      e = hipStreamCreateWithFlags(&b->lane_st[l], hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_ljoin[l], hipEventDisableTiming);
    }
  }
  if (e == hipSuccess) e = upload(&b->d_args, args);
  if (e == hipSuccess && !items.empty()) e = upload(&b->d_items, items);
  if (e == hipSuccess && !a1d.empty()) e = upload(&b->d_args1d, a1d);
  if (e == hipSuccess) e = upload(&b->d_pots, pots);
  if (e == hipSuccess) e = upload(&b->d_t0, t0);
  if (e == hipSuccess) e = upload(&b->d_dt, dt);
  if (e != hipSuccess) {
    batch_release(b);
    delete b;
    return e == hipErrorOutOfMemory ? WP_ENOMEM : WP_EDEVICE;
  }
  *out = b;
  return WP_OK;
}

wp_status wp_batch_set_graph_steps(wp_batch *b, uint32_t k) {
  if (!b) return WP_EINVAL;
  if (k > (uint32_t)kMaxSeqSteps) return bfail(b, WP_EINVAL, "graph steps must be in 0..64");
  b->graph_steps = k;
  return WP_OK;
}

wp_status wp_batch_propagate(wp_batch *b, uint64_t nsteps) {
  if (!b) return WP_EINVAL;
  if (nsteps == 0) return WP_OK;
  (void)hipSetDevice(b->device);
  const int count = (int)b->sims.size();
  // The members' host counters are authoritative: refresh the device copy.
  hipError_t e = b->step_pending ? hipEventSynchronize(b->ev_step) : hipSuccess;
  for (int i = 0; e == hipSuccess && i < count; ++i) b->h_step[i] = b->h_step[count + i] = (int64_t)b->sims[i]->step;
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_step, b->h_step, sizeof(int64_t) * 2 * count, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->ev_step, b->stream);
  if (e == hipSuccess) b->step_pending = true;
  // 1D members: all steps in one launch per line-length class.
  hipStream_t st1d = b->side ? b->side : b->stream;
  if (e == hipSuccess && b->side) {
    e = hipEventRecord(b->ev_fork, b->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->side, b->ev_fork, 0);
  }
  for (const Group1D &g : b->groups1d) {
    if (e != hipSuccess) break;
    e = wp::launch_solve1d_batch(g.prec, g.lgN, b->d_args1d + g.off, (int)g.count, (int64_t)nsteps, st1d);
  }
  // Mixed-length members: their own schedule, on the same stream as the 1D
  // solvers.
  for (int i : b->solo) {
    if (e != hipSuccess) break;
    wp_sim *s = b->sims[i];
    const hipStream_t own = s->stream;
    s->stream = st1d;
    e = run_schedule(s, nsteps, [](int, auto &&fn) { return fn(); });
    s->stream = own;
  }
  // 2D/3D members: open (potential half step at t_n and forward transform of
  // the first axis), nsteps-1 steady steps, and a final step closing with the
  // potential half step: the same sequence as wp_propagate, however the
  // steady steps are split between graph replays and direct launches.
  if (e == hipSuccess && !b->groups.empty()) {
    e = refresh_coef(b, b->stream, 1);
    if (e == hipSuccess) e = run_slot(b, b->stream, SLOT_V, V_FIRST, 0);
    uint64_t left = nsteps - 1;
    const uint32_t k = b->graph_steps;
    if (e == hipSuccess && k > 0 && left >= k) {
      if (!b->cap_stream) {
        e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
      }
      if (e == hipSuccess && (!b->exec || b->exec_steps != k)) {
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
        e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
          hipError_t ce = steady_steps(b, b->cap_stream, (int)k);
          e = hipStreamEndCapture(b->cap_stream, &b->graph);
          if (ce != hipSuccess) e = ce;
        }
        if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
        if (e == hipSuccess) b->exec_steps = k;
      }
      if (e == hipSuccess) e = hipEventRecord(b->ev_in, b->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->cap_stream, b->ev_in, 0);
      while (e == hipSuccess && left >= k) {
        e = hipGraphLaunch(b->exec, b->cap_stream);
        left -= k;
      }
      if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->cap_stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_out, 0);
    }
    while (e == hipSuccess && left > 0) {
      const int kk = (int)(left < (uint64_t)kMaxSeqSteps ? left : (uint64_t)kMaxSeqSteps);
      e = steady_steps(b, b->stream, kk);
      left -= (uint64_t)kk;
    }
    // final step
    if (e == hipSuccess) e = refresh_coef(b, b->stream, 2);
    if (e == hipSuccess) e = run_slot(b, b->stream, SLOT_FFWD, F_FWD, 0);
    if (e == hipSuccess) e = run_slot(b, b->stream, SLOT_K, K_LAST, 0);
    if (e == hipSuccess) e = run_slot(b, b->stream, SLOT_FINV, F_INV, 0);
    if (e == hipSuccess) e = run_slot(b, b->stream, SLOT_V, V_LAST, 1);
  }
  if (e == hipSuccess && b->side) {
    e = hipEventRecord(b->ev_join, b->side);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_join, 0);
  }
  if (e != hipSuccess) return bfail(b, WP_EDEVICE, std::string("batch_propagate: ") + hipGetErrorString(e));
  for (wp_sim *s : b->sims) s->step += nsteps;
  b->err.clear();
  return WP_OK;
}

wp_status wp_batch_autotune(wp_batch *b, uint32_t reps) {
  if (!b) return WP_EINVAL;
  if (reps < 1 || reps > 10000) return bfail(b, WP_EINVAL, "batch_autotune: reps must be in 1..10000");
  if (b->specs.empty()) {
    b->err.clear();
    return WP_OK;
  }
  (void)hipSetDevice(b->device);
  const int count = (int)b->sims.size();
  hipError_t e = hipStreamSynchronize(b->stream);
  // The candidates transform the members' states in place: save and restore.
  std::vector<char> saved(count, 0);
  for (const GroupSpec &sp : b->specs)
    for (auto &m : sp.members) saved[m.first] = 1;
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    if (!saved[i]) continue;
    wp_sim *s = b->sims[i];
    if (!s->scratch) e = dev_alloc(&s->scratch, s->psi_bytes);
    if (e == hipSuccess) e = hipMemcpyAsync(s->scratch, s->psi, s->psi_bytes, hipMemcpyDeviceToDevice, b->stream);
  }
  // Waveform rows for the members' current steps (potential passes read row 0).
  for (int i = 0; i < count && e == hipSuccess; ++i) b->h_step[i] = b->h_step[count + i] = (int64_t)b->sims[i]->step;
  if (e == hipSuccess)
    e = hipMemcpyAsync(b->d_step, b->h_step, sizeof(int64_t) * 2 * count, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = refresh_coef(b, b->stream, 1);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  b->step_pending = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = timing_event(&e0);
  if (e == hipSuccess) e = timing_event(&e1);
  for (const GroupSpec &sp : b->specs) {
    if (e != hipSuccess) break;
    const int var = sp.slot == SLOT_V ? V_STEADY : sp.slot == SLOT_K ? K_LAST : sp.slot == SLOT_FFWD ? F_FWD : F_INV;
    int cand[4];
    const int nc = wp::tune_candidates(sp.prec, sp.lgN, sp.kind, cand);
    if (nc < 2) continue;
    int best = 0;
    double best_ms = 0.0;
    for (int c = 0; c < nc && e == hipSuccess; ++c) {
      const int tile = wp::pass_tile(sp.prec, sp.lgN, sp.strided, sp.kind, cand[c]);
      std::vector<wp::BatchItem> items;
      for (auto &m : sp.members)
        for (int64_t t = 0; t < (m.second + tile - 1) / tile; ++t) items.push_back({m.first, (int32_t)t});
      wp::BatchItem *d_items = nullptr;
      e = upload(&d_items, items);
      wp::BatchLaunch L{};
      L.args = b->d_args;
      L.items = d_items;
      L.nblocks = (int)items.size();
      L.nvar = kVariants;
      L.var = var;
      L.row = 0;
      L.lgN = sp.lgN;
      L.strided = sp.strided;
      L.kind = sp.kind;
      L.tune = cand[c];
      if (e == hipSuccess) e = wp::launch_batch_pass(sp.prec, L, b->stream);  // warm-up
      if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
      for (uint32_t r = 0; r < reps && e == hipSuccess; ++r) e = wp::launch_batch_pass(sp.prec, L, b->stream);
      if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float m = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&m, e0, e1);
      if (d_items) (void)hipFree(d_items);
      if (e == hipSuccess && (c == 0 || m < best_ms)) {
        best = cand[c];
        best_ms = m;
      }
    }
    if (e == hipSuccess) tune_store(1, sp.prec, sp.lgN, sp.strided, sp.kind, best);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (int i = 0; i < count && e == hipSuccess; ++i)
    if (saved[i])
      e = hipMemcpyAsync(b->sims[i]->psi, b->sims[i]->scratch, b->sims[i]->psi_bytes, hipMemcpyDeviceToDevice,
                         b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  // New block maps for the chosen variants; the captured graph is stale.
  if (e == hipSuccess) {
    std::vector<wp::BatchItem> items = build_items(b);
    if (b->d_items) (void)hipFree(b->d_items);
    b->d_items = nullptr;
    if (!items.empty()) e = upload(&b->d_items, items);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->exec_steps = 0;
  }
  if (e != hipSuccess) return bfail(b, WP_EDEVICE, std::string("batch_autotune: ") + hipGetErrorString(e));
  b->err.clear();
  return WP_OK;
}

wp_status wp_tune_get(int32_t batched, int32_t prec, int32_t lg_n, int32_t strided, int32_t kind, int32_t *tune) {
  if (!tune) return WP_EINVAL;
  *tune = tune_for(batched ? 1 : 0, prec, lg_n, strided != 0, kind);
  return WP_OK;
}

wp_status wp_tune_set(int32_t batched, int32_t prec, int32_t lg_n, int32_t strided, int32_t kind, int32_t tune) {
  if (prec < WP_C64 || prec > WP_C64X || lg_n < 1 || lg_n > 12 || kind < 0 || kind > 4 || tune < 0 ||
      tune >= wp::kTuneSlots)
    return WP_EINVAL;
  tune_store(batched ? 1 : 0, prec, lg_n, strided != 0, kind, tune);
  return WP_OK;
}

void wp_tune_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune.clear();
}

wp_status wp_batch_destroy(wp_batch *b) {
  if (!b) return WP_EINVAL;
  (void)hipSetDevice(b->device);
  (void)hipStreamSynchronize(b->stream);
  batch_release(b);
  delete b;
  return WP_OK;
}

}  // extern "C"
