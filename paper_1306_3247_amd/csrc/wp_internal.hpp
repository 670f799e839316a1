// wp_internal.hpp -- kernel argument blocks and launcher entry points shared
// by the kernel translation unit and the C ABI.
#pragma once
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wp_device.hpp"

namespace wp {

// Operations of one line pass, applied in this order.
enum : uint32_t {
  OP_PRE_INV = 1u << 0,   // inverse line FFT (unnormalised)
  OP_V = 1u << 1,         // multiply by exp(-i V(x,t) vtau)
  OP_FWD = 1u << 2,       // forward line FFT
  OP_K = 1u << 3,         // multiply by the kinetic factor (1/N folded in)
  OP_POST_INV = 1u << 4,  // inverse line FFT
  // A 1D grid of n = n1*n2 points transformed as [n1][n2] (a four-step
  // transform): the pass along axis 0 applies the twiddles exp(-+2 pi i j2 k1/n)
  // next to its transforms, the pass along axis 1 the kinetic factor of bin
  // k1 + n1*k2.
  OP_SPLIT = 1u << 5,
  // Cache hints for the pass's HBM reads / writes (results unchanged).
  OP_LOAD_NT = 1u << 6,
  OP_STORE_NT = 1u << 7,
};

struct GridDev {
  int32_t ndim;
  int32_t lg[3];  // log2 of the axis lengths (0 on unused axes; power-of-two grids)
  double lo[3], dx[3];
  int32_t n[3];   // axis lengths (1 on unused axes)
  int32_t pow2;   // every length a power of two: indices by shifts, else by division
  // Storage: point i of the row-major grid sits at i + (i >> lg_plane) * pad,
  // i.e. consecutive first-axis planes of 2^lg_plane points lie
  // 2^lg_plane + pad points apart (pad = 0: contiguous).
  int32_t lg_plane;
  int32_t pad;
};

// Storage position of point i of the row-major grid.
__device__ __forceinline__ int64_t phys_index(const GridDev &g, int64_t i) {
  return i + (i >> g.lg_plane) * (int64_t)g.pad;
}

// Indices (i0, i1, i2) of point i of the row-major [n0][n1][n2] grid.
__device__ __forceinline__ void grid_index(const GridDev &g, int64_t i, int &i0, int &i1, int &i2) {
  if (g.pow2) {
    i2 = (int)(i & ((1 << g.lg[2]) - 1));
    i1 = (int)((i >> g.lg[2]) & ((1 << g.lg[1]) - 1));
    i0 = (int)(i >> (g.lg[1] + g.lg[2]));
  } else {
    i2 = (int)(i % g.n[2]);
    const int64_t r = i / g.n[2];
    i1 = (int)(r % g.n[1]);
    i0 = (int)(r / g.n[1]);
  }
}

// Time of a potential evaluation: t = t0 + (step + (step_dev ? *step_dev : 0)) * dt
// (time by multiplication, never by accumulation).
struct TimeDev {
  double t0, dt;
  int64_t step;
  const int64_t *step_dev;
  double half;  // 0.5 to sample at the step midpoint, else 0
};

__device__ __forceinline__ double time_of(const TimeDev &T) {
  int64_t n = T.step + (T.step_dev ? *T.step_dev : 0);
  return T.t0 + ((double)n + T.half) * T.dt;
}

// Time of step s after the first (plus `half` of a step).
__device__ __forceinline__ double step_time_of(const TimeDev &T, int64_t s, double half) {
  int64_t n = T.step + s + (T.step_dev ? *T.step_dev : 0);
  return T.t0 + ((double)n + half) * T.dt;
}

struct PassArgs {
  void *psi;
  GridDev g;
  int32_t axis;      // line axis
  int32_t lg_inner;  // log2 of the product of the axis lengths after `axis`
  int64_t n_lines;
  uint32_t ops;
  const double *coef;  // OP_V: the CO_COUNT waveform values at this pass's time
  double vtau;         // phase = V * vtau (dt/2hbar or dt/hbar)
  PotDev pot;
  const cx<double> *ktab[3];  // kinetic factors per axis (OP_K)
  const cx<double> *tw;       // twiddles exp(-2 pi i e/N), e < N
  // OP_SPLIT: exp(-2 pi i e/n) = wsplit[0][e >> split_h] * wsplit[1][e & (2^split_h - 1)]
  // for 0 <= e < n = 2^g.lg[0]; split_h = log2 n1.
  const cx<double> *wsplit[2];
  int32_t split_h;
  int32_t tune;  // kernel variant (see pass_cfg); 0 = default
  // Closing first-axis pass only (edge_pass_kernel): if set, workgroup b
  // also writes the FP64 moment sums of its final values to moments[8b ..]
  // in the slot layout of the observables' block partials.
  double *moments;
};

struct Solve1DArgs {
  void *psi;
  GridDev g;
  int64_t nsteps;
  TimeDev time;       // step = index of the first step
  double vtau_half;   // dt/2hbar
  double vtau_full;   // dt/hbar
  int32_t order;      // 0: V-K-V, 1: K-V-K
  PotDev pot;
  const cx<double> *kfull;  // exp(-i hbar k^2 dt/2m)/N
  const cx<double> *khalf;  // exp(-i hbar k^2 dt/4m)/N (K-V-K order)
  const cx<double> *tw;
};

struct ObsArgs {
  const void *psi;
  GridDev g;
  int64_t total;
  int32_t with_v;     // accumulate V|psi|^2
  int32_t kinetic;    // psi is in momentum space: accumulate k^2 |psi|^2
  double t;
  PotDev pot;
  const double *k2tab[3];  // k^2 per axis (kinetic)
  double *partials;        // [blocks][8]
  // kinetic on a split 1D grid: point i = k1*n2 + k2 holds bin k1 + n1*k2,
  // n1 = 2^split_h (0: not split)
  int32_t split_h;
};

// One workgroup of a batched pass: tile `tile` of solve `solve`.
struct BatchItem {
  int32_t solve;
  int32_t tile;
};

// A batched pass launch: `nblocks` workgroups described by `items`, all of
// the same precision, line length 2^lgN, layout and kind.
struct BatchLaunch {
  const PassArgs *args;
  const BatchItem *items;
  int nblocks;
  int nvar, var, row;
  int lgN;
  bool strided;
  int kind;  // 0 FFT only, 1 potential, 2 kinetic, 3 / 4 split 1D potential / kinetic
  int tune;  // kernel variant
};

// ---- mixed-radix lengths (any 2^a 3^b 5^c 7^d up to kMaxMixed) ----------
// Stage plan of one line transform (Stockham, radices 2, 3, 4, 5, 7, 8):
// stage s has radix radix[s], LS = product of the earlier radices, and its
// twiddles exp(-2 pi i r k/(radix LS)) at twoff[s] + (r-1) LS + k.
constexpr int kMaxStages = 12;
constexpr int kMaxMixed = 4096;
struct GPlan {
  int32_t nst;
  int32_t radix[kMaxStages], ls[kMaxStages], twoff[kMaxStages];
};

// A line pass on a grid with lengths that are not all powers of two.
struct GPassArgs {
  PassArgs p;     // as for the power-of-two passes (g.n gives the lengths)
  int64_t inner;  // product of the lengths after the line axis
  GPlan plan;     // of the line axis; p.tw holds its stage twiddles
};

// Events to attach to the next kernel dispatch of this host thread.  When
// `start` is set, the launchers of a single-handle schedule (line passes,
// mixed-radix passes, 1D solves, waveform coefficients) launch through
// hipExtLaunchKernel, so that the two events take the start and end times of
// that dispatch itself, with no marker between kernels, and set `used`.
struct DispatchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  bool used = false;
};
inline thread_local DispatchEvents tl_dispatch_events;

template <class K, class... A>
inline hipError_t launch_kernel(K kernel, dim3 grid, dim3 block, hipStream_t s, A... args) {
  DispatchEvents &d = tl_dispatch_events;
  if (d.start) {
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, d.start, d.stop, 0, args...);
    d.used = true;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
  }
  return hipGetLastError();
}

// The same with `shm` bytes of dynamic LDS.
template <class K, class... A>
inline hipError_t launch_kernel_shm(K kernel, dim3 grid, dim3 block, size_t shm, hipStream_t s, A... args) {
  DispatchEvents &d = tl_dispatch_events;
  if (d.start) {
    hipExtLaunchKernelGGL(kernel, grid, block, shm, s, d.start, d.stop, 0, args...);
    d.used = true;
  } else {
    hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
  }
  return hipGetLastError();
}

// Launchers (return hipSuccess or the launch error).
hipError_t launch_pass(int prec, const PassArgs &a, hipStream_t s);
hipError_t launch_solve1d(int prec, const Solve1DArgs &a, hipStream_t s);
// Mixed-radix line pass; prec is the handle's wp_precision (1 FP32, 2 FP64,
// 3 FP32 state with FP64 arithmetic).
hipError_t launch_gpass(int prec, const GPassArgs &a, hipStream_t s);
// 1D solve of any supported mixed length in one workgroup (a.g.n[0] points).
hipError_t launch_gsolve1d(int prec, const Solve1DArgs &a, const GPlan &plan, hipStream_t s);
hipError_t launch_gaussian(int prec, void *psi, const GridDev &g, const cx<double> *f0,
                           const cx<double> *f1, const cx<double> *f2, hipStream_t s);
hipError_t launch_observables(int prec, const ObsArgs &a, int blocks, double *out8, hipStream_t s);
// Sum `blocks` rows of 8 partials in index order into out8 (the final step
// of the observables' reduction).
hipError_t launch_reduce8(const double *partials, int blocks, double *out8, hipStream_t s);
// <phi|psi> without dV over `total` points: out8[0], out8[1] (precisions
// 1 = complex64, 2 = complex128); point i of phi (psi) is stored at
// i + (i >> lg_plane) * phi_pad (psi_pad).
hipError_t launch_inner(int phi_prec, const void *phi, int psi_prec, const void *psi, int64_t total, int lg_plane,
                        int phi_pad, int psi_pad, int blocks, double *partials, double *out8, hipStream_t s);
// Waveform values for `count` consecutive steps: out[j*CO_COUNT + w] is
// waveform w at the time of step T.step + j (plus T.half).
hipError_t launch_coefficients(const PotDev &p, const TimeDev &T, int count, double *out, hipStream_t s);

// Largest line length (points) supported by the line-pass kernels and by the
// single-workgroup 1D solver.
constexpr int kMaxLinePass = 4096;
constexpr int kMaxLine1D = 8192;
// Longer 1D grids use the split transform: n1, n2 between 128 and 1024.
constexpr int kMaxSplit1D = 1 << 20;
constexpr int kObsThreads = 256;
constexpr int kCoefChunk = 1024;  // steps per coefficient table

bool pass_supported(int prec, int lgN);
hipError_t launch_batch_pass(int prec, const BatchLaunch &b, hipStream_t s);
// Lines per workgroup of the variant that launch_*pass runs for `tune`.
int pass_tile(int prec, int lgN, bool strided, int kind, int tune);
// The variant actually run for a requested one (variants are compiled for
// some precisions, lengths and kinds only; elsewhere 0 runs).
int effective_tune(int prec, int lgN, int kind, int tune);
// Variants of a line pass (the tuning table's values are 0..kTuneSlots-1).
constexpr int kTuneSlots = 4;
// Distinct variants worth trying for a precision, line length and kind.
int tune_candidates(int prec, int lgN, int kind, int *out4);
// 1D solves in one launch, one workgroup each (all of line length 2^lgN).
hipError_t launch_solve1d_batch(int prec, int lgN, const Solve1DArgs *args, int count, int64_t nsteps,
                                hipStream_t s);
// step[i] += k for i < count.
hipError_t launch_step_advance(int64_t *step, int count, int64_t k, hipStream_t s);
// Waveform values for many solves: out[(i*stride + j)*CO_COUNT + w], j < rows,
// is waveform w of solve i at the time of step step_dev[i] + j (plus half).
hipError_t launch_coefficients_batch(const PotDev *pots, const double *t0, const double *dt,
                                     const int64_t *step_dev, double half, int count, int rows, int stride,
                                     double *out, hipStream_t s);

}  // namespace wp
