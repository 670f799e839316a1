// wp_kernels.hip -- HIP kernels of the split-operator step for gfx950.
//
// Data layout: psi is row-major [n0][n1][n2], interleaved complex, FP32 or
// FP64.  A multi-dimensional step is a sequence of line passes.  Each pass
// reads every line along one axis from HBM once, does all of its work in
// registers and LDS (inverse FFT, potential phase, forward FFT, kinetic
// phase, ...) and writes the line back once.
#include "wp_pass.hpp"

namespace wp {

#define WP_DECLARE_VARIANT(P, T)                                              \
  hipError_t dispatch_pass_##P##_##T(int lgN, const PassArgs &a, hipStream_t s); \
  hipError_t dispatch_batch_##P##_##T(const BatchLaunch &b, hipStream_t s);     \
  int pass_tile_##P##_##T(int lgN, bool strided, int kind);
WP_DECLARE_VARIANT(c64, 0)
WP_DECLARE_VARIANT(c64, 1)
WP_DECLARE_VARIANT(c64, 2)
WP_DECLARE_VARIANT(c64, 3)
WP_DECLARE_VARIANT(c128, 0)
WP_DECLARE_VARIANT(c128, 2)
WP_DECLARE_VARIANT(c64x, 0)
#undef WP_DECLARE_VARIANT

bool pass_supported(int prec, int lgN) { return prec >= 1 && prec <= 3 && lgN >= 1 && lgN <= 12; }

int effective_tune(int prec, int lgN, int kind, int tune) {
  if (kind > 2 || lgN < 6 || lgN > 10 || tune < 0) return 0;
  if (prec == 1) return tune & 3;
  if (prec == 2) return tune & 2;
  return 0;
}

int tune_candidates(int prec, int lgN, int kind, int *out4) {
  int n = 0;
  for (int t = 0; t < 4; ++t)
    if (effective_tune(prec, lgN, kind, t) == t) out4[n++] = t;
  return n;
}

// Line length of a pass: the axis length, or on a split 1D grid n1 =
// 2^split_h (axis 0) and n2 = n/n1 (axis 1).
static int pass_lgN(const PassArgs &a) {
  return a.split_h > 0 ? (a.axis == 0 ? a.split_h : a.g.lg[0] - a.split_h) : a.g.lg[a.axis];
}

hipError_t launch_pass(int prec, const PassArgs &a, hipStream_t s) {
  const int lgN = pass_lgN(a);
  if (!pass_supported(prec, lgN)) return hipErrorInvalidValue;
  if ((a.ops & OP_V) && (a.ops & OP_K)) return hipErrorInvalidValue;
  const int t = effective_tune(prec, lgN, pass_kind_of(a), a.tune);
  if (prec == 2) return t ? dispatch_pass_c128_2(lgN, a, s) : dispatch_pass_c128_0(lgN, a, s);
  if (prec == 3) return dispatch_pass_c64x_0(lgN, a, s);
  switch (t) {
    case 1: return dispatch_pass_c64_1(lgN, a, s);
    case 2: return dispatch_pass_c64_2(lgN, a, s);
    case 3: return dispatch_pass_c64_3(lgN, a, s);
    default: return dispatch_pass_c64_0(lgN, a, s);
  }
}

hipError_t launch_batch_pass(int prec, const BatchLaunch &b, hipStream_t s) {
  if (!pass_supported(prec, b.lgN) || b.nblocks <= 0) return hipErrorInvalidValue;
  const int t = effective_tune(prec, b.lgN, b.kind, b.tune);
  if (prec == 2) return t ? dispatch_batch_c128_2(b, s) : dispatch_batch_c128_0(b, s);
  if (prec == 3) return dispatch_batch_c64x_0(b, s);
  switch (t) {
    case 1: return dispatch_batch_c64_1(b, s);
    case 2: return dispatch_batch_c64_2(b, s);
    case 3: return dispatch_batch_c64_3(b, s);
    default: return dispatch_batch_c64_0(b, s);
  }
}

int pass_tile(int prec, int lgN, bool strided, int kind, int tune) {
  if (!pass_supported(prec, lgN)) return 0;
  const int t = effective_tune(prec, lgN, kind, tune);
  if (prec == 2) return t ? pass_tile_c128_2(lgN, strided, kind) : pass_tile_c128_0(lgN, strided, kind);
  if (prec == 3) return pass_tile_c64x_0(lgN, strided, kind);
  switch (t) {
    case 1: return pass_tile_c64_1(lgN, strided, kind);
    case 2: return pass_tile_c64_2(lgN, strided, kind);
    case 3: return pass_tile_c64_3(lgN, strided, kind);
    default: return pass_tile_c64_0(lgN, strided, kind);
  }
}

// ---------------------------------------------------------------------------
// 1D solve in one workgroup: the whole line stays in registers and LDS for
// all steps; HBM is read once and written once.
// ---------------------------------------------------------------------------
template <class S, class R, int N>
__device__ __forceinline__ void solve1d_body(const Solve1DArgs &a, int64_t nsteps) {
  using T = typename storage<S>::type;
  constexpr int L = fft_shape<N>::L, VPT = fft_shape<N>::VPT;
  static_assert(VPT <= 8, "one thread holds at most 8 values here");
  constexpr int NP = N >= 16 ? N + N / 16 : N;
  __shared__ cx<R> s_data[N > 8 ? NP : 1];
  __shared__ double s_coef[CO_COUNT];
  const int t = threadIdx.x;
  T *psi = (T *)a.psi;

  cx<R> v[VPT];
  cx<double> kf[VPT];
  double xs[VPT];
  const bool kvk = a.order == 1;
#pragma unroll
  for (int u = 0; u < VPT; ++u) {
    v[u] = load_as<R>(psi + t + L * u);
    kf[u] = kvk ? a.khalf[t + L * u] : a.kfull[t + L * u];
    xs[u] = a.g.lo[0] + (double)(t + L * u) * a.g.dx[0];
  }
  auto lds = [&](int p) -> cx<R> & { return s_data[p]; };

  auto apply_v = [&](double time, double vtau) {
    __syncthreads();
    for (int k = t; k < CO_COUNT; k += L) s_coef[k] = wave_value(a.pot.w[k], time);
    __syncthreads();
    const double ca = s_coef[CO_A], cb = s_coef[CO_B], cc = s_coef[CO_C], cs = s_coef[CO_S];
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      double th = cc + (ca * xs[u] + cb * xs[u] * xs[u]);
      if (a.pot.v0_kind != 0) th += cs * v0_value(a.pot, xs[u], 0.0, 0.0, 1);
      v[u] = mul_acc(v[u], expmi_wave(vtau * th));
    }
  };
  auto apply_k = [&](bool half_factor) {
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      cx<double> f = kf[u];
      if (half_factor) f = a.khalf[t + L * u];
      v[u] = mul_acc(v[u], f);
    }
  };

  const int64_t ns = nsteps;
  if (!kvk) {
    for (int64_t s = 0; s < ns; ++s) {
      if (s == 0) apply_v(step_time_of(a.time, 0, 0.0), a.vtau_half);
      line_fft<N, VPT, false>(v, t, a.tw, lds);
      apply_k(false);
      line_fft<N, VPT, true>(v, t, a.tw, lds);
      apply_v(step_time_of(a.time, s + 1, 0.0), s + 1 == ns ? a.vtau_half : a.vtau_full);
    }
  } else if (ns > 0) {
    // K/2 V K/2 with consecutive kinetic halves merged into full steps.
    line_fft<N, VPT, false>(v, t, a.tw, lds);
    apply_k(true);
    for (int64_t s = 0; s < ns; ++s) {
      line_fft<N, VPT, true>(v, t, a.tw, lds);
      apply_v(step_time_of(a.time, s, 0.5), a.vtau_full);
      line_fft<N, VPT, false>(v, t, a.tw, lds);
      if (s + 1 == ns) {
        apply_k(true);
      } else {
#pragma unroll
        for (int u = 0; u < VPT; ++u) v[u] = mul_acc(v[u], a.kfull[t + L * u]);
      }
    }
    line_fft<N, VPT, true>(v, t, a.tw, lds);
  }
#pragma unroll
  for (int u = 0; u < VPT; ++u) store_from(psi + t + L * u, v[u]);
}

template <class S, class R, int N>
__global__ void __launch_bounds__(fft_shape<N>::L) solve1d_kernel(Solve1DArgs a) {
  solve1d_body<S, R, N>(a, a.nsteps);
}

// One workgroup per solve.
template <class S, class R, int N>
__global__ void __launch_bounds__(fft_shape<N>::L) solve1d_batch_kernel(const Solve1DArgs *args, int64_t nsteps) {
  solve1d_body<S, R, N>(args[blockIdx.x], nsteps);
}

template <class S, class R, int N>
static hipError_t launch_solve1d_t(const Solve1DArgs &a, hipStream_t s, const Solve1DArgs *batch, int count) {
  if (batch)
    hipLaunchKernelGGL((solve1d_batch_kernel<S, R, N>), dim3(count), dim3(fft_shape<N>::L), 0, s, batch, a.nsteps);
  else
    return launch_kernel(solve1d_kernel<S, R, N>, dim3(1), dim3(fft_shape<N>::L), s, a);
  return hipGetLastError();
}

template <class S, class R>
static hipError_t dispatch_solve1d(int lgN, const Solve1DArgs &a, hipStream_t s, const Solve1DArgs *batch,
                                   int count) {
  switch (lgN) {
    case 1: return launch_solve1d_t<S, R, 2>(a, s, batch, count);
    case 2: return launch_solve1d_t<S, R, 4>(a, s, batch, count);
    case 3: return launch_solve1d_t<S, R, 8>(a, s, batch, count);
    case 4: return launch_solve1d_t<S, R, 16>(a, s, batch, count);
    case 5: return launch_solve1d_t<S, R, 32>(a, s, batch, count);
    case 6: return launch_solve1d_t<S, R, 64>(a, s, batch, count);
    case 7: return launch_solve1d_t<S, R, 128>(a, s, batch, count);
    case 8: return launch_solve1d_t<S, R, 256>(a, s, batch, count);
    case 9: return launch_solve1d_t<S, R, 512>(a, s, batch, count);
    case 10: return launch_solve1d_t<S, R, 1024>(a, s, batch, count);
    case 11: return launch_solve1d_t<S, R, 2048>(a, s, batch, count);
    case 12: return launch_solve1d_t<S, R, 4096>(a, s, batch, count);
    case 13: return launch_solve1d_t<S, R, 8192>(a, s, batch, count);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_solve1d(int prec, const Solve1DArgs &a, hipStream_t s) {
  const int lgN = a.g.lg[0];
  if (prec == 2) return dispatch_solve1d<double, double>(lgN, a, s, nullptr, 1);
  if (prec == 3) return dispatch_solve1d<float, double>(lgN, a, s, nullptr, 1);
  return dispatch_solve1d<float, float>(lgN, a, s, nullptr, 1);
}

hipError_t launch_solve1d_batch(int prec, int lgN, const Solve1DArgs *args, int count, int64_t nsteps,
                                hipStream_t s) {
  if (count <= 0) return hipErrorInvalidValue;
  Solve1DArgs unused{};
  unused.nsteps = nsteps;
  if (prec == 2) return dispatch_solve1d<double, double>(lgN, unused, s, args, count);
  if (prec == 3) return dispatch_solve1d<float, double>(lgN, unused, s, args, count);
  return dispatch_solve1d<float, float>(lgN, unused, s, args, count);
}

__global__ void step_advance_kernel(int64_t *step, int count, int64_t k) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) step[i] += k;
}

hipError_t launch_step_advance(int64_t *step, int count, int64_t k, hipStream_t s) {
  hipLaunchKernelGGL(step_advance_kernel, dim3((count + 255) / 256), dim3(256), 0, s, step, count, k);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// waveform coefficients of the potential for a run of steps
// ---------------------------------------------------------------------------
__global__ void coef_kernel(PotDev p, TimeDev T, int count, double *out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count * CO_COUNT) return;
  const int j = i / CO_COUNT, w = i % CO_COUNT;
  out[i] = wave_value(p.w[w], step_time_of(T, j, T.half));
}

hipError_t launch_coefficients(const PotDev &p, const TimeDev &T, int count, double *out, hipStream_t s) {
  const int n = count * CO_COUNT;
  return launch_kernel(coef_kernel, dim3((n + 255) / 256), dim3(256), s, p, T, count, out);
}

// Many solves at once; the step of solve i is read from step_dev[i] on the
// device, so the launch can be replayed from a graph.
__global__ void coef_batch_kernel(const PotDev *pots, const double *t0, const double *dt, const int64_t *step_dev,
                                  double half, int count, int rows, int stride, double *out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)count * rows * CO_COUNT) return;
  const int w = (int)(i % CO_COUNT);
  const int64_t jr = i / CO_COUNT;
  const int j = (int)(jr % rows);
  const int m = (int)(jr / rows);
  const double t = t0[m] + ((double)(step_dev[m] + j) + half) * dt[m];
  out[((int64_t)m * stride + j) * CO_COUNT + w] = wave_value(pots[m].w[w], t);
}

hipError_t launch_coefficients_batch(const PotDev *pots, const double *t0, const double *dt,
                                     const int64_t *step_dev, double half, int count, int rows, int stride,
                                     double *out, hipStream_t s) {
  if (rows > stride) return hipErrorInvalidValue;
  const int64_t n = (int64_t)count * rows * CO_COUNT;
  hipLaunchKernelGGL(coef_batch_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pots, t0, dt, step_dev,
                     half, count, rows, stride, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// initial state, conversions
// ---------------------------------------------------------------------------
template <class R>
__global__ void gaussian_kernel(void *out, GridDev g, const cx<double> *f0, const cx<double> *f1,
                                const cx<double> *f2, int64_t total) {
  using T = typename storage<R>::type;
  T *psi = (T *)out;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    int i0, i1, i2;
    grid_index(g, i, i0, i1, i2);
    const cx<double> f = cmul(cmul(f0[i0], f1[i1]), f2[i2]);
    store_from(psi + phys_index(g, i), f);
  }
}

static unsigned grid_blocks(int64_t total, int threads) {
  int64_t b = (total + threads - 1) / threads;
  if (b > 65536) b = 65536;
  if (b < 1) b = 1;
  return (unsigned)b;
}

hipError_t launch_gaussian(int prec, void *psi, const GridDev &g, const cx<double> *f0,
                           const cx<double> *f1, const cx<double> *f2, hipStream_t s) {
  const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
  const unsigned b = grid_blocks(total, 256);
  if (prec == 2) hipLaunchKernelGGL(gaussian_kernel<double>, dim3(b), dim3(256), 0, s, psi, g, f0, f1, f2, total);
  else hipLaunchKernelGGL(gaussian_kernel<float>, dim3(b), dim3(256), 0, s, psi, g, f0, f1, f2, total);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// observables: deterministic FP64 reductions.  Every block sums a fixed set
// of points (grid-stride order with a fixed grid), reduces in LDS by a fixed
// tree, and one final block adds the block partials in index order.
// ---------------------------------------------------------------------------
template <class R>
__global__ void __launch_bounds__(kObsThreads) obs_kernel(ObsArgs a) {
  using T = typename storage<R>::type;
  __shared__ double s_red[CO_COUNT][kObsThreads];
  __shared__ double s_coef[CO_COUNT];
  const int tid = threadIdx.x;
  if (a.with_v && tid < CO_COUNT) s_coef[tid] = wave_value(a.pot.w[tid], a.t);
  __syncthreads();
  const T *psi = (const T *)a.psi;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};

  for (int64_t i = (int64_t)blockIdx.x * kObsThreads + tid; i < a.total;
       i += (int64_t)gridDim.x * kObsThreads) {
    const T p = psi[phys_index(a.g, i)];
    const double pr = p.x, pi = p.y;
    const double w = pr * pr + pi * pi;
    int i0, i1, i2;
    grid_index(a.g, i, i0, i1, i2);
    if (a.kinetic && a.split_h) {
      // split 1D: point k1*n2 + k2 holds bin k1 + n1*k2
      const int lg2 = a.g.lg[0] - a.split_h;
      const int64_t m = (i >> lg2) + ((i & (((int64_t)1 << lg2) - 1)) << a.split_h);
      acc[0] += a.k2tab[0][m] * w;
    } else if (a.kinetic) {
      acc[0] += (a.k2tab[0][i0] + a.k2tab[1][i1] + a.k2tab[2][i2]) * w;
    } else {
      const double x0 = a.g.lo[0] + (double)i0 * a.g.dx[0];
      const double x1 = a.g.lo[1] + (double)i1 * a.g.dx[1];
      const double x2 = a.g.lo[2] + (double)i2 * a.g.dx[2];
      acc[0] += w;
      acc[1] += x0 * w;
      acc[2] += x1 * w;
      acc[3] += x2 * w;
      acc[4] += x0 * x0 * w;
      acc[5] += x1 * x1 * w;
      acc[6] += x2 * x2 * w;
      if (a.with_v) {
        const double xs[3] = {x0, x1, x2};
        double v = s_coef[CO_C];
        for (int d = 0; d < a.g.ndim; ++d) v += s_coef[CO_A + d] * xs[d] + s_coef[CO_B + d] * xs[d] * xs[d];
        if (a.pot.v0_kind != 0) v += s_coef[CO_S] * v0_value(a.pot, x0, x1, x2, a.g.ndim);
        acc[7] += v * w;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) s_red[k][tid] = acc[k];
  __syncthreads();
  for (int h = kObsThreads / 2; h > 0; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int k = 0; k < 8; ++k) s_red[k][tid] += s_red[k][tid + h];
    }
    __syncthreads();
  }
  if (tid < 8) a.partials[(int64_t)blockIdx.x * 8 + tid] = s_red[tid][0];
}

__global__ void __launch_bounds__(kObsThreads) obs_final_kernel(const double *partials, int blocks, double *out) {
  __shared__ double s_red[8][kObsThreads];
  const int tid = threadIdx.x;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = tid; b < blocks; b += kObsThreads)
    for (int k = 0; k < 8; ++k) acc[k] += partials[(int64_t)b * 8 + k];
  for (int k = 0; k < 8; ++k) s_red[k][tid] = acc[k];
  __syncthreads();
  for (int h = kObsThreads / 2; h > 0; h >>= 1) {
    if (tid < h)
      for (int k = 0; k < 8; ++k) s_red[k][tid] += s_red[k][tid + h];
    __syncthreads();
  }
  if (tid < 8) out[tid] = s_red[tid][0];
}

// <phi|psi>: per-block FP64 partials of conj(phi) psi in the first two of
// eight slots (the layout obs_final_kernel reduces), same fixed order.
template <class RP, class RS>
__global__ void __launch_bounds__(kObsThreads)
    inner_kernel(const void *phi_, const void *psi_, int64_t total, int lg_plane, int phi_pad, int psi_pad,
                 double *partials) {
  using TP = typename storage<RP>::type;
  using TS = typename storage<RS>::type;
  __shared__ double s_red[2][kObsThreads];
  const TP *phi = (const TP *)phi_;
  const TS *psi = (const TS *)psi_;
  const int tid = threadIdx.x;
  double re = 0.0, im = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kObsThreads + tid; i < total; i += (int64_t)gridDim.x * kObsThreads) {
    const int64_t plane = i >> lg_plane;
    const TP a = phi[i + plane * phi_pad];
    const TS b = psi[i + plane * psi_pad];
    const double ar = a.x, ai = a.y, br = b.x, bi = b.y;
    re += ar * br + ai * bi;
    im += ar * bi - ai * br;
  }
  s_red[0][tid] = re;
  s_red[1][tid] = im;
  __syncthreads();
  for (int h = kObsThreads / 2; h > 0; h >>= 1) {
    if (tid < h) {
      s_red[0][tid] += s_red[0][tid + h];
      s_red[1][tid] += s_red[1][tid + h];
    }
    __syncthreads();
  }
  if (tid < 8) partials[(int64_t)blockIdx.x * 8 + tid] = tid < 2 ? s_red[tid][0] : 0.0;
}

hipError_t launch_inner(int phi_prec, const void *phi, int psi_prec, const void *psi, int64_t total, int lg_plane,
                        int phi_pad, int psi_pad, int blocks, double *partials, double *out8, hipStream_t s) {
  const dim3 g(blocks), b(kObsThreads);
  if (phi_prec == 2 && psi_prec == 2)
    hipLaunchKernelGGL((inner_kernel<double, double>), g, b, 0, s, phi, psi, total, lg_plane, phi_pad, psi_pad, partials);
  else if (phi_prec == 2)
    hipLaunchKernelGGL((inner_kernel<double, float>), g, b, 0, s, phi, psi, total, lg_plane, phi_pad, psi_pad, partials);
  else if (psi_prec == 2)
    hipLaunchKernelGGL((inner_kernel<float, double>), g, b, 0, s, phi, psi, total, lg_plane, phi_pad, psi_pad, partials);
  else
    hipLaunchKernelGGL((inner_kernel<float, float>), g, b, 0, s, phi, psi, total, lg_plane, phi_pad, psi_pad, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(obs_final_kernel, dim3(1), dim3(kObsThreads), 0, s, (const double *)partials, blocks, out8);
  return hipGetLastError();
}

hipError_t launch_reduce8(const double *partials, int blocks, double *out8, hipStream_t s) {
  hipLaunchKernelGGL(obs_final_kernel, dim3(1), dim3(kObsThreads), 0, s, partials, blocks, out8);
  return hipGetLastError();
}

hipError_t launch_observables(int prec, const ObsArgs &a, int blocks, double *out8, hipStream_t s) {
  if (prec == 2) hipLaunchKernelGGL(obs_kernel<double>, dim3(blocks), dim3(kObsThreads), 0, s, a);
  else hipLaunchKernelGGL(obs_kernel<float>, dim3(blocks), dim3(kObsThreads), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(obs_final_kernel, dim3(1), dim3(kObsThreads), 0, s, (const double *)a.partials, blocks, out8);
  return hipGetLastError();
}

}  // namespace wp
