// wp_gpass.hip -- line passes and the 1D solver for axis lengths whose prime
// factors are 2, 3, 5 and 7 (the lengths advised for the transforms in
// Section 3.2.1, struct `parameters`, nx/ny/nz), up to 4096 points.
//
// A workgroup loads a tile of lines into LDS, transforms them stage by stage
// (Stockham autosort with radices 8, 4, 2, 3, 5, 7: butterfly j of a stage of
// radix R reads inputs j + r N/R, multiplies input r by
// exp(-+2 pi i r (j mod LS)/(R LS)), does an R-point DFT and writes output q
// to (j - j mod LS) R + (j mod LS) + q LS, alternating between two LDS
// buffers), applies the same phase factors as the power-of-two passes, and
// stores the lines back.  All arithmetic is FP64 whatever the storage type.
// Grid indices come from divisions by the runtime lengths.
#include "wp_pass.hpp"

namespace wp {

namespace {

// cos and sin of 2 pi m/R for m = 1..(R-1)/2.
__device__ __forceinline__ double root_cos(int R, int m) {
  if (R == 3) return -0.5;
  if (R == 5) return m == 1 ? 0.3090169943749474241023 : -0.8090169943749474241023;
  return m == 1 ? 0.623489801858733530525 : m == 2 ? -0.2225209339563144042889 : -0.9009688679024191262361;
}
__device__ __forceinline__ double root_sin(int R, int m) {
  if (R == 3) return 0.8660254037844386467637;
  if (R == 5) return m == 1 ? 0.9510565162951535721164 : 0.5877852522924731291687;
  return m == 1 ? 0.7818314824680298087084 : m == 2 ? 0.9749279121818236070181 : 0.4338837391175581204758;
}

// Odd prime R: mirrored inputs j and R - j are combined first; output q is
// t + s and output R - q is t - s, with t the cosine sum and s = (-+ i) times
// the sine sum.
template <int R, bool INV>
__device__ __forceinline__ void dft_odd(cx<double> *x) {
  constexpr int H = (R - 1) / 2;
  cx<double> a[H], b[H];
  cx<double> sum = x[0];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    a[j - 1] = cadd(x[j], x[R - j]);
    b[j - 1] = csub(x[j], x[R - j]);
    sum = cadd(sum, a[j - 1]);
  }
  cx<double> out[R];
  out[0] = sum;
#pragma unroll
  for (int q = 1; q <= H; ++q) {
    cx<double> t = x[0], u = {0.0, 0.0};
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const int m = (j * q) % R;
      const int mm = m <= H ? m : R - m;
      const double c = root_cos(R, mm), s = m <= H ? root_sin(R, mm) : -root_sin(R, mm);
      t = {t.x + a[j - 1].x * c, t.y + a[j - 1].y * c};
      u = {u.x + b[j - 1].x * s, u.y + b[j - 1].y * s};
    }
    const cx<double> iu = mul_mi<INV>(u);
    out[q] = cadd(t, iu);
    out[R - q] = csub(t, iu);
  }
#pragma unroll
  for (int q = 0; q < R; ++q) x[q] = out[q];
}

template <bool INV>
__device__ __forceinline__ void dft_any(cx<double> *x, int R) {
  switch (R) {
    case 2: dft2<INV>(x[0], x[1]); break;
    case 3: dft_odd<3, INV>(x); break;
    case 4: dft4<INV>(x[0], x[1], x[2], x[3]); break;
    case 5: dft_odd<5, INV>(x); break;
    case 7: dft_odd<7, INV>(x); break;
    default: dft8<INV>(x); break;
  }
}

constexpr int kGThreads = 256;
// LDS of one workgroup: two buffers of kMaxMixed FP64 complex values.
constexpr int kGBuf = kMaxMixed;

// Transform the `tile` lines of length N held in `a` (line tau at a + tau N)
// with the stages of `plan`; `b` is the other buffer.  Returns the buffer
// holding the result.  Every thread of the workgroup calls it.
template <bool INV>
__device__ cx<double> *gfft(cx<double> *a, cx<double> *b, int N, int tile, const GPlan &plan,
                           const cx<double> *tw) {
  for (int s = 0; s < plan.nst; ++s) {
    const int R = plan.radix[s], LS = plan.ls[s];
    const int nb = N / R;
    const cx<double> *tws = tw + plan.twoff[s];
    for (int e = threadIdx.x; e < tile * nb; e += kGThreads) {
      const int tau = e / nb, j = e - tau * nb;
      const int k = j % LS;
      const cx<double> *in = a + tau * N;
      cx<double> x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r)
        if (r < R) x[r] = in[j + r * nb];
      if (LS > 1) {
#pragma unroll
        for (int r = 1; r < 8; ++r) {
          if (r < R) {
            cx<double> w = tws[(r - 1) * LS + k];
            if (INV) w.y = -w.y;
            x[r] = cmul(x[r], w);
          }
        }
      }
      dft_any<INV>(x, R);
      cx<double> *out = b + tau * N + (j - k) * R + k;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < R) out[q * LS] = x[q];
    }
    __syncthreads();
    cx<double> *t = a;
    a = b;
    b = t;
  }
  return a;
}

// Multi-index of element j of line `line` along `axis`.
__device__ __forceinline__ void line_point(const GridDev &g, int axis, int64_t inner, int64_t line, int j,
                                           int idx[3]) {
  int64_t c = line % inner, o = line / inner;
#pragma unroll
  for (int d = 2; d >= 0; --d) {
    if (d > axis) {
      idx[d] = (int)(c % g.n[d]);
      c /= g.n[d];
    }
  }
#pragma unroll
  for (int d = 2; d >= 0; --d) {
    if (d < axis) {
      idx[d] = (int)(o % g.n[d]);
      o /= g.n[d];
    }
  }
  idx[axis] = j;
}

// Phase of the potential at a grid point: vtau * V(x, t), V from the
// waveform values `cf` (the same form as the power-of-two passes).
__device__ __forceinline__ double potential_phase(const PassArgs &a, const double *cf, const int idx[3]) {
  double xs[3] = {0.0, 0.0, 0.0};
  double v = cf[CO_C];
  for (int d = 0; d < a.g.ndim; ++d) {
    xs[d] = a.g.lo[d] + (double)idx[d] * a.g.dx[d];
    v += cf[CO_A + d] * xs[d] + cf[CO_B + d] * xs[d] * xs[d];
  }
  if (a.pot.v0_kind != 0) v += cf[CO_S] * v0_value(a.pot, xs[0], xs[1], xs[2], a.g.ndim);
  return a.vtau * v;
}

template <class S>
__device__ __forceinline__ void gpass_body(const GPassArgs &ga, int kind) {
  using T = typename storage<S>::type;
  __shared__ cx<double> s_buf[2 * kGBuf];
  const PassArgs &a = ga.p;
  const int N = a.g.n[a.axis];
  const int tile = kGBuf / N < 16 ? kGBuf / N : 16;
  const int64_t inner = ga.inner;
  const bool strided = inner > 1;
  const int64_t line0 = (int64_t)blockIdx.x * tile;
  T *psi = (T *)a.psi;
  const uint32_t ops = a.ops;
  auto addr = [&](int64_t line, int j) -> int64_t {
    return (line / inner) * N * inner + line % inner + (int64_t)j * inner;
  };
  // Strided lines: consecutive threads take neighbouring lines (contiguous in
  // memory); contiguous lines: consecutive points of one line.
  auto which = [&](int e, int &tau, int &j) {
    if (strided) {
      tau = e % tile;
      j = e / tile;
    } else {
      tau = e / N;
      j = e - tau * N;
    }
  };
  cx<double> *A = s_buf;
  for (int e = threadIdx.x; e < tile * N; e += kGThreads) {
    int tau, j;
    which(e, tau, j);
    const int64_t line = line0 + tau;
    A[tau * N + j] = line < a.n_lines ? load_as<double>(psi + addr(line, j)) : cx<double>{0.0, 0.0};
  }
  __syncthreads();
  auto other = [&](cx<double> *p) { return p == s_buf ? s_buf + kGBuf : s_buf; };
  if (kind == PK_F) {
    A = (ops & OP_PRE_INV) ? gfft<true>(A, other(A), N, tile, ga.plan, a.tw)
                           : gfft<false>(A, other(A), N, tile, ga.plan, a.tw);
  } else if (kind == PK_K) {
    A = gfft<false>(A, other(A), N, tile, ga.plan, a.tw);
    for (int e = threadIdx.x; e < tile * N; e += kGThreads) {
      int tau, j;
      which(e, tau, j);
      const int64_t line = line0 + tau;
      if (line >= a.n_lines) continue;
      int idx[3];
      line_point(a.g, a.axis, inner, line, j, idx);
      cx<double> f = {1.0, 0.0};
      for (int d = 0; d < a.g.ndim; ++d) f = cmul(f, a.ktab[d][idx[d]]);
      A[tau * N + j] = cmul(A[tau * N + j], f);
    }
    __syncthreads();
    A = gfft<true>(A, other(A), N, tile, ga.plan, a.tw);
  } else {
    if (ops & OP_PRE_INV) A = gfft<true>(A, other(A), N, tile, ga.plan, a.tw);
    if (ops & OP_V) {
      for (int e = threadIdx.x; e < tile * N; e += kGThreads) {
        int tau, j;
        which(e, tau, j);
        const int64_t line = line0 + tau;
        if (line >= a.n_lines) continue;
        int idx[3];
        line_point(a.g, a.axis, inner, line, j, idx);
        A[tau * N + j] = cmul(A[tau * N + j], expmi_wave(potential_phase(a, a.coef, idx)));
      }
      __syncthreads();
    }
    if (ops & OP_FWD) A = gfft<false>(A, other(A), N, tile, ga.plan, a.tw);
  }
  for (int e = threadIdx.x; e < tile * N; e += kGThreads) {
    int tau, j;
    which(e, tau, j);
    const int64_t line = line0 + tau;
    if (line < a.n_lines) store_from(psi + addr(line, j), A[tau * N + j]);
  }
}

template <class S, int KIND>
__global__ void __launch_bounds__(kGThreads) gpass_kernel(GPassArgs ga) {
  gpass_body<S>(ga, KIND);
}

// The whole 1D solve in one workgroup, as the power-of-two solver: merged
// potential halves (V-K-V) or merged kinetic halves (K-V-K).
template <class S>
__global__ void __launch_bounds__(kGThreads) gsolve1d_kernel(Solve1DArgs a, GPlan plan) {
  using T = typename storage<S>::type;
  __shared__ cx<double> s_buf[2 * kGBuf];
  __shared__ double s_coef[CO_COUNT];
  const int N = a.g.n[0];
  T *psi = (T *)a.psi;
  cx<double> *A = s_buf;
  auto other = [&](cx<double> *p) { return p == s_buf ? s_buf + kGBuf : s_buf; };
  for (int j = threadIdx.x; j < N; j += kGThreads) A[j] = load_as<double>(psi + j);
  __syncthreads();
  auto apply_v = [&](double time, double vtau) {
    for (int k = threadIdx.x; k < CO_COUNT; k += kGThreads) s_coef[k] = wave_value(a.pot.w[k], time);
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += kGThreads) {
      const double x = a.g.lo[0] + (double)j * a.g.dx[0];
      double th = s_coef[CO_C] + (s_coef[CO_A] * x + s_coef[CO_B] * x * x);
      if (a.pot.v0_kind != 0) th += s_coef[CO_S] * v0_value(a.pot, x, 0.0, 0.0, 1);
      A[j] = cmul(A[j], expmi_wave(vtau * th));
    }
    __syncthreads();
  };
  auto apply_k = [&](const cx<double> *kt) {
    for (int j = threadIdx.x; j < N; j += kGThreads) A[j] = cmul(A[j], kt[j]);
    __syncthreads();
  };
  const int64_t ns = a.nsteps;
  if (a.order == 0) {
    for (int64_t s = 0; s < ns; ++s) {
      if (s == 0) apply_v(step_time_of(a.time, 0, 0.0), a.vtau_half);
      A = gfft<false>(A, other(A), N, 1, plan, a.tw);
      apply_k(a.kfull);
      A = gfft<true>(A, other(A), N, 1, plan, a.tw);
      apply_v(step_time_of(a.time, s + 1, 0.0), s + 1 == ns ? a.vtau_half : a.vtau_full);
    }
  } else if (ns > 0) {
    A = gfft<false>(A, other(A), N, 1, plan, a.tw);
    apply_k(a.khalf);
    for (int64_t s = 0; s < ns; ++s) {
      A = gfft<true>(A, other(A), N, 1, plan, a.tw);
      apply_v(step_time_of(a.time, s, 0.5), a.vtau_full);
      A = gfft<false>(A, other(A), N, 1, plan, a.tw);
      apply_k(s + 1 == ns ? a.khalf : a.kfull);
    }
    A = gfft<true>(A, other(A), N, 1, plan, a.tw);
  }
  for (int j = threadIdx.x; j < N; j += kGThreads) store_from(psi + j, A[j]);
}

}  // namespace

hipError_t launch_gpass(int prec, const GPassArgs &ga, hipStream_t s) {
  const int N = ga.p.g.n[ga.p.axis];
  if (N < 2 || N > kMaxMixed || ga.plan.nst < 1 || ga.plan.nst > kMaxStages) return hipErrorInvalidValue;
  const int tile = kGBuf / N < 16 ? kGBuf / N : 16;
  const int64_t blocks = (ga.p.n_lines + tile - 1) / tile;
  if (blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const uint32_t ops = ga.p.ops;
  const int kind = (ops & OP_V) ? PK_V : (ops & OP_K) ? PK_K : PK_F;
  const dim3 g((unsigned)blocks), b(kGThreads);
  if (prec == 2) {
    if (kind == PK_V) return launch_kernel(gpass_kernel<double, PK_V>, g, b, s, ga);
    if (kind == PK_K) return launch_kernel(gpass_kernel<double, PK_K>, g, b, s, ga);
    return launch_kernel(gpass_kernel<double, PK_F>, g, b, s, ga);
  }
  if (kind == PK_V) return launch_kernel(gpass_kernel<float, PK_V>, g, b, s, ga);
  if (kind == PK_K) return launch_kernel(gpass_kernel<float, PK_K>, g, b, s, ga);
  return launch_kernel(gpass_kernel<float, PK_F>, g, b, s, ga);
}

hipError_t launch_gsolve1d(int prec, const Solve1DArgs &a, const GPlan &plan, hipStream_t s) {
  if (a.g.n[0] < 2 || a.g.n[0] > kMaxMixed || plan.nst < 1 || plan.nst > kMaxStages) return hipErrorInvalidValue;
  if (prec == 2) return launch_kernel(gsolve1d_kernel<double>, dim3(1), dim3(kGThreads), s, a, plan);
  return launch_kernel(gsolve1d_kernel<float>, dim3(1), dim3(kGThreads), s, a, plan);
}

}  // namespace wp
