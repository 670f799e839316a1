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
// stores the lines back.  All arithmetic is FP64; the line passes keep the
// values between stages in LDS as FP32 for an FP32 state (one rounding per
// stage, as the power-of-two FP32 passes round every addition) and as FP64
// otherwise.
//
// Line passes: the tile (T lines, a power of two chosen on the host so that
// two workgroups fit in a CU's LDS) sits in LDS point-major, element
// (j, line tau) at j (T + 1) + tau, so that neighbouring lanes take
// neighbouring lines when loading a strided axis and neighbouring points
// when loading the contiguous one; the storage offset of each line and its
// phase or kinetic constants (the terms of the other axes) are computed once
// per tile.
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

// ---- line passes -----------------------------------------------------------
constexpr int kLThreads = 512;
// Points of a tile per thread at most (the host caps T N at this times
// kLThreads).
constexpr int kLMaxPer = 16;

// Tile of a line pass: T lines (T = 2^lgT), TP = T + 1 (T > 1) entries per
// point in LDS.
struct LTile {
  int32_t T, lgT, TP;
};

// q = x / d and r = x mod d for 0 <= x, d < 2^16, from an FP32 estimate
// corrected by one step (inv = 1/d rounded to FP32).
__device__ __forceinline__ int divmod16(int x, int d, float inv, int &r) {
  int q = (int)((float)x * inv);
  r = x - q * d;
  if (r < 0) {
    --q;
    r += d;
  } else if (r >= d) {
    ++q;
    r -= d;
  }
  return q;
}

// One stage of radix R of the tile's transform, from buffer `a` into `b`.
template <bool INV, int R, class E>
__device__ __forceinline__ void lstage(const E *a, E *b, int N, int LS, const cx<double> *tws, const LTile &t) {
  const int nb = N / R;
  const float inv_ls = 1.0f / (float)LS;
  for (int e = threadIdx.x; e < (nb << t.lgT); e += kLThreads) {
    const int tau = e & (t.T - 1), jb = e >> t.lgT;
    int k;
    (void)divmod16(jb, LS, inv_ls, k);
    cx<double> x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const E *p = a + 2 * ((jb + r * nb) * t.TP + tau);
      x[r] = {(double)p[0], (double)p[1]};
    }
    if (LS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        cx<double> w = tws[(r - 1) * LS + k];
        if (INV) w.y = -w.y;
        x[r] = cmul(x[r], w);
      }
    }
    if constexpr (R == 3 || R == 5 || R == 7) dft_odd<R, INV>(x);
    else dft<R, INV>(x);
    const int o0 = (jb - k) * R + k;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      E *p = b + 2 * ((o0 + q * LS) * t.TP + tau);
      p[0] = (E)x[q].x;
      p[1] = (E)x[q].y;
    }
  }
}

// One transform of the tile, stage by stage from buffer `a` into `b` and
// back; returns the buffer holding the result.  Every thread calls it.
template <bool INV, class E>
__device__ E *lfft(E *a, E *b, int N, const LTile &t, const GPlan &plan, const cx<double> *tw) {
  for (int s = 0; s < plan.nst; ++s) {
    const int R = plan.radix[s], LS = plan.ls[s];
    const cx<double> *tws = tw + plan.twoff[s];
    switch (R) {
      case 2: lstage<INV, 2>(a, b, N, LS, tws, t); break;
      case 3: lstage<INV, 3>(a, b, N, LS, tws, t); break;
      case 4: lstage<INV, 4>(a, b, N, LS, tws, t); break;
      case 5: lstage<INV, 5>(a, b, N, LS, tws, t); break;
      case 7: lstage<INV, 7>(a, b, N, LS, tws, t); break;
      default: lstage<INV, 8>(a, b, N, LS, tws, t); break;
    }
    __syncthreads();
    E *tmp = a;
    a = b;
    b = tmp;
  }
  return a;
}

// Line pass of a mixed-length grid: kind PK_F (one transform), PK_K
// (transform, kinetic factor, inverse), PK_V ([inverse] potential phase
// [transform]), with the tile in dynamic LDS: two buffers of N (T + 1)
// complex E, then per line its storage offset and constants.
template <class S, class E, int KIND>
__global__ void __launch_bounds__(kLThreads) lpass_kernel(GPassArgs ga, LTile t) {
  using T = typename storage<S>::type;
  extern __shared__ __align__(16) unsigned char l_lds[];
  const PassArgs &a = ga.p;
  const int N = a.g.n[a.axis];
  const int64_t inner = ga.inner;
  const int tid = threadIdx.x;
  E *const buf0 = reinterpret_cast<E *>(l_lds), *const buf1 = buf0 + 2 * N * t.TP;
  auto other = [&](E *p) { return p == buf0 ? buf1 : buf0; };
  E *A = buf0;
  int64_t *lbase = reinterpret_cast<int64_t *>(buf1 + 2 * N * t.TP);  // T storage offsets (-1: no line)
  double *lc = reinterpret_cast<double *>(lbase + t.T);              // T x 4 constants
  const int64_t line0 = (int64_t)blockIdx.x << t.lgT;
  const uint32_t ops = a.ops;
  const int ax = a.axis;

  // Per line: storage offset of its first point, and the constants of the
  // other axes (potential: phase and r^2 terms; kinetic: factor product).
  if (tid < t.T) {
    const int64_t line = line0 + tid;
    double c0 = 0.0, c1 = 0.0, c2 = 1.0, c3 = 0.0;
    if (line < a.n_lines) {
      const int64_t o = line / inner, c = line - o * inner;
      lbase[tid] = o * (int64_t)N * inner + c;
      int idx[3] = {0, 0, 0};
      int64_t cc = c, oo = o;
#pragma unroll
      for (int d = 2; d >= 0; --d) {
        if (d > ax) {
          idx[d] = (int)(cc % a.g.n[d]);
          cc /= a.g.n[d];
        }
      }
#pragma unroll
      for (int d = 2; d >= 0; --d) {
        if (d < ax) {
          idx[d] = (int)(oo % a.g.n[d]);
          oo /= a.g.n[d];
        }
      }
      if (KIND == PK_V) {
        const double *cf = a.coef;
        double th = cf[CO_C], rho2 = 0.0;
        for (int d = 0; d < a.g.ndim; ++d) {
          if (d == ax) continue;
          const double x = a.g.lo[d] + (double)idx[d] * a.g.dx[d];
          th += cf[CO_A + d] * x + cf[CO_B + d] * x * x;
          rho2 += x * x;
        }
        c0 = th * a.vtau;
        c1 = rho2;
      } else if (KIND == PK_K) {
        cx<double> f = {1.0, 0.0};
        for (int d = 0; d < a.g.ndim; ++d)
          if (d != ax) f = cmul(f, a.ktab[d][idx[d]]);
        c2 = f.x;
        c3 = f.y;
      }
    } else {
      lbase[tid] = -1;
    }
    lc[4 * tid + 0] = c0;
    lc[4 * tid + 1] = c1;
    lc[4 * tid + 2] = c2;
    lc[4 * tid + 3] = c3;
  }
  __syncthreads();

  // Load: element e of the tile (e < N T, at most kLMaxPer per thread) is
  // point e >> lgT of line e & (T-1) on strided axes (neighbouring lanes on
  // neighbouring lines: one row segment per T lanes), and point e mod N of
  // line e / N on the contiguous axis.  Every load of a thread is issued
  // before the first is waited for.
  T *psi = (T *)a.psi;
  const int total = N << t.lgT;
  const float inv_n = 1.0f / (float)N;
  auto point = [&](int e, int &tau, int &j) {
    if (inner > 1) {
      tau = e & (t.T - 1);
      j = e >> t.lgT;
    } else {
      tau = divmod16(e, N, inv_n, j);
    }
  };
  {
    cx<double> v[kLMaxPer];
#pragma unroll
    for (int i = 0; i < kLMaxPer; ++i) {
      const int e = tid + i * kLThreads;
      v[i] = {0.0, 0.0};
      if (e < total) {
        int tau, j;
        point(e, tau, j);
        const int64_t b = lbase[tau];
        if (b >= 0) v[i] = load_as<double>(psi + b + (int64_t)j * inner);
      }
    }
#pragma unroll
    for (int i = 0; i < kLMaxPer; ++i) {
      const int e = tid + i * kLThreads;
      if (e < total) {
        int tau, j;
        point(e, tau, j);
        E *p = A + 2 * (j * t.TP + tau);
        p[0] = (E)v[i].x;
        p[1] = (E)v[i].y;
      }
    }
  }
  __syncthreads();

  if constexpr (KIND == PK_F) {
    A = (ops & OP_PRE_INV) ? lfft<true>(A, other(A), N, t, ga.plan, a.tw)
                           : lfft<false>(A, other(A), N, t, ga.plan, a.tw);
  } else if constexpr (KIND == PK_K) {
    A = lfft<false>(A, other(A), N, t, ga.plan, a.tw);
    const cx<double> *kt = a.ktab[ax];
    for (int e = tid; e < (N << t.lgT); e += kLThreads) {
      const int tau = e & (t.T - 1), j = e >> t.lgT;
      const cx<double> f = cmul(kt[j], cx<double>{lc[4 * tau + 2], lc[4 * tau + 3]});
      E *p = A + 2 * (j * t.TP + tau);
      const cx<double> v = cmul(cx<double>{(double)p[0], (double)p[1]}, f);
      p[0] = (E)v.x;
      p[1] = (E)v.y;
    }
    __syncthreads();
    A = lfft<true>(A, other(A), N, t, ga.plan, a.tw);
  } else {
    if (ops & OP_PRE_INV) A = lfft<true>(A, other(A), N, t, ga.plan, a.tw);
    if (ops & OP_V) {
      const double *cf = a.coef;
      const double vt = a.vtau;
      const double ca = vt * cf[CO_A + ax], cb = vt * cf[CO_B + ax], cs = vt * cf[CO_S];
      const int vk = a.pot.v0_kind;
      const double p0 = a.pot.v0_par[0], p1 = a.pot.v0_par[1], p2 = a.pot.v0_par[2];
      const double lo = a.g.lo[ax], dx = a.g.dx[ax];
      for (int e = tid; e < (N << t.lgT); e += kLThreads) {
        const int tau = e & (t.T - 1), j = e >> t.lgT;
        const double x = lo + (double)j * dx;
        double th = lc[4 * tau + 0] + x * fma(cb, x, ca);
        if (vk == 1) {
          th -= cs * p0 * rsqrt_fast(fma(x, x, lc[4 * tau + 1] + p1));
        } else if (vk == 2) {
          const double m = 1.0 - exp(-p1 * (x - p2));
          th += cs * p0 * m * m;
        }
        E *p = A + 2 * (j * t.TP + tau);
        const cx<double> v = cmul(cx<double>{(double)p[0], (double)p[1]}, expmi_wave(th));
        p[0] = (E)v.x;
        p[1] = (E)v.y;
      }
      __syncthreads();
    }
    if (ops & OP_FWD) A = lfft<false>(A, other(A), N, t, ga.plan, a.tw);
  }

#pragma unroll
  for (int i = 0; i < kLMaxPer; ++i) {
    const int e = tid + i * kLThreads;
    if (e < total) {
      int tau, j;
      point(e, tau, j);
      const int64_t b = lbase[tau];
      const E *p = A + 2 * (j * t.TP + tau);
      if (b >= 0) store_from(psi + b + (int64_t)j * inner, cx<double>{(double)p[0], (double)p[1]});
    }
  }
}

// LDS bytes of a tile of T lines of N points.
__host__ inline size_t ltile_bytes(int N, int T, int esize) {
  const int TP = T > 1 ? T + 1 : 1;
  return (size_t)2 * N * TP * 2 * esize + (size_t)T * (8 + 32);
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
  const uint32_t ops = ga.p.ops;
  const int kind = (ops & OP_V) ? PK_V : (ops & OP_K) ? PK_K : PK_F;
  // LDS element: FP32 for an FP32 state with FP32 arithmetic (prec 1), FP64
  // for the FP64 state (2) and for the FP32 state with FP64 arithmetic (3).
  const int esize = prec == 1 ? 4 : 8;
  // Lines per tile: up to 16 (FP32 storage) or 8 (FP64) neighbouring lines,
  // so that a strided row segment is up to 128 bytes; no more than LDS for
  // two workgroups per CU allows (one for the longest lines).
  int T = prec == 2 ? 8 : 16;
  while (T > 1 && (ltile_bytes(N, T, esize) > 80 * 1024 || T > ga.p.n_lines || N * T > kLMaxPer * kLThreads)) T >>= 1;
  const size_t shm = ltile_bytes(N, T, esize);
  if (shm > 160 * 1024) return hipErrorInvalidValue;
  LTile t{T, __builtin_ctz((unsigned)T), T > 1 ? T + 1 : 1};
  const int64_t blocks = (ga.p.n_lines + T - 1) / T;
  if (blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  const dim3 g((unsigned)blocks), b(kLThreads);
  auto go = [&](auto kernel) -> hipError_t {
    // Dynamic LDS beyond the default limit needs the attribute once per kernel.
    static bool ready = false;
    if (!ready) {
      hipError_t e = hipFuncSetAttribute((const void *)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         160 * 1024);
      if (e != hipSuccess) return e;
      ready = true;
    }
    return launch_kernel_shm(kernel, g, b, shm, s, ga, t);
  };
  if (prec == 2) {
    if (kind == PK_V) return go(lpass_kernel<double, double, PK_V>);
    if (kind == PK_K) return go(lpass_kernel<double, double, PK_K>);
    return go(lpass_kernel<double, double, PK_F>);
  }
  if (prec == 3) {
    if (kind == PK_V) return go(lpass_kernel<float, double, PK_V>);
    if (kind == PK_K) return go(lpass_kernel<float, double, PK_K>);
    return go(lpass_kernel<float, double, PK_F>);
  }
  if (kind == PK_V) return go(lpass_kernel<float, float, PK_V>);
  if (kind == PK_K) return go(lpass_kernel<float, float, PK_K>);
  return go(lpass_kernel<float, float, PK_F>);
}

hipError_t launch_gsolve1d(int prec, const Solve1DArgs &a, const GPlan &plan, hipStream_t s) {
  if (a.g.n[0] < 2 || a.g.n[0] > kMaxMixed || plan.nst < 1 || plan.nst > kMaxStages) return hipErrorInvalidValue;
  if (prec == 2) return launch_kernel(gsolve1d_kernel<double>, dim3(1), dim3(kGThreads), s, a, plan);
  return launch_kernel(gsolve1d_kernel<float>, dim3(1), dim3(kGThreads), s, a, plan);
}

}  // namespace wp
