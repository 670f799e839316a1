// wp_device.hpp -- device building blocks of the split-operator step on gfx950:
// complex arithmetic with FP64-accurate factor multiplies, the time-dependent
// potential family, and the LDS-staged line FFT.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace wp {

// ---------------------------------------------------------------------------
// complex values
// ---------------------------------------------------------------------------
template <class R>
struct cx {
  R x, y;
};

template <class R>
__device__ __forceinline__ cx<R> cadd(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R>
__device__ __forceinline__ cx<R> csub(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }

// Product of two FP64 factors.
__device__ __forceinline__ cx<double> cmul(cx<double> a, cx<double> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// Multiply a value by an FP64 factor and round the result once into the
// value's precision.  Rounding a phase or twiddle factor to FP32 first would
// bias |psi| by the same relative amount at every step; here the only
// rounding is that of the product.
__device__ __forceinline__ cx<double> mul_acc(cx<double> a, cx<double> w) { return cmul(a, w); }
__device__ __forceinline__ cx<float> mul_acc(cx<float> a, cx<double> w) {
  double ax = a.x, ay = a.y;
  return {(float)(ax * w.x - ay * w.y), (float)(ax * w.y + ay * w.x)};
}

// Multiply by -i (forward transform) or +i (inverse transform).
template <bool INV, class R>
__device__ __forceinline__ cx<R> mul_mi(cx<R> a) {
  return INV ? cx<R>{-a.y, a.x} : cx<R>{a.y, -a.x};
}

// s * sqrt(1/2) with one rounding: in FP32 the constant is carried as a
// two-term sum so that no rounded constant is applied at every transform.
__device__ __forceinline__ double mul_rsqrt2(double s) { return s * 0.70710678118654752440; }
__device__ __forceinline__ float mul_rsqrt2(float s) {
  constexpr float hi = 0.70710678118654752440f;
  constexpr float lo = (float)(0.70710678118654752440 - (double)hi);
  return fmaf(s, hi, s * lo);
}

// Multiply by exp(-+ 2 pi i/8) and exp(-+ 6 pi i/8) (the radix-8 inner
// twiddles; upper sign forward).
template <bool INV, class R>
__device__ __forceinline__ cx<R> mul_w8_1(cx<R> a) {
  // forward: (1 - i)/sqrt2 ; inverse: (1 + i)/sqrt2
  return INV ? cx<R>{mul_rsqrt2(a.x - a.y), mul_rsqrt2(a.x + a.y)}
             : cx<R>{mul_rsqrt2(a.x + a.y), mul_rsqrt2(a.y - a.x)};
}
template <bool INV, class R>
__device__ __forceinline__ cx<R> mul_w8_3(cx<R> a) {
  // forward: (-1 - i)/sqrt2 ; inverse: (-1 + i)/sqrt2
  return INV ? cx<R>{mul_rsqrt2(-a.x - a.y), mul_rsqrt2(a.x - a.y)}
             : cx<R>{mul_rsqrt2(a.y - a.x), mul_rsqrt2(-a.x - a.y)};
}

// Small DFTs in registers (unnormalised; INV selects exp(+2 pi i jm/n)).
template <bool INV, class R>
__device__ __forceinline__ void dft2(cx<R> &a, cx<R> &b) {
  cx<R> s = cadd(a, b), d = csub(a, b);
  a = s;
  b = d;
}

template <bool INV, class R>
__device__ __forceinline__ void dft4(cx<R> &u0, cx<R> &u1, cx<R> &u2, cx<R> &u3) {
  cx<R> s0 = cadd(u0, u2), s1 = csub(u0, u2);
  cx<R> s2 = cadd(u1, u3), s3 = mul_mi<INV>(csub(u1, u3));
  u0 = cadd(s0, s2);
  u1 = cadd(s1, s3);
  u2 = csub(s0, s2);
  u3 = csub(s1, s3);
}

// 8-point DFT as 2 x 4: radix-2 between r and r+4, inner twiddles W8^r on
// the difference terms, then two 4-point DFTs giving the even and odd outputs.
template <bool INV, class R>
__device__ __forceinline__ void dft8(cx<R> *v) {
  cx<R> a0 = cadd(v[0], v[4]), b0 = csub(v[0], v[4]);
  cx<R> a1 = cadd(v[1], v[5]), b1 = csub(v[1], v[5]);
  cx<R> a2 = cadd(v[2], v[6]), b2 = csub(v[2], v[6]);
  cx<R> a3 = cadd(v[3], v[7]), b3 = csub(v[3], v[7]);
  b1 = mul_w8_1<INV>(b1);
  b2 = mul_mi<INV>(b2);
  b3 = mul_w8_3<INV>(b3);
  dft4<INV>(a0, a1, a2, a3);
  dft4<INV>(b0, b1, b2, b3);
  v[0] = a0; v[2] = a1; v[4] = a2; v[6] = a3;
  v[1] = b0; v[3] = b1; v[5] = b2; v[7] = b3;
}

template <int RAD, bool INV, class R>
__device__ __forceinline__ void dft(cx<R> *x) {
  if constexpr (RAD == 2) dft2<INV>(x[0], x[1]);
  else if constexpr (RAD == 4) dft4<INV>(x[0], x[1], x[2], x[3]);
  else dft8<INV>(x);
}

// ---------------------------------------------------------------------------
// line FFT: N = 2^p points of one line held by L = N/VPT threads, VPT values
// each.  Thread t holds element t + L*u in slot u ("stride-L layout") on entry
// and on exit, in natural order, for both directions.
//
// Stages follow the Stockham autosort formulation (Stockham 1966; as used for
// GPUs by Govindaraju et al., SC 2008): with Ls the product of the radices
// done so far, butterfly j takes inputs j + r N/R, multiplies input r by
// exp(-+2 pi i r (j mod Ls)/(Ls R)), does an R-point DFT and writes output q
// to (j - j mod Ls) R + (j mod Ls) + q Ls.  The first stage takes its inputs
// straight from registers and the last leaves its outputs in registers, so a
// transform of 8^s points exchanges through LDS s-1 times.  The first stage
// has radix 2, 4 or 8 so that the rest are radix 8; a thread does VPT/R
// butterflies per stage.
//
// Twiddles are stored stage by stage ("stage order"): the stage with product
// Ls > 1 owns 7*Ls entries at offset tw_offset(Ls), entry (r-1)*Ls + k being
// exp(-2 pi i r k/(8 Ls)).  Lanes that run consecutive butterflies read
// consecutive entries, which keeps the table reads free of bank conflicts.
// ---------------------------------------------------------------------------
template <int N, int VPT_ = (N < 8 ? N : 8)>
struct fft_shape {
  static constexpr int lg = __builtin_ctz(N);
  static constexpr int VPT = VPT_ < N ? VPT_ : N;
  static constexpr int L = N / VPT;
  static constexpr int R0 = (N <= 8) ? N : ((lg % 3 == 0) ? 8 : (1 << (lg % 3)));
  static_assert(VPT >= R0 || N <= 8, "a thread must hold a whole first-stage butterfly");
};

template <int N>
constexpr int tw_offset(int LS) {
  int off = 0;
  for (int l = fft_shape<N>::R0; l < LS; l *= 8) off += 7 * l;
  return off;
}
// Entries of the stage-ordered twiddle table of an N-point line.
constexpr int tw_count(int N) {
  if (N <= 8) return 1;
  int lg = __builtin_ctz(N);
  int r0 = (lg % 3 == 0) ? 8 : (1 << (lg % 3));
  int off = 0;
  for (int l = r0; l < N; l *= 8) off += 7 * l;
  return off;
}

// LDS position of element i of a line: one padding slot after every 16
// elements.  In every index pattern of the stages below, the low four bits
// never carry when a multiple of Ls (writes) or of L (reads) is added, so
// pad(a + c) = pad(a) + c + (c >> 4) for those offsets c: each thread
// computes one base per butterfly and every other position is a constant
// offset (an immediate in the LDS instruction).
__device__ __forceinline__ constexpr int pad16(int i) { return i + (i >> 4); }

// FP32 passes whose whole twiddle table sits in LDS hold it as hi + lo
// pairs: w = (re_hi + re_lo) + i (im_hi + im_lo) with re_hi = (float)re and
// re_lo = (float)(re - re_hi), so w is carried to about 2^-48, and a
// product takes one multiply and three FMAs per component, smallest terms
// first.  That is the same count of vector instructions as the FP64 route
// of mul_acc (two conversions in, four FP64 operations, two conversions
// out), but the FP32 ones issue faster: the potential pass of the 512^3
// workload went from 0.573 to 0.551 ms.  The result is rounded a few times
// in FP32 instead of once, without bias: the norm does not drift (the
// factor's modulus is 1 to about 2^-48, unlike a rounded FP32 twiddle).
struct TwHiLo {
  const float4 *lds;  // entries {re_hi, im_hi, re_lo, im_lo} in stage order
};
template <int N, int LS>
__device__ __forceinline__ const float4 *stage_tw(const TwHiLo &tw) {
  return tw.lds + tw_offset<N>(LS);
}
__device__ __forceinline__ float4 hilo_of(cx<double> w) {
  const float hr = (float)w.x, hi = (float)w.y;
  return make_float4(hr, hi, (float)(w.x - (double)hr), (float)(w.y - (double)hi));
}
// a * w (or a * conj(w) for the inverse transform).
template <bool INV>
__device__ __forceinline__ cx<float> tw_mul(cx<float> a, float4 w) {
  const float wi = INV ? -w.y : w.y, wil = INV ? -w.w : w.w;
  float re = a.x * w.z;
  re = fmaf(-a.y, wil, re);
  re = fmaf(a.x, w.x, re);
  re = fmaf(-a.y, wi, re);
  float im = a.x * wil;
  im = fmaf(a.y, w.z, im);
  im = fmaf(a.x, wi, im);
  im = fmaf(a.y, w.x, im);
  return {re, im};
}
template <bool INV, class R>
__device__ __forceinline__ cx<R> tw_mul(cx<R> a, cx<double> w) {
  if (INV) w.y = -w.y;
  return mul_acc(a, w);
}

// Twiddle table in two places: its first TWL entries copied to LDS, the
// whole table in global memory.  A stage whose entries all lie below TWL
// reads the LDS copy, the others read global memory (through the caches).
template <int TWL>
struct TwSplit {
  const cx<double> *lds, *glob;
};
// Entries of the stage with product LS (see tw_offset).
template <int N, int LS>
__device__ __forceinline__ const cx<double> *stage_tw(const cx<double> *tw) {
  return tw + tw_offset<N>(LS);
}
template <int N, int LS, int TWL>
__device__ __forceinline__ const cx<double> *stage_tw(const TwSplit<TWL> &tw) {
  return (tw_offset<N>(LS) + 7 * LS <= TWL ? tw.lds : tw.glob) + tw_offset<N>(LS);
}

template <int N, int VPT, int RAD, int LS, bool INV, class R, class TW, class Lds>
__device__ __forceinline__ void fft_stage(cx<R> (&v)[VPT], int t, const TW &tw, Lds lds) {
  constexpr int L = N / VPT;
  constexpr int M = VPT / RAD;  // butterflies per thread
  constexpr bool LAST = (LS * RAD == N);
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int j = t + m * L;
    const int k = j & (LS - 1);
    cx<R> x[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) x[r] = v[m + r * M];
    if constexpr (LS > 1) {
      const auto *tws = stage_tw<N, LS>(tw) + k;
#pragma unroll
      for (int r = 1; r < RAD; ++r) x[r] = tw_mul<INV>(x[r], tws[(r - 1) * LS]);
    }
    dft<RAD, INV>(x);
    if constexpr (LAST) {
#pragma unroll
      for (int q = 0; q < RAD; ++q) v[m + q * M] = x[q];
    } else {
      const int p0 = pad16((j - k) * RAD + k);
#pragma unroll
      for (int q = 0; q < RAD; ++q) lds(p0 + q * LS + ((q * LS) >> 4)) = x[q];
    }
  }
}

// Ordering of an LDS exchange.  WAVE: every line is held by the threads of
// one wavefront and stored in its own part of LDS, so only that wavefront
// takes part; its LDS operations are performed in program order, and the
// wavefront-scope fence keeps the compiler from moving LDS accesses across.
// Otherwise the whole workgroup meets at a barrier.
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  } else {
    __syncthreads();
  }
}

template <int N, int VPT, int RAD, int LS, bool INV, bool WAVE, class R, class TW, class Lds>
__device__ __forceinline__ void fft_stages(cx<R> (&v)[VPT], int t, const TW &tw, Lds lds) {
  constexpr int L = N / VPT;
  fft_stage<N, VPT, RAD, LS, INV>(v, t, tw, lds);
  if constexpr (LS * RAD < N) {
    lds_sync<WAVE>();
    const int pt = pad16(t);
#pragma unroll
    for (int u = 0; u < VPT; ++u) v[u] = lds(pt + L * u + ((L * u) >> 4));
    // The next stage writes LDS only if it is not the last one.
    if constexpr (LS * RAD * 8 < N) lds_sync<WAVE>();
    fft_stages<N, VPT, 8, LS * RAD, INV, WAVE>(v, t, tw, lds);
  }
}

// Whole line transform.  Every thread of the workgroup must call it (it
// contains barriers) whether or not its line is valid.  It starts with a
// barrier so that earlier LDS reads of the same buffer are complete.
// `Lds` maps a padded position (see pad16) of this thread's line to an LDS
// reference.  WAVE (see lds_sync): each line lies within one wavefront, and
// the caller has already synchronised the workgroup after any LDS it fills
// together (twiddles, tables).
template <int N, int VPT, bool INV, bool WAVE = false, class R, class TW, class Lds>
__device__ __forceinline__ void line_fft(cx<R> (&v)[VPT], int t, const TW &tw, Lds lds) {
  if constexpr (N > 8) lds_sync<WAVE>();
  fft_stages<N, VPT, fft_shape<N, VPT>::R0, 1, INV, WAVE>(v, t, tw, lds);
}

// ---------------------------------------------------------------------------
// exp(-i theta) to FP64 accuracy, for the phase factors evaluated at every
// point: theta is reduced by the nearest multiple k of pi/2 with pi/2 split
// in three parts (Cody and Waite's method; k * PIO2_A is exact for
// |k| < 2^20), then sin and cos of the remainder |r| <= pi/4 come from their
// Taylor series (terms to r^19 and r^18: truncation below 1e-17), and the
// quadrant k mod 4 permutes and negates them.  Beyond |theta| ~ 1.6e6 the
// reduction error grows like ulp(theta), the same order as the rounding
// error theta itself carries, so no slower path is needed.
// ---------------------------------------------------------------------------
constexpr double fact(int n) { return n <= 1 ? 1.0 : n * fact(n - 1); }
// Taylor coefficients 1/n!, evaluated by the compiler.
template <int n>
struct inv_fact {
  static constexpr double value = 1.0 / fact(n);
};

// |theta| <= pi/4: no reduction needed (the same series as below).
__device__ __forceinline__ cx<double> expmi_quarter(double r) {
  const double r2 = r * r;
  double ps = -inv_fact<19>::value;
  ps = fma(ps, r2, inv_fact<17>::value);
  ps = fma(ps, r2, -inv_fact<15>::value);
  ps = fma(ps, r2, inv_fact<13>::value);
  ps = fma(ps, r2, -inv_fact<11>::value);
  ps = fma(ps, r2, inv_fact<9>::value);
  ps = fma(ps, r2, -inv_fact<7>::value);
  ps = fma(ps, r2, inv_fact<5>::value);
  ps = fma(ps, r2, -inv_fact<3>::value);
  double pc = inv_fact<18>::value;
  pc = fma(pc, r2, -inv_fact<16>::value);
  pc = fma(pc, r2, inv_fact<14>::value);
  pc = fma(pc, r2, -inv_fact<12>::value);
  pc = fma(pc, r2, inv_fact<10>::value);
  pc = fma(pc, r2, -inv_fact<8>::value);
  pc = fma(pc, r2, inv_fact<6>::value);
  pc = fma(pc, r2, -inv_fact<4>::value);
  pc = fma(pc, r2, inv_fact<2>::value);
  return {fma(-pc, r2, 1.0), -fma(ps * r2, r, r)};
}

// |theta| <= 1/16: the series to r^7 and r^8 (the next terms, r^9/9! and
// r^10/10!, are below 4e-17 and 3e-19).  The terms are summed from the
// smallest up over precomputed powers of r^2, so that every coefficient is a
// multiplier (kept in scalar registers) rather than the running sum;
// measured against extended precision both this order and Horner's rule
// stay within half an ulp for the cosine.
__device__ __forceinline__ cx<double> expmi_tiny(double r) {
  const double r2 = r * r, r4 = r2 * r2, r6 = r4 * r2, r8 = r4 * r4;
  double c = inv_fact<8>::value * r8;
  c = fma(-inv_fact<6>::value, r6, c);
  c = fma(inv_fact<4>::value, r4, c);
  c = fma(-0.5, r2, c);
  double s = -inv_fact<7>::value * r6;
  s = fma(inv_fact<5>::value, r4, s);
  s = fma(-inv_fact<3>::value, r2, s);
  return {c + 1.0, -fma(s, r, r)};
}

__device__ __forceinline__ cx<double> expmi_taylor(double th) {
  constexpr double TWO_OVER_PI = 0x1.45f306dc9c883p-1;
  constexpr double PIO2_A = 0x1.921fb54400000p+0;
  constexpr double PIO2_B = 0x1.0b4611a600000p-34;
  constexpr double PIO2_C = 0x1.3198a2e037073p-69;
  const double k = rint(th * TWO_OVER_PI);
  double r = fma(-k, PIO2_A, th);
  r = fma(-k, PIO2_B, r);
  r = fma(-k, PIO2_C, r);
  const double r2 = r * r;
  double ps = -inv_fact<19>::value;
  ps = fma(ps, r2, inv_fact<17>::value);
  ps = fma(ps, r2, -inv_fact<15>::value);
  ps = fma(ps, r2, inv_fact<13>::value);
  ps = fma(ps, r2, -inv_fact<11>::value);
  ps = fma(ps, r2, inv_fact<9>::value);
  ps = fma(ps, r2, -inv_fact<7>::value);
  ps = fma(ps, r2, inv_fact<5>::value);
  ps = fma(ps, r2, -inv_fact<3>::value);
  const double sn = fma(ps * r2, r, r);
  double pc = inv_fact<18>::value;
  pc = fma(pc, r2, -inv_fact<16>::value);
  pc = fma(pc, r2, inv_fact<14>::value);
  pc = fma(pc, r2, -inv_fact<12>::value);
  pc = fma(pc, r2, inv_fact<10>::value);
  pc = fma(pc, r2, -inv_fact<8>::value);
  pc = fma(pc, r2, inv_fact<6>::value);
  pc = fma(pc, r2, -inv_fact<4>::value);
  pc = fma(pc, r2, inv_fact<2>::value);
  const double cs = fma(-pc, r2, 1.0);
  // theta = k pi/2 + r: (cos, sin)(theta) for k mod 4 = 0, 1, 2, 3 is
  // (c, s), (-s, c), (-c, -s), (s, -c).
  const int q = (int)(long long)k & 3;
  const double c1 = (q & 1) ? sn : cs;
  const double s1 = (q & 1) ? cs : sn;
  const double cosv = (q == 1 || q == 2) ? -c1 : c1;
  const double sinv = (q >= 2) ? -s1 : s1;
  return {cosv, -sinv};
}

// 1/sqrt(q) for 1e-30 < q < 1e30: the FP32 estimate refined by one FP64
// Newton step, r + r (1/2 - q r^2/2) (relative error below 1e-13).
__device__ __forceinline__ double rsqrt_newton(double q) {
  const double r = (double)__frsqrt_rn((float)q);
  return fma(r, fma(-0.5 * q * r, r, 0.5), r);
}

// 1/sqrt(q) for q > 0: rsqrt_newton, with the FP64 library call for lanes
// outside the FP32 range (taken by the whole wavefront if any lane needs it).
__device__ __forceinline__ double rsqrt_fast(double q) {
  const bool in_range = q > 1e-30 && q < 1e30;
  return __all(in_range) ? rsqrt_newton(q) : rsqrt(q);
}

// exp(-i theta) choosing, for the whole wavefront at once (the branches stay
// uniform), the cheapest of the three evaluations that is exact for every
// lane's argument.  Phase increments per step are usually small, so the
// short series is the common case.
__device__ __forceinline__ cx<double> expmi_wave(double th) {
  const double a = fabs(th);
  if (__all(a <= 0.0625)) return expmi_tiny(th);
  if (__all(a <= 0.78539816339744830962)) return expmi_quarter(th);
  return expmi_taylor(th);
}


// ---------------------------------------------------------------------------
// time-dependent potential
// ---------------------------------------------------------------------------
struct WaveDev {
  int32_t kind;
  double A0, A1, omega, phase, tc, tau, ti, tf;
};

// Coefficient slots: a0 a1 a2 b0 b1 b2 c s.
enum { CO_A = 0, CO_B = 3, CO_C = 6, CO_S = 7, CO_COUNT = 8 };

struct PotDev {
  WaveDev w[CO_COUNT];
  int32_t v0_kind;  // 0 none, 1 soft-core, 2 Morse
  double v0_par[4];
};

__device__ __forceinline__ double wave_value(const WaveDev &w, double t) {
  switch (w.kind) {
    case 0: return w.A0;
    case 1: return w.A0 + w.A1 * sin(w.omega * t + w.phase);
    case 2: return w.A0 + w.A1 * cos(w.omega * t + w.phase);
    case 3: {
      double u = (t - w.tc) / w.tau;
      return w.A0 + w.A1 * exp(-u * u) * cos(w.omega * t + w.phase);
    }
    case 4: {
      if (t < w.ti || t > w.tf) return w.A0;
      double e = sin(M_PI * (t - w.ti) / (w.tf - w.ti));
      return w.A0 + w.A1 * e * e * cos(w.omega * t + w.phase);
    }
    default: return 0.0;
  }
}

// Non-separable part V0(x) of the potential.
__device__ __forceinline__ double v0_value(const PotDev &p, double x0, double x1, double x2, int ndim) {
  if (p.v0_kind == 1) {
    double r2 = x0 * x0;
    if (ndim > 1) r2 += x1 * x1;
    if (ndim > 2) r2 += x2 * x2;
    return -p.v0_par[0] / sqrt(r2 + p.v0_par[1]);
  }
  if (p.v0_kind == 2) {
    double e = 1.0 - exp(-p.v0_par[1] * (x0 - p.v0_par[2]));
    return p.v0_par[0] * e * e;
  }
  return 0.0;
}

// ---------------------------------------------------------------------------
// storage conversions
// ---------------------------------------------------------------------------
template <class R>
struct storage;
template <>
struct storage<double> {
  using type = double2;
};
template <>
struct storage<float> {
  using type = float2;
};

// Load a stored complex value (float2 or double2) into the compute type, and
// store back with one rounding.
template <class R, class T>
__device__ __forceinline__ cx<R> load_as(const T *p) {
  const T v = *p;
  return {(R)v.x, (R)v.y};
}
template <class R, class T>
__device__ __forceinline__ void store_from(T *p, cx<R> v) {
  T s;
  s.x = v.x;
  s.y = v.y;
  *p = s;
}

// The same with the non-temporal hint (data streamed through once: no
// point keeping it in the caches).
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef double nt_d2 __attribute__((ext_vector_type(2)));
template <class R>
__device__ __forceinline__ cx<R> load_nt_as(const float2 *p) {
  const nt_f2 v = __builtin_nontemporal_load((const nt_f2 *)p);
  return {(R)v.x, (R)v.y};
}
template <class R>
__device__ __forceinline__ cx<R> load_nt_as(const double2 *p) {
  const nt_d2 v = __builtin_nontemporal_load((const nt_d2 *)p);
  return {(R)v.x, (R)v.y};
}
template <class R>
__device__ __forceinline__ void store_nt_from(float2 *p, cx<R> v) {
  const nt_f2 s = {(float)v.x, (float)v.y};
  __builtin_nontemporal_store(s, (nt_f2 *)p);
}
template <class R>
__device__ __forceinline__ void store_nt_from(double2 *p, cx<R> v) {
  const nt_d2 s = {(double)v.x, (double)v.y};
  __builtin_nontemporal_store(s, (nt_d2 *)p);
}

}  // namespace wp
