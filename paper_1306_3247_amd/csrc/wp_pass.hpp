// wp_pass.hpp -- the line-pass kernel: every line along one axis is read from
// HBM once, transformed in registers and LDS, and written back once.
//
// Three kinds of pass (template parameter KIND):
//   PK_F  forward or inverse FFT only (middle axes of a 3D step);
//   PK_V  [inverse FFT] potential phase [forward FFT] (first axis): the
//         potential is evaluated on the device at the current time;
//   PK_K  forward FFT, kinetic phase, inverse FFT (last axis);
//   PK_VS, PK_KS  the two passes of a split 1D grid (OP_SPLIT): PK_VS is
//         [twiddle* inverse FFT] potential phase [forward FFT twiddle] along
//         axis 0 of [n1][n2], PK_KS forward FFT, kinetic phase, inverse FFT
//         along axis 1.
// Workgroup shapes are chosen per (precision, N, layout, kind) so that two or
// more workgroups fit in a CU's 160 KiB of LDS, letting one workgroup load
// while another computes; strided lines of 2048 points and more trade that
// for wider tiles (one workgroup per CU, see pass_cfg::WIDE).
#pragma once
#include <type_traits>

#include "wp_internal.hpp"

namespace wp {

enum PassKind : int { PK_F = 0, PK_V = 1, PK_K = 2, PK_VS = 3, PK_KS = 4 };

constexpr int pow2_floor(int x) {
  int p = 1;
  while (p * 2 <= x) p *= 2;
  return p;
}
constexpr int imin(int a, int b) { return a < b ? a : b; }
constexpr int imax(int a, int b) { return a > b ? a : b; }

// Tuning variants (picked per precision, line length, layout and kind by
// the autotuner of the C ABI): bit 0 gives FP32 passes 8 values per thread
// instead of 16; bit 1 aims at 256 threads and 52 KiB of LDS per workgroup
// (three per CU) instead of 512 threads and 80 KiB (two per CU).  Variants
// other than 0 are compiled for line lengths 64..1024 and kinds F, V, K.
constexpr int kTuneVariants = 4;
constexpr bool tune_compiled(int N, int KIND) { return N >= 64 && N <= 1024 && KIND <= 2; }

template <class S, class R, int N, bool STRIDED, int KIND, int TUNE = 0>
struct pass_cfg {
  static constexpr int ELEM = (int)sizeof(cx<R>);   // LDS element (compute type)
  static constexpr int GELEM = (int)sizeof(cx<S>);  // HBM element (storage type)
  // 16 values per thread in FP32 (8 in FP64) halves the threads per line;
  // the split 1D potential pass, with a twiddle and an FP64 phase per value,
  // keeps 8 to stay within its registers.
  static constexpr int VPT0 = (ELEM == 8 && N >= 16 && KIND != PK_VS) ? 16 : (N < 8 ? N : 8);
  static constexpr int VPT = ((TUNE & 1) && VPT0 == 16) ? 8 : VPT0;
  // Strided lines of 2048 points and more: one workgroup of up to 1024
  // threads per CU with most of the LDS, so that a tile spans more
  // neighbouring lines (longer row segments per cache line).
  static constexpr bool WIDE = STRIDED && N >= 2048 && TUNE == 0;
  static constexpr int TGT = (TUNE & 2) ? 256 : (WIDE ? 1024 : 512);  // threads aimed at
  static constexpr int L = N / VPT;
  static constexpr bool EXCH = N > 8;  // more than one stage: exchanges through LDS
  // Padded line length (see pad16).
  static constexpr int NP = N >= 16 ? N + N / 16 : N;
  // Twiddle entries copied to LDS: the whole table up to 512 points; for
  // longer lines (default variant) those of every stage but the last, which
  // then reads its entries through the caches.
  static constexpr bool TW_LDS = N <= 512;
  static constexpr int TWL = TW_LDS ? tw_count(N) : (TUNE == 0 ? tw_offset<N>(N / 8) : 0);
  static constexpr int TW_BYTES = 16 * TWL;
  // Kinetic factors of the line axis: staged in LDS up to 1024 points; longer
  // lines read them through the caches and leave the LDS to line data.
  static constexpr bool KT_LDS = N <= 1024;
  static constexpr int TAB_BYTES = (KIND == PK_K && KT_LDS) ? 16 * N : 0;
  // At most 80 KiB of LDS per workgroup (two per CU), 52 KiB in variant 2,
  // 156 KiB for WIDE.
  static constexpr int BUDGET = ((TUNE & 2) ? 53248 : (WIDE ? 159744 : 81920)) - 1024;
  static constexpr int DATA_BUDGET = BUDGET - TW_BYTES - TAB_BYTES;
  static constexpr int T_LDS = EXCH ? imax(1, pow2_floor(DATA_BUDGET / (NP * ELEM))) : 4096;
  static constexpr int T_THR = imax(1, TGT / L);
  // Strided lines: enough neighbouring lines that each row segment read is
  // a whole 128-byte cache line, within the thread target.
  static constexpr int T_MIN = STRIDED ? imin(128 / GELEM, imax(1, TGT / L)) : 1;
  static constexpr int TILE = imin(T_LDS, imax(T_THR, T_MIN));
  static constexpr int THREADS = TILE * L;
  // Row segments shorter than a cache line: the two workgroups that share
  // each line are placed on the same XCD (see pair_blocks).
  static constexpr bool PAIR = STRIDED && TILE * GELEM < 128;
  static_assert(THREADS <= 1024, "workgroup too large");
  // Line data; a PK_V pass also stages its per-axis phase table here while
  // the line data is in registers.
  static constexpr int DATA_BYTES = imax(EXCH ? TILE * NP * ELEM : 0, KIND == PK_V ? 16 * N : 0);
  // Waves per SIMD the register allocation must leave room for: two
  // workgroups per CU (at most 128 VGPRs for 512-thread workgroups); three
  // 256-thread workgroups in variant 2.
  static constexpr int WAVES_TARGET = (TUNE & 2) ? imax(1, imin(4, 3 * THREADS / 256)) : imax(1, imin(4, THREADS / 128));
  // No more waves than the LDS of a CU (160 KiB) lets in, so that the
  // register budget is not cut for occupancy that cannot happen.
  static constexpr int LDS_BYTES = DATA_BYTES + TW_BYTES + TAB_BYTES + 64;
  static constexpr int WAVES_LDS = imax(1, (163840 / LDS_BYTES) * ((THREADS + 63) / 64) / 4);
  static constexpr int WAVES_EU = imin(WAVES_TARGET, WAVES_LDS);
};

__device__ __forceinline__ void decode_line(const GridDev &g, int axis, int64_t o, int64_t c, int idx[3]) {
#pragma unroll
  for (int d = 2; d >= 0; --d) {
    if (d > axis) {
      idx[d] = (int)(c & ((1 << g.lg[d]) - 1));
      c >>= g.lg[d];
    }
  }
#pragma unroll
  for (int d = 2; d >= 0; --d) {
    if (d < axis) {
      idx[d] = (int)(o & ((1 << g.lg[d]) - 1));
      o >>= g.lg[d];
    }
  }
  idx[axis] = 0;
}

// Workgroups are handed to the 8 XCDs round-robin (block b to XCD b mod 8),
// each XCD with its own L2.  Within every 16 consecutive blocks this maps
// blocks b and b+8, which share an XCD, to the adjacent tiles 2r and 2r+1,
// so that a cache line split between two tiles is fetched into one L2.
__device__ __forceinline__ unsigned pair_blocks(unsigned b, unsigned nblocks) {
  if (nblocks % 16u != 0u) return b;
  return (b & ~15u) | ((b & 7u) << 1) | ((b >> 3) & 1u);
}

__device__ __forceinline__ double coord(const GridDev &g, int d, int i) {
  return g.lo[d] + (double)i * g.dx[d];
}

// exp(-2 pi i e/n) of a split 1D grid, from two short tables (e taken mod n).
__device__ __forceinline__ cx<double> split_twiddle(const PassArgs &a, int64_t e) {
  e &= ((int64_t)1 << a.g.lg[0]) - 1;
  const int h = a.split_h;
  return cmul(a.wsplit[0][e >> h], a.wsplit[1][e & ((1 << h) - 1)]);
}

// The work of one workgroup: tile `blk` of the lines described by `a`;
// `coef` holds the CO_COUNT waveform values at the pass's time (kind V).
template <class S, class R, int N, bool STRIDED, int KIND, int TUNE, bool EDGE = false>
__device__ __forceinline__ void pass_body(const PassArgs &a, const double *coef, unsigned blk) {
  using C = pass_cfg<S, R, N, STRIDED, KIND, TUNE>;
  using T = typename storage<S>::type;
  constexpr int L = C::L, VPT = C::VPT, TILE = C::TILE, NT = C::THREADS;

  __shared__ __align__(16) unsigned char s_raw[C::DATA_BYTES > 0 ? C::DATA_BYTES : 16];
  __shared__ cx<double> s_tw[C::TWL > 0 ? C::TWL : 1];
  __shared__ cx<double> s_ktab[KIND == PK_K && C::KT_LDS ? N : 1];
  cx<R> *s_data = reinterpret_cast<cx<R> *>(s_raw);

  const int tid = threadIdx.x;
  const int tau = STRIDED ? tid % TILE : tid / L;
  const int t = STRIDED ? tid / TILE : tid % L;
  const int64_t line = (int64_t)blk * TILE + tau;
  const bool valid = line < a.n_lines;
  // Contiguous lines are those of the last axis (nothing inside them).
  const int lgi = STRIDED ? a.lg_inner : 0;
  const int64_t o = line >> lgi, c = line & (((int64_t)1 << lgi) - 1);
  const int64_t base = (o << (fft_shape<N>::lg + lgi)) + c;
  // Element t + L*u of this thread's line is at pt + u*ustep (ustep is the
  // same for the whole workgroup).  A line of the first axis crosses the
  // planes, whose storage lies 2^lgi + pad points apart; the lines of the
  // other axes stay inside one plane.
  const int64_t lstride = STRIDED ? ((int64_t)1 << lgi) + (a.axis == 0 ? (int64_t)a.g.pad : 0) : 1;
  T *const pt = (T *)a.psi + phys_index(a.g, base) + t * lstride;
  const int64_t ustep = (int64_t)L * lstride;
  const uint32_t ops = a.ops;

  // Non-temporal stores only where a workgroup writes whole cache lines: a
  // line split between two workgroups is written twice and should meet its
  // other half in L2.
  constexpr uint32_t NT_OK = C::PAIR ? (uint32_t)OP_LOAD_NT : (OP_LOAD_NT | OP_STORE_NT);
  cx<R> v[VPT];
  if (valid && (ops & OP_LOAD_NT & NT_OK)) {
#pragma unroll
    for (int u = 0; u < VPT; ++u) v[u] = load_nt_as<R>(pt + u * ustep);
  } else if (valid) {
#pragma unroll
    for (int u = 0; u < VPT; ++u) v[u] = load_as<R>(pt + u * ustep);
  } else {
#pragma unroll
    for (int u = 0; u < VPT; ++u) v[u] = cx<R>{0, 0};
  }

  // FP32 passes with the whole table in LDS keep it as hi + lo pairs (the
  // same 16 bytes per entry; see TwHiLo), the others as FP64.
  constexpr bool HILO = std::is_same<R, float>::value && C::TW_LDS && C::TWL > 0;
  using TwT = std::conditional_t<HILO, TwHiLo, TwSplit<C::TWL>>;
  TwT tw;
  if constexpr (HILO) {
    float4 *s_tw4 = reinterpret_cast<float4 *>(s_tw);
    for (int e = tid; e < C::TWL; e += NT) s_tw4[e] = hilo_of(a.tw[e]);
    tw = TwHiLo{s_tw4};
  } else {
    if constexpr (C::TWL > 0)
      for (int e = tid; e < C::TWL; e += NT) s_tw[e] = a.tw[e];
    tw = TwSplit<C::TWL>{s_tw, a.tw};
  }
  if constexpr (KIND == PK_K && C::KT_LDS) {
    for (int e = tid; e < N; e += NT) s_ktab[e] = a.ktab[a.axis][e];
    __syncthreads();
  }

  // Indices of this thread's line on the other axes.
  int idx[3];
  decode_line(a.g, a.axis, o, c, idx);

  auto lds = [&](int p) -> cx<R> & {
    if constexpr (STRIDED) return s_data[p * TILE + tau];
    else return s_data[tau * C::NP + p];
  };

  if constexpr (KIND == PK_F) {
    if (ops & OP_PRE_INV) line_fft<N, VPT, true>(v, t, tw, lds);
    else line_fft<N, VPT, false>(v, t, tw, lds);
  } else if constexpr (KIND == PK_KS) {
    // Line k1 of [n1][n2]; after the forward transform position k2 holds
    // bin k1 + n1*k2 of the n-point transform (index taken mod n, so that
    // the idle lanes of a partial tile stay inside the table).
    const int64_t nmask = ((int64_t)1 << a.g.lg[0]) - 1;
    const cx<double> *kt = a.ktab[0];
    line_fft<N, VPT, false>(v, t, tw, lds);
#pragma unroll
    for (int u = 0; u < VPT; ++u) v[u] = mul_acc(v[u], kt[(line + a.n_lines * (int64_t)(t + L * u)) & nmask]);
    line_fft<N, VPT, true>(v, t, tw, lds);
  } else if constexpr (KIND == PK_VS) {
    // Column j2 = line of [n1][n2]; position j1 along it is the grid point
    // j1*n2 + j2.  Between the two line transforms of the n-point transform
    // sit the twiddles exp(-2 pi i j2 k1/n) (forward) and their conjugates
    // (inverse).
    const int64_t j2 = line;
    const int lg2 = lgi;
    if (ops & OP_PRE_INV) {
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const cx<double> w = split_twiddle(a, j2 * (int64_t)(t + L * u));
        v[u] = mul_acc(v[u], cx<double>{w.x, -w.y});
      }
      line_fft<N, VPT, true>(v, t, tw, lds);
    }
    if (ops & OP_V) {
      const double *s_coef = coef;  // uniform: scalar loads
      const double vt = a.vtau;
      const double cc = vt * s_coef[CO_C], ca = vt * s_coef[CO_A], cb = vt * s_coef[CO_B];
      const double cs = vt * s_coef[CO_S];
      const int kind = a.pot.v0_kind;
      const double p0 = a.pot.v0_par[0], p1 = a.pot.v0_par[1], p2 = a.pot.v0_par[2];
      const double lo = a.g.lo[0], dx = a.g.dx[0];
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const double x = lo + (double)(((int64_t)(t + L * u) << lg2) + j2) * dx;
        double th = cc + x * fma(cb, x, ca);
        if (kind == 1) {
          th -= cs * p0 * rsqrt_fast(fma(x, x, p1));
        } else if (kind == 2) {
          const double e = 1.0 - exp(-p1 * (x - p2));
          th += cs * p0 * e * e;
        }
        v[u] = mul_acc(v[u], expmi_wave(th));
      }
    }
    if (ops & OP_FWD) {
      line_fft<N, VPT, false>(v, t, tw, lds);
#pragma unroll
      for (int u = 0; u < VPT; ++u) v[u] = mul_acc(v[u], split_twiddle(a, j2 * (int64_t)(t + L * u)));
    }
  } else if constexpr (KIND == PK_K) {
    // Kinetic factor of this line on the other axes (1/N is in the table of
    // the last axis).
    cx<double> kl = {1.0, 0.0};
    for (int d = 0; d < a.g.ndim; ++d)
      if (d != a.axis) kl = cmul(kl, a.ktab[d][idx[d]]);
    // Last-axis lines of at most 64 threads lie within one wavefront each;
    // the tables were shared after the barrier above.
    constexpr bool WAVE = !STRIDED && L <= 64;
    const cx<double> *ktab = C::KT_LDS ? (const cx<double> *)s_ktab : a.ktab[a.axis];
    line_fft<N, VPT, false, WAVE>(v, t, tw, lds);
#pragma unroll
    for (int u = 0; u < VPT; ++u) v[u] = mul_acc(v[u], cmul(ktab[t + L * u], kl));
    line_fft<N, VPT, true, WAVE>(v, t, tw, lds);
  } else {
    const double *s_coef = coef;  // uniform: scalar loads
    const int ax = a.axis;
    const double vt = a.vtau;
    // phase = vt * (c + sum_d [a_d x_d + b_d x_d^2] + s V0(x)); the terms of
    // the other axes are constant along the line.
    double th_line = s_coef[CO_C], rho2 = 0.0;
    for (int d = 0; d < a.g.ndim; ++d) {
      if (d == ax) continue;
      const double x = coord(a.g, d, idx[d]);
      th_line += s_coef[CO_A + d] * x + s_coef[CO_B + d] * x * x;
      rho2 += x * x;
    }
    th_line *= vt;
    const double ca = vt * s_coef[CO_A + ax], cb = vt * s_coef[CO_B + ax];
    const double lo = a.g.lo[ax], dx = a.g.dx[ax];
    const bool separable = a.pot.v0_kind == 0;

    if (ops & OP_PRE_INV) line_fft<N, VPT, true>(v, t, tw, lds);
    if (separable) {
      // Phase table of the line axis, staged in the (now idle) line buffer.
      cx<double> *tab = reinterpret_cast<cx<double> *>(s_raw);
      if constexpr (C::EXCH) __syncthreads();  // every thread is done with the line buffer
      for (int e = tid; e < N; e += NT) {
        const double x = lo + (double)e * dx;
        tab[e] = expmi_taylor(x * fma(cb, x, ca));
      }
      const cx<double> fl = expmi_taylor(th_line);
      __syncthreads();
#pragma unroll
      for (int u = 0; u < VPT; ++u) v[u] = mul_acc(v[u], cmul(tab[t + L * u], fl));
    } else {
      const double cs = vt * s_coef[CO_S];
      const int kind = a.pot.v0_kind;
      const double p0 = a.pot.v0_par[0], p1 = a.pot.v0_par[1], p2 = a.pot.v0_par[2];
      const double r2off = rho2 + p1;
      // Soft core: on this line q = x^2 + r2off lies between r2off and
      // xm^2 + r2off (xm the largest |x|), so one check of the ends admits
      // the FP32-range reciprocal square root for every point, and
      // |th| <= |th_line| + |ca| xm + |cb| xm^2 + |cs p0| / sqrt(r2off)
      // admits the short series for every point; other lines choose point
      // by point.
      const double xm = fmax(fabs(lo), fabs(lo + (double)(N - 1) * dx));
      const bool soft_fast =
          kind == 1 && __all(r2off > 1e-30 && fma(xm, xm, r2off) < 1e30 &&
                             fabs(th_line) + xm * (fabs(ca) + xm * fabs(cb)) + fabs(cs * p0) * rsqrt(r2off) <= 0.0625);
      if (soft_fast) {
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
          const double x = lo + (double)(t + L * u) * dx;
          const double th = th_line + x * fma(cb, x, ca) - cs * p0 * rsqrt_newton(fma(x, x, r2off));
          v[u] = mul_acc(v[u], expmi_tiny(th));
        }
      } else {
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
          const double x = lo + (double)(t + L * u) * dx;
          double th = th_line + x * fma(cb, x, ca);
          if (kind == 1) {
            th -= cs * p0 * rsqrt_fast(fma(x, x, r2off));
          } else {
            const double e = 1.0 - exp(-p1 * (x - p2));
            th += cs * p0 * e * e;
          }
          v[u] = mul_acc(v[u], expmi_wave(th));
        }
      }
    }
    if (ops & OP_FWD) line_fft<N, VPT, false>(v, t, tw, lds);  // starts with a barrier
  }

  if constexpr (EDGE && KIND == PK_V && STRIDED) {
    // Moments of the final values, as the observables define them (the
    // value as stored, w = |psi|^2 in FP64): the line axis varies per
    // value, the other axes are constant along the line.  Fixed-order
    // workgroup tree in the (now idle) line buffer.
    if (a.moments) {
      double m0 = 0.0, m1 = 0.0, m2 = 0.0;
      if (valid) {
#pragma unroll
        for (int u = 0; u < VPT; ++u) {
          const double pr = (double)(S)v[u].x, pi = (double)(S)v[u].y;
          const double w = pr * pr + pi * pi;
          const double x = coord(a.g, a.axis, t + L * u);
          m0 += w;
          m1 += x * w;
          m2 += x * x * w;
        }
      }
      double m[8] = {m0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        if (d == a.axis) {
          m[1 + d] = m1;
          m[4 + d] = m2;
        } else {
          const double c = coord(a.g, d, idx[d]);
          m[1 + d] = c * m0;
          m[4 + d] = c * c * m0;
        }
      }
      // The line buffer holds the tree where it is large enough (every line
      // length that exchanges through LDS); short lines get their own.
      constexpr bool OWN = 8 * NT * sizeof(double) > sizeof(s_raw);
      __shared__ double s_own[OWN ? 8 * NT : 1];
      double *red = OWN ? s_own : reinterpret_cast<double *>(s_raw);
      __syncthreads();  // every thread is done with the line buffer
#pragma unroll
      for (int k = 0; k < 8; ++k) red[k * NT + tid] = m[k];
      __syncthreads();
      for (int h = NT / 2; h > 0; h >>= 1) {
        if (tid < h) {
#pragma unroll
          for (int k = 0; k < 8; ++k) red[k * NT + tid] += red[k * NT + tid + h];
        }
        __syncthreads();
      }
      if (tid < 8) a.moments[(int64_t)blk * 8 + tid] = red[tid * NT];
    }
  }

  if (valid && (ops & OP_STORE_NT & NT_OK)) {
#pragma unroll
    for (int u = 0; u < VPT; ++u) store_nt_from(pt + u * ustep, v[u]);
  } else if (valid) {
#pragma unroll
    for (int u = 0; u < VPT; ++u) store_from(pt + u * ustep, v[u]);
  }
}

template <class S, class R, int N, bool STRIDED, int KIND, int TUNE>
__global__ void __launch_bounds__((pass_cfg<S, R, N, STRIDED, KIND, TUNE>::THREADS),
                                  (pass_cfg<S, R, N, STRIDED, KIND, TUNE>::WAVES_EU))
    pass_kernel(PassArgs a) {
  using C = pass_cfg<S, R, N, STRIDED, KIND, TUNE>;
  const unsigned blk = C::PAIR ? pair_blocks(blockIdx.x, gridDim.x) : blockIdx.x;
  pass_body<S, R, N, STRIDED, KIND, TUNE>(a, a.coef, blk);
}

// The same first-axis potential pass under its own symbol, for the passes
// that open or close a propagation (one transform instead of two), so that
// per-kernel profiles report them apart from the steady-state pass; the
// closing pass can also reduce the moments of the final state
// (PassArgs::moments) without touching the steady kernel's registers.
template <class S, class R, int N, bool STRIDED, int KIND, int TUNE>
__global__ void __launch_bounds__((pass_cfg<S, R, N, STRIDED, KIND, TUNE>::THREADS),
                                  (pass_cfg<S, R, N, STRIDED, KIND, TUNE>::WAVES_EU))
    edge_pass_kernel(PassArgs a) {
  using C = pass_cfg<S, R, N, STRIDED, KIND, TUNE>;
  const unsigned blk = C::PAIR ? pair_blocks(blockIdx.x, gridDim.x) : blockIdx.x;
  pass_body<S, R, N, STRIDED, KIND, TUNE, true>(a, a.coef, blk);
}

// Batched: workgroup b runs tile items[b].tile of solve items[b].solve, whose
// argument block is args[items[b].solve * nvar + var]; `row` selects the
// waveform values of the step this launch belongs to.
template <class S, class R, int N, bool STRIDED, int KIND, int TUNE>
__global__ void __launch_bounds__((pass_cfg<S, R, N, STRIDED, KIND, TUNE>::THREADS),
                                  (pass_cfg<S, R, N, STRIDED, KIND, TUNE>::WAVES_EU))
    batch_pass_kernel(const PassArgs *args, const BatchItem *items, int nvar, int var, int row) {
  const BatchItem it = items[blockIdx.x];
  // A reference into global memory, not a copy: the fields are read with
  // scalar loads (the address is uniform), no private copy of the block.
  const PassArgs &a = args[it.solve * nvar + var];
  pass_body<S, R, N, STRIDED, KIND, TUNE>(a, a.coef ? a.coef + row * CO_COUNT : nullptr, (unsigned)it.tile);
}

template <class S, class R, int N, bool STRIDED, int KIND, int TUNE>
hipError_t launch_batch_t(const BatchLaunch &b, hipStream_t s) {
  using C = pass_cfg<S, R, N, STRIDED, KIND, TUNE>;
  hipLaunchKernelGGL((batch_pass_kernel<S, R, N, STRIDED, KIND, TUNE>), dim3(b.nblocks), dim3(C::THREADS), 0, s,
                     b.args, b.items, b.nvar, b.var, b.row);
  return hipGetLastError();
}

template <class S, class R, int N, bool STRIDED, int KIND, int TUNE>
hipError_t launch_pass_t(const PassArgs &a, hipStream_t s) {
  using C = pass_cfg<S, R, N, STRIDED, KIND, TUNE>;
  const int64_t blocks = (a.n_lines + C::TILE - 1) / C::TILE;
  if constexpr (KIND == PK_V && STRIDED) {
    if (!((a.ops & OP_PRE_INV) && (a.ops & OP_FWD)))
      return launch_kernel(edge_pass_kernel<S, R, N, STRIDED, KIND, TUNE>, dim3((unsigned)blocks), dim3(C::THREADS),
                           s, a);
  }
  return launch_kernel(pass_kernel<S, R, N, STRIDED, KIND, TUNE>, dim3((unsigned)blocks), dim3(C::THREADS), s, a);
}

// What one launch needs: kind (PK_*), layout, tuning variant.  The kind of a
// single pass follows from its operations.
__host__ inline int pass_kind_of(const PassArgs &a) {
  if (a.ops & OP_SPLIT) return a.axis == 0 ? PK_VS : PK_KS;
  if (a.ops & OP_V) return PK_V;
  if (a.ops & OP_K) return PK_K;
  return PK_F;
}

// Call f(integral_constant<N>) for N = 2^lgN, 1 <= lgN <= 12.
template <class F>
__host__ inline auto with_n(int lgN, F &&f) -> decltype(f(std::integral_constant<int, 2>{})) {
  switch (lgN) {
    case 1: return f(std::integral_constant<int, 2>{});
    case 2: return f(std::integral_constant<int, 4>{});
    case 3: return f(std::integral_constant<int, 8>{});
    case 4: return f(std::integral_constant<int, 16>{});
    case 5: return f(std::integral_constant<int, 32>{});
    case 6: return f(std::integral_constant<int, 64>{});
    case 7: return f(std::integral_constant<int, 128>{});
    case 8: return f(std::integral_constant<int, 256>{});
    case 9: return f(std::integral_constant<int, 512>{});
    case 10: return f(std::integral_constant<int, 1024>{});
    case 11: return f(std::integral_constant<int, 2048>{});
    default: return f(std::integral_constant<int, 4096>{});
  }
}

// Call f(KIND, STRIDED) as compile-time constants for the combinations that
// exist: F, V, K in both layouts; VS strided; KS contiguous.
template <int N, int TUNE, class F>
__host__ inline hipError_t with_kind(int kind, bool strided, F &&f) {
  using std::integral_constant;
  using T = integral_constant<bool, true>;
  using U = integral_constant<bool, false>;
  if constexpr (TUNE != 0 && !tune_compiled(N, 0)) {
    return hipErrorInvalidValue;
  } else {
    if (kind == PK_V) return strided ? f(integral_constant<int, PK_V>{}, T{}) : f(integral_constant<int, PK_V>{}, U{});
    if (kind == PK_K) return strided ? f(integral_constant<int, PK_K>{}, T{}) : f(integral_constant<int, PK_K>{}, U{});
    if (kind == PK_F) return strided ? f(integral_constant<int, PK_F>{}, T{}) : f(integral_constant<int, PK_F>{}, U{});
    if constexpr (TUNE == 0 && N >= 128 && N <= 1024) {
      if (kind == PK_VS && strided) return f(integral_constant<int, PK_VS>{}, T{});
      if (kind == PK_KS && !strided) return f(integral_constant<int, PK_KS>{}, U{});
    }
    return hipErrorInvalidValue;
  }
}

// The entry points each precision-and-variant translation unit instantiates.
template <class S, class R, int TUNE>
hipError_t dispatch_pass(int lgN, const PassArgs &a, hipStream_t s) {
  const int kind = pass_kind_of(a);
  const bool strided = a.lg_inner > 0;
  return with_n(lgN, [&](auto n) -> hipError_t {
    constexpr int NN = decltype(n)::value;
    return with_kind<NN, TUNE>(kind, strided, [&](auto k, auto st) -> hipError_t {
      return launch_pass_t<S, R, NN, decltype(st)::value, decltype(k)::value, TUNE>(a, s);
    });
  });
}

template <class S, class R, int TUNE>
hipError_t dispatch_batch(const BatchLaunch &b, hipStream_t s) {
  return with_n(b.lgN, [&](auto n) -> hipError_t {
    constexpr int NN = decltype(n)::value;
    return with_kind<NN, TUNE>(b.kind, b.strided, [&](auto k, auto st) -> hipError_t {
      return launch_batch_t<S, R, NN, decltype(st)::value, decltype(k)::value, TUNE>(b, s);
    });
  });
}

// Lines per workgroup of a pass configuration (the host sizes block maps
// with it); 0 for a combination that is not compiled.
template <class S, class R, int TUNE>
int pass_tile_t(int lgN, bool strided, int kind) {
  int tile = 0;
  (void)with_n(lgN, [&](auto n) -> hipError_t {
    constexpr int NN = decltype(n)::value;
    return with_kind<NN, TUNE>(kind, strided, [&](auto k, auto st) -> hipError_t {
      tile = pass_cfg<S, R, NN, decltype(st)::value, decltype(k)::value, TUNE>::TILE;
      return hipSuccess;
    });
  });
  return tile;
}

}  // namespace wp
