/*
 * oracle.c -- plain FP64 CPU reference of the split-operator time step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the GPU library.  It is written
 * for the reader, not for speed: a textbook radix-2 FFT, explicit loops, and
 * one OpenMP loop over independent lines or grid planes (which does not change
 * any result).  Build flags: -O2 -ffp-contract=off (no fused multiply-add).
 *
 * Every function cites the part of the paper it follows.  Where the paper is
 * silent or garbled, the reading taken is stated at the point of use.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

static const double ORC_PI = 3.14159265358979323846264338327950288;

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int is_pow2(int64_t n) { return n >= 1 && (n & (n - 1)) == 0; }

/* Any axis length n >= 2 is accepted: the transform below handles every
 * factorisation (the paper advises lengths with small prime factors for
 * speed, Section 3.2.1 under nx/ny/nz, not for correctness). */
static int grid_ok(const orc_grid *g) {
  if (g->ndim < 1 || g->ndim > 3) return 0;
  for (int d = 0; d < 3; ++d) {
    if (d < g->ndim) {
      if (g->n[d] < 2) return 0;
      if (!(g->hi[d] > g->lo[d])) return 0;
    } else if (g->n[d] != 1) {
      return 0;
    }
  }
  return g->mass > 0 && g->hbar > 0;
}

static int64_t grid_size(const orc_grid *g) { return g->n[0] * g->n[1] * g->n[2]; }

static double spacing(const orc_grid *g, int d) {
  return (g->hi[d] - g->lo[d]) / (double)g->n[d];
}

/* ---- time-dependent coefficients -------------------------------------- */

/* Scalar waveforms.  The sin^2 envelope is the pulse envelope of Section 4.1,
 * written as sin^2(pi (t - ti)/(tf - ti)) on [ti, tf] and zero outside; for
 * ti = 0 this is the paper's sin^2(pi t/(tf - ti)). */
double orc_wave_eval(const orc_wave *w, double t) {
  switch (w->kind) {
  case ORC_WAVE_CONST:
    return w->A0;
  case ORC_WAVE_SIN:
    return w->A0 + w->A1 * sin(w->omega * t + w->phase);
  case ORC_WAVE_COS:
    return w->A0 + w->A1 * cos(w->omega * t + w->phase);
  case ORC_WAVE_GAUSS_COS: {
    double u = (t - w->tc) / w->tau;
    return w->A0 + w->A1 * exp(-u * u) * cos(w->omega * t + w->phase);
  }
  case ORC_WAVE_SIN2_COS: {
    if (t < w->ti || t > w->tf) return w->A0;
    double e = sin(ORC_PI * (t - w->ti) / (w->tf - w->ti));
    return w->A0 + w->A1 * e * e * cos(w->omega * t + w->phase);
  }
  default:
    return NAN;
  }
}

/* ---- grids (Section 2.1) ------------------------------------------------ */

/* x_i = x_min + i dx (eq. grid).  The paper's dx = (x_max - x_min)/(n-1)
 * (eq. Deltax) with x_max the last point; with the period n dx that the
 * momentum grid implies, this is the half-open interval [lo, lo + n dx). */
int orc_coords(const orc_grid *g, int axis, double *out) {
  if (!grid_ok(g) || axis < 0 || axis > 2) return ORC_EINVAL;
  double dx = spacing(g, axis);
  for (int64_t i = 0; i < g->n[axis]; ++i) out[i] = g->lo[axis] + (double)i * dx;
  return ORC_OK;
}

/* Momentum grid p_i = 2 pi hbar i / (n dx) (Section 2.1, after eq. ft); the
 * wavenumber k = p / hbar is stored in DFT output order: index m < n/2 holds
 * m, index m >= n/2 holds m - n (the Nyquist bin m = n/2 of an even n becomes
 * -n/2; the paper's list i = -n/2..n/2 has one entry too many, and k^2 is the
 * same for either sign; for odd n the bins are -(n-1)/2..(n-1)/2). */
int orc_wavenumbers(const orc_grid *g, int axis, double *out) {
  if (!grid_ok(g) || axis < 0 || axis > 2) return ORC_EINVAL;
  int64_t n = g->n[axis];
  double L = (double)n * spacing(g, axis);
  for (int64_t m = 0; m < n; ++m) {
    int64_t mm = (2 * m < n) ? m : m - n;
    out[m] = 2.0 * ORC_PI * (double)mm / L;
  }
  if (n == 1) out[0] = 0.0;
  return ORC_OK;
}

/* V(x, t) at every grid point (the user function `potential` of Section 3.2,
 * here a fixed parametric family; the Morse term is the molecular potential
 * of Section 4.1 and the quadratic terms cover the Paul trap of Section 4.2). */
int orc_potential(const orc_grid *g, const orc_pot *p, double t, double *V) {
  if (!grid_ok(g)) return ORC_EINVAL;
  double *x[3];
  double a[3] = {0, 0, 0}, b[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    x[d] = (double *)malloc(sizeof(double) * (size_t)g->n[d]);
    if (!x[d]) return ORC_ENOMEM;
    orc_coords(g, d, x[d]);
    if (d < g->ndim) {
      a[d] = orc_wave_eval(&p->a[d], t);
      b[d] = orc_wave_eval(&p->b[d], t);
    }
  }
  double c = orc_wave_eval(&p->c, t);
  double s = (p->v0_kind == ORC_V0_NONE) ? 0.0 : orc_wave_eval(&p->s, t);
  int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for
  for (int64_t i = 0; i < nx; ++i) {
    for (int64_t j = 0; j < ny; ++j) {
      for (int64_t k = 0; k < nz; ++k) {
        double xs[3] = {x[0][i], x[1][j], x[2][k]};
        double v = c;
        for (int d = 0; d < g->ndim; ++d) v += a[d] * xs[d] + b[d] * xs[d] * xs[d];
        if (p->v0_kind == ORC_V0_SOFTCORE) {
          double r2 = 0.0;
          for (int d = 0; d < g->ndim; ++d) r2 += xs[d] * xs[d];
          v += s * (-p->v0_par[0] / sqrt(r2 + p->v0_par[1]));
        } else if (p->v0_kind == ORC_V0_MORSE) {
          double e = 1.0 - exp(-p->v0_par[1] * (xs[0] - p->v0_par[2]));
          v += s * (p->v0_par[0] * e * e);
        }
        V[(i * ny + j) * nz + k] = v;
      }
    }
  }
  for (int d = 0; d < 3; ++d) free(x[d]);
  return ORC_OK;
}

/* ---- discrete Fourier transforms (Section 2.1, eq. ft) ---------------- */

/* The definition, O(n^2): X_m = sum_j x_j exp(dir 2 pi i j m / n); the
 * inverse (dir = +1) also divides by n. */
int orc_dft1d(int64_t n, const double complex *in, double complex *out, int dir) {
  if (n < 1 || (dir != -1 && dir != 1)) return ORC_EINVAL;
  for (int64_t m = 0; m < n; ++m) {
    double complex acc = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      int64_t e = (j * m) % n; /* exact reduction keeps the angle small */
      double ang = 2.0 * ORC_PI * (double)e / (double)n;
      acc += in[j] * (cos(ang) + dir * I * sin(ang));
    }
    out[m] = (dir == 1) ? acc / (double)n : acc;
  }
  return ORC_OK;
}

/* Textbook iterative radix-2 decimation-in-time FFT: bit-reversal
 * permutation, then log2(n) butterfly stages.  tw[j] = exp(dir 2 pi i j / n)
 * for j < n/2, each computed directly from cos and sin. */
static void fft_line(int64_t n, double complex *a, const double complex *tw, int dir) {
  for (int64_t i = 1, j = 0; i < n; ++i) {
    int64_t bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) {
      double complex t = a[i];
      a[i] = a[j];
      a[j] = t;
    }
  }
  for (int64_t len = 2; len <= n; len <<= 1) {
    int64_t half = len >> 1, step = n / len;
    for (int64_t s = 0; s < n; s += len) {
      for (int64_t j = 0; j < half; ++j) {
        double complex u = a[s + j];
        double complex v = a[s + j + half] * tw[j * step];
        a[s + j] = u + v;
        a[s + j + half] = u - v;
      }
    }
  }
  if (dir == 1) {
    double inv = 1.0 / (double)n;
    for (int64_t i = 0; i < n; ++i) a[i] *= inv;
  }
}

/* exp(dir 2 pi i e / n), the exponent reduced exactly mod n first. */
static double complex unit_root(int64_t e, int64_t n, int dir) {
  double ang = 2.0 * ORC_PI * (double)(e % n) / (double)n;
  return cos(ang) + dir * I * sin(ang);
}

static int64_t smallest_factor(int64_t n) {
  for (int64_t p = 2; p * p <= n; ++p)
    if (n % p == 0) return p;
  return n;
}

/* Mixed-radix decimation in time (Cooley and Tukey) for any n: with p the
 * smallest prime factor of n and m = n/p, the m-point transforms Y_r of the
 * subsequences x[r + p j] (r < p) give X[k + m q] = sum_r W^(r (k + m q)) Y_r[k],
 * W = exp(dir 2 pi i / n).  Reads in[j*stride], writes out[0..n); tmp holds n
 * values.  Unnormalised. */
static void fft_mixed(int64_t n, const double complex *in, int64_t stride, double complex *out,
                      double complex *tmp, int dir) {
  if (n == 1) {
    out[0] = in[0];
    return;
  }
  int64_t p = smallest_factor(n), m = n / p;
  for (int64_t r = 0; r < p; ++r) fft_mixed(m, in + r * stride, stride * p, tmp + r * m, out + r * m, dir);
  for (int64_t k = 0; k < m; ++k)
    for (int64_t q = 0; q < p; ++q) {
      double complex acc = 0.0;
      for (int64_t r = 0; r < p; ++r) acc += unit_root(r * (k + m * q), n, dir) * tmp[r * m + k];
      out[k + m * q] = acc;
    }
}

/* One line of any length: radix 2 for powers of two, the mixed-radix
 * recursion otherwise; the inverse (dir = +1) divides by n. */
static int line_transform(int64_t n, double complex *a, const double complex *tw, int dir) {
  if (is_pow2(n)) {
    fft_line(n, a, tw, dir);
    return ORC_OK;
  }
  double complex *src = (double complex *)malloc(sizeof(double complex) * (size_t)n);
  double complex *tmp = (double complex *)malloc(sizeof(double complex) * (size_t)n);
  if (!src || !tmp) {
    free(src);
    free(tmp);
    return ORC_ENOMEM;
  }
  memcpy(src, a, sizeof(double complex) * (size_t)n);
  fft_mixed(n, src, 1, a, tmp, dir);
  if (dir == 1)
    for (int64_t i = 0; i < n; ++i) a[i] /= (double)n;
  free(src);
  free(tmp);
  return ORC_OK;
}

static double complex *twiddles(int64_t n, int dir) {
  double complex *tw = (double complex *)malloc(sizeof(double complex) * (size_t)(n / 2 + 1));
  if (!tw) return NULL;
  for (int64_t j = 0; j < n / 2 + 1; ++j) {
    double ang = 2.0 * ORC_PI * (double)j / (double)n;
    tw[j] = cos(ang) + dir * I * sin(ang);
  }
  return tw;
}

int orc_fft1d(int64_t n, double complex *data, int dir) {
  if (n < 1 || (dir != -1 && dir != 1)) return ORC_EINVAL;
  if (n == 1) return ORC_OK;
  double complex *tw = twiddles(n, dir);
  if (!tw) return ORC_ENOMEM;
  int rc = line_transform(n, data, tw, dir);
  free(tw);
  return rc;
}

/* 1D transform along one axis of the row-major array: each line is copied
 * out, transformed and copied back.  Lines are independent. */
static int fft_axis(const orc_grid *g, double complex *psi, int axis, int dir) {
  int64_t n = g->n[axis];
  if (n == 1) return ORC_OK;
  int64_t inner = 1, outer = 1;
  for (int d = axis + 1; d < 3; ++d) inner *= g->n[d];
  for (int d = 0; d < axis; ++d) outer *= g->n[d];
  double complex *tw = twiddles(n, dir);
  if (!tw) return ORC_ENOMEM;
  int64_t nlines = outer * inner;
  int fail = 0;
#pragma omp parallel
  {
    double complex *buf = (double complex *)malloc(sizeof(double complex) * (size_t)n);
    if (!buf) {
#pragma omp atomic write
      fail = 1;
    }
#pragma omp for
    for (int64_t l = 0; l < nlines; ++l) {
      if (!buf) continue;
      int64_t o = l / inner, c = l % inner;
      double complex *base = psi + o * n * inner + c;
      for (int64_t i = 0; i < n; ++i) buf[i] = base[i * inner];
      if (line_transform(n, buf, tw, dir) != ORC_OK) {
#pragma omp atomic write
        fail = 1;
      }
      for (int64_t i = 0; i < n; ++i) base[i * inner] = buf[i];
    }
    free(buf);
  }
  free(tw);
  return fail ? ORC_ENOMEM : ORC_OK;
}

/* Multi-dimensional DFT: the 1D transform applied along every axis. */
int orc_fftn(const orc_grid *g, double complex *psi, int dir) {
  if (!grid_ok(g) || (dir != -1 && dir != 1)) return ORC_EINVAL;
  for (int d = 0; d < 3; ++d) {
    int rc = fft_axis(g, psi, d, dir);
    if (rc) return rc;
  }
  return ORC_OK;
}

/* ---- initial state (Section 4.2, Gaussian wave packet) ---------------- */

/* psi0 = prod_d (2/pi)^(1/4) sigma_d^(-1/2)
 *            exp(-(x_d - c_d)^2 / sigma_d^2 + i k_d (x_d - c_d)),
 * k_d = p_d0 / hbar, then divided by its discrete norm so that
 * sum |psi|^2 dV = 1 exactly up to rounding. */
int orc_gaussian(const orc_grid *g, const double c[3], const double sigma[3],
                 const double k[3], double complex *psi) {
  if (!grid_ok(g)) return ORC_EINVAL;
  double complex *f[3];
  for (int d = 0; d < 3; ++d) {
    f[d] = (double complex *)malloc(sizeof(double complex) * (size_t)g->n[d]);
    double *x = (double *)malloc(sizeof(double) * (size_t)g->n[d]);
    if (!f[d] || !x) return ORC_ENOMEM;
    orc_coords(g, d, x);
    for (int64_t i = 0; i < g->n[d]; ++i) {
      if (d >= g->ndim) {
        f[d][i] = 1.0;
        continue;
      }
      double u = x[i] - c[d];
      double amp = pow(2.0 / ORC_PI, 0.25) / sqrt(sigma[d]) * exp(-u * u / (sigma[d] * sigma[d]));
      f[d][i] = amp * (cos(k[d] * u) + I * sin(k[d] * u));
    }
    free(x);
  }
  int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
  for (int64_t i = 0; i < nx; ++i)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t kk = 0; kk < nz; ++kk) psi[(i * ny + j) * nz + kk] = f[0][i] * f[1][j] * f[2][kk];
  for (int d = 0; d < 3; ++d) free(f[d]);
  double dV = 1.0, s = 0.0;
  for (int d = 0; d < g->ndim; ++d) dV *= spacing(g, d);
  int64_t N = grid_size(g);
  for (int64_t i = 0; i < N; ++i) s += creal(psi[i]) * creal(psi[i]) + cimag(psi[i]) * cimag(psi[i]);
  double nrm = sqrt(s * dV);
  for (int64_t i = 0; i < N; ++i) psi[i] /= nrm;
  return ORC_OK;
}

/* ---- the time step (Section 2.1, eqs. short-time and splitop) --------- */

/* psi <- psi * exp(-i theta(x)), theta = V(x, t) * tau / hbar, with
 * exp(-i theta) = cos(theta) - i sin(theta). */
static int apply_potential_phase(const orc_grid *g, const orc_pot *p, double complex *psi,
                                 double t, double tau, double *V) {
  int rc = orc_potential(g, p, t, V);
  if (rc) return rc;
  int64_t N = grid_size(g);
#pragma omp parallel for
  for (int64_t i = 0; i < N; ++i) {
    double th = V[i] * tau / g->hbar;
    psi[i] *= cos(th) - I * sin(th);
  }
  return ORC_OK;
}

/* psi <- F^-1 exp(-i hbar |k|^2 tau / 2m) F psi  (eq. ft with K = p^2/2m). */
static int apply_kinetic(const orc_grid *g, double complex *psi, double tau) {
  int rc = orc_fftn(g, psi, -1);
  if (rc) return rc;
  double *k[3];
  for (int d = 0; d < 3; ++d) {
    k[d] = (double *)malloc(sizeof(double) * (size_t)g->n[d]);
    if (!k[d]) return ORC_ENOMEM;
    orc_wavenumbers(g, d, k[d]);
  }
  int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2];
#pragma omp parallel for
  for (int64_t i = 0; i < nx; ++i)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t m = 0; m < nz; ++m) {
        double k2 = k[0][i] * k[0][i] + k[1][j] * k[1][j] + k[2][m] * k[2][m];
        double th = g->hbar * k2 * tau / (2.0 * g->mass);
        psi[(i * ny + j) * nz + m] *= cos(th) - I * sin(th);
      }
  for (int d = 0; d < 3; ++d) free(k[d]);
  return orc_fftn(g, psi, 1);
}

/* nsteps steps from t_n = t0 + n dt, n = n0, n0+1, ... (time by
 * multiplication, never by accumulation).  No two half steps are merged.
 *
 * ORC_ORDER_VKV: V half at t_n, full kinetic step, V half at t_{n+1}.  This
 *   is the Strang splitting with the potential integral of eq. short-time
 *   taken by the trapezoid rule; it is second order like eq. splitop.
 * ORC_ORDER_KVK: eq. splitop as printed -- kinetic half, potential at the
 *   midpoint t_n + dt/2 over a full dt, kinetic half. */
int orc_propagate(const orc_grid *g, const orc_pot *p, double complex *psi, double t0,
                  int64_t n0, int64_t nsteps, int order) {
  if (!grid_ok(g) || nsteps < 0 || (order != ORC_ORDER_VKV && order != ORC_ORDER_KVK))
    return ORC_EINVAL;
  double *V = (double *)malloc(sizeof(double) * (size_t)grid_size(g));
  if (!V) return ORC_ENOMEM;
  int rc = ORC_OK;
  double dt = g->dt;
  for (int64_t s = 0; s < nsteps && !rc; ++s) {
    int64_t n = n0 + s;
    double tn = t0 + (double)n * dt;
    double tn1 = t0 + (double)(n + 1) * dt;
    if (order == ORC_ORDER_VKV) {
      rc = apply_potential_phase(g, p, psi, tn, 0.5 * dt, V);
      if (!rc) rc = apply_kinetic(g, psi, dt);
      if (!rc) rc = apply_potential_phase(g, p, psi, tn1, 0.5 * dt, V);
    } else {
      double tmid = t0 + ((double)n + 0.5) * dt;
      rc = apply_kinetic(g, psi, 0.5 * dt);
      if (!rc) rc = apply_potential_phase(g, p, psi, tmid, dt, V);
      if (!rc) rc = apply_kinetic(g, psi, 0.5 * dt);
    }
  }
  free(V);
  return rc;
}

/* ---- observables (Section 3.2 utility functions; Table 3) ------------- */

/* out = {norm, <x>, <y>, <z>, <x^2>, <y^2>, <z^2>, E} with the integrals of
 * `norm` and `expectation1D` taken by the rectangle rule over the periodic
 * cell (sum f dV), and E = <psi|K + V(t)|psi> with the kinetic part taken
 * spectrally: (dV/N) sum_k (hbar^2 |k|^2 / 2m) |F psi|_k^2.  The moments
 * are not divided by the norm (expectation1D does not normalise). */
int orc_observables(const orc_grid *g, const orc_pot *p, const double complex *psi, double t,
                    double out[8]) {
  if (!grid_ok(g)) return ORC_EINVAL;
  int64_t nx = g->n[0], ny = g->n[1], nz = g->n[2], N = grid_size(g);
  double dV = 1.0;
  for (int d = 0; d < g->ndim; ++d) dV *= spacing(g, d);
  double *x[3], *k[3];
  for (int d = 0; d < 3; ++d) {
    x[d] = (double *)malloc(sizeof(double) * (size_t)g->n[d]);
    k[d] = (double *)malloc(sizeof(double) * (size_t)g->n[d]);
    if (!x[d] || !k[d]) return ORC_ENOMEM;
    orc_coords(g, d, x[d]);
    orc_wavenumbers(g, d, k[d]);
  }
  double *V = (double *)malloc(sizeof(double) * (size_t)N);
  double complex *ph = (double complex *)malloc(sizeof(double complex) * (size_t)N);
  if (!V || !ph) return ORC_ENOMEM;
  orc_potential(g, p, t, V);
  memcpy(ph, psi, sizeof(double complex) * (size_t)N);
  orc_fftn(g, ph, -1);
  double s0 = 0, s1[3] = {0, 0, 0}, s2[3] = {0, 0, 0}, sv = 0, sk = 0;
  for (int64_t i = 0; i < nx; ++i)
    for (int64_t j = 0; j < ny; ++j)
      for (int64_t m = 0; m < nz; ++m) {
        int64_t idx = (i * ny + j) * nz + m;
        double r = creal(psi[idx]), q = cimag(psi[idx]);
        double w = r * r + q * q;
        double xs[3] = {x[0][i], x[1][j], x[2][m]};
        s0 += w;
        for (int d = 0; d < 3; ++d) {
          s1[d] += xs[d] * w;
          s2[d] += xs[d] * xs[d] * w;
        }
        sv += V[idx] * w;
        double kr = creal(ph[idx]), kq = cimag(ph[idx]);
        double k2 = k[0][i] * k[0][i] + k[1][j] * k[1][j] + k[2][m] * k[2][m];
        sk += g->hbar * g->hbar * k2 / (2.0 * g->mass) * (kr * kr + kq * kq);
      }
  out[0] = sqrt(s0 * dV);
  for (int d = 0; d < 3; ++d) {
    out[1 + d] = (d < g->ndim) ? s1[d] * dV : 0.0;
    out[4 + d] = (d < g->ndim) ? s2[d] * dV : 0.0;
  }
  out[7] = sk * dV / (double)N + sv * dV;
  for (int d = 0; d < 3; ++d) {
    free(x[d]);
    free(k[d]);
  }
  free(V);
  free(ph);
  return ORC_OK;
}

/* <f1|f2> = sum conj(f1) f2 dV (the utility `integrate3D`, Section 3.2). */
int orc_inner(const orc_grid *g, const double complex *f1, const double complex *f2,
              double out[2]) {
  if (!grid_ok(g)) return ORC_EINVAL;
  double dV = 1.0;
  for (int d = 0; d < g->ndim; ++d) dV *= spacing(g, d);
  double complex acc = 0.0;
  int64_t N = grid_size(g);
  for (int64_t i = 0; i < N; ++i) acc += conj(f1[i]) * f2[i];
  out[0] = creal(acc) * dV;
  out[1] = cimag(acc) * dV;
  return ORC_OK;
}
