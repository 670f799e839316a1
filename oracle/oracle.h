/*
 * oracle.h -- plain FP64 CPU reference of the split-operator time step
 * (Dion, Hashemloo, Rahali, "Program for quantum wave-packet dynamics with
 * time-dependent potentials", Comput. Phys. Commun.).
 *
 * TEST INFRASTRUCTURE ONLY.  This code is the slow, obviously correct
 * definition against which the GPU library is checked.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or constant with the GPU library.
 *
 * Conventions (each one is restated where it is used in oracle.c):
 *   - grid: half-open [lo, hi) per axis, spacing (hi - lo) / n, point
 *     x_i = lo + i * spacing (Section 2.1, eqs. grid and Deltax, with the
 *     paper's x_max read as the last point hi - spacing);
 *   - wave function: row-major psi[nx][ny][nz], z fastest, interleaved
 *     (re, im) doubles (the layout of the paper's psi[nx_local][ny][nz]);
 *   - 1D problems lie along x and 2D problems in the xy-plane; unused axes
 *     have n = 1 (Section 2.2);
 *   - forward DFT uses exp(-2 pi i j m / n) and is unnormalised; the inverse
 *     uses exp(+2 pi i j m / n) and divides by n.
 */
#ifndef WAVEPACKET_ORACLE_H
#define WAVEPACKET_ORACLE_H

#include <complex.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Time-dependent scalar f(t) used for every coefficient of the potential. */
enum {
  ORC_WAVE_CONST = 0,    /* A0                                              */
  ORC_WAVE_SIN = 1,      /* A0 + A1 sin(omega t + phase)                    */
  ORC_WAVE_COS = 2,      /* A0 + A1 cos(omega t + phase)                    */
  ORC_WAVE_GAUSS_COS = 3,/* A0 + A1 exp(-((t-tc)/tau)^2) cos(omega t+phase) */
  ORC_WAVE_SIN2_COS = 4  /* A0 + A1 sin^2(pi (t-ti)/(tf-ti)) cos(omega t +  */
                         /* phase) for ti <= t <= tf, A0 otherwise          */
};

enum { ORC_V0_NONE = 0, ORC_V0_SOFTCORE = 1, ORC_V0_MORSE = 2 };

/* Operator order of one step. */
enum {
  ORC_ORDER_VKV = 0, /* exp(-iV(t_n+1)dt/2h) F^-1 exp(-iK dt/h) F exp(-iV(t_n)dt/2h) */
  ORC_ORDER_KVK = 1  /* exp(-iK dt/2h) exp(-iV(t_n + dt/2) dt/h) exp(-iK dt/2h)      */
};

typedef struct {
  int32_t kind;
  double A0, A1, omega, phase, tc, tau, ti, tf;
} orc_wave;

typedef struct {
  int32_t ndim;
  int64_t n[3];
  double lo[3], hi[3];
  double mass, hbar, dt;
} orc_grid;

/* V(x,t) = c(t) + sum_d [a_d(t) x_d + b_d(t) x_d^2] + s(t) V0(x)
 *   V0 SOFTCORE: -Z / sqrt(r^2 + eps2),  par = {Z, eps2}
 *   V0 MORSE   : D (1 - exp(-a (x - xe)))^2 along x, par = {D, a, xe}   */
typedef struct {
  orc_wave a[3], b[3], c, s;
  int32_t v0_kind;
  double v0_par[4];
} orc_pot;

double orc_wave_eval(const orc_wave *w, double t);
int orc_coords(const orc_grid *g, int axis, double *out);
int orc_wavenumbers(const orc_grid *g, int axis, double *out);
int orc_potential(const orc_grid *g, const orc_pot *p, double t, double *V);

int orc_dft1d(int64_t n, const double complex *in, double complex *out, int dir);
int orc_fft1d(int64_t n, double complex *data, int dir);
int orc_fftn(const orc_grid *g, double complex *psi, int dir);

int orc_gaussian(const orc_grid *g, const double c[3], const double sigma[3],
                 const double k[3], double complex *psi);
int orc_propagate(const orc_grid *g, const orc_pot *p, double complex *psi,
                  double t0, int64_t n0, int64_t nsteps, int order);
int orc_observables(const orc_grid *g, const orc_pot *p,
                    const double complex *psi, double t, double out[8]);
int orc_inner(const orc_grid *g, const double complex *f1,
              const double complex *f2, double out[2]);
int orc_num_threads(void);

#ifdef __cplusplus
}
#endif
#endif
