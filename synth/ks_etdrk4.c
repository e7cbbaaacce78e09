/*
 * Kuramoto-Sivashinsky trajectory generator (input data only; no part of the
 * decomposition method lives here).
 *
 * Equation: u_t = -u u_x - u_xx - u_xxxx on a periodic domain of length L
 * (the paper's Application section, eq. ks).  Fourier pseudospectral
 * discretisation with M = 64 grid points, i.e. modes |k| <= 31 kept (the
 * Nyquist mode is held at zero); the quadratic term is evaluated alias-free on
 * a padded grid of MP = 96 points (the 3/2 rule: products of two fields with
 * |k| <= 31 have |k| <= 62, and 62 - 96 = -34 lies outside the kept band, so
 * the retained modes are exact).  Time stepping is ETDRK4 (Cox & Matthews
 * 2002) with the phi-function coefficients evaluated by the contour-integral
 * average of Kassam & Trefethen (2005), SIAM J. Sci. Comput. 26(4).
 *
 * Mode k = 0 carries the spatial mean, which the equation conserves and the
 * nonlinear term never feeds; the initial condition has its mean removed, so
 * only modes k = 1..31 are stored (real and imaginary parts).
 *
 * The discrete transforms are written out as small dense cosine/sine sums:
 * with 31 modes and 96 points that is ~6k multiply-adds per transform, laid
 * out as axpy sweeps so the compiler vectorises them.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define KS_M 64
#define KS_K 31  /* stored modes k = 1..31 */
#define KS_MP 96 /* padded grid for the quadratic term */
#define KS_NC 64 /* contour points for the phi functions */

typedef struct {
  double inv_c[KS_K][KS_MP]; /* u(y_j) = sum_k inv_c[k][j]*vr_k + inv_s[k][j]*vi_k */
  double inv_s[KS_K][KS_MP];
  double fwd_c[KS_MP][KS_K]; /* (w)^_k real part = sum_j fwd_c[j][k] w_j */
  double fwd_s[KS_MP][KS_K]; /* imaginary part = sum_j fwd_s[j][k] w_j */
  double out_c[KS_K][KS_M];  /* samples on the 64-point grid */
  double out_s[KS_K][KS_M];
  double q[KS_K];            /* wave numbers 2*pi*k/L */
  double E[KS_K], E2[KS_K], Q[KS_K], f1[KS_K], f2[KS_K], f3[KS_K];
} ks_plan;

static void ks_setup(ks_plan* p, double L, double h) {
  const double twopi = 2.0 * M_PI;
  for (int k = 0; k < KS_K; ++k) {
    int kk = k + 1;
    for (int j = 0; j < KS_MP; ++j) {
      double a = twopi * kk * j / KS_MP;
      p->inv_c[k][j] = 2.0 * cos(a);
      p->inv_s[k][j] = -2.0 * sin(a);
      p->fwd_c[j][k] = cos(a) / KS_MP;
      p->fwd_s[j][k] = -sin(a) / KS_MP;
    }
    for (int j = 0; j < KS_M; ++j) {
      double a = twopi * kk * j / KS_M;
      p->out_c[k][j] = 2.0 * cos(a);
      p->out_s[k][j] = -2.0 * sin(a);
    }
    double q = twopi * kk / L;
    double lin = q * q - q * q * q * q; /* Fourier symbol of -d_xx - d_xxxx */
    p->q[k] = q;
    p->E[k] = exp(h * lin);
    p->E2[k] = exp(h * lin / 2.0);
    double complex sQ = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int j = 0; j < KS_NC; ++j) {
      double complex z = h * lin + cexp(I * twopi * (j + 0.5) / KS_NC);
      double complex ez = cexp(z), ez2 = cexp(z / 2.0);
      sQ += (ez2 - 1.0) / z;
      s1 += (-4.0 - z + ez * (4.0 - 3.0 * z + z * z)) / (z * z * z);
      s2 += (2.0 + z + ez * (-2.0 + z)) / (z * z * z);
      s3 += (-4.0 - 3.0 * z - z * z + ez * (4.0 - z)) / (z * z * z);
    }
    p->Q[k] = h * creal(sQ) / KS_NC;
    p->f1[k] = h * creal(s1) / KS_NC;
    p->f2[k] = h * creal(s2) / KS_NC;
    p->f3[k] = h * creal(s3) / KS_NC;
  }
}

/* N(v)_k = -(1/2) i q_k (u^2)^_k, evaluated alias-free on the padded grid. */
static void ks_nonlin(const ks_plan* p, const double* vr, const double* vi,
                      double* nr, double* ni) {
  double u[KS_MP];
  double wr[KS_K], wi[KS_K];
  memset(u, 0, sizeof u);
  for (int k = 0; k < KS_K; ++k) {
    const double a = vr[k], b = vi[k];
    for (int j = 0; j < KS_MP; ++j) u[j] += a * p->inv_c[k][j] + b * p->inv_s[k][j];
  }
  memset(wr, 0, sizeof wr);
  memset(wi, 0, sizeof wi);
  for (int j = 0; j < KS_MP; ++j) {
    const double w = u[j] * u[j];
    for (int k = 0; k < KS_K; ++k) {
      wr[k] += w * p->fwd_c[j][k];
      wi[k] += w * p->fwd_s[j][k];
    }
  }
  for (int k = 0; k < KS_K; ++k) {
    /* -0.5 i q (wr + i wi) = 0.5 q wi - 0.5 i q wr */
    nr[k] = 0.5 * p->q[k] * wi[k];
    ni[k] = -0.5 * p->q[k] * wr[k];
  }
}

static void ks_step(const ks_plan* p, double* vr, double* vi) {
  double Nvr[KS_K], Nvi[KS_K], ar[KS_K], ai[KS_K], Nar[KS_K], Nai[KS_K];
  double br[KS_K], bi[KS_K], Nbr[KS_K], Nbi[KS_K], cr[KS_K], ci[KS_K], Ncr[KS_K], Nci[KS_K];
  ks_nonlin(p, vr, vi, Nvr, Nvi);
  for (int k = 0; k < KS_K; ++k) {
    ar[k] = p->E2[k] * vr[k] + p->Q[k] * Nvr[k];
    ai[k] = p->E2[k] * vi[k] + p->Q[k] * Nvi[k];
  }
  ks_nonlin(p, ar, ai, Nar, Nai);
  for (int k = 0; k < KS_K; ++k) {
    br[k] = p->E2[k] * vr[k] + p->Q[k] * Nar[k];
    bi[k] = p->E2[k] * vi[k] + p->Q[k] * Nai[k];
  }
  ks_nonlin(p, br, bi, Nbr, Nbi);
  for (int k = 0; k < KS_K; ++k) {
    cr[k] = p->E2[k] * ar[k] + p->Q[k] * (2.0 * Nbr[k] - Nvr[k]);
    ci[k] = p->E2[k] * ai[k] + p->Q[k] * (2.0 * Nbi[k] - Nvi[k]);
  }
  ks_nonlin(p, cr, ci, Ncr, Nci);
  for (int k = 0; k < KS_K; ++k) {
    vr[k] = p->E[k] * vr[k] + Nvr[k] * p->f1[k] + 2.0 * (Nar[k] + Nbr[k]) * p->f2[k] + Ncr[k] * p->f3[k];
    vi[k] = p->E[k] * vi[k] + Nvi[k] * p->f1[k] + 2.0 * (Nai[k] + Nbi[k]) * p->f2[k] + Nci[k] * p->f3[k];
  }
}

static void ks_sample(const ks_plan* p, const double* vr, const double* vi, double* u) {
  memset(u, 0, KS_M * sizeof(double));
  for (int k = 0; k < KS_K; ++k)
    for (int j = 0; j < KS_M; ++j) u[j] += vr[k] * p->out_c[k][j] + vi[k] * p->out_s[k][j];
}

/*
 * Integrate from the 64-point initial field u0 (its mean is ignored), discard
 * `spinup` steps, then write `n_samples` snapshots, one every `every` steps,
 * the first one right after the spin-up.  out is n_samples x 64, row-major.
 * Returns 0 on success, -1 on bad arguments or allocation failure.
 */
static int ks_run(long n_samples, long spinup, long every, double dt, double L,
                  const double* u0, float* out32, double* out64) {
  if (n_samples < 0 || spinup < 0 || every < 1 || !(dt > 0) || !(L > 0) || !u0 ||
      (!out32 && !out64 && n_samples))
    return -1;
  ks_plan* p = (ks_plan*)malloc(sizeof(ks_plan));
  if (!p) return -1;
  ks_setup(p, L, dt);
  double vr[KS_K], vi[KS_K];
  for (int k = 0; k < KS_K; ++k) {
    double sr = 0, si = 0;
    for (int j = 0; j < KS_M; ++j) {
      double a = 2.0 * M_PI * (k + 1) * j / KS_M;
      sr += u0[j] * cos(a);
      si -= u0[j] * sin(a);
    }
    vr[k] = sr / KS_M;
    vi[k] = si / KS_M;
  }
  for (long s = 0; s < spinup; ++s) ks_step(p, vr, vi);
  for (long m = 0; m < n_samples; ++m) {
    if (m > 0)
      for (long s = 0; s < every; ++s) ks_step(p, vr, vi);
    double u[KS_M];
    ks_sample(p, vr, vi, u);
    for (int j = 0; j < KS_M; ++j) {
      if (out32) out32[m * KS_M + j] = (float)u[j];
      if (out64) out64[m * KS_M + j] = u[j];
    }
  }
  free(p);
  return 0;
}

int ks_generate(long n_samples, long spinup, long every, double dt, double L,
                const double* u0, float* out) {
  return ks_run(n_samples, spinup, every, dt, L, u0, out, 0);
}

/* Same trajectory with float64 snapshots (used to check the integrator). */
int ks_generate64(long n_samples, long spinup, long every, double dt, double L,
                  const double* u0, double* out) {
  return ks_run(n_samples, spinup, every, dt, L, u0, 0, out);
}
