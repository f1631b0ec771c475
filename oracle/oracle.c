/*
 * Plain double-precision CPU oracle for the spatiotemporal Hawkes
 * log-likelihood and its gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; it exists so the GPU library can be checked against a slow,
 * obviously correct evaluation of the paper's definitions.  It shares no code,
 * header or constant with the HIP library.
 *
 * Model (Holbrook, Ji & Suchard, arXiv 2010.02994, Sec. 2.1):
 *   rate            lambda(x,t) = mu(x,t) + xi(x,t)
 *   self-excitation xi(x,t) = theta*omega/h^D * sum_{t_n < t} exp(-omega (t-t_n)) phi((x-x_n)/h)
 *   background      mu(x,t) = mu0/(tau_x^D tau_t) * sum_n phi((x-x_n)/tau_x) phi((t-t_n)/tau_t) I[t != t_n]
 *   phi is the standard normal density in as many dimensions as its argument.
 *   compensator     Lambda_n = mu0 [Phi((t_N-t_n)/tau_t) - Phi(-t_n/tau_t)] + theta [1 - exp(-omega (t_N-t_n))]
 *   log-likelihood  ell = sum_n log lambda_n - sum_n Lambda_n          (eq. "likelihood")
 *   with lambda_n = sum_{n'} (mu_{nn'} + xi_{nn'}) the pair form of the same equation.
 *
 * Location gradient (App. A):
 *   d ell/d x_n = sum_{n'} [ (mu_{nn'}/lambda_n + mu_{n'n}/lambda_{n'}) / tau_x^2
 *                          + (xi_{nn'}/lambda_n + xi_{n'n}/lambda_{n'}) / h^2 ] (x_{n'} - x_n)
 *
 * Parameter gradient: not printed in the paper; obtained by differentiating
 * the pair terms and the compensator above term by term (the formulas are in
 * the comment of event_param_terms below).
 *
 * Readings where the paper is silent (each listed in the design notes):
 *  - t_N is the largest event time; the time integral runs over [0, t_N].
 *  - the spatial integral runs over all of R^D (no edge correction).
 *  - the background pair is excluded exactly when t_n == t_{n'}; the
 *    self-excitation pair needs t_{n'} < t_n strictly.  Input order is free.
 *  - parameter order in theta6 is (mu0, tau_x, tau_t, theta, omega, h), i.e.
 *    the library's (mu, h, tau, theta, omega, xi).
 *
 * Every sum over events uses Neumaier's compensated summation so the oracle's
 * own rounding stays far below the 1e-10 parity bar.  Rows are independent:
 * built with -fopenmp the row loops run in parallel and give bitwise the same
 * result as the single-threaded build.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ZERORATE (-4)

typedef struct { double s, c; } ksum;   /* Neumaier running sum */

static void ks_add(ksum* k, double v) {
  double t = k->s + v;
  if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
  else k->c += (v - t) + k->s;
  k->s = t;
}
static double ks_val(const ksum* k) { return k->s + k->c; }

static const double TWO_PI = 6.283185307179586476925286766559;

/* standard normal cdf written from its definition through erfc */
static double std_normal_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }
static double std_normal_pdf(double z) { return exp(-0.5 * z * z) / sqrt(TWO_PI); }

typedef struct {
  double mu0, tau_x, tau_t, theta, omega, h;
  double cbg_unit;   /* (2pi)^{-(D+1)/2} tau_x^{-D} tau_t^{-1}: background pair weight per unit mu0 */
  double cse_unit;   /* omega (2pi)^{-D/2} h^{-D}: self-excitation pair weight per unit theta */
  int d;
} model;

static int make_model(const double* th, int d, model* m) {
  for (int k = 0; k < 6; ++k) if (!isfinite(th[k])) return ORACLE_EINVAL;
  m->mu0 = th[0]; m->tau_x = th[1]; m->tau_t = th[2]; m->theta = th[3]; m->omega = th[4]; m->h = th[5];
  if (!(m->tau_x > 0) || !(m->tau_t > 0) || !(m->omega > 0) || !(m->h > 0)) return ORACLE_EINVAL;
  if (m->mu0 < 0 || m->theta < 0 || (m->mu0 == 0 && m->theta == 0)) return ORACLE_EINVAL;
  m->d = d;
  m->cbg_unit = pow(TWO_PI, -0.5 * (d + 1)) * pow(m->tau_x, -d) / m->tau_t;
  m->cse_unit = m->omega * pow(TWO_PI, -0.5 * d) * pow(m->h, -d);
  return ORACLE_OK;
}

/* Unweighted pair terms for the ordered pair (n, n'): the background kernel
 * value per unit mu0 and the self-excitation value per unit theta that event
 * n' contributes to the rate at event n.  Also returns r^2 and dt = t_n - t_n'. */
static void pair_terms(const model* m, const double* xn, const double* xm, double tn, double tm,
                       double* bg, double* se, double* r2_out, double* dt_out) {
  double r2 = 0.0;
  for (int k = 0; k < m->d; ++k) { double dx = xn[k] - xm[k]; r2 += dx * dx; }
  double dt = tn - tm;
  *bg = 0.0; *se = 0.0;
  if (dt != 0.0)
    *bg = m->cbg_unit * exp(-r2 / (2.0 * m->tau_x * m->tau_x) - dt * dt / (2.0 * m->tau_t * m->tau_t));
  if (dt > 0.0)
    *se = m->cse_unit * exp(-m->omega * dt - r2 / (2.0 * m->h * m->h));
  *r2_out = r2; *dt_out = dt;
}

/* Row sums for event n.  out6 = (K, R, U, J, V, W) with
 *   K = sum bg,  R = sum bg r^2,  U = sum bg dt^2,  J = sum se,  V = sum se r^2,  W = sum se dt
 * (unweighted: the weighted sums of the parameter-gradient formulas are
 *  M = mu0 K, A = mu0 R, B = mu0 U, S = theta J, P = theta V, Q = theta W). */
static void row_sums(const model* m, const double* x, const double* t, int64_t n, int64_t i, double* out6) {
  ksum acc[6];
  memset(acc, 0, sizeof(acc));
  const int d = m->d;
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    double bg, se, r2, dt;
    pair_terms(m, x + i * d, x + j * d, t[i], t[j], &bg, &se, &r2, &dt);
    if (bg != 0.0) { ks_add(&acc[0], bg); ks_add(&acc[1], bg * r2); ks_add(&acc[2], bg * dt * dt); }
    if (se != 0.0) { ks_add(&acc[3], se); ks_add(&acc[4], se * r2); ks_add(&acc[5], se * dt); }
  }
  for (int k = 0; k < 6; ++k) out6[k] = ks_val(&acc[k]);
}

static double row_rate(const model* m, const double* s6) { return m->mu0 * s6[0] + m->theta * s6[3]; }

/* lambda_n (and optionally the six row sums) for every event. */
int oracle_rates(const double* x, const double* t, int64_t n, int d, const double* theta6,
                 double* lam, double* sums6) {
  model m;
  if (n < 1 || d < 1 || !x || !t || !lam) return ORACLE_EINVAL;
  if (make_model(theta6, d, &m) != ORACLE_OK) return ORACLE_EINVAL;
  int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
  for (i = 0; i < n; ++i) {
    double s6[6];
    row_sums(&m, x, t, n, i, s6);
    lam[i] = row_rate(&m, s6);
    if (sums6) memcpy(sums6 + 6 * i, s6, sizeof(s6));
  }
  return ORACLE_OK;
}

/* The rates (Sec. 2.1) of the events listed in rows[], and their unweighted
 * row sums if sums6 is not NULL: the same per-event sums as oracle_rates,
 * O(n) work per listed event, for spot checks of inputs too large for the
 * full evaluation.  Every listed index must lie in [0, n). */
int oracle_rate_rows(const double* x, const double* t, int64_t n, int d, const double* theta6,
                     const int64_t* rows, int64_t nrows, double* lam, double* sums6) {
  model m;
  if (n < 1 || d < 1 || !x || !t || !rows || !lam || nrows < 0) return ORACLE_EINVAL;
  if (make_model(theta6, d, &m) != ORACLE_OK) return ORACLE_EINVAL;
  for (int64_t r = 0; r < nrows; ++r)
    if (rows[r] < 0 || rows[r] >= n) return ORACLE_EINVAL;
  int64_t r;
#pragma omp parallel for schedule(dynamic, 1)
  for (r = 0; r < nrows; ++r) {
    double s6[6];
    row_sums(&m, x, t, n, rows[r], s6);
    lam[r] = row_rate(&m, s6);
    if (sums6) memcpy(sums6 + 6 * r, s6, sizeof(s6));
  }
  return ORACLE_OK;
}

/* Location gradient rows (App. A) for the events listed in rows[], given the
 * rates lam[] of all events.  A partner whose three pair terms are exactly
 * zero adds exactly zero, so its rate is not needed beyond being finite.
 * scale (nrows, or NULL) receives each row's sum of the magnitudes of its
 * pair contributions, sum_{n'} |c_{nn'}| |x_{n'} - x_n|: the size against
 * which the rounding of any evaluation of that row is measured. */
int oracle_grad_rows_scaled(const double* x, const double* t, int64_t n, int d, const double* theta6,
                            const double* lam, const int64_t* rows, int64_t nrows, double* out, double* scale) {
  model m;
  if (n < 1 || d < 1 || d > 64 || !x || !t || !lam || !rows || !out) return ORACLE_EINVAL;
  if (make_model(theta6, d, &m) != ORACLE_OK) return ORACLE_EINVAL;
  const double itx2 = 1.0 / (m.tau_x * m.tau_x), ih2 = 1.0 / (m.h * m.h);
  int64_t r;
#pragma omp parallel for schedule(dynamic, 4)
  for (r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    ksum g[64], sc;
    memset(g, 0, sizeof(ksum) * d);
    memset(&sc, 0, sizeof(sc));
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double bg_ij, se_ij, se_ji, r2, dt, dummy_bg, dummy_r2, dummy_dt;
      pair_terms(&m, x + i * d, x + j * d, t[i], t[j], &bg_ij, &se_ij, &r2, &dt);
      pair_terms(&m, x + j * d, x + i * d, t[j], t[i], &dummy_bg, &se_ji, &dummy_r2, &dummy_dt);
      const double mu_ij = m.mu0 * bg_ij;             /* mu_{nn'} = mu_{n'n} */
      const double xi_ij = m.theta * se_ij;           /* from n' to n */
      const double xi_ji = m.theta * se_ji;           /* from n to n' */
      if (mu_ij == 0.0 && xi_ij == 0.0 && xi_ji == 0.0) continue;
      const double coef = (mu_ij / lam[i] + mu_ij / lam[j]) * itx2 + (xi_ij / lam[i] + xi_ji / lam[j]) * ih2;
      for (int k = 0; k < d; ++k) ks_add(&g[k], coef * (x[j * d + k] - x[i * d + k]));
      if (scale) ks_add(&sc, fabs(coef) * sqrt(r2));
    }
    for (int k = 0; k < d; ++k) out[r * d + k] = ks_val(&g[k]);
    if (scale) scale[r] = ks_val(&sc);
  }
  return ORACLE_OK;
}

int oracle_grad_rows(const double* x, const double* t, int64_t n, int d, const double* theta6,
                     const double* lam, const int64_t* rows, int64_t nrows, double* out) {
  return oracle_grad_rows_scaled(x, t, n, d, theta6, lam, rows, nrows, out, NULL);
}

/* Compensator terms per event: Lambda_n, and the pieces the parameter
 * gradient needs.  T is the largest event time (the paper's t_N). */
static void compensator(const model* m, double T, double tn, double* Lam, double* cdf_diff,
                        double* one_minus_decay, double* dtau, double* domega) {
  const double a = (T - tn) / m->tau_t, b = -tn / m->tau_t;
  *cdf_diff = std_normal_cdf(a) - std_normal_cdf(b);
  *one_minus_decay = 1.0 - exp(-m->omega * (T - tn));
  *Lam = m->mu0 * (*cdf_diff) + m->theta * (*one_minus_decay);
  /* d/d tau_t of mu0 [Phi(a) - Phi(b)] with a, b as above */
  *dtau = -m->mu0 / (m->tau_t * m->tau_t) * ((T - tn) * std_normal_pdf(a) + tn * std_normal_pdf(-b));
  /* d/d omega of theta [1 - exp(-omega (T - t_n))] */
  *domega = m->theta * (T - tn) * exp(-m->omega * (T - tn));
}

/* Event n's share of each parameter derivative of ell (the summands of the
 * parameter gradient), from its six unweighted row sums s = (K, R, U, J, V, W)
 * and its rate lam; Lam receives its compensator term Lambda_n.  In the
 * notation M = mu0 K, A = mu0 R, B = mu0 U, S = theta J, P = theta V, Q = theta W:
 *   d/d mu0   : M_n/(mu0 lambda_n) - [Phi(a_n) - Phi(b_n)]
 *   d/d tau_x : (A_n/tau_x^3 - D M_n/tau_x)/lambda_n
 *   d/d tau_t : (B_n/tau_t^3 - M_n/tau_t)/lambda_n - d Lambda_n/d tau_t
 *   d/d theta : S_n/(theta lambda_n) - [1 - exp(-omega (T - t_n))]
 *   d/d omega : (S_n/omega - Q_n)/lambda_n - theta (T - t_n) exp(-omega (T - t_n))
 *   d/d h     : (P_n/h^3 - D S_n/h)/lambda_n
 * (a_n = (T - t_n)/tau_t, b_n = -t_n/tau_t), obtained by differentiating the
 * pair terms and the compensator of Sec. 2.1 term by term. */
static void event_param_terms(const model* m, double T, double tn, const double* s, double lam, double* Lam,
                              double* v6) {
  double cdf_diff, omd, dtau, domega;
  compensator(m, T, tn, Lam, &cdf_diff, &omd, &dtau, &domega);
  const double il = 1.0 / lam;
  const int d = m->d;
  v6[0] = s[0] * il - cdf_diff;
  v6[1] = m->mu0 * (s[1] / (m->tau_x * m->tau_x * m->tau_x) - d * s[0] / m->tau_x) * il;
  v6[2] = m->mu0 * (s[2] / (m->tau_t * m->tau_t * m->tau_t) - s[0] / m->tau_t) * il - dtau;
  v6[3] = s[3] * il - omd;
  v6[4] = m->theta * (s[3] / m->omega - s[5]) * il - domega;
  v6[5] = m->theta * (s[4] / (m->h * m->h * m->h) - d * s[3] / m->h) * il;
}

/* Log-likelihood, location gradient and parameter gradient.
 * grad_x (n*d) and grad_theta (6) may be NULL.  Returns ORACLE_ZERORATE (with
 * ll = -inf) if some lambda_n is zero. */
int oracle_loglik_grad(const double* x, const double* t, int64_t n, int d, const double* theta6,
                       double* ll, double* grad_x, double* grad_theta) {
  model m;
  if (n < 1 || d < 1 || d > 64 || !x || !t || !ll) return ORACLE_EINVAL;
  if (make_model(theta6, d, &m) != ORACLE_OK) return ORACLE_EINVAL;
  for (int64_t i = 0; i < n; ++i) if (!isfinite(t[i])) return ORACLE_EINVAL;
  for (int64_t i = 0; i < n * d; ++i) if (!isfinite(x[i])) return ORACLE_EINVAL;

  double* lam = (double*)malloc(sizeof(double) * n);
  double* s6 = (double*)malloc(sizeof(double) * 6 * n);
  if (!lam || !s6) { free(lam); free(s6); return ORACLE_EINVAL; }
  oracle_rates(x, t, n, d, theta6, lam, s6);

  double T = t[0];
  for (int64_t i = 1; i < n; ++i) if (t[i] > T) T = t[i];

  int zero = 0;
  for (int64_t i = 0; i < n; ++i) if (!(lam[i] > 0.0)) zero = 1;

  ksum sl, sL, gk[6];
  memset(&sl, 0, sizeof(sl)); memset(&sL, 0, sizeof(sL)); memset(gk, 0, sizeof(gk));
  for (int64_t i = 0; i < n; ++i) {
    double Lam, v6[6];
    event_param_terms(&m, T, t[i], s6 + 6 * i, lam[i], &Lam, v6);
    ks_add(&sl, log(lam[i]));
    ks_add(&sL, Lam);
    for (int k = 0; k < 6; ++k) ks_add(&gk[k], v6[k]);
  }
  *ll = zero ? -INFINITY : ks_val(&sl) - ks_val(&sL);
  if (grad_theta) for (int k = 0; k < 6; ++k) grad_theta[k] = zero ? NAN : ks_val(&gk[k]);

  if (grad_x) {
    if (zero) {
      for (int64_t i = 0; i < n * d; ++i) grad_x[i] = NAN;
    } else {
      int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * n);
      if (!rows) { free(lam); free(s6); return ORACLE_EINVAL; }
      for (int64_t i = 0; i < n; ++i) rows[i] = i;
      oracle_grad_rows(x, t, n, d, theta6, lam, rows, n, grad_x);
      free(rows);
    }
  }
  free(lam); free(s6);
  return zero ? ORACLE_ZERORATE : ORACLE_OK;
}

/* log lambda_n for every event in the log domain, exact also where lambda_n
 * underflows double precision: each weighted pair term of Sec. 2.1 is kept as
 * its natural logarithm,
 *   log mu_{nn'} = log(mu0 (2 pi)^{-(D+1)/2} tau_x^{-D} tau_t^{-1}) - r^2/(2 tau_x^2) - dt^2/(2 tau_t^2)   (dt != 0)
 *   log xi_{nn'} = log(theta omega (2 pi)^{-D/2} h^{-D}) - omega dt - r^2/(2 h^2)                          (dt > 0)
 * and the row is summed relative to its largest term m_n:
 *   log lambda_n = m_n + log sum exp(log term - m_n).
 * max_log_term (or NULL) receives m_n; a row with no active pair gets -inf
 * for both.  A zero weight (mu0 = 0 or theta = 0) contributes no terms. */
int oracle_log_rates(const double* x, const double* t, int64_t n, int d, const double* theta6, double* log_lam,
                     double* max_log_term) {
  model m;
  if (n < 1 || d < 1 || !x || !t || !log_lam) return ORACLE_EINVAL;
  if (make_model(theta6, d, &m) != ORACLE_OK) return ORACLE_EINVAL;
  const double lbg = m.mu0 > 0 ? log(m.mu0 * m.cbg_unit) : -INFINITY;
  const double lse = m.theta > 0 ? log(m.theta * m.cse_unit) : -INFINITY;
  int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
  for (i = 0; i < n; ++i) {
    /* first sweep: the largest log term of the row */
    double mx = -INFINITY;
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double r2 = 0.0;
      for (int k = 0; k < d; ++k) { const double dx = x[i * d + k] - x[j * d + k]; r2 += dx * dx; }
      const double dt = t[i] - t[j];
      if (dt != 0.0) {
        const double e = lbg - r2 / (2.0 * m.tau_x * m.tau_x) - dt * dt / (2.0 * m.tau_t * m.tau_t);
        if (e > mx) mx = e;
      }
      if (dt > 0.0) {
        const double e = lse - m.omega * dt - r2 / (2.0 * m.h * m.h);
        if (e > mx) mx = e;
      }
    }
    if (max_log_term) max_log_term[i] = mx;
    if (mx == -INFINITY) { log_lam[i] = -INFINITY; continue; }
    /* second sweep: the terms relative to the largest one */
    ksum acc;
    memset(&acc, 0, sizeof(acc));
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      double r2 = 0.0;
      for (int k = 0; k < d; ++k) { const double dx = x[i * d + k] - x[j * d + k]; r2 += dx * dx; }
      const double dt = t[i] - t[j];
      if (dt != 0.0 && lbg > -INFINITY)
        ks_add(&acc, exp(lbg - r2 / (2.0 * m.tau_x * m.tau_x) - dt * dt / (2.0 * m.tau_t * m.tau_t) - mx));
      if (dt > 0.0 && lse > -INFINITY) ks_add(&acc, exp(lse - m.omega * dt - r2 / (2.0 * m.h * m.h) - mx));
    }
    log_lam[i] = mx + log(ks_val(&acc));
  }
  return ORACLE_OK;
}

/* The parameter gradient's summands over events (see event_param_terms):
 * sum6 receives sum_n v_k(n), the parameter gradient itself, and abs6 the
 * cancellation scale sum_n |v_k(n)| against which the rounding of any
 * evaluation of d ell/d Theta_k is measured.  Needs every lambda_n > 0. */
int oracle_param_terms(const double* x, const double* t, int64_t n, int d, const double* theta6, double* sum6,
                       double* abs6) {
  model m;
  if (n < 1 || d < 1 || !x || !t || !sum6 || !abs6) return ORACLE_EINVAL;
  if (make_model(theta6, d, &m) != ORACLE_OK) return ORACLE_EINVAL;
  double* lam = (double*)malloc(sizeof(double) * n);
  double* s6 = (double*)malloc(sizeof(double) * 6 * n);
  if (!lam || !s6) { free(lam); free(s6); return ORACLE_EINVAL; }
  oracle_rates(x, t, n, d, theta6, lam, s6);
  double T = t[0];
  for (int64_t i = 1; i < n; ++i) if (t[i] > T) T = t[i];
  int zero = 0;
  ksum sg[6], sa[6];
  memset(sg, 0, sizeof(sg)); memset(sa, 0, sizeof(sa));
  for (int64_t i = 0; i < n; ++i) {
    if (!(lam[i] > 0.0)) { zero = 1; break; }
    double Lam, v6[6];
    event_param_terms(&m, T, t[i], s6 + 6 * i, lam[i], &Lam, v6);
    for (int k = 0; k < 6; ++k) { ks_add(&sg[k], v6[k]); ks_add(&sa[k], fabs(v6[k])); }
  }
  for (int k = 0; k < 6; ++k) { sum6[k] = zero ? NAN : ks_val(&sg[k]); abs6[k] = zero ? NAN : ks_val(&sa[k]); }
  free(lam); free(s6);
  return zero ? ORACLE_ZERORATE : ORACLE_OK;
}

/* ------------------------------------------------------------------------
 * Bayesian multidimensional scaling (Sec. 2.2.3, eq. "bmdsLikelihood"):
 * observed dissimilarities delta_{nn'} (n > n') are independent normals with
 * mean d_{nn'} = |x_n - x_n'| and variance sigma^2, truncated to delta > 0:
 *   ell = -(M/2) log sigma^2 - sum_{n>n'} [ (delta - d)^2 / (2 sigma^2) + log Phi(d / sigma) ]
 * with M the number of pairs (the paper's exponent N(1-N)/4 of sigma^2 is -M/2
 * when every pair is observed).  A NaN delta marks a pair with no observation:
 * it contributes nothing and is not counted in M.
 * Derivatives, differentiating the summand term by term (z = d / sigma,
 * rho = phi(z) / Phi(z)):
 *   d ell/d x_n   = sum_{n' != n} [ (delta - d)/sigma^2 - rho/sigma ] (x_n - x_n') / d
 *   d ell/d sigma = -M/sigma + sum [ (delta - d)^2 / sigma^3 + rho z / sigma ]
 * A coincident pair (d = 0) contributes no direction to d ell/d x.
 * out3 = (ell, d ell/d sigma, M).  Status: EINVAL for a negative or infinite
 * delta, non-finite x or sigma <= 0. */
static void bmds_pair(const double* xi, const double* xj, int d, double delta, double sigma, double* term,
                      double* dsig, double* coef, double* dist) {
  double r2 = 0.0;
  for (int k = 0; k < d; ++k) { double v = xi[k] - xj[k]; r2 += v * v; }
  const double dd = sqrt(r2);
  const double z = dd / sigma;
  const double Phi = std_normal_cdf(z);
  const double rho = std_normal_pdf(z) / Phi;
  const double res = delta - dd;
  *term = -res * res / (2.0 * sigma * sigma) - log(Phi);
  *dsig = res * res / (sigma * sigma * sigma) + rho * z / sigma;
  *coef = dd > 0.0 ? (res / (sigma * sigma) - rho / sigma) / dd : 0.0;
  *dist = dd;
}

int oracle_bmds(const double* x, const double* delta, int64_t n, int d, double sigma, double* out3,
                double* grad_x) {
  if (n < 1 || d < 1 || d > 64 || !x || !delta || !out3) return ORACLE_EINVAL;
  if (!(sigma > 0.0) || !isfinite(sigma)) return ORACLE_EINVAL;
  for (int64_t i = 0; i < n * d; ++i) if (!isfinite(x[i])) return ORACLE_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < i; ++j) {
      const double v = delta[i * n + j];
      if (!isnan(v) && (v < 0.0 || isinf(v))) return ORACLE_EINVAL;
    }
  ksum sl, sd, sm;
  memset(&sl, 0, sizeof(sl)); memset(&sd, 0, sizeof(sd)); memset(&sm, 0, sizeof(sm));
  for (int64_t i = 0; i < n; ++i)
    for (int64_t j = 0; j < i; ++j) {
      const double v = delta[i * n + j];
      if (isnan(v)) continue;
      double term, dsig, coef, dist;
      bmds_pair(x + i * d, x + j * d, d, v, sigma, &term, &dsig, &coef, &dist);
      ks_add(&sl, term);
      ks_add(&sd, dsig);
      ks_add(&sm, 1.0);
    }
  const double M = ks_val(&sm);
  out3[0] = -0.5 * M * log(sigma * sigma) + ks_val(&sl);
  out3[1] = -M / sigma + ks_val(&sd);
  out3[2] = M;
  if (grad_x) {
    int64_t i;
#pragma omp parallel for schedule(dynamic, 16)
    for (i = 0; i < n; ++i) {
      ksum g[64];
      memset(g, 0, sizeof(ksum) * d);
      for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        const double v = i > j ? delta[i * n + j] : delta[j * n + i];
        if (isnan(v)) continue;
        double term, dsig, coef, dist;
        bmds_pair(x + i * d, x + j * d, d, v, sigma, &term, &dsig, &coef, &dist);
        for (int k = 0; k < d; ++k) ks_add(&g[k], coef * (x[i * d + k] - x[j * d + k]));
      }
      for (int k = 0; k < d; ++k) grad_x[i * d + k] = ks_val(&g[k]);
    }
  }
  return ORACLE_OK;
}
