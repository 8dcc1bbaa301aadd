/*
 * Driver for the sanitizer build of the CPU oracle (test infrastructure):
 * compiled together with oracle/h4_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitizers.py, it calls
 * every entry point of the oracle on small systems (with and without a
 * central particle, plain and compensated sums, index lists with repeats,
 * a short integration with block steps and dt_min clamps) and checks that
 * the results are finite and that the total momentum change of a full
 * force evaluation vanishes to rounding. Exit status 0 on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int or_max_threads(void);
int or_force(int64_t n, const double* m, const double* x, const double* v, double eps, double eps_bh,
             int64_t bh, int64_t n_act, const int64_t* idx, double* acc, double* jrk, int compensated,
             int nthreads);
int or_energy(int64_t n, const double* m, const double* x, const double* v, double eps, double eps_bh,
              int64_t bh, double* ekin, double* epot, double* epot_unsoft);
void or_predict(int64_t n, const double* x, const double* v, const double* a, const double* jk,
                const double* t_i, double t, double* xp, double* vp);
void or_hermite_derivs(const double* a0, const double* j0, const double* a1, const double* j1, double h,
                       double* a2, double* a3);
void or_correct(const double* xp, const double* vp, const double* a2, const double* a3, double h,
                double* x, double* v);
double or_dt_initial(const double* a, const double* jk, double eta);
double or_dt_aarseth(const double* a1, const double* j1, const double* a2, const double* a3, double h,
                     double eta);
double or_quantize(double dtstar, double dt_old, double t_new, double dt_max, double dt_min,
                   int64_t* clamps);
int or_init(int64_t n, const double* m, const double* x, const double* v, double eps, double eps_bh,
            int64_t bh, double eta, double dt_max, double dt_min, double* a, double* jk, double* t_i,
            double* dt_i, int64_t* clamps, int nthreads);
int64_t or_run(int64_t n, const double* m, double* x, double* v, double* a, double* jk, double* t_i,
               double* dt_i, double eps, double eps_bh, int64_t bh, double eta, double dt_max,
               double dt_min, double* t_now, double t_end, double e0, int64_t* stats, double* rows,
               int64_t max_rows, int nthreads);

static uint64_t lcg = 88172645463325252ULL;
static double uniform(void) {
  lcg = lcg * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

static int all_finite(const double* p, int64_t k) {
  for (int64_t q = 0; q < k; ++q)
    if (!isfinite(p[q])) return 0;
  return 1;
}

#define CHECK(cond, what)                      \
  do {                                         \
    if (!(cond)) {                             \
      fprintf(stderr, "FAILED: %s\n", what);   \
      return 1;                                \
    }                                          \
  } while (0)

static int run_case(int64_t n, int64_t bh) {
  const double eps = 1e-2, eps_bh = 1e-3, eta = 0.02, dt_max = 1.0 / 64, dt_min = 1.0 / 1048576;
  double* m = malloc(sizeof(double) * n);
  double* x = malloc(sizeof(double) * 3 * n);
  double* v = malloc(sizeof(double) * 3 * n);
  double* a = malloc(sizeof(double) * 3 * n);
  double* jk = malloc(sizeof(double) * 3 * n);
  double* ac = malloc(sizeof(double) * 3 * n);
  double* jc = malloc(sizeof(double) * 3 * n);
  double* xp = malloc(sizeof(double) * 3 * n);
  double* vp = malloc(sizeof(double) * 3 * n);
  double* t_i = malloc(sizeof(double) * n);
  double* dt_i = malloc(sizeof(double) * n);
  int64_t* idx = malloc(sizeof(int64_t) * n);
  double rows[8 * 8];
  if (!m || !x || !v || !a || !jk || !ac || !jc || !xp || !vp || !t_i || !dt_i || !idx) return 2;
  for (int64_t i = 0; i < n; ++i) {
    m[i] = 1.0 / (double)n;
    for (int d = 0; d < 3; ++d) {
      x[3 * i + d] = uniform() - 0.5;
      v[3 * i + d] = 0.3 * (uniform() - 0.5);
    }
    idx[i] = (i * 7) % n;
  }
  if (bh >= 0) m[bh] = 0.05;
  idx[n - 1] = idx[0];  // a repeated index

  CHECK(or_force(n, m, x, v, eps, eps_bh, bh, n, NULL, a, jk, 0, 1) == 0, "or_force plain");
  CHECK(or_force(n, m, x, v, eps, eps_bh, bh, n, idx, ac, jc, 1, 1) == 0, "or_force compensated");
  CHECK(all_finite(a, 3 * n) && all_finite(jk, 3 * n) && all_finite(ac, 3 * n) && all_finite(jc, 3 * n),
        "finite forces");
  for (int d = 0; d < 3; ++d) {
    double p = 0.0, s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      p += m[i] * a[3 * i + d];
      s += fabs(m[i] * a[3 * i + d]);
    }
    CHECK(fabs(p) <= 1e-12 * s, "momentum balance of the forces");
  }
  double ek, ep, eu;
  CHECK(or_energy(n, m, x, v, eps, eps_bh, bh, &ek, &ep, &eu) == 0 && isfinite(ek + ep + eu), "or_energy");

  for (int64_t i = 0; i < n; ++i) t_i[i] = 0.0;
  or_predict(n, x, v, a, jk, t_i, 1.0 / 128, xp, vp);
  CHECK(all_finite(xp, 3 * n) && all_finite(vp, 3 * n), "or_predict");
  double a2[3], a3[3], xc[3], vc[3];
  or_hermite_derivs(a, jk, a + 3, jk + 3, 1.0 / 256, a2, a3);
  or_correct(xp, vp, a2, a3, 1.0 / 256, xc, vc);
  CHECK(all_finite(xc, 3) && all_finite(vc, 3), "or_correct");
  int64_t clamps = 0;
  const double d0 = or_dt_initial(a, jk, eta);
  const double d1 = or_dt_aarseth(a, jk, a2, a3, 1.0 / 256, eta);
  CHECK(isfinite(d0) && d0 > 0 && isfinite(d1) && d1 > 0, "time-step criteria");
  CHECK(or_quantize(d1, 1.0 / 256, 1.0 / 128, dt_max, dt_min, &clamps) > 0, "or_quantize");
  CHECK(or_quantize(1e-30, 1.0 / 256, 1.0 / 128, dt_max, dt_min, &clamps) == dt_min && clamps == 1,
        "or_quantize clamp");

  clamps = 0;
  CHECK(or_init(n, m, x, v, eps, eps_bh, bh, eta, dt_max, dt_min, a, jk, t_i, dt_i, &clamps, 1) == 0,
        "or_init");
  double t_now = 0.0;
  int64_t stats[4] = {0, 0, 0, clamps};
  const int64_t nrows = or_run(n, m, x, v, a, jk, t_i, dt_i, eps, eps_bh, bh, eta, dt_max, dt_min, &t_now,
                               2 * dt_max, ek + ep, stats, rows, 8, 1);
  CHECK(nrows == 2 && t_now == 2 * dt_max && stats[0] > 0 && stats[1] >= n, "or_run");
  CHECK(all_finite(x, 3 * n) && all_finite(v, 3 * n) && all_finite(rows, 8 * nrows), "finite state");
  printf("n=%lld bh=%lld: block steps %lld, particle steps %lld, drift %.2e\n", (long long)n, (long long)bh,
         (long long)stats[0], (long long)stats[1], rows[8 * (nrows - 1) + 5]);
  free(m); free(x); free(v); free(a); free(jk); free(ac); free(jc); free(xp); free(vp);
  free(t_i); free(dt_i); free(idx);
  return 0;
}

int main(void) {
  CHECK(or_max_threads() >= 1, "or_max_threads");
  if (run_case(2, -1)) return 1;
  if (run_case(67, -1)) return 1;
  if (run_case(129, 5)) return 1;
  printf("sanitized oracle ok\n");
  return 0;
}
