/*
 * FP64 CPU oracle for the GraviDy Hermite-4 block-time-step integrator with
 * Plummer softening (arXiv:1702.00440).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may load, call or link
 * this file: it is used by the tests, by the smoke check and by the CPU
 * baseline leg of the benchmark. It shares no code, header or constant with the
 * HIP library; the two meet only at the seeded inputs.
 *
 * Plain, slow and obviously correct on purpose: double arithmetic compiled
 * without FMA contraction, every sum in ascending index order, the steps of
 * the method in the paper's order. Optional OpenMP splits independent i
 * particles over threads; each i's sum is still taken serially in j order, so
 * the result does not depend on the thread count.
 *
 * Readings of points the paper leaves open are marked READING and follow the
 * mathematics:
 *   - jerk: the exact time derivative of the softened acceleration, Eq. (3);
 *     the paper only warns that the Makino & Aarseth (1992) print of it has a
 *     sign typo in its second term (Sec. 2.4, footnote);
 *   - predictor / corrector / time-step criterion: the standard Hermite-4
 *     forms of Makino & Aarseth (1992), to which the paper defers (Sec. 2.1,
 *     Sec. 2.4, Sec. 3.2);
 *   - energy: the kinetic plus the softened potential, the quantity that the
 *     softened dynamics conserve (Eq. (2) prints the unsoftened one, which is
 *     also returned);
 *   - central massive particle (the paper's planned extension, Sec. 6): when
 *     bh >= 0, every pair that involves particle bh is softened with eps_bh
 *     instead of eps (symmetric, so Newton's third law still holds); bh < 0
 *     means no such particle.
 *
 * Array conventions: positions, velocities, accelerations and jerks are
 * row-major (n, 3) double arrays; index arrays are int64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2
#define OR_ESTATE -4

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Neumaier's compensated summation: running sum s with compensation c. */
static inline void neumaier_add(double* s, double* c, double x) {
  double t = *s + x;
  if (fabs(*s) >= fabs(x))
    *c += (*s - t) + x;
  else
    *c += (x - t) + *s;
  *s = t;
}

/* Squared softening of pair (i, j): eps_bh^2 when either is the central
 * particle bh, eps^2 otherwise. */
static inline double pair_eps2(int64_t i, int64_t j, double eps2, double eps2_bh, int64_t bh) {
  return (bh >= 0 && (i == bh || j == bh)) ? eps2_bh : eps2;
}

/*
 * Softened acceleration and jerk of particle i from all j != i.
 *
 * Acceleration, Eq. (3) with G = 1 (Sec. 3.1): a_i = sum_j m_j r / s^(3/2),
 * where r = x_j - x_i and s = |r|^2 + eps^2 (Eq. (1) and (3) write the same
 * sum with r_i - r_j and a leading minus sign).
 * Jerk (READING, see header): the time derivative of that sum along the
 * motion, d/dt [r / s^(3/2)] = w / s^(3/2) - 3 (r . w) r / s^(5/2), with
 * w = v_j - v_i. The j = i term is excluded as in Eq. (1).
 */
static void pair_sum(int64_t n, const double* m, const double* x, const double* v,
                     double eps2, double eps2_bh, int64_t bh, int64_t i, int compensated,
                     double* acc, double* jrk) {
  double s_acc[3] = {0, 0, 0}, c_acc[3] = {0, 0, 0};
  double s_jrk[3] = {0, 0, 0}, c_jrk[3] = {0, 0, 0};
  const double* xi = x + 3 * i;
  const double* vi = v + 3 * i;
  for (int64_t j = 0; j < n; ++j) {
    if (j == i) continue;
    double r[3], w[3];
    for (int d = 0; d < 3; ++d) {
      r[d] = x[3 * j + d] - xi[d];
      w[d] = v[3 * j + d] - vi[d];
    }
    double s = r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + pair_eps2(i, j, eps2, eps2_bh, bh);
    double s32 = s * sqrt(s);
    double s52 = s32 * s;
    double rw = r[0] * w[0] + r[1] * w[1] + r[2] * w[2];
    for (int d = 0; d < 3; ++d) {
      double ta = m[j] * r[d] / s32;
      double tj = m[j] * (w[d] / s32 - 3.0 * rw * r[d] / s52);
      if (compensated) {
        neumaier_add(&s_acc[d], &c_acc[d], ta);
        neumaier_add(&s_jrk[d], &c_jrk[d], tj);
      } else {
        s_acc[d] += ta;
        s_jrk[d] += tj;
      }
    }
  }
  for (int d = 0; d < 3; ++d) {
    acc[d] = s_acc[d] + c_acc[d];
    jrk[d] = s_jrk[d] + c_jrk[d];
  }
}

/*
 * Force (acceleration and jerk) of the listed i particles from all n
 * particles: the O(N_act * N) step of the integration (Sec. 2.4, step 7(c)ii;
 * Sec. 2.5). idx == NULL means every particle (the initial O(N^2) evaluation,
 * Sec. 2.4 step 3). compensated != 0 sums with Neumaier compensation, used as
 * a higher-accuracy reference; the plain mode is the definition itself.
 */
int or_force(int64_t n, const double* m, const double* x, const double* v, double eps,
             double eps_bh, int64_t bh, int64_t n_act, const int64_t* idx, double* acc,
             double* jrk, int compensated, int nthreads) {
  if (n < 1 || n_act < 0 || bh >= n) return OR_EINVAL;
  double eps2 = eps * eps;
  double eps2_bh = eps_bh * eps_bh;
  set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < n_act; ++k) {
    int64_t i = idx ? idx[k] : k;
    pair_sum(n, m, x, v, eps2, eps2_bh, bh, i, compensated, acc + 3 * k, jrk + 3 * k);
  }
  return OR_OK;
}

/*
 * Energy, Eq. (2) with G = 1: E = 1/2 sum_i m_i v_i^2 - sum_{i<j} m_i m_j / d_ij.
 * epot uses the softened distance d_ij = sqrt(|r_ij|^2 + eps^2) (READING, see
 * header); epot_unsoft uses d_ij = |r_ij| exactly as printed (pairs at zero
 * distance would give -inf). Pairs are visited in the order (i ascending,
 * j > i ascending); sums are compensated.
 */
int or_energy(int64_t n, const double* m, const double* x, const double* v, double eps,
              double eps_bh, int64_t bh, double* ekin, double* epot, double* epot_unsoft) {
  if (n < 1 || bh >= n) return OR_EINVAL;
  double eps2 = eps * eps;
  double eps2_bh = eps_bh * eps_bh;
  double sk = 0, ck = 0, sp = 0, cp = 0, su = 0, cu = 0;
  for (int64_t i = 0; i < n; ++i) {
    double v2 = v[3 * i] * v[3 * i] + v[3 * i + 1] * v[3 * i + 1] + v[3 * i + 2] * v[3 * i + 2];
    neumaier_add(&sk, &ck, 0.5 * m[i] * v2);
    for (int64_t j = i + 1; j < n; ++j) {
      double dx = x[3 * i] - x[3 * j], dy = x[3 * i + 1] - x[3 * j + 1], dz = x[3 * i + 2] - x[3 * j + 2];
      double r2 = dx * dx + dy * dy + dz * dz;
      double mm = m[i] * m[j];
      neumaier_add(&sp, &cp, -mm / sqrt(r2 + pair_eps2(i, j, eps2, eps2_bh, bh)));
      if (epot_unsoft) neumaier_add(&su, &cu, -mm / sqrt(r2));
    }
  }
  if (ekin) *ekin = sk + ck;
  if (epot) *epot = sp + cp;
  if (epot_unsoft) *epot_unsoft = su + cu;
  return OR_OK;
}

/*
 * Predictor (Sec. 2.1: the explicit third-order extrapolation of H4; Sec. 2.4
 * step 7(a)). Each particle j is advanced from its own time t_j to t by the
 * Taylor series through the jerk term, Delta = t - t_j:
 *   x_p = x + v Delta + a Delta^2 / 2 + jerk Delta^3 / 6
 *   v_p = v + a Delta + jerk Delta^2 / 2
 */
void or_predict(int64_t n, const double* x, const double* v, const double* a, const double* jk,
                const double* t_i, double t, double* xp, double* vp) {
  for (int64_t j = 0; j < n; ++j) {
    double dt = t - t_i[j];
    for (int d = 0; d < 3; ++d) {
      int64_t q = 3 * j + d;
      xp[q] = x[q] + v[q] * dt + a[q] * dt * dt / 2.0 + jk[q] * dt * dt * dt / 6.0;
      vp[q] = v[q] + a[q] * dt + jk[q] * dt * dt / 2.0;
    }
  }
}

/*
 * Hermite interpolation of the force over one step (Sec. 2.1: the fourth-order
 * corrector of H4). With a0, j0 at the start of a step of length h and a1, j1
 * at its end, the unique cubic a(t) matching all four has second and third
 * derivatives at the start
 *   a2 = (-6 (a0 - a1) - h (4 j0 + 2 j1)) / h^2
 *   a3 = (12 (a0 - a1) + 6 h (j0 + j1)) / h^3
 */
void or_hermite_derivs(const double* a0, const double* j0, const double* a1, const double* j1,
                       double h, double* a2, double* a3) {
  for (int d = 0; d < 3; ++d) {
    a2[d] = (-6.0 * (a0[d] - a1[d]) - h * (4.0 * j0[d] + 2.0 * j1[d])) / (h * h);
    a3[d] = (12.0 * (a0[d] - a1[d]) + 6.0 * h * (j0[d] + j1[d])) / (h * h * h);
  }
}

/*
 * Corrector: the predicted state plus the integrals of the two higher terms of
 * the cubic,
 *   x = x_p + a2 h^4 / 24 + a3 h^5 / 120
 *   v = v_p + a2 h^3 / 6  + a3 h^4 / 24
 */
void or_correct(const double* xp, const double* vp, const double* a2, const double* a3,
                double h, double* x, double* v) {
  for (int d = 0; d < 3; ++d) {
    x[d] = xp[d] + a2[d] * h * h * h * h / 24.0 + a3[d] * h * h * h * h * h / 120.0;
    v[d] = vp[d] + a2[d] * h * h * h / 6.0 + a3[d] * h * h * h * h / 24.0;
  }
}

static double norm3(const double* u) { return sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]); }

/*
 * Time-step criteria controlled by eta (Sec. 3.2; the criterion itself is the
 * Aarseth form used with H4 by Makino & Aarseth 1992 — READING, see header).
 * Initial step (the same eta is used "from the initial calculation to the
 * update"): dt* = eta |a| / |jerk|.
 * Regular step, from the new force a1, j1 and the derivatives at the end of
 * the step, a2e = a2 + h a3 and a3:
 *   dt* = sqrt(eta (|a1| |a2e| + |j1|^2) / (|j1| |a3| + |a2e|^2))
 */
double or_dt_initial(const double* a, const double* jk, double eta) {
  return eta * norm3(a) / norm3(jk);
}

double or_dt_aarseth(const double* a1, const double* j1, const double* a2, const double* a3,
                     double h, double eta) {
  double a2e[3];
  for (int d = 0; d < 3; ++d) a2e[d] = a2[d] + h * a3[d];
  double na1 = norm3(a1), nj1 = norm3(j1), na2 = norm3(a2e), na3 = norm3(a3);
  return sqrt(eta * (na1 * na2 + nj1 * nj1) / (nj1 * na3 + na2 * na2));
}

/*
 * Block time steps (Sec. 2.4, block-time-step item, after Press 1986): steps
 * are dt_max / 2^k, k >= 0 (READING of the quantisation rule, which the paper
 * does not print):
 *   - the candidate is the largest dt_max / 2^k that is <= dt* (dt* that is
 *     not a finite number below dt_max gives dt_max);
 *   - a smaller candidate is taken at once (any number of halvings);
 *   - a larger one grows the step by one doubling only, and only when the new
 *     time t_new is a multiple of the doubled step and that step is <= dt_max;
 *   - the result is clamped below at dt_min, and each clamp is counted.
 * dt_old = INFINITY selects the initial step (no doubling rule applies).
 */
double or_quantize(double dtstar, double dt_old, double t_new, double dt_max, double dt_min,
                   int64_t* clamps) {
  double cand = dt_max;
  if (dtstar < dt_max) {
    while (cand > dtstar && cand >= dt_min) cand *= 0.5;
  }
  double dt_new;
  if (cand <= dt_old) {
    dt_new = cand;
  } else if (2.0 * dt_old <= dt_max && fmod(t_new, 2.0 * dt_old) == 0.0) {
    dt_new = 2.0 * dt_old;
  } else {
    dt_new = dt_old;
  }
  if (dt_new < dt_min) {
    dt_new = dt_min;
    if (clamps) ++*clamps;
  }
  return dt_new;
}

/*
 * Initialisation (Sec. 2.4 steps 2-3): forces of all particles at t = 0
 * (O(N^2)), t_i = 0, and the initial block step of every particle.
 */
int or_init(int64_t n, const double* m, const double* x, const double* v, double eps,
            double eps_bh, int64_t bh, double eta, double dt_max, double dt_min, double* a,
            double* jk, double* t_i, double* dt_i, int64_t* clamps, int nthreads) {
  int rc = or_force(n, m, x, v, eps, eps_bh, bh, n, NULL, a, jk, 0, nthreads);
  if (rc) return rc;
  for (int64_t i = 0; i < n; ++i) {
    t_i[i] = 0.0;
    dt_i[i] = or_quantize(or_dt_initial(a + 3 * i, jk + 3 * i, eta), INFINITY, 0.0, dt_max, dt_min,
                          clamps);
  }
  return OR_OK;
}

/*
 * One block step (Sec. 2.4 steps 5-7):
 *   5. find the active particles: every i with t_i + dt_i equal to the
 *      earliest such time t_next (dyadic times compare exactly), in ascending
 *      index order;
 *   6. keep their current a, jerk for the corrector;
 *   7a. predict every particle to t_next;
 *   7c. new a, jerk of the active particles from the predicted state of all;
 *   7d. correct the active particles, give each a new block step, and move
 *       them to t_next.
 * Writes the active indices to active_out (capacity n) and returns N_act
 * (negative on error). *t_now is set to t_next.
 */
int64_t or_block_step(int64_t n, const double* m, double* x, double* v, double* a, double* jk,
                      double* t_i, double* dt_i, double eps, double eps_bh, int64_t bh,
                      double eta, double dt_max, double dt_min, double* t_now,
                      int64_t* active_out, int64_t* clamps, int nthreads) {
  double t_next = INFINITY;
  for (int64_t i = 0; i < n; ++i)
    if (t_i[i] + dt_i[i] < t_next) t_next = t_i[i] + dt_i[i];
  int64_t n_act = 0;
  for (int64_t i = 0; i < n; ++i)
    if (t_i[i] + dt_i[i] == t_next) active_out[n_act++] = i;

  double* xp = (double*)malloc(sizeof(double) * 3 * n);
  double* vp = (double*)malloc(sizeof(double) * 3 * n);
  double* a1 = (double*)malloc(sizeof(double) * 3 * n_act);
  double* j1 = (double*)malloc(sizeof(double) * 3 * n_act);
  if (!xp || !vp || !a1 || !j1) {
    free(xp); free(vp); free(a1); free(j1);
    return OR_ENOMEM;
  }
  or_predict(n, x, v, a, jk, t_i, t_next, xp, vp);
  or_force(n, m, xp, vp, eps, eps_bh, bh, n_act, active_out, a1, j1, 0, nthreads);
  for (int64_t k = 0; k < n_act; ++k) {
    int64_t i = active_out[k];
    double h = dt_i[i];
    double a2[3], a3[3];
    or_hermite_derivs(a + 3 * i, jk + 3 * i, a1 + 3 * k, j1 + 3 * k, h, a2, a3);
    or_correct(xp + 3 * i, vp + 3 * i, a2, a3, h, x + 3 * i, v + 3 * i);
    double dtstar = or_dt_aarseth(a1 + 3 * k, j1 + 3 * k, a2, a3, h, eta);
    for (int d = 0; d < 3; ++d) {
      a[3 * i + d] = a1[3 * k + d];
      jk[3 * i + d] = j1[3 * k + d];
    }
    t_i[i] = t_next;
    dt_i[i] = or_quantize(dtstar, h, t_next, dt_max, dt_min, clamps);
  }
  free(xp); free(vp); free(a1); free(j1);
  *t_now = t_next;
  return n_act;
}

/*
 * Integration from the current state (all particles synchronised at *t_now)
 * to t_end, a multiple of dt_max. Every time a multiple of dt_max is reached
 * all particles are synchronised and a log row is written, the columns of the
 * paper's run log (Appendix A, example run): time, block steps, particle
 * steps, total energy, relative energy change since the previous row and
 * since the start. Each row holds 8 doubles:
 *   t, block_steps, particle_steps, E, |E - E_prev| / |E_prev|, |E - E0| / |E0|,
 *   ekin, epot
 * stats[0..3] accumulate block steps, particle steps, pair interactions
 * (sum of N_act * N) and dt_min clamps. Returns the number of rows written,
 * negative on error.
 */
int64_t or_run(int64_t n, const double* m, double* x, double* v, double* a, double* jk,
               double* t_i, double* dt_i, double eps, double eps_bh, int64_t bh, double eta,
               double dt_max, double dt_min, double* t_now, double t_end, double e0,
               int64_t* stats, double* rows, int64_t max_rows, int nthreads) {
  int64_t* active = (int64_t*)malloc(sizeof(int64_t) * n);
  if (!active) return OR_ENOMEM;
  int64_t nrows = 0;
  double e_prev = e0;
  while (*t_now < t_end) {
    int64_t n_act = or_block_step(n, m, x, v, a, jk, t_i, dt_i, eps, eps_bh, bh, eta, dt_max,
                                  dt_min, t_now, active, &stats[3], nthreads);
    if (n_act < 0) {
      free(active);
      return n_act;
    }
    stats[0] += 1;
    stats[1] += n_act;
    stats[2] += n_act * n;
    if (fmod(*t_now, dt_max) == 0.0) {
      for (int64_t i = 0; i < n; ++i)
        if (t_i[i] != *t_now) {
          free(active);
          return OR_ESTATE;
        }
      double ek, ep;
      or_energy(n, m, x, v, eps, eps_bh, bh, &ek, &ep, NULL);
      double e = ek + ep;
      if (nrows < max_rows) {
        double* r = rows + 8 * nrows;
        r[0] = *t_now;
        r[1] = (double)stats[0];
        r[2] = (double)stats[1];
        r[3] = e;
        r[4] = fabs(e - e_prev) / fabs(e_prev);
        r[5] = fabs(e - e0) / fabs(e0);
        r[6] = ek;
        r[7] = ep;
        ++nrows;
      }
      e_prev = e;
    }
  }
  free(active);
  return nrows;
}
