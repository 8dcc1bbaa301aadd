// C ABI of the gfx950 Hermite-4 block-step library (declared in
// include/gravidy_hip.h): argument validation, workspace carve-up, launch
// sequencing, hipGraph capture of block-step sequences, status readback.
//
// The host never takes part in a block step: the schedule, the active set,
// the block size and every stop condition live in device memory, so a
// sequence of steps is captured once into a graph and replayed; the host
// synchronises once per replay to see whether the stop time was reached.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <string>

#include "gd_internal.h"
#include "../../include/gravidy_hip.h"

using namespace gd;

namespace {

constexpr int kGraphSteps = 64;  // block steps per captured graph

enum Phase { kIdle = 0, kPredictedAuto = 1, kPredictedExplicit = 2, kForcedAuto = 3, kForcedExplicit = 4 };

thread_local std::string g_init_error;

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Byte offsets of every array in the workspace.
struct Layout {
  size_t sc, m, jm, x[3], v[3], a[3], j[3], p[3], pv[3], tick, lev, active, ip[3], ipv[3], ia[3], ij[3], ilev,
      part, ebuf, total;
};

Layout make_layout(long long n) {
  Layout L;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  const size_t nd = sizeof(double) * (size_t)n;
  L.sc = take(sizeof(Sched));
  L.m = take(nd);
  L.jm = take(nd);
  for (int d = 0; d < 3; ++d) L.x[d] = take(nd);
  for (int d = 0; d < 3; ++d) L.v[d] = take(nd);
  for (int d = 0; d < 3; ++d) L.a[d] = take(nd);
  for (int d = 0; d < 3; ++d) L.j[d] = take(nd);
  for (int d = 0; d < 3; ++d) L.p[d] = take(nd);
  for (int d = 0; d < 3; ++d) L.pv[d] = take(nd);
  L.tick = take(sizeof(long long) * (size_t)n);
  L.lev = take(sizeof(int) * (size_t)n);
  L.active = take(sizeof(int) * (size_t)n);
  for (int d = 0; d < 3; ++d) L.ip[d] = take(nd);
  for (int d = 0; d < 3; ++d) L.ipv[d] = take(nd);
  for (int d = 0; d < 3; ++d) L.ia[d] = take(nd);
  for (int d = 0; d < 3; ++d) L.ij[d] = take(nd);
  L.ilev = take(sizeof(int) * (size_t)n);
  L.part = take(sizeof(double) * 6 * (size_t)partial_rows(n));
  const long long eitems = std::max<long long>((n + kBlock - 1) / kBlock, kEnergyGrid);
  L.ebuf = take(sizeof(double) * 3 * (size_t)(eitems + 1));
  L.total = off;
  return L;
}

bool is_pow2(double v) {
  if (!(v > 0.0) || !std::isfinite(v)) return false;
  int e;
  return std::frexp(v, &e) == 0.5;
}

}  // namespace

struct gd_ctx {
  gd_params p{};
  long long n = 0;
  Consts c{};
  Dev d{};
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  bool prof = false, ev_ready = false;
  hipEvent_t ev_s[kGraphSteps + 1] = {}, ev_e[kGraphSteps + 1] = {};
  double prof_ms = 0.0;
  long long prof_launches = 0, prof_pairs = 0;
  Sched* h_sc = nullptr;    // pinned host mirror of the device record
  double* h_e = nullptr;    // pinned host energy result (3 doubles)
  double* d_eres = nullptr; // device energy result
  int phase = kIdle;
  bool synced = true;       // every particle at t_now
  long long t_now = 0;      // host copy, valid when synced
  double e0 = 0, e_last = 0;
  std::string err;

  gd_status fail(gd_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return st;
  }
  gd_status hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return GD_OK;
    return fail(GD_EHIP, "%s: %s", what, hipGetErrorString(e));
  }
};

#define GD_TRY(expr)              \
  do {                            \
    gd_status _st = (expr);       \
    if (_st != GD_OK) return _st; \
  } while (0)

namespace {

gd_status read_sched(gd_ctx* c) {
  GD_TRY(c->hip(hipMemcpyAsync(c->h_sc, c->d.sc, sizeof(Sched), hipMemcpyDeviceToHost, c->stream),
                "read status"));
  return c->hip(hipStreamSynchronize(c->stream), "synchronise");
}

gd_status energy_now(gd_ctx* c, int unsoft, double out[3]) {
  GD_TRY(c->hip(launch_energy(c->d, c->c, unsoft, c->stream), "energy kernel"));
  GD_TRY(c->hip(hipMemcpyAsync(c->h_e, c->d_eres, 3 * sizeof(double), hipMemcpyDeviceToHost,
                               c->stream),
                "read energy"));
  GD_TRY(c->hip(hipStreamSynchronize(c->stream), "synchronise"));
  for (int k = 0; k < 3; ++k) out[k] = c->h_e[k];
  return GD_OK;
}

// One block step: predict (auto schedule), force, correct. With events
// (direct launches only), the force launch records its own start and end.
gd_status enqueue_step(gd_ctx* c, hipStream_t s, hipEvent_t ev_s, hipEvent_t ev_e) {
  GD_TRY(c->hip(launch_predict(c->d, c->c, kPredAuto, 0.0, s), "predict kernel"));
  GD_TRY(c->hip(launch_force(c->d, c->c, s, ev_s, ev_e), "force kernel"));
  return c->hip(launch_correct(c->d, c->c, s), "correct kernel");
}

// Captures kGraphSteps block steps into *out.
gd_status build_graph(gd_ctx* c, hipGraphExec_t* out) {
  if (*out) return GD_OK;
  hipGraph_t g = nullptr;
  GD_TRY(c->hip(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal),
                "begin capture"));
  gd_status st = GD_OK;
  for (int k = 0; k < kGraphSteps && st == GD_OK; ++k)
    st = enqueue_step(c, c->capture_stream, nullptr, nullptr);
  hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
  if (st != GD_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  GD_TRY(c->hip(e, "end capture"));
  e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return c->hip(e, "instantiate graph");
}

// Initialisation (Sec. 2.4 steps 2-3): load m, x, v at t = 0, force of every
// particle (O(N^2)), initial block steps, energy. Shared by gd_init and
// gd_reinit; statistics restart from zero.
gd_status initialise(gd_ctx* c, const double* m, const double* x, const double* v) {
  const Dev& d = c->d;
  GD_TRY(c->hip(launch_reset_sched(d, 0, c->stream), "reset"));
  GD_TRY(c->hip(launch_load(d, c->c, m, x, v, c->stream), "load kernel"));
  GD_TRY(c->hip(launch_predict(d, c->c, kPredAll, 0.0, c->stream), "predict kernel"));
  GD_TRY(c->hip(launch_force(d, c->c, c->stream, c->prof ? c->ev_s[kGraphSteps] : nullptr,
                             c->prof ? c->ev_e[kGraphSteps] : nullptr),
                "force kernel"));
  GD_TRY(c->hip(launch_init_dt(d, c->c, c->stream), "init dt kernel"));
  GD_TRY(read_sched(c));
  if (c->h_sc->bad_input) return c->fail(GD_EINVAL, "non-finite or negative input (m, x or v)");
  if (c->h_sc->nonfinite) return c->fail(GD_ENONFINITE, "non-finite initial acceleration or jerk");
  if (c->prof) {
    float ms = 0.f;
    GD_TRY(c->hip(hipEventElapsedTime(&ms, c->ev_s[kGraphSteps], c->ev_e[kGraphSteps]), "event time"));
    c->prof_ms += ms;
    c->prof_launches += 1;
    c->prof_pairs += c->n * c->n;
  }
  double e[3];
  GD_TRY(energy_now(c, 0, e));
  c->e0 = c->e_last = e[0] + e[1];
  c->t_now = 0;
  c->synced = true;
  c->phase = kIdle;
  return GD_OK;
}

}  // namespace

extern "C" {

gd_status gd_workspace_bytes(int64_t n, const gd_params* p, size_t* bytes) {
  (void)p;
  if (!bytes || n < 2 || n > (int64_t)std::numeric_limits<int>::max() / 2) return GD_EINVAL;
  *bytes = make_layout(n).total;
  return GD_OK;
}

gd_status gd_init(gd_ctx** out, const gd_params* p, int64_t n, const double* m, const double* x,
                  const double* v, void* workspace, size_t ws_bytes, void* hip_stream) {
  if (!out) return GD_EINVAL;
  *out = nullptr;
  auto bad = [](gd_status st, const char* msg) {
    g_init_error = msg;
    return st;
  };
  if (!p || !m || !x || !v || !workspace) return bad(GD_EINVAL, "NULL argument");
  if (n < 2 || n > (int64_t)std::numeric_limits<int>::max() / 2) return bad(GD_EINVAL, "n out of range");
  if (!(p->eta > 0.0) || !std::isfinite(p->eta)) return bad(GD_EINVAL, "eta must be finite and > 0");
  if (!(p->eps == 0.0 || (p->eps >= 1e-30 && std::isfinite(p->eps))))
    return bad(GD_EINVAL, "eps must be 0 or in [1e-30, inf)");
  if (p->bh_index < -1 || p->bh_index >= n) return bad(GD_EINVAL, "bh_index must be -1 or in [0, n)");
  if (p->bh_index >= 0 && !(p->eps >= 1e-30 && p->eps_bh >= 1e-30 && std::isfinite(p->eps_bh)))
    return bad(GD_EINVAL, "with a central particle, eps and eps_bh must be in [1e-30, inf)");
  if (!is_pow2(p->dt_max) || !is_pow2(p->dt_min) || p->dt_min > p->dt_max)
    return bad(GD_EINVAL, "dt_max and dt_min must be powers of two with dt_min <= dt_max");
  int kmax = (int)std::lround(std::log2(p->dt_max / p->dt_min));
  if (kmax > 40) return bad(GD_EINVAL, "log2(dt_max / dt_min) must be <= 40");
  if (p->flags != 0) return bad(GD_EINVAL, "flags must be 0");
  if (((uintptr_t)workspace & 255) != 0) return bad(GD_EINVAL, "workspace must be 256-byte aligned");
  const Layout L = make_layout(n);
  if (ws_bytes < L.total) return bad(GD_ENOMEM, "workspace smaller than gd_workspace_bytes()");

  gd_ctx* c = new (std::nothrow) gd_ctx();
  if (!c) return bad(GD_EINVAL, "out of host memory");
  c->p = *p;
  c->n = n;
  c->c.n = (int)n;
  c->c.kmax = kmax;
  c->c.dt_min = p->dt_min;
  c->c.dt_max = p->dt_max;
  c->c.eta = p->eta;
  c->c.eps2 = p->eps * p->eps;
  c->c.bh = (int)p->bh_index;
  c->c.eps2_bh = p->bh_index >= 0 ? p->eps_bh * p->eps_bh : c->c.eps2;
  launch_grids((int)n, &c->c.force_grid, &c->c.correct_grid);
  c->stream = (hipStream_t)hip_stream;
  char* w = (char*)workspace;
  Dev& d = c->d;
  d.sc = (Sched*)(w + L.sc);
  d.m = (double*)(w + L.m);
  d.jm = (double*)(w + L.jm);
  double** xs[3] = {&d.x, &d.y, &d.z};
  double** vs[3] = {&d.vx, &d.vy, &d.vz};
  double** as[3] = {&d.ax, &d.ay, &d.az};
  double** js[3] = {&d.jx, &d.jy, &d.jz};
  double** ps[3] = {&d.px, &d.py, &d.pz};
  double** pvs[3] = {&d.pvx, &d.pvy, &d.pvz};
  for (int k = 0; k < 3; ++k) {
    *xs[k] = (double*)(w + L.x[k]);
    *vs[k] = (double*)(w + L.v[k]);
    *as[k] = (double*)(w + L.a[k]);
    *js[k] = (double*)(w + L.j[k]);
    *ps[k] = (double*)(w + L.p[k]);
    *pvs[k] = (double*)(w + L.pv[k]);
  }
  d.tick = (long long*)(w + L.tick);
  d.lev = (int*)(w + L.lev);
  d.active = (int*)(w + L.active);
  double** is[3] = {&d.ix, &d.iy, &d.iz};
  double** ivs[3] = {&d.ivx, &d.ivy, &d.ivz};
  double** ias[3] = {&d.iax, &d.iay, &d.iaz};
  double** ijs[3] = {&d.ijx, &d.ijy, &d.ijz};
  for (int k = 0; k < 3; ++k) {
    *is[k] = (double*)(w + L.ip[k]);
    *ivs[k] = (double*)(w + L.ipv[k]);
    *ias[k] = (double*)(w + L.ia[k]);
    *ijs[k] = (double*)(w + L.ij[k]);
  }
  d.ilev = (int*)(w + L.ilev);
  d.part = (double*)(w + L.part);
  d.ebuf = (double*)(w + L.ebuf);

  auto cleanup_fail = [&](gd_status st) {
    g_init_error = c->err;
    gd_destroy(c);
    return st;
  };
  gd_status st;
  if ((st = c->hip(hipHostMalloc((void**)&c->h_sc, sizeof(Sched), hipHostMallocDefault),
                   "pinned status buffer")) != GD_OK)
    return cleanup_fail(st);
  if ((st = c->hip(hipHostMalloc((void**)&c->h_e, 4 * sizeof(double), hipHostMallocDefault),
                   "pinned energy buffer")) != GD_OK)
    return cleanup_fail(st);
  if ((st = c->hip(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking),
                   "capture stream")) != GD_OK)
    return cleanup_fail(st);

  c->d_eres = d.ebuf + 3 * (size_t)make_eplan((int)n).items;
  if ((st = initialise(c, m, x, v)) != GD_OK) return cleanup_fail(st);
  *out = c;
  return GD_OK;
}

gd_status gd_reinit(gd_ctx* c, const double* m, const double* x, const double* v) {
  if (!c) return GD_EINVAL;
  if (!m || !x || !v) return c->fail(GD_EINVAL, "NULL argument");
  return initialise(c, m, x, v);
}

gd_status gd_profile_force(gd_ctx* c, int enable) {
  if (!c) return GD_EINVAL;
  if (enable && !c->ev_ready) {
    for (int k = 0; k < kGraphSteps + 1; ++k) {
      GD_TRY(c->hip(hipEventCreate(&c->ev_s[k]), "event create"));
      GD_TRY(c->hip(hipEventCreate(&c->ev_e[k]), "event create"));
    }
    c->ev_ready = true;
  }
  c->prof = enable != 0;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  c->prof_pairs = 0;
  return GD_OK;
}

gd_status gd_profile_get(gd_ctx* c, double* force_ms, int64_t* launches, int64_t* pairs) {
  if (!c) return GD_EINVAL;
  if (force_ms) *force_ms = c->prof_ms;
  if (launches) *launches = c->prof_launches;
  if (pairs) *pairs = c->prof_pairs;
  return GD_OK;
}

gd_status gd_predict(gd_ctx* c, const double* t) {
  if (!c) return GD_EINVAL;
  if (t == nullptr) {
    GD_TRY(c->hip(launch_set_tend(c->d, std::numeric_limits<long long>::max(), c->stream), "prepare"));
    GD_TRY(c->hip(launch_predict(c->d, c->c, kPredAuto, 0.0, c->stream), "predict kernel"));
    c->phase = kPredictedAuto;
  } else {
    if (!std::isfinite(*t)) return c->fail(GD_EINVAL, "t must be finite");
    GD_TRY(c->hip(launch_predict(c->d, c->c, kPredExplicit, *t, c->stream), "predict kernel"));
    c->phase = kPredictedExplicit;
  }
  return GD_OK;
}

gd_status gd_force(gd_ctx* c, const int32_t* idx, int64_t n_act, double* acc, double* jerk) {
  if (!c) return GD_EINVAL;
  if (c->phase == kIdle) return c->fail(GD_ESTATE, "gd_force before gd_predict");
  if (idx == nullptr) {
    if (c->phase != kPredictedAuto && c->phase != kForcedAuto)
      return c->fail(GD_ESTATE, "no active set: use gd_predict(NULL) or pass indices");
    c->phase = kForcedAuto;
  } else {
    if (n_act < 0 || n_act > c->n) return c->fail(GD_EINVAL, "n_act out of range");
    if (n_act == 0) {
      c->phase = kForcedExplicit;
      return GD_OK;
    }
    GD_TRY(c->hip(launch_set_active(c->d, c->c, idx, (int)n_act, c->stream), "set active"));
    c->phase = kForcedExplicit;
  }
  GD_TRY(c->hip(launch_force(c->d, c->c, c->stream), "force kernel"));
  if (acc || jerk) GD_TRY(c->hip(launch_reduce_out(c->d, c->c, acc, jerk, c->stream), "force output"));
  if (idx != nullptr) {
    GD_TRY(read_sched(c));
    if (c->h_sc->bad_input) {
      c->h_sc->bad_input = 0;
      GD_TRY(c->hip(hipMemcpyAsync(&c->d.sc->bad_input, &c->h_sc->bad_input, sizeof(int),
                                   hipMemcpyHostToDevice, c->stream),
                    "clear flag"));
      GD_TRY(c->hip(hipStreamSynchronize(c->stream), "synchronise"));
      return c->fail(GD_EINVAL, "index out of range in idx");
    }
  }
  return GD_OK;
}

gd_status gd_active(gd_ctx* c, int32_t* idx, int64_t* n_act) {
  if (!c || !n_act) return GD_EINVAL;
  if (c->phase != kPredictedAuto && c->phase != kForcedAuto)
    return c->fail(GD_ESTATE, "no active set: call gd_predict(NULL) first");
  if (idx) GD_TRY(c->hip(launch_copy_active(c->d, c->c, idx, c->stream), "copy active"));
  GD_TRY(read_sched(c));
  *n_act = c->h_sc->n_act;
  return GD_OK;
}

gd_status gd_correct(gd_ctx* c) {
  if (!c) return GD_EINVAL;
  if (c->phase != kForcedAuto) return c->fail(GD_ESTATE, "gd_correct needs gd_predict(NULL) then gd_force(NULL, ...)");
  GD_TRY(c->hip(launch_correct(c->d, c->c, c->stream), "correct kernel"));
  c->phase = kIdle;
  c->synced = false;
  return GD_OK;
}

gd_status gd_step_to(gd_ctx* c, double t_end, gd_stats* st) {
  if (!c) return GD_EINVAL;
  if (c->phase == kPredictedAuto || c->phase == kForcedAuto)
    return c->fail(GD_ESTATE, "a block step is in progress (gd_predict without gd_correct)");
  // Current time (exact): synchronised contexts know it; otherwise read it.
  if (!c->synced) {
    GD_TRY(read_sched(c));
    c->t_now = c->h_sc->t_now;
  }
  const double q = t_end / c->p.dt_max;
  if (!std::isfinite(t_end) || q != std::floor(q) || q < 0 || q > 9.0e15 / (1LL << c->c.kmax))
    return c->fail(GD_EINVAL, "t_end must be a non-negative multiple of dt_max");
  const long long per_max = 1LL << c->c.kmax;
  const long long target = (long long)q * per_max;
  if (target < c->t_now) return c->fail(GD_EINVAL, "t_end is before the current time");
  // Profiling runs the same steps as direct launches (the force launches
  // carry timing events); otherwise a captured graph is replayed.
  if (!c->prof) GD_TRY(build_graph(c, &c->graph));
  c->phase = kIdle;
  GD_TRY(read_sched(c));
  long long steps_before = c->h_sc->block_steps, pairs_before = c->h_sc->pairs;
  while (c->t_now < target) {
    // Advance to the next multiple of dt_max, where all particles meet.
    const long long chunk_end = (c->t_now / per_max + 1) * per_max;
    GD_TRY(c->hip(launch_set_tend(c->d, chunk_end, c->stream), "prepare"));
    for (;;) {
      if (c->prof) {
        for (int k = 0; k < kGraphSteps; ++k) GD_TRY(enqueue_step(c, c->stream, c->ev_s[k], c->ev_e[k]));
      } else {
        GD_TRY(c->hip(hipGraphLaunch(c->graph, c->stream), "graph launch"));
      }
      GD_TRY(read_sched(c));
      if (c->h_sc->nonfinite) return c->fail(GD_ENONFINITE, "non-finite acceleration or jerk");
      if (c->prof) {
        // Steps run in order; the first (block_steps delta) of the replay were real.
        const long long ran = c->h_sc->block_steps - steps_before;
        for (long long k = 0; k < ran && k < kGraphSteps; ++k) {
          float ms = 0.f;
          GD_TRY(c->hip(hipEventElapsedTime(&ms, c->ev_s[k], c->ev_e[k]), "event time"));
          c->prof_ms += ms;
        }
        c->prof_launches += ran;
        c->prof_pairs += c->h_sc->pairs - pairs_before;
      }
      steps_before = c->h_sc->block_steps;
      pairs_before = c->h_sc->pairs;
      if (c->h_sc->t_now >= chunk_end) break;
    }
    c->t_now = c->h_sc->t_now;
    double e[3];
    GD_TRY(energy_now(c, 0, e));
    c->e_last = e[0] + e[1];
  }
  c->synced = true;
  if (st) GD_TRY(gd_stats_get(c, st));
  return GD_OK;
}

gd_status gd_energy(gd_ctx* c, double* ekin, double* epot, double* epot_unsoft) {
  if (!c) return GD_EINVAL;
  if (!c->synced || c->phase != kIdle)
    return c->fail(GD_ESTATE, "particles are not synchronised (use gd_step_to to a multiple of dt_max)");
  double e[3];
  GD_TRY(energy_now(c, epot_unsoft != nullptr, e));
  if (ekin) *ekin = e[0];
  if (epot) *epot = e[1];
  if (epot_unsoft) *epot_unsoft = e[2];
  return GD_OK;
}

gd_status gd_get_state(gd_ctx* c, double* x, double* v, double* a, double* jerk, double* t_i,
                       double* dt_i, double* t_now) {
  if (!c) return GD_EINVAL;
  GD_TRY(c->hip(launch_get_state(c->d, c->c, x, v, a, jerk, t_i, dt_i, c->stream), "get state"));
  GD_TRY(read_sched(c));
  if (t_now) *t_now = (double)c->h_sc->t_now * c->c.dt_min;
  return GD_OK;
}

gd_status gd_set_state(gd_ctx* c, const double* x, const double* v, const double* a,
                       const double* jerk, const double* t_i, const double* dt_i, double t_now) {
  if (!c) return GD_EINVAL;
  if (!x || !v || !a || !jerk || !t_i || !dt_i) return c->fail(GD_EINVAL, "NULL argument");
  const double q = t_now / c->c.dt_min;
  if (!std::isfinite(q) || q < 0 || q > 9.0e15 || q != std::floor(q))
    return c->fail(GD_EINVAL, "t_now must be a non-negative multiple of dt_min");
  const long long tn = (long long)q;
  GD_TRY(c->hip(launch_reset_sched(c->d, tn, c->stream), "reset"));
  GD_TRY(c->hip(launch_set_state(c->d, c->c, x, v, a, jerk, t_i, dt_i, tn, c->stream), "set state"));
  GD_TRY(read_sched(c));
  if (c->h_sc->bad_input) return c->fail(GD_EINVAL, "invalid state (times, steps or non-finite values)");
  c->t_now = tn;
  c->phase = kIdle;
  // Synchronised only when every particle sits at t_now.
  c->synced = (tn % (1LL << c->c.kmax)) == 0;
  return GD_OK;
}

gd_status gd_stats_get(gd_ctx* c, gd_stats* st) {
  if (!c || !st) return GD_EINVAL;
  GD_TRY(read_sched(c));
  st->t = (double)c->h_sc->t_now * c->c.dt_min;
  st->block_steps = c->h_sc->block_steps;
  st->particle_steps = c->h_sc->particle_steps;
  st->pair_interactions = c->h_sc->pairs;
  st->dtmin_clamps = c->h_sc->clamps;
  st->e0 = c->e0;
  st->e = c->e_last;
  return GD_OK;
}

void gd_destroy(gd_ctx* c) {
  if (!c) return;
  if (c->graph) (void)hipGraphExecDestroy(c->graph);
  if (c->ev_ready)
    for (int k = 0; k < kGraphSteps + 1; ++k) {
      (void)hipEventDestroy(c->ev_s[k]);
      (void)hipEventDestroy(c->ev_e[k]);
    }
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  if (c->h_sc) (void)hipHostFree(c->h_sc);
  if (c->h_e) (void)hipHostFree(c->h_e);
  delete c;
}

const char* gd_last_error(const gd_ctx* c) {
  if (!c) return g_init_error.c_str();
  return c->err.c_str();
}

}  // extern "C"
