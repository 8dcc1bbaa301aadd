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
#include <mutex>
#include <algorithm>
#include <chrono>
#include <string>
#include <vector>

#include "gd_internal.h"
#include "../../include/gravidy_hip.h"

using namespace gd;

namespace {

constexpr int kGraphSteps = 64;  // block steps per captured graph
constexpr int kSchedWords = (int)((sizeof(Sched) + 7) / 8);  // 8-byte words of a status copy
// Force-timing buckets by N_act: lower edges (the last bucket is open).
constexpr int kProfBuckets = GD_PROFILE_BUCKETS;
constexpr long long kProfEdges[kProfBuckets] = {1, 2, 8, 64, 1024, 4096};

int prof_bucket(long long n_act) {
  int b = 0;
  while (b + 1 < kProfBuckets && n_act >= kProfEdges[b + 1]) ++b;
  return b;
}

enum Phase { kIdle = 0, kPredictedAuto = 1, kPredictedExplicit = 2, kForcedAuto = 3, kForcedExplicit = 4 };

thread_local std::string g_init_error;

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

// Byte offsets of every array in the workspace.
struct Layout {
  size_t sc, m, jm, x[3], v[3], a[3], j[3], p[3], pv[3], tick, lev, active, ip[3], ipv[3], ia[3], ij[3], ilev,
      tag, part, ebuf, nact_log, total;
};

// i particles per lane of a context's force kernel (see kIPerLaneLarge).
int ipl_for(const gd_params* p, long long n) {
  return (n >= kLargeN && p->eps > 0.0) ? kIPerLaneLarge : kIPerLane;
}

// The workspace of a context of n particles whose force kernel holds ipl i
// per lane (pools use the size a context would have).
Layout make_layout(long long n, int ipl) {
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
  L.lev = take((size_t)n);
  // two active lists
  L.active = take(2 * sizeof(int) * (size_t)n);
  for (int d = 0; d < 3; ++d) L.ip[d] = take(2 * nd);
  for (int d = 0; d < 3; ++d) L.ipv[d] = take(2 * nd);
  for (int d = 0; d < 3; ++d) L.ia[d] = take(2 * nd);
  for (int d = 0; d < 3; ++d) L.ij[d] = take(2 * nd);
  L.ilev = take(2 * sizeof(int) * (size_t)n);
  L.tag = take(2 * sizeof(long long) * (size_t)n);
  L.part = take(sizeof(double) * 6 * (size_t)partial_rows(n, ipl));
  // At least kEnergyGrid entries: the diagnostics reuse the buffer for their results.
  const long long eitems = std::max<long long>(make_eplan((int)n).items, kEnergyGrid);
  L.ebuf = take(sizeof(double) * 3 * (size_t)(eitems + 1));
  L.nact_log = take(sizeof(int) * 72);
  L.total = off;
  return L;
}

// Device pointers of a workspace laid out by make_layout.
Dev carve(void* workspace, const Layout& L) {
  char* w = (char*)workspace;
  Dev d{};
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
  d.lev = (unsigned char*)(w + L.lev);
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
  d.tag = (long long*)(w + L.tag);
  d.part = (double*)(w + L.part);
  d.ebuf = (double*)(w + L.ebuf);
  d.nact_log = (int*)(w + L.nact_log);
  return d;
}

bool is_pow2(double v) {
  if (!(v > 0.0) || !std::isfinite(v)) return false;
  int e;
  return std::frexp(v, &e) == 0.5;
}

// Host-side validation shared by gd_init and gd_pool_admit; returns the
// reason of the first failed check, or null.
const char* check_params(const gd_params* p, int64_t n, int* kmax_out) {
  if (n < 2 || n > (int64_t)std::numeric_limits<int>::max() / 2) return "n out of range";
  if (!(p->eta > 0.0) || !std::isfinite(p->eta)) return "eta must be finite and > 0";
  if (!(p->eps == 0.0 || (p->eps >= 1e-30 && std::isfinite(p->eps))))
    return "eps must be 0 or in [1e-30, inf)";
  if (p->bh_index < -1 || p->bh_index >= n) return "bh_index must be -1 or in [0, n)";
  if (p->bh_index >= 0 && !(p->eps >= 1e-30 && p->eps_bh >= 1e-30 && std::isfinite(p->eps_bh)))
    return "with a central particle, eps and eps_bh must be in [1e-30, inf)";
  if (!is_pow2(p->dt_max) || !is_pow2(p->dt_min) || p->dt_min > p->dt_max)
    return "dt_max and dt_min must be powers of two with dt_min <= dt_max";
  const int kmax = (int)std::lround(std::log2(p->dt_max / p->dt_min));
  if (kmax > 40) return "log2(dt_max / dt_min) must be <= 40";
  if ((p->flags & ~GD_FLAG_MIXED) != 0) return "flags: unknown bits";
  // Mixed precision rounds m q^3 of the softened self pair (q = 1 / eps) to
  // FP32; below eps^2 = 1e-20 it would overflow, and inf * 0 gives NaN.
  if ((p->flags & GD_FLAG_MIXED) && p->eps > 0.0 && p->eps * p->eps < 1e-20)
    return "with GD_FLAG_MIXED, eps must be 0 or have eps^2 >= 1e-20";
  *kmax_out = kmax;
  return nullptr;
}

// Constants of n particles whose force kernel holds ipl i per lane, without
// the launch grids.
Consts consts_of(const gd_params* p, int64_t n, int kmax, int ipl) {
  Consts c{};
  c.n = (int)n;
  c.kmax = kmax;
  c.dt_min = p->dt_min;
  c.dt_max = p->dt_max;
  c.inv_dt_min = 1.0 / p->dt_min;
  c.inv_dt_max = 1.0 / p->dt_max;
  c.eta = p->eta;
  c.eps2 = p->eps * p->eps;
  c.bh = (int)p->bh_index;
  c.eps2_bh = p->bh_index >= 0 ? p->eps_bh * p->eps_bh : c.eps2;
  c.mixed = (p->flags & GD_FLAG_MIXED) ? 1 : 0;
  const Plan p1 = make_plan(1, (int)n, ipl);
  c.lj1_ipl = p1.lj | (ipl << 8);  // n1 = 0: see make_consts
  c.s1 = p1.s;
  c.part_cs = partial_rows(n, ipl);
  return c;
}

// Constants of a context (pool == false) or of a pool's cluster (pool ==
// true: pools run the force kernel with kIPerLane i per lane), with launch
// grids for every block size.
Consts make_consts(const gd_params* p, int64_t n, int kmax, bool pool) {
  const int ipl = pool ? kIPerLane : ipl_for(p, n);
  Consts c = consts_of(p, n, kmax, ipl);
  launch_grids((int)n, ipl, &c.force_grid, &c.correct_grid);
  // n1: every block of up to n1 particles has the one-particle decomposition
  // (the kernels then take one_plan instead of make_plan's search)
  int n1 = 1;
  while (n1 < n && n1 < 65535) {
    const Plan q = make_plan(n1 + 1, (int)n, ipl);
    if (q.lj != lj1_of(c) || q.s != c.s1) break;
    ++n1;
  }
  c.lj1_ipl |= n1 << 16;
  return c;
}

}  // namespace

struct gd_ctx {
  gd_params p{};
  long long n = 0;
  Consts c{};
  Dev d{};
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;
  // Two instances of the captured block steps, each ending with a copy of the
  // schedule record into its own pinned buffer (h_ring[0] / h_ring[1]), with
  // an event recorded after each launch: replays can then be queued ahead of
  // the host reading an earlier replay's status.
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  Sched* h_ring[2] = {nullptr, nullptr};
  hipEvent_t ev_ring[2] = {nullptr, nullptr};
  bool prof = false, ev_ready = false;
  hipEvent_t ev_s[kGraphSteps + 1] = {}, ev_e[kGraphSteps + 1] = {};
  double prof_ms = 0.0;
  long long prof_launches = 0, prof_pairs = 0;
  double bucket_ms[GD_PROFILE_BUCKETS] = {};
  long long bucket_launches[GD_PROFILE_BUCKETS] = {}, bucket_pairs[GD_PROFILE_BUCKETS] = {};
  int* h_nact = nullptr;    // pinned host copy of the N_act log
  Sched* h_sc = nullptr;    // pinned host mirror of the device record
  double* h_e = nullptr;    // pinned host energy result (3 doubles)
  double* d_eres = nullptr; // device energy result
  int phase = kIdle;
  bool synced = true;       // every particle at t_now
  long long t_now = 0;      // host copy, valid when synced
  double e0 = 0, e_last = 0;
  double wall_s = 0.0;  // host seconds spent in gd_step_to since the state was set
  // Progress report of gd_step_to (0: off): at most one line per interval,
  // written when the host reads the schedule record of a finished replay.
  double progress_s = 0.0;
  double prog_target = 0.0;
  std::chrono::steady_clock::time_point prog_t0, prog_last;
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

// One progress line from the schedule record the host holds (h_sc), if the
// interval has passed since the last one.
void report_progress(gd_ctx* c) {
  if (c->progress_s <= 0.0) return;
  const auto now = std::chrono::steady_clock::now();
  if (std::chrono::duration<double>(now - c->prog_last).count() < c->progress_s) return;
  c->prog_last = now;
  std::fprintf(stderr, "gd_step_to: t = %.9g of %.9g, %lld block steps, %lld particle steps, %.1f s\n",
               (double)c->h_sc->t_now * c->p.dt_min, c->prog_target, c->h_sc->block_steps,
               c->h_sc->particle_steps, std::chrono::duration<double>(now - c->prog_t0).count());
  std::fflush(stderr);
}

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

// One block step of parity par: the force kernel (which finds the step from
// the level histogram and checks the list and j stream the previous step's
// corrector prepared) and the corrector (which also prepares the next step's).
// With events (direct launches only), the force launch records its own start
// and end.
gd_status enqueue_step(gd_ctx* c, hipStream_t s, int par, hipEvent_t ev_s, hipEvent_t ev_e) {
  GD_TRY(c->hip(launch_step_force(c->d, c->c, par, s, ev_s, ev_e), "force kernel"));
  return c->hip(launch_step_correct(c->d, c->c, par, s), "correct kernel");
}

// Captures kGraphSteps block steps into *out.
}  // namespace

// The schedule record copied, word by word, to pinned host memory: the last
// node of a replayed graph, so that the host reads a replay's status without
// a separate copy.
static_assert(sizeof(Sched) % 8 == 0, "the status copy moves whole 8-byte words");
__global__ void k_status_out(const unsigned long long* __restrict__ sc, unsigned long long* __restrict__ out) {
  for (int k = threadIdx.x; k < kSchedWords; k += blockDim.x) out[k] = sc[k];
  __threadfence_system();
}

namespace {

gd_status build_graph(gd_ctx* c, int ring) {
  hipGraphExec_t* out = &c->graph[ring];
  if (*out) return GD_OK;
  hipGraph_t g = nullptr;
  GD_TRY(c->hip(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal),
                "begin capture"));
  gd_status st = GD_OK;
  for (int k = 0; k < kGraphSteps && st == GD_OK; ++k)
    st = enqueue_step(c, c->capture_stream, k & 1, nullptr, nullptr);
  if (st == GD_OK) {
    hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, c->capture_stream,
                       (const unsigned long long*)c->d.sc, (unsigned long long*)c->h_ring[ring]);
    st = c->hip(hipGetLastError(), "status kernel");
  }
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
    const int b = prof_bucket(c->n);
    c->bucket_ms[b] += ms;
    c->bucket_launches[b] += 1;
    c->bucket_pairs[b] += c->n * c->n;
  }
  double e[3];
  GD_TRY(energy_now(c, 0, e));
  c->e0 = c->e_last = e[0] + e[1];
  c->t_now = 0;
  c->wall_s = 0.0;
  c->synced = true;
  c->phase = kIdle;
  return GD_OK;
}

}  // namespace

extern "C" {

gd_status gd_workspace_bytes(int64_t n, const gd_params* p, size_t* bytes) {
  if (!bytes || n < 2 || n > (int64_t)std::numeric_limits<int>::max() / 2) return GD_EINVAL;
  // Without parameters: the larger of the two sizes.
  *bytes = make_layout(n, p ? ipl_for(p, n) : kIPerLaneLarge).total;
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
  int kmax = 0;
  if (const char* why = check_params(p, n, &kmax)) return bad(GD_EINVAL, why);
  if (((uintptr_t)workspace & 255) != 0) return bad(GD_EINVAL, "workspace must be 256-byte aligned");
  const Layout L = make_layout(n, ipl_for(p, n));
  if (ws_bytes < L.total) return bad(GD_ENOMEM, "workspace smaller than gd_workspace_bytes()");

  gd_ctx* c = new (std::nothrow) gd_ctx();
  if (!c) return bad(GD_EINVAL, "out of host memory");
  c->p = *p;
  c->n = n;
  c->c = make_consts(p, n, kmax, false);
  c->stream = (hipStream_t)hip_stream;
  c->d = carve(workspace, L);
  Dev& d = c->d;

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
  for (int r = 0; r < 2; ++r) {
    if ((st = c->hip(hipHostMalloc((void**)&c->h_ring[r], 8 * (size_t)kSchedWords, hipHostMallocDefault),
                     "pinned status ring")) != GD_OK)
      return cleanup_fail(st);
    if ((st = c->hip(hipEventCreateWithFlags(&c->ev_ring[r], hipEventDisableTiming), "status event")) != GD_OK)
      return cleanup_fail(st);
  }

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
    // All events or none: a partial set is destroyed again, so that a later
    // call (or gd_destroy) never sees events it did not record as made.
    int k = 0;
    hipError_t e = hipSuccess;
    for (; k < kGraphSteps + 1; ++k) {
      if ((e = hipEventCreate(&c->ev_s[k])) != hipSuccess) break;
      if ((e = hipEventCreate(&c->ev_e[k])) != hipSuccess) {
        (void)hipEventDestroy(c->ev_s[k]);
        break;
      }
    }
    if (e != hipSuccess) {
      for (int q = 0; q < k; ++q) {
        (void)hipEventDestroy(c->ev_s[q]);
        (void)hipEventDestroy(c->ev_e[q]);
      }
      return c->hip(e, "event create");
    }
    c->ev_ready = true;
  }
  if (enable && !c->h_nact)
    GD_TRY(c->hip(hipHostMalloc((void**)&c->h_nact, sizeof(int) * kGraphSteps, hipHostMallocDefault),
                  "pinned alloc"));
  c->prof = enable != 0;
  c->prof_ms = 0.0;
  c->prof_launches = 0;
  c->prof_pairs = 0;
  for (int b = 0; b < kProfBuckets; ++b) {
    c->bucket_ms[b] = 0.0;
    c->bucket_launches[b] = 0;
    c->bucket_pairs[b] = 0;
  }
  return GD_OK;
}

gd_status gd_profile_buckets(gd_ctx* c, int64_t* n_act_min, double* force_ms, int64_t* launches,
                             int64_t* pairs) {
  if (!c) return GD_EINVAL;
  for (int b = 0; b < kProfBuckets; ++b) {
    if (n_act_min) n_act_min[b] = kProfEdges[b];
    if (force_ms) force_ms[b] = c->bucket_ms[b];
    if (launches) launches[b] = c->bucket_launches[b];
    if (pairs) pairs[b] = c->bucket_pairs[b];
  }
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

}  // extern "C"

namespace {

// The force of the current active set (idx == NULL) or of an index list,
// with make_plan's decomposition (forced_lj == 0) or a forced one.
gd_status force_of(gd_ctx* c, const int32_t* idx, int64_t n_act, double* acc, double* jerk, int forced_lj,
                   int forced_s) {
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
    GD_TRY(c->hip(launch_set_active(c->d, c->c, idx, (int)n_act, c->stream, forced_lj, forced_s), "set active"));
    c->phase = kForcedExplicit;
  }
  // With timing on, an explicit list's launch records its own start and end.
  const bool timed = c->prof && idx != nullptr;
  GD_TRY(c->hip(launch_force(c->d, c->c, c->stream, timed ? c->ev_s[kGraphSteps] : nullptr,
                             timed ? c->ev_e[kGraphSteps] : nullptr),
                "force kernel"));
  if (acc || jerk) GD_TRY(c->hip(launch_reduce_out(c->d, c->c, acc, jerk, c->stream), "force output"));
  if (idx != nullptr) {
    GD_TRY(read_sched(c));
    if (timed) {
      float ms = 0.f;
      GD_TRY(c->hip(hipEventElapsedTime(&ms, c->ev_s[kGraphSteps], c->ev_e[kGraphSteps]), "event time"));
      c->prof_ms += ms;
      c->prof_launches += 1;
      c->prof_pairs += n_act * c->n;
      const int b = prof_bucket(n_act);
      c->bucket_ms[b] += ms;
      c->bucket_launches[b] += 1;
      c->bucket_pairs[b] += n_act * c->n;
    }
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

}  // namespace

extern "C" {

gd_status gd_force(gd_ctx* c, const int32_t* idx, int64_t n_act, double* acc, double* jerk) {
  if (!c) return GD_EINVAL;
  return force_of(c, idx, n_act, acc, jerk, 0, 0);
}

gd_status gd_force_plan(gd_ctx* c, const int32_t* idx, int64_t n_act, int32_t lanes_per_i, int32_t slices,
                        double* acc, double* jerk) {
  if (!c) return GD_EINVAL;
  if (!idx) return c->fail(GD_EINVAL, "gd_force_plan needs an index list");
  const int lj = lanes_per_i == 16 ? 4 : lanes_per_i == 32 ? 5 : lanes_per_i == 64 ? 6 : 0;
  if (lj == 0) return c->fail(GD_EINVAL, "lanes_per_i must be 16, 32 or 64");
  const long long tiles = (c->n + kTileJ - 1) / kTileJ;
  if (slices < 1 || slices > tiles) return c->fail(GD_EINVAL, "slices must be in [1, ceil(n / 256)]");
  if (n_act < 0 || n_act > c->n) return c->fail(GD_EINVAL, "n_act out of range");
  const Plan p = plan_with((int)n_act, (int)c->n, lj, slices, ipl_of(c->c));
  if ((long long)p.s * n_act > c->c.part_cs)
    return c->fail(GD_EINVAL, "%d slices of %lld particles exceed the partial-force buffer", p.s,
                   (long long)n_act);
  return force_of(c, idx, n_act, acc, jerk, lj, slices);
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

namespace {

// Graph replays until the schedule reaches chunk_end; on return h_sc holds
// the status after the last replay that did work. The next replay is queued
// before the host reads the previous one's status, so that the device does
// not wait for the host between replays, unless the replay in flight is
// likely to end the chunk (the time left is under twice what the last replay
// covered). A replay queued after the stop time is reached does nothing: the
// device skips every step past it.
gd_status replay_chunk(gd_ctx* c, long long chunk_end) {
  int next = 0, head = 0, inflight = 0;
  long long t_prev = c->t_now, adv = 0;
  auto queue = [&]() -> gd_status {
    GD_TRY(c->hip(hipGraphLaunch(c->graph[next], c->stream), "graph launch"));
    GD_TRY(c->hip(hipEventRecord(c->ev_ring[next], c->stream), "status event"));
    next ^= 1;
    ++inflight;
    return GD_OK;
  };
  GD_TRY(queue());
  for (;;) {
    if (inflight == 1 && adv > 0 && chunk_end - t_prev > 2 * adv) GD_TRY(queue());
    GD_TRY(c->hip(hipEventSynchronize(c->ev_ring[head]), "status wait"));
    *c->h_sc = *c->h_ring[head];
    head ^= 1;
    --inflight;
    if (c->h_sc->nonfinite) {
      (void)hipStreamSynchronize(c->stream);
      return c->fail(GD_ENONFINITE, "non-finite acceleration or jerk");
    }
    report_progress(c);
    adv = c->h_sc->t_now - t_prev;
    t_prev = c->h_sc->t_now;
    if (c->h_sc->t_now >= chunk_end) return GD_OK;
    if (inflight == 0) GD_TRY(queue());
  }
}

}  // namespace

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
  if (!c->prof) {
    GD_TRY(build_graph(c, 0));
    GD_TRY(build_graph(c, 1));
  }
  c->phase = kIdle;
  c->prog_t0 = c->prog_last = std::chrono::steady_clock::now();
  c->prog_target = t_end;
  GD_TRY(read_sched(c));
  long long steps_before = c->h_sc->block_steps, pairs_before = c->h_sc->pairs;
  bool prepared = false;
  while (c->t_now < target) {
    // Advance to the next multiple of dt_max, where all particles meet.
    const long long chunk_end = (c->t_now / per_max + 1) * per_max;
    GD_TRY(c->hip(launch_set_tend(c->d, chunk_end, c->stream), "prepare"));
    if (!prepared) {
      // The list and j stream of the first step, for parity 0.
      GD_TRY(c->hip(launch_prepare(c->d, c->c, c->stream), "prepare kernel"));
      prepared = true;
    }
    if (!c->prof) {
      GD_TRY(replay_chunk(c, chunk_end));
      c->t_now = c->h_sc->t_now;
      double e[3];
      GD_TRY(energy_now(c, 0, e));
      c->e_last = e[0] + e[1];
      continue;
    }
    // Timing: the same steps as direct launches, 64 at a time, each force
    // launch between its own events and each step's N_act logged.
    for (;;) {
      for (int k = 0; k < kGraphSteps; ++k) {
        GD_TRY(enqueue_step(c, c->stream, k & 1, c->ev_s[k], c->ev_e[k]));
        GD_TRY(c->hip(launch_log_nact(c->d, c->d.nact_log + k, c->stream), "log kernel"));
      }
      GD_TRY(c->hip(hipMemcpyAsync(c->h_nact, c->d.nact_log, sizeof(int) * kGraphSteps,
                                   hipMemcpyDeviceToHost, c->stream),
                    "read log"));
      GD_TRY(read_sched(c));
      if (c->h_sc->nonfinite) return c->fail(GD_ENONFINITE, "non-finite acceleration or jerk");
      report_progress(c);
      // The steps that computed a force logged their N_act (the others, past
      // the stop time or rebuilding their list, logged 0).
      const long long ran = c->h_sc->block_steps - steps_before;
      long long timed = 0;
      for (int k = 0; k < kGraphSteps; ++k) {
        if (c->h_nact[k] <= 0) continue;
        float ms = 0.f;
        GD_TRY(c->hip(hipEventElapsedTime(&ms, c->ev_s[k], c->ev_e[k]), "event time"));
        c->prof_ms += ms;
        const int b = prof_bucket(c->h_nact[k]);
        c->bucket_ms[b] += ms;
        c->bucket_launches[b] += 1;
        c->bucket_pairs[b] += (long long)c->h_nact[k] * c->n;
        ++timed;
      }
      if (timed != ran) return c->fail(GD_EHIP, "force timing: %lld logged steps, %lld taken", timed, ran);
      c->prof_launches += ran;
      c->prof_pairs += c->h_sc->pairs - pairs_before;
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
  c->wall_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - c->prog_t0).count();
  if (st) GD_TRY(gd_stats_get(c, st));
  return GD_OK;
}

gd_status gd_progress(gd_ctx* c, double interval_s) {
  if (!c) return GD_EINVAL;
  if (!(interval_s >= 0.0) || !std::isfinite(interval_s))
    return c->fail(GD_EINVAL, "the progress interval must be finite and >= 0");
  c->progress_s = interval_s;
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

gd_status gd_diagnostics(gd_ctx* c, const double* fractions, int32_t n_frac, double* radii,
                         double* t_rh, double* r_half, int64_t* level_counts, int32_t n_levels) {
  if (!c) return GD_EINVAL;
  if (n_frac < 0 || n_frac > kMaxDiagFractions || (n_frac > 0 && (!fractions || !radii)) || n_levels < 0 ||
      (n_levels > 0 && !level_counts))
    return c->fail(GD_EINVAL, "bad fractions or level buffer");
  if (!c->synced || c->phase != kIdle)
    return c->fail(GD_ESTATE, "particles are not synchronised (use gd_step_to to a multiple of dt_max)");
  // Ascending fractions for the single pass; results are returned in the
  // caller's order.
  std::vector<std::pair<double, int>> fr;
  for (int q = 0; q < n_frac; ++q) {
    if (!(fractions[q] > 0.0 && fractions[q] <= 1.0)) return c->fail(GD_EINVAL, "fractions must be in (0, 1]");
    fr.push_back({fractions[q], q});
  }
  std::sort(fr.begin(), fr.end());
  double sorted[kMaxDiagFractions];
  for (int q = 0; q < n_frac; ++q) sorted[q] = fr[q].first;
  GD_TRY(c->hip(launch_diagnostics(c->d, c->c, sorted, n_frac, c->d.ebuf, c->stream), "diagnostics"));
  double out[kMaxDiagFractions + 2];
  GD_TRY(c->hip(hipMemcpyAsync(out, c->d.ebuf, sizeof(double) * (n_frac + 2), hipMemcpyDeviceToHost,
                               c->stream),
                "read diagnostics"));
  GD_TRY(read_sched(c));  // synchronises; also brings the level histogram
  for (int q = 0; q < n_frac; ++q) radii[fr[q].second] = out[q];
  if (t_rh) *t_rh = out[n_frac];
  if (r_half) *r_half = out[n_frac + 1];
  for (int k = 0; k < n_levels; ++k) level_counts[k] = k <= c->c.kmax ? c->h_sc->hist[k] : 0;
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
  c->wall_s = 0.0;
  c->phase = kIdle;
  // Synchronised only when every particle sits at t_now.
  c->synced = (tn % (1LL << c->c.kmax)) == 0;
  return GD_OK;
}

static_assert(GD_NACT_BINS == kNactBins, "histogram bins of the header and the schedule record");

gd_status gd_nact_histogram(gd_ctx* c, int64_t* counts) {
  if (!c) return GD_EINVAL;
  if (!counts) return c->fail(GD_EINVAL, "NULL argument");
  GD_TRY(read_sched(c));
  for (int b = 0; b < kNactBins; ++b) counts[b] = c->h_sc->nact_hist[b];
  return GD_OK;
}

gd_status gd_refills(gd_ctx* c, int64_t* refills) {
  if (!c) return GD_EINVAL;
  if (!refills) return c->fail(GD_EINVAL, "NULL argument");
  GD_TRY(read_sched(c));
  *refills = c->h_sc->refills;
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
  st->wall_s = c->wall_s;
  return GD_OK;
}

void gd_destroy(gd_ctx* c) {
  if (!c) return;
  for (int r = 0; r < 2; ++r) {
    if (c->graph[r]) (void)hipGraphExecDestroy(c->graph[r]);
    if (c->ev_ring[r]) (void)hipEventDestroy(c->ev_ring[r]);
    if (c->h_ring[r]) (void)hipHostFree(c->h_ring[r]);
  }
  if (c->ev_ready)
    for (int k = 0; k < kGraphSteps + 1; ++k) {
      (void)hipEventDestroy(c->ev_s[k]);
      (void)hipEventDestroy(c->ev_e[k]);
    }
  if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
  if (c->h_sc) (void)hipHostFree(c->h_sc);
  if (c->h_e) (void)hipHostFree(c->h_e);
  if (c->h_nact) (void)hipHostFree(c->h_nact);
  delete c;
}

const char* gd_last_error(const gd_ctx* c) {
  if (!c) return g_init_error.c_str();
  return c->err.c_str();
}

}  // extern "C"

// ===========================================================================
// Force evaluation without device allocation (gd_force_noalloc)
// ===========================================================================
//
// The arrays a context keeps in its workspace for one force evaluation (the
// schedule record, the j stream, the listed particles' state and the slice
// partials) live here in one file-scope device array per GPU. Host code never
// uses the array's name as an address: the first call on a device resolves
// that device's copy with hipGetSymbolAddress and keeps the pointer.

namespace {

constexpr long long kNoallocMaxN = GD_NOALLOC_MAX_N;

constexpr size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Byte offsets of the arrays of one call with n particles.
struct NoallocLayout {
  size_t sc, jm, p[3], pv[3], active, ip[3], ipv[3], part, total;
};

constexpr NoallocLayout noalloc_layout(long long n) {
  NoallocLayout L{};
  size_t off = 0;
  const size_t nd = sizeof(double) * (size_t)n;
  L.sc = off;
  off = align256(off + sizeof(Sched));
  L.jm = off;
  off = align256(off + nd);
  for (int d = 0; d < 3; ++d) {
    L.p[d] = off;
    off = align256(off + nd);
  }
  for (int d = 0; d < 3; ++d) {
    L.pv[d] = off;
    off = align256(off + nd);
  }
  L.active = off;
  off = align256(off + sizeof(int) * (size_t)n);
  for (int d = 0; d < 3; ++d) {
    L.ip[d] = off;
    off = align256(off + nd);
  }
  for (int d = 0; d < 3; ++d) {
    L.ipv[d] = off;
    off = align256(off + nd);
  }
  L.part = off;
  off = align256(off + sizeof(double) * 6 * (size_t)partial_rows(n, kIPerLane));
  L.total = off;
  return L;
}

// Every size up to the maximum fits: each offset grows with n.
constexpr size_t kNoallocScratchBytes = noalloc_layout(kNoallocMaxN).total;
static_assert(kNoallocMaxN < kLargeN, "calls of this size hold two i per lane, as contexts do");

}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// This device's copy of the scratch array (resolved once per device).
gd_status noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    g_init_error = std::string("current device: ") + hipGetErrorString(e);
    return GD_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    g_init_error = "device ordinal beyond the library's table";
    return GD_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      g_init_error = std::string("scratch address: ") + hipGetErrorString(e);
      return GD_EHIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return GD_OK;
}

}  // namespace

// The inputs of one gd_force_noalloc call in the force kernel's layout: the
// j stream (structure of arrays; masses with the central particle's zeroed),
// the listed particles' state by list position, and the schedule record of a
// step with those n_act particles. A listed index outside [0, n) gives its
// position a NaN state (so NaN output rows) and the list entry -1.
__global__ void k_noalloc_load(Dev d, int n, int bh, int ipl, const double* __restrict__ m,
                               const double* __restrict__ x, const double* __restrict__ v,
                               const int32_t* __restrict__ idx, int n_act) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t == 0) {
    Sched* sc = d.sc;
    sc->n_act = n_act;
    sc->done = 0;
    sc->nonfinite = 0;
    sc->bad_input = 0;
    sc->plan = make_plan(n_act, n, ipl);
  }
  if (t < n) {
    d.px[t] = x[3 * t]; d.py[t] = x[3 * t + 1]; d.pz[t] = x[3 * t + 2];
    d.pvx[t] = v[3 * t]; d.pvy[t] = v[3 * t + 1]; d.pvz[t] = v[3 * t + 2];
    if (bh >= 0) d.jm[t] = t == bh ? 0.0 : m[t];
  }
  if (t < n_act) {
    const int i = idx[t];
    const bool ok = i >= 0 && i < n;
    const int k = ok ? i : 0;
    const double nan = __builtin_nan("");
    d.active[t] = ok ? i : -1;
    d.ix[t] = ok ? x[3 * k] : nan;
    d.iy[t] = ok ? x[3 * k + 1] : nan;
    d.iz[t] = ok ? x[3 * k + 2] : nan;
    d.ivx[t] = ok ? v[3 * k] : nan;
    d.ivy[t] = ok ? v[3 * k + 1] : nan;
    d.ivz[t] = ok ? v[3 * k + 2] : nan;
  }
}

extern "C" {

gd_status gd_force_noalloc(const gd_params* p, int64_t n, const double* m, const double* x,
                           const double* v, const int32_t* idx, int64_t n_act, double* acc,
                           double* jerk, void* hip_stream) {
  auto bad = [](gd_status st, const char* msg) {
    g_init_error = msg;
    return st;
  };
  if (!p) return bad(GD_EINVAL, "NULL parameters");
  int kmax = 0;
  if (const char* why = check_params(p, n, &kmax)) return bad(GD_EINVAL, why);
  if (n > kNoallocMaxN) return bad(GD_EINVAL, "n exceeds GD_NOALLOC_MAX_N (65536)");
  if (n_act < 0 || n_act > n) return bad(GD_EINVAL, "n_act out of range");
  if (n_act == 0) return GD_OK;
  if (!m || !x || !v || !idx) return bad(GD_EINVAL, "NULL argument");
  void* base = nullptr;
  GD_TRY(noalloc_scratch(&base));

  const NoallocLayout L = noalloc_layout(n);
  char* w = (char*)base;
  Dev d{};
  d.sc = (Sched*)(w + L.sc);
  d.m = const_cast<double*>(m);  // read only
  d.jm = (double*)(w + L.jm);
  d.px = (double*)(w + L.p[0]);
  d.py = (double*)(w + L.p[1]);
  d.pz = (double*)(w + L.p[2]);
  d.pvx = (double*)(w + L.pv[0]);
  d.pvy = (double*)(w + L.pv[1]);
  d.pvz = (double*)(w + L.pv[2]);
  d.active = (int*)(w + L.active);
  d.ix = (double*)(w + L.ip[0]);
  d.iy = (double*)(w + L.ip[1]);
  d.iz = (double*)(w + L.ip[2]);
  d.ivx = (double*)(w + L.ipv[0]);
  d.ivy = (double*)(w + L.ipv[1]);
  d.ivz = (double*)(w + L.ipv[2]);
  d.part = (double*)(w + L.part);

  // The constants of a context of this size; the grids follow this call's
  // own decomposition (the kernels' results do not depend on the grid).
  Consts c = consts_of(p, n, kmax, kIPerLane);
  const Plan plan = make_plan((int)n_act, (int)n, kIPerLane);
  c.force_grid = std::min(plan.items, kForceGrid);
  const long long lanes = n_act * correct_lanes(plan.s);
  c.correct_grid = (int)std::min<long long>((lanes + kBlock - 1) / kBlock, kCorrectGrid);

  hipStream_t s = (hipStream_t)hip_stream;
  const int grid = (int)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(k_noalloc_load, dim3(grid), dim3(kBlock), 0, s, d, (int)n, c.bh, kIPerLane, m, x,
                     v, idx, (int)n_act);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = launch_force(d, c, s);
  if (e == hipSuccess) e = launch_reduce_out(d, c, acc, jerk, s);
  if (e != hipSuccess) {
    g_init_error = std::string("force launch: ") + hipGetErrorString(e);
    return GD_EHIP;
  }
  return GD_OK;
}

}  // extern "C"

// ===========================================================================
// Pools of independent clusters (continuous batching)
// ===========================================================================
//
// A pool owns one caller-provided arena: the device tables (slot descriptors,
// the table of resident clusters, the status array), then the clusters'
// workspaces, placed first-fit as clusters are admitted and freed as they
// are released. Admission is by footprint: a cluster is admitted when a slot
// and a gap of gd_workspace_bytes(n) bytes are free. One call of
// gd_pool_run replays a captured graph of kPoolSteps pool steps; each pool
// step advances every resident cluster by one of its own block steps, with
// one launch per phase for all of them. Clusters that reach their end time
// stop (their steps become no-ops) and are reported.

namespace {

constexpr int kPoolSteps = 32;  // pool steps per captured graph

struct PoolSlotHost {
  bool used = false;      // slot holds a cluster (running or finished)
  bool resident = false;  // in the device table (still stepping)
  int64_t n = 0;
  size_t off = 0, bytes = 0;  // workspace block in the arena
  long long t_end = 0;
  double e0 = 0.0;
  gd_status status = GD_OK;
  // host clock at admission and at retirement (the replay that finished it)
  std::chrono::steady_clock::time_point t_admit, t_done;
  Dev d{};
  Consts c{};
};

}  // namespace

struct gd_pool {
  gd_params p{};
  int kmax = 0;
  int max_clusters = 0;
  hipStream_t stream = nullptr;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  char* arena = nullptr;
  size_t arena_bytes = 0, heap_off = 0;
  PoolSlot* d_slots = nullptr;
  PoolTable* d_tab = nullptr;
  PoolStatus* d_status = nullptr;
  PoolWork* d_work = nullptr;
  PoolStatus* h_status = nullptr;  // pinned
  PoolTable* h_tab = nullptr;      // pinned staging
  PoolSlot* h_slot = nullptr;      // pinned staging
  double* h_e = nullptr;           // pinned energy result
  std::vector<PoolSlotHost> slots;
  std::string err;

  gd_status fail(gd_status st, const char* msg) {
    err = msg;
    return st;
  }
  gd_status hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return GD_OK;
    err = std::string(what) + ": " + hipGetErrorString(e);
    return GD_EHIP;
  }
};

namespace {

size_t pool_table_bytes(int max_clusters) {
  return align_up(sizeof(PoolSlot) * (size_t)max_clusters) + align_up(sizeof(PoolTable)) +
         align_up(sizeof(PoolStatus) * (size_t)max_clusters) + align_up(sizeof(PoolWork));
}

// First-fit placement of `bytes` in the arena heap, between the blocks of the
// clusters that hold slots.
bool pool_place(gd_pool* P, size_t bytes, size_t* off) {
  std::vector<std::pair<size_t, size_t>> blocks;
  for (const auto& s : P->slots)
    if (s.used) blocks.push_back({s.off, s.bytes});
  std::sort(blocks.begin(), blocks.end());
  size_t cur = P->heap_off;
  for (const auto& b : blocks) {
    if (b.first >= cur + bytes) break;
    cur = std::max(cur, align_up(b.first + b.second));
  }
  if (cur + bytes > P->arena_bytes) return false;
  *off = cur;
  return true;
}

// Uploads the table of resident clusters (stream-ordered).
gd_status pool_upload_table(gd_pool* P) {
  PoolTable& t = *P->h_tab;
  t.count = 0;
  int acc = 0;
  for (int sl = 0; sl < P->max_clusters; ++sl) {
    const PoolSlotHost& s = P->slots[sl];
    if (!s.resident) continue;
    t.order[t.count] = sl;
    t.pred_off[t.count] = acc;
    acc += (int)((s.n + kBlock - 1) / kBlock);
    ++t.count;
  }
  t.pred_off[t.count] = acc;
  GD_TRY(P->hip(hipMemcpyAsync(P->d_tab, P->h_tab, sizeof(PoolTable), hipMemcpyHostToDevice, P->stream),
                "upload pool table"));
  // The staging buffer is reused by the next call: wait for the copy.
  return P->hip(hipStreamSynchronize(P->stream), "synchronise");
}

gd_status pool_energy(gd_pool* P, PoolSlotHost& s, double* e) {
  GD_TRY(P->hip(launch_energy(s.d, s.c, 0, P->stream), "energy kernel"));
  const double* res = s.d.ebuf + 3 * (size_t)make_eplan(s.c.n).items;
  GD_TRY(P->hip(hipMemcpyAsync(P->h_e, res, 3 * sizeof(double), hipMemcpyDeviceToHost, P->stream),
                "read energy"));
  GD_TRY(P->hip(hipStreamSynchronize(P->stream), "synchronise"));
  *e = P->h_e[0] + P->h_e[1];
  return GD_OK;
}

gd_status pool_build_graph(gd_pool* P) {
  if (P->graph) return GD_OK;
  hipGraph_t g = nullptr;
  GD_TRY(P->hip(hipStreamBeginCapture(P->capture_stream, hipStreamCaptureModeThreadLocal),
                "begin capture"));
  hipError_t e = hipSuccess;
  for (int k = 0; k < kPoolSteps && e == hipSuccess; ++k)
    e = launch_pool_step(P->d_slots, P->d_tab, P->d_work, (P->p.flags & GD_FLAG_MIXED) != 0,
                         P->capture_stream);
  if (e == hipSuccess) e = launch_pool_status(P->d_slots, P->d_tab, P->d_status, P->capture_stream);
  hipError_t e2 = hipStreamEndCapture(P->capture_stream, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return P->hip(e != hipSuccess ? e : e2, "capture pool graph");
  }
  e = hipGraphInstantiate(&P->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return P->hip(e, "instantiate pool graph");
}

}  // namespace

extern "C" {

gd_status gd_pool_arena_bytes(int32_t max_clusters, const int64_t* n, int32_t count, size_t* bytes) {
  if (!bytes || max_clusters < 1 || max_clusters > kMaxPool || count < 0 || (count > 0 && !n))
    return GD_EINVAL;
  size_t b = pool_table_bytes(max_clusters);
  for (int k = 0; k < count; ++k) {
    if (n[k] < 2 || n[k] > (int64_t)std::numeric_limits<int>::max() / 2) return GD_EINVAL;
    b += make_layout(n[k], kIPerLaneLarge).total;
  }
  *bytes = b;
  return GD_OK;
}

gd_status gd_pool_create(gd_pool** out, const gd_params* p, int32_t max_clusters, void* arena,
                         size_t arena_bytes, void* hip_stream) {
  if (!out) return GD_EINVAL;
  *out = nullptr;
  auto bad = [](gd_status st, const char* msg) {
    g_init_error = msg;
    return st;
  };
  if (!p || !arena) return bad(GD_EINVAL, "NULL argument");
  if (max_clusters < 1 || max_clusters > kMaxPool) return bad(GD_EINVAL, "max_clusters must be in [1, 256]");
  int kmax = 0;
  if (const char* why = check_params(p, 2, &kmax)) return bad(GD_EINVAL, why);
  if (p->bh_index != -1 || !(p->eps > 0.0))
    return bad(GD_EINVAL, "pools take softened clusters without a central particle (eps > 0, bh_index = -1)");
  if (((uintptr_t)arena & 255) != 0) return bad(GD_EINVAL, "arena must be 256-byte aligned");
  if (arena_bytes < pool_table_bytes(max_clusters)) return bad(GD_ENOMEM, "arena smaller than the pool tables");
  gd_pool* P = new (std::nothrow) gd_pool();
  if (!P) return bad(GD_EINVAL, "out of host memory");
  P->p = *p;
  P->kmax = kmax;
  P->max_clusters = max_clusters;
  P->stream = (hipStream_t)hip_stream;
  P->arena = (char*)arena;
  P->arena_bytes = arena_bytes;
  P->slots.resize(max_clusters);
  size_t off = 0;
  P->d_slots = (PoolSlot*)(P->arena + off);
  off += align_up(sizeof(PoolSlot) * (size_t)max_clusters);
  P->d_tab = (PoolTable*)(P->arena + off);
  off += align_up(sizeof(PoolTable));
  P->d_status = (PoolStatus*)(P->arena + off);
  off += align_up(sizeof(PoolStatus) * (size_t)max_clusters);
  P->d_work = (PoolWork*)(P->arena + off);
  off += align_up(sizeof(PoolWork));
  P->heap_off = off;
  gd_status st = GD_OK;
  if (st == GD_OK) st = P->hip(hipHostMalloc((void**)&P->h_status, sizeof(PoolStatus) * max_clusters, 0), "pinned status");
  if (st == GD_OK) st = P->hip(hipHostMalloc((void**)&P->h_tab, sizeof(PoolTable), 0), "pinned table");
  if (st == GD_OK) st = P->hip(hipHostMalloc((void**)&P->h_slot, sizeof(PoolSlot), 0), "pinned slot");
  if (st == GD_OK) st = P->hip(hipHostMalloc((void**)&P->h_e, 4 * sizeof(double), 0), "pinned energy");
  if (st == GD_OK)
    st = P->hip(hipStreamCreateWithFlags(&P->capture_stream, hipStreamNonBlocking), "capture stream");
  if (st == GD_OK) st = pool_upload_table(P);
  if (st != GD_OK) {
    g_init_error = P->err;
    gd_pool_destroy(P);
    return st;
  }
  *out = P;
  return GD_OK;
}

gd_status gd_pool_admit(gd_pool* P, int64_t n, const double* m, const double* x, const double* v,
                        double t_end, int32_t* slot_out) {
  if (!P || !slot_out) return GD_EINVAL;
  *slot_out = -1;
  if (!m || !x || !v) return P->fail(GD_EINVAL, "NULL argument");
  int kmax = 0;
  if (const char* why = check_params(&P->p, n, &kmax)) return P->fail(GD_EINVAL, why);
  const double q = t_end / P->p.dt_max;
  if (!std::isfinite(t_end) || !(q > 0) || q != std::floor(q) || q > 9.0e15 / (1LL << kmax))
    return P->fail(GD_EINVAL, "t_end must be a positive multiple of dt_max");
  int sl = -1;
  for (int k = 0; k < P->max_clusters; ++k)
    if (!P->slots[k].used) {
      sl = k;
      break;
    }
  if (sl < 0) return P->fail(GD_ENOMEM, "no free slot");
  const Layout L = make_layout(n, ipl_for(&P->p, n));
  size_t off = 0;
  if (!pool_place(P, L.total, &off)) return P->fail(GD_ENOMEM, "no room in the arena");
  PoolSlotHost& s = P->slots[sl];
  s = PoolSlotHost();
  s.t_admit = std::chrono::steady_clock::now();
  s.used = true;
  s.n = n;
  s.off = off;
  s.bytes = L.total;
  s.t_end = (long long)q * (1LL << kmax);
  s.d = carve(P->arena + off, L);
  s.c = make_consts(&P->p, n, kmax, true);
  // Initialisation of the cluster (Sec. 2.4 steps 2-3) on the pool stream.
  auto undo = [&](gd_status st) {
    s = PoolSlotHost();
    return st;
  };
  gd_status st;
  if ((st = P->hip(launch_reset_sched(s.d, 0, P->stream), "reset")) != GD_OK) return undo(st);
  if ((st = P->hip(launch_load(s.d, s.c, m, x, v, P->stream), "load kernel")) != GD_OK) return undo(st);
  if ((st = P->hip(launch_predict(s.d, s.c, kPredAll, 0.0, P->stream), "predict kernel")) != GD_OK)
    return undo(st);
  if ((st = P->hip(launch_force(s.d, s.c, P->stream), "force kernel")) != GD_OK) return undo(st);
  if ((st = P->hip(launch_init_dt(s.d, s.c, P->stream), "init dt kernel")) != GD_OK) return undo(st);
  if ((st = P->hip(launch_set_tend(s.d, s.t_end, P->stream), "prepare")) != GD_OK) return undo(st);
  Sched chk;
  if ((st = P->hip(hipMemcpyAsync(&chk, s.d.sc, sizeof(Sched), hipMemcpyDeviceToHost, P->stream),
                   "read status")) != GD_OK)
    return undo(st);
  if ((st = P->hip(hipStreamSynchronize(P->stream), "synchronise")) != GD_OK) return undo(st);
  if (chk.bad_input) return undo(P->fail(GD_EINVAL, "non-finite or negative input (m, x or v)"));
  if (chk.nonfinite) return undo(P->fail(GD_ENONFINITE, "non-finite initial acceleration or jerk"));
  if ((st = pool_energy(P, s, &s.e0)) != GD_OK) return undo(st);
  // Descriptor, then the table that makes the cluster resident.
  P->h_slot->d = s.d;
  P->h_slot->c = s.c;
  if ((st = P->hip(hipMemcpyAsync(&P->d_slots[sl], P->h_slot, sizeof(PoolSlot), hipMemcpyHostToDevice,
                                  P->stream),
                   "upload slot")) != GD_OK)
    return undo(st);
  s.resident = true;
  if ((st = pool_upload_table(P)) != GD_OK) return undo(st);
  *slot_out = sl;
  return GD_OK;
}

gd_status gd_pool_run(gd_pool* P, int32_t* finished, int32_t* n_finished) {
  if (!P || !n_finished) return GD_EINVAL;
  *n_finished = 0;
  int resident = 0;
  for (const auto& s : P->slots) resident += s.resident;
  if (resident == 0) return GD_OK;
  GD_TRY(pool_build_graph(P));
  GD_TRY(P->hip(hipGraphLaunch(P->graph, P->stream), "pool graph launch"));
  GD_TRY(P->hip(hipMemcpyAsync(P->h_status, P->d_status, sizeof(PoolStatus) * P->max_clusters,
                               hipMemcpyDeviceToHost, P->stream),
                "read pool status"));
  GD_TRY(P->hip(hipStreamSynchronize(P->stream), "synchronise"));
  bool changed = false;
  for (int sl = 0; sl < P->max_clusters; ++sl) {
    PoolSlotHost& s = P->slots[sl];
    if (!s.resident) continue;
    const PoolStatus& st = P->h_status[sl];
    const bool failed = st.nonfinite != 0;
    if (st.t_now >= s.t_end || failed) {
      s.resident = false;
      s.t_done = std::chrono::steady_clock::now();
      s.status = failed ? GD_ENONFINITE : GD_OK;
      changed = true;
      if (finished) finished[*n_finished] = sl;
      ++*n_finished;
    }
  }
  if (changed) GD_TRY(pool_upload_table(P));
  return GD_OK;
}

gd_status gd_pool_result(gd_pool* P, int32_t sl, double* x, double* v, gd_stats* st) {
  if (!P || sl < 0 || sl >= P->max_clusters) return GD_EINVAL;
  PoolSlotHost& s = P->slots[sl];
  if (!s.used) return P->fail(GD_EINVAL, "slot holds no cluster");
  if (s.resident) return P->fail(GD_ESTATE, "cluster still running");
  if (s.status != GD_OK) return P->fail(s.status, "cluster produced a non-finite acceleration or jerk");
  if (x || v) GD_TRY(P->hip(launch_get_state(s.d, s.c, x, v, nullptr, nullptr, nullptr, nullptr, P->stream),
                            "get state"));
  if (st) {
    double e = 0.0;
    GD_TRY(pool_energy(P, s, &e));
    const PoolStatus& ps = P->h_status[sl];
    st->t = (double)ps.t_now * s.c.dt_min;
    st->block_steps = ps.block_steps;
    st->particle_steps = ps.particle_steps;
    st->pair_interactions = ps.pairs;
    st->dtmin_clamps = ps.clamps;
    st->e0 = s.e0;
    st->e = e;
    st->wall_s = std::chrono::duration<double>(s.t_done - s.t_admit).count();
  } else {
    GD_TRY(P->hip(hipStreamSynchronize(P->stream), "synchronise"));
  }
  return GD_OK;
}

gd_status gd_pool_release(gd_pool* P, int32_t sl) {
  if (!P || sl < 0 || sl >= P->max_clusters) return GD_EINVAL;
  PoolSlotHost& s = P->slots[sl];
  if (!s.used) return P->fail(GD_EINVAL, "slot holds no cluster");
  const bool was_resident = s.resident;
  s = PoolSlotHost();
  if (was_resident) GD_TRY(pool_upload_table(P));
  return GD_OK;
}

gd_status gd_pool_resident(gd_pool* P, int32_t* count) {
  if (!P || !count) return GD_EINVAL;
  int c = 0;
  for (const auto& s : P->slots) c += s.resident;
  *count = c;
  return GD_OK;
}

void gd_pool_destroy(gd_pool* P) {
  if (!P) return;
  if (P->graph) (void)hipGraphExecDestroy(P->graph);
  if (P->capture_stream) (void)hipStreamDestroy(P->capture_stream);
  if (P->h_status) (void)hipHostFree(P->h_status);
  if (P->h_tab) (void)hipHostFree(P->h_tab);
  if (P->h_slot) (void)hipHostFree(P->h_slot);
  if (P->h_e) (void)hipHostFree(P->h_e);
  delete P;
}

const char* gd_pool_last_error(const gd_pool* P) {
  if (!P) return g_init_error.c_str();
  return P->err.c_str();
}

}  // extern "C"
