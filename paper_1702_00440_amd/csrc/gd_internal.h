// Internal declarations shared by the kernels (gd_kernels.hip) and the C ABI
// runtime (gd_api.hip). Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gd {

// Launch geometry. Every kernel runs 256-lane workgroups (4 wave64s).
constexpr int kBlock = 256;
// j particles staged per LDS tile.
constexpr int kTileJ = 256;
// i particles held per lane by the force kernel: kIPerLane, or
// kIPerLaneLarge in contexts of at least kLargeN particles with eps > 0. More
// i per lane give each lane more independent pair chains and each LDS read
// of j more pairs, which long items repay; at smaller N the mid-size blocks
// are faster with 2 (and pools always use 2).
constexpr int kIPerLane = 2;
constexpr int kIPerLaneLarge = 4;
constexpr int kLargeN = 131072;
// Items the force decomposition aims for: slices are added (in powers of
// two) while i tiles times slices stays within kSliceItems, about two items
// per workgroup of the grid.
constexpr int kSliceItems = 2048;
// Fewest work units (i tiles times j tiles, times the i per lane) at which
// the decomposition stops widening the lanes per i.
constexpr int kMinUnits = 1536;
// Upper bound of the force grid: workgroups loop over items beyond it.
constexpr int kForceGrid = 1024;
// Upper bound of the corrector grid.
constexpr int kCorrectGrid = 2048;
// Shortest j slice (one LDS tile): it bounds the number of slice partials a
// particle has (N / kMinSlice). Small blocks shorten each lane's serial
// chain of pair evaluations with more lanes per i instead (LJ up to 64).
constexpr int kMinSlice = kTileJ;
// Smallest log2 of the lanes that share one i: i tiles hold at most
// (kBlock >> kMinLj) * ipl = 32 (or 64) particles, which keeps the number of
// j slices (and so the partial sums to reduce) small for large blocks.
constexpr int kMinLj = 4;
// Energy: i particles per lane from kEnergyLargeN particles on (one below,
// where four would leave most lanes idle), and the nominal number of
// workgroups a call is split into.
constexpr int kEnergyIPerLane = 4;
constexpr int kEnergyLargeN = 16384;
constexpr int kEnergyGrid = 1024;
// Maximum block-step level (dt = dt_max / 2^level).
constexpr int kMaxLevels = 41;

// Bins of the block-size histogram: bin b counts the block steps whose N_act
// lies in [2^b, 2^(b+1)).
constexpr int kNactBins = 32;

// Mass fractions one diagnostics call can take.
constexpr int kMaxDiagFractions = 32;

// Predictor modes.
enum : int { kPredAuto = 0, kPredAll = 1, kPredExplicit = 2 };

// Decomposition of one force launch over (i tile, j slice) items.
//   lj   : log2 of the lanes sharing one i (LJ = 1 << lj, 1..64, in one wave)
//   it   : i particles per workgroup tile = (kBlock >> lj) * ipl
//   nit  : number of i tiles
//   s    : number of j slices; item = itile * s + slice
//   len  : j particles per slice
struct Plan {
  int lj, it, nit, s, len, items;
};

// Device-resident scheduling and bookkeeping record (lives in the workspace).
//
// Block steps replayed from a graph run two kernels each (k_step_force,
// k_step_correct), and the step's parity (0/1, a kernel argument) picks one of
// two active lists: the corrector of a step predicts every particle to the
// speculated next block time and builds the next step's list in the other
// list, and the next force kernel checks the speculation (see k_step_force).
struct Sched {
  long long t_now;   // current block time, in dt_min ticks
  long long t_next;  // block time of the step in flight
  long long t_end;   // steps whose t_next would exceed this are skipped
  // The prepared list and j stream: (block time << 1) | list. One 64-bit word,
  // so that a kernel that reads it while another workgroup rewrites it sees
  // either the old pair or the new one.
  long long spec;
  int n_act;         // active particles of the step in flight
  int kthr;          // a particle is active when its level >= kthr
  int done;          // 1: the step in flight is skipped (t_end reached)
  int lcnt[2];       // compaction counters of the two active lists
  int nonfinite;     // set when a non-finite force or jerk is seen
  int bad_input;     // set by input / state validation
  int refill;        // 1: the step in flight rebuilt the list (no force, no correction)
  int fine;          // finest occupied level of the step in flight
  long long block_steps, particle_steps, pairs, clamps;
  long long refills;  // replayed steps that rebuilt their list instead of stepping
  long long nact_hist[kNactBins];  // block steps by floor(log2 N_act)
  Plan plan;                 // force decomposition of the step in flight
  int hist[kMaxLevels + 1];  // particles per level
};

// The plan depends only on (n_act, n). The kernel that fixes n_act for a
// step (predictor, or the explicit index list) stores it in the Sched record,
// and the force kernel and every slice reduction read that one copy.
// The decomposition with LJ = 2^lj lanes per i, ipl i per lane and at most
// s_req slices of whole LDS tiles (as many as keep each slice's tile count,
// with none empty).
__host__ __device__ inline Plan plan_with(int n_act, int n, int lj, int s_req, int ipl) {
  int tiles = (n + kTileJ - 1) / kTileJ;
  if (tiles < 1) tiles = 1;
  const int s0 = s_req < 1 ? 1 : (s_req > tiles ? tiles : s_req);
  // it and (in make_plan's plans) s0 are powers of two: shifts, not divisions
  const int lg_it = (8 - lj) + __builtin_ctz((unsigned)ipl);  // kBlock = 2^8
  const int tps = (s0 & (s0 - 1)) == 0 ? (tiles + s0 - 1) >> __builtin_ctz((unsigned)s0)
                                       : (tiles + s0 - 1) / s0;  // tiles per slice
  Plan p;
  p.lj = lj;
  p.it = (kBlock >> lj) * ipl;
  p.nit = (n_act + p.it - 1) >> lg_it;
  if (p.nit < 1) p.nit = 1;
  p.s = (tiles + tps - 1) / tps;
  p.len = tps * kTileJ;
  p.items = p.nit * p.s;
  return p;
}

// The decomposition make_plan considers at lj: slice count the largest power
// of two (at most one per tile) for which i tiles times slices stays within
// kSliceItems. *stop tells whether make_plan takes it: enough work units for
// the grid at this lj with i tiles at least half full, or the last
// candidate (LJ = 64).
__host__ __device__ inline Plan plan_for_lj(int n_act, int n, int lj, int ipl, bool* stop) {
  int tiles = (n + kTileJ - 1) / kTileJ;
  if (tiles < 1) tiles = 1;
  const int it = (kBlock >> lj) * ipl;
  int nit = (n_act + it - 1) >> ((8 - lj) + __builtin_ctz((unsigned)ipl));  // it = 2^(8 - lj) * ipl
  if (nit < 1) nit = 1;
  int s = 1;
  while (2 * s <= tiles && 2 * s * nit <= kSliceItems) s *= 2;
  *stop = lj == 6 || ((long long)nit * tiles * ipl >= kMinUnits && 2 * n_act >= nit * it);
  return plan_with(n_act, n, lj, s, ipl);
}

// The first lj from kMinLj up that gives enough work units (or the last one).
__host__ __device__ inline Plan make_plan(int n_act, int n, int ipl) {
  for (int lj = kMinLj;; ++lj) {
    bool stop = false;
    const Plan p = plan_for_lj(n_act, n, lj, ipl, &stop);
    if (stop) return p;
  }
}

// Rows of the partial-force buffer a context of n particles with ipl i per
// lane needs: for every plan, s * n_act <= s * nit * it <= max(nit,
// kSliceItems) * it with it <= (kBlock >> kMinLj) * ipl, and
// s * n_act <= (n / kMinSlice rounded up) * n. More i per lane never needs
// fewer rows.
constexpr long long partial_rows(long long n, int ipl) {
  const long long it_max = (long long)(kBlock >> kMinLj) * ipl;
  const long long by_items = n + it_max + (long long)kSliceItems * it_max;
  const long long by_slices = ((n + kMinSlice - 1) / kMinSlice) * n;
  const long long rows = by_items < by_slices ? by_items : by_slices;
  // Also scratch of the diagnostics sort: 1.5 * 2n + n / 64 + 8 doubles.
  return rows > n + 16 ? rows : n + 16;
}

// Energy decomposition: items are (i tile of kBlock * ipl, j slice). Slices
// are whole LDS tiles; about 8 items per workgroup of the nominal grid keep
// the tail of the launch short.
struct EPlan {
  int ipl, nit, s, len, items;
};
__host__ __device__ inline EPlan make_eplan(int n) {
  EPlan e;
  e.ipl = n >= kEnergyLargeN ? kEnergyIPerLane : 1;
  const int tile = kBlock * e.ipl;
  e.nit = (n + tile - 1) / tile;
  const int max_s = (n + kTileJ - 1) / kTileJ;
  int s = (8 * kEnergyGrid + e.nit - 1) / e.nit;
  if (s > max_s) s = max_s;
  if (s < 1) s = 1;
  e.s = s;
  e.len = (((n + s - 1) / s + kTileJ - 1) / kTileJ) * kTileJ;
  e.items = e.nit * s;
  return e;
}

// Device pointers of one context, carved from the caller's workspace.
struct Dev {
  Sched* sc;
  double* m;
  double* jm;                              // j-stream masses (central particle's zeroed)
  double *x, *y, *z, *vx, *vy, *vz;        // corrected state at t_i
  double *ax, *ay, *az, *jx, *jy, *jz;     // acceleration, jerk at t_i
  double *px, *py, *pz, *pvx, *pvy, *pvz;  // predicted j stream
  long long* tick;                         // t_i in dt_min ticks
  unsigned char* lev;                      // dt_i = dt_max / 2^lev
  // Two active lists, list q at offset q * n of each array (positions
  // 0..n_act-1), with the listed particles' predicted state, a and jerk at
  // t_i, and level, by position.
  int* active;
  double *ix, *iy, *iz, *ivx, *ivy, *ivz;
  double *iax, *iay, *iaz, *ijx, *ijy, *ijz;
  int* ilev;
  // tag[q * n + j]: the block time for which particle j was put in list q
  // (-1: never since the state was loaded).
  long long* tag;
  double* part;                            // [6][partial_rows(n)]: position * s + slot
  double* ebuf;                            // energy partials [items][3] + result [3]
  int* nact_log;                           // force-timing pass: N_act of each timed step
};

struct Consts {
  int n;
  int kmax;          // log2(dt_max / dt_min)
  int force_grid;    // workgroups of a force launch
  int correct_grid;  // workgroups of a corrector launch
  int bh;            // index of the central particle, -1 if none
  int mixed;         // 1: pair arithmetic in mixed precision (GD_FLAG_MIXED)
  double dt_min, dt_max, eta, eps2, eps2_bh;
  double inv_dt_min, inv_dt_max;  // exact reciprocals (powers of two)
  // The decomposition of a one-particle block (log2 lanes per i; j slices
  // s1), the force kernel's i count per lane, and the largest block size up
  // to which every block has the one-particle decomposition (at most
  // 65535), packed as lj1 | ipl << 8 | n1 << 16: one field more would split
  // the corrector's kernel-argument loads into two dependent batches (its
  // scalar registers are full).
  int lj1_ipl, s1;
  long long part_cs;  // component stride of the partial-force buffer (partial_rows(n, ipl))
};
__host__ __device__ inline int lj1_of(const Consts& c) { return c.lj1_ipl & 255; }
__host__ __device__ inline int ipl_of(const Consts& c) { return (c.lj1_ipl >> 8) & 255; }
__host__ __device__ inline int n1_of(const Consts& c) { return (int)((unsigned)c.lj1_ipl >> 16); }

// make_plan(n_act, n, ipl_of(c)) for n_act <= n1_of(c): the one-particle
// decomposition with the i tiles that n_act needs (a few shifts, where
// make_plan's search is a long dependent chain).
__host__ __device__ inline Plan one_plan(int n_act, int n, const Consts& c) {
  const int lj = lj1_of(c), ipl = ipl_of(c);
  const int tiles = (n + kTileJ - 1) / kTileJ;
  Plan p;
  p.lj = lj;
  p.it = (kBlock >> lj) * ipl;
  p.nit = (n_act + p.it - 1) >> ((8 - lj) + __builtin_ctz((unsigned)ipl));
  if (p.nit < 1) p.nit = 1;
  p.s = c.s1;
  p.len = ((tiles + c.s1 - 1) / c.s1) * kTileJ;
  p.items = p.nit * p.s;
  return p;
}

// Lanes the corrector gives one active particle: one per j slice of the
// force plan (rounded up to a power of two), at most a wave.
__host__ __device__ inline int correct_lanes(int s) {
  int l = 1;
  while (l < s && l < 64) l <<= 1;
  return l;
}

// Launch sizes for a context of n particles: enough workgroups for the
// largest force decomposition and corrector layout over all block sizes
// (sampled), capped; kernels loop over anything beyond the grid.
inline void launch_grids(int n, int ipl, int* force_grid, int* correct_grid) {
  long long fmax = 1, cmax = 1;
  const int step = n > 8192 ? n / 8192 : 1;
  for (int a = 1;; a += step) {
    if (a > n) a = n;
    const Plan p = make_plan(a, n, ipl);
    if (p.items > fmax) fmax = p.items;
    const long long lanes = (long long)a * correct_lanes(p.s);
    const long long wg = (lanes + kBlock - 1) / kBlock;
    if (wg > cmax) cmax = wg;
    if (a == n) break;
  }
  *force_grid = (int)(fmax < kForceGrid ? fmax : kForceGrid);
  *correct_grid = (int)(cmax < kCorrectGrid ? cmax : kCorrectGrid);
}

// ---------------------------------------------------------------------------
// Pools of independent clusters (continuous batching)
// ---------------------------------------------------------------------------
// A pool keeps up to kMaxPool clusters resident; one pool step advances every
// resident cluster by one of its own block steps, with one launch per phase
// (predict, force, correct) for all of them. The tables live in device memory
// at the head of the pool's arena.
constexpr int kMaxPool = 256;

struct PoolSlot {
  Dev d;
  Consts c;
};

struct PoolTable {
  int count;                   // resident clusters
  int order[kMaxPool];         // slot index of each resident cluster
  int pred_off[kMaxPool + 1];  // prefix sum of the clusters' predictor blocks
};

// A cluster's block step as the pool predictor fixed it: block size, block
// time and decomposition (what the force and corrector otherwise read from
// the cluster's record).
struct PoolStep {
  long long t_next;
  int n_act;
  Plan plan;
};

// Work of each resident cluster in the current pool step (by table
// position), written by the pool predictor for the force and corrector
// launches: force items, corrector workgroups (0 once the cluster is done)
// and the step itself.
struct PoolWork {
  int force_n[kMaxPool];
  int correct_n[kMaxPool];
  PoolStep step[kMaxPool];
};

// Per-slot status gathered after each batch of pool steps.
struct PoolStatus {
  long long t_now, block_steps, particle_steps, pairs, clamps;
  int done, nonfinite;
};

hipError_t launch_pool_step(const PoolSlot* slots, const PoolTable* tab, PoolWork* work, bool mixed,
                            hipStream_t s);
// Lagrange radii of the ascending fractions frac[0..n_frac) into out[0..n_frac),
// Eq. (5) into out[n_frac], the half-mass radius into out[n_frac + 1].
hipError_t launch_diagnostics(const Dev& d, const Consts& c, const double* frac, int n_frac,
                              double* out, hipStream_t s);
hipError_t launch_pool_status(const PoolSlot* slots, const PoolTable* tab, PoolStatus* out,
                              hipStream_t s);

// Launchers (gd_kernels.hip). Each returns the hipGetLastError() of its launch.
hipError_t launch_load(const Dev& d, const Consts& c, const double* m, const double* x,
                       const double* v, hipStream_t s);
hipError_t launch_predict(const Dev& d, const Consts& c, int mode, double t_explicit, hipStream_t s);
// ev_start/ev_stop (may be null): events that record the launch's own start
// and end (hipExtLaunchKernelGGL), for per-launch timing outside graphs.
hipError_t launch_force(const Dev& d, const Consts& c, hipStream_t s, hipEvent_t ev_start = nullptr,
                        hipEvent_t ev_stop = nullptr);
hipError_t launch_correct(const Dev& d, const Consts& c, hipStream_t s);
// The two kernels of a graph-replayed block step with parity par (see Sched).
hipError_t launch_step_force(const Dev& d, const Consts& c, int par, hipStream_t s,
                             hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
hipError_t launch_step_correct(const Dev& d, const Consts& c, int par, hipStream_t s);
// Predicts every particle to the next block time and builds list 0 for it,
// so that a step of parity 0 finds its list prepared.
hipError_t launch_prepare(const Dev& d, const Consts& c, hipStream_t s);
// Copies the N_act of the step in flight (0 if it was skipped or rebuilt its
// list) to *out.
hipError_t launch_log_nact(const Dev& d, int* out, hipStream_t s);
hipError_t launch_init_dt(const Dev& d, const Consts& c, hipStream_t s);
hipError_t launch_reduce_out(const Dev& d, const Consts& c, double* acc, double* jerk, hipStream_t s);
hipError_t launch_energy(const Dev& d, const Consts& c, int unsoft, hipStream_t s);
hipError_t launch_set_tend(const Dev& d, long long t_end, hipStream_t s);
hipError_t launch_reset_sched(const Dev& d, long long t_now, hipStream_t s);
// forced_lj > 0: the decomposition plan_with(n_act, n, forced_lj, forced_s)
// instead of make_plan's.
hipError_t launch_set_active(const Dev& d, const Consts& c, const int32_t* idx, int n_act, hipStream_t s,
                             int forced_lj = 0, int forced_s = 0);
hipError_t launch_copy_active(const Dev& d, const Consts& c, int32_t* idx, hipStream_t s);
hipError_t launch_get_state(const Dev& d, const Consts& c, double* x, double* v, double* a,
                            double* jerk, double* t_i, double* dt_i, hipStream_t s);
hipError_t launch_set_state(const Dev& d, const Consts& c, const double* x, const double* v,
                            const double* a, const double* jerk, const double* t_i,
                            const double* dt_i, long long t_now, hipStream_t s);

}  // namespace gd
