// HIP kernels for gfx950 (MI355X): the device side of the Hermite-4
// block-time-step integrator with Plummer softening of GraviDy
// (arXiv:1702.00440). Every step of the paper's integration scheme (Sec. 2.4,
// numbered step list) runs here: prediction of all particles, the active-set
// search, the O(N_act * N) acceleration and jerk, the Hermite corrector with
// the Aarseth block time step, and the O(N^2) energy.
//
// Layout: structure-of-arrays FP64 in one caller-owned workspace (gd_api.hip
// carves it). Times are integers in units of dt_min; a particle's step is
// dt_max / 2^lev, i.e. 2^(kmax - lev) ticks.
//
// Determinism: no floating-point atomics anywhere. Every sum has a fixed
// order that depends only on (n_act, n), never on scheduling or on the order
// of the active list, so results are bitwise reproducible.

#include <hip/hip_ext.h>

#include "gd_internal.h"

namespace gd {

// ---------------------------------------------------------------------------
// Pair arithmetic (FP64)
// ---------------------------------------------------------------------------

// 1/sqrt(s) to full FP64 accuracy. v_rsq_f64 alone is good to about 2^-24
// (measured), so one third-order step follows: with e = 1 - s y^2,
// y' = y (1 + e/2 + 3 e^2 / 8) is the Taylor series of y (1 - e)^(-1/2) and
// leaves a relative error of about (5/16) e^3, far below 2^-53.
__device__ __forceinline__ double rsqrt_fp64(double s) {
  double y = __builtin_amdgcn_rsq(s);
  double e = fma(-s, y * y, 1.0);
  double p = fma(e, 0.375, 0.5);
  return fma(y * e, p, y);
}

// Accumulators of one i particle: acceleration and jerk.
struct Acc6 {
  double ax, ay, az, jx, jy, jz;
};

// Contribution of particle j to particle i (Eq. (3) and its time derivative):
//   r = x_j - x_i, w = v_j - v_i, s = r.r + eps^2, q = s^(-1/2)
//   a    += m_j q^3 r
//   jerk += m_j q^3 (w - 3 (r.w) q^2 r)
__device__ __forceinline__ void pair_fp64(double xi, double yi, double zi, double vxi, double vyi,
                                          double vzi, double xj, double yj, double zj, double vxj,
                                          double vyj, double vzj, double mj, double eps2,
                                          Acc6& A) {
  const double dx = xj - xi, dy = yj - yi, dz = zj - zi;
  const double dvx = vxj - vxi, dvy = vyj - vyi, dvz = vzj - vzi;
  const double s = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
  const double rv = fma(dz, dvz, fma(dy, dvy, dx * dvx));
  const double q = rsqrt_fp64(s);
  const double q2 = q * q;
  const double mq3 = (mj * q) * q2;
  const double b3 = (rv * q2) * -3.0;
  A.ax = fma(mq3, dx, A.ax);
  A.ay = fma(mq3, dy, A.ay);
  A.az = fma(mq3, dz, A.az);
  const double wx = fma(b3, dx, dvx), wy = fma(b3, dy, dvy), wz = fma(b3, dz, dvz);
  A.jx = fma(mq3, wx, A.jx);
  A.jy = fma(mq3, wy, A.jy);
  A.jz = fma(mq3, wz, A.jz);
}

// FP32 acceleration sums of one i particle over one LDS tile (mixed precision).
struct Acc3f {
  float ax, ay, az;
};

// The same pair in mixed precision: the acceleration terms in FP32, the jerk
// in FP64. The scalar factors are FP64: the differences r = x_j - x_i and
// w = v_j - v_i, s = r.r + eps^2, r.w, and q = s^(-1/2) from v_rsq_f64 with
// one Newton step y (3 - s y^2) / 2 (relative error about 2^-47). m q^3 and r
// are rounded to FP32 once each; the acceleration terms m q^3 r are formed
// and summed in FP32 over each LDS tile (at most 256 / LJ terms per lane),
// and the caller adds the tile sums into FP64 accumulators. The jerk terms
// m q^3 (w - 3 (r.w) q^2 r) are formed and accumulated in FP64: a particle's
// jerk sum can cancel by two orders of magnitude, and FP32 terms (each
// rounded to about 6e-8 of its size) then miss a relative error of 2e-6.
__device__ __forceinline__ void pair_mixed(double xi, double yi, double zi, double vxi, double vyi,
                                           double vzi, double xj, double yj, double zj, double vxj,
                                           double vyj, double vzj, double mj, double eps2,
                                           Acc6& A, Acc3f& F) {
  const double dx = xj - xi, dy = yj - yi, dz = zj - zi;
  const double dvx = vxj - vxi, dvy = vyj - vyi, dvz = vzj - vzi;
  const double s = fma(dz, dz, fma(dy, dy, fma(dx, dx, eps2)));
  const double rv = fma(dz, dvz, fma(dy, dvy, dx * dvx));
  const double y = __builtin_amdgcn_rsq(s);
  const double q = fma(y * fma(-s, y * y, 1.0), 0.5, y);
  const double q2 = q * q;
  const double mq3 = (mj * q) * q2;
  const double b3 = (rv * q2) * -3.0;
  const float fm = (float)mq3;
  F.ax = fmaf(fm, (float)dx, F.ax);
  F.ay = fmaf(fm, (float)dy, F.ay);
  F.az = fmaf(fm, (float)dz, F.az);
  const double wx = fma(b3, dx, dvx), wy = fma(b3, dy, dvy), wz = fma(b3, dz, dvz);
  A.jx = fma(mq3, wx, A.jx);
  A.jy = fma(mq3, wy, A.jy);
  A.jz = fma(mq3, wz, A.jz);
}

// Value held by lane (lane ^ kOff) of the wave, kOff in {1, 2, 4, 8, 16, 32},
// by register-only lane exchanges instead of the LDS crossbar: DPP quad
// permutations (1, 2), a half-row mirror followed by a quad reversal (4), a
// row rotation by 8 (8), and the permlane16/32 swaps (16, 32), of which each
// lane takes the half that holds its partner. Every lane of the wave must be
// active. The partner is exactly lane ^ kOff, so a butterfly built on it sums
// in the same order as one built on __shfl_xor.
template <int kOff>
__device__ __forceinline__ int xor_partner_i(int v) {
  if constexpr (kOff == 1) {
    return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (kOff == 2) {
    return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (kOff == 4) {
    const int m = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    return __builtin_amdgcn_mov_dpp(m, 0x1B, 0xF, 0xF, false);         // quad_perm [3,2,1,0]
  } else if constexpr (kOff == 8) {
    return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (kOff == 16) {
    const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (threadIdx.x & 16) ? r[0] : r[1];
  } else {
    static_assert(kOff == 32, "lane exchange offsets are 1..32");
    const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (threadIdx.x & 32) ? r[0] : r[1];
  }
}

template <int kOff>
__device__ __forceinline__ double xor_partner_d(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)xor_partner_i<kOff>((int)(unsigned)b);
  const unsigned hi = (unsigned)xor_partner_i<kOff>((int)(unsigned)(b >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <int kOff, int kN>
__device__ __forceinline__ void xor_add(double (&v)[kN]) {
#pragma unroll
  for (int k = 0; k < kN; ++k) v[k] += xor_partner_d<kOff>(v[k]);
}

// The pair (a, b) combined with the pair of lane (lane ^ kOff): lanes with
// the kOff bit clear return a + a', lanes with it set b' + b (primes mark the
// partner's values), so each lane of an exchanging pair keeps one of the two
// sums. At offsets 16 and 32 one row swap per 32-bit word moves both halves
// (v_permlane16/32_swap exchange the odd rows of their first operand with the
// even rows of their second); smaller offsets send the half that the partner
// keeps. IEEE addition commutes, so both forms give the same value.
template <int kOff>
__device__ __forceinline__ double split_add(double a, double b) {
  if constexpr (kOff >= 16) {
    const unsigned long long ua = (unsigned long long)__double_as_longlong(a);
    const unsigned long long ub = (unsigned long long)__double_as_longlong(b);
    const int alo = (int)(unsigned)ua, ahi = (int)(unsigned)(ua >> 32);
    const int blo = (int)(unsigned)ub, bhi = (int)(unsigned)(ub >> 32);
    auto swap = [](int x, int y) {
      if constexpr (kOff == 16) return __builtin_amdgcn_permlane16_swap(x, y, false, false);
      else return __builtin_amdgcn_permlane32_swap(x, y, false, false);
    };
    const auto lo = swap(alo, blo);
    const auto hi = swap(ahi, bhi);
    const double r0 = __longlong_as_double(
        (long long)(((unsigned long long)(unsigned)hi[0] << 32) | (unsigned)lo[0]));
    const double r1 = __longlong_as_double(
        (long long)(((unsigned long long)(unsigned)hi[1] << 32) | (unsigned)lo[1]));
    return r0 + r1;
  } else {
    const bool up = (threadIdx.x & kOff) != 0;
    const double send = up ? a : b;
    const double keep = up ? b : a;
    return keep + xor_partner_d<kOff>(send);
  }
}

// Sum of v over each aligned group of g consecutive lanes (g a power of two,
// at most 64), left in every lane of the group: a butterfly with offsets
// g/2, ..., 1 (one uniform branch per level).
template <int kN>
__device__ __forceinline__ void group_sum(double (&v)[kN], int g) {
  if (g > 32) xor_add<32>(v);
  if (g > 16) xor_add<16>(v);
  if (g > 8) xor_add<8>(v);
  if (g > 4) xor_add<4>(v);
  if (g > 2) xor_add<2>(v);
  if (g > 1) xor_add<1>(v);
}

// Acceleration and jerk (f[0..2], f[3..5]) summed over each aligned group of
// kL consecutive lanes, left in every lane of the group: the first exchange
// keeps the acceleration in the lower half of the group and the jerk in the
// upper, a butterfly sums those 3 values over the half, and one more exchange
// gives each lane the other half's totals.
template <int kL>
__device__ __forceinline__ void force_sums(double (&f)[6]) {
  if constexpr (kL > 1) {
    double t[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) t[k] = split_add<kL / 2>(f[k], f[3 + k]);
    if constexpr (kL / 2 > 1) group_sum(t, kL / 2);
    const bool lower = (threadIdx.x & (kL / 2)) == 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double o = xor_partner_d<kL / 2>(t[k]);
      f[k] = lower ? t[k] : o;
      f[3 + k] = lower ? o : t[k];
    }
  }
}

// force_sums for a group size known at run time (a power of two up to 64).
__device__ __forceinline__ void force_sums(double (&f)[6], int L) {
  switch (L) {
    case 64: force_sums<64>(f); break;
    case 32: force_sums<32>(f); break;
    case 16: force_sums<16>(f); break;
    case 8: force_sums<8>(f); break;
    case 4: force_sums<4>(f); break;
    case 2: force_sums<2>(f); break;
    default: break;
  }
}

// ---------------------------------------------------------------------------
// Block time steps
// ---------------------------------------------------------------------------

// Smallest k >= 0 with dt_max / 2^k <= dtstar; kmax + 1 when even dt_min is
// too large (the caller clamps and counts); 0 when dtstar is not a number
// below dt_max (including +inf and NaN). With dtstar / dt_max = f 2^e,
// f in [0.5, 1), the answer is exactly 1 - e. dt_max is a power of two, so
// the quotient is the exact product with inv_dt_max = 1 / dt_max.
__device__ __forceinline__ int level_for(double dtstar, double dt_max, double inv_dt_max, int kmax) {
  if (!(dtstar < dt_max)) return 0;
  if (!(dtstar > 0.0)) return kmax + 1;
  int e;
  (void)frexp(dtstar * inv_dt_max, &e);
  return min(1 - e, kmax + 1);
}

__device__ __forceinline__ double norm3(double a, double b, double c) {
  return sqrt(a * a + b * b + c * c);
}

// Predicted position and velocity (Sec. 2.1): the Taylor series through the
// jerk over dt, as x + dt (v + dt/2 (a + dt/3 jerk)) and v + dt (a + dt/2 jerk).
// Every kernel that predicts uses this one sequence of operations.
__device__ __forceinline__ void taylor6(double dt, double x0, double y0, double z0, double vx0,
                                        double vy0, double vz0, double ax0, double ay0, double az0,
                                        double jx0, double jy0, double jz0, double o[6]) {
  const double h2 = 0.5 * dt, h3 = dt * (1.0 / 3.0);
  o[0] = fma(dt, fma(h2, fma(h3, jx0, ax0), vx0), x0);
  o[1] = fma(dt, fma(h2, fma(h3, jy0, ay0), vy0), y0);
  o[2] = fma(dt, fma(h2, fma(h3, jz0, az0), vz0), z0);
  o[3] = fma(dt, fma(h2, jx0, ax0), vx0);
  o[4] = fma(dt, fma(h2, jy0, ay0), vy0);
  o[5] = fma(dt, fma(h2, jz0, az0), vz0);
}

// Uses a value on a path that otherwise ignores it (an empty asm that takes
// it in a register). A load whose only uses lie past an early-exit branch
// would otherwise be moved below that branch, into a second round trip after
// the one that decides the branch; held on the exit path, it stays above and
// travels with the branch's own loads.
template <typename T>
__device__ __forceinline__ void hold(const T& v) {
  asm volatile("" ::"v"(v));
}

struct NextStep {
  long long t_next;
  int kthr, n_act, done;
  int fine;  // finest occupied level
};

// Sum over a wave (every lane gets it), by a register butterfly.
__device__ __forceinline__ int wave_sum(int v) {
  v += xor_partner_i<32>(v);
  v += xor_partner_i<16>(v);
  v += xor_partner_i<8>(v);
  v += xor_partner_i<4>(v);
  v += xor_partner_i<2>(v);
  v += xor_partner_i<1>(v);
  return v;
}

// The next block step from the level histogram (Sec. 2.4 steps 5-6),
// evaluated by one whole wave; lane l holds h = hist[l] (0 for l > kmax).
// Every particle of level k sits on a multiple of its step 2^(kmax-k) ticks,
// so the next block time is the next multiple of the smallest step present
// (the finest occupied level is the highest set bit of a ballot), the active
// particles are those with level >= kmax - ctz(t_next), and their number is
// the histogram's tail sum (a wave sum). Every lane returns the
// same result.
__device__ __forceinline__ NextStep next_step_wave(int h, int lane, int kmax, long long t_now,
                                                   long long t_end) {
  const unsigned long long occ = __ballot(h > 0);
  const int kmx = occ ? 63 - __clzll((long long)occ) : 0;
  const int sh = kmax - kmx;
  NextStep r;
  r.t_next = ((t_now >> sh) + 1) << sh;
  const int tz = __builtin_ctzll((unsigned long long)r.t_next);
  r.kthr = max(0, kmax - tz);
  // (read back from lane 0: the compiler then knows the count is uniform and
  // keeps the decomposition and the loops that depend on it scalar)
  r.n_act = __builtin_amdgcn_readfirstlane(wave_sum(lane >= r.kthr ? h : 0));
  r.done = r.t_next > t_end;
  r.fine = kmx;
  return r;
}

// make_plan evaluated by one whole wave: lane l tries lj = kMinLj + l with
// the same plan_for_lj, and the first lane that stops wins (its plan read
// back lane by lane), so every lane returns make_plan(n_act, n, ipl).
__device__ __forceinline__ Plan make_plan_wave(int n_act, int n, int ipl, int lane) {
  const int lj = kMinLj + lane;
  bool stop = false;
  Plan p{};
  if (lj <= 6) p = plan_for_lj(n_act, n, lj, ipl, &stop);
  const unsigned long long st = __ballot(stop);
  const int first = __ffsll((long long)st) - 1;
  Plan q;
  q.lj = __builtin_amdgcn_readlane(p.lj, first);
  q.it = __builtin_amdgcn_readlane(p.it, first);
  q.nit = __builtin_amdgcn_readlane(p.nit, first);
  q.s = __builtin_amdgcn_readlane(p.s, first);
  q.len = __builtin_amdgcn_readlane(p.len, first);
  q.items = __builtin_amdgcn_readlane(p.items, first);
  return q;
}

// A plan that every lane of the wave holds, read back from lane 0 so that its
// fields live in scalar registers.
__device__ __forceinline__ Plan uniform_plan(const Plan& p) {
  Plan q;
  q.lj = __builtin_amdgcn_readfirstlane(p.lj);
  q.it = __builtin_amdgcn_readfirstlane(p.it);
  q.nit = __builtin_amdgcn_readfirstlane(p.nit);
  q.s = __builtin_amdgcn_readfirstlane(p.s);
  q.len = __builtin_amdgcn_readfirstlane(p.len);
  q.items = __builtin_amdgcn_readfirstlane(p.items);
  return q;
}

// ---------------------------------------------------------------------------
// Active lists and prediction to a block time (shared by the predictor, the
// force kernel of a replayed step and its corrector)
// ---------------------------------------------------------------------------

// Positions in a list for the threads of the workgroup with take == true:
// ranks by wave ballot, one atomic on the list's counter per workgroup. Every
// thread of the workgroup must call it. The list order depends on which
// workgroup's atomic lands first, but no result depends on the order: a
// particle's force sums are the same at every list position.
__device__ __forceinline__ int wg_append(bool take, int* counter) {
  __shared__ int s_cnt[kBlock / 64];
  __shared__ int s_base;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const unsigned long long ball = __ballot(take);
  const int before = __popcll(ball & ((1ULL << lane) - 1ULL));
  if (lane == 0) s_cnt[wave] = __popcll(ball);
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      const int cw = s_cnt[w];
      s_cnt[w] = tot;
      tot += cw;
    }
    s_base = tot ? atomicAdd(counter, tot) : 0;
  }
  __syncthreads();
  const int pos = s_base + s_cnt[wave] + before;
  __syncthreads();  // the shared words are reused by the next call
  return pos;
}

// k_step_correct's view of a context's arrays: the first array of each group
// that the workspace layout places one stride apart (the state x .. jz, the j
// stream px .. pvz, the list arrays ix .. ijz), with the two strides. Array k
// of a group is addressed where it is used (st_arr, pj_arr, il_arr). Passing
// the 41 pointers of Dev, or computing them all when the kernel starts, left
// the kernel short of scalar registers: its argument loads came in dependent
// batches and many values were spilled to vector lanes.
struct DevC {
  Sched* sc;
  double *m, *jm, *st, *pj, *il, *part;
  long long* tick;
  unsigned char* lev;
  int *active, *ilev;
  long long* tag;
  long long sn, sl;  // strides in doubles: state and j stream; list arrays
};

// Array k of the state (x .. jz), j stream (px .. pvz) and list (ix .. ijz)
// groups, for either view (k is a constant at every use; the j stream has the
// first six).
enum : int { kX = 0, kY, kZ, kVx, kVy, kVz, kAx, kAy, kAz, kJx, kJy, kJz };
__device__ __forceinline__ double* st_arr(const Dev& d, int k) {
  double* const a[12] = {d.x, d.y, d.z, d.vx, d.vy, d.vz, d.ax, d.ay, d.az, d.jx, d.jy, d.jz};
  return a[k];
}
__device__ __forceinline__ double* pj_arr(const Dev& d, int k) {
  double* const a[6] = {d.px, d.py, d.pz, d.pvx, d.pvy, d.pvz};
  return a[k];
}
__device__ __forceinline__ double* il_arr(const Dev& d, int k) {
  double* const a[12] = {d.ix, d.iy, d.iz, d.ivx, d.ivy, d.ivz, d.iax, d.iay, d.iaz, d.ijx, d.ijy, d.ijz};
  return a[k];
}
__device__ __forceinline__ double* st_arr(const DevC& d, int k) { return d.st + k * d.sn; }
__device__ __forceinline__ double* pj_arr(const DevC& d, int k) { return d.pj + k * d.sn; }
__device__ __forceinline__ double* il_arr(const DevC& d, int k) { return d.il + k * d.sl; }

// Entry pos of list q: particle j with its predicted state o, its a and jerk
// at t_i and its level; and j's tag in list q (the block time of the step).
template <class D>
__device__ __forceinline__ void list_store(const D& d, int n, int q, int pos, int j, const double (&o)[6],
                                           double ax, double ay, double az, double jx, double jy, double jz,
                                           int lv, long long tag) {
  const size_t k = (size_t)q * n + pos;
  d.active[k] = j;
  il_arr(d, kX)[k] = o[0]; il_arr(d, kY)[k] = o[1]; il_arr(d, kZ)[k] = o[2];
  il_arr(d, kVx)[k] = o[3]; il_arr(d, kVy)[k] = o[4]; il_arr(d, kVz)[k] = o[5];
  il_arr(d, kAx)[k] = ax; il_arr(d, kAy)[k] = ay; il_arr(d, kAz)[k] = az;
  il_arr(d, kJx)[k] = jx; il_arr(d, kJy)[k] = jy; il_arr(d, kJz)[k] = jz;
  d.ilev[k] = lv;
  d.tag[(size_t)q * n + j] = tag;
}

// Stored state of one particle (corrected state, a and jerk at t_i, t_i, level).
struct PState {
  double x, y, z, vx, vy, vz, ax, ay, az, jx, jy, jz;
  long long tick;
  int lev;
};

template <class D>
__device__ __forceinline__ PState load_pstate(const D& d, int j) {
  PState p;
  p.x = st_arr(d, kX)[j]; p.y = st_arr(d, kY)[j]; p.z = st_arr(d, kZ)[j];
  p.vx = st_arr(d, kVx)[j]; p.vy = st_arr(d, kVy)[j]; p.vz = st_arr(d, kVz)[j];
  p.ax = st_arr(d, kAx)[j]; p.ay = st_arr(d, kAy)[j]; p.az = st_arr(d, kAz)[j];
  p.jx = st_arr(d, kJx)[j]; p.jy = st_arr(d, kJy)[j]; p.jz = st_arr(d, kJz)[j];
  p.tick = d.tick[j];
  p.lev = d.lev[j];
  return p;
}

// Particle j (valid) predicted over dt into the j stream (o receives the
// predicted state).
template <class D>
__device__ __forceinline__ void predict_store(const D& d, int j, double dt, const PState& p, double (&o)[6]) {
  taylor6(dt, p.x, p.y, p.z, p.vx, p.vy, p.vz, p.ax, p.ay, p.az, p.jx, p.jy, p.jz, o);
  pj_arr(d, kX)[j] = o[0]; pj_arr(d, kY)[j] = o[1]; pj_arr(d, kZ)[j] = o[2];
  pj_arr(d, kVx)[j] = o[3]; pj_arr(d, kVy)[j] = o[4]; pj_arr(d, kVz)[j] = o[5];
}

// The workgroup's particles [blk * kBlock, (blk + 1) * kBlock) predicted to
// block time t (ticks) into the j stream; those with level >= kthr appended
// to list q, tagged with t. p holds the thread's particle (loaded by the
// caller, index min(j, n - 1)).
__device__ __forceinline__ void predict_append(const Dev& d, const Consts& c, int blk, const PState& p,
                                               long long t, int kthr, int q) {
  const int j = blk * kBlock + threadIdx.x;
  bool act = false;
  double o[6];
  if (j < c.n) {
    predict_store(d, j, (double)(t - p.tick) * c.dt_min, p, o);
    act = p.lev >= kthr;
  }
  const int pos = wg_append(act, &d.sc->lcnt[q]);
  if (act) list_store(d, c.n, q, pos, j, o, p.ax, p.ay, p.az, p.jx, p.jy, p.jz, p.lev, t);
}

// The next block step from the Sched record, by one wave (next_step_wave):
// every lane returns the same result.
__device__ __forceinline__ NextStep schedule_wave(const Sched* __restrict__ sc, const Consts& c) {
  const int lane = threadIdx.x & 63;
  const int h = lane <= c.kmax ? sc->hist[lane] : 0;
  return next_step_wave(h, lane, c.kmax, sc->t_now, sc->t_end);
}

// ---------------------------------------------------------------------------
// Force kernel: O(N_act * N) acceleration and jerk (Sec. 2.4 step 7(c), Sec. 2.5)
// ---------------------------------------------------------------------------
//
// One launch shape serves every block size. The decomposition (make_plan)
// is computed on the device from n_act, so a captured graph never needs the
// host to know the block size:
//   - items are (i tile, j slice) pairs; workgroups loop over items;
//   - inside a workgroup, LJ = 2^lj consecutive lanes share the same i
//     particles and split the slice's j between them (LJ = 16 for most block
//     sizes, up to 64 inside one wave);
//   - each lane holds kI i particles (2, or 4 in large contexts), so one LDS read of j feeds
//     several pair evaluations;
//   - j particles of the slice go through LDS in tiles of kTileJ, loaded
//     with coalesced SoA reads and prefetched into registers one tile ahead;
//   - the LJ lanes of one i pair reduce their sums by halving (quarter_sums)
//     inside the wave, and each slice writes its partial sum to
//     part[component][position][slot], so that the slices of one particle
//     are contiguous for the reduction (slice_slot keeps the slices that one
//     XCD computes next to each other).
// The slices of a particle are summed afterwards by the kernel that consumes
// the force (corrector, initial steps, or output), in an order that depends
// only on (n_act, n).
// i particles of one lane: predicted state, index, softening, accumulators.
template <int kI>
struct ILane {
  double x[kI], y[kI], z[kI];
  double vx[kI], vy[kI], vz[kI], e2[kI];
  int g[kI], pos[kI];
  Acc6 A[kI];
  Acc3f Af[kI];  // mixed precision: acceleration sums of the current tile
};

// Pairs of one LDS tile of cnt j (first index jt). Lane jsub of each group of
// LJ lanes takes j = jsub, jsub + LJ, ...: a uniform trip count over whole
// groups of LJ (scalar loop control, no per-lane exit masks), then at most
// one partial group.
template <bool kMaskSelf, bool kMixed, int kI>
__device__ __forceinline__ void tile_pairs(const double (*sj)[kTileJ], int cnt, int LJ, int jsub,
                                           int jt, double eps2, ILane<kI>& I) {
  const int full = cnt & ~(LJ - 1);
  if (kMixed) {
#pragma unroll
    for (int q = 0; q < kI; ++q) I.Af[q] = Acc3f{0.f, 0.f, 0.f};
  }
  auto pairs_with = [&](int k) {
    const double xj = sj[0][k], yj = sj[1][k], zj = sj[2][k];
    const double vxj = sj[3][k], vyj = sj[4][k], vzj = sj[5][k];
    const double mj = sj[6][k];
#pragma unroll
    for (int q = 0; q < kI; ++q) {
      // eps = 0: the j = i term (r = 0) is excluded explicitly; with eps > 0
      // it is exactly zero (r = w = 0, finite q).
      const bool self = kMaskSelf && (jt + k) == I.g[q];
      const double xjq = self ? I.x[q] + 1.0 : xj;
      if (kMixed) {
        pair_mixed(I.x[q], I.y[q], I.z[q], I.vx[q], I.vy[q], I.vz[q], xjq, yj, zj, vxj, vyj, vzj,
                   self ? 0.0 : mj, kMaskSelf ? eps2 : I.e2[q], I.A[q], I.Af[q]);
      } else {
        pair_fp64(I.x[q], I.y[q], I.z[q], I.vx[q], I.vy[q], I.vz[q], xjq, yj, zj, vxj, vyj, vzj,
                  self ? 0.0 : mj, kMaskSelf ? eps2 : I.e2[q], I.A[q]);
      }
    }
  };
#pragma unroll 2
  for (int kk = 0; kk < full; kk += LJ) pairs_with(kk + jsub);
  if (full + jsub < cnt) pairs_with(full + jsub);
  if (kMixed) {
    // At most kTileJ / LJ acceleration terms per lane in FP32, then into FP64.
#pragma unroll
    for (int q = 0; q < kI; ++q) {
      I.A[q].ax += (double)I.Af[q].ax;
      I.A[q].ay += (double)I.Af[q].ay;
      I.A[q].az += (double)I.Af[q].az;
    }
  }
}

// Storage slot of slice sl among the s slices of one particle. When s is a
// multiple of 8, item and workgroup index agree mod 8, so slice sl runs on
// XCD sl % 8; its slices are stored together, and each XCD's L2 writes back
// whole sectors instead of 8-byte pieces of lines that all eight share.
__device__ __forceinline__ int slice_slot(int sl, int s) {
  return (s & 7) ? sl : (sl & 7) * (s >> 3) + (sl >> 3);
}

// The 12 sums of a group of kLJ lanes that share two i (acceleration and
// jerk of each) reduced over the group by halving: the first exchange keeps
// the first i in the lower half of the group and the second in the upper
// half, the next keeps the acceleration in the lower quarter of each half and
// the jerk in the upper, and a butterfly sums the remaining 3 values over the
// quarter. Every lane of quarter k ends with the totals of block k of 3.
template <int kLJ>
__device__ __forceinline__ void quarter_sums(const double (&v)[12], double (&t)[3]) {
  double h[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) h[k] = split_add<kLJ / 2>(v[k], v[6 + k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) t[k] = split_add<kLJ / 4>(h[k], h[3 + k]);
  if constexpr (kLJ / 8 >= 1) group_sum(t, kLJ / 4);
}

// The 24 sums of a group of kLJ lanes that share four i, reduced the same
// way: the first exchange keeps i 0-1 in the lower half of the group and
// i 2-3 in the upper, the next keeps the first i of each pair in the lower
// quarter of the half, the next the acceleration in the lower eighth of the
// quarter, and a butterfly sums the remaining 3 values over the eighth.
template <int kLJ>
__device__ __forceinline__ void eighth_sums(const double (&v)[24], double (&t)[3]) {
  double h[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) h[k] = split_add<kLJ / 2>(v[k], v[12 + k]);
  double u[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) u[k] = split_add<kLJ / 4>(h[k], h[6 + k]);
#pragma unroll
  for (int k = 0; k < 3; ++k) t[k] = split_add<kLJ / 8>(u[k], u[3 + k]);
  if constexpr (kLJ / 16 >= 1) group_sum(t, kLJ / 8);
}

// Reduction over the LJ lanes that share the lane's kI i (consecutive lanes),
// then the slice partials by list position: each 3-vector (one i's
// acceleration or jerk) is stored by the first lane of the part of the group
// that holds it (LJ / (2 kI) lanes). The central particle's pairs (softened
// with eps_bh, once per i, on slice 0; bx.. its predicted state) are added to
// the first lane's sums before the reduction.
template <bool kCentral, int kI>
__device__ __forceinline__ void finish_item(const Dev& d, const Consts& c, int LJ, int jsub,
                                            int slice, int s, int n_act, ILane<kI>& I, double bx,
                                            double by, double bz, double bvx, double bvy,
                                            double bvz) {
  static_assert(kI == 2 || kI == 4, "the reduction splits the sums of two or four i");
  if (kCentral && slice == 0 && jsub == 0) {
    const int b = c.bh;
    const double bm = d.m[b];
#pragma unroll
    for (int q = 0; q < kI; ++q)
      if (I.g[q] != b)
        pair_fp64(I.x[q], I.y[q], I.z[q], I.vx[q], I.vy[q], I.vz[q], bx, by, bz, bvx, bvy, bvz, bm,
                  c.eps2_bh, I.A[q]);
  }
  double v[6 * kI];
#pragma unroll
  for (int q = 0; q < kI; ++q) {
    v[6 * q + 0] = I.A[q].ax; v[6 * q + 1] = I.A[q].ay; v[6 * q + 2] = I.A[q].az;
    v[6 * q + 3] = I.A[q].jx; v[6 * q + 4] = I.A[q].jy; v[6 * q + 5] = I.A[q].jz;
  }
  double t[3];
  if constexpr (kI == 2) {
    if (LJ == 64) quarter_sums<64>(v, t);
    else if (LJ == 32) quarter_sums<32>(v, t);
    else quarter_sums<16>(v, t);
  } else {
    if (LJ == 64) eighth_sums<64>(v, t);
    else if (LJ == 32) eighth_sums<32>(v, t);
    else eighth_sums<16>(v, t);
  }
  const int part = LJ / (2 * kI);  // lanes that end with one 3-vector
  if ((jsub & (part - 1)) == 0) {
    // which i: the half, then (four i) the quarter; acceleration or jerk: the
    // lower or upper part within that
    const int q = kI == 2 ? (jsub >= LJ / 2) : 2 * (jsub >= LJ / 2) + ((jsub & (LJ / 4)) != 0);
    const int comp = (jsub & part) ? 3 : 0;
    // (explicit selects: an indexed read would keep the lane's i in memory)
    int pos;
    if constexpr (kI == 2) pos = q ? I.pos[1] : I.pos[0];
    else pos = q == 0 ? I.pos[0] : q == 1 ? I.pos[1] : q == 2 ? I.pos[2] : I.pos[3];
    if (pos < n_act) {
      // part[component][position][slot], components part_cs apart
      const size_t cs = (size_t)c.part_cs;
      double* o = d.part + (size_t)pos * s + slice_slot(slice, s) + comp * cs;
      o[0 * cs] = t[0];
      o[1 * cs] = t[1];
      o[2 * cs] = t[2];
    }
  }
}

// kStep: the force kernel of a graph-replayed block step (k_step_force), with
// the active list of parity par; otherwise that of a step whose predictor ran
// before (list 0).
template <bool kMaskSelf, bool kCentral, bool kMixed, int kI, bool kStep = false>
__device__ __forceinline__ void force_body(const Dev& d, const Consts& c, int blk, int nblk, int par = 0,
                                           const PoolStep* step = nullptr) {
  Sched* __restrict__ sc = d.sc;
  const int n = c.n;
  const size_t lo = (size_t)par * n;  // list offset
  const double* __restrict__ px = d.px;
  const double* __restrict__ py = d.py;
  const double* __restrict__ pz = d.pz;
  const double* __restrict__ pvx = d.pvx;
  const double* __restrict__ pvy = d.pvy;
  const double* __restrict__ pvz = d.pvz;
  // With a central particle its mass is zero in the j stream (jm); its pairs
  // are added separately with their own softening.
  const double* __restrict__ pm = kCentral ? d.jm : d.m;

  __shared__ double sj[7][kTileJ];
  const int tid = threadIdx.x;

  // The i particles of an item. The predicted state of the active list is
  // stored by list position (one load level instead of an index gather).
  // Positions past the list read entry kc instead: any entry in bounds
  // serves, since their sums are never stored.
  ILane<kI> I;
  auto load_i = [&](int itile, int it, int ilane, int ilanes, int kc) {
#pragma unroll
    for (int q = 0; q < kI; ++q) {
      I.pos[q] = itile * it + ilane + q * ilanes;
      const size_t k = lo + min(I.pos[q], kc);
      I.g[q] = (kMaskSelf || kCentral) ? d.active[k] : 0;
      // Softening enters only as the addend of r.r, so a per-i value costs
      // nothing: the central particle takes eps_bh for all of its pairs.
      I.e2[q] = (kCentral && I.g[q] == c.bh) ? c.eps2_bh : c.eps2;
      I.x[q] = d.ix[k];
      I.y[q] = d.iy[k];
      I.z[q] = d.iz[k];
      I.vx[q] = d.ivx[k];
      I.vy[q] = d.ivy[k];
      I.vz[q] = d.ivz[k];
      I.A[q] = Acc6{0, 0, 0, 0, 0, 0};
    }
  };
  // Tile loads and LDS stores are lane-uniform (indices clamped into the
  // slice, lanes past its end store a duplicate that is never read): the
  // i loads are then drained on every path before the first tile, and the
  // inner loop does not wait on the prefetch of the next tile.
  static_assert(kTileJ == kBlock, "one j per thread per tile");
  double rx = 0, ry = 0, rz = 0, rvx = 0, rvy = 0, rvz = 0, rm = 0;
  auto load_tile = [&](int base, int j1) {
    const int j = min(base + tid, j1 - 1);
    rx = px[j]; ry = py[j]; rz = pz[j];
    rvx = pvx[j]; rvy = pvy[j]; rvz = pvz[j];
    rm = pm[j];
  };

  // Small blocks share the decomposition of a one-particle block (lj1, s1),
  // which n alone fixes: one i tile, whose items are the first s1
  // workgroups. Those request their item before the schedule record is
  // read, so that the two memory round trips overlap; a step with another
  // decomposition loads its items afresh.
  const bool spec = blk < c.s1;
  if (spec) {
    // Slices are whole tiles: s1 slices of ceil(tiles / s1) tiles each (the
    // slice length of plan_with for that slice count).
    const int tiles = (n + kTileJ - 1) / kTileJ;
    const int len1 = ((tiles + c.s1 - 1) / c.s1) * kTileJ;
    const int j0 = blk * len1, j1 = min(n, j0 + len1);
    const int lj1 = lj1_of(c);
    load_i(0, (kBlock >> lj1) * kI, tid >> lj1, kBlock >> lj1, n - 1);
    if (j0 < j1) load_tile(j0, j1);
  }

  int n_act;
  Plan p;
  if constexpr (kStep) {
    // The step from the level histogram, in every wave (each wave gets the
    // same result), then the check of the prepared list and j stream.
    const NextStep nx = schedule_wave(sc, c);
    // A plain 64-bit load (one access: either the old word or the new one);
    // an agent-scope atomic load would bypass the caches.
    const long long word = __hip_atomic_load(&sc->spec, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    // (the word is the same in every lane; from lane 0 the branches on it are
    // uniform)
    const long long prepared =
        (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(word >> 32)) << 32) |
                    (unsigned)__builtin_amdgcn_readfirstlane((int)word));
    if (nx.done) {
      if (blk == 0 && tid == 0) {
        sc->done = 1;
        sc->refill = 0;
      }
      return;
    }
    if (prepared != ((nx.t_next << 1) | par)) {
      // The corrector of the previous step predicted another block time, or
      // prepared the other list: predict every particle to t_next and build
      // list par ^ 1 instead of a force. The corrector then does nothing,
      // and the next step (parity par ^ 1) finds its list prepared. A
      // workgroup that reads the new record sees the other list as prepared
      // and takes this path as well.
      for (int b = blk; b < (n + kBlock - 1) / kBlock; b += nblk) {
        const PState ps = load_pstate(d, min(b * kBlock + tid, n - 1));
        predict_append(d, c, b, ps, nx.t_next, nx.kthr, par ^ 1);
      }
      if (blk == 0 && tid == 0) {
        __hip_atomic_store(&sc->spec, (nx.t_next << 1) | (par ^ 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sc->refill = 1;
        sc->done = 0;
      }
      return;
    }
    n_act = nx.n_act;
    p = n_act <= n1_of(c) ? one_plan(n_act, n, c) : make_plan_wave(n_act, n, ipl_of(c), tid & 63);
    p = uniform_plan(p);
    if (blk == 0 && tid == 0) {
      sc->t_next = nx.t_next;
      sc->kthr = nx.kthr;
      sc->n_act = n_act;
      sc->plan = p;
      sc->fine = nx.fine;
      sc->done = 0;
      sc->refill = 0;
    }
  } else if (step) {
    // a pool launch: the step as its predictor fixed it (only clusters that
    // have work get items)
    n_act = __builtin_amdgcn_readfirstlane(step->n_act);
    p = uniform_plan(step->plan);
  } else {
    if (__builtin_amdgcn_readfirstlane(sc->done)) return;
    n_act = __builtin_amdgcn_readfirstlane(sc->n_act);
    if (n_act <= 0) return;
    p = uniform_plan(sc->plan);
  }
  if (blk >= p.items) return;
  // Same lanes per i and slices: same tile size, slice length and item map.
  const bool early = spec && p.lj == lj1_of(c) && p.s == c.s1;
  const int LJ = 1 << p.lj;
  const int jsub = tid & (LJ - 1);
  const int ilane = tid >> p.lj;
  const int ilanes = kBlock >> p.lj;

  for (int item = blk; item < p.items; item += nblk) {
    const int itile = item / p.s;
    const int slice = item - itile * p.s;
    const int j0 = slice * p.len;
    const int j1 = min(n, j0 + p.len);
    if (item != blk || !early) {
      load_i(itile, p.it, ilane, ilanes, n_act - 1);
      if (j0 < j1) load_tile(j0, j1);
    }
    for (int jt = j0; jt < j1; jt += kTileJ) {
      const int cnt = min(kTileJ, j1 - jt);
      __syncthreads();
      sj[0][tid] = rx; sj[1][tid] = ry; sj[2][tid] = rz;
      sj[3][tid] = rvx; sj[4][tid] = rvy; sj[5][tid] = rvz;
      sj[6][tid] = rm;
      __syncthreads();
      if (jt + kTileJ < j1) load_tile(jt + kTileJ, j1);
      tile_pairs<kMaskSelf, kMixed, kI>(sj, cnt, LJ, jsub, jt, c.eps2, I);
    }
    double bx = 0, by = 0, bz = 0, bvx = 0, bvy = 0, bvz = 0;
    if (kCentral) {
      const int b = c.bh;
      bx = px[b]; by = py[b]; bz = pz[b];
      bvx = pvx[b]; bvy = pvy[b]; bvz = pvz[b];
    }
    finish_item<kCentral, kI>(d, c, LJ, jsub, slice, p.s, n_act, I, bx, by, bz, bvx, bvy, bvz);
  }
}

template <bool kMaskSelf, bool kCentral, bool kMixed, int kI>
__global__ __launch_bounds__(kBlock) void k_force(Dev d, Consts c) {
  force_body<kMaskSelf, kCentral, kMixed, kI>(d, c, blockIdx.x, gridDim.x);
}

// The force kernel of a graph-replayed block step of parity par (see Sched).
template <bool kMaskSelf, bool kCentral, bool kMixed, int kI>
__global__ __launch_bounds__(kBlock) void k_step_force(Dev d, Consts c, int par) {
  force_body<kMaskSelf, kCentral, kMixed, kI, true>(d, c, blockIdx.x, gridDim.x, par);
}

// ---------------------------------------------------------------------------
// Slice reduction and per-particle finishing
// ---------------------------------------------------------------------------

// The s slice partials of active position k (contiguous in
// part[component][position][slot]), summed by the L consecutive lanes of a
// group (lane r takes slots r, r + L, ...: coalesced) and combined across
// the group by force_sums, in a fixed order: every lane of the group ends
// with the totals. One memory round trip instead of s dependent ones. All
// lanes of the wave must call it (valid == false contributes zeros).
__device__ __forceinline__ void reduce_slices(const double* __restrict__ part, int s, long long cs,
                                              int k, int L, int r, bool valid, double (&f)[6]) {
#pragma unroll
  for (int q = 0; q < 6; ++q) f[q] = 0.0;
  if (valid) {
    const double* o = part + (size_t)k * s;
    for (int sl = r; sl < s; sl += L) {
#pragma unroll
      for (int q = 0; q < 6; ++q) f[q] += o[q * cs + sl];
    }
  }
  force_sums(f, L);
}

// Workgroup-local bookkeeping, flushed to the Sched record with one atomic
// per field and workgroup.
struct LocalBook {
  int hist[kMaxLevels + 1];
  int clamp, bad;
};

__device__ __forceinline__ void book_init(LocalBook& b, int tid) {
  if (tid <= kMaxLevels) b.hist[tid] = 0;
  if (tid == 0) { b.clamp = 0; b.bad = 0; }
}

__device__ __forceinline__ void book_flush(LocalBook& b, Sched* sc, int kmax, int tid) {
  if (tid <= kmax && b.hist[tid] != 0) atomicAdd(&sc->hist[tid], b.hist[tid]);
  if (tid == 0) {
    if (b.clamp) atomicAdd((unsigned long long*)&sc->clamps, (unsigned long long)b.clamp);
    if (b.bad) atomicOr(&sc->nonfinite, 1);
  }
}

__device__ __forceinline__ bool finite6(const double f[6]) {
  bool ok = true;
#pragma unroll
  for (int q = 0; q < 6; ++q) ok = ok && isfinite(f[q]);
  return ok;
}

// ---------------------------------------------------------------------------
// Corrector and new block step (Sec. 2.4 step 7(d); Sec. 3.2)
// ---------------------------------------------------------------------------
//
// Per active particle: the summed new force (a1, j1); Hermite interpolation
// of (a0, j0, a1, j1) over h gives the 2nd and 3rd derivatives a2, a3 at the
// start of the step; corrected
//   x = x_p + a2 h^4/24 + a3 h^5/120,  v = v_p + a2 h^3/6 + a3 h^4/24;
// new step from the Aarseth criterion with the derivatives carried to the end
// of the step, quantised to a power of two (shrink freely, grow by one level
// only where the doubled step divides the new time, clamp at dt_min).
// Everything the particle needs (slice partials, predicted state, a0, j0,
// level) is read by list position in one memory round trip; L lanes per
// particle share the slice reduction and the first lane corrects.
// kStep: the corrector of a graph-replayed block step of parity par, which
// also predicts every corrected particle to the speculated next block time
// (the next multiple of the finest step of this step: t_next + 2^(kmax -
// fine)) into the j stream and appends those active then to list par ^ 1;
// k_step_correct's other workgroups do the same for the particles this step
// did not correct (predict_rest). Otherwise the corrector of a step whose
// list is list 0.
template <bool kStep, class D = Dev>
__device__ __forceinline__ void correct_body(const D& d, const Consts& c, int blk, int nblk, int par = 0,
                                             const PoolStep* step = nullptr) {
  Sched* __restrict__ sc = d.sc;
  const int tid = threadIdx.x;
  const size_t lo = (size_t)par * c.n;  // list offset
  // Small blocks use the slice count of a one-particle block (s1, which n
  // alone fixes) and fill at most its first i tile. The workgroups that hold
  // those positions request their state, and their slice partials when one
  // slot per lane covers them, before the schedule record is read, so that
  // the two memory round trips overlap; a step with another layout loads
  // afresh. Lanes past the list read entries in bounds (positions below n
  // and below part_cs / s1, which every block with s1 slices satisfies).
  const int L1 = correct_lanes(c.s1);
  const int per1 = kBlock / L1;
  const bool spec = blk * per1 < (kBlock >> lj1_of(c)) * ipl_of(c);
  const bool one_slot = c.s1 <= L1;
  int i = 0, lv = 0;
  double a0[3] = {0.0, 0.0, 0.0}, j0[3] = {0.0, 0.0, 0.0};
  double xp[3] = {0.0, 0.0, 0.0}, vp[3] = {0.0, 0.0, 0.0};
  double g1[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (spec) {
    const int r1 = tid & (L1 - 1);
    const int kcap = (int)min((long long)c.n, c.part_cs / c.s1) - 1;
    const int k1 = min(blk * per1 + tid / L1, kcap);
    i = d.active[lo + k1];
    lv = d.ilev[lo + k1];
    a0[0] = il_arr(d, kAx)[lo + k1]; a0[1] = il_arr(d, kAy)[lo + k1]; a0[2] = il_arr(d, kAz)[lo + k1];
    j0[0] = il_arr(d, kJx)[lo + k1]; j0[1] = il_arr(d, kJy)[lo + k1]; j0[2] = il_arr(d, kJz)[lo + k1];
    xp[0] = il_arr(d, kX)[lo + k1]; xp[1] = il_arr(d, kY)[lo + k1]; xp[2] = il_arr(d, kZ)[lo + k1];
    vp[0] = il_arr(d, kVx)[lo + k1]; vp[1] = il_arr(d, kVy)[lo + k1]; vp[2] = il_arr(d, kVz)[lo + k1];
    if (one_slot) {
      // (lanes past the slices read the last one; their sums are not used)
      const double* o = d.part + (size_t)k1 * c.s1 + min(r1, c.s1 - 1);
#pragma unroll
      for (int q = 0; q < 6; ++q) g1[q] = o[q * c.part_cs];
    }
  }

  int n_act, fine = 0;
  long long t_next;
  Plan p;
  if constexpr (kStep) {
    // every field the step needs in one round trip, with the loads above
    // (both flags read: no short-circuit load after the first)
    const int done = sc->done, refill = sc->refill;
    n_act = sc->n_act;
    t_next = sc->t_next;
    p = sc->plan;
    fine = sc->fine;
    if (done | refill) {
      hold(i); hold(lv);
#pragma unroll
      for (int q = 0; q < 3; ++q) { hold(a0[q]); hold(j0[q]); hold(xp[q]); hold(vp[q]); }
#pragma unroll
      for (int q = 0; q < 6; ++q) hold(g1[q]);
      hold(n_act); hold(t_next); hold(fine);
      hold(p.lj); hold(p.it); hold(p.nit); hold(p.s); hold(p.len); hold(p.items);
      // the list this step's corrector would have built next stays free
      if (blk == 0 && tid == 0) {
        sc->lcnt[par] = 0;
        if (refill) atomicAdd((unsigned long long*)&sc->refills, 1ULL);
      }
      return;
    }
  } else {
    // (a pool launch gives workgroups only to clusters whose step runs)
    if (!step && sc->done) return;
    n_act = step ? step->n_act : sc->n_act;
    t_next = step ? step->t_next : sc->t_next;
    p = step ? step->plan : sc->plan;
  }
  // speculated next block time (kStep)
  const long long t_spec = kStep ? t_next + (1LL << (c.kmax - fine)) : 0;
  const int kthr_spec = kStep ? max(0, c.kmax - (int)__builtin_ctzll((unsigned long long)t_spec)) : 0;
  const int L = correct_lanes(p.s);
  const int per_wg = kBlock / L;
  if (blk * per_wg >= n_act && blk != 0) return;
  // Same slice count: same lanes per particle and the same positions.
  const bool early = spec && p.s == c.s1;
  __shared__ LocalBook bk;
  book_init(bk, tid);
  __syncthreads();
  if (blk == 0 && tid == 0) {
    // Counters by atomics whose result is not used: no memory round trip
    // before the wave goes on.
    atomicAdd((unsigned long long*)&sc->block_steps, 1ULL);
    atomicAdd((unsigned long long*)&sc->particle_steps, (unsigned long long)n_act);
    atomicAdd((unsigned long long*)&sc->pairs, (unsigned long long)n_act * (unsigned long long)c.n);
    if (n_act > 0) atomicAdd((unsigned long long*)&sc->nact_hist[31 - __clz(n_act)], 1ULL);
    sc->t_now = t_next;
    if (kStep) {
      sc->lcnt[par] = 0;
      sc->spec = (t_spec << 1) | (par ^ 1);
    } else {
      sc->lcnt[0] = 0;
    }
  }
  const int r = tid & (L - 1);
  for (int base = blk * per_wg; base < n_act; base += nblk * per_wg) {
    const int k = base + tid / L;
    const bool valid = k < n_act;
    const int kk = valid ? k : 0;
    const bool first = early && base == blk * per_wg;
    if (!first) {
      // Loads that do not depend on the reduction, issued with it.
      i = d.active[lo + kk];
      lv = d.ilev[lo + kk];
      a0[0] = il_arr(d, kAx)[lo + kk]; a0[1] = il_arr(d, kAy)[lo + kk]; a0[2] = il_arr(d, kAz)[lo + kk];
      j0[0] = il_arr(d, kJx)[lo + kk]; j0[1] = il_arr(d, kJy)[lo + kk]; j0[2] = il_arr(d, kJz)[lo + kk];
      xp[0] = il_arr(d, kX)[lo + kk]; xp[1] = il_arr(d, kY)[lo + kk]; xp[2] = il_arr(d, kZ)[lo + kk];
      vp[0] = il_arr(d, kVx)[lo + kk]; vp[1] = il_arr(d, kVy)[lo + kk]; vp[2] = il_arr(d, kVz)[lo + kk];
    }
    double f[6];
    if (first && one_slot) {
      // The sum reduce_slices forms from the same one slot per lane.
#pragma unroll
      for (int q = 0; q < 6; ++q) f[q] = (valid && r < p.s) ? 0.0 + g1[q] : 0.0;
      force_sums(f, L);
    } else {
      reduce_slices(d.part, p.s, c.part_cs, k, L, r, valid, f);
    }
    const bool owner = r == 0 && valid;  // the lane that corrects position k
    bool take = false;
    double o[6];
    int nl = 0;
    if (owner) {
      if (!finite6(f)) bk.bad = 1;

      // h and its powers are powers of two: dividing by h^2 and h^3 is the exact
      // product with their reciprocals (from 1 / dt_min, scaled by 2^(lv - kmax)).
      const double h = (double)(1LL << (c.kmax - lv)) * c.dt_min;
      const double h2 = h * h, h3 = h2 * h;
      const double ih = ldexp(c.inv_dt_min, lv - c.kmax);
      const double ih2 = ih * ih, ih3 = ih2 * ih;
      double a2[3], a3[3], a2e[3], xn[3], vn[3];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double da = a0[q] - f[q];
        a2[q] = (-6.0 * da - h * (4.0 * j0[q] + 2.0 * f[3 + q])) * ih2;
        a3[q] = (12.0 * da + 6.0 * h * (j0[q] + f[3 + q])) * ih3;
        xn[q] = xp[q] + a2[q] * (h2 * h2) / 24.0 + a3[q] * (h2 * h3) / 120.0;
        vn[q] = vp[q] + a2[q] * h3 / 6.0 + a3[q] * (h2 * h2) / 24.0;
        a2e[q] = a2[q] + h * a3[q];
      }
      const double na1 = norm3(f[0], f[1], f[2]);
      const double nj1 = norm3(f[3], f[4], f[5]);
      const double na2 = norm3(a2e[0], a2e[1], a2e[2]);
      const double na3 = norm3(a3[0], a3[1], a3[2]);
      const double dtstar = sqrt(c.eta * (na1 * na2 + nj1 * nj1) / (nj1 * na3 + na2 * na2));
      const int kc = level_for(dtstar, c.dt_max, c.inv_dt_max, c.kmax);
      if (kc >= lv) {
        nl = kc;
      } else if (lv >= 1 && (t_next & ((1LL << (c.kmax - lv + 1)) - 1)) == 0) {
        nl = lv - 1;
      } else {
        nl = lv;
      }
      if (nl > c.kmax) {
        nl = c.kmax;
        atomicAdd(&bk.clamp, 1);
      }
      st_arr(d, kX)[i] = xn[0]; st_arr(d, kY)[i] = xn[1]; st_arr(d, kZ)[i] = xn[2];
      st_arr(d, kVx)[i] = vn[0]; st_arr(d, kVy)[i] = vn[1]; st_arr(d, kVz)[i] = vn[2];
      st_arr(d, kAx)[i] = f[0]; st_arr(d, kAy)[i] = f[1]; st_arr(d, kAz)[i] = f[2];
      st_arr(d, kJx)[i] = f[3]; st_arr(d, kJy)[i] = f[4]; st_arr(d, kJz)[i] = f[5];
      d.tick[i] = t_next;
      d.lev[i] = (unsigned char)nl;
      if (nl != lv) {
        atomicAdd(&bk.hist[lv], -1);
        atomicAdd(&bk.hist[nl], 1);
      }
      if (kStep) {
        // the corrected state predicted to the speculated next block time
        taylor6((double)(t_spec - t_next) * c.dt_min, xn[0], xn[1], xn[2], vn[0], vn[1], vn[2], f[0], f[1],
                f[2], f[3], f[4], f[5], o);
        pj_arr(d, kX)[i] = o[0]; pj_arr(d, kY)[i] = o[1]; pj_arr(d, kZ)[i] = o[2];
        pj_arr(d, kVx)[i] = o[3]; pj_arr(d, kVy)[i] = o[4]; pj_arr(d, kVz)[i] = o[5];
        take = nl >= kthr_spec;
      }
    }
    if (kStep) {
      const int pos = wg_append(take, &sc->lcnt[par ^ 1]);
      if (take) list_store(d, c.n, par ^ 1, pos, i, o, f[0], f[1], f[2], f[3], f[4], f[5], nl, t_spec);
    }
  }
  __syncthreads();
  book_flush(bk, sc, c.kmax, tid);
}

// The particles that the corrector of a replayed step of parity par did not
// correct (those not tagged in list par with this step's block time): each
// predicted to the speculated next block time into the j stream, and those
// active then appended to list par ^ 1. Workgroups take blocks of kBlock
// particles.
template <class D>
__device__ __forceinline__ void predict_rest(const D& d, const Consts& c, int blk, int nblk, int par) {
  const Sched* __restrict__ sc = d.sc;
  const int n = c.n, tid = threadIdx.x;
  const int nb = (n + kBlock - 1) / kBlock;
  if (blk >= nb) return;
  // The first block's state is requested with the schedule record.
  PState ps = load_pstate(d, min(blk * kBlock + tid, n - 1));
  long long tg = d.tag[(size_t)par * n + min(blk * kBlock + tid, n - 1)];
  const int stop = sc->done | sc->refill;
  const long long t_next = sc->t_next;
  const int fine = sc->fine;
  if (stop) {
    hold(ps.x); hold(ps.y); hold(ps.z); hold(ps.vx); hold(ps.vy); hold(ps.vz);
    hold(ps.ax); hold(ps.ay); hold(ps.az); hold(ps.jx); hold(ps.jy); hold(ps.jz);
    hold(ps.tick); hold(ps.lev); hold(tg); hold(t_next); hold(fine);
    return;
  }
  const long long t_spec = t_next + (1LL << (c.kmax - fine));
  const int kthr_spec = max(0, c.kmax - (int)__builtin_ctzll((unsigned long long)t_spec));
  for (int b = blk; b < nb; b += nblk) {
    if (b != blk) {
      ps = load_pstate(d, min(b * kBlock + tid, n - 1));
      tg = d.tag[(size_t)par * n + min(b * kBlock + tid, n - 1)];
    }
    const int j = b * kBlock + tid;
    bool take = false;
    double o[6];
    if (j < n && tg != t_next) {
      predict_store(d, j, (double)(t_spec - ps.tick) * c.dt_min, ps, o);
      take = ps.lev >= kthr_spec;
    }
    const int pos = wg_append(take, &d.sc->lcnt[par ^ 1]);
    if (take) list_store(d, n, par ^ 1, pos, j, o, ps.ax, ps.ay, ps.az, ps.jx, ps.jy, ps.jz, ps.lev, t_spec);
  }
}

__global__ __launch_bounds__(kBlock) void k_correct(Dev d, Consts c) {
  correct_body<false>(d, c, blockIdx.x, gridDim.x);
}

// The corrector of a graph-replayed block step of parity par: the first
// ceil(n / kBlock) workgroups predict the particles this step does not
// correct (predict_rest), the others correct the active particles
// (correct_body). The prediction workgroups come first: in a small step they
// are the longer path (every particle's state, the list counter's round
// trip), and workgroups start in index order (same-box timing of the
// N = 16384 integration: 548 ms this way, 563 ms the other way round).

__global__ __launch_bounds__(kBlock) void k_step_correct(DevC d, Consts c, int par) {
  const int nb = (c.n + kBlock - 1) / kBlock;
  if ((int)blockIdx.x < nb)
    predict_rest(d, c, blockIdx.x, nb, par);
  else
    correct_body<true>(d, c, blockIdx.x - nb, gridDim.x - nb, par);
}

// Prediction of every particle to the next block time into the j stream and
// list 0 for it (t_end as set before), for a step of parity 0.
__global__ __launch_bounds__(kBlock) void k_prepare(Dev d, Consts c) {
  Sched* __restrict__ sc = d.sc;
  const int n = c.n;
  const NextStep nx = schedule_wave(sc, c);
  for (int b = blockIdx.x; b < (n + kBlock - 1) / kBlock; b += gridDim.x) {
    const PState ps = load_pstate(d, min(b * kBlock + (int)threadIdx.x, n - 1));
    predict_append(d, c, b, ps, nx.t_next, nx.kthr, 0);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) sc->spec = nx.t_next << 1;
}

// Initial block steps (Sec. 2.4 step 3; Sec. 3.2: the same eta from the
// initial calculation on): dt* = eta |a| / |jerk|, quantised to the largest
// dt_max / 2^k <= dt*, clamped at dt_min. Stores a, jerk, t_i = t_now and the
// level histogram (zeroed beforehand).
__global__ __launch_bounds__(kBlock) void k_init_dt(Dev d, Consts c) {
  Sched* __restrict__ sc = d.sc;
  const int n_act = sc->n_act;
  const long long t_now = sc->t_now;
  const Plan p = sc->plan;
  const int L = correct_lanes(p.s);
  const int per_wg = kBlock / L;
  const int tid = threadIdx.x;
  __shared__ LocalBook bk;
  book_init(bk, tid);
  __syncthreads();
  const int r = tid & (L - 1);
  for (int base = blockIdx.x * per_wg; base < n_act; base += gridDim.x * per_wg) {
    const int k = base + tid / L;
    const bool valid = k < n_act;
    const int i = d.active[valid ? k : 0];
    double f[6];
    reduce_slices(d.part, p.s, c.part_cs, k, L, r, valid, f);
    if (r != 0 || !valid) continue;
    if (!finite6(f)) bk.bad = 1;
    const double dtstar = c.eta * norm3(f[0], f[1], f[2]) / norm3(f[3], f[4], f[5]);
    int nl = level_for(dtstar, c.dt_max, c.inv_dt_max, c.kmax);
    if (nl > c.kmax) {
      nl = c.kmax;
      atomicAdd(&bk.clamp, 1);
    }
    d.ax[i] = f[0]; d.ay[i] = f[1]; d.az[i] = f[2];
    d.jx[i] = f[3]; d.jy[i] = f[4]; d.jz[i] = f[5];
    d.tick[i] = t_now;
    d.lev[i] = (unsigned char)nl;
    atomicAdd(&bk.hist[nl], 1);
  }
  __syncthreads();
  book_flush(bk, sc, c.kmax, tid);
}

// Summed forces of the current active list as (n_act, 3) row-major arrays
// (gd_force outputs; either may be null).
__global__ __launch_bounds__(kBlock) void k_reduce_out(Dev d, Consts c, double* __restrict__ acc,
                                                       double* __restrict__ jerk) {
  Sched* __restrict__ sc = d.sc;
  const int n_act = sc->n_act;
  const Plan p = sc->plan;
  const int L = correct_lanes(p.s);
  const int per_wg = kBlock / L;
  const int tid = threadIdx.x;
  const int r = tid & (L - 1);
  bool bad = false;
  for (int base = blockIdx.x * per_wg; base < n_act; base += gridDim.x * per_wg) {
    const int k = base + tid / L;
    const bool valid = k < n_act;
    double f[6];
    reduce_slices(d.part, p.s, c.part_cs, k, L, r, valid, f);
    if (r != 0 || !valid) continue;
    if (!finite6(f)) bad = true;
    if (acc) {
      acc[3 * k] = f[0]; acc[3 * k + 1] = f[1]; acc[3 * k + 2] = f[2];
    }
    if (jerk) {
      jerk[3 * k] = f[3]; jerk[3 * k + 1] = f[4]; jerk[3 * k + 2] = f[5];
    }
  }
  if (bad) atomicOr(&sc->nonfinite, 1);
}

// ---------------------------------------------------------------------------
// Predictor with the active-set search (Sec. 2.4 steps 5 and 7(a))
// ---------------------------------------------------------------------------
//
// Every workgroup first derives the step from the level histogram: all
// particles at level k sit on multiples of their step 2^(kmax-k) ticks, so
// the earliest next time is the next multiple of the smallest step present,
// and the active set is every particle whose step divides that time, i.e.
// level >= kmax - ctz(t_next). No O(N) search is needed for the time, and the
// block size is the histogram's tail sum. The histogram and the clock are
// read by parallel lanes in one memory round trip.
//
// Then each lane predicts one particle to t_next (Taylor series through the
// jerk, Delta = t_next - t_j) into the j stream, and active particles are
// appended to the active list (wave ballot + one atomic per workgroup; the
// list order is not deterministic, but no result depends on it), together
// with their predicted state (for the force kernel) and their a, jerk and
// level (for the corrector), stored by list position.

// work (pool predictor, may be NULL): the cluster's force items, corrector
// workgroups and step for this pool step, written by its workgroup 0 at
// table position k.
__device__ __forceinline__ void predict_body(const Dev& d, const Consts& c, int mode,
                                             double t_explicit, int blk, PoolWork* work = nullptr, int k = 0) {
  Sched* __restrict__ sc = d.sc;
  const int n = c.n, kmax = c.kmax;
  __shared__ long long s_tnext;
  __shared__ int s_kthr, s_done;
  const int tid = threadIdx.x;
  // The particle's state does not depend on the schedule: its loads are
  // issued first and overlap the read of the histogram and the clock.
  const PState p = load_pstate(d, min(blk * kBlock + tid, n - 1));
  // The step, by wave 0 (next_step_wave, make_plan_wave).
  const int wave = tid >> 6, lane = tid & 63;
  if (wave == 0) {
    long long t_next;
    int kthr, nact = 0, done = 0;
    if (mode == kPredAuto) {
      const NextStep nx = schedule_wave(sc, c);
      t_next = nx.t_next;
      kthr = nx.kthr;
      nact = nx.n_act;
      done = nx.done;
    } else if (mode == kPredAll) {
      t_next = sc->t_now;
      kthr = 0;
      nact = n;
    } else {
      t_next = sc->t_now;
      kthr = kmax + 1;  // nobody active
    }
    Plan pl{};
    if (blk == 0 && nact > 0) pl = nact <= n1_of(c) ? one_plan(nact, n, c) : make_plan_wave(nact, n, ipl_of(c), lane);
    if (lane == 0) {
      s_tnext = t_next;
      s_kthr = kthr;
      s_done = done;
      if (blk == 0) {
        sc->t_next = t_next;
        sc->kthr = kthr;
        sc->n_act = nact;
        sc->done = done;
        if (nact > 0) sc->plan = pl;
        if (work) {
          const bool w = !done && nact > 0;
          const int per_wg = w ? kBlock / correct_lanes(pl.s) : 1;
          work->force_n[k] = w ? pl.items : 0;
          work->correct_n[k] = w ? (nact + per_wg - 1) / per_wg : 0;
          work->step[k].t_next = t_next;
          work->step[k].n_act = nact;
          work->step[k].plan = pl;
        }
      }
    }
  }
  __syncthreads();
  if (s_done) return;
  if (mode == kPredExplicit) {
    // prediction to an explicit time: the j stream only, nobody listed
    const int j = blk * kBlock + tid;
    double o[6];
    if (j < n) predict_store(d, j, t_explicit - (double)p.tick * c.dt_min, p, o);
    return;
  }
  predict_append(d, c, blk, p, s_tnext, s_kthr, 0);
}

__global__ __launch_bounds__(kBlock) void k_predict(Dev d, Consts c, int mode, double t_explicit) {
  predict_body(d, c, mode, t_explicit, blockIdx.x);
}

// ---------------------------------------------------------------------------
// Energy (Eq. (2), softened and unsoftened potentials)
// ---------------------------------------------------------------------------
//
// The potential sums each pair once: a lane holds kI i particles
// (EPlan::ipl) and sums phi_i = sum_{j > i} m_j / sqrt(r_ij^2 + eps_ij^2)
// over the j of its item (i tile, j slice); the workgroup then reduces
// -m_i phi_i (and the kinetic term, on slice 0) in a fixed tree, and a second
// kernel sums the item partials in a fixed order. Tiles wholly left of the i
// tile are skipped and only those that overlap it test j > i. The central
// particle's column enters the tile with mass 0 and is added once for each
// i below it, with its own softening, by the slice that holds it.
template <int kI, bool kMask, bool kUnsoft>
__device__ __forceinline__ void energy_tile(const double (*sj)[4], int cnt, int jt,
                                            const int (&ii)[kI],
                                            const double (&xi)[kI],
                                            const double (&yi)[kI],
                                            const double (&zi)[kI],
                                            const double (&e2)[kI],
                                            double (&phi)[kI],
                                            double (&phiu)[kI]) {
#pragma unroll 2
  for (int k = 0; k < cnt; ++k) {
    const double2 xy = *reinterpret_cast<const double2*>(&sj[k][0]);
    const double2 zm = *reinterpret_cast<const double2*>(&sj[k][2]);
#pragma unroll
    for (int q = 0; q < kI; ++q) {
      const double dx = xy.x - xi[q], dy = xy.y - yi[q], dz = zm.x - zi[q];
      double r2 = 0.0, s2;
      if constexpr (kUnsoft) {
        r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        s2 = r2 + e2[q];
      } else {
        s2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, e2[q])));
      }
      double mj = zm.y;
      if constexpr (kMask) {
        const bool lower = jt + k <= ii[q];
        s2 = lower ? 1.0 : s2;
        mj = lower ? 0.0 : mj;
      }
      phi[q] = fma(mj, rsqrt_fp64(s2), phi[q]);
      if constexpr (kUnsoft) {
        const double u2 = kMask && jt + k <= ii[q] ? 1.0 : r2;
        phiu[q] = fma(mj, rsqrt_fp64(u2), phiu[q]);
      }
    }
  }
}

template <int kI, bool kUnsoft>
__global__ __launch_bounds__(kBlock) void k_energy(int n, double eps2, double eps2_bh, int bh,
                                                   const double* __restrict__ x,
                                                   const double* __restrict__ y,
                                                   const double* __restrict__ z,
                                                   const double* __restrict__ vx,
                                                   const double* __restrict__ vy,
                                                   const double* __restrict__ vz,
                                                   const double* __restrict__ m,
                                                   double* __restrict__ ebuf) {
  const EPlan e = make_eplan(n);
  __shared__ __align__(16) double sj[kTileJ][4];
  __shared__ double red[3][kBlock];
  const int tid = threadIdx.x;
  for (int item = blockIdx.x; item < e.items; item += gridDim.x) {
    // The slice is rotated by the i tile: consecutive workgroups go to
    // different XCDs, and under j > i the slices hold unequal work.
    const int itile = item / e.s, slice = (item - itile * e.s + itile) % e.s;
    const int i0 = itile * kBlock * kI;
    const int j0 = min(n, slice * e.len), j1 = min(n, j0 + e.len);
    int ii[kI];
    double xi[kI], yi[kI], zi[kI], e2[kI], phi[kI], phiu[kI];
#pragma unroll
    for (int q = 0; q < kI; ++q) {
      ii[q] = min(i0 + q * kBlock + tid, n - 1);
      xi[q] = x[ii[q]]; yi[q] = y[ii[q]]; zi[q] = z[ii[q]];
      e2[q] = ii[q] == bh ? eps2_bh : eps2;
      phi[q] = 0.0; phiu[q] = 0.0;
    }
    // i0 and j0 are multiples of kTileJ, so max(j0, i0) starts a tile.
    for (int jt = max(j0, i0); jt < j1; jt += kTileJ) {
      const int cnt = min(kTileJ, j1 - jt);
      __syncthreads();
      if (tid < cnt) {
        const int j = jt + tid;
        *reinterpret_cast<double2*>(&sj[tid][0]) = make_double2(x[j], y[j]);
        *reinterpret_cast<double2*>(&sj[tid][2]) = make_double2(z[j], j == bh ? 0.0 : m[j]);
      }
      __syncthreads();
      if (jt < i0 + kBlock * kI)
        energy_tile<kI, true, kUnsoft>(sj, cnt, jt, ii, xi, yi, zi, e2, phi, phiu);
      else
        energy_tile<kI, false, kUnsoft>(sj, cnt, jt, ii, xi, yi, zi, e2, phi, phiu);
    }
    if (bh >= j0 && bh < j1) {
      const double xb = x[bh], yb = y[bh], zb = z[bh], mb = m[bh];
#pragma unroll
      for (int q = 0; q < kI; ++q) {
        if (ii[q] >= bh) continue;
        const double dx = xb - xi[q], dy = yb - yi[q], dz = zb - zi[q];
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        phi[q] = fma(mb, rsqrt_fp64(r2 + eps2_bh), phi[q]);
        if constexpr (kUnsoft) phiu[q] = fma(mb, rsqrt_fp64(r2), phiu[q]);
      }
    }
    double kin = 0.0, pot = 0.0, potu = 0.0;
#pragma unroll
    for (int q = 0; q < kI; ++q) {
      const int i = i0 + q * kBlock + tid;
      if (i < n) {
        const double mi = m[i];
        pot -= mi * phi[q];
        potu -= mi * phiu[q];
        if (slice == 0) kin += 0.5 * mi * fma(vz[i], vz[i], fma(vy[i], vy[i], vx[i] * vx[i]));
      }
    }
    red[0][tid] = kin;
    red[1][tid] = pot;
    red[2][tid] = potu;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if (tid < w) {
        red[0][tid] += red[0][tid + w];
        red[1][tid] += red[1][tid + w];
        red[2][tid] += red[2][tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      ebuf[3 * item + 0] = red[0][0];
      ebuf[3 * item + 1] = red[1][0];
      ebuf[3 * item + 2] = red[2][0];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_energy_final(int n, double* __restrict__ ebuf,
                                                         double* __restrict__ out) {
  const EPlan e = make_eplan(n);
  __shared__ double red[3][kBlock];
  const int tid = threadIdx.x;
  double s0 = 0, s1 = 0, s2 = 0;
  for (int it = tid; it < e.items; it += kBlock) {
    s0 += ebuf[3 * it + 0];
    s1 += ebuf[3 * it + 1];
    s2 += ebuf[3 * it + 2];
  }
  red[0][tid] = s0;
  red[1][tid] = s1;
  red[2][tid] = s2;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] += red[0][tid + w];
      red[1][tid] += red[1][tid + w];
      red[2][tid] += red[2][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = red[0][0];
    out[1] = red[1][0];
    out[2] = red[2][0];
  }
}

// ---------------------------------------------------------------------------
// State movement and small bookkeeping kernels
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool fin3(double a, double b, double c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

// Row-major (n, 3) inputs to SoA; masses copied; validation of the inputs.
__global__ void k_load(Sched* __restrict__ sc, int n, int bh, const double* __restrict__ m_in,
                       const double* __restrict__ x_in, const double* __restrict__ v_in,
                       double* __restrict__ m, double* __restrict__ jm, double* __restrict__ x,
                       double* __restrict__ y,
                       double* __restrict__ z, double* __restrict__ vx, double* __restrict__ vy,
                       double* __restrict__ vz, double* __restrict__ ax, double* __restrict__ ay,
                       double* __restrict__ az, double* __restrict__ jx, double* __restrict__ jy,
                       double* __restrict__ jz, long long* __restrict__ tick,
                       unsigned char* __restrict__ lev, long long* __restrict__ tag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  tag[i] = -1;
  tag[n + i] = -1;
  const double mi = m_in[i];
  const double x0 = x_in[3 * i], x1 = x_in[3 * i + 1], x2 = x_in[3 * i + 2];
  const double v0 = v_in[3 * i], v1 = v_in[3 * i + 1], v2 = v_in[3 * i + 2];
  if (!(isfinite(mi) && mi >= 0.0 && fin3(x0, x1, x2) && fin3(v0, v1, v2))) atomicOr(&sc->bad_input, 1);
  m[i] = mi;
  jm[i] = i == bh ? 0.0 : mi;
  x[i] = x0; y[i] = x1; z[i] = x2;
  vx[i] = v0; vy[i] = v1; vz[i] = v2;
  ax[i] = 0; ay[i] = 0; az[i] = 0;
  jx[i] = 0; jy[i] = 0; jz[i] = 0;
  tick[i] = 0;
  lev[i] = 0;
}

__global__ void k_reset_sched(Sched* __restrict__ sc, long long t_now) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->t_now = t_now;
    sc->t_next = 0;
    sc->t_end = 0;
    sc->n_act = 0;
    sc->kthr = 0;
    sc->done = 0;
    sc->lcnt[0] = 0;
    sc->lcnt[1] = 0;
    sc->spec = -2;  // no list prepared (block time -1)
    sc->refill = 0;
    sc->fine = 0;
    sc->nonfinite = 0;
    sc->bad_input = 0;
    sc->block_steps = 0;
    sc->particle_steps = 0;
    sc->pairs = 0;
    sc->clamps = 0;
    sc->refills = 0;
  }
  if (blockIdx.x == 0 && threadIdx.x <= kMaxLevels) sc->hist[threadIdx.x] = 0;
  if (blockIdx.x == 0 && threadIdx.x < kNactBins) sc->nact_hist[threadIdx.x] = 0;
}

// N_act of the step in flight, for the force-timing pass (0 when the step was
// skipped because the stop time was reached, or rebuilt its list).
__global__ void k_log_nact(const Sched* __restrict__ sc, int* __restrict__ out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = (sc->done || sc->refill) ? 0 : sc->n_act;
}

// Prepares a sequence of automatic steps: sets the stop time and clears the
// compaction counter.
__global__ void k_set_tend(Sched* __restrict__ sc, long long t_end) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    sc->t_end = t_end;
    sc->lcnt[0] = 0;
    sc->lcnt[1] = 0;
    sc->done = 0;
  }
}

// Explicit active list for gd_force(idx, ...): range-checked copy.
__global__ void k_set_active(Sched* __restrict__ sc, int n, int ipl, int forced_lj, int forced_s,
                             const int32_t* __restrict__ idx, int n_act, int* __restrict__ active, const double* __restrict__ px,
                             const double* __restrict__ py, const double* __restrict__ pz,
                             const double* __restrict__ pvx, const double* __restrict__ pvy,
                             const double* __restrict__ pvz, double* __restrict__ ix,
                             double* __restrict__ iy, double* __restrict__ iz,
                             double* __restrict__ ivx, double* __restrict__ ivy,
                             double* __restrict__ ivz) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) {
    sc->n_act = n_act;
    sc->done = 0;
    sc->plan = forced_lj > 0 ? plan_with(n_act, n, forced_lj, forced_s, ipl) : make_plan(n_act, n, ipl);
  }
  if (k >= n_act) return;
  int i = idx[k];
  if (i < 0 || i >= n) {
    atomicOr(&sc->bad_input, 1);
    i = 0;
  }
  active[k] = i;
  ix[k] = px[i]; iy[k] = py[i]; iz[k] = pz[i];
  ivx[k] = pvx[i]; ivy[k] = pvy[i]; ivz[k] = pvz[i];
}

__global__ void k_copy_active(const Sched* __restrict__ sc, const int* __restrict__ active,
                              int32_t* __restrict__ out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < sc->n_act) out[k] = active[k];
}

__global__ void k_get_state(int n, int kmax, double dt_min, const double* __restrict__ x,
                            const double* __restrict__ y, const double* __restrict__ z,
                            const double* __restrict__ vx, const double* __restrict__ vy,
                            const double* __restrict__ vz, const double* __restrict__ ax,
                            const double* __restrict__ ay, const double* __restrict__ az,
                            const double* __restrict__ jx, const double* __restrict__ jy,
                            const double* __restrict__ jz, const long long* __restrict__ tick,
                            const unsigned char* __restrict__ lev, double* __restrict__ xo,
                            double* __restrict__ vo, double* __restrict__ ao,
                            double* __restrict__ jo, double* __restrict__ to,
                            double* __restrict__ dto) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (xo) { xo[3 * i] = x[i]; xo[3 * i + 1] = y[i]; xo[3 * i + 2] = z[i]; }
  if (vo) { vo[3 * i] = vx[i]; vo[3 * i + 1] = vy[i]; vo[3 * i + 2] = vz[i]; }
  if (ao) { ao[3 * i] = ax[i]; ao[3 * i + 1] = ay[i]; ao[3 * i + 2] = az[i]; }
  if (jo) { jo[3 * i] = jx[i]; jo[3 * i + 1] = jy[i]; jo[3 * i + 2] = jz[i]; }
  if (to) to[i] = (double)tick[i] * dt_min;
  if (dto) dto[i] = (double)(1LL << (kmax - lev[i])) * dt_min;
}

// Inverse of k_get_state with validation: dt_i must be dt_min * 2^k for
// k in [0, kmax], t_i an exact multiple of dt_i, t_i <= t_now < t_i + dt_i.
__global__ void k_set_state(Sched* __restrict__ sc, int n, int kmax, double dt_min,
                            long long t_now, const double* __restrict__ xi,
                            const double* __restrict__ vi, const double* __restrict__ ai,
                            const double* __restrict__ ji, const double* __restrict__ ti,
                            const double* __restrict__ dti, double* __restrict__ x,
                            double* __restrict__ y, double* __restrict__ z,
                            double* __restrict__ vx, double* __restrict__ vy,
                            double* __restrict__ vz, double* __restrict__ ax,
                            double* __restrict__ ay, double* __restrict__ az,
                            double* __restrict__ jx, double* __restrict__ jy,
                            double* __restrict__ jz, long long* __restrict__ tick,
                            unsigned char* __restrict__ lev, long long* __restrict__ tag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  tag[i] = -1;
  tag[n + i] = -1;
  bool ok = fin3(xi[3 * i], xi[3 * i + 1], xi[3 * i + 2]) &&
            fin3(vi[3 * i], vi[3 * i + 1], vi[3 * i + 2]) &&
            fin3(ai[3 * i], ai[3 * i + 1], ai[3 * i + 2]) &&
            fin3(ji[3 * i], ji[3 * i + 1], ji[3 * i + 2]);
  const double steps = dti[i] / dt_min;  // exact for powers of two
  int e = 0;
  const double f = frexp(steps, &e);
  const int lg = e - 1;  // steps = 2^lg when f == 0.5
  ok = ok && f == 0.5 && lg >= 0 && lg <= kmax;
  const int lv = kmax - (ok ? lg : 0);
  const double tt = ti[i] / dt_min;
  ok = ok && isfinite(tt) && tt >= 0.0 && tt < 9.0e15 && tt == floor(tt);
  const long long tk = ok ? (long long)tt : 0;
  const long long st = 1LL << (kmax - lv);
  ok = ok && (tk % st) == 0 && tk <= t_now && t_now < tk + st;
  if (!ok) atomicOr(&sc->bad_input, 1);
  x[i] = xi[3 * i]; y[i] = xi[3 * i + 1]; z[i] = xi[3 * i + 2];
  vx[i] = vi[3 * i]; vy[i] = vi[3 * i + 1]; vz[i] = vi[3 * i + 2];
  ax[i] = ai[3 * i]; ay[i] = ai[3 * i + 1]; az[i] = ai[3 * i + 2];
  jx[i] = ji[3 * i]; jy[i] = ji[3 * i + 1]; jz[i] = ji[3 * i + 2];
  tick[i] = tk;
  lev[i] = (unsigned char)lv;
  atomicAdd(&sc->hist[lv], 1);
}

// ---------------------------------------------------------------------------
// Pool kernels: one launch per phase for every resident cluster
// ---------------------------------------------------------------------------
//
// Each cluster keeps its own decomposition, which depends only on its own
// (n_act, n): a pool launch assigns every workgroup task (a predictor block,
// a force item, or a corrector block of one cluster) to the same body the
// single-cluster kernels run. So a cluster's results are bitwise the same
// alone and packed with others.

constexpr int kPoolGrid = 1024;

static_assert(kMaxPool <= kBlock, "one thread per resident cluster loads its record");

// The last entry k with off[k] <= g (count entries, off in LDS, off[0] = 0,
// non-decreasing: clusters without work have equal offsets), by the whole
// wave: lane l tests entries l + 1, l + 65, ..., and k is the number that
// pass. Every lane of the wave must be active.
__device__ __forceinline__ int pool_find(const int* off, int count, int g) {
  int k = 0;
  for (int base = 1; base < count; base += 64) {
    const int e = base + (threadIdx.x & 63);
    k += __popcll(__ballot(e < count && off[e] <= g));
  }
  return k;
}

// off[k] = n[0] + ... + n[k - 1] for k = 0..count (arrays in LDS), by the
// first wave: inclusive scans of n across its lanes, 64 entries at a time
// with the carry of the ones before. The caller synchronises the workgroup
// before and after.
__device__ __forceinline__ void pool_offsets(const int* n, int count, int* off) {
  const int tid = threadIdx.x;
  if (tid >= 64) return;
  if (tid == 0) off[0] = 0;
  int carry = 0;
  for (int base = 0; base < count; base += 64) {
    const int e = base + tid;
    int v = e < count ? n[e] : 0;
#pragma unroll
    for (int d = 1; d < 64; d *= 2) {
      const int u = __shfl_up(v, d, 64);
      if (tid >= d) v += u;
    }
    v += carry;
    if (e < count) off[e + 1] = v;
    carry = __shfl(v, 63, 64);
  }
}

// Work item g of a pool launch: the cluster's slot, the workgroup index
// within that cluster's launch and (n given) its number of workgroups. The
// same in every lane; read back from lane 0 so that the slot's record is
// read with scalar loads and the cluster's loops stay scalar.
struct PoolItem {
  int k, slot, blk, nblk;  // k: position in the table
};

__device__ __forceinline__ PoolItem pool_item(const int* off, const int* order, const int* n, int count,
                                              int g) {
  const int k = __builtin_amdgcn_readfirstlane(pool_find(off, count, g));
  PoolItem it;
  it.k = k;
  it.slot = __builtin_amdgcn_readfirstlane(order[k]);
  it.blk = g - __builtin_amdgcn_readfirstlane(off[k]);
  it.nblk = n ? __builtin_amdgcn_readfirstlane(n[k]) : 0;
  return it;
}

// The table is read whole (entries past count are in bounds and unused), so
// that its loads do not wait for the count.
__global__ __launch_bounds__(kBlock) void k_pool_predict(const PoolSlot* __restrict__ slots,
                                                         const PoolTable* __restrict__ tab,
                                                         PoolWork* __restrict__ work) {
  __shared__ int s_off[kMaxPool + 1], s_order[kMaxPool];
  const int tid = threadIdx.x;
  const int count = tab->count;
  for (int k = tid; k <= kMaxPool; k += kBlock) s_off[k] = tab->pred_off[k];
  for (int k = tid; k < kMaxPool; k += kBlock) s_order[k] = tab->order[k];
  __syncthreads();
  const int total = s_off[count];
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    const PoolItem it = pool_item(s_off, s_order, nullptr, count, g);
    const PoolSlot& ps = slots[it.slot];
    predict_body(ps.d, ps.c, kPredAuto, 0.0, it.blk, work, it.k);
  }
}

template <bool kMixed>
__device__ __forceinline__ void pool_force_body(const PoolSlot* __restrict__ slots,
                                                const PoolTable* __restrict__ tab,
                                                const PoolWork* __restrict__ work) {
  __shared__ int s_off[kMaxPool + 1], s_order[kMaxPool], s_n[kMaxPool];
  const int tid = threadIdx.x;
  const int count = tab->count;
  for (int k = tid; k < kMaxPool; k += kBlock) {
    s_order[k] = tab->order[k];
    s_n[k] = work->force_n[k];
  }
  __syncthreads();
  pool_offsets(s_n, count, s_off);
  __syncthreads();
  const int total = s_off[count];
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    const PoolItem it = pool_item(s_off, s_order, s_n, count, g);
    const PoolSlot& ps = slots[it.slot];
    force_body<false, false, kMixed, kIPerLane>(ps.d, ps.c, it.blk, it.nblk, 0, &work->step[it.k]);
  }
}

// Both variants fit 128 VGPRs (4 waves per SIMD) without spills, once the
// cluster's record is read with scalar loads (pool_item).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_pool_force(
    const PoolSlot* __restrict__ slots, const PoolTable* __restrict__ tab, const PoolWork* __restrict__ work) {
  pool_force_body<false>(slots, tab, work);
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_pool_force_mixed(
    const PoolSlot* __restrict__ slots, const PoolTable* __restrict__ tab, const PoolWork* __restrict__ work) {
  pool_force_body<true>(slots, tab, work);
}

__global__ __launch_bounds__(kBlock) void k_pool_correct(const PoolSlot* __restrict__ slots,
                                                         const PoolTable* __restrict__ tab,
                                                         const PoolWork* __restrict__ work) {
  __shared__ int s_off[kMaxPool + 1], s_order[kMaxPool], s_n[kMaxPool];
  const int tid = threadIdx.x;
  const int count = tab->count;
  for (int k = tid; k < kMaxPool; k += kBlock) {
    s_order[k] = tab->order[k];
    s_n[k] = work->correct_n[k];
  }
  __syncthreads();
  pool_offsets(s_n, count, s_off);
  __syncthreads();
  const int total = s_off[count];
  for (int g = blockIdx.x; g < total; g += gridDim.x) {
    const PoolItem it = pool_item(s_off, s_order, s_n, count, g);
    const PoolSlot& ps = slots[it.slot];
    correct_body<false>(ps.d, ps.c, it.blk, it.nblk, 0, &work->step[it.k]);
  }
}

__global__ void k_pool_status(const PoolSlot* __restrict__ slots, const PoolTable* __restrict__ tab,
                              PoolStatus* __restrict__ out) {
  const int t = threadIdx.x;
  if (t >= tab->count) return;
  const int sl = tab->order[t];
  const Sched* sc = slots[sl].d.sc;
  PoolStatus st;
  st.t_now = sc->t_now;
  st.block_steps = sc->block_steps;
  st.particle_steps = sc->particle_steps;
  st.pairs = sc->pairs;
  st.clamps = sc->clamps;
  st.done = sc->done;
  st.nonfinite = sc->nonfinite;
  out[sl] = st;
}

// ---------------------------------------------------------------------------
// Diagnostics: Lagrange radii and half-mass relaxation time (Sec. 4.2, Eq. (5))
// ---------------------------------------------------------------------------
//
// Lagrange radius of mass fraction f: about the centre of mass, the distance
// of the first particle (in ascending distance, ties by index) at which the
// cumulative mass reaches f times the total. The distances are sorted on the
// device (bitonic network over the bit patterns of r^2, which order like the
// values for r^2 >= 0) and the masses are accumulated in sorted order by one
// lane, so the cumulative sums are the plain sequential ones.

struct DiagArgs {
  int n_frac;
  double frac[kMaxDiagFractions];  // ascending
};

// Per-workgroup partial sums of m, m x, m y, m z (fixed-order tree).
__global__ __launch_bounds__(kBlock) void k_diag_com(int n, const double* __restrict__ m,
                                                     const double* __restrict__ x,
                                                     const double* __restrict__ y,
                                                     const double* __restrict__ z,
                                                     double* __restrict__ wg_out) {
  __shared__ double red[4][kBlock];
  const int tid = threadIdx.x;
  const int i = blockIdx.x * kBlock + tid;
  double v[4] = {0, 0, 0, 0};
  if (i < n) {
    v[0] = m[i];
    v[1] = m[i] * x[i];
    v[2] = m[i] * y[i];
    v[3] = m[i] * z[i];
  }
  for (int q = 0; q < 4; ++q) red[q][tid] = v[q];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (tid < w)
      for (int q = 0; q < 4; ++q) red[q][tid] += red[q][tid + w];
    __syncthreads();
  }
  if (tid == 0)
    for (int q = 0; q < 4; ++q) wg_out[4 * blockIdx.x + q] = red[q][0];
}

// Sort keys: bit pattern of r^2 about the centre of mass (padding: max key).
__global__ __launch_bounds__(kBlock) void k_diag_keys(int n, int npow2, int nwg,
                                                      const double* __restrict__ wg,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ y,
                                                      const double* __restrict__ z,
                                                      unsigned long long* __restrict__ key,
                                                      int* __restrict__ idx) {
  __shared__ double com[4];
  const int tid = threadIdx.x;
  if (tid < 4) {
    double acc = 0.0;
    for (int b = 0; b < nwg; ++b) acc += wg[4 * b + tid];
    com[tid] = acc;
  }
  __syncthreads();
  const int i = blockIdx.x * kBlock + tid;
  if (i >= npow2) return;
  if (i < n) {
    const double dx = x[i] - com[1] / com[0], dy = y[i] - com[2] / com[0], dz = z[i] - com[3] / com[0];
    const double r2 = dx * dx + dy * dy + dz * dz;
    key[i] = (unsigned long long)__double_as_longlong(r2);
  } else {
    key[i] = ~0ULL;
  }
  idx[i] = i;
}

// One compare-exchange stage of the bitonic network on (key, index) pairs.
__global__ __launch_bounds__(kBlock) void k_bitonic(int npow2, int j, int k,
                                                    unsigned long long* __restrict__ key,
                                                    int* __restrict__ idx) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= npow2) return;
  const int l = i ^ j;
  if (l <= i) return;
  const bool up = (i & k) == 0;
  const unsigned long long ki = key[i], kl = key[l];
  const int ii = idx[i], il = idx[l];
  const bool greater = ki > kl || (ki == kl && ii > il);
  if (greater == up) {
    key[i] = kl;
    key[l] = ki;
    idx[i] = il;
    idx[l] = ii;
  }
}

// One lane: total mass in index order, cumulative mass in sorted order, the
// radius for each fraction, and Eq. (5) for the half-mass radius
// (out[n_frac]; out[n_frac + 1] is the radius at f = 1/2).
__global__ void k_diag_scan(int n, const double* __restrict__ m,
                            const unsigned long long* __restrict__ key, const int* __restrict__ idx,
                            DiagArgs a, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double mt = 0.0;
  for (int i = 0; i < n; ++i) mt += m[i];
  double cum = 0.0;
  int f = 0;
  double rh = 0.0;
  bool rh_set = false;
  for (int r = 0; r < n && (f < a.n_frac || !rh_set); ++r) {
    cum += m[idx[r]];
    const double rad = sqrt(__longlong_as_double((long long)key[r]));
    while (f < a.n_frac && cum >= a.frac[f] * mt) out[f++] = rad;
    if (!rh_set && cum >= 0.5 * mt) {
      rh = rad;
      rh_set = true;
    }
  }
  const double last = sqrt(__longlong_as_double((long long)key[n - 1]));
  while (f < a.n_frac) out[f++] = last;
  if (!rh_set) rh = last;
  out[a.n_frac + 1] = rh;
  out[a.n_frac] = 0.138 * sqrt((double)n * rh * rh * rh / (mt / n)) / log(0.1 * n);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static inline int grid_for(int n) { return (n + kBlock - 1) / kBlock; }

hipError_t launch_load(const Dev& d, const Consts& c, const double* m, const double* x,
                       const double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_load, dim3(grid_for(c.n)), dim3(kBlock), 0, s, d.sc, c.n, c.bh, m, x, v, d.m,
                     d.jm, d.x, d.y, d.z, d.vx, d.vy, d.vz, d.ax, d.ay, d.az, d.jx, d.jy, d.jz, d.tick,
                     d.lev, d.tag);
  return hipGetLastError();
}

hipError_t launch_predict(const Dev& d, const Consts& c, int mode, double t_explicit,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_predict, dim3(grid_for(c.n)), dim3(kBlock), 0, s, d, c, mode, t_explicit);
  return hipGetLastError();
}

hipError_t launch_force(const Dev& d, const Consts& c, hipStream_t s, hipEvent_t ev_start,
                        hipEvent_t ev_stop) {
  // Four i per lane only with eps > 0 (no self mask): see make_consts.
  auto kern = ipl_of(c) == kIPerLaneLarge
                  ? (c.mixed ? (c.bh >= 0 ? k_force<false, true, true, kIPerLaneLarge>
                                          : k_force<false, false, true, kIPerLaneLarge>)
                             : (c.bh >= 0 ? k_force<false, true, false, kIPerLaneLarge>
                                          : k_force<false, false, false, kIPerLaneLarge>))
              : c.mixed ? (c.bh >= 0 ? k_force<false, true, true, kIPerLane>
                                     : (c.eps2 > 0.0 ? k_force<false, false, true, kIPerLane>
                                                     : k_force<true, false, true, kIPerLane>))
                        : (c.bh >= 0 ? k_force<false, true, false, kIPerLane>
                                     : (c.eps2 > 0.0 ? k_force<false, false, false, kIPerLane>
                                                     : k_force<true, false, false, kIPerLane>));
  if (ev_start) {
    // The events take the dispatch's own start and end timestamps.
    hipExtLaunchKernelGGL(kern, dim3(c.force_grid), dim3(kBlock), 0, s, ev_start, ev_stop, 0, d, c);
  } else {
    hipLaunchKernelGGL(kern, dim3(c.force_grid), dim3(kBlock), 0, s, d, c);
  }
  return hipGetLastError();
}

hipError_t launch_step_force(const Dev& d, const Consts& c, int par, hipStream_t s, hipEvent_t ev_start,
                             hipEvent_t ev_stop) {
  auto kern = ipl_of(c) == kIPerLaneLarge
                  ? (c.mixed ? (c.bh >= 0 ? k_step_force<false, true, true, kIPerLaneLarge>
                                          : k_step_force<false, false, true, kIPerLaneLarge>)
                             : (c.bh >= 0 ? k_step_force<false, true, false, kIPerLaneLarge>
                                          : k_step_force<false, false, false, kIPerLaneLarge>))
              : c.mixed ? (c.bh >= 0 ? k_step_force<false, true, true, kIPerLane>
                                     : (c.eps2 > 0.0 ? k_step_force<false, false, true, kIPerLane>
                                                     : k_step_force<true, false, true, kIPerLane>))
                        : (c.bh >= 0 ? k_step_force<false, true, false, kIPerLane>
                                     : (c.eps2 > 0.0 ? k_step_force<false, false, false, kIPerLane>
                                                     : k_step_force<true, false, false, kIPerLane>));
  if (ev_start) {
    hipExtLaunchKernelGGL(kern, dim3(c.force_grid), dim3(kBlock), 0, s, ev_start, ev_stop, 0, d, c, par);
  } else {
    hipLaunchKernelGGL(kern, dim3(c.force_grid), dim3(kBlock), 0, s, d, c, par);
  }
  return hipGetLastError();
}

hipError_t launch_step_correct(const Dev& d, const Consts& c, int par, hipStream_t s) {
  DevC e{};
  e.sc = d.sc; e.m = d.m; e.jm = d.jm; e.st = d.x; e.pj = d.px; e.il = d.ix; e.part = d.part;
  e.tick = d.tick; e.lev = d.lev; e.active = d.active; e.ilev = d.ilev; e.tag = d.tag;
  e.sn = d.y - d.x;
  e.sl = d.iy - d.ix;
  // (make_layout places each group one stride apart; any other layout is refused)
  const double* st[12] = {d.x, d.y, d.z, d.vx, d.vy, d.vz, d.ax, d.ay, d.az, d.jx, d.jy, d.jz};
  const double* pj[6] = {d.px, d.py, d.pz, d.pvx, d.pvy, d.pvz};
  const double* il[12] = {d.ix, d.iy, d.iz, d.ivx, d.ivy, d.ivz, d.iax, d.iay, d.iaz, d.ijx, d.ijy, d.ijz};
  for (int k = 0; k < 12; ++k)
    if (st[k] != d.x + k * e.sn || il[k] != d.ix + k * e.sl || (k < 6 && pj[k] != d.px + k * e.sn))
      return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_step_correct, dim3(c.correct_grid + grid_for(c.n)), dim3(kBlock), 0, s, e, c, par);
  return hipGetLastError();
}

hipError_t launch_prepare(const Dev& d, const Consts& c, hipStream_t s) {
  hipLaunchKernelGGL(k_prepare, dim3(grid_for(c.n)), dim3(kBlock), 0, s, d, c);
  return hipGetLastError();
}

hipError_t launch_correct(const Dev& d, const Consts& c, hipStream_t s) {
  hipLaunchKernelGGL(k_correct, dim3(c.correct_grid), dim3(kBlock), 0, s, d, c);
  return hipGetLastError();
}

hipError_t launch_init_dt(const Dev& d, const Consts& c, hipStream_t s) {
  hipLaunchKernelGGL(k_init_dt, dim3(c.correct_grid), dim3(kBlock), 0, s, d, c);
  return hipGetLastError();
}

hipError_t launch_reduce_out(const Dev& d, const Consts& c, double* acc, double* jerk,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_out, dim3(c.correct_grid), dim3(kBlock), 0, s, d, c, acc, jerk);
  return hipGetLastError();
}

hipError_t launch_energy(const Dev& d, const Consts& c, int unsoft, hipStream_t s) {
  const EPlan ep = make_eplan(c.n);
  auto kern = ep.ipl == kEnergyIPerLane ? (unsoft ? k_energy<kEnergyIPerLane, true>
                                                  : k_energy<kEnergyIPerLane, false>)
                                        : (unsoft ? k_energy<1, true> : k_energy<1, false>);
  hipLaunchKernelGGL(kern, dim3(ep.items), dim3(kBlock), 0, s, c.n, c.eps2, c.eps2_bh, c.bh, d.x,
                     d.y, d.z, d.vx, d.vy, d.vz, d.m, d.ebuf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kBlock), 0, s, c.n, d.ebuf,
                     d.ebuf + 3 * (size_t)ep.items);
  return hipGetLastError();
}

hipError_t launch_set_tend(const Dev& d, long long t_end, hipStream_t s) {
  hipLaunchKernelGGL(k_set_tend, dim3(1), dim3(64), 0, s, d.sc, t_end);
  return hipGetLastError();
}

hipError_t launch_log_nact(const Dev& d, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_log_nact, dim3(1), dim3(64), 0, s, d.sc, out);
  return hipGetLastError();
}

hipError_t launch_reset_sched(const Dev& d, long long t_now, hipStream_t s) {
  hipLaunchKernelGGL(k_reset_sched, dim3(1), dim3(64), 0, s, d.sc, t_now);
  return hipGetLastError();
}

hipError_t launch_set_active(const Dev& d, const Consts& c, const int32_t* idx, int n_act,
                             hipStream_t s, int forced_lj, int forced_s) {
  hipLaunchKernelGGL(k_set_active, dim3(grid_for(n_act > 0 ? n_act : 1)), dim3(kBlock), 0, s,
                     d.sc, c.n, ipl_of(c), forced_lj, forced_s, idx, n_act, d.active, d.px, d.py, d.pz, d.pvx, d.pvy, d.pvz, d.ix,
                     d.iy, d.iz, d.ivx, d.ivy, d.ivz);
  return hipGetLastError();
}

hipError_t launch_copy_active(const Dev& d, const Consts& c, int32_t* idx, hipStream_t s) {
  hipLaunchKernelGGL(k_copy_active, dim3(grid_for(c.n)), dim3(kBlock), 0, s, d.sc, d.active, idx);
  return hipGetLastError();
}

hipError_t launch_get_state(const Dev& d, const Consts& c, double* x, double* v, double* a,
                            double* jerk, double* t_i, double* dt_i, hipStream_t s) {
  hipLaunchKernelGGL(k_get_state, dim3(grid_for(c.n)), dim3(kBlock), 0, s, c.n, c.kmax, c.dt_min,
                     d.x, d.y, d.z, d.vx, d.vy, d.vz, d.ax, d.ay, d.az, d.jx, d.jy, d.jz, d.tick,
                     d.lev, x, v, a, jerk, t_i, dt_i);
  return hipGetLastError();
}

hipError_t launch_set_state(const Dev& d, const Consts& c, const double* x, const double* v,
                            const double* a, const double* jerk, const double* t_i,
                            const double* dt_i, long long t_now, hipStream_t s) {
  hipLaunchKernelGGL(k_set_state, dim3(grid_for(c.n)), dim3(kBlock), 0, s, d.sc, c.n, c.kmax,
                     c.dt_min, t_now, x, v, a, jerk, t_i, dt_i, d.x, d.y, d.z, d.vx, d.vy, d.vz,
                     d.ax, d.ay, d.az, d.jx, d.jy, d.jz, d.tick, d.lev, d.tag);
  return hipGetLastError();
}

hipError_t launch_diagnostics(const Dev& d, const Consts& c, const double* frac, int n_frac,
                              double* out, hipStream_t s) {
  const int n = c.n;
  int npow2 = 1;
  while (npow2 < n) npow2 <<= 1;
  const int nwg = grid_for(n);
  // Scratch in the partial-force buffer (unused between block steps): the
  // workgroup sums, then keys and indices.
  double* wg = d.part;
  unsigned long long* key = (unsigned long long*)(d.part + 4 * (size_t)nwg + 8);
  int* idx = (int*)(key + npow2);
  hipLaunchKernelGGL(k_diag_com, dim3(nwg), dim3(kBlock), 0, s, n, d.m, d.x, d.y, d.z, wg);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diag_keys, dim3(grid_for(npow2)), dim3(kBlock), 0, s, n, npow2, nwg, wg, d.x,
                     d.y, d.z, key, idx);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int k = 2; k <= npow2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      hipLaunchKernelGGL(k_bitonic, dim3(grid_for(npow2)), dim3(kBlock), 0, s, npow2, j, k, key, idx);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  DiagArgs a{};
  a.n_frac = n_frac;
  for (int q = 0; q < n_frac; ++q) a.frac[q] = frac[q];
  hipLaunchKernelGGL(k_diag_scan, dim3(1), dim3(64), 0, s, n, d.m, key, idx, a, out);
  return hipGetLastError();
}

hipError_t launch_pool_step(const PoolSlot* slots, const PoolTable* tab, PoolWork* work, bool mixed,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_pool_predict, dim3(kPoolGrid), dim3(kBlock), 0, s, slots, tab, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const PoolWork* cw = work;
  if (mixed)
    hipLaunchKernelGGL(k_pool_force_mixed, dim3(kPoolGrid), dim3(kBlock), 0, s, slots, tab, cw);
  else
    hipLaunchKernelGGL(k_pool_force, dim3(kPoolGrid), dim3(kBlock), 0, s, slots, tab, cw);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pool_correct, dim3(kPoolGrid), dim3(kBlock), 0, s, slots, tab, cw);
  return hipGetLastError();
}

hipError_t launch_pool_status(const PoolSlot* slots, const PoolTable* tab, PoolStatus* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_pool_status, dim3(1), dim3(kMaxPool), 0, s, slots, tab, out);
  return hipGetLastError();
}

}  // namespace gd
