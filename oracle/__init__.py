"""FP64 CPU oracle for the Hermite-4 block-step integrator (arXiv:1702.00440).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg may use it; the product path never does. It shares no code with
the HIP library (see h4_oracle.c for the method and the readings it takes).

The C source is compiled with gcc into liboracle_h4.so next to this file, by
build() (called from the repository's build entry point) or on first use when
no library is there yet.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import math

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "h4_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_h4.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build() -> str:
    """Compile the oracle: plain -O2, no FMA contraction, OpenMP over i only."""
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    _lib = _bind(C.CDLL(_LIB))
    return _lib


class using:
    """Context manager: route every oracle call through another build of the
    oracle source (e.g. a copy with a planted mistake, in the tests)."""

    def __init__(self, lib_path):
        self.path = lib_path

    def __enter__(self):
        global _lib
        self.saved = _load()
        _lib = _bind(C.CDLL(self.path))
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def compile_source(src_path, out_path):
    """Compile an oracle source file with the same flags as build()."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-o", out_path, src_path, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    return out_path


def _bind(lib):
    i64, dbl, cint = C.c_int64, C.c_double, C.c_int
    lib.or_force.argtypes = [i64, _dp, _dp, _dp, dbl, dbl, i64, i64, C.c_void_p, _dp, _dp, cint, cint]
    lib.or_force.restype = cint
    lib.or_energy.argtypes = [i64, _dp, _dp, _dp, dbl, dbl, i64, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(dbl)]
    lib.or_energy.restype = cint
    lib.or_predict.argtypes = [i64, _dp, _dp, _dp, _dp, _dp, dbl, _dp, _dp]
    lib.or_predict.restype = None
    lib.or_hermite_derivs.argtypes = [_dp, _dp, _dp, _dp, dbl, _dp, _dp]
    lib.or_hermite_derivs.restype = None
    lib.or_correct.argtypes = [_dp, _dp, _dp, _dp, dbl, _dp, _dp]
    lib.or_correct.restype = None
    lib.or_dt_initial.argtypes = [_dp, _dp, dbl]
    lib.or_dt_initial.restype = dbl
    lib.or_dt_aarseth.argtypes = [_dp, _dp, _dp, _dp, dbl, dbl]
    lib.or_dt_aarseth.restype = dbl
    lib.or_quantize.argtypes = [dbl, dbl, dbl, dbl, dbl, C.POINTER(i64)]
    lib.or_quantize.restype = dbl
    lib.or_init.argtypes = [i64, _dp, _dp, _dp, dbl, dbl, i64, dbl, dbl, dbl, _dp, _dp, _dp, _dp,
                            C.POINTER(i64), cint]
    lib.or_init.restype = cint
    lib.or_block_step.argtypes = [i64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, dbl, dbl, i64, dbl, dbl, dbl,
                                  C.POINTER(dbl), _ip, C.POINTER(i64), cint]
    lib.or_block_step.restype = i64
    lib.or_run.argtypes = [i64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, dbl, dbl, i64, dbl, dbl, dbl,
                           C.POINTER(dbl), dbl, dbl, _ip, _dp, i64, cint]
    lib.or_run.restype = i64
    lib.or_max_threads.argtypes = []
    lib.or_max_threads.restype = cint
    return lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and a.shape != shape:
        a = a.reshape(shape)
    return a


def max_threads() -> int:
    return int(_load().or_max_threads())


def force(m, x, v, eps, idx=None, compensated=False, threads=1, eps_bh=None, bh=-1):
    """Softened acceleration and jerk of particles idx (all when None) from all
    particles; pairs with particle bh (if >= 0) are softened with eps_bh.
    Returns (acc[n_act, 3], jerk[n_act, 3])."""
    lib = _load()
    m = _f64(m)
    n = m.shape[0]
    x, v = _f64(x, (n, 3)), _f64(v, (n, 3))
    if idx is None:
        n_act, ip = n, None
        keep = None
    else:
        keep = np.ascontiguousarray(idx, dtype=np.int64)
        if keep.size and (keep.min() < 0 or keep.max() >= n):
            raise IndexError("active index out of range")
        n_act, ip = keep.shape[0], keep.ctypes.data_as(C.c_void_p)
    acc = np.zeros((n_act, 3))
    jrk = np.zeros((n_act, 3))
    e_bh = float(eps if eps_bh is None else eps_bh)
    rc = lib.or_force(n, m, x, v, float(eps), e_bh, int(bh), n_act, ip, acc, jrk, int(bool(compensated)),
                      int(threads))
    if rc:
        raise ValueError(f"or_force failed ({rc})")
    return acc, jrk


def energy(m, x, v, eps, unsoftened=False, eps_bh=None, bh=-1):
    """(ekin, epot_softened[, epot_unsoftened]) of a synchronised state."""
    lib = _load()
    m = _f64(m)
    n = m.shape[0]
    x, v = _f64(x, (n, 3)), _f64(v, (n, 3))
    ek, ep, eu = C.c_double(), C.c_double(), C.c_double()
    e_bh = float(eps if eps_bh is None else eps_bh)
    rc = lib.or_energy(n, m, x, v, float(eps), e_bh, int(bh), C.byref(ek), C.byref(ep),
                       C.byref(eu) if unsoftened else None)
    if rc:
        raise ValueError(f"or_energy failed ({rc})")
    if unsoftened:
        return ek.value, ep.value, eu.value
    return ek.value, ep.value


def predict(x, v, a, jk, t_i, t):
    lib = _load()
    x = _f64(x)
    n = x.shape[0]
    v, a, jk = _f64(v, (n, 3)), _f64(a, (n, 3)), _f64(jk, (n, 3))
    t_i = _f64(np.broadcast_to(np.asarray(t_i, dtype=np.float64), (n,)))
    xp, vp = np.zeros((n, 3)), np.zeros((n, 3))
    lib.or_predict(n, x, v, a, jk, t_i, float(t), xp, vp)
    return xp, vp


def hermite_derivs(a0, j0, a1, j1, h):
    lib = _load()
    a2, a3 = np.zeros(3), np.zeros(3)
    lib.or_hermite_derivs(_f64(a0), _f64(j0), _f64(a1), _f64(j1), float(h), a2, a3)
    return a2, a3


def correct(xp, vp, a2, a3, h):
    lib = _load()
    x, v = np.zeros(3), np.zeros(3)
    lib.or_correct(_f64(xp), _f64(vp), _f64(a2), _f64(a3), float(h), x, v)
    return x, v


def dt_initial(a, jk, eta):
    return float(_load().or_dt_initial(_f64(a), _f64(jk), float(eta)))


def dt_aarseth(a1, j1, a2, a3, h, eta):
    return float(_load().or_dt_aarseth(_f64(a1), _f64(j1), _f64(a2), _f64(a3), float(h), float(eta)))


def quantize(dtstar, dt_old, t_new, dt_max, dt_min):
    """Returns (dt_new, clamped)."""
    c = C.c_int64(0)
    r = _load().or_quantize(float(dtstar), float(dt_old), float(t_new), float(dt_max), float(dt_min), C.byref(c))
    return float(r), int(c.value)


def _is_pow2(x: float) -> bool:
    if not (x > 0 and math.isfinite(x)):
        return False
    mant, _ = math.frexp(x)
    return mant == 0.5


class State:
    """Oracle integrator state: the particle arrays plus per-particle times and
    block steps (row-major (n, 3) arrays)."""

    def __init__(self, m, x, v, eps, eta, dt_max, dt_min, threads=1, eps_bh=None, bh=-1):
        if not (_is_pow2(dt_max) and _is_pow2(dt_min) and dt_min <= dt_max):
            raise ValueError("dt_max and dt_min must be powers of two with dt_min <= dt_max")
        self.m = _f64(m).copy()
        n = self.m.shape[0]
        if n < 2:
            raise ValueError("need at least two particles")
        self.n = n
        self.x = _f64(x, (n, 3)).copy()
        self.v = _f64(v, (n, 3)).copy()
        self.eps, self.eta, self.dt_max, self.dt_min = float(eps), float(eta), float(dt_max), float(dt_min)
        self.eps_bh, self.bh = float(eps if eps_bh is None else eps_bh), int(bh)
        self.threads = int(threads)
        self.a = np.zeros((n, 3))
        self.jk = np.zeros((n, 3))
        self.t_i = np.zeros(n)
        self.dt_i = np.zeros(n)
        self.t_now = 0.0
        # block steps, particle steps, pair interactions, dt_min clamps
        self.stats = np.zeros(4, dtype=np.int64)
        clamps = C.c_int64(0)
        rc = _load().or_init(n, self.m, self.x, self.v, self.eps, self.eps_bh, self.bh, self.eta, self.dt_max,
                             self.dt_min, self.a, self.jk, self.t_i, self.dt_i, C.byref(clamps), self.threads)
        if rc:
            raise ValueError(f"or_init failed ({rc})")
        self.stats[3] += clamps.value
        ek, ep = energy(self.m, self.x, self.v, self.eps, eps_bh=self.eps_bh, bh=self.bh)
        self.e0 = ek + ep

    @classmethod
    def from_arrays(cls, m, x, v, a, jk, t_i, dt_i, t_now, eps, eta, dt_max, dt_min, threads=1,
                    eps_bh=None, bh=-1):
        """A state set from saved arrays (no initial force evaluation)."""
        self = cls.__new__(cls)
        self.m = _f64(m).copy()
        n = self.n = self.m.shape[0]
        self.x, self.v = _f64(x, (n, 3)).copy(), _f64(v, (n, 3)).copy()
        self.a, self.jk = _f64(a, (n, 3)).copy(), _f64(jk, (n, 3)).copy()
        self.t_i, self.dt_i = _f64(t_i).copy(), _f64(dt_i).copy()
        self.t_now = float(t_now)
        self.eps, self.eta, self.dt_max, self.dt_min = float(eps), float(eta), float(dt_max), float(dt_min)
        self.eps_bh, self.bh = float(eps if eps_bh is None else eps_bh), int(bh)
        self.threads = int(threads)
        self.stats = np.zeros(4, dtype=np.int64)
        self.e0 = float("nan")
        return self

    def block_step(self):
        """One block step; returns the active indices (ascending)."""
        active = np.zeros(self.n, dtype=np.int64)
        t_now = C.c_double(self.t_now)
        clamps = C.c_int64(0)
        n_act = _load().or_block_step(self.n, self.m, self.x, self.v, self.a, self.jk, self.t_i, self.dt_i,
                                      self.eps, self.eps_bh, self.bh, self.eta, self.dt_max, self.dt_min,
                                      C.byref(t_now), active, C.byref(clamps), self.threads)
        if n_act < 0:
            raise RuntimeError(f"or_block_step failed ({n_act})")
        self.t_now = t_now.value
        self.stats += np.array([1, n_act, n_act * self.n, clamps.value], dtype=np.int64)
        return active[:n_act].copy()

    def run(self, t_end, max_rows=100000):
        """Integrate to t_end (a multiple of dt_max). Returns the log rows
        (t, block_steps, particle_steps, E, RelE, CumE, ekin, epot)."""
        q = t_end / self.dt_max
        if q != math.floor(q) or t_end < self.t_now:
            raise ValueError("t_end must be a multiple of dt_max and not before the current time")
        rows = np.zeros((max_rows, 8))
        t_now = C.c_double(self.t_now)
        stats = np.zeros(4, dtype=np.int64)
        nrows = _load().or_run(self.n, self.m, self.x, self.v, self.a, self.jk, self.t_i, self.dt_i,
                               self.eps, self.eps_bh, self.bh, self.eta, self.dt_max, self.dt_min, C.byref(t_now),
                               float(t_end), float(self.e0), stats, rows, max_rows, self.threads)
        if nrows < 0:
            raise RuntimeError(f"or_run failed ({nrows})")
        self.t_now = t_now.value
        self.stats += stats
        return rows[:nrows].copy()

    def energy(self):
        ek, ep = energy(self.m, self.x, self.v, self.eps, eps_bh=self.eps_bh, bh=self.bh)
        return ek + ep


def lagrange_radii(m, x, fractions):
    """Lagrange radii (the paper's Sec. 4.2: radii of the spheres that hold
    given mass fractions), about the centre of mass: particles in ascending
    distance (ties by index), cumulative mass in that order; the radius for
    fraction f is the distance of the first particle at which the cumulative
    mass reaches f times the total mass. Plain numpy."""
    m = np.asarray(m, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
    mt = 0.0
    for mi in m:
        mt += mi
    com = np.zeros(3)
    for d in range(3):
        acc = 0.0
        for mi, xi in zip(m, x[:, d]):
            acc += mi * xi
        com[d] = acc / mt
    r2 = ((x - com) ** 2).sum(axis=1)
    order = np.argsort(r2, kind="stable")
    cum = np.cumsum(m[order])
    out = []
    for f in fractions:
        k = int(np.searchsorted(cum, f * mt, side="left"))
        k = min(k, len(m) - 1)
        out.append(float(np.sqrt(r2[order[k]])))
    return np.array(out)


def half_mass_relaxation_time(n, total_mass, r_h):
    """Half-mass relaxation time, Eq. (5) with G = 1:
    0.138 (N r_h^3 / m)^(1/2) / ln(0.1 N), m the mean particle mass."""
    mean_m = total_mass / n
    return 0.138 * math.sqrt(n * r_h ** 3 / mean_m) / math.log(0.1 * n)
