"""Python binding of the C ABI in include/gravidy_hip.h (argument marshalling only).

Every function here has the name of the C entry point it calls; all
arithmetic runs in the HIP library. PyTorch supplies device memory (the
workspace and the array arguments, as CUDA/HIP tensors) and the stream.

The library must have been built (paper_1702_00440_amd/build.py, or the
repository's build entry point); importing it fails loudly otherwise. torch is
imported first so that the library binds to the HIP runtime torch loaded.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgravidy_hip.so")

GD_OK, GD_EINVAL, GD_ENOMEM, GD_EHIP, GD_ESTATE, GD_ENONFINITE = 0, -1, -2, -3, -4, -5
GD_FLAG_MIXED = 1
GD_POOL_MAX_CLUSTERS = 256
_NAMES = {GD_EINVAL: "GD_EINVAL", GD_ENOMEM: "GD_ENOMEM", GD_EHIP: "GD_EHIP",
          GD_ESTATE: "GD_ESTATE", GD_ENONFINITE: "GD_ENONFINITE"}


def status_name(status: int) -> str:
    """Name of a gd_status value ("GD_OK", "GD_EINVAL", ...)."""
    return "GD_OK" if status == GD_OK else _NAMES.get(status, str(status))


class GdError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_NAMES.get(status, status)}: {message}")
        self.status = status


class gd_params(C.Structure):
    _fields_ = [("eta", C.c_double), ("eps", C.c_double), ("eps_bh", C.c_double), ("dt_max", C.c_double),
                ("dt_min", C.c_double), ("bh_index", C.c_int64), ("flags", C.c_int32)]


class gd_stats(C.Structure):
    _fields_ = [("t", C.c_double), ("block_steps", C.c_int64), ("particle_steps", C.c_int64),
                ("pair_interactions", C.c_int64), ("dtmin_clamps", C.c_int64),
                ("e0", C.c_double), ("e", C.c_double), ("wall_s", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None
_VP = C.c_void_p


def library():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"HIP library not built: {LIB_PATH} is missing "
                          "(run paper_1702_00440_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    i64, st = C.c_int64, C.c_int
    lib.gd_workspace_bytes.argtypes = [i64, C.POINTER(gd_params), C.POINTER(C.c_size_t)]
    lib.gd_init.argtypes = [C.POINTER(_VP), C.POINTER(gd_params), i64, _VP, _VP, _VP, _VP, C.c_size_t, _VP]
    lib.gd_reinit.argtypes = [_VP, _VP, _VP, _VP]
    lib.gd_profile_force.argtypes = [_VP, C.c_int]
    lib.gd_profile_get.argtypes = [_VP, C.POINTER(C.c_double), C.POINTER(i64), C.POINTER(i64)]
    lib.gd_profile_buckets.argtypes = [_VP, C.POINTER(i64), C.POINTER(C.c_double), C.POINTER(i64),
                                       C.POINTER(i64)]
    lib.gd_predict.argtypes = [_VP, C.POINTER(C.c_double)]
    lib.gd_force.argtypes = [_VP, _VP, i64, _VP, _VP]
    lib.gd_force_plan.argtypes = [_VP, _VP, i64, C.c_int32, C.c_int32, _VP, _VP]
    lib.gd_force_plan.restype = st
    lib.gd_active.argtypes = [_VP, _VP, C.POINTER(i64)]
    lib.gd_correct.argtypes = [_VP]
    lib.gd_step_to.argtypes = [_VP, C.c_double, C.POINTER(gd_stats)]
    lib.gd_progress.argtypes = [_VP, C.c_double]
    lib.gd_energy.argtypes = [_VP, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.gd_get_state.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, _VP, C.POINTER(C.c_double)]
    lib.gd_set_state.argtypes = [_VP, _VP, _VP, _VP, _VP, _VP, _VP, C.c_double]
    lib.gd_stats_get.argtypes = [_VP, C.POINTER(gd_stats)]
    lib.gd_nact_histogram.argtypes = [_VP, C.POINTER(i64)]
    lib.gd_refills.argtypes = [_VP, C.POINTER(i64)]
    lib.gd_refills.restype = st
    lib.gd_diagnostics.argtypes = [_VP, C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_double),
                                   C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(i64), C.c_int32]
    lib.gd_diagnostics.restype = st
    for name in ["gd_workspace_bytes", "gd_init", "gd_reinit", "gd_profile_force", "gd_profile_get", "gd_profile_buckets", "gd_predict", "gd_force", "gd_active", "gd_correct",
                 "gd_step_to", "gd_energy", "gd_get_state", "gd_set_state", "gd_stats_get", "gd_nact_histogram"]:
        getattr(lib, name).restype = st
    lib.gd_pool_arena_bytes.argtypes = [C.c_int32, C.POINTER(i64), C.c_int32, C.POINTER(C.c_size_t)]
    lib.gd_pool_create.argtypes = [C.POINTER(_VP), C.POINTER(gd_params), C.c_int32, _VP, C.c_size_t, _VP]
    lib.gd_pool_admit.argtypes = [_VP, i64, _VP, _VP, _VP, C.c_double, C.POINTER(C.c_int32)]
    lib.gd_pool_run.argtypes = [_VP, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.gd_pool_result.argtypes = [_VP, C.c_int32, _VP, _VP, C.POINTER(gd_stats)]
    lib.gd_pool_release.argtypes = [_VP, C.c_int32]
    lib.gd_pool_resident.argtypes = [_VP, C.POINTER(C.c_int32)]
    for name in ["gd_pool_arena_bytes", "gd_pool_create", "gd_pool_admit", "gd_pool_run", "gd_pool_result",
                 "gd_pool_release", "gd_pool_resident"]:
        getattr(lib, name).restype = st
    lib.gd_pool_destroy.argtypes = [_VP]
    lib.gd_pool_destroy.restype = None
    lib.gd_pool_last_error.argtypes = [_VP]
    lib.gd_pool_last_error.restype = C.c_char_p
    lib.gd_destroy.argtypes = [_VP]
    lib.gd_destroy.restype = None
    lib.gd_last_error.argtypes = [_VP]
    lib.gd_last_error.restype = C.c_char_p
    lib.gd_force_noalloc.argtypes = [C.POINTER(gd_params), i64, _VP, _VP, _VP, _VP, i64, _VP, _VP, _VP]
    lib.gd_force_noalloc.restype = st
    _lib = lib
    return lib


def _check(rc: int, ctx) -> None:
    if rc != GD_OK:
        msg = library().gd_last_error(ctx)
        raise GdError(rc, msg.decode() if msg else "")


def _check_pool(rc: int, pool) -> None:
    if rc != GD_OK:
        msg = library().gd_pool_last_error(pool)
        raise GdError(rc, msg.decode() if msg else "")


def _ptr(t, dtype, shape=None, name="array"):
    """Device pointer of a contiguous tensor of the given dtype (None -> NULL)."""
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


# One int32 element per device whose address stands for an empty index list:
# an empty tensor has no storage (its data pointer is NULL), and the C ABI
# reads a NULL index list as "the current active set". With n_act = 0 the
# library never reads through the pointer.
_EMPTY_LIST = {}


def _list_ptr(idx, name="idx"):
    """Device pointer of an int32 index list; an empty list gets a non-NULL address."""
    p = _ptr(idx, torch.int32, None, name)
    if idx is not None and idx.numel() == 0 and not p:
        key = idx.device
        if key not in _EMPTY_LIST:
            _EMPTY_LIST[key] = torch.zeros(1, dtype=torch.int32, device=key)
        p = _EMPTY_LIST[key].data_ptr()
    return p


def _stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def make_params(eta=0.01, eps=1e-4, dt_max=0.125, dt_min=2.0 ** -22, flags=0, eps_bh=None,
                bh_index=-1) -> gd_params:
    e_bh = float(eps if eps_bh is None else eps_bh)
    return gd_params(float(eta), float(eps), e_bh, float(dt_max), float(dt_min), int(bh_index), int(flags))


def gd_workspace_bytes(n: int, params: gd_params | None = None) -> int:
    out = C.c_size_t()
    rc = library().gd_workspace_bytes(int(n), C.byref(params) if params is not None else None, C.byref(out))
    _check(rc, None)
    return int(out.value)


def gd_init(params: gd_params, m, x, v, workspace, stream=None):
    """Returns the context handle (an opaque pointer)."""
    n = m.shape[0]
    ctx = _VP()
    rc = library().gd_init(C.byref(ctx), C.byref(params), n, _ptr(m, torch.float64, (n,), "m"),
                           _ptr(x, torch.float64, (n, 3), "x"), _ptr(v, torch.float64, (n, 3), "v"),
                           _ptr(workspace, torch.uint8, None, "workspace"), workspace.numel(),
                           _stream_handle(stream))
    _check(rc, None)
    return ctx


def gd_reinit(ctx, m, x, v) -> None:
    n = m.shape[0]
    _check(library().gd_reinit(ctx, _ptr(m, torch.float64, (n,), "m"), _ptr(x, torch.float64, (n, 3), "x"),
                               _ptr(v, torch.float64, (n, 3), "v")), ctx)


def gd_profile_force(ctx, enable: bool = True) -> None:
    _check(library().gd_profile_force(ctx, int(bool(enable))), ctx)


def gd_profile_get(ctx) -> dict:
    ms, launches, pairs = C.c_double(), C.c_int64(), C.c_int64()
    _check(library().gd_profile_get(ctx, C.byref(ms), C.byref(launches), C.byref(pairs)), ctx)
    return {"force_ms": ms.value, "launches": int(launches.value), "pairs": int(pairs.value)}


GD_PROFILE_BUCKETS = 6


def gd_profile_buckets(ctx) -> list:
    """Force-launch timing by block size: one dict per N_act bucket."""
    nb = GD_PROFILE_BUCKETS
    lo, ms, launches, pairs = (C.c_int64 * nb)(), (C.c_double * nb)(), (C.c_int64 * nb)(), (C.c_int64 * nb)()
    _check(library().gd_profile_buckets(ctx, lo, ms, launches, pairs), ctx)
    out = []
    for b in range(nb):
        hi = int(lo[b + 1]) - 1 if b + 1 < nb else None
        out.append({"n_act_min": int(lo[b]), "n_act_max": hi, "force_ms": ms[b], "launches": int(launches[b]),
                    "pairs": int(pairs[b])})
    return out


def gd_predict(ctx, t: float | None = None) -> None:
    tp = C.byref(C.c_double(t)) if t is not None else None
    _check(library().gd_predict(ctx, tp), ctx)


def gd_force(ctx, idx=None, acc=None, jerk=None) -> None:
    n_act = 0 if idx is None else idx.shape[0]
    _check(library().gd_force(ctx, _list_ptr(idx), n_act,
                              _ptr(acc, torch.float64, None, "acc"), _ptr(jerk, torch.float64, None, "jerk")), ctx)


def gd_force_plan(ctx, idx, lanes_per_i: int, slices: int, acc=None, jerk=None) -> None:
    """gd_force of an index list with a chosen decomposition of the force
    kernel (lanes per listed particle, j slices)."""
    n_act = idx.shape[0]
    _check(library().gd_force_plan(ctx, _list_ptr(idx), n_act, int(lanes_per_i),
                                   int(slices), _ptr(acc, torch.float64, None, "acc"),
                                   _ptr(jerk, torch.float64, None, "jerk")), ctx)


GD_NOALLOC_MAX_N = 65536


def gd_force_noalloc(params: gd_params, m, x, v, idx, acc=None, jerk=None, stream=None) -> None:
    """Acceleration and jerk of the listed particles without a context or any
    device allocation (the library's scratch array); queued, not synchronised."""
    n = m.shape[0]
    n_act = idx.shape[0]
    rc = library().gd_force_noalloc(C.byref(params), n, _ptr(m, torch.float64, (n,), "m"),
                                    _ptr(x, torch.float64, (n, 3), "x"), _ptr(v, torch.float64, (n, 3), "v"),
                                    _ptr(idx, torch.int32, (n_act,), "idx"), n_act,
                                    _ptr(acc, torch.float64, (n_act, 3), "acc"),
                                    _ptr(jerk, torch.float64, (n_act, 3), "jerk"), _stream_handle(stream))
    _check(rc, None)


def gd_active(ctx, idx=None) -> int:
    n = C.c_int64()
    _check(library().gd_active(ctx, _ptr(idx, torch.int32, None, "idx"), C.byref(n)), ctx)
    return int(n.value)


def gd_correct(ctx) -> None:
    _check(library().gd_correct(ctx), ctx)


def gd_step_to(ctx, t_end: float) -> dict:
    st = gd_stats()
    _check(library().gd_step_to(ctx, float(t_end), C.byref(st)), ctx)
    return st.as_dict()


def gd_progress(ctx, interval_s: float) -> None:
    _check(library().gd_progress(ctx, float(interval_s)), ctx)


def gd_energy(ctx, unsoftened: bool = False):
    ek, ep, eu = C.c_double(), C.c_double(), C.c_double()
    _check(library().gd_energy(ctx, C.byref(ek), C.byref(ep), C.byref(eu) if unsoftened else None), ctx)
    return (ek.value, ep.value, eu.value) if unsoftened else (ek.value, ep.value)


def gd_get_state(ctx, x=None, v=None, a=None, jerk=None, t_i=None, dt_i=None) -> float:
    t_now = C.c_double()
    f = torch.float64
    _check(library().gd_get_state(ctx, _ptr(x, f, None, "x"), _ptr(v, f, None, "v"), _ptr(a, f, None, "a"),
                                  _ptr(jerk, f, None, "jerk"), _ptr(t_i, f, None, "t_i"),
                                  _ptr(dt_i, f, None, "dt_i"), C.byref(t_now)), ctx)
    return t_now.value


def gd_set_state(ctx, x, v, a, jerk, t_i, dt_i, t_now: float) -> None:
    f = torch.float64
    _check(library().gd_set_state(ctx, _ptr(x, f, None, "x"), _ptr(v, f, None, "v"), _ptr(a, f, None, "a"),
                                  _ptr(jerk, f, None, "jerk"), _ptr(t_i, f, None, "t_i"),
                                  _ptr(dt_i, f, None, "dt_i"), float(t_now)), ctx)


def gd_diagnostics(ctx, fractions=(0.01, 0.05, 0.1, 0.25, 0.5, 0.75, 0.9), n_levels=41) -> dict:
    """Lagrange radii at the given mass fractions, half-mass relaxation time
    (Eq. 5) and the particles per block-step level, from the device."""
    nf = len(fractions)
    fr = (C.c_double * max(1, nf))(*[float(f) for f in fractions])
    radii = (C.c_double * max(1, nf))()
    t_rh, r_half = C.c_double(), C.c_double()
    levels = (C.c_int64 * max(1, n_levels))()
    _check(library().gd_diagnostics(ctx, fr, nf, radii, C.byref(t_rh), C.byref(r_half), levels, n_levels), ctx)
    return {"fractions": list(fractions), "radii": [radii[k] for k in range(nf)], "t_rh": t_rh.value,
            "r_half": r_half.value, "levels": [int(levels[k]) for k in range(n_levels)]}


def gd_stats_get(ctx) -> dict:
    st = gd_stats()
    _check(library().gd_stats_get(ctx, C.byref(st)), ctx)
    return st.as_dict()


GD_NACT_BINS = 32


def gd_nact_histogram(ctx) -> list:
    """Block steps since init / reinit / set_state by active-block size:
    entry b counts the steps with 2^b <= N_act < 2^(b+1)."""
    counts = (C.c_int64 * GD_NACT_BINS)()
    _check(library().gd_nact_histogram(ctx, counts), ctx)
    return [int(c) for c in counts]


def gd_refills(ctx) -> int:
    """Replayed steps that rebuilt their active list instead of stepping."""
    r = C.c_int64()
    _check(library().gd_refills(ctx, C.byref(r)), ctx)
    return int(r.value)


def gd_destroy(ctx) -> None:
    if ctx:
        library().gd_destroy(ctx)


def gd_last_error(ctx=None) -> str:
    msg = library().gd_last_error(ctx)
    return msg.decode() if msg else ""


def gd_pool_arena_bytes(max_clusters: int, ns) -> int:
    arr = (C.c_int64 * max(1, len(ns)))(*[int(v) for v in ns])
    out = C.c_size_t()
    _check_pool(library().gd_pool_arena_bytes(int(max_clusters), arr, len(ns), C.byref(out)), None)
    return int(out.value)


def gd_pool_create(params: gd_params, max_clusters: int, arena, stream=None):
    pool = _VP()
    rc = library().gd_pool_create(C.byref(pool), C.byref(params), int(max_clusters),
                                  _ptr(arena, torch.uint8, None, "arena"), arena.numel(), _stream_handle(stream))
    _check_pool(rc, None)
    return pool


def gd_pool_admit(pool, m, x, v, t_end: float):
    """Slot of the admitted cluster, or None when no slot or arena room is free."""
    n = m.shape[0]
    slot = C.c_int32(-1)
    rc = library().gd_pool_admit(pool, n, _ptr(m, torch.float64, (n,), "m"), _ptr(x, torch.float64, (n, 3), "x"),
                                 _ptr(v, torch.float64, (n, 3), "v"), float(t_end), C.byref(slot))
    if rc == GD_ENOMEM:
        return None
    _check_pool(rc, pool)
    return int(slot.value)


def gd_pool_run(pool) -> list:
    fin = (C.c_int32 * GD_POOL_MAX_CLUSTERS)()
    nf = C.c_int32(0)
    _check_pool(library().gd_pool_run(pool, fin, C.byref(nf)), pool)
    return [int(fin[k]) for k in range(nf.value)]


def gd_pool_result(pool, slot: int, x=None, v=None) -> dict:
    st = gd_stats()
    f = torch.float64
    _check_pool(library().gd_pool_result(pool, int(slot), _ptr(x, f, None, "x"), _ptr(v, f, None, "v"),
                                         C.byref(st)), pool)
    return st.as_dict()


def gd_pool_release(pool, slot: int) -> None:
    _check_pool(library().gd_pool_release(pool, int(slot)), pool)


def gd_pool_resident(pool) -> int:
    c = C.c_int32()
    _check_pool(library().gd_pool_resident(pool, C.byref(c)), pool)
    return int(c.value)


def gd_pool_destroy(pool) -> None:
    if pool:
        library().gd_pool_destroy(pool)


class Cluster:
    """One context plus the device workspace it owns (a torch uint8 tensor)."""

    def __init__(self, m, x, v, eta=0.01, eps=1e-4, dt_max=0.125, dt_min=2.0 ** -22,
                 device="cuda", stream=None, eps_bh=None, bh_index=-1, flags=0):
        self.params = make_params(eta, eps, dt_max, dt_min, flags=flags, eps_bh=eps_bh,
                                  bh_index=bh_index)
        dev = torch.device(device)
        self.m = torch.as_tensor(m, dtype=torch.float64).to(dev).contiguous()
        self.n = self.m.shape[0]
        xt = torch.as_tensor(x, dtype=torch.float64).to(dev).reshape(self.n, 3).contiguous()
        vt = torch.as_tensor(v, dtype=torch.float64).to(dev).reshape(self.n, 3).contiguous()
        nbytes = gd_workspace_bytes(self.n, self.params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream
        self.ctx = gd_init(self.params, self.m, xt, vt, self.workspace, stream)

    def close(self):
        if getattr(self, "ctx", None):
            gd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def state(self):
        """(x, v, a, jerk, t_i, dt_i, t_now) as device tensors (+ float)."""
        dev = self.m.device
        x, v, a, j = (torch.empty(self.n, 3, dtype=torch.float64, device=dev) for _ in range(4))
        t_i, dt_i = (torch.empty(self.n, dtype=torch.float64, device=dev) for _ in range(2))
        t_now = gd_get_state(self.ctx, x, v, a, j, t_i, dt_i)
        return x, v, a, j, t_i, dt_i, t_now
