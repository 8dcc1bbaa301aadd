"""CPU-side checks of the HIP library: it is built for gfx950, it exports
every entry point the public header declares, and the host-side argument
checks answer without touching a GPU."""
import ctypes as C
import os
import re
import subprocess

import pytest
import torch  # noqa: F401  (binds the library to torch's HIP runtime)

from paper_1702_00440_amd import gravidy as g

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gravidy_hip.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(gd_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for want in ["gd_init", "gd_predict", "gd_force", "gd_correct", "gd_step_to", "gd_energy",
                 "gd_workspace_bytes", "gd_active", "gd_get_state", "gd_set_state", "gd_stats_get",
                 "gd_destroy", "gd_last_error"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(g.LIB_PATH), "run the build first"
    out = subprocess.run(["nm", "-D", "--defined-only", g.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\bT (gd_[a-z_]+)\b", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing
    lib = g.library()
    for n in _declared():
        assert hasattr(lib, n)


def test_binding_constants_match_the_header():
    """Every #define GD_<NAME> <integer> of the public header has the same
    value in the binding (buffers the binding sizes from them must hold what
    the library writes)."""
    text = open(HEADER).read()
    found = re.findall(r"#define\s+(GD_[A-Z0-9_]+)\s+(\d+)\b", text)
    assert len(found) >= 5
    for name, value in found:
        assert getattr(g, name) == int(value), name


def test_library_has_gfx950_code_object():
    data = open(g.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_workspace_bytes_host_only():
    b1 = g.gd_workspace_bytes(1024)
    b2 = g.gd_workspace_bytes(16384)
    assert b2 > b1 > 1024 * 8 * 25
    assert b1 % 256 == 0
    with pytest.raises(g.GdError) as e:
        g.gd_workspace_bytes(1)
    assert e.value.status == g.GD_EINVAL


def test_workspace_bytes_follow_items_per_lane():
    # Contexts of 131072 or more softened particles hold four i per lane, which
    # needs a larger partial-force buffer; NULL parameters give the larger size.
    big = 131072
    soft = g.make_params(eps=1e-4)
    hard = g.make_params(eps=0.0)
    b_soft = g.gd_workspace_bytes(big, soft)
    b_hard = g.gd_workspace_bytes(big, hard)
    assert b_soft > b_hard
    assert g.gd_workspace_bytes(big) == b_soft
    assert g.gd_workspace_bytes(big - 1, soft) == g.gd_workspace_bytes(big - 1, hard)
    assert g.gd_workspace_bytes(big - 1) >= g.gd_workspace_bytes(big - 1, soft)


def test_init_rejects_workspace_sized_for_two_i_per_lane():
    lib = g.library()
    n = 131072
    p = g.make_params(eps=1e-4)
    short = g.gd_workspace_bytes(n, g.make_params(eps=0.0))
    assert short < g.gd_workspace_bytes(n, p)
    ctx = C.c_void_p()
    dummy = C.c_void_p(256)
    rc = lib.gd_init(C.byref(ctx), C.byref(p), n, dummy, dummy, dummy, dummy, short, None)
    assert rc == g.GD_ENOMEM
    assert "workspace" in g.gd_last_error(None)


@pytest.mark.parametrize("kw,msg", [
    (dict(eta=0.0), "eta"),
    (dict(eta=float("nan")), "eta"),
    (dict(eps=-1.0), "eps"),
    (dict(eps=1e-40), "eps"),
    (dict(dt_max=0.1), "power"),
    (dict(dt_min=0.25), "power"),
    (dict(dt_min=2.0 ** -60), "40"),
    (dict(flags=2), "flags"),
    (dict(flags=g.GD_FLAG_MIXED, eps=1e-11), "eps^2 >= 1e-20"),
    (dict(flags=g.GD_FLAG_MIXED, eps=5e-11), "eps^2 >= 1e-20"),
])
def test_init_rejects_bad_params_before_any_device_work(kw, msg):
    """Parameter validation happens on the host before any HIP call, so it can
    run here with dummy (never dereferenced) pointers."""
    lib = g.library()
    p = g.make_params(**kw)
    ctx = C.c_void_p()
    dummy = C.c_void_p(256)
    rc = lib.gd_init(C.byref(ctx), C.byref(p), 16, dummy, dummy, dummy, dummy, 1 << 30, None)
    assert rc == g.GD_EINVAL
    assert not ctx.value
    assert msg in g.gd_last_error(None)


def test_mixed_softening_bound_accepts_zero_and_1e_minus_10():
    """GD_FLAG_MIXED takes eps = 0 (the self pair is masked) and eps^2 >=
    1e-20; those pass the host checks and stop only at the workspace size."""
    lib = g.library()
    ctx = C.c_void_p()
    dummy = C.c_void_p(256)
    for eps in (0.0, 1e-10, 1e-4):
        p = g.make_params(flags=g.GD_FLAG_MIXED, eps=eps)
        rc = lib.gd_init(C.byref(ctx), C.byref(p), 16, dummy, dummy, dummy, dummy, 1, None)
        assert rc == g.GD_ENOMEM, eps


def test_init_rejects_short_workspace_and_null():
    lib = g.library()
    p = g.make_params()
    ctx = C.c_void_p()
    dummy = C.c_void_p(256)
    need = g.gd_workspace_bytes(16)
    rc = lib.gd_init(C.byref(ctx), C.byref(p), 16, dummy, dummy, dummy, dummy, need - 1, None)
    assert rc == g.GD_ENOMEM
    rc = lib.gd_init(C.byref(ctx), C.byref(p), 16, None, dummy, dummy, dummy, need, None)
    assert rc == g.GD_EINVAL
    rc = lib.gd_init(C.byref(ctx), C.byref(p), 1, dummy, dummy, dummy, dummy, need, None)
    assert rc == g.GD_EINVAL
    misaligned = C.c_void_p(256 + 8)
    rc = lib.gd_init(C.byref(ctx), C.byref(p), 16, dummy, dummy, dummy, misaligned, need, None)
    assert rc == g.GD_EINVAL


def test_null_context_is_rejected():
    lib = g.library()
    assert lib.gd_predict(None, None) == g.GD_EINVAL
    assert lib.gd_correct(None) == g.GD_EINVAL
    assert lib.gd_step_to(None, 1.0, None) == g.GD_EINVAL
    assert lib.gd_progress(None, 1.0) == g.GD_EINVAL
    counts = (C.c_int64 * g.GD_NACT_BINS)()
    assert lib.gd_nact_histogram(None, counts) == g.GD_EINVAL
    assert lib.gd_profile_buckets(None, None, None, None, None) == g.GD_EINVAL
    lib.gd_destroy(None)


def test_binding_refuses_host_tensors():
    with pytest.raises(TypeError):
        g._ptr(torch.zeros(3, dtype=torch.float64), torch.float64)


def test_init_rejects_bad_central_particle():
    lib = g.library()
    ctx = C.c_void_p()
    dummy = C.c_void_p(256)
    for kw in [dict(bh_index=16), dict(bh_index=-2), dict(bh_index=3, eps_bh=0.0), dict(bh_index=3, eps=0.0)]:
        p = g.make_params(**kw)
        rc = lib.gd_init(C.byref(ctx), C.byref(p), 16, dummy, dummy, dummy, dummy, 1 << 30, None)
        assert rc == g.GD_EINVAL, kw


def test_pool_create_validation_host_only():
    lib = g.library()
    pool = C.c_void_p()
    dummy = C.c_void_p(256)
    for kw, mc in [(dict(), 0), (dict(), 257), (dict(eps=0.0), 4), (dict(bh_index=1, eps_bh=1e-6), 4)]:
        p = g.make_params(**kw)
        rc = lib.gd_pool_create(C.byref(pool), C.byref(p), mc, dummy, 1 << 30, None)
        assert rc == g.GD_EINVAL, (kw, mc)
    assert g.gd_pool_arena_bytes(4, [256, 512]) > g.gd_workspace_bytes(256) + g.gd_workspace_bytes(512)


def test_force_noalloc_checks_sizes_on_the_host():
    """gd_force_noalloc rejects sizes beyond its scratch array, and an empty
    list, before any device work (so these answer without a GPU)."""
    lib = g.library()
    p = g.make_params()
    rc = lib.gd_force_noalloc(C.byref(p), g.GD_NOALLOC_MAX_N + 1, None, None, None, None, 4, None, None, None)
    assert rc == g.GD_EINVAL
    assert b"GD_NOALLOC_MAX_N" in lib.gd_last_error(None)
    assert lib.gd_force_noalloc(C.byref(p), 1000, None, None, None, None, 1001, None, None, None) == g.GD_EINVAL
    assert lib.gd_force_noalloc(C.byref(p), 1000, None, None, None, None, -1, None, None, None) == g.GD_EINVAL
    assert lib.gd_force_noalloc(C.byref(p), 1000, None, None, None, None, 0, None, None, None) == g.GD_OK
    bad = g.make_params(eps=-1.0)
    assert lib.gd_force_noalloc(C.byref(bad), 1000, None, None, None, None, 4, None, None, None) == g.GD_EINVAL
