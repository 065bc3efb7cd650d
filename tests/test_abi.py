"""CPU checks of the C-ABI library: it loads, exports every entry point that
include/lbf.h declares, and validates arguments before touching a device
(no GPU call is made here)."""
import ctypes
import os
import re

import pytest

from paper_0707_1581_amd import lb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "lbf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = header_functions()
    for n in ("lb_init", "lb_step", "lb_moments", "lb_modes", "lb_populations", "lb_check",
              "lb_batch_init", "lb_batch_step", "lb_batch_view", "lb_autotune"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = lb.lib()
    for n in header_functions():
        assert hasattr(L, n), n
    # the binding marshals exactly the declared set
    assert sorted(s[0] for s in lb.SIGNATURES) == header_functions()


def test_state_bytes():
    L = lb.lib()
    for storage, size in (("f32", 4), ("f16", 2), ("bf16", 2)):
        p = lb.make_params(5, 7, 3, storage=storage)
        assert L.lb_state_bytes(ctypes.byref(p)) == 19 * 5 * 7 * 3 * size
    p = lb.make_params(512, 512, 512)
    assert L.lb_state_bytes(ctypes.byref(p)) == 19 * 512 ** 3 * 4
    for storage, size in (("f32", 4), ("bf16", 2)):
        p = lb.make_params(6, 5, 1, storage=storage, lattice="d2q9")
        assert L.lb_state_bytes(ctypes.byref(p)) == 9 * 6 * 5 * size


def test_d2q9_needs_a_flat_box():
    L = lb.lib()
    p = lb.make_params(8, 8, 2, lattice="d2q9")
    assert L.lb_state_bytes(ctypes.byref(p)) == 0
    ctx = ctypes.c_void_p()
    assert L.lb_init(ctypes.byref(p), ctypes.c_void_p(256), None, 0, None, 0, ctypes.byref(ctx)) == lb.LB_EINVAL
    assert "nz = 1" in L.lb_last_error().decode()


@pytest.mark.parametrize("field,value", [
    ("nx", 0), ("ny", -3), ("storage", 7), ("rho0", 0.0), ("rho0", float("nan")), ("kT", -1e-4),
    ("gamma_bulk", 1.5), ("gamma_shear", -1.01), ("gamma_odd", float("inf")), ("thermal_modes", 5),
    ("lattice", 2), ("lattice", -1)])
def test_invalid_params_rejected_without_device(field, value):
    L = lb.lib()
    p = lb.make_params(4, 4, 4)
    setattr(p, field, value)
    assert L.lb_state_bytes(ctypes.byref(p)) == 0
    ctx = ctypes.c_void_p()
    buf = ctypes.c_void_p(256)  # never dereferenced: validation fails first
    rc = L.lb_init(ctypes.byref(p), buf, None, 0, None, 0, ctypes.byref(ctx))
    assert rc == lb.LB_EINVAL
    assert ctx.value is None
    assert L.lb_last_error().decode()


def test_too_many_sites_unsupported():
    L = lb.lib()
    p = lb.make_params(2048, 2048, 1024)
    assert L.lb_state_bytes(ctypes.byref(p)) == 0
    ctx = ctypes.c_void_p()
    assert L.lb_init(ctypes.byref(p), ctypes.c_void_p(256), None, 0, None, 0,
                     ctypes.byref(ctx)) == lb.LB_EUNSUPPORTED
    # just below 2^32, but a grid of whole workgroups would wrap the 32-bit site index
    p = lb.make_params(512, 8388607, 1, storage="f16", lattice="d2q9")
    assert L.lb_state_bytes(ctypes.byref(p)) == 0
    assert L.lb_init(ctypes.byref(p), ctypes.c_void_p(256), None, 0, None, 0,
                     ctypes.byref(ctx)) == lb.LB_EUNSUPPORTED
    # the largest size used by the tests is accepted
    p = lb.make_params(65536, 65535, 1, storage="f16", lattice="d2q9")
    assert L.lb_state_bytes(ctypes.byref(p)) == 9 * 65536 * 65535 * 2


def test_other_argument_errors():
    L = lb.lib()
    p = lb.make_params(4, 4, 4)
    ctx = ctypes.c_void_p()
    # NULL state, misaligned state, bad init kind, fields missing, negative t0
    assert L.lb_init(ctypes.byref(p), None, None, 0, None, 0, ctypes.byref(ctx)) == lb.LB_EINVAL
    assert L.lb_init(ctypes.byref(p), ctypes.c_void_p(260), None, 0, None, 0, ctypes.byref(ctx)) == lb.LB_EINVAL
    assert L.lb_init(ctypes.byref(p), ctypes.c_void_p(256), None, 9, None, 0, ctypes.byref(ctx)) == lb.LB_EINVAL
    assert L.lb_init(ctypes.byref(p), ctypes.c_void_p(256), None, 2, None, 0, ctypes.byref(ctx)) == lb.LB_EINVAL
    assert L.lb_init(ctypes.byref(p), ctypes.c_void_p(256), None, 0, None, -1, ctypes.byref(ctx)) == lb.LB_EINVAL
    assert L.lb_step(None, 1) == lb.LB_EINVAL
    assert L.lb_propagate(None, 1) == lb.LB_EINVAL
    # copy calibration: argument errors are caught before any device call
    out = ctypes.c_double(0.0)
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30)
    assert L.lb_copy_rate(None, b, 1024, 1, None, ctypes.byref(out)) == lb.LB_EINVAL
    assert L.lb_copy_rate(a, b, 1024, 1, None, None) == lb.LB_EINVAL
    assert L.lb_copy_rate(ctypes.c_void_p((1 << 20) + 16), b, 1024, 1, None, ctypes.byref(out)) == lb.LB_EINVAL
    assert L.lb_copy_rate(a, b, 1000, 1, None, ctypes.byref(out)) == lb.LB_EINVAL
    assert L.lb_copy_rate(a, b, 0, 1, None, ctypes.byref(out)) == lb.LB_EINVAL
    assert L.lb_copy_rate(a, b, 1024, 0, None, ctypes.byref(out)) == lb.LB_EINVAL
    assert L.lb_copy_rate(a, ctypes.c_void_p((1 << 20) + 512), 1024, 1, None, ctypes.byref(out)) == lb.LB_EINVAL
    assert L.lb_moments(None, None) == lb.LB_EINVAL
    assert L.lb_step_count(None) == -1
    L.lb_destroy(None)


def test_batch_pool_layout_and_validation():
    L = lb.lib()
    reps = [lb.make_params(3, 3, 3), lb.make_params(5, 4, 3), lb.make_params(2, 2, 2)]
    arr = (lb.LbParams * 3)(*reps)
    sizes = [19 * 27 * 4, 19 * 60 * 4, 19 * 8 * 4]
    up = [(s + 255) // 256 * 256 for s in sizes]
    assert L.lb_batch_pool_bytes(arr, 3) == sum(up)
    assert [L.lb_batch_offset(arr, 3, r) for r in range(3)] == [0, up[0], up[0] + up[1]]
    mixed = (lb.LbParams * 2)(lb.make_params(3, 3, 3), lb.make_params(3, 3, 3, storage="f16"))
    ctx = ctypes.c_void_p()
    assert L.lb_batch_init(mixed, 2, ctypes.c_void_p(256), None, 1, 0, ctypes.byref(ctx)) == lb.LB_EINVAL
    assert L.lb_batch_init(arr, 3, ctypes.c_void_p(256), None, 2, 0, ctypes.byref(ctx)) == lb.LB_EUNSUPPORTED
    assert L.lb_batch_init(arr, 0, ctypes.c_void_p(256), None, 1, 0, ctypes.byref(ctx)) == lb.LB_EINVAL
    two = (lb.LbParams * 2)(lb.make_params(3, 3, 1), lb.make_params(3, 3, 1, lattice="d2q9"))
    assert L.lb_batch_init(two, 2, ctypes.c_void_p(256), None, 1, 0, ctypes.byref(ctx)) == lb.LB_EINVAL
    assert "same lattice" in L.lb_last_error().decode()


def test_strerror():
    L = lb.lib()
    for code in (0, -1, -2, -3, -4, 17):
        assert L.lb_strerror(code).decode()


def test_workloads_generators_are_deterministic():
    import workloads
    a = workloads.ensemble_replicas()
    b = workloads.ensemble_replicas()
    assert a == b and len(a) == 96
    assert {r["nx"] for r in a} <= set(workloads.ENSEMBLE_SIZES)
    assert len({r["seed"] for r in a}) == 96
    assert all(1e-5 <= r["kT"] <= 1e-3 and 0 <= r["gamma_shear"] <= 0.9 for r in a)


def test_step_noalloc_validates_before_touching_a_device():
    L = lb.lib()
    p = lb.make_params(8, 8, 8)
    arr = (lb.LbParams * 65)(*([p] * 65))
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: every check below fails first
    assert L.lb_step_noalloc(arr, 65, fake, None, 0, 1) == lb.LB_EUNSUPPORTED
    assert "64" in L.lb_last_error().decode()
    assert L.lb_step_noalloc(arr, 0, fake, None, 0, 1) == lb.LB_EINVAL
    assert L.lb_step_noalloc(None, 1, fake, None, 0, 1) == lb.LB_EINVAL
    assert L.lb_step_noalloc(arr, 1, ctypes.c_void_p((1 << 20) + 4), None, 0, 1) == lb.LB_EINVAL  # misaligned
    assert L.lb_step_noalloc(arr, 1, None, None, 0, 1) == lb.LB_EINVAL
    assert L.lb_step_noalloc(arr, 1, fake, None, -1, 1) == lb.LB_EINVAL
    assert L.lb_step_noalloc(arr, 1, fake, None, 0, -1) == lb.LB_EINVAL
    mixed = (lb.LbParams * 2)(p, lb.make_params(8, 8, 8, storage="f16"))
    assert L.lb_step_noalloc(mixed, 2, fake, None, 0, 1) == lb.LB_EINVAL
    bad = (lb.LbParams * 1)(lb.make_params(0, 8, 8))
    assert L.lb_step_noalloc(bad, 1, fake, None, 0, 1) == lb.LB_EINVAL
    assert L.lb_step_noalloc(arr, 1, fake, None, 0, 0) == lb.LB_OK  # nothing to do: no device call
