"""C ABI checks that need no GPU: the library loads, exports every entry
point the header declares, and rejects bad arguments before touching the
device."""
import ctypes
import math
import os

import numpy as np
import pytest

import paper_1801_10187_amd as m
from paper_1801_10187_amd import binding

LIB = binding.LIB_PATH


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmpcd.so is not built (run python -m paper_1801_10187_amd.build)")
    return m.load()


def test_header_declares_the_step_entry_points():
    names = m.declared_symbols()
    for n in ("mpcd_create", "mpcd_stream", "mpcd_bin", "mpcd_collide", "mpcd_step",
              "mpcd_get_state", "mpcd_get_cells", "mpcd_destroy", "mpcd_last_error"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    out = os.popen(f"nm -D --defined-only {LIB}").read()
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in m.declared_symbols() if n not in exported]
    assert not missing, f"declared but not exported: {missing}"


def test_library_is_built_for_gfx950():
    data = open(LIB, "rb").read()
    assert b"gfx950" in data


def _create(lib, p, n=1, pos=None, vel=None):
    pos = np.full((max(n, 1), 3), 0.5) if pos is None else pos
    vel = np.zeros_like(pos) if vel is None else vel
    ctx = ctypes.c_void_p()
    st = lib.mpcd_create(ctypes.byref(p), n, binding._ptr(pos), binding._ptr(vel), 0,
                         None, None, None, 0, None, ctypes.byref(ctx))
    return st, ctx


@pytest.mark.parametrize("field,value", [("a", 0.0), ("a", -1.0), ("dt", -0.1),
                                         ("kT", -1.0), ("solvent_mass", 0.0),
                                         ("precision", 7), ("thermostat", 2),
                                         ("grid_shift", 5), ("flags", 4),
                                         ("alpha", float("nan")), ("collision", 2)])
def test_create_rejects_bad_parameters(lib, field, value):
    p = m.make_params((4, 4, 4))
    setattr(p, field, value)
    st, ctx = _create(lib, p)
    assert st == binding.MPCD_EINVAL
    assert ctx.value is None
    assert lib.mpcd_last_error().decode() != ""


def test_create_rejects_bad_sizes(lib):
    p = m.make_params((0, 4, 4))
    assert _create(lib, p)[0] == binding.MPCD_EINVAL
    p = m.make_params((2000, 4, 4), precision=m.FP32)
    assert _create(lib, p)[0] == binding.MPCD_EINVAL
    p = m.make_params((4, 4, 4))
    assert _create(lib, p, n=-1)[0] == binding.MPCD_EINVAL


def test_null_context_is_an_error(lib):
    for fn in (lib.mpcd_stream, lib.mpcd_bin, lib.mpcd_collide, lib.mpcd_sync):
        assert fn(None) == binding.MPCD_EINVAL
    assert lib.mpcd_step(None, 1) == binding.MPCD_EINVAL
    lib.mpcd_destroy(None)   # no-op


def test_bad_copy_and_philox_arguments(lib):
    assert lib.mpcd_copy_kernel(None, None, -1, None) == binding.MPCD_EINVAL
    assert lib.mpcd_philox4x32_10(None, -5, 0, None) == binding.MPCD_EINVAL


def _create_batch(lib, plist, counts):
    arr = (binding.Params * len(plist))(*plist)
    n = np.asarray(counts, dtype=np.int64)
    tot = int(n.sum())
    pos = np.full((max(tot, 1), 3), 0.5)
    vel = np.zeros((max(tot, 1), 3))
    ctx = ctypes.c_void_p()
    st = lib.mpcd_create_batch(len(plist), arr, n.ctypes.data_as(ctypes.c_void_p),
                               pos.ctypes.data_as(ctypes.c_void_p),
                               vel.ctypes.data_as(ctypes.c_void_p), 0, None, ctypes.byref(ctx))
    return st, ctx


def test_batch_create_rejects_bad_boxes(lib):
    """Validation happens before any device work: no GPU needed."""
    good = m.make_params((4, 4, 4))
    assert lib.mpcd_create_batch(0, None, None, None, None, 0, None,
                                 ctypes.byref(ctypes.c_void_p())) == binding.MPCD_EINVAL
    bad = m.make_params((4, 4, 4), dt=-1.0)
    st, ctx = _create_batch(lib, [good, bad], [3, 3])
    assert st == binding.MPCD_EINVAL and ctx.value is None
    assert lib.mpcd_last_error().decode().startswith("box 1")
    mixed = m.make_params((4, 4, 4), precision=m.FP32)
    st, _ = _create_batch(lib, [good, mixed], [3, 3])
    assert st == binding.MPCD_EINVAL
    assert "must match box 0" in lib.mpcd_last_error().decode()
    st, _ = _create_batch(lib, [good, good], [3, -1])
    assert st == binding.MPCD_EINVAL


def test_at_rule_excludes_the_rotation_thermostat(lib):
    p = m.make_params((4, 4, 4), thermostat=True, collision=m.AT)
    st, ctx = _create(lib, p)
    assert st == binding.MPCD_EINVAL and ctx.value is None
    assert "AT rule" in lib.mpcd_last_error().decode()
