"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function declared in include/hlbm.h, and validates configurations
before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2312_14172_amd import hlbm as H

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "hlbm.h")).read()
    return sorted(set(re.findall(r"\b(hlbm_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_function():
    L = H.lib()
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(H.EXPORTED)


def test_particle_record_layout_matches_header():
    # 21 doubles + 2 int32 = 176 bytes, field order as declared
    assert H.HLBM_PARTICLE.itemsize == 176
    # 8 int32, 9 doubles, the stream pointer, 2 int32, 1 double, 2 int32
    assert ctypes.sizeof(H.hlbm_config) == 4 * 8 + 8 * 9 + 8 + 4 + 4 + 8 + 4 + 4
    assert H.hlbm_config.max_mesh_triangles.offset == 128
    assert H.hlbm_config.coupling.offset == 132


def _size(**kw):
    cfg = H.make_config(**kw)
    n = ctypes.c_size_t(0)
    rc = H.lib().hlbm_workspace_size(ctypes.byref(cfg), ctypes.byref(n))
    return rc, n.value


def test_workspace_size_counts_both_population_buffers():
    rc64, b64 = _size(n=(64, 32, 16), precision="fp64")
    rc32, b32 = _size(n=(64, 32, 16), precision="fp32")
    rc16, b16 = _size(n=(64, 32, 16), precision="fp16s")
    assert rc64 == rc32 == rc16 == 0
    N = 64 * 32 * 16
    assert b64 - b32 == 2 * 19 * N * 4
    assert b32 - b16 == 2 * 19 * N * 2


@pytest.mark.parametrize("kw,code", [
    (dict(n=(0, 4, 4)), -1),
    (dict(n=(8, 8, 8), tau=0.5), -1),
    (dict(n=(8, 8, 8), tau=float("nan")), -1),
    (dict(n=(8, 8, 8), eps=0.0), -1),
    (dict(n=(8, 8, 8), bc=(0, 2, 0)), -1),
    (dict(n=(8, 8, 8), precision=7), -1),
    (dict(n=(8, 8, 8), max_particles=-1), -1),
    # distance tables of (2 (27 + 100) + 2)^3 cells per particle
    (dict(n=(8, 8, 8), max_particles=1, learned_max_circumradius=27.0, max_mesh_triangles=4, eps=200.0), -6),
])
def test_invalid_configurations_are_rejected(kw, code):
    rc, _ = _size(**kw)
    assert rc == code
    assert H.lib().hlbm_last_error().decode()


def test_init_rejects_null_workspace():
    cfg = H.make_config(n=(8, 8, 8))
    ctx = ctypes.c_void_p()
    rc = H.lib().hlbm_init(ctypes.byref(cfg), None, 1 << 20, ctypes.byref(ctx))
    assert rc == -1 and not ctx.value
