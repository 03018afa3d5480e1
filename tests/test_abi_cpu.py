"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and validates configurations on the host (these calls do
not touch a device)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2101_02745_amd import _lib, inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("fpic.h", "fpic_particles.h")]


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(fpic_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libflavorpic.so not built")
    return _lib.load()


def test_header_declares_the_abi():
    names = declared_functions()
    for must in ("fpic_create", "fpic_set_state", "fpic_step", "fpic_moments",
                 "fpic_flavor_totals", "fpic_batch_step", "fpic_autotune",
                 "fpic_particles_create", "fpic_particles_set", "fpic_particles_step"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name
    # and the binding covers the same set
    assert set(_lib.EXPORTS) == set(declared_functions())


def cfg_of(**kw):
    w = I.workload("1d_32x26")
    hc = _lib.HostConfig.from_workload(w)
    for k, v in kw.items():
        if k == "dt":
            hc.c.dt = v
        elif k == "shape_order":
            hc.c.shape_order = v
        elif k == "hvac":
            hc.c.hvac[:] = v
        elif k == "vmat":
            hc.c.vmat[:] = v
        elif k == "dirs":
            hc.dirs[:] = v
        elif k == "ncell":
            hc.c.ncell[:] = v
    return hc


def ws_bytes(lib, hc, tune=None):
    n = C.c_size_t()
    t = _lib.tuning(tune)
    rc = lib.fpic_workspace_bytes(C.byref(hc.c), C.byref(t) if t else None, C.byref(n))
    return rc, n.value


def test_workspace_size_is_consistent(lib):
    hc = cfg_of()
    rc, n = ws_bytes(lib, hc)
    assert rc == 0
    P = 26 * 32
    assert n >= (18 + 3 * 16) * 8 * P   # state + three slopes of 16 reals
    assert n < 64 * 18 * 8 * P + (1 << 20)
    rc2, n2 = ws_bytes(lib, hc, {"waves": 1, "dirs_per_wave": 1})
    assert rc2 == 0 and n2 > n          # more direction groups, more partials


@pytest.mark.parametrize("kw,code", [
    ({"dt": 5.0}, _lib.FPIC_EUNSUPPORTED),       # crosses a cell per stage
    ({"dt": -0.1}, _lib.FPIC_EINVAL),
    ({"dt": float("nan")}, _lib.FPIC_EINVAL),
    ({"shape_order": 3}, _lib.FPIC_EUNSUPPORTED),
    ({"shape_order": 3, "ncell": [4, 4, 4]}, _lib.FPIC_EUNSUPPORTED),   # 3D path
    ({"hvac": [0.0, 1.0] + [0.0] * 16}, _lib.FPIC_EINVAL),   # not Hermitian
    ({"vmat": [0.0, float("inf"), 0.0]}, _lib.FPIC_EINVAL),
    ({"vmat": [0.0, float("inf"), 0.0], "ncell": [4, 4, 4]}, _lib.FPIC_EINVAL),   # 3D path
    ({"dirs": 2.0}, _lib.FPIC_EINVAL),           # not unit vectors
    ({"ncell": [1, 1, 0]}, _lib.FPIC_EINVAL),
])
def test_bad_configs_rejected(lib, kw, code):
    hc = cfg_of(**kw)
    rc, _ = ws_bytes(lib, hc)
    assert rc == code
    assert len(lib.fpic_last_error()) > 0
    if "vmat" in kw:
        assert b"vmat" in lib.fpic_last_error()


def test_bad_tuning_rejected(lib):
    hc = cfg_of()
    rc, _ = ws_bytes(lib, hc, {"waves": 3})
    assert rc == _lib.FPIC_EINVAL
    rc, _ = ws_bytes(lib, hc, {"steps_per_graph": 1000})
    assert rc == _lib.FPIC_EINVAL
    rc, _ = ws_bytes(lib, hc, {"cache_policy": 3})
    assert rc == _lib.FPIC_EINVAL
    for policy in (0, 1, 2):
        rc, _ = ws_bytes(lib, hc, {"cache_policy": policy})
        assert rc == _lib.FPIC_OK
    # 1D slope forms: 0 k1 and k2 formed again, 1 k1 only, 2 every slope
    # stored; the workspace holds every form's buffers, so its size is one
    sizes = set()
    for fused in (0, 1, 2):
        rc, n = ws_bytes(lib, hc, {"fused": fused})
        assert rc == _lib.FPIC_OK
        sizes.add(n)
    assert len(sizes) == 1
    for fused in (-1, 3):
        rc, _ = ws_bytes(lib, hc, {"fused": fused})
        assert rc == _lib.FPIC_EINVAL
        assert b"fused" in lib.fpic_last_error()


def test_batch_rejects_3d(lib):
    hc = cfg_of(ncell=[2, 2, 2])
    arr = (_lib.Config * 1)(hc.c)
    n = C.c_size_t()
    assert lib.fpic_batch_workspace_bytes(1, arr, None, C.byref(n)) == _lib.FPIC_EINVAL


def test_null_arguments(lib):
    n = C.c_size_t()
    assert lib.fpic_workspace_bytes(None, None, C.byref(n)) == _lib.FPIC_EINVAL
    assert lib.fpic_step(None, 1) == _lib.FPIC_EINVAL
    assert lib.fpic_sync(None) == _lib.FPIC_EINVAL
    lib.fpic_destroy(None)          # no-op


def test_quadratic_shape_accepted_in_1d(lib):
    hc = cfg_of(shape_order=2)
    rc, n = ws_bytes(lib, hc)
    assert rc == 0
    rc1, n1 = ws_bytes(lib, cfg_of())
    assert rc1 == 0 and n > n1          # three edge partials per tile instead of one


def test_batch_needs_one_shape_order(lib):
    a, b = cfg_of(), cfg_of(shape_order=2)
    cfgs = (_lib.Config * 2)(a.c, b.c)
    n = C.c_size_t()
    rc = lib.fpic_batch_workspace_bytes(2, cfgs, None, C.byref(n))
    assert rc == _lib.FPIC_EINVAL
    assert b"shape_order" in lib.fpic_last_error()


def pcfg(**kw):
    w = I.particle_workload("1d_64x16_random")
    c = _lib.pconfig(w.ncell, w.dx, w.nparticles, w.hvac(), w.dt)
    for k, v in kw.items():
        if k == "ncell":
            c.ncell[:] = v
        elif k == "hvac_im":
            c.hvac[1] = v
        else:
            setattr(c, k, v)
    return c


def test_particles_workspace_size(lib):
    n = C.c_size_t()
    assert lib.fpic_particles_workspace_bytes(C.byref(pcfg()), C.byref(n)) == 0
    small = n.value
    assert lib.fpic_particles_workspace_bytes(C.byref(pcfg(npart=4096)), C.byref(n)) == 0
    # two particle sets (18 + 3 + 3 + 2 reals and an index each) and three
    # 16-real slopes per particle
    assert n.value - small >= (4096 - 1024) * (2 * (26 * 8 + 4) + 48 * 8)


@pytest.mark.parametrize("kw,code", [({"npart": 0}, _lib.FPIC_EINVAL),
                                     ({"dt": 0.0}, _lib.FPIC_EINVAL),
                                     ({"dt": float("nan")}, _lib.FPIC_EINVAL),
                                     ({"shape_order": 3}, _lib.FPIC_EUNSUPPORTED),
                                     ({"sort_every": -1}, _lib.FPIC_EINVAL),
                                     ({"sort_every": 2000}, _lib.FPIC_EINVAL),
                                     ({"ncell": [1, 0, 4]}, _lib.FPIC_EINVAL),
                                     ({"hvac_im": 0.5}, _lib.FPIC_EINVAL)])
def test_particles_bad_configs_rejected(lib, kw, code):
    n = C.c_size_t()
    assert lib.fpic_particles_workspace_bytes(C.byref(pcfg(**kw)), C.byref(n)) == code
    assert lib.fpic_last_error()
    assert lib.fpic_particles_create(C.byref(pcfg(**kw)), None, 0, None, C.byref(C.c_void_p())) == code
