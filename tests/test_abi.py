"""The C-ABI library loads and exports every entry point include/psfd.h declares.

Host-side checks only (no device calls): option and problem validation errors
that the library reports before touching the GPU are exercised through plan
creation, which builds the FP64 tables on the host.
"""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psfd.h")
LIB = os.path.join(ROOT, "paper_2606_25541_amd", "libpsfd.so")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"\b(psfd_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2606_25541_amd import build
        build.build()
    from paper_2606_25541_amd import _lib
    return _lib.load(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared()
    assert len(names) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], stdout=subprocess.PIPE, text=True).stdout
    exported = set(re.findall(r"\sT\s(psfd_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


def test_binding_covers_header():
    from paper_2606_25541_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()


def test_status_strings_and_version(lib):
    assert lib.psfd_version().decode().startswith("psfd")
    assert lib.psfd_status_string(0).decode() == "ok"
    assert "singular" in lib.psfd_status_string(-4).decode()


def _problem(nx=8, ny=8, nz=4, theta=6.0):
    from paper_2606_25541_amd import _lib as L
    layers = (L.psfd_layer * 1)(L.psfd_layer(0.9, 0.01, 3.0))
    return L.psfd_problem(nx, ny, nz, 16.0, 16.0, 8.0, 13.5, 1.0, theta, 0.0, 0, 1,
                          C.cast(layers, C.POINTER(L.psfd_layer)), 0.9, 0.02), layers


def test_plan_validation_errors(lib):
    from paper_2606_25541_amd import _lib as L
    h = C.c_void_p()
    p, keep = _problem(nx=12)
    assert lib.psfd_plan_create(C.byref(p), None, C.byref(h)) == L.PSFD_ERR_UNSUPPORTED_SIZE
    assert "powers of two" in lib.psfd_last_error().decode()
    p, keep = _problem(nz=256)
    assert lib.psfd_plan_create(C.byref(p), None, C.byref(h)) == L.PSFD_ERR_UNSUPPORTED_SIZE
    p, keep = _problem()
    o = L.psfd_opts(1e-6, 0.0, 64, 100, 10, 1, 0.0)
    assert lib.psfd_plan_create(C.byref(p), C.byref(o), C.byref(h)) == L.PSFD_ERR_INVALID_ARG
    assert lib.psfd_plan_create(None, None, C.byref(h)) == L.PSFD_ERR_INVALID_ARG


def test_wood_anomaly_is_singular(lib):
    """An order with kt = k_bg exactly: incidence sin(theta) = lambda / lx - 1 ... picked so kx(-1) = -k_bg."""
    import math
    from paper_2606_25541_amd import _lib as L
    lam, lx = 13.5, 16.0
    # kx0 - 2 pi / lx = -k0  ->  sin(theta) = 1 - lam / lx
    theta = math.degrees(math.asin(1.0 - lam / lx))
    p, keep = _problem(theta=theta)
    h = C.c_void_p()
    assert lib.psfd_plan_create(C.byref(p), None, C.byref(h)) == L.PSFD_ERR_SINGULAR


def test_plan_create_and_footprint_on_host(lib):
    from paper_2606_25541_amd import _lib as L
    p, keep = _problem()
    h = C.c_void_p()
    rc = lib.psfd_plan_create(C.byref(p), None, C.byref(h))
    if rc == L.PSFD_ERR_HIP:
        pytest.skip("no HIP runtime device")
    assert rc == 0
    v = C.c_size_t()
    assert lib.psfd_plan_footprint(h, C.byref(v)) == 0
    assert v.value > 31 * 3 * 8 * 8 * 4 * 8
    lib.psfd_plan_destroy(h)


def test_release_cached_workspaces_without_cache(lib):
    # only the host-side cache is touched: returns OK with nothing kept
    assert lib.psfd_release_cached_workspaces() == 0


def test_isolated_plan_validation_errors(lib):
    """psfd_iso_plan_create rejects bad grids, sizes, media and radii before any
    device call."""
    from paper_2606_25541_amd import _lib as L
    h = C.c_void_p()

    def P(nx=8, ny=8, nz=4, d=(2.0, 2.0, 1.0), lam=13.5, e=(1.0, 0.0), R=0.0):
        return L.psfd_iso_problem(nx, ny, nz, d[0], d[1], d[2], lam, e[0], e[1], R)

    cases = [
        (P(nx=12), L.PSFD_ERR_UNSUPPORTED_SIZE),
        (P(nz=256), L.PSFD_ERR_UNSUPPORTED_SIZE),
        (P(ny=1), L.PSFD_ERR_UNSUPPORTED_SIZE),
        (P(d=(2.0, 0.0, 1.0)), L.PSFD_ERR_INVALID_ARG),
        (P(lam=-1.0), L.PSFD_ERR_INVALID_ARG),
        (P(e=(1.0, -0.1)), L.PSFD_ERR_INVALID_ARG),
        # a radius far beyond the box needs an oversampled grid longer than 1024
        (P(nx=128, R=1e6), L.PSFD_ERR_UNSUPPORTED_SIZE),
    ]
    for p, code in cases:
        assert lib.psfd_iso_plan_create(C.byref(p), C.byref(h)) == code, (p.nx, p.ny, p.nz)
        assert lib.psfd_last_error().decode()
    assert lib.psfd_iso_plan_create(None, C.byref(h)) == L.PSFD_ERR_INVALID_ARG
    assert lib.psfd_iso_apply(None, None, None, None, 0, None) == L.PSFD_ERR_INVALID_ARG
