"""The allocation-free apply (psfd_apply_noalloc) against psfd_apply, through the C ABI.

Both run the same kernels on the same inputs; the allocation-free entry point
takes its workspace from the library's static per-device array. Checked on two
calls in a row, the second on a smaller grid (so the array holds the first
call's larger workspace when the second starts), in FP32 and FP64, with the
plain, transposed and coupled operators; and a grid whose workspace exceeds
the array is refused with UNSUPPORTED_SIZE before any launch.
"""
import ctypes as C

import numpy as np
import pytest

from paper_2606_25541_amd import clips

from gpu_util import device, rel, say, torch

pytestmark = pytest.mark.gpu


def _plan(n, nz, lx):
    from paper_2606_25541_amd import api
    layers, es = clips.mo_si_stack(40)
    p = clips.Problem(nx=n, ny=n, nz=nz, lx_nm=lx, ly_nm=lx, t_nm=60.0, theta_deg=6.0, phi_deg=15.0, pol=1,
                      layers=layers, eps_sub=es)
    return p, api.Plan(p, rtol=1e-6)


def _call(name, plan, d, x, y, code, flags):
    from paper_2606_25541_amd import _lib as L
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(L.lib(), name)(plan._h, C.c_void_p(d.data_ptr()), C.c_void_p(x.data_ptr()),
                                C.c_void_p(y.data_ptr()), code, flags, s)
    return rc


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_apply_equals_apply_two_calls(dtype):
    from paper_2606_25541_amd import _lib as L
    dev = device()
    tdt, code, bar = {"c64": (torch.complex64, L.PSFD_C64, 1e-6),
                      "c128": (torch.complex128, L.PSFD_C128, 1e-13)}[dtype]
    for (n, nz, lx) in ((128, 64, 256.0), (64, 32, 128.0)):  # second call smaller
        p, plan = _plan(n, nz, lx)
        d = torch.from_numpy(clips.contact_holes(n, n, nz, lx, lx, 6, seed=n)).to(dev).to(tdt)
        x = torch.from_numpy(clips.random_complex((3, nz, n, n), seed=n + 1)).to(dev).to(tdt)
        for flags in (0, L.PSFD_APPLY_TRANSPOSE, L.PSFD_APPLY_REFLECT | L.PSFD_APPLY_K_ONLY):
            y0 = torch.empty_like(x)
            y1 = torch.full_like(x, float("nan"))
            say("noalloc", dtype, (n, nz), "flags", flags)
            assert _call("psfd_apply", plan, d, x, y0, code, flags) == 0
            assert _call("psfd_apply_noalloc", plan, d, x, y1, code, flags) == 0
            torch.cuda.synchronize()
            e = rel(y1.cpu().numpy(), y0.cpu().numpy())
            say("  rel diff %.2e bitwise %s" % (e, torch.equal(y0, y1)))
            assert np.isfinite(e) and e <= bar


def test_noalloc_apply_refuses_oversized_workspace():
    from paper_2606_25541_amd import _lib as L
    dev = device()
    # 256 x 256 x 64 complex128: 3 N values of 16 bytes = 192 MiB > 128 MiB
    p, plan = _plan(256, 64, 512.0)
    d = torch.zeros((64, 256, 256), dtype=torch.complex128, device=dev)
    x = torch.zeros((3, 64, 256, 256), dtype=torch.complex128, device=dev)
    y = torch.empty_like(x)
    rc = _call("psfd_apply_noalloc", plan, d, x, y, L.PSFD_C128, 0)
    assert rc == L.PSFD_ERR_UNSUPPORTED_SIZE
    assert "static scratch" in L.lib().psfd_last_error().decode()
