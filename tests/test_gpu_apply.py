"""Parity of the HIP operator apply (eq. (18) left side) with the oracle.

Element-wise comparison on seeded inputs; shapes cover the fused-plane and the
split row/column transverse paths of both precisions, odd tails of the
z-pencil blocking (nx < 16) and the transposed and K-only variants.
Tolerances: FP64 1e-12 relative (rounding of O(log N) FFT passes), FP32 2e-6
relative (single-precision FFTs of length <= 256 in each axis).
"""
import numpy as np
import pytest

import oracle as O
from paper_2606_25541_amd import clips

from gpu_util import device, rel, say, torch

pytestmark = pytest.mark.gpu

# (128, 128, 4): square-plane kernel in FP32, row/column strips in FP64;
# (256, 256, 2): strips in both precisions; (16, 16, 32) and (16, 8, 64): the
# z-pencil with compile-time padded lengths 64 and 128; (128, 128, 32) and
# (128, 128, 64): the quarter-plane kernels with the quarter-layout pencil at
# both compile-time lengths, in both precisions; (256, 256, 32): quarter planes
# in FP32, strips in FP64
SHAPES = [
    (4, 4, 2), (8, 8, 4), (16, 8, 8), (32, 32, 16), (64, 32, 8), (128, 128, 4), (256, 64, 2), (64, 256, 2),
    (256, 256, 2), (16, 16, 32), (16, 8, 64), (128, 128, 32), (128, 128, 64), (256, 256, 32),
]


def make(nx, ny, nz, theta=6.0, phi=25.0, pol=0):
    layers, es = clips.mo_si_stack(10)
    return clips.Problem(nx=nx, ny=ny, nz=nz, lx_nm=2.0 * nx, ly_nm=2.0 * ny, t_nm=60.0 * nz / 32 + 1.0,
                         theta_deg=theta, phi_deg=phi, pol=pol, layers=layers, eps_sub=es)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_apply_matches_oracle(shape, dtype):
    from paper_2606_25541_amd import api
    dev = device()
    nx, ny, nz = shape
    say("apply", shape, dtype)
    p = make(nx, ny, nz)
    de = clips.manhattan(nx, ny, nz, p.lx_nm, p.ly_nm, seed=nx + ny + nz)
    x = clips.random_complex((3, nz, ny, nx), seed=17)
    S = O.Setup(p)
    ref = O.apply_A(S, de, x)
    refk = O.conv_K(S, O.potential(S, de)[None] * x)
    reft = O.apply_A(S, de, x, transpose=True)
    td = torch.complex128 if dtype == "c128" else torch.complex64
    tol = 1e-12 if dtype == "c128" else 2e-6
    plan = api.Plan(p)
    dd = torch.from_numpy(de).to(dev, td)
    xx = torch.from_numpy(x).to(dev, td)
    y = plan.psfd_apply(dd, xx).cpu().numpy()
    yk = plan.psfd_apply(dd, xx, k_only=True).cpu().numpy()
    yt = plan.psfd_apply(dd, xx, transpose=True).cpu().numpy()
    assert rel(y, ref) < tol, rel(y, ref)
    assert rel(yk, refk) < tol * 3, rel(yk, refk)
    assert rel(yt, reft) < tol, rel(yt, reft)
    if dtype == "c128":
        assert np.max(np.abs(y - ref)) < 1e-11 * np.max(np.abs(ref))


@pytest.mark.parametrize("shape", [(8, 8, 4), (16, 8, 8), (32, 32, 16), (128, 128, 4), (64, 256, 2), (128, 128, 32),
                                   (128, 128, 64), (256, 256, 32)])
@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_coupled_apply_matches_oracle(shape, dtype):
    """y = u - M V u with M = K + R_vol T_R K_top (and its bilinear transpose)."""
    from paper_2606_25541_amd import api
    dev = device()
    nx, ny, nz = shape
    say("coupled apply", shape, dtype)
    p = make(nx, ny, nz, phi=10.0, pol=1)
    de = clips.manhattan(nx, ny, nz, p.lx_nm, p.ly_nm, seed=3 * nx + nz)
    u = clips.random_complex((3, nz, ny, nx), seed=23)
    S = O.Setup(p)
    Vu = O.potential(S, de)[None] * u
    ref = u - O.apply_M(S, Vu)
    reft = u - O.apply_M_T(S, Vu)
    td = torch.complex128 if dtype == "c128" else torch.complex64
    tol = 1e-12 if dtype == "c128" else 3e-6
    plan = api.Plan(p)
    dd = torch.from_numpy(de).to(dev, td)
    uu = torch.from_numpy(u).to(dev, td)
    y = plan.psfd_apply(dd, uu, reflect=True).cpu().numpy()
    yt = plan.psfd_apply(dd, uu, reflect=True, transpose=True).cpu().numpy()
    assert rel(y, ref) < tol, rel(y, ref)
    assert rel(yt, reft) < tol, rel(yt, reft)


@pytest.mark.parametrize("n,nz,dtype", [(128, 32, "c64"), (128, 64, "c64"), (128, 32, "c128"), (128, 64, "c128"),
                                        (256, 64, "c64")])
def test_quarter_planes_match_full_planes(n, nz, dtype, monkeypatch):
    """n x n planes: the quarter-plane kernels (four blocks per plane, the
    radix-4 y combine in the pencil) against the one-block-per-plane kernels
    (FP32, 128 x 128) or the row and column strips (FP64; FP32 at 256 x 256), in
    every apply variant (plain, K only, transposed, coupled)."""
    from paper_2606_25541_amd import api
    dev = device()
    say("quarter vs full planes", n, nz, dtype)
    p = make(n, n, nz, phi=10.0)
    de = clips.manhattan(n, n, nz, p.lx_nm, p.ly_nm, seed=nz + 5)
    x = clips.random_complex((3, nz, n, n), seed=29)
    plan = api.Plan(p)
    td = torch.complex64 if dtype == "c64" else torch.complex128
    dd = torch.from_numpy(de).to(dev, td)
    xx = torch.from_numpy(x).to(dev, td)
    variants = [{}, {"k_only": True}, {"transpose": True}, {"reflect": True}, {"reflect": True, "transpose": True}]
    ys = {}
    for q in ("1", "0"):
        monkeypatch.setenv("PSFD_QUARTER_PLANES", q)
        ys[q] = [plan.psfd_apply(dd, xx, **v).cpu().numpy() for v in variants]
    tol = 1e-6 if dtype == "c64" else 1e-13
    for v, a, b in zip(variants, ys["1"], ys["0"]):
        assert rel(a, b) < tol, (v, rel(a, b))


def test_apply_is_deterministic():
    from paper_2606_25541_amd import api
    dev = device()
    p = make(64, 64, 16)
    de = clips.manhattan(64, 64, 16, p.lx_nm, p.ly_nm, seed=3)
    x = clips.random_complex((3, 16, 64, 64), seed=4)
    plan = api.Plan(p)
    dd = torch.from_numpy(de).to(dev, torch.complex64)
    xx = torch.from_numpy(x).to(dev, torch.complex64)
    a = plan.psfd_apply(dd, xx).cpu()
    b = plan.psfd_apply(dd, xx).cpu()
    assert torch.equal(a, b)


def test_apply_full_size_sampled():
    """128 x 128 x 64 (the large-solve grid): sampled outputs vs a per-point oracle sum.

    K is diagonal per transverse order, so one order's z-profile of K(Vx) is
    computed from the oracle's kernel table column by direct DFT sums.
    """
    from paper_2606_25541_amd import api
    dev = device()
    p = clips.config_problem("G3")
    de = clips.contact_holes(128, 128, 64, 256.0, 256.0, 8, seed=2001)
    x = clips.random_complex((3, 64, 128, 128), seed=5)
    plan = api.Plan(p)
    say("apply full size G3 fp64")
    y = plan.psfd_apply(torch.from_numpy(de).to(dev), torch.from_numpy(x).to(dev), k_only=True)
    torch.cuda.synchronize()
    yh = np.fft.fft2(y.cpu().numpy(), axes=(-2, -1))
    S = O.Setup(p)
    f = np.fft.fft2(O.potential(S, de)[None] * x, axes=(-2, -1))      # (3, nz, ny, nx) spectra
    rng = np.random.default_rng(9)
    kap = S.kappa
    for _ in range(6):
        j, i = int(rng.integers(0, 128)), int(rng.integers(0, 128))
        G = O.gtilde_periodic(S.KX[j, i], S.KY[j, i], kap, S.beta[j, i], S.kbg, S.L, S.sgn)  # (pz, 3, 3)
        G[S.l == -S.pz // 2, 0:2, 2] = 0
        G[S.l == -S.pz // 2, 2, 0:2] = 0
        G *= S.keep[j, i]
        fp = np.zeros((3, S.pz), complex)
        fp[:, :64] = f[:, :, j, i]
        F = np.fft.fft(fp, axis=1)
        out = np.einsum("lab,bl->al", G, F)
        prof = np.fft.ifft(out, axis=1)[:, :64]
        assert rel(yh[:, :, j, i], prof) < 1e-11
