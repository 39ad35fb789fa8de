"""Parity of the HIP adjoint (vector-Jacobian product of the orders) with the oracle and with finite differences.

psfd_solve_adjoint takes the forward total field and the cotangent of the
orders of any real loss, and returns the gradient with respect to delta_eps
(dL/dRe + i dL/dIm) from the transposed coupled solve. Losses: J = sum over
the 0 and +-1 orders (x and y) of ||a_q||^2 (through torch autograd), and
L = Re(w . a_(+1,0)) - ||a_(-1,0)||^2, which is not an intensity. Oracle parity:
relative L2 <= 1e-7 (both sides solve to <= 1e-11). Finite differences
(central, FP64 solves at 1e-12) agree to 1e-4 relative, the bar the adjoint
workload sets.
"""
import numpy as np
import pytest

import oracle as O
from paper_2606_25541_amd import clips

from gpu_util import device, rel, say, torch

pytestmark = pytest.mark.gpu

ORDERS = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
W_PLUS1 = np.array([0.7 - 0.2j, -0.4 + 0.9j, 0.3 + 0.1j])


def problem(nx=8, ny=8, nz=4, pol=0, phi=10.0):
    layers, es = clips.mo_si_stack(10)
    return clips.Problem(nx=nx, ny=ny, nz=nz, lx_nm=3.0 * nx, ly_nm=3.0 * ny, t_nm=20.0, theta_deg=6.0,
                         phi_deg=phi, pol=pol, layers=layers, eps_sub=es)


def loss_and_cotangent(a):
    """L = Re(w . a_(+1,0)) - ||a_(-1,0)||^2 and G = dL/dRe a + i dL/dIm a (numpy, [ny][nx][3])."""
    L = float(np.real(W_PLUS1 @ a[0, 1]) - np.sum(np.abs(a[0, -1]) ** 2))
    G = np.zeros_like(a)
    G[0, 1] = np.conj(W_PLUS1)
    G[0, -1] = -2.0 * a[0, -1]
    return L, G


def intensity_cotangent(a, ny, nx):
    G = np.zeros_like(a)
    for (m, n) in ORDERS:
        G[n % ny, m % nx] = 2.0 * a[n % ny, m % nx]
    return G


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("pol", [0, 1])
@pytest.mark.parametrize("loss", ["intensity", "general"])
def test_adjoint_matches_oracle(prec, pol, loss):
    from paper_2606_25541_amd import api
    dev = device()
    p = problem(pol=pol)
    de, _ = clips.smooth_density_eps(8, 8, 4, p.lx_nm, p.ly_nm, p.t_nm, seed=5, sigma_xy_nm=3.0, sigma_z_nm=3.0)
    say("adjoint", prec, pol, loss)
    fwd = O.solve_monolithic(p, de, rtol=1e-13)
    G = intensity_cotangent(fwd["orders"], 8, 8) if loss == "intensity" else loss_and_cotangent(fwd["orders"])[1]
    ref = O.order_vjp(p, de, G, u=fwd["u"], rtol=1e-13)
    plan = api.Plan(p, rtol=1e-11, precision=prec, restart=20)
    d = torch.from_numpy(de).to(dev)
    u = torch.empty((3, 4, 8, 8), dtype=torch.complex128, device=dev)
    _, orders, fi = plan.psfd_solve(d, u=u)
    assert rel(u.cpu().numpy(), fwd["u"]) < 1e-9
    # the cotangent of the GPU's own orders (what autograd hands the backward)
    a = orders.cpu().numpy()
    Gg = intensity_cotangent(a, 8, 8) if loss == "intensity" else loss_and_cotangent(a)[1]
    grad, ai = plan.psfd_solve_adjoint(d, u, torch.from_numpy(Gg).to(dev))
    say("  fwd", fi, "adj", ai)
    assert ai["status"] == 0
    assert rel(grad.cpu().numpy(), ref["grad"]) < 1e-7


def test_adjoint_finite_differences_and_autograd():
    """Orders through torch autograd: the intensity J via order_intensity and a
    general loss of the orders, each against central differences of FP64 solves."""
    from paper_2606_25541_amd import api
    dev = device()
    nx, ny, nz = 32, 32, 16
    p = problem(nx, ny, nz, phi=0.0)
    de, _ = clips.smooth_density_eps(nx, ny, nz, p.lx_nm, p.ly_nm, p.t_nm, seed=7, sigma_xy_nm=6.0, sigma_z_nm=4.0)
    plan = api.Plan(p, rtol=1e-12, precision="fp64", restart=30)
    d = torch.from_numpy(de).to(dev).requires_grad_(True)
    J = api.order_intensity(d, plan, ORDERS)
    J.backward()
    gJ = d.grad.detach().cpu().numpy()
    d.grad = None
    a = api.Orders.apply(d, plan)
    w = torch.from_numpy(W_PLUS1).to(dev)
    Lg = (w * a[0, 1]).sum().real - (a[0, -1].abs() ** 2).sum()
    Lg.backward()
    gL = d.grad.detach().cpu().numpy()
    em = torch.empty((3, nz, ny, nx), dtype=torch.complex128, device=dev)
    od = torch.empty((ny, nx, 3), dtype=torch.complex128, device=dev)

    def losses(x):
        plan.psfd_solve(torch.from_numpy(x).to(dev), em, od)
        a = od.cpu().numpy()
        Jv = sum(float(np.sum(np.abs(a[n % ny, m % nx]) ** 2)) for (m, n) in ORDERS)
        return Jv, loss_and_cotangent(a)[0]

    rng = np.random.default_rng(21)
    for _ in range(4):
        k, j, i = int(rng.integers(0, nz)), int(rng.integers(0, ny)), int(rng.integers(0, nx))
        for part in (1.0, 1j):
            h = 1e-5
            dp = de.copy(); dp[k, j, i] += h * part
            dm = de.copy(); dm[k, j, i] -= h * part
            (jp, lp), (jm, lm) = losses(dp), losses(dm)
            for fd, g in (((jp - jm) / (2 * h), gJ), ((lp - lm) / (2 * h), gL)):
                an = g[k, j, i].real if part == 1.0 else g[k, j, i].imag
                say("  fd", fd, "adjoint", an)
                assert abs(fd - an) <= 1e-4 * abs(fd) + 1e-10


@pytest.mark.parametrize("n", [64, 128])
def test_adjoint_fused_krylov_kernels_match_separate_passes(n, monkeypatch):
    """n x n x 32 (n = 64, 128), mixed: the forward and the transposed solve of
    the adjoint run the Gram-Schmidt projections and update inside the transform
    kernels (the pencil carrying the Givens step of the transposed operator
    too); the gradient and J agree with the separate passes
    (PSFD_FUSE_DOTS=0, PSFD_FUSE_UPDATE=0) to the solve tolerance."""
    from paper_2606_25541_amd import api
    dev = device()
    nz = 32
    p = problem(n, n, nz, phi=20.0)
    de, _ = clips.smooth_density_eps(n, n, nz, p.lx_nm, p.ly_nm, p.t_nm, seed=11, sigma_xy_nm=4.0, sigma_z_nm=3.0)
    d = torch.from_numpy(de).to(dev)
    plan = api.Plan(p, rtol=1e-10, precision="mixed", restart=8)
    say("adjoint %dx%dx%d fused vs separate" % (n, n, nz))

    def run():
        u = torch.empty((3, nz, n, n), dtype=torch.complex128, device=dev)
        _, orders, fi = plan.psfd_solve(d, u=u)
        G = torch.from_numpy(intensity_cotangent(orders.cpu().numpy(), n, n)).to(dev)
        g, ai = plan.psfd_solve_adjoint(d, u, G)
        return g, fi, ai

    g1, f1, a1 = run()
    monkeypatch.setenv("PSFD_FUSE_DOTS", "0")
    monkeypatch.setenv("PSFD_FUSE_UPDATE", "0")
    g2, f2, a2 = run()
    say("  fused", f1, a1, "separate", f2, a2)
    assert f1["status"] == 0 and a1["status"] == 0
    assert abs(f1["iters"] - f2["iters"]) <= 8 and abs(a1["iters"] - a2["iters"]) <= 8
    assert rel(g1.cpu().numpy(), g2.cpu().numpy()) < 1e-7
