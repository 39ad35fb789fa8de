"""Parity of the HIP differential PSFD operator and solver with the oracle (Sec. 3, eqs. (6)-(8)).

* The apply y = A x (and D A x with the spectral damping) against the oracle's,
  element by element, on grids whose transverse passes take the fused square
  plane, the split row / column and the tile kernels, FP64 (<= 1e-11 of the
  largest output) and FP32 (<= 2e-5).
* The background-field solve (outer reflection loop around GMRES) and the
  full-domain solve (multilayer on the grid) against the oracle's, with and
  without preconditioning: field <= 1e-8 relative, orders <= 1e-9 of the largest.
* The preconditioner study's ordering on a small clip: the Green's-function
  (Lippmann-Schwinger) solve takes fewer GMRES steps than the damped
  differential solve, which takes fewer than the unpreconditioned one.
"""
import numpy as np
import pytest

import oracle as O
from oracle import differential as Df
from paper_2606_25541_amd import clips

from gpu_util import device, rel, say, torch

pytestmark = pytest.mark.gpu


def problem(nx, ny, nz, t, L, theta=6.0, phi=20.0, pol=0, pairs=10, es=None):
    layers, esub = clips.mo_si_stack(pairs)
    return clips.Problem(nx=nx, ny=ny, nz=nz, lx_nm=L, ly_nm=L * ny / nx, t_nm=t, theta_deg=theta, phi_deg=phi,
                         pol=pol, layers=layers, eps_sub=esub if es is None else es)


APPLY_CASES = [
    # nx, ny, nz (absorber), pe, pml
    (8, 8, 4, 32, 6),
    (16, 8, 8, 64, 12),
    (32, 32, 8, 64, 16),
    (64, 64, 16, 128, 24),
    (256, 16, 4, 16, 2),
]


@pytest.mark.parametrize("case", APPLY_CASES, ids=["%dx%dx%d" % (c[0], c[1], c[3]) for c in APPLY_CASES])
@pytest.mark.parametrize("precond", ["none", "damping"])
def test_diff_apply_matches_oracle(case, precond):
    from paper_2606_25541_amd import api
    dev = device()
    nx, ny, nz, pe, npml = case
    p = problem(nx, ny, nz, 2.0 * nz, 2.0 * nx, pol=1)
    zc0 = (pe - nz) // 2
    D = Df.DiffSetup(p, pe, zc0, nz, npml)
    plan = api.DiffPlan(p, pe, zc0, nz, npml)
    de = clips.manhattan(nx, ny, nz, p.lx_nm, p.ly_nm, seed=nx + pe)
    x = clips.random_complex((3, pe, ny, nx), seed=pe)
    ref = Df.apply_diff(D, de, x, precond)
    say("diff apply", case, precond)
    for dt, bar in ((torch.complex128, 1e-11), (torch.complex64, 2e-5)):
        y = plan.apply(torch.from_numpy(de).to(dev).to(dt), torch.from_numpy(x).to(dev).to(dt), precond=precond)
        err = np.abs(y.cpu().numpy() - ref).max() / np.abs(ref).max()
        say("  ", dt, "err %.2e" % err)
        assert err <= bar


@pytest.mark.parametrize("precond", ["none", "damping"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_diff_background_solve_matches_oracle(precond, prec):
    """4 x 4 x 16 planes (768 unknowns): the oracle solves every outer step
    directly (dense LU), the GPU by GMRES(64) to 1e-11."""
    from paper_2606_25541_amd import api
    dev = device()
    nx, ny, nz, pe, npml = 4, 4, 4, 16, 3
    p = problem(nx, ny, nz, 8.0, 8.0, pol=0, pairs=20)
    zc0 = (pe - nz) // 2
    D = Df.DiffSetup(p, pe, zc0, nz, npml)
    de = clips.manhattan(nx, ny, nz, p.lx_nm, p.ly_nm, seed=5)
    ref = Df.solve_background(D, de, precond, rtol=1e-13, dense=True)
    plan = api.DiffPlan(p, pe, zc0, nz, npml)
    e, orders, info = plan.solve(torch.from_numpy(de).to(dev), precond, rtol=1e-11, restart=64, max_iters=200000,
                                 max_outer=200, precision=prec)
    say("diff background", precond, prec, info, "oracle outer", ref["outer_iters"])
    assert info["status"] == 0
    assert rel(e.cpu().numpy(), ref["E"]) < 1e-8
    o = orders.cpu().numpy()
    assert np.abs(o - ref["orders"]).max() < 1e-9 * np.abs(ref["orders"]).max()


@pytest.mark.parametrize("precond", ["none", "damping"])
def test_diff_full_domain_solve_matches_oracle(precond):
    """4 Mo/Si pairs on the grid below a 4-plane absorber, spacing 0.69 nm (Si 6,
    Mo 4 planes), 4 x 4 x 64 planes; the oracle's dense solve against GMRES(64)."""
    from paper_2606_25541_amd import api
    dev = device()
    layers, _ = clips.mo_si_stack(4)
    nx, ny, nz, pe, npml = 4, 4, 4, 64, 6
    nl = 40
    p = clips.Problem(nx=nx, ny=ny, nz=nz, lx_nm=8.0, ly_nm=8.0, t_nm=4 * 0.69, theta_deg=6.0, phi_deg=0.0,
                      pol=0, layers=[], eps_sub=1.0)
    zc0 = npml + 6
    D = Df.DiffSetup(p, pe, zc0, nz + nl, npml)
    dabs = clips.manhattan(nx, ny, nz, 8.0, 8.0, seed=9)
    dc = clips.layered_contrast(nz + nl, nz, 0.69, layers, dabs)
    ref = Df.solve_full_domain(D, dc, precond, dense=True)
    plan = api.DiffPlan(p, pe, zc0, nz + nl, npml, form="full")
    e, orders, info = plan.solve(torch.from_numpy(dc).to(dev), precond, rtol=1e-11, restart=64, max_iters=200000)
    say("diff full domain", precond, info)
    assert info["status"] == 0
    assert rel(e.cpu().numpy(), ref["E"]) < 1e-8
    assert np.abs(orders.cpu().numpy() - ref["orders"]).max() < 1e-9 * np.abs(ref["orders"]).max()


def test_green_function_solve_takes_fewer_steps_on_a_small_clip():
    """16 x 16 x 8 Manhattan clip, rtol 1e-6: the Lippmann-Schwinger solve
    (outer coupling, the same background decomposition) takes fewer GMRES steps
    than the differential solve with either preconditioner; the three counts
    are printed for the record."""
    from paper_2606_25541_amd import api
    dev = device()
    nx, ny, nz, pe, npml = 16, 16, 8, 64, 16
    p = problem(nx, ny, nz, 16.0, 32.0, pol=0, pairs=40)
    de = clips.manhattan(nx, ny, nz, p.lx_nm, p.ly_nm, seed=31)
    d = torch.from_numpy(de).to(dev)
    plan = api.DiffPlan(p, pe, (pe - nz) // 2, nz, npml)
    its = {}
    for pc in ("none", "damping"):
        _, _, info = plan.solve(d, pc, rtol=1e-6, restart=30, max_iters=100000, max_outer=200, precision="mixed")
        assert info["status"] == 0, info
        its[pc] = info["iters"]
    ls = api.Plan(p, rtol=1e-6, precision="mixed", restart=30, coupling="outer", max_outer=200)
    _, _, li = ls.solve(d)
    its["ls"] = li["iters"]
    say("iterations", its)
    assert its["ls"] < min(its["none"], its["damping"])
