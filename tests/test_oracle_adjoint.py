"""Pins of the oracle's adjoint (gradient of order intensities w.r.t. delta_eps).

* Every transposed map satisfies <A x, y> = <x, A^T y> (bilinear) on random
  vectors, i.e. it is the transpose of the forward map, checked by brute force.
* The gradient agrees with central finite differences of full forward solves.
"""
import numpy as np
import pytest

import oracle as O
from paper_2606_25541_amd import clips as C


def setup():
    layers, es = C.mo_si_stack(10)
    p = C.Problem(nx=8, ny=4, nz=4, lx_nm=24.0, ly_nm=12.0, t_nm=20.0, theta_deg=6.0, phi_deg=15.0,
                  pol=1, layers=layers, eps_sub=es)
    return p, O.Setup(p)


def bil(a, b):
    return np.sum(a * b)


def test_transposes_are_bilinear_transposes():
    p, S = setup()
    x = C.random_complex((3, 4, 4, 8), 1)
    y = C.random_complex((3, 4, 4, 8), 2)
    a = C.random_complex((4, 8, 3), 3)
    for fwd, adj, u, v in [
        (lambda f: O.conv_K(S, f), lambda f: O.conv_K(S, f, transpose=True), x, y),
        (lambda f: O.apply_M(S, f), lambda f: O.apply_M_T(S, f), x, y),
        (lambda f: O.read_down(S, f), lambda c: O.read_down_T(S, c), x, a),
        (lambda f: O.read_up(S, f), lambda c: O.read_up_T(S, c), x, a),
        (lambda c: O.inject_up(S, c), lambda f: O.inject_up_T(S, f), a, x),
        (lambda c: O.reflect(S, c), lambda c: O.reflect_T(S, c), a, a[::-1].copy()),
    ]:
        lhs = bil(fwd(u), v)
        rhs = bil(u, adj(v))
        assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1e-30)


def test_transpose_of_K_is_flipped_table():
    """K^T equals K built from G~ at the negated wavevector (base -k0)."""
    p, S = setup()
    x = C.random_complex((3, 4, 4, 8), 5)
    kt = O.conv_K(S, x, transpose=True)
    p2 = C.Problem(**{**p.__dict__, "phi_deg": p.phi_deg + 180.0})
    S2 = O.Setup(p2)
    # the table at the negated index of base k0 is the table of base -k0
    k2 = O.conv_K(S2, x)
    assert np.max(np.abs(kt - k2)) < 1e-12 * np.max(np.abs(kt))


def test_gradient_matches_finite_differences():
    layers, es = C.mo_si_stack(10)
    p = C.Problem(nx=8, ny=8, nz=4, lx_nm=24.0, ly_nm=24.0, t_nm=20.0, theta_deg=6.0, phi_deg=10.0,
                  pol=0, layers=layers, eps_sub=es)
    de, _ = C.smooth_density_eps(8, 8, 4, 24.0, 24.0, 20.0, seed=5, sigma_xy_nm=3.0, sigma_z_nm=3.0)
    orders = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    adj = O.adjoint_gradient(p, de, orders, rtol=1e-13)
    rng = np.random.default_rng(11)
    S = O.Setup(p)
    for _ in range(4):
        k, j, i = int(rng.integers(0, 4)), int(rng.integers(0, 8)), int(rng.integers(0, 8))
        for part in (1.0, 1j):
            h = 1e-5
            dp = de.copy()
            dp[k, j, i] += h * part
            dm = de.copy()
            dm[k, j, i] -= h * part
            jp = O.objective(S, O.solve(p, dp, rtol=1e-13, S=S)["orders"], orders)
            jm = O.objective(S, O.solve(p, dm, rtol=1e-13, S=S)["orders"], orders)
            fd = (jp - jm) / (2 * h)
            g = adj["grad"][k, j, i]
            an = g.real if part == 1.0 else g.imag
            assert abs(fd - an) <= 1e-6 * abs(fd) + 1e-12


def _vjp_problem():
    layers, es = C.mo_si_stack(10)
    p = C.Problem(nx=8, ny=8, nz=4, lx_nm=24.0, ly_nm=24.0, t_nm=20.0, theta_deg=6.0, phi_deg=10.0,
                  pol=1, layers=layers, eps_sub=es)
    de, _ = C.smooth_density_eps(8, 8, 4, 24.0, 24.0, 20.0, seed=6, sigma_xy_nm=3.0, sigma_z_nm=3.0)
    return p, de


W_PLUS1 = np.array([0.7 - 0.2j, -0.4 + 0.9j, 0.3 + 0.1j])


def non_intensity_loss(a):
    """L(a) = Re(w . a_(+1,0)) - ||a_(-1,0)||^2 and its gradient dL/dRe a + i dL/dIm a."""
    L = float(np.real(W_PLUS1 @ a[0, 1]) - np.sum(np.abs(a[0, -1]) ** 2))
    G = np.zeros_like(a)
    G[0, 1] = np.conj(W_PLUS1)
    G[0, -1] = -2.0 * a[0, -1]
    return L, G


def test_order_vjp_matches_finite_differences_for_a_general_loss():
    """The vector-Jacobian product of the orders (any cotangent) against central
    differences of full FP64 monolithic solves, for a loss that is not an intensity."""
    p, de = _vjp_problem()
    fwd = O.solve_monolithic(p, de, rtol=1e-13)
    _, G = non_intensity_loss(fwd["orders"])
    v = O.order_vjp(p, de, G, u=fwd["u"], rtol=1e-13)
    rng = np.random.default_rng(21)
    for _ in range(4):
        k, j, i = int(rng.integers(0, 4)), int(rng.integers(0, 8)), int(rng.integers(0, 8))
        for part in (1.0, 1j):
            h = 1e-5
            lp = non_intensity_loss(O.solve_monolithic(p, de + _bump(de, k, j, i, h * part), rtol=1e-13)["orders"])[0]
            lm = non_intensity_loss(O.solve_monolithic(p, de - _bump(de, k, j, i, h * part), rtol=1e-13)["orders"])[0]
            fd = (lp - lm) / (2 * h)
            g = v["grad"][k, j, i]
            an = g.real if part == 1.0 else g.imag
            assert abs(fd - an) <= 1e-6 * abs(fd) + 1e-12, (k, j, i, part, fd, an)


def _bump(de, k, j, i, h):
    d = np.zeros_like(de)
    d[k, j, i] = h
    return d


def test_order_vjp_of_the_intensity_is_the_intensity_gradient():
    """With the cotangent 2 a on the selected orders (the gradient of sum ||a_q||^2),
    the monolithic vector-Jacobian product equals the outer-splitting adjoint."""
    p, de = _vjp_problem()
    orders = [(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1)]
    adj = O.adjoint_gradient(p, de, orders, rtol=1e-13)
    S = adj["fwd"]["setup"]
    G = np.where(O.order_mask(S, orders)[..., None], 2.0 * adj["fwd"]["orders"], 0.0)
    v = O.order_vjp(p, de, G, rtol=1e-13)
    assert np.max(np.abs(v["grad"] - adj["grad"])) <= 1e-8 * np.max(np.abs(adj["grad"]))
