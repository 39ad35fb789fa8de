"""Pins of the oracle's discrete solver (eqs. (8), (9), (11)-(12), (18)).

* GMRES and the outer reflection loop agree with a dense direct solve of the
  monolithic system (I - (K + R_vol T_R K_top) V) u = e_bg on tiny grids.
* With no absorber the reflected order is exactly T_R E_inc (bare mirror).
* A laterally uniform absorber film converges, as dz -> 0, to the exact
  reflection of the composite stack [film + multilayer] from the independent
  layered-media recursion, at second order in dz, for TE and TM.
* Reciprocity under swapped incidence holds to solver precision.
* Born limit: (u - e_bg) / t -> M V e_bg with O(t) error.
* Energy balance of a lossless free-standing grating converges to 1.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_25541_amd import clips as C

K0 = 2 * math.pi / 13.5


def small_problem(nx, ny, nz, l=16.0, t=16.0, theta=6.0, phi=20.0, pol=0, pairs=10):
    layers, es = C.mo_si_stack(pairs)
    return C.Problem(nx=nx, ny=ny, nz=nz, lx_nm=l, ly_nm=l, t_nm=t, theta_deg=theta, phi_deg=phi,
                     pol=pol, layers=layers, eps_sub=es)


@pytest.mark.parametrize("shape,pol", [((4, 4, 4), 0), ((8, 8, 4), 1), ((8, 4, 2), 0)])
def test_gmres_outer_loop_equals_dense_direct(shape, pol):
    nx, ny, nz = shape
    rng = np.random.default_rng(7)
    m2 = rng.random((ny, nx)) < 0.5
    de = C.extrude(m2, nz)
    p = small_problem(nx, ny, nz, pol=pol)
    d = O.dense_solve_monolithic(p, de)
    r = O.solve(p, de, rtol=1e-13)
    assert np.linalg.norm(r["u"] - d["u"]) <= 1e-11 * np.linalg.norm(d["u"])
    # the mask field is K V u
    S = r["setup"]
    xm = O.conv_K(S, O.potential(S, de)[None] * d["u"])
    assert np.linalg.norm(r["emask"] - xm) <= 1e-11 * np.linalg.norm(xm)


def test_dense_gmres_of_eq18_alone():
    p = small_problem(4, 4, 4)
    de = C.extrude(np.eye(4, dtype=bool), 4)
    S = O.Setup(p)
    b = C.random_complex((3, 4, 4, 4), seed=3)
    A = O.dense_matrix(lambda v: O.apply_A(S, de, v), 192, b.shape)
    x_ref = np.linalg.solve(A, b.reshape(-1)).reshape(b.shape)
    x, info = O.gmres(lambda v: O.apply_A(S, de, v), b, None, 1e-13, 30, 1000)
    assert np.linalg.norm(x - x_ref) <= 1e-12 * np.linalg.norm(x_ref)
    x5, info5 = O.gmres(lambda v: O.apply_A(S, de, v), b, None, 1e-13, 5, 2000)
    assert np.linalg.norm(x5 - x_ref) <= 1e-12 * np.linalg.norm(x_ref)
    assert info5["iters"] > info["iters"]


@pytest.mark.parametrize("pol", [0, 1])
def test_bare_multilayer(pol):
    p = small_problem(8, 8, 4, pol=pol, pairs=40)
    de = np.zeros((4, 8, 8), dtype=complex)
    r = O.solve(p, de, rtol=1e-12)
    S = r["setup"]
    a = r["orders"]
    ref = S.TR[0, 0] @ S.e_inc * np.exp(1j * S.beta[0, 0] * S.t)
    assert np.max(np.abs(a[0, 0] - ref)) < 1e-14
    a2 = a.copy()
    a2[0, 0] = 0
    assert np.max(np.abs(a2)) == 0.0
    assert np.max(np.abs(r["emask"])) == 0.0
    eta = O.efficiencies(S, a)[0, 0]
    rr = S.rs[0, 0] if pol == 0 else S.rp[0, 0]
    assert abs(eta - abs(rr) ** 2) < 1e-14


@pytest.mark.parametrize("pol", [0, 1])
def test_uniform_film_converges_to_layered_reflection(pol):
    layers, es = C.mo_si_stack(40)
    eabs = C.eps_of(C.N_ABSORBER)
    kt = K0 * math.sin(math.radians(6.0))
    r_exact = O.generalized_reflection(K0, 1.0, [(eabs, 60.0)] + layers, es, np.array([kt]), pol)[0]
    errs = []
    for nz in (16, 32, 64):
        p = C.Problem(nx=4, ny=4, nz=nz, lx_nm=16.0, ly_nm=16.0, t_nm=60.0, theta_deg=6.0, phi_deg=0.0,
                      pol=pol, layers=layers, eps_sub=es)
        de = np.full((nz, 4, 4), eabs - 1.0, dtype=complex)
        r = O.solve(p, de, rtol=1e-11)
        S = r["setup"]
        a0 = r["orders"][0, 0]
        vec = S.s_hat[0, 0] if pol == 0 else S.p_plus[0, 0]
        rr = (vec @ a0) * np.exp(1j * S.beta[0, 0] * 60.0)
        # only the specular order is excited by a laterally uniform film
        others = r["orders"].copy()
        others[0, 0] = 0
        assert np.max(np.abs(others)) < 1e-13
        errs.append(abs(rr - r_exact))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.8, (errs, rates)
    assert errs[-1] < 2e-3 * abs(r_exact) / 0.18 + 1e-3


@pytest.mark.parametrize("pol", [0, 1])
def test_reciprocity_swapped_incidence(pol):
    nx, ny, nz = 16, 8, 8
    layers, es = C.mo_si_stack(10)
    m2 = np.zeros((ny, nx), bool)
    m2[:, 2:5] = True
    m2[:, 7:13] = True
    m2[1:3, 10:15] = True            # no mirror symmetry
    de = C.extrude(m2, nz)
    mk = lambda phi: C.Problem(nx=nx, ny=ny, nz=nz, lx_nm=32.0, ly_nm=32.0, t_nm=30.0, theta_deg=6.0,
                               phi_deg=phi, pol=pol, layers=layers, eps_sub=es)
    r1 = O.solve(mk(0.0), de, rtol=1e-12)
    r2 = O.solve(mk(180.0), de, rtol=1e-12)
    e1 = O.efficiencies(r1["setup"], r1["orders"])
    e2 = O.efficiencies(r2["setup"], r2["orders"])
    assert abs(e1[0, 0] - e2[0, 0]) < 1e-9 * e1[0, 0]
    # k_in -> k_in + G_1  versus  -(k_in + G_1) -> -k_in
    r3 = O.solve(mk(180.0), de, rtol=1e-12, inc_order=(-1, 0))
    e3 = O.efficiencies(r3["setup"], r3["orders"])
    assert abs(e1[0, 1] - e3[0, 0]) < 1e-9 * e1[0, 1]


def test_born_limit():
    p = small_problem(8, 8, 8, phi=0.0)
    S = O.Setup(p)
    de = C.extrude(np.eye(8, dtype=bool) | np.roll(np.eye(8, dtype=bool), 1, 1), 8)
    ebg = O.background_field(S)
    born = O.apply_M(S, O.potential(S, de)[None] * ebg)
    errs = []
    for t in (1e-2, 1e-3):
        r = O.solve(p, t * de, rtol=1e-13, S=S)
        errs.append(np.linalg.norm((r["u"] - ebg) / t - born) / np.linalg.norm(born))
    assert errs[1] < 0.12 * errs[0]
    assert errs[1] < 1e-3


def test_energy_balance_lossless_grating():
    out = []
    for nz in (8, 16, 32):
        p = C.Problem(nx=16, ny=4, nz=nz, lx_nm=32.0, ly_nm=8.0, t_nm=30.0, theta_deg=6.0, phi_deg=0.0,
                      pol=0, layers=[], eps_sub=1.0)
        m2 = np.zeros((4, 16), bool)
        m2[:, 3:9] = True
        de = C.extrude(m2, nz, n_abs=0.95 + 0j)
        r = O.solve(p, de, rtol=1e-12)
        S = r["setup"]
        prop = S.beta.real > 0
        R = O.efficiencies(S, r["orders"])[prop].sum()
        T = O.efficiencies(S, O.transmitted_down(S, de, r["u"]))[prop].sum()
        out.append(abs(R + T - 1.0))
    assert out[0] > out[1] > out[2]
    assert out[2] < 5e-6


def test_outer_loop_stops_on_reflection_change():
    p = small_problem(8, 8, 8, pairs=40)
    de = C.manhattan(8, 8, 8, 16.0, 16.0, seed=4)
    r = O.solve(p, de, rtol=1e-10)
    assert r["outer_change"] <= 1e-10
    assert 2 <= r["outer_iters"] <= 40
    assert r["mono_residual"] < 1e-8
