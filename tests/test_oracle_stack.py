"""Pins of the oracle's layered-stack reflection (Sec. 2: reflection operator R;
Sec. 3, eq. (9): T_R built from the stack's generalized reflection).

The recursion in the oracle is checked against an independent 2x2
characteristic-matrix propagation written here, the single-interface Fresnel
formulas, and the closed form of a lossless quarter-wave stack at normal
incidence.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2606_25541_amd import clips as C

K0 = 2 * math.pi / 13.5


def char_matrix_reflection(k0, eps0, layers, eps_s, kt, pol):
    """Reflection of U = E_y (TE) or H_y (TM) at the top surface.

    Propagates (U, U'/p) from the substrate (one downgoing wave) up through each
    layer with its 2x2 characteristic matrix, then splits the result at z = 0
    into down- and upgoing waves of the ambient medium. p = 1 (TE), eps (TM).
    """
    def kz(e):
        r = np.sqrt(complex(k0 * k0 * e - kt * kt))
        return -r if (r.imag < 0 or (r.imag == 0 and r.real < 0)) else r

    p = (lambda e: 1.0) if pol == 0 else (lambda e: complex(e))
    ks = kz(eps_s)
    vec = np.array([1.0 + 0j, -1j * ks / p(eps_s)])
    for e, d in reversed(layers):
        k = kz(e)
        q = k / p(e)
        dl = k * d
        m = np.array([[np.cos(dl), np.sin(dl) / q], [-q * np.sin(dl), np.cos(dl)]])
        vec = m @ vec
    k0z = kz(eps0)
    F, G = vec
    b = (F + G * p(eps0) / (1j * k0z)) / 2
    a = (F - G * p(eps0) / (1j * k0z)) / 2
    return b / a


@pytest.mark.parametrize("pol", [0, 1])
@pytest.mark.parametrize("theta", [0.0, 6.0, 25.0, 80.0])
def test_recursion_matches_characteristic_matrix(pol, theta):
    layers, es = C.mo_si_stack(40)
    layers = [(C.eps_of(C.N_ABSORBER), 60.0)] + layers
    kt = K0 * math.sin(math.radians(theta))
    r_rec = O.generalized_reflection(K0, 1.0, layers, es, np.array([kt]), pol)[0]
    r_cm = char_matrix_reflection(K0, 1.0, layers, es, kt, pol)
    assert abs(r_rec - r_cm) <= 1e-12 * max(1.0, abs(r_cm))


@pytest.mark.parametrize("pol", [0, 1])
def test_recursion_evanescent_orders(pol):
    layers, es = C.mo_si_stack(10)
    for kt in (1.2 * K0, 2.0 * K0, 5.0 * K0):
        r_rec = O.generalized_reflection(K0, 1.0, layers, es, np.array([kt]), pol)[0]
        r_cm = char_matrix_reflection(K0, 1.0, layers, es, kt, pol)
        assert abs(r_rec - r_cm) <= 1e-10 * max(1.0, abs(r_cm))


def test_single_interface_fresnel():
    n1, n2 = 1.0, 1.5 + 0.01j
    th = math.radians(30.0)
    kt = K0 * math.sin(th)
    c1 = math.cos(th)
    c2 = np.sqrt(1 - (n1 * math.sin(th) / n2) ** 2)
    rs = (n1 * c1 - n2 * c2) / (n1 * c1 + n2 * c2)
    # H-field ratio for TM (tangential H continuous)
    rp_h = (n2 * c1 - n1 * c2) / (n2 * c1 + n1 * c2)
    got_s = O.generalized_reflection(K0, n1 ** 2, [], n2 ** 2, np.array([kt]), 0)[0]
    got_p = O.generalized_reflection(K0, n1 ** 2, [], n2 ** 2, np.array([kt]), 1)[0]
    assert abs(got_s - rs) < 1e-14
    assert abs(got_p - rp_h) < 1e-14


def test_quarter_wave_stack_closed_form():
    nh, nl, ns, n0, npair = 2.3, 1.38, 1.52, 1.0, 7
    lam = 13.5
    layers = [(nh ** 2, lam / (4 * nh)), (nl ** 2, lam / (4 * nl))] * npair
    x = (nl / nh) ** (2 * npair)
    r_exact = (n0 * x - ns) / (n0 * x + ns)
    got = O.generalized_reflection(K0, n0 ** 2, layers, ns ** 2, np.array([0.0]), 0)[0]
    assert abs(got - r_exact) < 1e-13
    got_tm = O.generalized_reflection(K0, n0 ** 2, layers, ns ** 2, np.array([0.0]), 1)[0]
    assert abs(got_tm + r_exact) < 1e-13  # H ratio = -E ratio at normal incidence


def test_reflection_matrix_normal_incidence_basis_free():
    """At kt = 0, T_R = r_s (I - z z^T) whatever the azimuth (r_p = -r_s)."""
    layers, es = C.mo_si_stack(40)
    for phi in (0.0, 37.0):
        p = C.Problem(nx=4, ny=4, nz=2, lx_nm=8.0, ly_nm=8.0, t_nm=4.0, theta_deg=0.0,
                      phi_deg=phi, layers=layers, eps_sub=es)
        S = O.Setup(p)
        T = S.TR[0, 0]
        ref = S.rs[0, 0] * np.diag([1.0, 1.0, 0.0])
        assert np.max(np.abs(T - ref)) < 1e-14


def test_mo_si_mirror_reflectance_plausible():
    """40 Mo/Si pairs at 13.5 nm: the mirror reflects ~70 % (Bragg peak)."""
    layers, es = C.mo_si_stack(40)
    r = O.generalized_reflection(K0, 1.0, layers, es, np.array([K0 * math.sin(math.radians(6))]), 0)[0]
    assert 0.6 < abs(r) ** 2 < 0.8
