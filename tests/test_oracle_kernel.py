"""Pins of the oracle's windowed dyadic Green's function (eqs. (13)-(17)).

For the xy-periodic clip the kernel is windowed in z only. The closed form in
the oracle is checked against direct numerical quadrature of the spatial
kernel over the window (a route that never uses the closed form), against the
unwindowed free-space transform of eq. (14) in the limit of a large window with
a lossy background, and against the symmetries the discrete reciprocity needs.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O

K0 = 2 * math.pi / 13.5


def quad_c(f, a, b):
    re = integrate.quad(lambda z: f(z).real, a, b, limit=400, epsabs=1e-14, epsrel=1e-12)[0]
    im = integrate.quad(lambda z: f(z).imag, a, b, limit=400, epsabs=1e-14, epsrel=1e-12)[0]
    return re + 1j * im


def windowed_by_quadrature(kx, ky, kappa, kbg, L):
    """int_{-L}^{L} G(kt, z) exp(-i kappa z) dz from the spatial kernel.

    Mixed-domain scalar kernel g = i exp(i beta |z|) / (2 beta); the dyadic
    kernel (I + grad grad / kbg^2) g has grad = (i kx, i ky, d/dz); away from
    z = 0, d/dz g = -sign(z) exp(i beta |z|) / 2 and d2/dz2 g = -beta^2 g, and
    the zz entry carries the local term -delta(z) / kbg^2.
    """
    beta = np.sqrt(complex(kbg * kbg - kx * kx - ky * ky))
    if beta.imag < 0:
        beta = -beta
    g = lambda z: 1j * np.exp(1j * beta * abs(z)) / (2 * beta)
    dg = lambda z: -np.sign(z) * np.exp(1j * beta * abs(z)) / 2
    k2 = kbg * kbg
    ent = {
        (0, 0): lambda z: (1 - kx * kx / k2) * g(z),
        (1, 1): lambda z: (1 - ky * ky / k2) * g(z),
        (0, 1): lambda z: (-kx * ky / k2) * g(z),
        (0, 2): lambda z: (1j * kx / k2) * dg(z),
        (1, 2): lambda z: (1j * ky / k2) * dg(z),
        (2, 2): lambda z: (1 - beta * beta / k2) * g(z),
    }
    out = np.zeros((3, 3), dtype=complex)
    for (i, j), f in ent.items():
        w = lambda z, f=f: f(z) * np.exp(-1j * kappa * z)
        out[i, j] = quad_c(w, -L, 0.0) + quad_c(w, 0.0, L)
        out[j, i] = out[i, j]
    out[2, 2] += -1.0 / k2
    return out


@pytest.mark.parametrize("kx,ky,l", [(0.0487, 0.0, 3), (0.3, -0.2, 5), (0.9, 0.4, -7), (0.0, 0.0, 1),
                                     (0.1, 0.05, 0), (0.6, 0.3, 12)])
def test_gtilde_matches_quadrature(kx, ky, l):
    L = 60.0
    kappa = math.pi * l / L
    sgn = (-1.0) ** l
    beta = O.kz_branch(K0 ** 2 - kx * kx - ky * ky)
    G = O.gtilde_periodic(kx, ky, kappa, beta, K0, L, sgn)
    Q = windowed_by_quadrature(kx, ky, kappa, K0, L)
    assert np.max(np.abs(G - Q)) <= 1e-9 * np.max(np.abs(Q))


def test_large_window_limit_is_free_space_transform():
    """Lossy background, L -> inf: F[G] = (I - k k^T / kbg^2) / (k^2 - kbg^2)."""
    kbg = K0 * (1 + 0.05j)
    kx, ky, kappa = 0.2, -0.1, 0.37
    L = 4000.0
    beta = O.kz_branch(kbg ** 2 - kx * kx - ky * ky)
    G = O.gtilde_periodic(kx, ky, kappa, beta, kbg, L, 1.0)
    k = np.array([kx, ky, kappa])
    ref = (np.eye(3) - np.outer(k, k) / kbg ** 2) / (k @ k - kbg ** 2)
    assert np.max(np.abs(G - ref)) < 1e-12 * np.max(np.abs(ref))


def test_resonance_is_continuous():
    """At kappa = beta the closed form is 0/0; the series branch is continuous."""
    L = 60.0
    l = 5
    kappa = math.pi * l / L
    beta0 = kappa
    vals = []
    for d in (0.0, 1e-9, 1e-7, 2e-6, 1e-5):
        b = beta0 + d / L
        vals.append(O.window_scalar(b, kappa, L, (-1.0) ** l))
    lim = 1j * L / (2 * beta0)
    assert abs(vals[0] - lim) < 1e-14 * abs(lim)
    for v in vals[1:]:
        assert abs(v - lim) < 1e-4 * abs(lim)


def test_table_even_and_symmetric():
    from paper_2606_25541_amd import clips as C
    layers, es = C.mo_si_stack(4)
    p = C.Problem(nx=8, ny=4, nz=4, lx_nm=24.0, ly_nm=12.0, t_nm=16.0, theta_deg=9.0, phi_deg=20.0,
                  layers=layers, eps_sub=es)
    S = O.Setup(p)
    G = S.G
    assert np.max(np.abs(G - np.swapaxes(G, -1, -2))) == 0.0
    # base -k0 problem: G(-k) at the flipped index must equal G(k)
    p2 = C.Problem(**{**p.__dict__, "phi_deg": 200.0})
    S2 = O.Setup(p2)
    flip = lambda a: np.roll(np.flip(a, axis=(0, 1, 2)), 1, axis=(0, 1, 2))
    assert np.max(np.abs(S2.G - flip(S.G))) < 1e-12 * np.max(np.abs(S.G))
