"""Pins of the differential PSFD oracle (Sec. 3: eqs. (6)-(8), the preconditioner study).

* The pseudo-spectral curl curl of a decaying wave packet converges
  exponentially to the analytic curl curl (the convergence study of Sec. 3).
* curl grad = 0 and div curl = 0 hold to rounding, with the PML stretch too
  (a sign or component slip in the curl breaks them).
* The PML absorbs an outgoing wave: a source sheet's field against the analytic
  outgoing solution, with the error falling as the layer thickens; without PML
  the periodic wrap spoils it.
* GMRES with either preconditioner reproduces a dense direct solve.
* The spectral-damping multiplier is min(1, k_bg^2 / |k|^2) on Fourier modes.
* Background-field form: a laterally uniform film on the multilayer converges to
  the exact layered reflection of [film + multilayer] as the grid is refined.
* Full-domain form: with no layers it is the background form with an empty stack.
"""
import math
import warnings

import numpy as np
import pytest
from scipy import integrate

import oracle as O
from oracle import differential as Df
from paper_2606_25541_amd import clips as C

K0 = 2 * math.pi / 13.5


def _setup(nx, ny, nz, pe, zc0, ncz, npml, L=16.0, t=8.0, theta=0.0, pol=0, layers=None, es=1.0, p=3):
    prob = C.Problem(nx=nx, ny=ny, nz=nz, lx_nm=L, ly_nm=L, t_nm=t, theta_deg=theta, phi_deg=0.0, pol=pol,
                     layers=layers or [], eps_sub=es)
    return Df.DiffSetup(prob, pe, zc0, ncz, npml, p)


def _packet(D, Lz, q, w):
    """phi = exp(i q.r) exp(-|r - c|^2 / (2 w^2)) on the grid (centre of the box) and its Hessian."""
    S = D.S
    x = np.arange(D.nx) * S.lx / D.nx
    y = np.arange(D.ny) * S.ly / D.ny
    z = D.z
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    c = (S.lx / 2, S.ly / 2, z[D.pe // 2])
    R = [X - c[0], Y - c[1], Z - c[2]]
    phi = np.exp(1j * (q[0] * X + q[1] * Y + q[2] * Z)) * np.exp(-(R[0] ** 2 + R[1] ** 2 + R[2] ** 2) / (2 * w * w))
    g = [1j * q[i] - R[i] / w ** 2 for i in range(3)]
    H = [[phi * (g[i] * g[j] - (1.0 / w ** 2 if i == j else 0.0)) for j in range(3)] for i in range(3)]
    return phi, H


@pytest.mark.parametrize("n", [24, 32, 48])
def test_curl_curl_of_a_wave_packet_converges_spectrally(n):
    """curl curl (p phi) = Hess(phi) p - lap(phi) p for the packet; the error falls
    exponentially with the points per axis (1e-2 at 16, below 1e-9 at 48)."""
    L = 24.0
    errs = []
    for m in (16, n):
        D = _setup(m, m, 2, m, m // 2, 2, 0, L=L, t=2 * L / m)
        q = (2 * np.pi * 2 / L, -2 * np.pi / L, 2 * np.pi * 3 / L)
        phi, H = _packet(D, L, q, L / 18)
        p = np.array([0.3, -0.7 + 0.2j, 0.5])
        f = np.stack([p[c] * phi for c in range(3)])
        lap = H[0][0] + H[1][1] + H[2][2]
        exact = np.stack([sum(H[i][j] * p[j] for j in range(3)) - lap * p[i] for i in range(3)])
        got = Df.curl(D, Df.curl(D, f))
        errs.append(np.abs(got - exact).max() / np.abs(exact).max())
    assert errs[0] > 1e-4
    assert errs[1] < {24: 2e-2, 32: 5e-4, 48: 1e-9}[n], errs


def test_curl_identities_with_pml():
    D = _setup(8, 8, 4, 32, 14, 4, 6, theta=10.0)
    rng = np.random.default_rng(4)
    phi = rng.normal(size=(32, 8, 8)) + 1j * rng.normal(size=(32, 8, 8))
    grad = np.stack([Df._dx(D, phi), Df._dy(D, phi), Df._dz(D, phi)])
    assert np.abs(Df.curl(D, grad)).max() <= 1e-12 * np.abs(grad).max() * 10
    f = rng.normal(size=(3, 32, 8, 8)) + 1j * rng.normal(size=(3, 32, 8, 8))
    c = Df.curl(D, f)
    div = Df._dx(D, c[0]) + Df._dy(D, c[1]) + Df._dz(D, c[2])
    assert np.abs(div).max() <= 1e-12 * np.abs(c).max() * 10


def _sheet_error(npml, pe=192, p=3):
    """-E'' - k^2 E = f for a Gaussian sheet f (normal incidence, one order): the
    discrete solution against the outgoing solution (i / 2k) int exp(ik|z - z'|) f dz'
    on the planes outside the PML."""
    D = _setup(1, 1, 2, pe, pe // 2, 2, npml, L=8.0, t=1.0)
    k = D.S.kbg
    zc, w = D.z[pe // 2], 1.5
    f = np.exp(-(D.z - zc) ** 2 / (2 * w * w))
    b = np.zeros((3, pe, 1, 1), dtype=complex)
    b[0, :, 0, 0] = f
    n3 = 3 * pe
    A = O.dense_matrix(lambda v: Df.apply_diff(D, np.zeros((2, 1, 1)), v), n3, b.shape)
    E = np.linalg.solve(A, b.ravel()).reshape(b.shape)[0, :, 0, 0]
    inner = np.arange(npml, pe - npml)
    ref = []
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        for kk in inner:
            z = D.z[kk]
            g = lambda s: np.exp(1j * k * abs(z - s)) * np.exp(-(s - zc) ** 2 / (2 * w * w))
            re = integrate.quad(lambda s: g(s).real, zc - 12 * w, zc + 12 * w, points=[z], limit=200)[0]
            im = integrate.quad(lambda s: g(s).imag, zc - 12 * w, zc + 12 * w, points=[z], limit=200)[0]
            ref.append(1j / (2 * k) * (re + 1j * im))
    ref = np.array(ref)
    return np.abs(E[inner] - ref).max() / np.abs(ref).max()


def test_pml_absorbs_outgoing_waves():
    errs = [_sheet_error(n) for n in (4, 8, 16, 32)]
    assert errs[-1] < 1e-4, errs
    assert errs[0] > errs[1] > errs[2] > errs[-1], errs
    assert _sheet_error(0) > 10 * errs[-1]       # no PML: the wave wraps around


@pytest.mark.parametrize("precond", ["none", "damping"])
def test_gmres_matches_dense_solve(precond):
    layers, es = C.mo_si_stack(4)
    D = _setup(4, 4, 2, 16, 6, 2, 3, L=12.0, t=3.0, theta=8.0, pol=1, layers=layers, es=es)
    rng = np.random.default_rng(8)
    de = 0.2 * (rng.normal(size=(2, 4, 4)) + 0.3j)
    b = Df.rhs(D, de, rng.normal(size=(3, 2, 4, 4)) + 1j * rng.normal(size=(3, 2, 4, 4)))
    n3 = b.size
    A = O.dense_matrix(lambda v: Df.apply_diff(D, de, v), n3, b.shape)
    x_ref = np.linalg.solve(A, b.ravel()).reshape(b.shape)
    x, info = Df.solve_linear(D, de, b, precond, rtol=1e-13, restart=n3)
    assert info["rel_residual"] <= 1e-13
    assert np.linalg.norm(x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)


def test_damping_multiplier_on_fourier_modes():
    D = _setup(8, 8, 4, 16, 6, 4, 2, L=20.0, t=8.0, theta=12.0)
    S = D.S
    for (l, j, i) in ((0, 0, 0), (1, 0, 2), (3, 5, 1), (8, 4, 7)):
        mode = np.zeros((3, 16, 8, 8), dtype=complex)
        spec = np.zeros((16, 8, 8), dtype=complex)
        spec[l, j, i] = 1.0
        mode[1] = np.fft.ifftn(spec)
        k2 = S.kx[i] ** 2 + S.ky[j] ** 2 + D.kappa[l] ** 2
        want = min(1.0, S.kbg ** 2 / k2)
        assert np.allclose(Df.damping(D, mode), want * mode, rtol=0, atol=1e-15)


def test_uniform_film_background_converges_to_layered_reflection():
    """TE, 60 nm film on 40 Mo/Si pairs at 6 deg: the specular order of the
    differential background-field method against the exact reflection of
    [film + stack]; refining dz (and the PML with it) from 3.75 to 1.875 nm cuts
    the error by more than 5x (2.8e-2 -> 3.0e-3)."""
    layers, es = C.mo_si_stack(40)
    eabs = C.eps_of(C.N_ABSORBER)
    kt = K0 * math.sin(math.radians(6.0))
    r_exact = O.generalized_reflection(K0, 1.0, [(eabs, 60.0)] + layers, es, np.array([kt]), 0)[0]
    errs = []
    for nz, pe, npml in ((16, 64, 8), (32, 128, 16)):
        D = _setup(4, 4, nz, pe, (pe - nz) // 2, nz, npml, L=16.0, t=60.0, theta=6.0, layers=layers, es=es)
        de = np.full((nz, 4, 4), eabs - 1.0, dtype=complex)
        r = Df.solve_background(D, de, "damping", rtol=1e-11)
        others = r["orders"].copy()
        others[0, 0] = 0
        assert np.abs(others).max() < 1e-10
        rr = (D.S.s_hat[0, 0] @ r["orders"][0, 0]) * np.exp(1j * D.S.beta[0, 0] * 60.0)
        errs.append(abs(rr - r_exact))
    assert errs[1] < 5e-3 and errs[0] > 5 * errs[1], errs


def test_full_domain_without_layers_is_the_background_form_without_stack():
    D = _setup(8, 8, 4, 32, 14, 4, 6, L=16.0, t=8.0, theta=6.0, pol=1)
    de = C.manhattan(8, 8, 4, 16.0, 16.0, seed=3)
    rb = Df.solve_background(D, de, "none", rtol=1e-12)
    rf = Df.solve_full_domain(D, de, "none", rtol=1e-12)
    assert rb["outer_iters"] == 1
    assert np.linalg.norm(rf["E"] - rb["E"]) <= 1e-10 * np.linalg.norm(rb["E"])
    assert np.abs(rf["orders"] - rb["orders"]).max() <= 1e-10 * np.abs(rb["orders"]).max()
