"""Pins of the spherically windowed dyadic kernel (isolated-domain mode, eqs. (15)-(17)).

The closed forms are checked against an independent derivation by radial
quadrature. With g = exp(i k r) / (4 pi r), the truncated dyadic kernel is, as
a distribution on the ball,

    G_R = (2/3) g I - delta(r) I / (3 k^2) + (g'' - g'/r) (r^ r^ - I/3) / k^2,

whose transform, from the angular integrals of 1 and of r^ r^ - I/3 (the j0 and
j2 terms of the plane-wave expansion), is A I + B k^ k^ with

    S0 = 4 pi int_0^R g j0(kr) r^2 dr,   T2 = (4 pi / k^2) int_0^R (g'' - g'/r) j2(kr) r^2 dr,
    A = (2/3) S0 - 1 / (3 k^2) + T2 / 3,   B = -T2.

The printed h(k; R) (R in place of R^2) and the printed A(0) (no 4 pi) fail the
same check, which is what the readings of the windowed kernel rest on.
"""
import warnings

import numpy as np
import pytest
from scipy import integrate, special

from oracle import isolated as I

K0 = 2 * np.pi / 13.5


def cquad(f, a, b):
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", integrate.IntegrationWarning)
        re = integrate.quad(lambda r: f(r).real, a, b, limit=400, epsabs=1e-14, epsrel=1e-12)[0]
        im = integrate.quad(lambda r: f(r).imag, a, b, limit=400, epsabs=1e-14, epsrel=1e-12)[0]
    return re + 1j * im


def by_quadrature(k, kbg, R):
    """(A, B, S0) from the radial integrals of the distributional decomposition."""
    S0 = cquad(lambda r: np.exp(1j * kbg * r) * r * special.spherical_jn(0, k * r), 0.0, R)
    # (g'' - g'/r) r^2 4 pi = exp(i k r) (3 - 3 i k r - k^2 r^2) / r
    T2 = cquad(lambda r: np.exp(1j * kbg * r) * (3 - 3j * kbg * r - kbg ** 2 * r ** 2)
               * special.spherical_jn(2, k * r) / r, 0.0, R) / kbg ** 2
    return 2.0 / 3.0 * S0 - 1.0 / (3.0 * kbg ** 2) + T2 / 3.0, -T2, S0


CASES = [(K0 * (1 + 0.02j), 40.0), (K0 * (1 + 0.05j), 25.0), (0.9 * K0 * (1 + 0.01j), 60.0)]
KS = [0.02, 0.1, 0.3, K0, 0.9, 2.0, 5.0]


@pytest.mark.parametrize("kbg,R", CASES)
def test_scalar_window_matches_quadrature(kbg, R):
    for k in KS:
        F = I.window_sphere_scalar(k, kbg, R)
        _, _, S0 = by_quadrature(k, kbg, R)
        assert abs(F - S0) <= 1e-9 * abs(S0), (k, F, S0)
    # k = 0: 4 pi int_0^R g r^2 dr
    S00 = cquad(lambda r: np.exp(1j * kbg * r) * r, 0.0, R)
    assert abs(I.window_sphere_scalar(0.0, kbg, R) - S00) <= 1e-9 * abs(S00)


@pytest.mark.parametrize("kbg,R", CASES)
def test_dyadic_window_matches_quadrature(kbg, R):
    for k in KS:
        A, B = I.window_sphere_AB(k, kbg, R)
        Aq, Bq, _ = by_quadrature(k, kbg, R)
        assert abs(A - Aq) <= 1e-9 * abs(Aq), (k, A, Aq)
        assert abs(B - Bq) <= 1e-9 * abs(Bq), (k, B, Bq)


@pytest.mark.parametrize("kbg,R", CASES)
def test_limits_at_k0(kbg, R):
    """A is continuous at k = 0 (with the 4 pi of the corrected A(0)) and B -> 0 as k^2."""
    A0, B0 = I.window_sphere_AB(0.0, kbg, R)
    assert B0 == 0
    for k in (1e-4 / R, 1e-3 / R, 1e-2 / R):
        A, B = I.window_sphere_AB(k, kbg, R)
        assert abs(A - A0) <= 1e-4 * abs(A0)
        assert abs(B) <= 0.2 * (k * R) ** 2 * abs(A0)
    # the quadrature at k = 0 (j2 vanishes: B = 0, A = (2/3) S0 - 1/(3 k^2))
    S00 = cquad(lambda r: np.exp(1j * kbg * r) * r, 0.0, R)
    assert abs(A0 - (2.0 / 3.0 * S00 - 1.0 / (3.0 * kbg ** 2))) <= 1e-9 * abs(A0)


def test_lossless_resonance_limit():
    """For a real k_bg the scalar transform has a removable point at k = k_bg."""
    kbg, R = K0, 30.0
    F0 = I.window_sphere_scalar(kbg, kbg, R)
    for d in (1e-5, -1e-5, 1e-4):
        assert abs(I.window_sphere_scalar(kbg * (1 + d), kbg, R) - F0) <= 5e-3 * abs(F0) * abs(d) / 1e-5
    _, _, S0 = by_quadrature(kbg, kbg, R)
    assert abs(F0 - S0) <= 1e-9 * abs(S0)


def test_printed_forms_fail_quadrature():
    """The printed h (R instead of R^2) and the printed A(0) (no 4 pi) disagree with the kernel."""
    kbg, R, k = K0 * (1 + 0.02j), 40.0, 0.3
    Aq, Bq, _ = by_quadrature(k, kbg, R)
    F = I.window_sphere_scalar(k, kbg, R)
    h_printed = I.window_sphere_h(k, kbg, R) / R  # 4 pi R g'(R) j1(kR) / (k^2 kR)
    assert abs((F + h_printed) - Aq) > 1e-2 * abs(Aq)
    assert abs((-F - 3 * h_printed - 1 / kbg ** 2) - Bq) > 1e-2 * abs(Bq)
    A0, _ = I.window_sphere_AB(0.0, kbg, R)
    A0_printed = I.window_sphere_scalar(0.0, kbg, R) + R ** 2 * (
        I.g_prime_times_4pi_r2(kbg, R) / (4 * np.pi * R ** 2)) / (3 * kbg ** 2)
    assert abs(A0_printed - A0) > 1e-2 * abs(A0)


def test_dyadic_structure():
    """F[G_R] is symmetric and even in k, k^ is an eigenvector (A + B), the transverse plane A."""
    kbg, R = K0 * (1 + 0.02j), 40.0
    rng = np.random.default_rng(9)
    kv = rng.normal(size=(20, 3)) * 0.4
    G = I.gtilde_isolated(kv[:, 0], kv[:, 1], kv[:, 2], kbg, R)
    Gm = I.gtilde_isolated(-kv[:, 0], -kv[:, 1], -kv[:, 2], kbg, R)
    assert np.allclose(G, np.swapaxes(G, -1, -2), rtol=0, atol=1e-14)
    assert np.allclose(G, Gm, rtol=0, atol=1e-14)
    k = np.linalg.norm(kv, axis=1)
    A, B = I.window_sphere_AB(k, kbg, R)
    kh = kv / k[:, None]
    assert np.allclose(np.einsum("nij,nj->ni", G, kh), (A + B)[:, None] * kh, atol=1e-12)
    t = np.cross(kh, np.array([0.3, -0.2, 0.9]))
    t /= np.linalg.norm(t, axis=1)[:, None]
    assert np.allclose(np.einsum("nij,nj->ni", G, t), A[:, None] * t, atol=1e-12)
    # k = 0: A(0) I
    G0 = I.gtilde_isolated(0.0, 0.0, 0.0, kbg, R)
    assert np.allclose(G0, I.window_sphere_AB(0.0, kbg, R)[0] * np.eye(3), atol=1e-14)


def test_isolated_apply_is_the_discrete_linear_convolution():
    """The 2x-padded FFT apply equals the direct sum over voxel pairs with the
    kernel samples of the 4x-oversampled precompute (a tiny grid, so that the
    O(N^2) sum is cheap): y_i = x_i - sum_j K[i - j] V_j x_j dV."""
    shape, spacing = (3, 4, 5), (2.0, 1.5, 1.0)
    kbg = K0 * (1 + 0.02j)
    nz, ny, nx = shape
    R = 1.2 * np.sqrt((nz * spacing[0]) ** 2 + (ny * spacing[1]) ** 2 + (nx * spacing[2]) ** 2)
    rng = np.random.default_rng(3)
    vol = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    x = rng.normal(size=(3,) + shape) + 1j * rng.normal(size=(3,) + shape)
    K = I.kernel_samples(shape, spacing, kbg, R)
    y = I.apply_isolated(I.isolated_table(shape, spacing, kbg, R), vol, x)
    dV = spacing[0] * spacing[1] * spacing[2]
    ref = x.copy()
    for iz in range(nz):
        for iy in range(ny):
            for ix in range(nx):
                acc = np.zeros(3, dtype=complex)
                for jz in range(nz):
                    for jy in range(ny):
                        for jx in range(nx):
                            k = K[(iz - jz) % (2 * nz), (iy - jy) % (2 * ny), (ix - jx) % (2 * nx)]
                            acc += k @ (vol[jz, jy, jx] * x[:, jz, jy, jx])
                ref[:, iz, iy, ix] -= acc * dV
    assert np.max(np.abs(y - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_isolated_kernel_samples_even_and_symmetric():
    """The kernel samples are symmetric 3x3 and even in the offset, so the
    discrete isolated operator is complex-symmetric (reciprocal)."""
    shape, spacing = (4, 4, 6), (1.0, 1.0, 1.0)
    kbg = K0 * (1 + 0.03j)
    R = 1.1 * np.sqrt(4 ** 2 + 4 ** 2 + 6 ** 2)
    K = I.kernel_samples(shape, spacing, kbg, R)
    assert np.allclose(K, np.swapaxes(K, -1, -2), rtol=0, atol=1e-12 * np.abs(K).max())
    # K at offset -j (FFT order on 2n); the offset -n of each axis has no stored
    # partner +n, so those planes are left out
    Kneg = np.roll(np.flip(K, axis=(0, 1, 2)), shift=(1, 1, 1), axis=(0, 1, 2))
    inner = np.ones(K.shape[:3], dtype=bool)
    inner[shape[0]] = False
    inner[:, shape[1]] = False
    inner[:, :, shape[2]] = False
    assert np.allclose(K[inner], Kneg[inner], rtol=0, atol=1e-12 * np.abs(K).max())
    # reciprocity of the apply: <a, (I - A) b> = <b, (I - A) a> (bilinear) for V = 1
    rng = np.random.default_rng(5)
    T = I.isolated_table(shape, spacing, kbg, R)
    a = rng.normal(size=(3,) + shape) + 1j * rng.normal(size=(3,) + shape)
    b = rng.normal(size=(3,) + shape) + 1j * rng.normal(size=(3,) + shape)
    one = np.ones(shape)
    lhs = np.sum(a * (b - I.apply_isolated(T, one, b)))
    rhs = np.sum(b * (a - I.apply_isolated(T, one, a)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_isolated_dense_solve():
    """The dense solve satisfies the isolated system to rounding, reduces to
    u = b without contrast, and agrees with scipy's GMRES on the operator."""
    from scipy.sparse.linalg import LinearOperator, gmres
    shape, spacing = (2, 4, 4), (1.0, 2.0, 2.0)
    kbg = K0 * (1 + 0.02j)
    R = float(np.sqrt(sum((n * h) ** 2 for n, h in zip(shape, spacing))))
    T = I.isolated_table(shape, spacing, kbg, R, I.oversampling(shape, spacing, R))
    rng = np.random.default_rng(12)
    vol = K0 ** 2 * (0.3 * rng.normal(size=shape) + 0.1j * rng.random(size=shape))
    b = rng.normal(size=(3,) + shape) + 1j * rng.normal(size=(3,) + shape)
    u = I.solve_isolated_dense(T, vol, b)
    r = b - I.apply_isolated(T, vol, u)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(b)
    assert np.allclose(I.solve_isolated_dense(T, np.zeros(shape), b), b, rtol=0, atol=1e-14)
    op = LinearOperator((b.size, b.size), dtype=complex,
                        matvec=lambda v: I.apply_isolated(T, vol, v.reshape(b.shape)).ravel())
    ug, info = gmres(op, b.ravel(), rtol=1e-13, atol=0.0, restart=b.size, maxiter=10)
    assert info == 0
    assert np.linalg.norm(ug - u.ravel()) <= 1e-10 * np.linalg.norm(u)


@pytest.mark.parametrize("shape,spacing", [((4, 8, 8), (1.0, 3.0, 3.0)), ((8, 4, 16), (2.0, 2.0, 1.0))])
def test_isolated_offset_minus_n_plane_is_inert(shape, spacing):
    """The padded convolution meets offsets in (-n, n) only, so zeroing the kernel
    samples at the offset plane jz = -nz leaves the operator unchanged. Without
    that plane the samples are even along z in xx, yy, zz, xy and odd in xz, yz,
    so the table is even / odd in kz and kz = 0 .. nz determines it (what the
    z-pencil order of the apply stores)."""
    kbg = K0 * (1 + 0.02j)
    nz = shape[0]
    R = float(np.sqrt(sum((n * h) ** 2 for n, h in zip(shape, spacing))))
    K = I.kernel_samples(shape, spacing, kbg, R, I.oversampling(shape, spacing, R))
    dV = np.prod(spacing)
    T = np.fft.fftn(K, axes=(0, 1, 2)) * dV
    Ke = K.copy()
    Ke[nz] = 0
    Te = np.fft.fftn(Ke, axes=(0, 1, 2)) * dV
    sgn = np.array([[1, 1, -1], [1, 1, -1], [-1, -1, 1]])
    kz = np.arange(1, 2 * nz)
    assert np.abs(Te[kz] - sgn * Te[2 * nz - kz]).max() <= 1e-14 * np.abs(Te).max()
    rng = np.random.default_rng(1)
    vol = rng.normal(size=shape) + 0.3j
    x = rng.normal(size=(3,) + shape) + 1j * rng.normal(size=(3,) + shape)
    y0 = I.apply_isolated(T, vol, x)
    Th = Te.copy()
    Th[nz + 1:] = sgn * Te[2 * nz - np.arange(nz + 1, 2 * nz)]
    assert np.abs(I.apply_isolated(Th, vol, x) - y0).max() <= 1e-14 * np.abs(y0).max()
    # the plane itself is not negligible: dropping another plane does change the operator
    Kb = K.copy()
    Kb[1] = 0
    Tb = np.fft.fftn(Kb, axes=(0, 1, 2)) * dV
    assert np.abs(I.apply_isolated(Tb, vol, x) - y0).max() > 1e-6 * np.abs(y0).max()


# ---------------------------------------------------------------------------
# Pin of the discretised precompute (kernel samples, 1/dV, per-axis period and
# restriction, then the padded apply): the discrete convolution of a smooth
# density converges to the continuous convolution with the windowed dyadic
# kernel (eqs. (13)-(17) and the zero-padded apply of eq. (18)). The
# continuous reference comes from a radial quadrature of the scalar potential
# of a Gaussian, with no FFT and none of the precompute's arithmetic.
# ---------------------------------------------------------------------------

def _gauss_potential(r, k, s):
    """phi, phi', phi'' of phi = g * f for f = exp(-rho^2 / (2 s^2)), g = exp(i k d) / (4 pi d).

    The spherical mean of g over |r'| = rho is (exp(ik(r + rho)) - exp(ik|r - rho|)) / (8 pi i k r rho),
    so phi = J / (2 i k r) with J(r) = int_0^inf rho f (exp(ik(r + rho)) - exp(ik|r - rho|)) d rho;
    J' is the same integral differentiated under the sign, and J'' = -k^2 J - 2 i k r f(r)
    (the jump of the sign term), which is the Helmholtz equation of phi with source f.
    """
    f = lambda q: np.exp(-q * q / (2 * s * s))
    top = 14 * s
    pts = [r] if r < top else None

    def quad(fn):
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", integrate.IntegrationWarning)
            re = integrate.quad(lambda q: fn(q).real, 0, top, points=pts, limit=400, epsabs=1e-15, epsrel=1e-12)[0]
            im = integrate.quad(lambda q: fn(q).imag, 0, top, points=pts, limit=400, epsabs=1e-15, epsrel=1e-12)[0]
        return re + 1j * im

    J = quad(lambda q: q * f(q) * (np.exp(1j * k * (r + q)) - np.exp(1j * k * abs(r - q))))
    Jp = quad(lambda q: q * f(q) * 1j * k * (np.exp(1j * k * (r + q)) - np.sign(r - q) * np.exp(1j * k * abs(r - q))))
    Jpp = -k * k * J - 2j * k * r * f(r)
    c = 1.0 / (2j * k)
    return c * J / r, c * (Jp / r - J / r ** 2), c * (Jpp / r - 2 * Jp / r ** 2 + 2 * J / r ** 3)


def _gauss_field(rxyz, k, s, p):
    """E(r) = (I + grad grad / k^2)(g * f) p: for a radial phi,
    grad grad phi = phi'' r^ r^ + (phi' / r)(I - r^ r^)."""
    out = np.empty((len(rxyz), 3), dtype=complex)
    for i, rv in enumerate(rxyz):
        r = float(np.linalg.norm(rv))
        phi, d1, d2 = _gauss_potential(r, k, s)
        rh = rv / r
        out[i] = (phi + d1 / (k * k * r)) * p + ((d2 - d1 / r) / (k * k)) * np.dot(rh, p) * rh
    return out


def _gauss_apply_error(spacing, over=None, scale=1.0, swap=False, npts=30):
    """Max error (relative to the largest reference value) of K(f p) at sampled voxels against the
    continuous field, for a Gaussian (s = 1.6 nm) at the centre of a 16 x 24 x 32 nm box with an
    anisotropic voxel `spacing` (dz, dy, dx); R is the box diagonal."""
    box, s = (16.0, 24.0, 32.0), 1.6
    kbg = K0 * (1 + 0.02j)
    p = np.array([0.3, -0.5, 0.8 + 0.2j])
    shape = tuple(int(round(b / h)) for b, h in zip(box, spacing))
    R = float(np.sqrt(sum(b * b for b in box)))
    over = over or I.oversampling(shape, spacing, R)
    T = I.isolated_table(shape, spacing[::-1] if swap else spacing, kbg, R, over) * scale
    axes = [(np.arange(n) + 0.5) * h - b / 2 for n, h, b in zip(shape, spacing, box)]
    Z, Y, X = np.meshgrid(*axes, indexing="ij")
    f = np.exp(-(X * X + Y * Y + Z * Z) / (2 * s * s))
    x = np.broadcast_to(p[:, None, None, None], (3,) + shape).astype(complex)
    w = x - I.apply_isolated(T, f, x)              # K (f p)
    rng = np.random.default_rng(0)
    idx = [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(npts)]
    rxyz = np.array([[X[i], Y[i], Z[i]] for i in idx])
    E = _gauss_field(rxyz, kbg, s, p)
    got = np.array([[w[c][i] for c in range(3)] for i in idx])
    return float(np.abs(got - E).max() / np.abs(E).max())


def test_isolated_precompute_converges_to_the_continuous_convolution():
    """Refining an anisotropic grid over a fixed box, the discrete isolated
    operator applied to a Gaussian density converges spectrally to the
    continuous windowed-kernel convolution: 1.8e-2 at voxels (2, 1.5, 1) nm,
    6e-7 at (1, 0.75, 0.5) nm. A wrong cell-volume factor, swapped spacings
    or a period without the oversampling each leave an O(1e-1..1) error."""
    coarse = _gauss_apply_error((2.0, 1.5, 1.0))
    fine = _gauss_apply_error((1.0, 0.75, 0.5))
    assert fine <= 1e-5, fine
    assert coarse >= 100 * fine, (coarse, fine)
    sp = (1.0, 0.75, 0.5)
    assert _gauss_apply_error(sp, scale=2.0, npts=8) > 0.1    # a factor 2 in 1/dV
    assert _gauss_apply_error(sp, swap=True, npts=8) > 0.1    # (dz, dy, dx) taken as (dx, dy, dz)
    assert _gauss_apply_error(sp, over=(2, 2, 2), npts=8) > 0.05  # period 2 L: ball images wrap in
