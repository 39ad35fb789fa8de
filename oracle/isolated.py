"""Spherically windowed dyadic Green's function of the isolated-domain mode
(test infrastructure only, see the package doc).

The isolated-domain form of the method convolves with the free-space dyadic
Green's function truncated to a ball of radius R, whose transform is analytic
(the windowed kernel section, eqs. (13)-(17)):

    F[G_R](k) = A(k) I + B(k) k^ k^,
    A(k) = F[g_R](k) + h(k; R),   B(k) = -F[g_R](k) - 3 h(k; R) - 1 / k_bg^2   (k > 0),
    A(0) = F[g_R](0) + h(0; R),   B(0) = 0,

with g(r) = exp(i k_bg r) / (4 pi r), the windowed scalar transform F[g_R] of
eq. (17), and h(k; R) = 4 pi R^2 g'(R) j1(kR) / (k_bg^2 kR). The printed h has
R where R^2 belongs, and the printed A(0) lacks the factor 4 pi; both readings
are pinned by a radial quadrature of the windowed kernel (tests). With the
corrections, A(0) is the k -> 0 limit of A(k), and B(k) -> 0 there.

Below the kernel: its real-space samples by the oversampled precompute (4x, or
more along an axis where the ball of radius R needs a longer period) and the
isolated-domain apply with padding by 2 on all three axes. None of this is
on the periodic hot path.
"""
from __future__ import annotations

import numpy as np


def _j1_over_x(x):
    """j1(x) / x, with its series below |x| = 1e-3 (the limit at 0 is 1/3)."""
    x = np.asarray(x, dtype=float)
    small = np.abs(x) < 1e-3
    xs = np.where(small, 1.0, x)
    val = (np.sin(xs) / xs - np.cos(xs)) / (xs * xs)
    ser = 1.0 / 3.0 - x * x / 30.0 + x ** 4 / 840.0
    return np.where(small, ser, val)


def g_prime_times_4pi_r2(kbg: complex, R: float) -> complex:
    """4 pi R^2 g'(R) = exp(i k_bg R) (i k_bg R - 1) for g = exp(i k_bg r) / (4 pi r)."""
    return np.exp(1j * kbg * R) * (1j * kbg * R - 1.0)


def window_sphere_scalar(k, kbg: complex, R: float):
    """F[g_R](k) = 4 pi int_0^R g(r) j0(kr) r^2 dr in closed form (eq. (17)).

    k = 0 and the removable point k^2 = k_bg^2 take their limits (the latter
    only arises for a lossless background)."""
    k = np.asarray(k, dtype=float)
    e = np.exp(1j * kbg * R)
    kk = np.where(k == 0.0, 1.0, k)
    den = kbg * kbg - kk * kk
    near = np.abs(den) < 1e-10 * np.abs(kbg * kbg)
    den = np.where(near, 1.0, den)
    gen = (e * (np.cos(kk * R) - 1j * kbg / kk * np.sin(kk * R)) - 1.0) / den
    at0 = (e * (1.0 - 1j * R * kbg) - 1.0) / (kbg * kbg)
    atkb = 1j * R / (2.0 * kbg) - 1j / (2.0 * kbg * kbg) * e * np.sin(kbg * R)
    return np.where(k == 0.0, at0, np.where(near, atkb, gen))


def window_sphere_h(k, kbg: complex, R: float):
    """h(k; R) = 4 pi R^2 g'(R) j1(kR) / (k_bg^2 kR) (the corrected reading of the
    auxiliary function of the windowed kernel)."""
    k = np.asarray(k, dtype=float)
    return g_prime_times_4pi_r2(kbg, R) * _j1_over_x(k * R) / (kbg * kbg)


def window_sphere_AB(k, kbg: complex, R: float):
    """A(k), B(k) of F[G_R](k) = A I + B k^ k^ (k >= 0)."""
    k = np.asarray(k, dtype=float)
    F = window_sphere_scalar(k, kbg, R)
    h = window_sphere_h(k, kbg, R)
    A = F + h
    B = np.where(k == 0.0, 0.0 + 0.0j, -F - 3.0 * h - 1.0 / (kbg * kbg))
    return A, B


def gtilde_isolated(kx, ky, kz, kbg: complex, R: float) -> np.ndarray:
    """F[G_R] at wavevectors (kx, ky, kz): array [..., 3, 3] (symmetric, even in k)."""
    kx, ky, kz = np.broadcast_arrays(np.asarray(kx, float), np.asarray(ky, float), np.asarray(kz, float))
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    A, B = window_sphere_AB(k, kbg, R)
    ks = np.where(k == 0.0, 1.0, k)
    kh = np.stack([kx / ks, ky / ks, kz / ks], axis=-1)
    out = A[..., None, None] * np.eye(3) + B[..., None, None] * kh[..., :, None] * kh[..., None, :]
    return out


def oversampling(shape, spacing, R: float) -> tuple:
    """Per-axis oversampling factor of the kernel precompute: the smallest power
    of two that is at least 4 (the factor the windowed kernel section uses) and
    at least 1 + R / L_a, L_a = n_a h_a. The inverse DFT of samples of F[G_R] at
    spacing 2 pi / P_a has the images of the ball of radius R at multiples of
    the period P_a; the offsets |j| <= L_a that the padded convolution meets
    stay clear of them when P_a >= L_a + R (for a cube with R at the diagonal
    the factor 4 suffices; a flat absorber needs more along its thin axis)."""
    out = []
    for n, h in zip(shape, spacing):
        f = 4
        while f < 1.0 + R / (n * h):
            f *= 2
        out.append(f)
    return tuple(out)


def kernel_samples(shape, spacing, kbg: complex, R: float, over=4) -> np.ndarray:
    """Real-space samples of the windowed dyadic kernel on the lattice offsets of
    a grid of `shape` (nz, ny, nx) with `spacing` (dz, dy, dx): K[j] for every
    offset j in [-n, n) per axis, in FFT order on the 2n grid, shape
    (2nz, 2ny, 2nx, 3, 3).

    The transform F[G_R] is sampled on the grid oversampled `over` times (an int,
    or one factor per axis (z, y, x); period over * n * h per axis; its Nyquist
    planes zeroed), brought to real space by the inverse DFT (divided by
    the cell volume, so that a Riemann sum of K against a density is the
    convolution), and restricted to the offsets a 2n-padded convolution meets
    (the precompute of the truncated-kernel method the windowed kernel section
    cites)."""
    nz, ny, nx = shape
    dz, dy, dx = spacing
    oz, oy, ox = (over, over, over) if np.isscalar(over) else over
    M = (oz * nz, oy * ny, ox * nx)
    kz = 2 * np.pi * np.fft.fftfreq(M[0], d=dz)
    ky = 2 * np.pi * np.fft.fftfreq(M[1], d=dy)
    kx = 2 * np.pi * np.fft.fftfreq(M[2], d=dx)
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    G = gtilde_isolated(KX, KY, KZ, kbg, R)                      # (Mz, My, Mx, 3, 3)
    # the Nyquist planes have no partner of opposite sign, and the off-diagonal
    # entries are odd in each component of k: zeroed, as on the periodic path,
    # so that the samples are exactly even in the offset
    G[M[0] // 2] = 0
    G[:, M[1] // 2] = 0
    G[:, :, M[2] // 2] = 0
    g = np.fft.ifftn(G, axes=(0, 1, 2)) / (dx * dy * dz)          # samples at offsets, FFT order
    iz = np.r_[0:nz, M[0] - nz:M[0]]
    iy = np.r_[0:ny, M[1] - ny:M[1]]
    ix = np.r_[0:nx, M[2] - nx:M[2]]
    return g[np.ix_(iz, iy, ix)]                                   # offsets [-n, n) in FFT order on 2n


def isolated_table(shape, spacing, kbg: complex, R: float, over=4) -> np.ndarray:
    """The kernel of the isolated-domain apply on the 2n grid: the DFT of the
    kernel samples (times the cell volume), shape (2nz, 2ny, 2nx, 3, 3)."""
    dz, dy, dx = spacing
    K = kernel_samples(shape, spacing, kbg, R, over)
    return np.fft.fftn(K, axes=(0, 1, 2)) * (dx * dy * dz)


def apply_isolated(table: np.ndarray, vol: np.ndarray, x: np.ndarray) -> np.ndarray:
    """y = x - P IFFT(table . FFT(Z (vol x))) with Z the zero padding of every axis
    to twice its length and P the restriction back (eq. (18) for an isolated
    scatterer). vol is the potential V per voxel (nz, ny, nx); x is (3, nz, ny, nx)."""
    _, nz, ny, nx = x.shape
    f = np.zeros((3, 2 * nz, 2 * ny, 2 * nx), dtype=complex)
    f[:, :nz, :ny, :nx] = vol[None] * x
    fh = np.fft.fftn(f, axes=(1, 2, 3))
    wh = np.einsum("zyxij,jzyx->izyx", table, fh)
    w = np.fft.ifftn(wh, axes=(1, 2, 3))[:, :nz, :ny, :nx]
    return x - w


def solve_isolated_dense(table: np.ndarray, vol: np.ndarray, b: np.ndarray) -> np.ndarray:
    """u with u - P IFFT(table . FFT(Z (vol u))) = b (eq. (18) for the isolated
    scatterer with right-hand side b): the operator is assembled column by
    column by applying it to unit vectors, then solved by LU. Small grids only
    (3 N unknowns, a dense 3N x 3N matrix)."""
    shape = b.shape
    n = b.size
    A = np.empty((n, n), dtype=complex)
    e = np.zeros(n, dtype=complex)
    for j in range(n):
        e[j] = 1.0
        A[:, j] = apply_isolated(table, vol, e.reshape(shape)).ravel()
        e[j] = 0.0
    return np.linalg.solve(A, b.ravel()).reshape(shape)
