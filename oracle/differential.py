"""Differential PSFD operator with a z-PML (test infrastructure only, see the package doc).

The comparison solver of the paper's preconditioner study (Sec. 3): the curl-curl
equation of the mask field, eq. (8) on the homogeneous background,

    curl curl E - k_bg^2 E - V E = V e_bg,     V = k0^2 delta_eps,

discretised pseudo-spectrally: every derivative is a Fourier derivative along its
axis (eq. (6)), and along z, where the domain is open, the derivative is
stretched inside the perfectly matched layers, d/dz -> (1 / (1 + i s(z))) d/dz
(eq. (7)). The clip is periodic in x and y (Floquet envelopes, as on the main
path); z covers an extended grid of planes, spacing dz, with the absorber (or,
for the full-domain form, the absorber and the multilayer) inside and PML
layers at both ends. Readings, recorded in the design notes:

* planes z_k = (k - z0 + 1/2) dz: the absorber's first plane z0 sits at dz/2, as
  on the main path; z = 0 is the multilayer surface;
* x, y derivatives multiply the envelope spectrum by i (k_x0 + 2 pi m / L_x)
  (i k_y likewise), Nyquist index included; the first z derivative zeroes the
  z-Nyquist wavenumber (the usual odd-derivative choice);
* PML: s(z) = s_max (d / L)^p at depth d of the plane centre into a layer of L =
  n_pml dz, zero outside; s_max = (p + 1) ln(1 / R0) / (2 k_bg L), so that a
  normally incident wave returns with amplitude R0 after a round trip;
* spectral damping (the Table's "spectral damping" preconditioner):
  D(k) = min(1, k_bg^2 / |k|^2) on the full 3-D wavevector (k_x, k_y, kappa),
  applied on the left: D A x = D b; "none": A x = b;
* background-field form (eqs. (8)-(9)): the downgoing mask field at z = 0 is read
  on the plane below the absorber (z = -dz/2) as per-order amplitudes
  a_q = FFT_xy(E)_q exp(-i beta_q dz / 2) / (N_x N_y), the upgoing one on the
  plane above (z = T + dz/2) the same way; E_up = T_R (a_inc + a_dn); the orders
  at z = T are E_up exp(i beta T) + a_up;
* full-domain form (the paper's baseline without the background decomposition):
  the multilayer is on the grid as permittivity (the contrast planes below the
  absorber, built by the input generators), the source is V E_inc with the
  incident wave alone, and the substrate is the background medium.
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np

from . import psfd as P


class DiffSetup:
    """Grid, PML and tables of one differential problem.

    prob: the clip, incidence and multilayer (prob.nz, prob.t_nm: the absorber,
    spacing dz = t / nz); nz_ext planes in z with the contrast region on planes
    [zc0, zc0 + ncz) whose top nz planes are the absorber.
    """

    def __init__(self, prob, nz_ext: int, zc0: int, ncz: int, pml_cells: int, pml_order: int = 3,
                 pml_reflection: float = 1e-8):
        self.S = P.Setup(prob)
        S = self.S
        self.nx, self.ny, self.nz = S.nx, S.ny, S.nz
        self.pe, self.zc0, self.ncz = int(nz_ext), int(zc0), int(ncz)
        self.z0 = self.zc0 + self.ncz - self.nz          # first absorber plane
        self.dz = S.dz
        self.npml = int(pml_cells)
        if not (self.npml + 1 <= self.zc0 and self.z0 + self.nz + 1 <= self.pe - self.npml and self.ncz >= self.nz):
            raise ValueError("the contrast region and one readout plane on each side must lie outside the PML")
        self.z = (np.arange(self.pe) - self.z0 + 0.5) * self.dz
        l = np.rint(np.fft.fftfreq(self.pe) * self.pe).astype(int)
        self.kappa = 2.0 * math.pi * l / (self.pe * self.dz)
        self.kappa_d = np.where(l == -self.pe // 2, 0.0, self.kappa)
        L = self.npml * self.dz
        p = int(pml_order)
        smax = (p + 1) * math.log(1.0 / pml_reflection) / (2.0 * S.kbg * L) if self.npml > 0 else 0.0
        k = np.arange(self.pe)
        depth = np.zeros(self.pe)
        bot = k < self.npml
        top = k >= self.pe - self.npml
        depth[bot] = (self.npml - k[bot] - 0.5) * self.dz
        depth[top] = (k[top] - (self.pe - self.npml) + 0.5) * self.dz
        self.sigma = np.where(bot | top, smax * (depth / max(L, 1e-300)) ** p, 0.0)
        self.inv_s = 1.0 / (1.0 + 1j * self.sigma)
        self.sigma_max = smax
        K2 = (S.KX[None] ** 2 + S.KY[None] ** 2 + self.kappa[:, None, None] ** 2)
        with np.errstate(divide="ignore"):
            self.damp = np.minimum(1.0, np.where(K2 > 0, S.kbg ** 2 / K2, np.inf))


def _dx(D: DiffSetup, f):
    return np.fft.ifft(1j * D.S.kx * np.fft.fft(f, axis=-1), axis=-1)


def _dy(D: DiffSetup, f):
    return np.fft.ifft(1j * D.S.ky[:, None] * np.fft.fft(f, axis=-2), axis=-2)


def _dz(D: DiffSetup, f):
    """Stretched spectral z derivative (eqs. (6)-(7)): (1 / s(z)) IFFT_z(i kappa FFT_z f)."""
    d = np.fft.ifft(1j * D.kappa_d[:, None, None] * np.fft.fft(f, axis=0), axis=0)
    return D.inv_s[:, None, None] * d


def curl(D: DiffSetup, f: np.ndarray) -> np.ndarray:
    """curl f of a field (3, pe, ny, nx) with the pseudo-spectral derivatives."""
    return np.stack([_dy(D, f[2]) - _dz(D, f[1]),
                     _dz(D, f[0]) - _dx(D, f[2]),
                     _dx(D, f[1]) - _dy(D, f[0])])


def potential_ext(D: DiffSetup, deps_c: np.ndarray) -> np.ndarray:
    """V = k0^2 delta_eps on the extended grid, from the contrast planes (ncz, ny, nx)."""
    V = np.zeros((D.pe, D.ny, D.nx), dtype=complex)
    V[D.zc0:D.zc0 + D.ncz] = D.S.vscale * np.asarray(deps_c, dtype=complex)
    return V


def damping(D: DiffSetup, f: np.ndarray) -> np.ndarray:
    """Spectral-damping preconditioner: IFFT_xyz(min(1, k_bg^2 / |k|^2) FFT_xyz f) per component."""
    return np.fft.ifftn(D.damp[None] * np.fft.fftn(f, axes=(1, 2, 3)), axes=(1, 2, 3))


def apply_diff(D: DiffSetup, deps_c: np.ndarray, x: np.ndarray, precond: str = "none") -> np.ndarray:
    """A x = curl curl x - k_bg^2 x - V x, or D A x with precond = "damping"."""
    V = potential_ext(D, deps_c)
    y = curl(D, curl(D, x)) - D.S.kbg ** 2 * x - V[None] * x
    return damping(D, y) if precond == "damping" else y


def rhs(D: DiffSetup, deps_c: np.ndarray, e_src_c: np.ndarray) -> np.ndarray:
    """b = V e on the contrast planes (e: the source field there, (3, ncz, ny, nx))."""
    b = np.zeros((3, D.pe, D.ny, D.nx), dtype=complex)
    b[:, D.zc0:D.zc0 + D.ncz] = D.S.vscale * np.asarray(deps_c)[None] * e_src_c
    return b


def solve_linear(D: DiffSetup, deps_c, b, precond="none", x0=None, rtol=1e-10, restart=30, max_iters=20000,
                 dense=None):
    """GMRES(m) on A x = b ("none") or D A x = D b ("damping"); with `dense` (the
    assembled matrix of A, tiny grids) a direct solve of A x = b instead."""
    if dense is not None:
        x = np.linalg.solve(dense, np.asarray(b).ravel()).reshape(b.shape)
        return x, {"iters": 0, "rel_residual": float(np.linalg.norm(dense @ x.ravel() - b.ravel())
                                                     / max(np.linalg.norm(b), 1e-300))}
    bb = damping(D, b) if precond == "damping" else b
    return P.gmres(lambda v: apply_diff(D, deps_c, v, precond), bb, x0, rtol, restart, max_iters)


def dense_operator(D: DiffSetup, deps_c) -> np.ndarray:
    """A assembled column by column (3 nz_ext ny nx unknowns: tiny grids only)."""
    shape = (3, D.pe, D.ny, D.nx)
    return P.dense_matrix(lambda v: apply_diff(D, deps_c, v), int(np.prod(shape)), shape)


def read_plane(D: DiffSetup, E: np.ndarray, k: int, dist: float) -> np.ndarray:
    """Per-order amplitudes (ny, nx, 3) of the field on plane k, carried over `dist`
    (> 0) away from the sources: FFT_xy(E(z_k))_q exp(-i beta_q dist) / (N_x N_y)."""
    S = D.S
    a = P.spectrum_xy(S, E[:, k])                                    # (3, ny, nx)
    a = np.transpose(a, (1, 2, 0)) * np.exp(-1j * S.beta * dist)[..., None]
    return a * S.keep[..., None]


def solve_background(D: DiffSetup, deps: np.ndarray, precond: str = "none", rtol: float = 1e-10,
                     outer_rtol: Optional[float] = None, restart: int = 30, max_iters: int = 20000,
                     max_outer: int = 200, dense: bool = False) -> Dict:
    """The background-field method with the differential operator (eqs. (8)-(9)):
    outer fixed point over the multilayer reflection around GMRES on the
    curl-curl equation of the mask field; returns E_mask on the extended grid,
    the orders at z = T and the counters."""
    S = D.S
    assert D.ncz == D.nz
    outer_rtol = rtol if outer_rtol is None else outer_rtol
    a_inc = P.incident_down(S)
    a_up = P.reflect(S, a_inc)
    e_inc = P.incident_field(S)
    E = np.zeros((3, D.pe, D.ny, D.nx), dtype=complex)
    Ad = dense_operator(D, deps) if dense else None
    its, change = 0, float("inf")
    for outer in range(1, max_outer + 1):
        e = e_inc + P.inject_up(S, a_up)
        E, info = solve_linear(D, deps, rhs(D, deps, e), precond, E, rtol, restart, max_iters, Ad)
        its += info["iters"]
        a_dn = read_plane(D, E, D.z0 - 1, 0.5 * D.dz)
        a_new = P.reflect(S, a_inc + a_dn)
        nrm = np.linalg.norm(a_new)
        change = np.linalg.norm(a_new - a_up) / nrm if nrm > 0 else 0.0
        a_up = a_new
        if change <= outer_rtol:
            break
    a_mask_up = read_plane(D, E, D.z0 + D.nz, 0.5 * D.dz)
    orders = a_up * np.exp(1j * S.beta * S.t)[..., None] + a_mask_up
    return {"E": E, "emask": E[:, D.z0:D.z0 + D.nz], "orders": orders, "iters": its, "outer_iters": outer,
            "outer_change": change, "rel_residual": info["rel_residual"]}


def solve_full_domain(D: DiffSetup, deps_c: np.ndarray, precond: str = "none", rtol: float = 1e-10,
                      restart: int = 30, max_iters: int = 20000, dense: bool = False) -> Dict:
    """Full-domain PSFD: the multilayer is part of the contrast (planes [zc0, zc0 + ncz)),
    the source is V E_inc, and the reflected orders at z = T are read above the absorber."""
    S = D.S
    e_inc = np.zeros((3, D.ncz, D.ny, D.nx), dtype=complex)
    zc = (np.arange(D.zc0, D.zc0 + D.ncz) - D.z0 + 0.5) * D.dz
    ii, jj = S.inc_order
    b0 = S.beta[jj, ii]
    spec = np.zeros((3, D.ncz, D.ny, D.nx), dtype=complex)
    for c in range(3):
        spec[c, :, jj, ii] = S.e_inc[c] * np.exp(-1j * b0 * zc)
    e_inc = P.field_from_spectrum(S, spec)
    E, info = solve_linear(D, deps_c, rhs(D, deps_c, e_inc), precond, None, rtol, restart, max_iters,
                           dense_operator(D, deps_c) if dense else None)
    orders = read_plane(D, E, D.z0 + D.nz, 0.5 * D.dz)
    return {"E": E, "orders": orders, "iters": info["iters"], "rel_residual": info["rel_residual"]}
