"""Seeded synthetic inputs: mask clips, multilayer stacks and incidence sets.

This module only builds inputs (geometry, material indices, angles). It holds
no part of the solver's arithmetic, so both the HIP path and the CPU oracle can
be fed from it.

The paper's experiments use a Ta absorber on a Mo/Si Bragg reflector
(Sec. 2 and Sec. 3, cuboid and layout experiments) with mask layouts taken
from a public layout dataset that is not available here; the generators below
stand in for those layouts with seeded Manhattan geometry of the same kind
(rectangles snapped to the lateral grid, extruded through the absorber).

Array conventions
-----------------
* Permittivity contrast volumes are complex128 arrays of shape ``(nz, ny, nx)``.
  Voxel ``(k, j, i)`` covers ``x in [i*dx, (i+1)*dx)``, ``y in [j*dy, (j+1)*dy)``
  and ``z in [k*dz, (k+1)*dz)`` with ``z = 0`` the multilayer surface and
  ``z = t`` the top of the absorber.
* A layer stack is a list of ``(eps, thickness_nm)`` from the top down, plus a
  substrate permittivity.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Material indices used by every workload (refractive index n = n' + i n'').
N_ABSORBER = 0.95 + 0.031j
N_MO = 0.92 + 0.0064j
N_SI = 0.999 + 0.0018j

TE, TM = 0, 1


def eps_of(n: complex) -> complex:
    """Relative permittivity of a material with refractive index ``n``."""
    return complex(n) ** 2


def mo_si_stack(n_pairs: int = 40, period_nm: float = 6.9, mo_fraction: float = 0.4,
                n_mo: complex = N_MO, n_si: complex = N_SI) -> Tuple[List[Tuple[complex, float]], complex]:
    """Mo/Si bilayer mirror, Si on top of each pair, on a Si half-space."""
    d_mo = period_nm * mo_fraction
    d_si = period_nm - d_mo
    layers: List[Tuple[complex, float]] = []
    for _ in range(n_pairs):
        layers.append((eps_of(n_si), d_si))
        layers.append((eps_of(n_mo), d_mo))
    return layers, eps_of(n_si)


@dataclasses.dataclass
class Problem:
    """One scattering problem: grid, clip, illumination and layer stack."""
    nx: int
    ny: int
    nz: int
    lx_nm: float
    ly_nm: float
    t_nm: float
    wavelength_nm: float = 13.5
    eps_bg: float = 1.0
    theta_deg: float = 6.0
    phi_deg: float = 0.0
    pol: int = TE
    layers: List[Tuple[complex, float]] = dataclasses.field(default_factory=list)
    eps_sub: complex = 1.0 + 0.0j

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


def _box_mask(nx: int, ny: int, lx: float, ly: float, rects: Sequence[Tuple[float, float, float, float]]) -> np.ndarray:
    """Binary (ny, nx) mask of the union of periodic rectangles (x0, y0, w, h) in nm."""
    dx, dy = lx / nx, ly / ny
    m = np.zeros((ny, nx), dtype=bool)
    for (x0, y0, w, h) in rects:
        i0 = int(round(x0 / dx)); i1 = i0 + max(1, int(round(w / dx)))
        j0 = int(round(y0 / dy)); j1 = j0 + max(1, int(round(h / dy)))
        ii = np.arange(i0, i1) % nx
        jj = np.arange(j0, j1) % ny
        m[np.ix_(jj, ii)] = True
    return m


def extrude(mask2d: np.ndarray, nz: int, n_abs: complex = N_ABSORBER, eps_bg: float = 1.0) -> np.ndarray:
    """Contrast volume: absorber where ``mask2d`` is set, background elsewhere."""
    de = eps_of(n_abs) - eps_bg
    vol = np.where(mask2d, de, 0.0).astype(np.complex128)
    return np.ascontiguousarray(np.broadcast_to(vol, (nz,) + mask2d.shape))


def line_space(nx: int, ny: int, nz: int, lx: float, ly: float, x0: float, x1: float,
               n_abs: complex = N_ABSORBER) -> np.ndarray:
    """y-invariant absorber line covering ``x in [x0, x1)`` nm."""
    return extrude(_box_mask(nx, ny, lx, ly, [(x0, 0.0, x1 - x0, ly)]), nz, n_abs)


def contact_holes(nx: int, ny: int, nz: int, lx: float, ly: float, n_holes: int, seed: int,
                  side_nm: Tuple[float, float] = (20.0, 40.0), n_abs: complex = N_ABSORBER) -> np.ndarray:
    """Dark-field absorber with ``n_holes`` square openings.

    Hole side ~ U[side_nm], snapped to the lateral grid; centres uniform;
    periodic wrap; overlapping holes merge.
    """
    rng = np.random.default_rng(seed)
    dx = lx / nx
    rects = []
    for _ in range(n_holes):
        s = rng.uniform(*side_nm)
        s = max(dx, round(s / dx) * dx)
        cx, cy = rng.uniform(0, lx), rng.uniform(0, ly)
        rects.append((cx - s / 2, cy - s / 2, s, s))
    holes = _box_mask(nx, ny, lx, ly, rects)
    return extrude(~holes, nz, n_abs)


def manhattan(nx: int, ny: int, nz: int, lx: float, ly: float, seed: int,
              n_rect: Tuple[int, int] = (4, 12), n_abs: complex = N_ABSORBER) -> np.ndarray:
    """Random Manhattan clip: union of 4-12 rectangles, sides U[dx, L/2] nm."""
    rng = np.random.default_rng(seed)
    dx, dy = lx / nx, ly / ny
    rects = []
    for _ in range(int(rng.integers(n_rect[0], n_rect[1] + 1))):
        w = max(dx, round(rng.uniform(min(4 * dx, lx / 2), lx / 2) / dx) * dx)
        h = max(dy, round(rng.uniform(min(4 * dy, ly / 2), ly / 2) / dy) * dy)
        rects.append((rng.uniform(0, lx), rng.uniform(0, ly), w, h))
    return extrude(_box_mask(nx, ny, lx, ly, rects), nz, n_abs)


def smooth_density_eps(nx: int, ny: int, nz: int, lx: float, ly: float, t: float, seed: int,
                       sigma_xy_nm: float = 8.0, sigma_z_nm: float = 4.0, slope: float = 4.0,
                       n_abs: complex = N_ABSORBER) -> Tuple[np.ndarray, np.ndarray]:
    """Smooth random absorber: n = 1 + rho (n_abs - 1), rho = sigmoid(slope * s).

    ``s`` is seeded white noise Gaussian-filtered (periodic in x, y; zero-padded
    in z) and scaled to unit standard deviation. Returns ``(delta_eps, rho)``.
    """
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((nz, ny, nx))
    fx = np.fft.fftfreq(nx, d=lx / nx)
    fy = np.fft.fftfreq(ny, d=ly / ny)
    fz = np.fft.fftfreq(2 * nz, d=t / nz)
    gx = np.exp(-2 * (math.pi * sigma_xy_nm * fx) ** 2)
    gy = np.exp(-2 * (math.pi * sigma_xy_nm * fy) ** 2)
    gz = np.exp(-2 * (math.pi * sigma_z_nm * fz) ** 2)
    wp = np.zeros((2 * nz, ny, nx))
    wp[:nz] = w
    s = np.fft.ifftn(np.fft.fftn(wp) * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]).real[:nz]
    s = (s - s.mean()) / s.std()
    rho = 1.0 / (1.0 + np.exp(-slope * s))
    n = 1.0 + rho * (complex(n_abs) - 1.0)
    return (n * n - 1.0).astype(np.complex128), rho


def pupil_angles(na: float = 0.33, mag: float = 4.0, theta0_deg: float = 6.0,
                 sigma_min: float = 0.2, sigma_max: float = 0.9, n: int = 9) -> List[Tuple[float, float]]:
    """Illumination directions (theta_deg, phi_deg) from a 9x9 pupil grid.

    sigma points on linspace(-0.9, 0.9, 9)^2 with 0.2 <= |sigma| <= 0.9 are kept;
    the mask-side direction sine is (sin theta0, 0) + sigma * na / mag.
    """
    out = []
    g = np.linspace(-sigma_max, sigma_max, n)
    for sx in g:
        for sy in g:
            r = math.hypot(sx, sy)
            if r < sigma_min - 1e-12 or r > sigma_max + 1e-12:
                continue
            ux = math.sin(math.radians(theta0_deg)) + sx * na / mag
            uy = sy * na / mag
            st = math.hypot(ux, uy)
            out.append((math.degrees(math.asin(st)), math.degrees(math.atan2(uy, ux))))
    return out


def config_problem(name: str, pol: int = TE, theta_deg: float = 6.0, phi_deg: float = 0.0,
                   n_pairs: int = 40) -> Problem:
    """Grid, clip size and stack of the named workload (no contrast volume)."""
    layers, eps_sub = mo_si_stack(n_pairs)
    sizes = {
        "G1": (32, 32, 32, 64.0),
        "G2": (64, 64, 32, 128.0),
        "G3": (128, 128, 64, 256.0),
        "G4": (256, 256, 64, 512.0),
    }
    nx, ny, nz, l = sizes[name]
    return Problem(nx=nx, ny=ny, nz=nz, lx_nm=l, ly_nm=l, t_nm=60.0, theta_deg=theta_deg,
                   phi_deg=phi_deg, pol=pol, layers=layers, eps_sub=eps_sub)


def random_complex(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """Seeded standard complex Gaussian array (test vectors)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)).astype(dtype)


def manhattan_set(grids: Sequence[str], seed0: int, angles: Sequence[Tuple[float, float]],
                  rng: Optional[np.random.Generator] = None):
    """``(grid, problem, delta_eps)`` per grid name: a pupil angle each and a Manhattan clip.

    The angle of item i is drawn from ``rng`` when given, else it is
    ``angles[(7 i) mod len(angles)]``; the clip of item i has seed ``seed0 + i``.
    """
    items = []
    for i, g in enumerate(grids):
        th, ph = angles[int(rng.integers(len(angles))) if rng is not None else (7 * i) % len(angles)]
        p = config_problem(g, theta_deg=th, phi_deg=ph)
        items.append((g, p, manhattan(p.nx, p.ny, p.nz, p.lx_nm, p.ly_nm, seed=seed0 + i)))
    return items


def batched_set():
    """The 64 batched instances: 64x64x32 and 128x128x64 Manhattan clips alternating,
    pupil angles drawn with seed 3000, clip seeds 3000 + i."""
    return manhattan_set(["G2", "G3"] * 32, 3000, pupil_angles(), np.random.default_rng(3000))


def serving_pool():
    """The 12 requests of the serving pool: 64x64x32, 128x128x64 and 256x256x64 in turn,
    pupil angle (7 i) mod 48, clip seeds 4000 + i."""
    return manhattan_set(["G2", "G3", "G4"] * 4, 4000, pupil_angles(), None)


def headline_clip() -> np.ndarray:
    """The 128x128x64 contact-hole clip of the headline solve (8 holes, seed 2001)."""
    return contact_holes(128, 128, 64, 256.0, 256.0, 8, seed=2001)


def layered_contrast(ncz: int, nz: int, dz: float, layers: Sequence[Tuple[complex, float]], deps_abs: np.ndarray,
                     eps_bg: float = 1.0) -> np.ndarray:
    """Contrast planes (ncz, ny, nx) of a full-domain grid: the multilayer below the
    absorber (each plane takes the layer containing its centre, layers listed from
    the top down, plane spacing dz) under the absorber's own nz planes on top."""
    ny, nx = deps_abs.shape[1:]
    out = np.zeros((ncz, ny, nx), dtype=np.complex128)
    nl = ncz - nz
    bounds = np.cumsum([0.0] + [float(d) for _, d in layers])      # depth below the absorber
    for k in range(nl):
        depth = (nl - k - 0.5) * dz
        i = int(np.searchsorted(bounds, depth, side="right")) - 1
        if 0 <= i < len(layers):
            out[k] = complex(layers[i][0]) - eps_bg
    out[nl:] = deps_abs
    return out


def cuboid(nx: int, ny: int, nz: int, lx: float, ly: float, wx: float, wy: float,
           n_abs: complex = N_ABSORBER) -> np.ndarray:
    """A single absorber block wx x wy nm centred on the clip, through the absorber."""
    return extrude(_box_mask(nx, ny, lx, ly, [((lx - wx) / 2, (ly - wy) / 2, wx, wy)]), nz, n_abs)
