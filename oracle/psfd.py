"""Plain FP64 reference implementation (test infrastructure only, see package doc).

Conventions (the paper fixes the physics; the discrete choices below are the
readings recorded in the design notes):

* time dependence exp(-i w t); absorbing media have Im n > 0;
  k0 = 2 pi / wavelength, k_bg = k0 sqrt(eps_bg), V = k0^2 (eps - eps_bg)
  (the w^2 mu factor of eq. (1) with relative permittivities).
* x, y periodic with Floquet (Bloch) phase; the unknowns are envelopes
  u = E exp(-i (kx0 x + ky0 y)), sample (j, i) at x = i dx, y = j dy.
* z covers the absorber [0, T] (z = 0 is the multilayer surface) with
  cell-centred planes z_k = (k + 1/2) dz, zero padded to Pz = 2 Nz for the
  z convolution (eq. (18) and the padding remark after it).
* transverse orders in FFT order: kx_m = kx0 + 2 pi m / Lx, likewise y;
  beta = sqrt(k_bg^2 - kt^2) with Im beta >= 0.
* FFTs are unnormalised forward / 1/M inverse (NumPy), so
  IFFT(G ~ FFT(f)) is the Riemann-sum convolution int G(r - r') f(r') dr'.
"""
from __future__ import annotations

import math
from typing import Dict, Optional, Sequence, Tuple

import numpy as np
import scipy.fft as sfft

WORKERS = 1  # scipy.fft worker threads


def set_workers(n: int) -> None:
    global WORKERS
    WORKERS = int(max(1, n))


def _fftn(a, axes):
    return sfft.fftn(a, axes=axes, workers=WORKERS)


def _ifftn(a, axes):
    return sfft.ifftn(a, axes=axes, workers=WORKERS)


# ---------------------------------------------------------------------------
# Branch of the longitudinal wavenumber
# ---------------------------------------------------------------------------

def kz_branch(kz2) -> np.ndarray:
    """sqrt(kz2) on the branch Im >= 0 (Re >= 0 on the real axis).

    This is the outgoing / decaying choice required by the radiation condition
    attached to eq. (1).
    """
    r = np.sqrt(np.asarray(kz2, dtype=np.complex128))
    flip = (r.imag < 0) | ((r.imag == 0) & (r.real < 0))
    return np.where(flip, -r, r)


# ---------------------------------------------------------------------------
# Layered stack: generalized reflection coefficients (Sec. 2, reflection
# operator of eq. (3); Sec. 3, eq. (9) uses T_R built from them)
# ---------------------------------------------------------------------------

def fresnel(kzi, kzj, epsi, epsj, pol: int):
    """Single-interface reflection from region i into region j.

    TE: ratio of reflected to incident E (tangential E continuous);
    TM: ratio of reflected to incident H (tangential H continuous).
    """
    if pol == 0:
        return (kzi - kzj) / (kzi + kzj)
    return (epsj * kzi - epsi * kzj) / (epsj * kzi + epsi * kzj)


def generalized_reflection(k0: float, eps_top, layers: Sequence[Tuple[complex, float]], eps_sub,
                           kt, pol: int) -> np.ndarray:
    """Recursive generalized reflection coefficient of the stack at its top surface.

    Regions: 0 = medium above the stack (eps_top), 1..N = layers (top down),
    N+1 = substrate half-space. Starting from the bottom interface, each step
    folds the layer below into the reflection seen from the layer above, with
    the round trip phase exp(2 i kz d) of that layer.
    """
    kt = np.asarray(kt, dtype=np.float64)
    eps = [complex(eps_top)] + [complex(e) for e, _ in layers] + [complex(eps_sub)]
    thick = [0.0] + [float(d) for _, d in layers] + [0.0]
    kz = [kz_branch(k0 * k0 * e - kt * kt) for e in eps]
    nreg = len(eps)
    rt = fresnel(kz[nreg - 2], kz[nreg - 1], eps[nreg - 2], eps[nreg - 1], pol)
    for i in range(nreg - 3, -1, -1):
        r = fresnel(kz[i], kz[i + 1], eps[i], eps[i + 1], pol)
        ph = np.exp(2j * kz[i + 1] * thick[i + 1])
        rt = (r + rt * ph) / (1.0 + r * rt * ph)
    return rt


# ---------------------------------------------------------------------------
# Windowed dyadic Green's function, xy-periodic clip, window |z| < L
# (eqs. (13)-(17) specialised to the periodic clip: reading R1/R2/O4)
# ---------------------------------------------------------------------------

def window_scalar(beta, kappa, L, sgn):
    """z-windowed transform of the 1-D scalar kernel i exp(i beta |z|) / (2 beta).

    F = (s exp(i beta L) - 1) / (beta^2 - kappa^2) with s = exp(i kappa L) = +-1.
    Near the resonance kappa = +-beta the removable singularity is evaluated
    through its Taylor series F = L (i - u/2 - i u^2/6) / (beta + |kappa|),
    u = (beta - |kappa|) L, which at u = 0 is the limit i L / (2 beta).
    """
    beta = np.asarray(beta, dtype=np.complex128)
    kappa = np.asarray(kappa, dtype=np.float64)
    beta, kappa, sgn = np.broadcast_arrays(beta, kappa, np.asarray(sgn, dtype=np.float64))
    num = sgn * np.exp(1j * beta * L) - 1.0
    den = beta * beta - kappa * kappa
    akap = np.abs(kappa)
    u = (beta - akap) * L
    near = np.abs(u) < 1e-6
    with np.errstate(divide="ignore", invalid="ignore"):
        f = num / den
    series = L * (1j - u / 2 - 1j * u * u / 6) / (beta + akap)
    return np.where(near, series, f)


def gtilde_periodic(kx, ky, kappa, beta, kbg, L, sgn) -> np.ndarray:
    """F[G_L](k): windowed dyadic kernel at k = (kx, ky, kappa), shape (..., 3, 3).

    From the dyadic/scalar relation eq. (14), G = (I + grad grad / k_bg^2) g,
    transformed over the window |z| < L with the transverse dependence exact:
    G~ = F (I - k k^T / k_bg^2) - (s exp(i beta L) / k_bg^2) z z^T,
    where the last term is the boundary term of the zz second derivative (the
    zz entry equals (kt^2 / k_bg^2) F - 1 / k_bg^2, which contains the local
    -delta(z) / k_bg^2 part of the dyadic kernel).
    """
    F = window_scalar(beta, kappa, L, sgn)
    kx, ky, kappa, F, sgn_b, beta_b = np.broadcast_arrays(
        np.asarray(kx, float), np.asarray(ky, float), np.asarray(kappa, float), F,
        np.asarray(sgn, float), np.asarray(beta, complex))
    kv = [kx, ky, kappa]
    out = np.empty(F.shape + (3, 3), dtype=np.complex128)
    k2 = kbg * kbg
    for i in range(3):
        for j in range(3):
            out[..., i, j] = F * ((1.0 if i == j else 0.0) - kv[i] * kv[j] / k2)
    out[..., 2, 2] -= sgn_b * np.exp(1j * beta_b * L) / k2
    return out


# ---------------------------------------------------------------------------
# Problem setup: grids, orders, kernel table, reflection matrices
# ---------------------------------------------------------------------------

class Setup:
    """All FP64 tables of one problem (grid, orders, T_R, kernel, incidence)."""

    def __init__(self, prob, inc_order: Tuple[int, int] = (0, 0), nyquist_zero: bool = True):
        self.prob = prob
        nx, ny, nz = int(prob.nx), int(prob.ny), int(prob.nz)
        self.nx, self.ny, self.nz = nx, ny, nz
        self.lx, self.ly, self.t = float(prob.lx_nm), float(prob.ly_nm), float(prob.t_nm)
        self.k0 = 2.0 * math.pi / float(prob.wavelength_nm)
        eps_bg = float(prob.eps_bg)
        self.eps_bg = eps_bg
        self.kbg = self.k0 * math.sqrt(eps_bg)
        th, ph = math.radians(float(prob.theta_deg)), math.radians(float(prob.phi_deg))
        self.phi = ph
        self.kx0 = self.kbg * math.sin(th) * math.cos(ph)
        self.ky0 = self.kbg * math.sin(th) * math.sin(ph)
        self.m = np.rint(np.fft.fftfreq(nx) * nx).astype(int)
        self.n = np.rint(np.fft.fftfreq(ny) * ny).astype(int)
        self.kx = self.kx0 + 2.0 * math.pi * self.m / self.lx          # (nx,)
        self.ky = self.ky0 + 2.0 * math.pi * self.n / self.ly          # (ny,)
        self.KX = np.broadcast_to(self.kx[None, :], (ny, nx)).copy()
        self.KY = np.broadcast_to(self.ky[:, None], (ny, nx)).copy()
        self.kt = np.hypot(self.KX, self.KY)
        self.beta = kz_branch(self.kbg ** 2 - self.kt ** 2)          # (ny, nx)
        if np.any(np.abs(self.beta) < 1e-6 * self.kbg):
            raise ValueError("Wood anomaly: an order grazes (beta = 0)")
        keep = np.ones((ny, nx), dtype=bool)
        if nyquist_zero:
            if nx % 2 == 0 and nx > 1:
                keep[:, self.m == -nx // 2] = False
            if ny % 2 == 0 and ny > 1:
                keep[self.n == -ny // 2, :] = False
        self.keep = keep
        self.dz = self.t / nz
        self.z = (np.arange(nz) + 0.5) * self.dz
        self.pz = 2 * nz
        self.L = self.t
        self.l = np.rint(np.fft.fftfreq(self.pz) * self.pz).astype(int)
        self.kappa = 2.0 * math.pi * self.l / (self.pz * self.dz)
        self.sgn = np.where(self.l % 2 == 0, 1.0, -1.0)
        self.vscale = self.k0 ** 2
        # polarisation basis per order (bilinear, valid for evanescent orders)
        s = np.zeros((ny, nx, 3))
        with np.errstate(divide="ignore", invalid="ignore"):
            s[..., 0] = np.where(self.kt > 0, -self.KY / self.kt, -math.sin(ph))
            s[..., 1] = np.where(self.kt > 0, self.KX / self.kt, math.cos(ph))
        self.s_hat = s.astype(np.complex128)
        kp = np.stack([self.KX + 0j, self.KY + 0j, self.beta], axis=-1)
        km = np.stack([self.KX + 0j, self.KY + 0j, -self.beta], axis=-1)
        self.k_plus, self.k_minus = kp, km
        self.p_plus = np.cross(kp, self.s_hat) / self.kbg
        self.p_minus = np.cross(km, self.s_hat) / self.kbg
        self.rs = generalized_reflection(self.k0, eps_bg, prob.layers, prob.eps_sub, self.kt, 0)
        self.rp = generalized_reflection(self.k0, eps_bg, prob.layers, prob.eps_sub, self.kt, 1)
        TR = (self.rs[..., None, None] * self.s_hat[..., :, None] * self.s_hat[..., None, :]
              + self.rp[..., None, None] * self.p_plus[..., :, None] * self.p_minus[..., None, :])
        self.TR = TR * keep[..., None, None]
        eye = np.eye(3)
        self.P_minus = eye - km[..., :, None] * km[..., None, :] / self.kbg ** 2
        self.P_plus = eye - kp[..., :, None] * kp[..., None, :] / self.kbg ** 2
        # incidence (unit amplitude at z = 0, downgoing, in order inc_order)
        self.inc_order = (int(inc_order[0]) % nx, int(inc_order[1]) % ny)
        ii, jj = self.inc_order
        if int(prob.pol) == 0:
            self.e_inc = self.s_hat[jj, ii].copy()
        else:
            self.e_inc = self.p_minus[jj, ii].copy()
        self._G = None

    # -- kernel table ------------------------------------------------------
    @property
    def G(self) -> np.ndarray:
        """F[G_L] on the padded grid, shape (pz, ny, nx, 3, 3).

        Orders on the x- or y-Nyquist index are zeroed (reading R5); on the
        z-Nyquist plane the entries odd in kappa (xz, yz) are zeroed so that
        the table is exactly even in k, i.e. the operator is reciprocal.
        """
        if self._G is None:
            kap = self.kappa[:, None, None]
            G = gtilde_periodic(self.KX[None], self.KY[None], kap, self.beta[None], self.kbg,
                                self.L, self.sgn[:, None, None])
            nyqz = self.l == -self.pz // 2
            for (a, b) in ((0, 2), (2, 0), (1, 2), (2, 1)):
                G[nyqz, :, :, a, b] = 0.0
            G *= self.keep[None, :, :, None, None]
            self._G = G
        return self._G


# ---------------------------------------------------------------------------
# Operators on envelope fields f[c, z, y, x] (complex128, shape (3, nz, ny, nx))
# ---------------------------------------------------------------------------

def potential(S: Setup, deps: np.ndarray) -> np.ndarray:
    """V = k0^2 delta_eps per voxel (the diagonal mask potential of eq. (10))."""
    return S.vscale * np.asarray(deps, dtype=np.complex128)


def conv_K(S: Setup, f: np.ndarray, transpose: bool = False) -> np.ndarray:
    """K f = P IFFT_xyz(F[G_L] . FFT_xyz(Z f)), the convolution of eq. (18).

    Z pads z to Pz = 2 Nz with zeros, P keeps the Nz physical planes. The
    bilinear transpose is P FFT(F[G_L] . IFFT(Z f)) (the DFT matrix is
    symmetric and F[G_L] is a symmetric 3x3 per k).
    """
    nz = S.nz
    fp = np.zeros((3, S.pz, S.ny, S.nx), dtype=np.complex128)
    fp[:, :nz] = f
    F = _ifftn(fp, (1, 2, 3)) if transpose else _fftn(fp, (1, 2, 3))
    G = S.G
    out = np.empty_like(F)
    for i in range(3):
        out[i] = G[..., i, 0] * F[0] + G[..., i, 1] * F[1] + G[..., i, 2] * F[2]
    out = _fftn(out, (1, 2, 3)) if transpose else _ifftn(out, (1, 2, 3))
    return out[:, :nz]


def apply_A(S: Setup, deps: np.ndarray, x: np.ndarray, transpose: bool = False) -> np.ndarray:
    """Left side of eq. (18): x - K(V x)  (with K^T for the transposed system)."""
    V = potential(S, deps)
    return x - conv_K(S, V[None] * x, transpose)


def spectrum_xy(S: Setup, f: np.ndarray) -> np.ndarray:
    """Normalised transverse Fourier coefficients per plane: FFT_xy(f) / (Nx Ny)."""
    return _fftn(f, (-2, -1)) / (S.nx * S.ny)


def field_from_spectrum(S: Setup, a: np.ndarray) -> np.ndarray:
    """Inverse of spectrum_xy: sum over orders of a_q exp(i G_q . rho)."""
    return _ifftn(a, (-2, -1)) * (S.nx * S.ny)


def read_down(S: Setup, f: np.ndarray) -> np.ndarray:
    """Downgoing order amplitudes at z = 0 radiated by the source density f.

    Plane-wave form of the dyadic kernel below the sources:
    a_q = (i dz / (2 beta_q)) P-_q sum_k exp(i beta_q z_k) f^_q(z_k),
    the midpoint rule over the cell-centred planes. This is E_mask(z_top) of
    eq. (9) in the transverse Fourier domain. Shape (ny, nx, 3).
    """
    fh = spectrum_xy(S, f)                                   # (3, nz, ny, nx)
    ph = np.exp(1j * S.beta[None] * S.z[:, None, None])      # (nz, ny, nx)
    acc = np.einsum("kyx,ckyx->yxc", ph, fh) * (1j * S.dz / (2 * S.beta))[..., None]
    a = np.einsum("yxij,yxj->yxi", S.P_minus, acc)
    return a * S.keep[..., None]


def read_up(S: Setup, f: np.ndarray) -> np.ndarray:
    """Upgoing order amplitudes at z = T radiated by the source density f."""
    fh = spectrum_xy(S, f)
    ph = np.exp(1j * S.beta[None] * (S.t - S.z)[:, None, None])
    acc = np.einsum("kyx,ckyx->yxc", ph, fh) * (1j * S.dz / (2 * S.beta))[..., None]
    a = np.einsum("yxij,yxj->yxi", S.P_plus, acc)
    return a * S.keep[..., None]


def inject_up(S: Setup, a: np.ndarray) -> np.ndarray:
    """Upgoing plane waves with amplitudes a_q at z = 0, sampled on the planes.

    This is the volume field of eq. (9): IFFT_xy of the per-order amplitude
    times exp(i k_z (z - z_top)), the propagation applied per order.
    """
    ph = np.exp(1j * S.beta[None] * S.z[:, None, None])      # (nz, ny, nx)
    spec = np.transpose(a, (2, 0, 1))[:, None] * ph[None]   # (3, nz, ny, nx)
    return field_from_spectrum(S, spec)


def reflect(S: Setup, a_dn: np.ndarray) -> np.ndarray:
    """Per-order reflection T_R . a (T_R = r_s s s^T + r_p p+ p-^T)."""
    return np.einsum("yxij,yxj->yxi", S.TR, a_dn)


def incident_field(S: Setup) -> np.ndarray:
    """Unit downgoing plane wave in order inc_order, envelope on the grid."""
    ii, jj = S.inc_order
    spec = np.zeros((3, S.nz, S.ny, S.nx), dtype=np.complex128)
    b = S.beta[jj, ii]
    for c in range(3):
        spec[c, :, jj, ii] = S.e_inc[c] * np.exp(-1j * b * S.z)
    return field_from_spectrum(S, spec)


def incident_down(S: Setup) -> np.ndarray:
    """Order amplitudes of the incident wave at z = 0."""
    a = np.zeros((S.ny, S.nx, 3), dtype=np.complex128)
    ii, jj = S.inc_order
    a[jj, ii] = S.e_inc
    return a


def apply_M(S: Setup, f: np.ndarray) -> np.ndarray:
    """M f = K f + R_vol T_R K_top f: free-space plus layered-stack response."""
    return conv_K(S, f) + inject_up(S, reflect(S, read_down(S, f)))


def background_field(S: Setup) -> np.ndarray:
    """e_bg = E_inc + R[E_inc]: incident plus its multilayer reflection."""
    return incident_field(S) + inject_up(S, reflect(S, incident_down(S)))


def apply_monolithic(S: Setup, deps: np.ndarray, u: np.ndarray) -> np.ndarray:
    """(I - M V) u for the total field u in the slab (eq. (3) with eqs. (11)-(12))."""
    V = potential(S, deps)
    return u - apply_M(S, V[None] * u)


# ---------------------------------------------------------------------------
# GMRES(m) with modified Gram-Schmidt and Givens rotations (Saad & Schultz)
# ---------------------------------------------------------------------------

def gmres(matvec, b: np.ndarray, x0: Optional[np.ndarray] = None, rtol: float = 1e-8,
          restart: int = 30, max_iters: int = 10000) -> Tuple[np.ndarray, Dict]:
    """Restarted GMRES on a complex system; stops at ||b - A x|| <= rtol ||b||."""
    shape = b.shape
    bv = b.reshape(-1)
    x = np.zeros_like(bv) if x0 is None else x0.reshape(-1).astype(np.complex128).copy()
    bnorm = np.linalg.norm(bv)
    hist = []
    its = 0
    if bnorm == 0.0:
        return np.zeros(shape, dtype=np.complex128), {"iters": 0, "rel_residual": 0.0, "history": hist}

    def mv(v):
        return matvec(v.reshape(shape)).reshape(-1)

    r = bv - mv(x)
    rnorm = np.linalg.norm(r)
    while True:
        hist.append(rnorm / bnorm)
        if rnorm <= rtol * bnorm or its >= max_iters:
            break
        m = restart
        Vb = np.zeros((m + 1, bv.size), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.float64)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = rnorm
        Vb[0] = r / rnorm
        j_used = 0
        for j in range(m):
            w = mv(Vb[j])
            its += 1
            for i in range(j + 1):
                H[i, j] = np.vdot(Vb[i], w)
                w = w - H[i, j] * Vb[i]
            H[j + 1, j] = np.linalg.norm(w)
            for i in range(j):
                a, bb = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * bb
                H[i + 1, j] = -np.conj(sn[i]) * a + cs[i] * bb
            a, bb = H[j, j], H[j + 1, j]
            den = math.hypot(abs(a), abs(bb))
            if abs(a) == 0.0:
                cs[j], sn[j] = 0.0, 1.0
            else:
                cs[j] = abs(a) / den
                sn[j] = (a / abs(a)) * np.conj(bb) / den
            H[j, j] = cs[j] * a + sn[j] * bb
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            j_used = j + 1
            if abs(H[j + 1, j]) == 0.0 and den == 0.0:
                break
            nrm = np.linalg.norm(w)
            if nrm > 0:
                Vb[j + 1] = w / nrm
            if abs(g[j + 1]) <= rtol * bnorm or its >= max_iters or nrm == 0:
                break
        k = j_used
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + y @ Vb[:k]
        r = bv - mv(x)
        rnorm = np.linalg.norm(r)
    return x.reshape(shape), {"iters": its, "rel_residual": rnorm / bnorm, "history": hist}


# ---------------------------------------------------------------------------
# Forward solve: outer fixed-point loop over the reflection (eqs. (8)-(9))
# around the Lippmann-Schwinger solve (eq. (18))
# ---------------------------------------------------------------------------

def solve(prob, deps: np.ndarray, rtol: float = 1e-8, outer_rtol: Optional[float] = None,
          restart: int = 30, max_iters: int = 20000, max_outer: int = 100,
          inc_order: Tuple[int, int] = (0, 0), S: Optional[Setup] = None) -> Dict:
    """Background-field LS solve. Returns fields, order amplitudes and counters.

    Outer step i: E_up = T_R (E_inc + E_mask^(i-1))(z_top) per order; the
    layered field E_layer = R_vol E_up; solve eq. (18)
    x - K V x = K V (E_inc + E_layer) for x = E_mask (warm started); update the
    downgoing mask field at z_top; stop when the relative change of E_up is at
    most outer_rtol. E_mask^(0) = 0.
    """
    if S is None:
        S = Setup(prob, inc_order)
    if outer_rtol is None:
        outer_rtol = rtol
    deps = np.asarray(deps, dtype=np.complex128)
    V = potential(S, deps)
    e_inc = incident_field(S)
    a_inc = incident_down(S)
    a_mask_dn = np.zeros_like(a_inc)
    a_up = reflect(S, a_inc + a_mask_dn)
    x = np.zeros((3, S.nz, S.ny, S.nx), dtype=np.complex128)
    total_its, outer, change = 0, 0, float("inf")
    for outer in range(1, max_outer + 1):
        e = e_inc + inject_up(S, a_up)
        rhs = conv_K(S, V[None] * e)
        x, info = gmres(lambda v: apply_A(S, deps, v), rhs, x, rtol, restart, max_iters)
        total_its += info["iters"]
        u = e + x
        a_mask_dn = read_down(S, V[None] * u)
        a_up_new = reflect(S, a_inc + a_mask_dn)
        nrm = np.linalg.norm(a_up_new)
        change = np.linalg.norm(a_up_new - a_up) / nrm if nrm > 0 else 0.0
        a_up = a_up_new
        if change <= outer_rtol:
            break
    e_layer = inject_up(S, a_up)
    u = e_inc + e_layer + x
    orders = reflected_orders(S, deps, u, a_up)
    mono = apply_monolithic(S, deps, u)
    ebg = background_field(S)
    return {
        "emask": x, "u": u, "e_layer": e_layer, "a_up": a_up, "a_dn": a_inc + a_mask_dn,
        "orders": orders, "iters": total_its, "outer_iters": outer, "outer_change": change,
        "rel_residual": info["rel_residual"],
        "mono_residual": np.linalg.norm(mono - ebg) / np.linalg.norm(ebg), "setup": S,
    }


def reflected_orders(S: Setup, deps: np.ndarray, u: np.ndarray, a_up: np.ndarray) -> np.ndarray:
    """Total upgoing order amplitudes at z = T, shape (ny, nx, 3).

    a_q = E_up,q exp(i beta_q T) + (upgoing mask field at T)_q, with E_up the
    layered-stack reflection at z = 0 and the mask part radiated by V u.
    """
    V = potential(S, deps)
    return a_up * np.exp(1j * S.beta * S.t)[..., None] + read_up(S, V[None] * u)


def transmitted_down(S: Setup, deps: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Downgoing order amplitudes at z = 0 (incident plus mask scattering)."""
    V = potential(S, deps)
    return incident_down(S) + read_down(S, V[None] * u)


def efficiencies(S: Setup, a: np.ndarray) -> np.ndarray:
    """eta_q = ||a_q||^2 Re beta_q / Re beta_inc (power per order)."""
    ii, jj = S.inc_order
    return np.sum(np.abs(a) ** 2, axis=-1) * S.beta.real / S.beta[jj, ii].real


# ---------------------------------------------------------------------------
# Dense references for tiny grids
# ---------------------------------------------------------------------------

def dense_matrix(op, n3: int, shape) -> np.ndarray:
    """Assemble a linear operator column by column from unit vectors."""
    A = np.zeros((n3, n3), dtype=np.complex128)
    e = np.zeros(n3, dtype=np.complex128)
    for j in range(n3):
        e[:] = 0
        e[j] = 1
        A[:, j] = op(e.reshape(shape)).reshape(-1)
    return A


def dense_solve_monolithic(prob, deps: np.ndarray, inc_order=(0, 0)) -> Dict:
    """Direct solve of (I - M V) u = e_bg, the fixed point of the outer loop."""
    S = Setup(prob, inc_order)
    shape = (3, S.nz, S.ny, S.nx)
    n3 = int(np.prod(shape))
    A = dense_matrix(lambda v: apply_monolithic(S, deps, v), n3, shape)
    ebg = background_field(S)
    u = np.linalg.solve(A, ebg.reshape(-1)).reshape(shape)
    return {"u": u, "A": A, "setup": S}


# ---------------------------------------------------------------------------
# Adjoint: gradient of J = sum_{q in Q} ||a_q||^2 with respect to delta_eps
# ---------------------------------------------------------------------------

def read_down_T(S: Setup, a: np.ndarray) -> np.ndarray:
    """Bilinear transpose of read_down: order amplitudes -> source density."""
    b = np.einsum("yxji,yxj->yxi", S.P_minus, a * S.keep[..., None])
    b = b * (1j * S.dz / (2 * S.beta))[..., None]
    ph = np.exp(1j * S.beta[None] * S.z[:, None, None])
    spec = np.transpose(b, (2, 0, 1))[:, None] * ph[None]   # (3, nz, ny, nx)
    # transpose of FFT_xy / (NxNy) is FFT_xy / (NxNy) (symmetric DFT matrix)
    return _fftn(spec, (-2, -1)) / (S.nx * S.ny)


def read_up_T(S: Setup, a: np.ndarray) -> np.ndarray:
    b = np.einsum("yxji,yxj->yxi", S.P_plus, a * S.keep[..., None])
    b = b * (1j * S.dz / (2 * S.beta))[..., None]
    ph = np.exp(1j * S.beta[None] * (S.t - S.z)[:, None, None])
    spec = np.transpose(b, (2, 0, 1))[:, None] * ph[None]
    return _fftn(spec, (-2, -1)) / (S.nx * S.ny)


def inject_up_T(S: Setup, f: np.ndarray) -> np.ndarray:
    """Bilinear transpose of inject_up: field -> order amplitudes."""
    # transpose of (NxNy) IFFT_xy is (NxNy) IFFT_xy
    spec = _ifftn(f, (-2, -1)) * (S.nx * S.ny)
    ph = np.exp(1j * S.beta[None] * S.z[:, None, None])
    return np.einsum("kyx,ckyx->yxc", ph, spec)


def reflect_T(S: Setup, a: np.ndarray) -> np.ndarray:
    return np.einsum("yxji,yxj->yxi", S.TR, a)


def apply_M_T(S: Setup, f: np.ndarray) -> np.ndarray:
    """M^T f = K^T f + K_top^T T_R^T R_vol^T f."""
    return conv_K(S, f, transpose=True) + read_down_T(S, reflect_T(S, inject_up_T(S, f)))


def readout_T(S: Setup, c: np.ndarray) -> np.ndarray:
    """W^T c for the readout a = c0 + W V u, W = diag(e^{i beta T}) T_R K_top + K_up."""
    ph = np.exp(1j * S.beta * S.t)[..., None]
    return read_down_T(S, reflect_T(S, ph * c)) + read_up_T(S, c)


def order_mask(S: Setup, orders: Sequence[Tuple[int, int]]) -> np.ndarray:
    msk = np.zeros((S.ny, S.nx), dtype=bool)
    for (m, n) in orders:
        msk[n % S.ny, m % S.nx] = True
    return msk


def objective(S: Setup, a: np.ndarray, orders: Sequence[Tuple[int, int]]) -> float:
    """J = sum over the selected orders of ||a_q||^2 (Cartesian components)."""
    return float(np.sum(np.abs(a[order_mask(S, orders)]) ** 2))


def adjoint_gradient(prob, deps: np.ndarray, orders: Sequence[Tuple[int, int]],
                     fwd: Optional[Dict] = None, rtol: float = 1e-10, restart: int = 30,
                     max_iters: int = 20000, max_outer: int = 200) -> Dict:
    """Gradient of J with respect to delta_eps (torch convention dJ/dRe + i dJ/dIm).

    lambda solves (I - M^T V) lambda = W^T conj(dJ/da) with the outer splitting
    (I - K^T V) lambda^(i) = s + K_top^T T_R^T R_vol^T V lambda^(i-1);
    dJ = 2 Re sum_r k0^2 d(delta_eps) sum_c lambda_c u_c, so the torch gradient
    is 2 conj(k0^2 sum_c lambda_c u_c).
    """
    if fwd is None:
        fwd = solve(prob, deps, rtol=rtol, restart=restart, max_iters=max_iters)
    S = fwd["setup"]
    deps = np.asarray(deps, dtype=np.complex128)
    V = potential(S, deps)
    u = fwd["u"]
    a = fwd["orders"]
    msk = order_mask(S, orders)
    c = np.where(msk[..., None], np.conj(a), 0.0)
    s = readout_T(S, c)
    lam = np.zeros_like(u)
    couple = np.zeros_like(u)
    its = 0
    for outer in range(1, max_outer + 1):
        rhs = s + couple
        lam, info = gmres(lambda v: apply_A(S, deps, v, transpose=True), rhs, lam, rtol, restart, max_iters)
        its += info["iters"]
        new = read_down_T(S, reflect_T(S, inject_up_T(S, V[None] * lam)))
        ch = np.linalg.norm(new - couple) / max(np.linalg.norm(new), 1e-300)
        couple = new
        if ch <= rtol:
            break
    g = S.vscale * np.sum(lam * u, axis=0)
    return {"grad": 2.0 * np.conj(g), "lam": lam, "J": objective(S, a, orders), "iters": its,
            "outer_iters": outer, "fwd": fwd}


def order_vjp(prob, deps: np.ndarray, grad_orders: np.ndarray, u: Optional[np.ndarray] = None,
              rtol: float = 1e-10, restart: int = 30, max_iters: int = 20000) -> Dict:
    """Vector-Jacobian product of the reflected orders a(delta_eps) for any real loss L(a).

    grad_orders = dL/dRe a + i dL/dIm a, shape (ny, nx, 3) (PyTorch's convention for
    complex tensors). The orders a = c0 + W V u are holomorphic in delta_eps, with u
    the total field of the monolithic system (I - M V) u = e_bg (eqs. (3), (8)-(9),
    (18)); so dL = Re sum_q conj(G_q) . da_q and, by the push-through identity,
    da = W (I - V M)^{-1} dV u. With lambda = (I - M^T V)^{-1} W^T conj(G),
    dL = Re sum_r k0^2 d(delta_eps)(r) sum_c lambda_c u_c, and the gradient in the
    same convention is conj(k0^2 sum_c lambda_c u_c). u (the forward total field)
    is solved for when not given. Returns grad, lambda, u and the GMRES counters.
    """
    S = Setup(prob)
    deps = np.asarray(deps, dtype=np.complex128)
    V = potential(S, deps)
    its_fwd = 0
    if u is None:
        u, fi = gmres(lambda v: apply_monolithic(S, deps, v), background_field(S), None, rtol, restart, max_iters)
        its_fwd = fi["iters"]
    s = readout_T(S, np.conj(np.asarray(grad_orders, dtype=np.complex128)))
    lam, info = gmres(lambda v: v - apply_M_T(S, V[None] * v), s, None, rtol, restart, max_iters)
    g = S.vscale * np.sum(lam * u, axis=0)
    return {"grad": np.conj(g), "lam": lam, "u": u, "iters_fwd": its_fwd, "iters_adj": info["iters"],
            "rel_residual_adj": info["rel_residual"], "setup": S}


def orders_of_total_field(S: Setup, deps: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Reflected orders at z = T of a total field u in the slab: the layered-stack
    reflection of the downgoing field at z = 0 propagated to T, plus the upgoing
    mask field (eq. (9) and its readouts)."""
    V = potential(S, deps)
    a_up = reflect(S, incident_down(S) + read_down(S, V[None] * u))
    return reflected_orders(S, deps, u, a_up)


def solve_monolithic(prob, deps: np.ndarray, rtol: float = 1e-10, restart: int = 30,
                     max_iters: int = 20000) -> Dict:
    """GMRES(m) on the monolithic system (I - M V) u = e_bg (the fixed point of the
    outer loop of eqs. (8)-(9)): total field u, E_mask = K V u and the orders."""
    S = Setup(prob)
    deps = np.asarray(deps, dtype=np.complex128)
    u, info = gmres(lambda v: apply_monolithic(S, deps, v), background_field(S), None, rtol, restart, max_iters)
    V = potential(S, deps)
    return {"u": u, "emask": conv_K(S, V[None] * u), "orders": orders_of_total_field(S, deps, u),
            "iters": info["iters"], "rel_residual": info["rel_residual"], "setup": S}
