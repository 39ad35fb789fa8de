"""Python front end over the C ABI: torch tensors in, torch tensors out.

PyTorch only provides device memory and the current HIP stream; every
operation runs in libpsfd.so. Names follow the C entry points.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Optional, Sequence, Tuple

import torch

from . import _lib as L


def _c_problem(p) -> Tuple[L.psfd_problem, object]:
    layers = (L.psfd_layer * max(1, len(p.layers)))()
    for i, (e, d) in enumerate(p.layers):
        e = complex(e)
        layers[i] = L.psfd_layer(e.real, e.imag, float(d))
    es = complex(p.eps_sub)
    cp = L.psfd_problem(int(p.nx), int(p.ny), int(p.nz), float(p.lx_nm), float(p.ly_nm), float(p.t_nm),
                        float(p.wavelength_nm), float(p.eps_bg), float(p.theta_deg), float(p.phi_deg),
                        int(p.pol), len(p.layers), C.cast(layers, C.POINTER(L.psfd_layer)), es.real, es.imag)
    return cp, layers


def _c_opts(rtol=1e-6, outer_rtol=None, restart=30, max_iters=5000, max_outer=100, precision="mixed",
            inner_eta=1e-4, coupling="mono") -> L.psfd_opts:
    prec = {"fp64": L.PSFD_FP64, "mixed": L.PSFD_MIXED}[precision] if isinstance(precision, str) else int(precision)
    cpl = {"outer": L.PSFD_COUPLING_OUTER, "mono": L.PSFD_COUPLING_MONO}[coupling] if isinstance(coupling, str) \
        else int(coupling)
    return L.psfd_opts(float(rtol), float(outer_rtol if outer_rtol is not None else rtol), int(restart),
                       int(max_iters), int(max_outer), prec, float(inner_eta), cpl)


def _stream() -> C.c_void_p:
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Plan:
    """A problem's FP64 tables and (lazily) its solve workspace on the current device."""

    def __init__(self, prob, **opts):
        self.prob = prob
        self.nx, self.ny, self.nz = int(prob.nx), int(prob.ny), int(prob.nz)
        self._cp, self._keep = _c_problem(prob)
        self._opts = _c_opts(**opts)
        h = C.c_void_p()
        L.check(L.lib().psfd_plan_create(C.byref(self._cp), C.byref(self._opts), C.byref(h)), "psfd_plan_create")
        self._h = h
        # held here so that a plan collected at interpreter exit can still be freed
        self._destroy = L.lib().psfd_plan_destroy

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._destroy(self._h)
            self._h = None

    __del__ = close

    def footprint(self) -> int:
        v = C.c_size_t()
        L.check(L.lib().psfd_plan_footprint(self._h, C.byref(v)), "psfd_plan_footprint")
        return int(v.value)

    @property
    def field_shape(self):
        return (3, self.nz, self.ny, self.nx)

    def psfd_apply(self, deps: torch.Tensor, x: torch.Tensor, out: Optional[torch.Tensor] = None,
                   transpose: bool = False, k_only: bool = False, reflect: bool = False) -> torch.Tensor:
        """y = x - K(V x) (or K(V x)); reflect: K -> M = K + R_vol T_R K_top."""
        dt = x.dtype
        code = {torch.complex64: L.PSFD_C64, torch.complex128: L.PSFD_C128}[dt]
        _dev(deps, dt, "deps")
        _dev(x, dt, "x")
        if tuple(x.shape) != self.field_shape or tuple(deps.shape) != self.field_shape[1:]:
            raise ValueError("shape mismatch")
        if out is None:
            out = torch.empty_like(x)
        _dev(out, dt, "out")
        flags = (L.PSFD_APPLY_TRANSPOSE if transpose else 0) | (L.PSFD_APPLY_K_ONLY if k_only else 0) | \
            (L.PSFD_APPLY_REFLECT if reflect else 0)
        L.check(L.lib().psfd_apply(self._h, C.c_void_p(deps.data_ptr()), C.c_void_p(x.data_ptr()),
                                   C.c_void_p(out.data_ptr()), code, flags, _stream()), "psfd_apply")
        return out

    apply = psfd_apply

    def psfd_solve(self, deps: torch.Tensor, emask: Optional[torch.Tensor] = None,
                   orders: Optional[torch.Tensor] = None,
                   u: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, torch.Tensor, Dict]:
        """(E_mask, orders, info); u (optional, complex128 [3][nz][ny][nx]) receives the total field."""
        _dev(deps, torch.complex128, "deps")
        if tuple(deps.shape) != self.field_shape[1:]:
            raise ValueError("deps shape mismatch")
        if emask is None:
            emask = torch.empty(self.field_shape, dtype=torch.complex128, device=deps.device)
        if orders is None:
            orders = torch.empty((self.ny, self.nx, 3), dtype=torch.complex128, device=deps.device)
        _dev(emask, torch.complex128, "emask")
        _dev(orders, torch.complex128, "orders")
        if tuple(emask.shape) != self.field_shape or tuple(orders.shape) != (self.ny, self.nx, 3):
            raise ValueError("output shape mismatch")
        up = None
        if u is not None:
            _dev(u, torch.complex128, "u")
            if tuple(u.shape) != self.field_shape:
                raise ValueError("u shape mismatch")
            up = C.c_void_p(u.data_ptr())
        info = L.psfd_info()
        L.check(L.lib().psfd_solve(self._h, C.c_void_p(deps.data_ptr()), C.c_void_p(emask.data_ptr()),
                                   C.c_void_p(orders.data_ptr()), up, C.byref(info), _stream()), "psfd_solve")
        return emask, orders, info.as_dict()

    solve = psfd_solve

    def psfd_solve_adjoint(self, deps: torch.Tensor, u: torch.Tensor, grad_orders: torch.Tensor,
                           grad: Optional[torch.Tensor] = None) -> Tuple[torch.Tensor, Dict]:
        """dL/dRe + i dL/dIm of delta_eps from the forward total field u and the cotangent
        grad_orders = dL/dRe a + i dL/dIm a of the orders (complex128 [ny][nx][3])."""
        _dev(deps, torch.complex128, "deps")
        _dev(u, torch.complex128, "u")
        _dev(grad_orders, torch.complex128, "grad_orders")
        if tuple(deps.shape) != self.field_shape[1:] or tuple(u.shape) != self.field_shape or \
                tuple(grad_orders.shape) != (self.ny, self.nx, 3):
            raise ValueError("shape mismatch")
        if grad is None:
            grad = torch.empty_like(deps)
        _dev(grad, torch.complex128, "grad")
        info = L.psfd_info()
        L.check(L.lib().psfd_solve_adjoint(self._h, C.c_void_p(deps.data_ptr()), C.c_void_p(u.data_ptr()),
                                           C.c_void_p(grad_orders.data_ptr()), C.c_void_p(grad.data_ptr()),
                                           C.byref(info), _stream()), "psfd_solve_adjoint")
        return grad, info.as_dict()

    adjoint = psfd_solve_adjoint


def psfd_solve_batch(probs: Sequence, deps: Sequence[torch.Tensor], **opts):
    """Lock-step batched solves of same-shape instances; returns lists of fields, orders, infos."""
    n = len(probs)
    cps = (L.psfd_problem * n)()
    keep = []
    for i, p in enumerate(probs):
        cps[i], k = _c_problem(p)
        keep.append(k)
    o = _c_opts(**opts)
    em = [torch.empty((3, p.nz, p.ny, p.nx), dtype=torch.complex128, device=deps[0].device) for p in probs]
    od = [torch.empty((p.ny, p.nx, 3), dtype=torch.complex128, device=deps[0].device) for p in probs]
    for d in deps:
        _dev(d, torch.complex128, "deps")
    ad = (C.c_void_p * n)(*[d.data_ptr() for d in deps])
    ae = (C.c_void_p * n)(*[t.data_ptr() for t in em])
    ao = (C.c_void_p * n)(*[t.data_ptr() for t in od])
    info = (L.psfd_info * n)()
    L.check(L.lib().psfd_solve_batch(n, cps, C.byref(o), ad, ae, ao, info, _stream()), "psfd_solve_batch")
    return em, od, [info[i].as_dict() for i in range(n)]


solve_batch = psfd_solve_batch


def psfd_release_cached_workspaces() -> None:
    """Free the device workspaces psfd_solve_batch keeps for reuse."""
    L.check(L.lib().psfd_release_cached_workspaces(), "psfd_release_cached_workspaces")


class Server:
    """Continuous-batching solve server (a worker thread and stream per group of requests)."""

    def __init__(self, hbm_budget: int, max_slots: int, **opts):
        self._opts = _c_opts(**opts)
        self._defaults = dict(opts)
        h = C.c_void_p()
        L.check(L.lib().psfd_server_create(int(hbm_budget), int(max_slots), C.byref(self._opts), C.byref(h)),
                "psfd_server_create")
        self._h = h
        self._keep = {}

    def psfd_server_submit(self, prob, deps: torch.Tensor, emask: torch.Tensor, orders: torch.Tensor,
                           **opts) -> int:
        """Submit one solve; opts (rtol, restart, precision, ...) override the server's defaults."""
        cp, k = _c_problem(prob)
        for name, t, shape in (("deps", deps, (prob.nz, prob.ny, prob.nx)),
                               ("emask", emask, (3, prob.nz, prob.ny, prob.nx)),
                               ("orders", orders, (prob.ny, prob.nx, 3))):
            _dev(t, torch.complex128, name)
            if tuple(t.shape) != shape:
                raise ValueError(f"{name} shape mismatch")
        o = C.byref(_c_opts(**{**self._defaults, **opts})) if opts else None
        t = C.c_uint64()
        L.check(L.lib().psfd_server_submit(self._h, C.byref(cp), o, C.c_void_p(deps.data_ptr()),
                                           C.c_void_p(emask.data_ptr()), C.c_void_p(orders.data_ptr()),
                                           C.byref(t)), "psfd_server_submit")
        self._keep[int(t.value)] = (deps, emask, orders)
        return int(t.value)

    submit = psfd_server_submit

    def psfd_server_poll(self, ticket: int):
        done = C.c_int32()
        info = L.psfd_info()
        lat = C.c_double()
        L.check(L.lib().psfd_server_poll(self._h, C.c_uint64(ticket), C.byref(done), C.byref(info), C.byref(lat)),
                "psfd_server_poll")
        if done.value:
            self._keep.pop(int(ticket), None)
        return bool(done.value), info.as_dict(), float(lat.value)

    poll = psfd_server_poll

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            h, self._h = self._h, None
            if L is not None:
                L.check(L.lib().psfd_server_destroy(h), "psfd_server_destroy")

    __del__ = close


class Orders(torch.autograd.Function):
    """a(delta_eps): the reflected order amplitudes [ny][nx][3] of the plan's problem.

    Forward runs psfd_solve and keeps the total field; backward runs the
    hand-written adjoint solve (psfd_solve_adjoint) on the incoming cotangent,
    so any real loss of the orders can be differentiated. Gradients follow
    torch's convention for complex tensors (dL/dRe + i dL/dIm).
    """

    @staticmethod
    def forward(ctx, deps: torch.Tensor, plan: Plan):
        d = deps.detach().contiguous()
        u = torch.empty(plan.field_shape, dtype=torch.complex128, device=deps.device)
        _, orders, info = plan.psfd_solve(d, u=u)
        ctx.save_for_backward(d, u)
        ctx.plan = plan
        ctx.info = info
        return orders

    @staticmethod
    def backward(ctx, gout):
        d, u = ctx.saved_tensors
        grad, info = ctx.plan.psfd_solve_adjoint(d, u, gout.to(torch.complex128).contiguous())
        ctx.adjoint_info = info
        return grad, None


def order_intensity(deps: torch.Tensor, plan: Plan, orders_sel: Sequence[Tuple[int, int]]) -> torch.Tensor:
    """J = sum over the selected orders (m, n) of ||a_q||^2, differentiable in deps through Orders."""
    a = Orders.apply(deps, plan)
    ny, nx = a.shape[0], a.shape[1]
    idx = torch.tensor([(n % ny) * nx + (m % nx) for (m, n) in orders_sel], device=a.device)
    sel = a.reshape(ny * nx, 3).index_select(0, idx)
    return (sel.real ** 2 + sel.imag ** 2).sum()


class IsoPlan:
    """Isolated-domain mode: a scatterer in free space with the spherically
    windowed dyadic kernel and padding by 2 on all axes (psfd_iso_* entry
    points). The kernel table is precomputed on the current device at
    construction."""

    def __init__(self, nx: int, ny: int, nz: int, spacing_nm: Tuple[float, float, float],
                 wavelength_nm: float = 13.5, eps_bg: complex = 1.0, radius_nm: float = 0.0):
        dz, dy, dx = (float(v) for v in spacing_nm)
        e = complex(eps_bg)
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self._cp = L.psfd_iso_problem(self.nx, self.ny, self.nz, dx, dy, dz, float(wavelength_nm), e.real, e.imag,
                                      float(radius_nm))
        h = C.c_void_p()
        L.check(L.lib().psfd_iso_plan_create(C.byref(self._cp), C.byref(h)), "psfd_iso_plan_create")
        self._h = h
        self._destroy = L.lib().psfd_iso_plan_destroy

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._destroy(self._h)
            self._h = None

    __del__ = close

    @property
    def field_shape(self):
        return (3, self.nz, self.ny, self.nx)

    def _check(self, deps, x, out):
        dt = x.dtype
        code = {torch.complex64: L.PSFD_C64, torch.complex128: L.PSFD_C128}[dt]
        _dev(deps, dt, "deps")
        _dev(x, dt, "x")
        if tuple(x.shape) != self.field_shape or tuple(deps.shape) != self.field_shape[1:]:
            raise ValueError("shape mismatch")
        if out is None:
            out = torch.empty_like(x)
        _dev(out, dt, "out")
        return code, out

    def psfd_iso_apply(self, deps: torch.Tensor, x: torch.Tensor, out: Optional[torch.Tensor] = None) -> torch.Tensor:
        """y = x - P IFFT(table . FFT(Z V x)), V = k0^2 deps."""
        code, out = self._check(deps, x, out)
        L.check(L.lib().psfd_iso_apply(self._h, C.c_void_p(deps.data_ptr()), C.c_void_p(x.data_ptr()),
                                       C.c_void_p(out.data_ptr()), code, _stream()), "psfd_iso_apply")
        return out

    apply = psfd_iso_apply

    def psfd_iso_solve(self, deps: torch.Tensor, b: torch.Tensor, rtol: float = 1e-8, restart: int = 30,
                       max_iters: int = 2000, out: Optional[torch.Tensor] = None, precision: str = "fp64"):
        """u with u - K(V u) = b by GMRES (precision "fp64" or "mixed"); returns (u, info dict)."""
        if b.dtype != torch.complex128:
            raise ValueError("b must be complex128")
        _, out = self._check(deps, b, out)
        info = L.psfd_info()
        L.check(L.lib().psfd_iso_solve(self._h, C.c_void_p(deps.data_ptr()), C.c_void_p(b.data_ptr()),
                                       C.c_void_p(out.data_ptr()), float(rtol), int(restart), int(max_iters),
                                       {"fp64": L.PSFD_FP64, "mixed": L.PSFD_MIXED}[precision], C.byref(info),
                                       _stream()), "psfd_iso_solve")
        return out, info.as_dict()

    solve = psfd_iso_solve

    def psfd_iso_table(self):
        """(table complex128 [6][2nz][2ny][2nx] on the device, (o_z, o_y, o_x), R)."""
        t = torch.empty((6, 2 * self.nz, 2 * self.ny, 2 * self.nx), dtype=torch.complex128, device="cuda")
        over = (C.c_int32 * 3)()
        r = C.c_double()
        L.check(L.lib().psfd_iso_table(self._h, C.c_void_p(t.data_ptr()), over, C.byref(r), _stream()),
                "psfd_iso_table")
        return t, tuple(int(v) for v in over), float(r.value)

    table = psfd_iso_table

    def bench_stage(self, stage: int, deps: torch.Tensor, x: torch.Tensor, out: torch.Tensor, reps: int) -> float:
        code, out = self._check(deps, x, out)
        ms = C.c_float()
        L.check(L.lib().psfd_iso_bench_stage(self._h, int(stage), C.c_void_p(deps.data_ptr()),
                                             C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()), code, int(reps),
                                             C.byref(ms), _stream()), "psfd_iso_bench_stage")
        return float(ms.value)


class DiffPlan:
    """Differential PSFD operator with a z-PML on an extended z grid (psfd_diff_* entry
    points): the comparison solver of the preconditioner study, in the background-field
    form (outer reflection loop) or the full-domain form (multilayer on the grid)."""

    def __init__(self, prob, nz_ext: int, zc0: int, ncz: int, pml_cells: int, pml_order: int = 3,
                 pml_reflection: float = 1e-8, form: str = "background"):
        self.prob = prob
        self.nx, self.ny, self.nz = int(prob.nx), int(prob.ny), int(prob.nz)
        self.nz_ext, self.zc0, self.ncz = int(nz_ext), int(zc0), int(ncz)
        cp, self._keep = _c_problem(prob)
        self._cp = L.psfd_diff_problem(cp, self.nz_ext, self.zc0, self.ncz, int(pml_cells), int(pml_order),
                                       float(pml_reflection),
                                       {"background": L.PSFD_DIFF_BACKGROUND, "full": L.PSFD_DIFF_FULL_DOMAIN}[form])
        h = C.c_void_p()
        L.check(L.lib().psfd_diff_plan_create(C.byref(self._cp), C.byref(h)), "psfd_diff_plan_create")
        self._h = h
        self._destroy = L.lib().psfd_diff_plan_destroy

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._destroy(self._h)
            self._h = None

    __del__ = close

    @property
    def field_shape(self):
        return (3, self.nz_ext, self.ny, self.nx)

    @staticmethod
    def _pc(precond):
        return {"none": L.PSFD_PRECOND_NONE, "damping": L.PSFD_PRECOND_DAMPING}[precond]

    def psfd_diff_apply(self, deps: torch.Tensor, x: torch.Tensor, out: Optional[torch.Tensor] = None,
                        precond: str = "none") -> torch.Tensor:
        """y = A x (or D A x): curl curl x - k_bg^2 x - V x on the extended grid."""
        dt = x.dtype
        code = {torch.complex64: L.PSFD_C64, torch.complex128: L.PSFD_C128}[dt]
        _dev(deps, dt, "deps")
        _dev(x, dt, "x")
        if tuple(x.shape) != self.field_shape or tuple(deps.shape) != (self.ncz, self.ny, self.nx):
            raise ValueError("shape mismatch")
        if out is None:
            out = torch.empty_like(x)
        _dev(out, dt, "out")
        L.check(L.lib().psfd_diff_apply(self._h, C.c_void_p(deps.data_ptr()), C.c_void_p(x.data_ptr()),
                                        C.c_void_p(out.data_ptr()), code, self._pc(precond), _stream()),
                "psfd_diff_apply")
        return out

    apply = psfd_diff_apply

    def psfd_diff_solve(self, deps: torch.Tensor, precond: str = "none", e: Optional[torch.Tensor] = None,
                        orders: Optional[torch.Tensor] = None, **opts):
        """(field on the extended grid, orders, info) of the background-field or full-domain solve."""
        _dev(deps, torch.complex128, "deps")
        if tuple(deps.shape) != (self.ncz, self.ny, self.nx):
            raise ValueError("deps shape mismatch")
        if e is None:
            e = torch.empty(self.field_shape, dtype=torch.complex128, device=deps.device)
        if orders is None:
            orders = torch.empty((self.ny, self.nx, 3), dtype=torch.complex128, device=deps.device)
        _dev(e, torch.complex128, "e")
        _dev(orders, torch.complex128, "orders")
        o = _c_opts(**opts)
        info = L.psfd_info()
        L.check(L.lib().psfd_diff_solve(self._h, C.c_void_p(deps.data_ptr()), C.c_void_p(e.data_ptr()),
                                        C.c_void_p(orders.data_ptr()), C.byref(o), self._pc(precond),
                                        C.byref(info), _stream()), "psfd_diff_solve")
        return e, orders, info.as_dict()

    solve = psfd_diff_solve
