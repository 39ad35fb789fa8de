"""Batched solves and the continuous-batching server.

* A batch of instances (different angles, polarisations, clips) gives the same
  result per instance as solving each alone (bitwise: every reduction runs per
  instance with a fixed layout).
* Requests submitted while others are running are admitted as slots free up;
  each served result equals the same problem solved alone, and agrees with the
  oracle.
* Admission respects the device-memory budget.
"""
import time

import numpy as np
import pytest

import oracle as O
from paper_2606_25541_amd import clips

from gpu_util import device, rel, say, torch

pytestmark = pytest.mark.gpu


def prob(n, nz, theta, phi, pol, pairs=20):
    layers, es = clips.mo_si_stack(pairs)
    return clips.Problem(nx=n, ny=n, nz=nz, lx_nm=2.0 * n, ly_nm=2.0 * n, t_nm=30.0, theta_deg=theta,
                         phi_deg=phi, pol=pol, layers=layers, eps_sub=es)


def cases():
    out = []
    angles = clips.pupil_angles()
    for i in range(6):
        n, nz = (16, 8) if i % 2 == 0 else (32, 8)
        th, ph = angles[(7 * i) % len(angles)]
        p = prob(n, nz, th, ph, i % 2 if i < 4 else 0)
        out.append((p, clips.manhattan(n, n, nz, p.lx_nm, p.ly_nm, seed=100 + i)))
    return out


OPTS = dict(rtol=1e-9, precision="mixed", restart=16)


def alone(p, de, dev):
    from paper_2606_25541_amd import api
    plan = api.Plan(p, **OPTS)
    em, od, info = plan.psfd_solve(torch.from_numpy(de).to(dev))
    torch.cuda.synchronize()
    return em.cpu().numpy(), od.cpu().numpy(), info


def test_batch_equals_single():
    from paper_2606_25541_amd import api
    dev = device()
    cs = [c for c in cases() if c[0].nx == 16]
    say("batch of", len(cs))
    em, od, infos = api.psfd_solve_batch([c[0] for c in cs], [torch.from_numpy(c[1]).to(dev) for c in cs], **OPTS)
    torch.cuda.synchronize()
    for (p, de), e, o, inf in zip(cs, em, od, infos):
        e1, o1, i1 = alone(p, de, dev)
        assert inf["status"] == 0
        assert np.array_equal(e.cpu().numpy(), e1), rel(e.cpu().numpy(), e1)
        assert np.array_equal(o.cpu().numpy(), o1)
        assert inf["iters"] == i1["iters"]


@pytest.mark.parametrize("n,prec", [(64, "mixed"), (128, "mixed"), (128, "fp64")])
def test_batch_equals_single_128_planes(n, prec):
    """FP32 square planes (64 x 64 and 128 x 128), 32 per component (padded z length 64, pencil
    blocks large enough for the Givens task): the lock-step batch runs the
    Gram-Schmidt update in the forward plane kernel, the projections in the
    inverse one and the last column's Givens step from the projections. FP64 at
    128 x 128: the Arnoldi steps on quarter planes with a separate Givens launch.
    Three instances, one of which converges cycles before the others, must each
    equal their lone solve bitwise."""
    from paper_2606_25541_amd import api
    dev = device()
    angles = clips.pupil_angles()
    cs = []
    for i in range(3):
        th, ph = angles[(11 * i + 3) % len(angles)]
        p = prob(n, 32, th, ph, i % 2)
        de = clips.manhattan(n, n, 32, p.lx_nm, p.ly_nm, seed=300 + i)
        if i == 2:
            de = de * 0.25  # weaker contrast: converges in fewer cycles
        cs.append((p, de))
    opts = dict(rtol=1e-9, precision=prec, restart=8)
    say("batch of 3 at %dx%dx32 %s" % (n, n, prec))
    em, od, infos = api.psfd_solve_batch([c[0] for c in cs], [torch.from_numpy(c[1]).to(dev) for c in cs], **opts)
    torch.cuda.synchronize()
    iters = []
    for (p, de), e, o, inf in zip(cs, em, od, infos):
        plan = api.Plan(p, **opts)
        e1, o1, i1 = plan.psfd_solve(torch.from_numpy(de).to(dev))
        torch.cuda.synchronize()
        say("  batched", inf, "alone", i1)
        assert inf["status"] == 0
        assert inf["iters"] == i1["iters"]
        assert np.array_equal(e.cpu().numpy(), e1.cpu().numpy()), rel(e.cpu().numpy(), e1.cpu().numpy())
        assert np.array_equal(o.cpu().numpy(), o1.cpu().numpy())
        iters.append(inf["iters"])
    assert min(iters) < max(iters)


@pytest.mark.parametrize("n,prec", [(64, "mixed"), (128, "mixed"), (128, "fp64")])
def test_server_matches_alone_128_planes(n, prec):
    """n x n x 32 (n = 64, 128), mixed: the lone (lock-step) solve and the server's slots
    (each at its own step, with a per-slot pending-update flag) run the same
    fused kernels: the Gram-Schmidt update in the forward plane kernel, the
    projections in the inverse one, the Givens step in the pencil and the last
    column's from the projections. FP64 at 128 x 128: the quarter-plane steps,
    the Givens step in its own launch (lone) or in the update pass (slots).
    Two requests submitted apart, so that their slots stand at different steps,
    each equal their lone solve bit for bit."""
    from paper_2606_25541_amd import api
    dev = device()
    opts = dict(rtol=1e-10, precision=prec, restart=8)
    reqs = []
    for i, (th, ph, pol) in enumerate(((6.0, 0.0, 0), (7.5, 40.0, 1))):
        p = prob(n, 32, th, ph, pol)
        de = clips.manhattan(n, n, 32, p.lx_nm, p.ly_nm, seed=401 + i)
        reqs.append((p, torch.from_numpy(de).to(dev)))
    srv = api.Server(hbm_budget=8 << 30, max_slots=2, **opts)
    outs, tickets = [], []
    for k, (p, d) in enumerate(reqs):
        e = torch.empty((3, p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
        o = torch.empty((p.ny, p.nx, 3), dtype=torch.complex128, device=dev)
        tickets.append(srv.submit(p, d, e, o))
        outs.append((e, o))
        if k == 0:
            time.sleep(0.003)  # the second request joins while the first runs
    infos = {}
    deadline = time.perf_counter() + 60
    while len(infos) < len(tickets) and time.perf_counter() < deadline:
        for t in tickets:
            if t not in infos:
                done, info, _ = srv.poll(t)
                if done:
                    infos[t] = info
        time.sleep(0.002)
    srv.close()
    assert len(infos) == len(tickets), "served requests not finished within 60 s"
    for (p, d), (e2, o2), t in zip(reqs, outs, tickets):
        plan = api.Plan(p, **opts)
        e1, o1, i1 = plan.psfd_solve(d)
        torch.cuda.synchronize()
        i2 = infos[t]
        say("  alone", i1, "served", i2)
        assert i1["status"] == 0 and i2["status"] == 0
        assert i1["iters"] == i2["iters"]
        assert torch.equal(e1, e2), rel(e2.cpu().numpy(), e1.cpu().numpy())
        assert torch.equal(o1, o2)


def test_batch_reuses_cached_workspace():
    # a second call of the same kind runs in the kept workspace: same results;
    # after the cache is released the call allocates afresh, same results again
    from paper_2606_25541_amd import api
    dev = device()
    cs = [c for c in cases() if c[0].nx == 32][:2]
    ds = [torch.from_numpy(c[1]).to(dev) for c in cs]
    runs = []
    for k in range(3):
        if k == 2:
            api.psfd_release_cached_workspaces()
        em, od, infos = api.psfd_solve_batch([c[0] for c in cs], ds, **OPTS)
        torch.cuda.synchronize()
        assert all(i["status"] == 0 for i in infos)
        runs.append(([e.cpu().numpy() for e in em], [o.cpu().numpy() for o in od], [i["iters"] for i in infos]))
    for r in runs[1:]:
        assert r[2] == runs[0][2]
        for a, b in zip(r[0] + r[1], runs[0][0] + runs[0][1]):
            assert np.array_equal(a, b)
    api.psfd_release_cached_workspaces()


def test_server_mix_equals_alone_and_oracle():
    from paper_2606_25541_amd import api
    dev = device()
    cs = cases()
    srv = api.Server(hbm_budget=8 << 30, max_slots=2, **OPTS)
    outs, tickets = [], []
    for k, (p, de) in enumerate(cs):
        d = torch.from_numpy(de).to(dev)
        e = torch.empty((3, p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
        o = torch.empty((p.ny, p.nx, 3), dtype=torch.complex128, device=dev)
        torch.cuda.synchronize()
        tickets.append(srv.submit(p, d, e, o))
        outs.append((d, e, o))
        if k == 2:
            time.sleep(0.05)  # later requests arrive while the first ones run
    results = {}
    t0 = time.time()
    while len(results) < len(tickets) and time.time() - t0 < 120:
        for t in tickets:
            if t in results:
                continue
            done, info, lat = srv.poll(t)
            if done:
                results[t] = (info, lat)
        time.sleep(0.002)
    srv.close()
    assert len(results) == len(tickets)
    for (p, de), t, (d, e, o) in zip(cs, tickets, outs):
        info, lat = results[t]
        say("served", p.nx, info, "latency %.3f s" % lat)
        assert info["status"] == 0 and lat > 0
        e1, o1, i1 = alone(p, de, dev)
        assert np.array_equal(e.cpu().numpy(), e1), rel(e.cpu().numpy(), e1)
        assert np.array_equal(o.cpu().numpy(), o1)
    p, de = cs[1]
    ref = O.solve(p, de, rtol=1e-11)
    assert rel(outs[1][1].cpu().numpy(), ref["emask"]) < 1e-7


def test_server_budget_admission():
    from paper_2606_25541_amd import api
    dev = device()
    p, de = cases()[0]
    plan = api.Plan(p, **OPTS)
    per_slot = plan.footprint()
    # budget below one slot: the request is refused with an out-of-memory status
    srv = api.Server(hbm_budget=per_slot // 2, max_slots=4, **OPTS)
    d = torch.from_numpy(de).to(dev)
    e = torch.empty((3, p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
    o = torch.empty((p.ny, p.nx, 3), dtype=torch.complex128, device=dev)
    t = srv.submit(p, d, e, o)
    for _ in range(2000):
        done, info, lat = srv.poll(t)
        if done:
            break
        time.sleep(0.005)
    assert done and info["status"] == -3
    srv.close()
    # budget for one slot: three requests run one after another, all complete
    srv = api.Server(hbm_budget=int(per_slot * 1.5), max_slots=4, **OPTS)
    bufs = [(torch.empty_like(e), torch.empty_like(o)) for _ in range(3)]
    ts = [srv.submit(p, d, bb[0], bb[1]) for bb in bufs]
    lats = []
    for t in ts:
        for _ in range(20000):
            done, info, lat = srv.poll(t)
            if done:
                break
            time.sleep(0.001)
        assert done and info["status"] == 0
        lats.append(lat)
    srv.close()
    assert lats[0] < lats[1] < lats[2]
    for bb in bufs[1:]:
        assert torch.equal(bb[0], bufs[0][0])


def _drain(srv, tickets, limit_s=120.0):
    infos = {}
    deadline = time.perf_counter() + limit_s
    while len(infos) < len(tickets) and time.perf_counter() < deadline:
        for t in tickets:
            if t not in infos:
                done, info, lat = srv.poll(t)
                if done:
                    infos[t] = (info, lat)
        time.sleep(0.002)
    return infos


def test_server_binding_budget_queues_mixed_shapes():
    """A budget that holds one slot of either shape but not one of each: requests
    of the second shape wait (no OOM) until the first shape's group is drained
    and released, and every result still equals its lone solve bitwise."""
    from paper_2606_25541_amd import api
    dev = device()
    cs = cases()  # 16x16x8 and 32x32x8 alternating
    per = {c[0].nx: api.Plan(c[0], **OPTS).footprint() for c in cs[:2]}
    budget = int(max(per.values()) * 1.2)
    assert budget < sum(per.values())
    say("budget", budget, "per slot", per)
    srv = api.Server(hbm_budget=budget, max_slots=4, **OPTS)
    outs, tickets = [], []
    for p, de in cs:
        d = torch.from_numpy(de).to(dev)
        e = torch.empty((3, p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
        o = torch.empty((p.ny, p.nx, 3), dtype=torch.complex128, device=dev)
        torch.cuda.synchronize()
        tickets.append(srv.submit(p, d, e, o))
        outs.append((e, o))
    infos = _drain(srv, tickets)
    srv.close()
    assert len(infos) == len(tickets), "served requests not finished"
    for (p, de), t, (e, o) in zip(cs, tickets, outs):
        info, lat = infos[t]
        say("  served", p.nx, info["status"], info["iters"], "latency %.3f" % lat)
        assert info["status"] == 0
        e1, o1, i1 = alone(p, de, dev)
        assert info["iters"] == i1["iters"]
        assert np.array_equal(e.cpu().numpy(), e1)
        assert np.array_equal(o.cpu().numpy(), o1)


def test_server_per_request_options():
    """Options per request: a tighter tolerance and an FP64 request (another
    kind, its own group) next to the server's defaults; each equals the lone
    solve with the same options."""
    from paper_2606_25541_amd import api
    dev = device()
    cs = [c for c in cases() if c[0].nx == 16]
    variants = [dict(), dict(rtol=1e-11), dict(precision="fp64", restart=12)]
    srv = api.Server(hbm_budget=8 << 30, max_slots=2, **OPTS)
    outs, tickets = [], []
    for (p, de), v in zip(cs, variants):
        d = torch.from_numpy(de).to(dev)
        e = torch.empty((3, p.nz, p.ny, p.nx), dtype=torch.complex128, device=dev)
        o = torch.empty((p.ny, p.nx, 3), dtype=torch.complex128, device=dev)
        torch.cuda.synchronize()
        tickets.append(srv.submit(p, d, e, o, **v))
        outs.append((d, e, o))
    infos = _drain(srv, tickets)
    srv.close()
    assert len(infos) == len(tickets)
    for (p, de), v, t, (d, e, o) in zip(cs, variants, tickets, outs):
        info, _ = infos[t]
        plan = api.Plan(p, **{**OPTS, **v})
        e1, o1, i1 = plan.psfd_solve(d)
        torch.cuda.synchronize()
        say("  opts", v, "served", info["iters"], info["rel_residual"], "alone", i1["iters"])
        assert info["status"] == 0 and info["iters"] == i1["iters"]
        assert info["rel_residual"] <= {**OPTS, **v}["rtol"]
        assert torch.equal(e, e1) and torch.equal(o, o1)


@pytest.mark.parametrize("n", [16, 64])
def test_graph_replay_equals_eager_launches(n, monkeypatch):
    """Restart cycles replayed as a captured HIP graph against the same launches
    issued one by one (PSFD_GRAPH=0): bitwise equal fields, orders and counts,
    over several solves in a row (each replays the graph many times, with
    eager launches and host synchronisation between the replays)."""
    from paper_2606_25541_amd import api
    dev = device()
    p = prob(n, 32 if n == 64 else 8, 6.0, 20.0, 1)
    de = clips.manhattan(n, n, p.nz, p.lx_nm, p.ly_nm, seed=500 + n)
    d = torch.from_numpy(de).to(dev)
    opts = dict(rtol=1e-9, precision="mixed", restart=8)
    plan = api.Plan(p, **opts)
    runs = [plan.psfd_solve(d) for _ in range(3)]
    monkeypatch.setenv("PSFD_GRAPH", "0")
    e0, o0, i0 = plan.psfd_solve(d)
    torch.cuda.synchronize()
    say("  graph", runs[0][2], "eager", i0)
    assert i0["status"] == 0
    for e, o, i in runs:
        assert i == i0
        assert torch.equal(e, e0) and torch.equal(o, o0)


@pytest.mark.parametrize("n", [16, 64])
def test_restarts_without_residual_keep_results(n, monkeypatch):
    """Restarts that leave out the FP64 b - A x they do not use (the default)
    against restarts that all form it (PSFD_LITE_RESTARTS=0), and against a host
    blind to the residual ratio (PSFD_NEAR_RATIO=0), whose instances ask for b -
    A x at restarts without it and wait for one: bitwise equal fields, orders,
    step and cycle counts."""
    from paper_2606_25541_amd import api
    dev = device()
    p = prob(n, 32 if n == 64 else 8, 6.0, 20.0, 1)
    de = clips.manhattan(n, n, p.nz, p.lx_nm, p.ly_nm, seed=700 + n)
    d = torch.from_numpy(de).to(dev)
    plan = api.Plan(p, rtol=1e-9, precision="mixed", restart=8)
    res = {}
    for name, env in (("default", {}), ("blind", {"PSFD_NEAR_RATIO": "0"}),
                      ("all", {"PSFD_NEAR_RATIO": "0", "PSFD_LITE_RESTARTS": "0"})):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        res[name] = plan.psfd_solve(d)
        torch.cuda.synchronize()
    e0, o0, i0 = res["all"]
    say("  restarts", {k: v[2]["iters"] for k, v in res.items()})
    assert i0["status"] == 0
    for e, o, i in res.values():
        assert i == i0
        assert torch.equal(e, e0) and torch.equal(o, o0)


def test_iteration_limit_with_restarts_without_residual(monkeypatch):
    """A solve stopped by its iteration limit (11 steps of GMRES(4)) reports
    NOT_CONVERGED with the same steps, residual and field whether its restarts
    leave out the unused b - A x (the default), make instances wait for it
    (PSFD_NEAR_RATIO=0) or all form it (PSFD_LITE_RESTARTS=0)."""
    from paper_2606_25541_amd import _lib as L, api
    dev = device()
    p = prob(64, 32, 6.0, 20.0, 1)
    de = clips.manhattan(64, 64, p.nz, p.lx_nm, p.ly_nm, seed=901)
    d = torch.from_numpy(de).to(dev)
    plan = api.Plan(p, rtol=1e-12, precision="mixed", restart=4, max_iters=11)
    res = {}
    for name, env in (("default", {}), ("blind", {"PSFD_NEAR_RATIO": "0"}),
                      ("all", {"PSFD_NEAR_RATIO": "0", "PSFD_LITE_RESTARTS": "0"})):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        res[name] = plan.psfd_solve(d)
        torch.cuda.synchronize()
    e0, o0, i0 = res["all"]
    say("  limit", {k: (v[2]["iters"], v[2]["status"]) for k, v in res.items()})
    assert i0["status"] == L.PSFD_NOT_CONVERGED and 11 <= i0["iters"] <= 12
    for e, o, i in res.values():
        assert i == i0
        assert torch.equal(e, e0) and torch.equal(o, o0)
