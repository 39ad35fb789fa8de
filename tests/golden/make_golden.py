"""Write the oracle reference solutions of the measured workloads (calls only the oracle).

Each case is the oracle's FP64 GMRES(30) solve of the monolithic system
(I - M V) u = e_bg (eqs. (3), (8)-(9) and (18): the fixed point of the outer
reflection loop, with M = K + R_vol T_R K_top) to a relative residual of 1e-10,
from the seeded inputs of ``paper_2606_25541_amd.clips``. Stored per case
(``<case>.npz``):

* ``emask_sample``: E_mask = K V u (envelope) on a lattice of 8 z-planes and
  16 x 16 (x, y) points, complex128 [3][8][16][16], with its indices
  ``zi``, ``yi``, ``xi``;
* ``emask_norm``: the 2-norm of the whole E_mask field;
* ``orders``: the reflected order amplitudes a_q at z = T for |m|, |n| <= 8,
  complex128 [17][17][3] (order (m, n) at [n + 8][m + 8]);
* ``meta``: JSON with the case recipe and the oracle's iteration count and
  final relative residual.

With ``--iterations`` it records instead the oracle's own GMRES(30) iteration
counts on the headline solve to rtol 1e-6 and 3e-7
(``oracle_headline_iterations.json``).

Usage: ``python tests/golden/make_golden.py [case ...] [--workers N] [--iterations]``.
A 128 x 128 x 64 case takes about 10 minutes on 6 host threads, the
256 x 256 x 64 case about 40.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2606_25541_amd import clips  # noqa: E402

RTOL = 1e-10
RESTART = 30
NORD = 8


def cases():
    """name -> (description, problem, delta_eps)."""
    out = {}
    d2 = clips.headline_clip()
    for pol, tag in ((clips.TE, "te"), (clips.TM, "tm")):
        out["contact_holes_128x128x64_" + tag] = (
            "128x128x64 contact holes (256 nm, 8 holes, seed 2001), %s 6 deg" % tag.upper(),
            clips.config_problem("G3", pol=pol), d2)
    pool = clips.serving_pool()
    for i in range(3):
        g, p, d = pool[i]
        out["serving_pool_%d_%dx%dx%d" % (i, p.nx, p.ny, p.nz)] = (
            "serving pool request %d: %s Manhattan clip seed %d, theta %.4f phi %.4f TE" % (
                i, g, 4000 + i, p.theta_deg, p.phi_deg), p, d)
    bat = clips.batched_set()
    for i in range(2):
        g, p, d = bat[i]
        out["batched_%d_%dx%dx%d" % (i, p.nx, p.ny, p.nz)] = (
            "batched instance %d: %s Manhattan clip seed %d, theta %.4f phi %.4f TE" % (
                i, g, 3000 + i, p.theta_deg, p.phi_deg), p, d)
    return out


def sample_index(n: int, k: int) -> np.ndarray:
    """k evenly spaced indices of [0, n), starting at 0."""
    return (np.arange(k) * (n // k)).astype(np.int64)


def make(name, desc, p, d):
    t0 = time.perf_counter()
    S = O.Setup(p)
    ebg = O.background_field(S)
    u, info = O.gmres(lambda v: O.apply_monolithic(S, d, v), ebg, None, RTOL, RESTART, 20000)
    V = O.potential(S, d)
    x = O.conv_K(S, V[None] * u)
    a_up = O.reflect(S, O.incident_down(S) + O.read_down(S, V[None] * u))
    orders = O.reflected_orders(S, d, u, a_up)
    zi, yi, xi = sample_index(p.nz, 8), sample_index(p.ny, 16), sample_index(p.nx, 16)
    mi = np.arange(-NORD, NORD + 1)
    osel = orders[np.ix_(mi % p.ny, mi % p.nx)]
    meta = {"case": name, "description": desc, "grid": [p.nx, p.ny, p.nz], "clip_nm": [p.lx_nm, p.ly_nm, p.t_nm],
            "theta_deg": p.theta_deg, "phi_deg": p.phi_deg, "pol": p.pol,
            "solver": "oracle GMRES(%d) on (I - M V) u = e_bg, rtol %g" % (RESTART, RTOL),
            "iters": info["iters"], "rel_residual": float(info["rel_residual"]),
            "seconds": time.perf_counter() - t0}
    np.savez(os.path.join(HERE, name + ".npz"), emask_sample=x[:, zi][:, :, yi][:, :, :, xi], zi=zi, yi=yi, xi=xi,
             emask_norm=np.linalg.norm(x), orders=osel, meta=json.dumps(meta))
    print(json.dumps(meta), flush=True)


def iterations(workers):
    """The oracle's own GMRES(30) iteration counts on the headline solve (the monolithic
    system of the 128x128x64 contact holes, TE) to the benchmark's tolerances, from zero:
    the count by which the timed CPU sample of the benchmark is scaled to a full solve."""
    p, d = clips.config_problem("G3", pol=clips.TE), clips.headline_clip()
    S = O.Setup(p)
    ebg = O.background_field(S)
    res = {"case": "contact_holes_128x128x64_te", "solver": "oracle GMRES(%d) on (I - M V) u = e_bg" % RESTART,
           "workers": workers, "runs": []}
    for rtol in (1e-6, 3e-7):
        t0 = time.perf_counter()
        _, info = O.gmres(lambda v: O.apply_monolithic(S, d, v), ebg, None, rtol, RESTART, 20000)
        res["runs"].append({"rtol": rtol, "iters": info["iters"], "rel_residual": float(info["rel_residual"]),
                            "seconds": time.perf_counter() - t0})
        print(json.dumps(res["runs"][-1]), flush=True)
    with open(os.path.join(HERE, "oracle_headline_iterations.json"), "w") as f:
        json.dump(res, f, indent=1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cases", nargs="*")
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--iterations", action="store_true",
                    help="record the oracle's iteration counts on the headline solve instead")
    a = ap.parse_args()
    O.set_workers(a.workers)
    if a.iterations:
        iterations(a.workers)
        return
    cs = cases()
    for name in (a.cases or list(cs)):
        make(name, *cs[name])


if __name__ == "__main__":
    main()
