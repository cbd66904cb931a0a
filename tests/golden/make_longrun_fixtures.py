#!/usr/bin/env python3
"""Writes tests/golden/longrun_<case>.json: the oracle's state at sampled cells after 10, 100, 500,
1000 and 2000 steps (the backstep) or 10, 100 and 500 steps (the airfoil) of two full-size workloads, for the GPU long-run parity tests.

  backstep: the 122,876-cell backward-facing step (Re_h 3.6e4, SST, dt = min(60 tau0, 0.9 of the
            advective Courant limit)), from rest, 2000 steps;
  airfoil:  the 512 x 384 O-mesh around the 12 % section (Re 6e6, 10 degrees, dt = min(180 tau0, 0.9
            of the Courant limit), face-value limiter of reading r32, developed near-wall start), 500
            steps.  From about step 900 omega falls in a few cells at the trailing edge and reaches
            its floor (1e-20) by step 1300; nu_t = a1 k / max(a1 omega, S F2) is then bounded only
            by S F2, and runs that differ by rounding separate (the oracle's own run had left the
            GPU's by step 1000, while the oracle restarted from the GPU's FP64 state at step 500
            still tracked it at step 1000).

Per checkpoint: f (9 values), k, omega, nu_t at 160 sampled cells (seeded: anywhere, wall cells, and where
the flow starts), the
totals, the wall force and for the airfoil the lift and drag coefficients.  The file is rewritten at
every checkpoint.  Calls only the oracle and the seeded mesh generator.  Runs for hours:

    python tests/golden/make_longrun_fixtures.py backstep
    python tests/golden/make_longrun_fixtures.py airfoil
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fvlbm_oracle as O                  # noqa: E402
from paper_1812_00394_amd import meshgen as mg        # noqa: E402

CHECKPOINTS = (10, 100, 500, 1000, 2000)


def mesh_sha(m):
    h = hashlib.sha256()
    for key in ("nodes", "cell_ptr", "cell_nodes", "bface_nodes", "bface_group", "group_kind"):
        h.update(np.ascontiguousarray(m[key]).tobytes())
    return h.hexdigest()


def courant_dt(G):
    en = np.maximum(O.EX[:, None] * G.nl[:, 0] + O.EY[:, None] * G.nl[:, 1], 0.0)
    out = np.stack([np.bincount(G.cell, weights=en[a], minlength=G.n) for a in range(9)])
    return 1.0 / (out / G.area).max()


def case(name):
    """(mesh, params, f0, k0, w0, steps, wall mask, lift/drag (u_ref, chord) or None)"""
    if name == "backstep":
        m = mg.backstep()
        U, Re = 0.05, 3.6e4
        nu = U / Re
        G = O.Geometry(m)
        p = O.default_params(nu=nu, dt=min(60 * 3 * nu, 0.9 * courant_dt(G)), sst=True,
                             group_u=[[0, 0], [U, 0], [0, 0]], group_rho=[1, 1, 1], group_k=[0, 1e-6, 0],
                             group_w=[0, 1e-2, 0])
        n = G.n
        orc = O.Oracle(m, p)
        f0, k0, w0 = orc.init_state(np.ones(n), np.zeros(n), np.zeros(n), np.full(n, 1e-6), np.full(n, 1e-2))
        return m, p, orc, f0, k0, w0, 2000, 1, None
    if name == "airfoil":
        m = mg.naca_omesh()
        U, c, Re, alpha = 0.05, 1.0, 6e6, np.deg2rad(10.0)
        nu = U * c / Re
        kinf, winf = 1e-3 * U * U / Re, 5 * U / c
        G = O.Geometry(m)
        p = O.default_params(nu=nu, dt=min(180 * 3 * nu, 0.9 * courant_dt(G)), sst=True, theta=alpha, limiter=1,
                             group_u=[[0, 0], [U, 0]], group_rho=[1, 1], group_k=[0, kinf], group_w=[0, winf])
        wd = G.wall_dist
        fac = np.minimum(1.0, (wd / 0.01) ** (1 / 7))
        w0 = np.maximum(winf, 6 * nu / (0.075 * wd ** 2))
        orc = O.Oracle(m, p)
        n = G.n
        f0, k0, w0 = orc.init_state(np.ones(n), U * np.cos(alpha) * fac, U * np.sin(alpha) * fac, np.full(n, kinf), w0)
        return m, p, orc, f0, k0, w0, 500, 1, (U, c)
    raise SystemExit(f"unknown case {name}")


def samples(orc, rng):
    """64 cells anywhere, 32 wall cells and 64 cells where the flow starts: within 0.3 of the inlet
    edges (the backstep; over its 2000 steps the start-up front travels about 0.2 h), or within 0.2
    chord of the section (the airfoil)."""
    G = orc.g
    n = G.n
    walls = np.unique(G.cell[G.bidx[(orc.b_kind == O.WALL)]])
    inlet = orc.b_kind == O.INLET
    if inlet.any():
        x0 = G.xf[G.bidx[inlet], 0].min()
        near = np.nonzero(G.xc[:, 0] < x0 + 0.3)[0]
    else:
        near = np.nonzero(G.wall_dist < 0.2)[0]
    return np.unique(np.concatenate([rng.choice(n, 64, replace=False), rng.choice(walls, 32, replace=False),
                                     rng.choice(near, 64, replace=False)]))


def main(name):
    t0 = time.time()
    m, p, orc, f, k, w, steps, mask, ld = case(name)
    cells = samples(orc, np.random.default_rng(2024))
    out = {"what": f"oracle state at sampled cells of the {name} workload after the listed steps",
           "script": "tests/golden/make_longrun_fixtures.py", "mesh_sha256": mesh_sha(m), "n_cells": int(orc.g.n),
           "params": {kk: (v.tolist() if isinstance(v, np.ndarray) else v) for kk, v in p.items()},
           "cells": cells.tolist(), "wall_mask": mask, "lift_drag_ref": ld, "checkpoints": {}}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"longrun_{name}.json")
    done = 0
    for cp in CHECKPOINTS:
        if cp > steps:
            break
        f, k, w = orc.run(f, k, w, cp - done)
        done = cp
        Fv, jr = orc.forces(f, mask)
        rec = {"f": f[:, cells].tolist(), "k": k[cells].tolist(), "omega": w[cells].tolist(),
               "nu_t": orc.last_nut[cells].tolist(), "totals": orc.totals(f).tolist(),
               "force": Fv.tolist(), "j_r": float(jr),
               "f_dev_scale": float(np.abs(f - O.WT[:, None] * p["rho0"]).max()),
               "finite": bool(np.isfinite(f).all()), "seconds": round(time.time() - t0, 1)}
        if ld:
            rec["lift_drag"] = orc.lift_drag(f, mask, ld[0], ld[1]).tolist()
        out["checkpoints"][str(cp)] = rec
        with open(path + ".tmp", "w") as fh:
            json.dump(out, fh)
        os.replace(path + ".tmp", path)
        print(name, "step", cp, "written", round(time.time() - t0), "s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
