#!/usr/bin/env python3
"""Writes tests/golden/c4_piece_400.json: the oracle's derivatives of J = w . (F_x, F_y, J_R) after
400 IMEX + SST steps on the seeded piece of tests/c4case.py with respect to (theta, sigma_k1,
sigma_w1, beta*, a1), by complex step (h = 1e-30, exact to rounding) and by centred differences
(eps = 1e-6 max(|p|, 1)).  Calls only the oracle (and the seeded input module).  About 2 minutes.

    python tests/golden/make_c4_fixture.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import fvlbm_oracle as O          # noqa: E402
from tests import c4case as C                 # noqa: E402

PARAMS = ("theta", "sigma_k1", "sigma_w1", "beta_star", "a1")


def main():
    t0 = time.time()
    m = C.piece()
    G = O.Geometry(m)
    en = np.maximum(O.EX[:, None] * G.nl[:, 0] + O.EY[:, None] * G.nl[:, 1], 0.0)
    out = np.stack([np.bincount(G.cell, weights=en[a], minlength=G.n) for a in range(9)])
    courant = 1.0 / (out / G.area).max()
    U, Re = 0.05, 3.6e4
    nu = U / Re
    ng = len(m["group_kind"])            # wall, inlet, outlet of the step; the far-field cut edges
    assert ng == 4
    p = O.default_params(nu=nu, dt=min(60 * 3 * nu, 0.9 * courant), sst=True, theta=0.03,
                         group_u=[[0, 0], [U, 0], [0, 0], [0.02, 0]], group_rho=[1, 1, 1, 1],
                         group_k=[0, 1e-6, 0, 1e-6], group_w=[0, 1e-2, 0, 1e-2],
                         jr_group=0, jr_xmin=0.0, eps_tau=1e-4)
    rho, ux, uy, noise, k0, w0 = C.initial_fields(m)
    f0 = O.feq(rho, ux, uy) + 1e-5 * O.WT[:, None] * noise
    w = np.array(C.FUNCTIONAL)

    def J(pp, cplx=False):
        o = O.Oracle(m, pp)
        dt = complex if cplx else float
        fN, _, _ = o.run(f0.astype(dt), k0.astype(dt), w0.astype(dt), C.N_STEPS)
        Fv, JR = o.forces(fN, 1)
        return w[0] * Fv[0] + w[1] * Fv[1] + w[2] * JR, Fv, JR

    J0, F0, JR0 = J(p)
    cs, fd, eps_used = [], [], []
    for key in PARAMS:
        H = 1e-30
        pc = dict(p)
        pc[key] = p[key] + 1j * H
        cs.append(float(np.imag(J(pc, True)[0]) / H))
        eps = 1e-6 * max(abs(p[key]), 1.0)
        pp, pm = dict(p), dict(p)
        pp[key] = p[key] + eps
        pm[key] = p[key] - eps
        fd.append(float((J(pp)[0] - J(pm)[0]) / (2 * eps)))
        eps_used.append(eps)
        print(key, cs[-1], fd[-1], flush=True)
    fx = {
        "what": "oracle derivatives of J = w . (F_x, F_y, J_R) after the recorded run, piece of the backstep",
        "script": "tests/golden/make_c4_fixture.py",
        "mesh": m["name"], "mesh_sha256": C.mesh_sha(m), "n_cells": int(G.n),
        "n_steps": C.N_STEPS, "functional_weights": list(C.FUNCTIONAL), "wall_mask": 1,
        "params": {k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in p.items()},
        "param_names": list(PARAMS),
        "J": float(J0), "force": [float(F0[0]), float(F0[1])], "j_r": float(JR0),
        "complex_step": cs, "central_difference": fd, "fd_eps": eps_used,
        "seconds": round(time.time() - t0, 1),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_piece_400.json")
    with open(path, "w") as fh:
        json.dump(fx, fh, indent=1)
    print("wrote", path, "in", fx["seconds"], "s")


if __name__ == "__main__":
    main()
