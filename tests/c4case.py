"""Seeded inputs of the derivative check on a piece of the backward-facing step (the adjoint
workload: 400 IMEX steps with a checkpoint every 20).

The piece: the cells within R edge rings of the wall cell nearest (h, 0.01 h) behind the step of the
122,876-cell backstep mesh, R the least giving at least 800 cells.  Its original edges keep their
groups (the walls); the edges cut from the rest of the mesh form one far-field group, so that the
inflow angle (which turns far-field and inlet velocities) acts on the piece.  The initial fields are a
reversed near-wall shear stream with seeded noise, uniform-ish k and omega.  Plain numpy: mesh
plumbing and random numbers only, none of the method's arithmetic (the equilibrium that turns the
fields into f is applied by the caller)."""
import hashlib

import numpy as np

from paper_1812_00394_amd import meshgen as mg
from tests import submesh as sm

FARFIELD = 5
N_STEPS = 400
CKPT = 20
FUNCTIONAL = (0.7, -1.3, 2.0)     # J = w . (F_x, F_y, J_R)


def piece():
    mesh = mg.backstep()
    xc = sm.centroids(mesh)
    seed_cell = int(np.argmin((xc[:, 0] - 1.0) ** 2 + (xc[:, 1] - 0.01) ** 2))
    R = 1
    while sm.rings(mesh, [seed_cell], R).sum() < 800:
        R += 1
    p, cells = sm.cut(mesh, sm.rings(mesh, [seed_cell], R))
    kinds = np.array(p["group_kind"]).copy()
    kinds[-1] = FARFIELD
    p["group_kind"] = kinds
    p["name"] = f"{len(cells)}-cell piece of the backstep ({R} rings), far-field cut edges"
    return p


def mesh_sha(m):
    h = hashlib.sha256()
    for key in ("nodes", "cell_ptr", "cell_nodes", "bface_nodes", "bface_group", "group_kind"):
        h.update(np.ascontiguousarray(m[key]).tobytes())
    return h.hexdigest()


def initial_fields(m):
    """rho, u_x, u_y, the non-equilibrium noise [9, n] (to be scaled by 1e-5 w_a), k, omega."""
    xc = sm.centroids(m)
    n = len(xc)
    rng = np.random.default_rng(95)
    x, y = xc[:, 0], xc[:, 1]
    ux = 0.03 * np.tanh(4 * (y - 0.5)) + 0.002 * rng.standard_normal(n)
    uy = 0.003 * np.sin(3 * x) + 0.002 * rng.standard_normal(n)
    rho = 1 + 0.001 * rng.standard_normal(n)
    noise = rng.standard_normal((9, n))
    k0, w0 = 1e-6 * (1 + 0.5 * rng.random(n)), 1e-2 * (1 + 0.5 * rng.random(n))
    return rho, ux, uy, noise, k0, w0
