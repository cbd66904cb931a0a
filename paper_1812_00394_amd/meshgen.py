"""Seeded synthetic meshes: the only module that both the oracle and the HIP path read.

It produces *inputs* only — node coordinates, cell-to-node lists and tagged boundary edges —
and holds none of the method's arithmetic (no areas, normals, gradients or fluxes; each side
derives those itself).  Every generator is deterministic for a given seed (numpy PCG64).

Mesh dictionary (all numpy, C-contiguous):
  nodes          float64 [n_nodes, 2]
  cell_ptr       int64   [n_cells + 1]   CSR offsets into cell_nodes
  cell_nodes     int64   [nnz]           3 or 4 node ids per cell, counter-clockwise
  bface_nodes    int64   [n_bfaces, 2]   boundary edges (any orientation)
  bface_group    int32   [n_bfaces]      group id of each boundary edge
  group_kind     int32   [n_groups]      WALL=1 MOVING_WALL=2 INLET=3 OUTLET=4 FARFIELD=5 PERIODIC=6
  periodic_shift float64 [n_groups, 2]   for PERIODIC groups: the translation that maps this
                                         group's edges onto their partner edges
  name           str
The paper's own meshes (Salome-generated cavity, backward-facing step and NACA0012 grids of its
numerical-experiments section) are not available; these generators stand in for them.
"""
from __future__ import annotations

import numpy as np

WALL, MOVING_WALL, INLET, OUTLET, FARFIELD, PERIODIC = 1, 2, 3, 4, 5, 6


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _finish(nodes, cells, bfaces, bgroups, kinds, shifts=None, name=""):
    """Pack python lists / arrays into the mesh dictionary, dropping unused nodes."""
    if isinstance(cells, np.ndarray) and cells.ndim == 2:
        cell_ptr = np.arange(cells.shape[0] + 1, dtype=np.int64) * cells.shape[1]
        cell_nodes = cells.reshape(-1).astype(np.int64)
    else:
        lens = np.array([len(c) for c in cells], dtype=np.int64)
        cell_ptr = np.zeros(len(cells) + 1, dtype=np.int64)
        np.cumsum(lens, out=cell_ptr[1:])
        cell_nodes = np.concatenate([np.asarray(c, dtype=np.int64) for c in cells])
    bfaces = np.asarray(bfaces, dtype=np.int64).reshape(-1, 2)
    used = np.zeros(len(nodes), dtype=bool)
    used[cell_nodes] = True
    remap = -np.ones(len(nodes), dtype=np.int64)
    remap[used] = np.arange(int(used.sum()), dtype=np.int64)
    nodes = np.ascontiguousarray(np.asarray(nodes, dtype=np.float64)[used])
    cell_nodes = remap[cell_nodes]
    bfaces = remap[bfaces]
    assert (bfaces >= 0).all(), "boundary edge references a node of no cell"
    ng = len(kinds)
    if shifts is None:
        shifts = np.zeros((ng, 2))
    return dict(nodes=nodes, cell_ptr=cell_ptr, cell_nodes=np.ascontiguousarray(cell_nodes),
                bface_nodes=np.ascontiguousarray(bfaces),
                bface_group=np.ascontiguousarray(np.asarray(bgroups, dtype=np.int32)),
                group_kind=np.asarray(kinds, dtype=np.int32),
                periodic_shift=np.ascontiguousarray(np.asarray(shifts, dtype=np.float64).reshape(ng, 2)),
                name=name)


def _lattice_cells(nx, ny, split, rng, keep=None):
    """Cells of an (nx+1) x (ny+1) node lattice (node id = j*(nx+1)+i).

    split: 'none' (quads), 'random' (each quad cut along a seeded diagonal) or a boolean
    [ny, nx] array selecting which quads are cut (the diagonal still seeded).
    keep: optional boolean [ny, nx] mask of the quads that exist.
    Returns a list of CCW node tuples.
    """
    cells = []
    if isinstance(split, str):
        cut = np.full((ny, nx), split == "random")
    else:
        cut = split
    diag = rng.integers(0, 2, size=(ny, nx)) if rng is not None else np.zeros((ny, nx), dtype=np.int64)
    for j in range(ny):
        for i in range(nx):
            if keep is not None and not keep[j, i]:
                continue
            a = j * (nx + 1) + i          # (i, j)
            b = a + 1                     # (i+1, j)
            c = b + (nx + 1)              # (i+1, j+1)
            d = a + (nx + 1)              # (i, j+1)
            if not cut[j, i]:
                cells.append((a, b, c, d))
            elif diag[j, i] == 0:
                cells.append((a, b, c))
                cells.append((a, c, d))
            else:
                cells.append((a, b, d))
                cells.append((b, c, d))
    return cells


def _sides(nx, ny):
    """Boundary edges of the full lattice, per side, as (a, b) node pairs."""
    w = nx + 1
    bottom = [(i, i + 1) for i in range(nx)]
    top = [(ny * w + i, ny * w + i + 1) for i in range(nx)]
    left = [(j * w, (j + 1) * w) for j in range(ny)]
    right = [(j * w + nx, (j + 1) * w + nx) for j in range(ny)]
    return bottom, right, top, left


def _jitter(nodes, nx, ny, amp, rng, movable=None):
    """Independent uniform perturbation U(-amp, amp) per component of interior lattice nodes."""
    nodes = nodes.copy()
    J, I = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    interior = (I > 0) & (I < nx) & (J > 0) & (J < ny)
    if movable is not None:
        interior &= movable
    noise = rng.uniform(-1.0, 1.0, size=(ny + 1, nx + 1, 2))
    amp = np.broadcast_to(np.asarray(amp, dtype=np.float64), (ny + 1, nx + 1, 2)) if np.ndim(amp) else amp
    pert = noise * amp
    nodes = nodes.reshape(ny + 1, nx + 1, 2)
    nodes[interior] += pert[interior]
    return nodes.reshape(-1, 2)


def lattice_nodes(xs, ys):
    X, Y = np.meshgrid(np.asarray(xs, float), np.asarray(ys, float), indexing="xy")
    return np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)


# ----------------------------------------------------------------------------------------------
# Lid-driven cavity (laminar case): unit square, n x n quads cut along seeded diagonals,
# interior nodes jittered by U(-jitter*h, jitter*h) per component.  Group 0: the three
# resting walls, group 1: the moving lid (y = 1).
# ----------------------------------------------------------------------------------------------
def cavity(n=48, jitter=0.15, seed=1, split="random"):
    rng = _rng(seed)
    h = 1.0 / n
    nodes = lattice_nodes(np.linspace(0, 1, n + 1), np.linspace(0, 1, n + 1))
    cells = _lattice_cells(n, n, split, rng)
    nodes = _jitter(nodes, n, n, jitter * h, rng)
    bottom, right, top, left = _sides(n, n)
    bf = bottom + right + left + top
    bg = [0] * (len(bottom) + len(right) + len(left)) + [1] * len(top)
    return _finish(nodes, cells, bf, bg, [WALL, MOVING_WALL], name=f"cavity{n}")


# ----------------------------------------------------------------------------------------------
# Rectangles for the analytic-flow pins.
#   kind='periodic'  : periodic in x and y (Taylor-Green vortex, free-stream tests)
#   kind='couette'   : periodic in x, resting wall at y=0 (group 2), moving wall at y=Ly (group 3)
#   kind='channel'   : inlet x=0 (group 0), outlet x=Lx (group 1), walls y=0 / y=Ly (group 2)
#   kind='duct'      : inlet x=0 (group 0), outlet x=Lx (group 1), far field y=0 / y=Ly (group 2)
#   kind='open'      : far field on all four sides (group 0)
# ----------------------------------------------------------------------------------------------
def rectangle(nx, ny, Lx=1.0, Ly=1.0, kind="periodic", split="random", jitter=0.0, seed=0):
    rng = _rng(seed)
    nodes = lattice_nodes(np.linspace(0, Lx, nx + 1), np.linspace(0, Ly, ny + 1))
    cells = _lattice_cells(nx, ny, split, rng)
    if jitter:
        nodes = _jitter(nodes, nx, ny, np.array([jitter * Lx / nx, jitter * Ly / ny]), rng)
    bottom, right, top, left = _sides(nx, ny)
    if kind == "periodic":
        bf = left + right + bottom + top
        bg = [0] * ny + [1] * ny + [2] * nx + [3] * nx
        kinds = [PERIODIC] * 4
        shifts = [(Lx, 0.0), (-Lx, 0.0), (0.0, Ly), (0.0, -Ly)]
    elif kind == "couette":
        bf = left + right + bottom + top
        bg = [0] * ny + [1] * ny + [2] * nx + [3] * nx
        kinds = [PERIODIC, PERIODIC, WALL, MOVING_WALL]
        shifts = [(Lx, 0.0), (-Lx, 0.0), (0.0, 0.0), (0.0, 0.0)]
    elif kind == "channel":
        bf = left + right + bottom + top
        bg = [0] * ny + [1] * ny + [2] * (2 * nx)
        kinds = [INLET, OUTLET, WALL]
        shifts = None
    elif kind == "duct":
        bf = left + right + bottom + top
        bg = [0] * ny + [1] * ny + [2] * (2 * nx)
        kinds = [INLET, OUTLET, FARFIELD]
        shifts = None
    elif kind == "open":
        bf = left + right + bottom + top
        bg = [0] * (2 * nx + 2 * ny)
        kinds = [FARFIELD]
        shifts = None
    else:
        raise ValueError(kind)
    return _finish(nodes, cells, bf, bg, kinds, shifts, name=f"{kind}{nx}x{ny}")


# ----------------------------------------------------------------------------------------------
# Backward-facing-step-like channel (turbulent case).  Inlet channel x in [-4h, 0], y in [h, 2h];
# downstream x in [0, 26h], y in [0, 2h] (domain 30h x 2h).  Quads with geometric wall
# stretching (ratio 1.12, first spacing y1) near every wall; away from walls the quads are cut
# into triangles along seeded diagonals and their nodes jittered.
# Groups: 0 wall (all solid walls), 1 inlet (x=-4h), 2 outlet (x=26h).
# ----------------------------------------------------------------------------------------------
def _graded(a, b, d_end, ratio, d_core, both=True):
    """1-D node positions on [a, b]: geometric growth from spacing d_end at a (and at b when
    both=True) by `ratio` until the spacing reaches d_core, uniform core in between."""
    L = b - a
    grow = []
    s = d_end
    while s < d_core and sum(grow) + s < (0.45 if both else 0.9) * L:
        grow.append(s)
        s *= ratio
    grow = np.array(grow)
    used = grow.sum() * (2 if both else 1)
    n_core = max(1, int(round((L - used) / d_core)))
    core = np.full(n_core, (L - used) / n_core)
    steps = np.concatenate([grow, core, grow[::-1]]) if both else np.concatenate([grow, core])
    x = a + np.concatenate([[0.0], np.cumsum(steps)])
    x[-1] = b
    return x


def backstep(h=1.0, y1=5.4e-4, ratio=1.12, core=0.035, dx_core=0.058, dx_corner=0.004,
             wall_layers=24, jitter=0.15, seed=2):
    rng = _rng(seed)
    # y: lower block [0, h] and upper block [h, 2h], clustered at 0, h and 2h.
    y_lo = _graded(0.0, h, y1 * h, ratio, core * h)
    y_up = _graded(h, 2 * h, y1 * h, ratio, core * h)
    ys = np.concatenate([y_lo, y_up[1:]])
    # x: clustered at the step corner x = 0 from both sides, uniform elsewhere.
    x_in = _graded(-4 * h, 0.0, dx_corner * h, ratio, dx_core * h, both=False)[::-1]
    x_in = -4 * h + (0.0 - x_in)  # mirror so the clustering sits at x = 0
    x_in = np.sort(x_in)
    x_dn = _graded(0.0, 26 * h, dx_corner * h, ratio, dx_core * h, both=False)
    xs = np.concatenate([x_in, x_dn[1:]])
    nx, ny = len(xs) - 1, len(ys) - 1
    i0 = int(np.argmin(np.abs(xs)))          # node column at x = 0
    jh = int(np.argmin(np.abs(ys - h)))      # node row at y = h
    keep = np.ones((ny, nx), dtype=bool)
    keep[:jh, :i0] = False                   # the step itself (x < 0, y < h)
    # distance (in cell rows/columns) to the nearest wall, to decide quads vs triangles
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    rows_to_wall = np.minimum(J, ny - 1 - J)               # bottom / top walls
    rows_to_wall = np.where(I < i0, np.minimum(ny - 1 - J, J - jh), rows_to_wall)  # inlet channel
    # the grid lines clustered like walls (y = h downstream of the step, x = 0 above it) keep quads
    # as well: their thin cells cut in two would be sliver triangles
    rows_to_line = np.where(I >= i0, np.where(J >= jh, J - jh, jh - 1 - J), 10 ** 6)
    cols_to_step = np.where(I >= i0, I - i0, i0 - 1 - I)
    split = (rows_to_wall >= wall_layers) & (rows_to_line >= wall_layers) & (cols_to_step >= wall_layers) & keep
    nodes = lattice_nodes(xs, ys)
    cells = _lattice_cells(nx, ny, split, rng, keep=keep)
    # jitter only the nodes surrounded by triangle cells (core), by a fraction of local spacing
    movable = np.zeros((ny + 1, nx + 1), dtype=bool)
    core_nodes = np.zeros((ny + 1, nx + 1), dtype=np.int64)
    for dj in (0, 1):
        for di in (0, 1):
            core_nodes[dj:ny + dj, di:nx + di] += split
    movable = core_nodes == 4
    dxl = np.minimum(np.diff(xs)[np.clip(np.arange(nx + 1) - 1, 0, nx - 1)], np.diff(xs)[np.clip(np.arange(nx + 1), 0, nx - 1)])
    dyl = np.minimum(np.diff(ys)[np.clip(np.arange(ny + 1) - 1, 0, ny - 1)], np.diff(ys)[np.clip(np.arange(ny + 1), 0, ny - 1)])
    amp = np.stack(np.broadcast_arrays(dxl[None, :], dyl[:, None]), axis=-1) * jitter
    nodes = _jitter(nodes, nx, ny, amp, rng, movable=movable)
    w = nx + 1
    nid = lambda i, j: j * w + i
    walls, inlet, outlet = [], [], []
    for i in range(nx):
        if i >= i0:
            walls.append((nid(i, 0), nid(i + 1, 0)))          # bottom wall downstream
        else:
            walls.append((nid(i, jh), nid(i + 1, jh)))        # inlet channel floor
        walls.append((nid(i, ny), nid(i + 1, ny)))            # top wall
    for j in range(jh):
        walls.append((nid(i0, j), nid(i0, j + 1)))            # step face
    for j in range(jh, ny):
        inlet.append((nid(0, j), nid(0, j + 1)))
    for j in range(ny):
        outlet.append((nid(nx, j), nid(nx, j + 1)))
    bf = walls + inlet + outlet
    bg = [0] * len(walls) + [1] * len(inlet) + [2] * len(outlet)
    return _finish(nodes, cells, bf, bg, [WALL, INLET, OUTLET], name="backstep")


# ----------------------------------------------------------------------------------------------
# O-mesh around a NACA 4-digit symmetric section (sharp trailing edge), chord 1, leading edge at
# the origin.  n_wall cells around the section (cosine-clustered at LE and TE), n_normal layers
# growing geometrically from y1 to a circle of radius `radius` centred at mid-chord.
# Groups: 0 wall (the section), 1 far field.
# ----------------------------------------------------------------------------------------------
def naca_thickness(x, t=0.12):
    return 5 * t * (0.2969 * np.sqrt(x) - 0.1260 * x - 0.3516 * x ** 2 + 0.2843 * x ** 3 - 0.1036 * x ** 4)


def geometric_ratio(y1, n, total):
    """Solve y1 * (r^n - 1)/(r - 1) = total for r > 1 by bisection."""
    lo, hi = 1.0 + 1e-12, 2.0
    for _ in range(200):
        r = 0.5 * (lo + hi)
        s = y1 * (r ** n - 1) / (r - 1)
        lo, hi = (r, hi) if s < total else (lo, r)
    return 0.5 * (lo + hi)


def naca_omesh(n_wall=512, n_normal=384, t=0.12, y1=4.5e-6, radius=20.0, blend=0.2):
    assert n_wall % 2 == 0
    half = n_wall // 2
    # wall points: TE -> lower surface -> LE -> upper surface -> TE (counter-clockwise seen from
    # outside would be clockwise; orientation fixed below)
    beta = np.linspace(0.0, np.pi, half + 1)
    xc = 0.5 * (1 + np.cos(beta))           # 1 -> 0 (TE to LE)
    yt = naca_thickness(xc, t)
    yt[0] = 0.0
    lower = np.stack([xc, -yt], axis=1)                  # TE -> LE along the lower surface
    upper = np.stack([xc[::-1], yt[::-1]], axis=1)       # LE -> TE along the upper surface
    wall = np.concatenate([lower[:-1], upper[:-1]])      # n_wall points, closed loop
    # outward normals from the polygon (central differences), TE normal along +x
    nxt = np.roll(wall, -1, axis=0)
    prv = np.roll(wall, 1, axis=0)
    tang = nxt - prv
    nrm = np.stack([-tang[:, 1], tang[:, 0]], axis=1)  # loop TE->lower->LE->upper is clockwise
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    nrm[0] = (1.0, 0.0)
    if np.dot(nrm[half // 2], np.array([0.0, -1.0])) < 0:   # lower-surface normal must point down
        nrm = -nrm
        nrm[0] = (1.0, 0.0)
    centre = np.array([0.5, 0.0])
    ang = np.arctan2(wall[:, 1] - centre[1], wall[:, 0] - centre[0])
    outer = centre + radius * np.stack([np.cos(ang), np.sin(ang)], axis=1)
    r = geometric_ratio(y1, n_normal, radius)
    eta = np.concatenate([[0.0], y1 * (r ** np.arange(1, n_normal + 1) - 1) / (r - 1)])
    eta = eta / eta[-1]                                   # fraction of the wall-to-circle distance
    R = np.linalg.norm(outer - wall, axis=1)
    radial = (outer - wall) / R[:, None]
    nodes = np.zeros((n_normal + 1, n_wall, 2))
    for j in range(n_normal + 1):
        s = eta[j] * radius
        b = 1.0 - np.exp(-s / blend)                      # 0 at the wall (normal), -> 1 (radial)
        d = (1 - b) * nrm + b * radial
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        pts_normal = wall + (eta[j] * R)[:, None] * d
        pts_lin = wall + eta[j] * (outer - wall)
        g = min(1.0, eta[j] * 4.0)                        # fade to straight interpolation far out
        nodes[j] = (1 - g) * pts_normal + g * pts_lin
    nodes[-1] = outer
    nodes = nodes.reshape(-1, 2)
    nid = lambda i, j: j * n_wall + (i % n_wall)
    cells = []
    for j in range(n_normal):
        for i in range(n_wall):
            cells.append((nid(i, j), nid(i + 1, j), nid(i + 1, j + 1), nid(i, j + 1)))
    cells = np.array(cells, dtype=np.int64)
    # orientation: make every cell counter-clockwise
    p = nodes[cells]
    area = 0.5 * np.sum(p[:, :, 0] * np.roll(p[:, :, 1], -1, axis=1) - np.roll(p[:, :, 0], -1, axis=1) * p[:, :, 1], axis=1)
    if np.median(area) < 0:
        cells = cells[:, ::-1].copy()
    bf = [(nid(i, 0), nid(i + 1, 0)) for i in range(n_wall)]
    bf += [(nid(i, n_normal), nid(i + 1, n_normal)) for i in range(n_wall)]
    bg = [0] * n_wall + [1] * n_wall
    m = _finish(nodes, cells, bf, bg, [WALL, FARFIELD], name=f"naca_omesh{n_wall}x{n_normal}")
    m["meta_ratio"] = r
    return m


# ----------------------------------------------------------------------------------------------
# Throughput-stress mesh: Delaunay triangulation of stratified-jittered points in a Lx x H
# rectangle, point density graded linearly from `grade` (at y=0) to 1 (at y=H).
# Groups: 0 wall (y=0 and y=H), 1 inlet (x=0), 2 outlet (x=Lx).
# ----------------------------------------------------------------------------------------------
def delaunay_rect(n_points=2_000_000, Lx=4.0, H=1.0, grade=3.0, seed=5):
    from scipy.spatial import Delaunay
    rng = _rng(seed)
    # rows: density proportional to (grade - (grade-1) y/H); choose ny, nx so ny*nx ~ n_points
    a, b = grade, 1.0 - grade        # density g(s) = a + b s on s in [0,1]
    area = a + 0.5 * b

    def rows(ny):
        # inverse CDF of the linear density for the row positions:
        # solve a s + b s^2/2 = q * area for s
        q = np.linspace(0.0, 1.0, ny + 1)
        s = (-a + np.sqrt(a * a + 2 * b * q * area)) / b if b != 0 else q
        return s * H

    def row_spacing(ys, j, ny):
        return (ys[min(j + 1, ny)] - ys[max(j - 1, 0)]) / (2 if 0 < j < ny else 1)

    ny = int(round(np.sqrt(n_points * H / Lx)))
    for _ in range(3):               # points grow like ny^2: rescale ny to hit n_points
        ys = rows(ny)
        total = sum(int(round(Lx / row_spacing(ys, j, ny))) + 1 for j in range(ny + 1))
        ny = max(2, int(round(ny * np.sqrt(n_points / total))))
    ys = rows(ny)
    pts = []
    for j in range(ny + 1):
        dy_loc = row_spacing(ys, j, ny)
        nx_j = max(4, int(round(Lx / dy_loc)))
        xs = np.linspace(0.0, Lx, nx_j + 1)
        if 0 < j < ny:
            dx = Lx / nx_j
            xj = xs[1:-1] + rng.uniform(-0.3, 0.3, size=nx_j - 1) * dx
            yj = ys[j] + rng.uniform(-0.3, 0.3, size=nx_j - 1) * dy_loc
            pts.append(np.stack([np.concatenate([[0.0], xj, [Lx]]),
                                 np.concatenate([[ys[j]], yj, [ys[j]]])], axis=1))
        else:
            pts.append(np.stack([xs, np.full_like(xs, ys[j])], axis=1))
    pts = np.concatenate(pts)
    tri = Delaunay(pts, qhull_options="Qbb Qc Qz Q12")
    cells = tri.simplices.astype(np.int64)
    p = pts[cells]
    area = 0.5 * ((p[:, 1, 0] - p[:, 0, 0]) * (p[:, 2, 1] - p[:, 0, 1]) - (p[:, 2, 0] - p[:, 0, 0]) * (p[:, 1, 1] - p[:, 0, 1]))
    flip = area < 0
    cells[flip] = cells[flip][:, ::-1]
    # boundary edges = edges used by exactly one triangle
    e = np.concatenate([cells[:, [0, 1]], cells[:, [1, 2]], cells[:, [2, 0]]])
    key = np.sort(e, axis=1)
    uniq, inv, cnt = np.unique(key, axis=0, return_inverse=True, return_counts=True)
    bedges = uniq[cnt == 1]
    mid = 0.5 * (pts[bedges[:, 0]] + pts[bedges[:, 1]])
    tol = 1e-9 * max(Lx, H)
    grp = np.full(len(bedges), -1, dtype=np.int32)
    grp[(np.abs(mid[:, 1]) < tol) | (np.abs(mid[:, 1] - H) < tol)] = 0
    grp[np.abs(mid[:, 0]) < tol] = 1
    grp[np.abs(mid[:, 0] - Lx) < tol] = 2
    assert (grp >= 0).all(), "a hull edge lies off the rectangle"
    return _finish(pts, cells, bedges, grp, [WALL, INLET, OUTLET], name=f"delaunay{len(cells)}")


def save(mesh, path):
    np.savez(path, **{k: v for k, v in mesh.items() if k != "name"}, name=np.array(mesh["name"]))


def load(path):
    with np.load(path, allow_pickle=False) as z:
        m = {k: z[k] for k in z.files}
    m["name"] = str(m["name"])
    return m
