"""Pieces of a mesh for sampled parity checks at full size.

One IMEX step changes a cell only through cells within a few edge rings of it (the SST update
gathers two rings, each of the three stage sweeps two more).  A piece of the mesh made of every
cell within R rings of some sample cells, stepped by the oracle, therefore gives the sample
cells' new values exactly when R exceeds that reach: the piece's cut edges (made outlet edges
here) cannot influence them within the step.  The wall distance is the one quantity of a cell
that depends on the whole mesh; the oracle measures it to the whole mesh's walls
(Oracle(..., wall_segments=...)).  Plain numpy, no part of the library.
"""
import numpy as np

WALL, MOVING_WALL, OUTLET, PERIODIC = 1, 2, 4, 6


def _edges(mesh):
    """Half-edges (cell, node a, node b, edge key) and the interior edges as cell pairs with the
    node pair of the first cell's half-edge."""
    ptr = np.asarray(mesh["cell_ptr"], np.int64)
    cn = np.asarray(mesh["cell_nodes"], np.int64)
    n = len(ptr) - 1
    nv = np.diff(ptr)
    cell = np.repeat(np.arange(n), nv)
    local = np.arange(len(cn)) - ptr[cell]
    nxt = ptr[cell] + (local + 1) % nv[cell]
    a, b = cn, cn[nxt]
    nn = len(mesh["nodes"]) + 1
    key = np.minimum(a, b) * nn + np.maximum(a, b)
    o = np.argsort(key, kind="stable")
    ks = key[o]
    same = np.nonzero(ks[1:] == ks[:-1])[0]
    pairs = np.stack([cell[o[same]], cell[o[same + 1]]], axis=1)
    pair_nodes = np.stack([a[o[same]], b[o[same]]], axis=1)
    return cell, key, pairs, pair_nodes


def rings(mesh, seeds, R):
    """Boolean mask of the cells within R edge rings of the seed cells."""
    import scipy.sparse as sp
    if np.any(np.asarray(mesh["group_kind"]) == PERIODIC):
        raise ValueError("periodic meshes are not supported")
    n = len(mesh["cell_ptr"]) - 1
    _, _, pairs, _ = _edges(mesh)
    A = sp.csr_matrix((np.ones(2 * len(pairs)), (np.r_[pairs[:, 0], pairs[:, 1]], np.r_[pairs[:, 1], pairs[:, 0]])),
                      shape=(n, n))
    mask = np.zeros(n, bool)
    mask[np.asarray(seeds)] = True
    front = mask.copy()
    for _ in range(R):
        reach = (A @ front.astype(np.float64)) > 0
        front = reach & ~mask
        mask |= reach
    return mask


def cut(mesh, mask):
    """The cells in mask as a mesh of their own: the original boundary edges of those cells keep
    their groups; edges to cells outside the mask become outlet edges of one extra group (the
    last).  Returns (piece, cells) with cells[i] the original index of piece cell i."""
    ptr = np.asarray(mesh["cell_ptr"], np.int64)
    cn = np.asarray(mesh["cell_nodes"], np.int64)
    cells = np.nonzero(mask)[0]
    nv = np.diff(ptr)[cells]
    new_ptr = np.r_[0, np.cumsum(nv)]
    idx = np.concatenate([np.arange(ptr[c], ptr[c + 1]) for c in cells]) if len(cells) else np.zeros(0, np.int64)
    old_nodes = cn[idx]
    used, new_cn = np.unique(old_nodes, return_inverse=True)
    nodes = np.asarray(mesh["nodes"], np.float64)[used]
    # boundary edges: original ones owned by kept cells, plus the cut edges
    cell, key, pairs, pair_nodes = _edges(mesh)
    bfn = np.asarray(mesh["bface_nodes"], np.int64)
    bgrp = np.asarray(mesh["bface_group"], np.int64)
    nn = len(mesh["nodes"]) + 1
    bkey = np.minimum(bfn[:, 0], bfn[:, 1]) * nn + np.maximum(bfn[:, 0], bfn[:, 1])
    keep_b = np.isin(bkey, key[mask[cell]])
    is_cut = mask[pairs[:, 0]] != mask[pairs[:, 1]]
    cut_nodes = pair_nodes[is_cut]
    n_groups = len(mesh["group_kind"])
    bf_nodes = np.concatenate([bfn[keep_b], cut_nodes])
    bf_group = np.concatenate([bgrp[keep_b], np.full(len(cut_nodes), n_groups)])
    piece = {
        "nodes": nodes,
        "cell_ptr": new_ptr,
        "cell_nodes": new_cn.astype(np.int64),
        "bface_nodes": np.searchsorted(used, bf_nodes),
        "bface_group": bf_group,
        "group_kind": np.r_[np.asarray(mesh["group_kind"]), OUTLET],
        "periodic_shift": np.zeros((n_groups + 1, 2)),
        "name": f"piece of {mesh.get('name', 'mesh')} ({len(cells)} cells)",
    }
    return piece, cells


def wall_segments(mesh):
    """[m, 2, 2] end points of the mesh's WALL / MOVING_WALL boundary edges."""
    kinds = np.asarray(mesh["group_kind"])
    bfn = np.asarray(mesh["bface_nodes"], np.int64)
    sel = np.isin(kinds[np.asarray(mesh["bface_group"], np.int64)], [WALL, MOVING_WALL])
    nodes = np.asarray(mesh["nodes"], np.float64)
    return np.stack([nodes[bfn[sel, 0]], nodes[bfn[sel, 1]]], axis=1)


def centroids(mesh):
    """Polygon centroids (shoelace), plain numpy."""
    ptr = np.asarray(mesh["cell_ptr"], np.int64)
    cn = np.asarray(mesh["cell_nodes"], np.int64)
    nodes = np.asarray(mesh["nodes"], np.float64)
    n = len(ptr) - 1
    nv = np.diff(ptr)
    cell = np.repeat(np.arange(n), nv)
    local = np.arange(len(cn)) - ptr[cell]
    nxt = ptr[cell] + (local + 1) % nv[cell]
    p, q = nodes[cn], nodes[cn[nxt]]
    cross = p[:, 0] * q[:, 1] - q[:, 0] * p[:, 1]
    area = np.bincount(cell, weights=cross, minlength=n) * 0.5
    cx = np.bincount(cell, weights=(p[:, 0] + q[:, 0]) * cross, minlength=n) / (6 * area)
    cy = np.bincount(cell, weights=(p[:, 1] + q[:, 1]) * cross, minlength=n) / (6 * area)
    return np.stack([cx, cy], axis=1)


def boundary_cells(mesh, group):
    """Cells owning a boundary edge of the given group."""
    cell, key, _, _ = _edges(mesh)
    bfn = np.asarray(mesh["bface_nodes"], np.int64)
    sel = np.asarray(mesh["bface_group"]) == group
    nn = len(mesh["nodes"]) + 1
    bkey = np.minimum(bfn[sel, 0], bfn[sel, 1]) * nn + np.maximum(bfn[sel, 0], bfn[sel, 1])
    return np.unique(cell[np.isin(key, bkey)])
