"""CPU tests of the C-ABI library's host side (no GPU needed): it loads, exports every symbol the
header declares, and its FP64 mesh preprocessing agrees with the oracle's geometry; malformed
meshes are rejected with FVLBM_EMESH."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import fvlbm_oracle as O
from paper_1812_00394_amd import fvlbm as F
from paper_1812_00394_amd import meshgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "fvlbm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fvlbm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = F.lib()
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name
    assert sorted(F.EXPORTS) == names


MESHES = {
    "cavity": lambda: mg.cavity(n=12, jitter=0.2, seed=3),
    "periodic": lambda: mg.rectangle(7, 5, kind="periodic", jitter=0.2, seed=4),
    "channel": lambda: mg.rectangle(9, 6, Lx=2.0, kind="channel", jitter=0.2, seed=5),
    "backstep": lambda: mg.backstep(core=0.25, dx_core=0.5, y1=1e-2, dx_corner=0.05, wall_layers=3),
    "naca": lambda: mg.naca_omesh(n_wall=32, n_normal=12, y1=1e-3),
}


@pytest.mark.parametrize("name", sorted(MESHES))
@pytest.mark.parametrize("order", ["none", "morton", "rcm", "tiles"])
def test_geometry_matches_oracle(name, order):
    m = MESHES[name]()
    M = F.Mesh(m, order=order)
    G = O.Geometry(m)
    area, cen, wd = M.geometry()
    np.testing.assert_allclose(area, G.area, rtol=1e-12)
    np.testing.assert_allclose(cen, G.xc, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(wd, G.wall_dist, rtol=1e-12, atol=1e-15)
    p = M.permutation()
    assert sorted(p.tolist()) == list(range(G.n))
    assert M.n_cells == G.n
    assert M.n_boundary_edges == int((~G.interior).sum())
    assert M.n_interior_edges == int(G.interior.sum()) // 2


def test_morton_order_is_local():
    m = mg.cavity(n=32, jitter=0.1, seed=1)
    G = O.Geometry(m)
    for order, bound in (("morton", 0.2), ("none", None)):
        p = F.Mesh(m, order=order).permutation()
        jumps = np.linalg.norm(np.diff(G.xc[p], axis=0), axis=1)
        if bound is not None:
            assert np.median(jumps) < bound / 4


def _broken(kind):
    m = mg.cavity(n=4, jitter=0.0, seed=0, split="none")
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    if kind == "clockwise":
        cn = m["cell_nodes"].reshape(-1, 4)
        cn[3] = cn[3, ::-1]
        m["cell_nodes"] = cn.reshape(-1)
    elif kind == "missing_bface":
        m["bface_nodes"] = m["bface_nodes"][1:]
        m["bface_group"] = m["bface_group"][1:]
    elif kind == "extra_bface":
        m["bface_nodes"] = np.concatenate([m["bface_nodes"], [[6, 7]]])
        m["bface_group"] = np.concatenate([m["bface_group"], [0]]).astype(np.int32)
    elif kind == "triple_edge":
        cn = m["cell_nodes"].reshape(-1, 4)
        m["cell_nodes"] = np.concatenate([cn, cn[5:6]]).reshape(-1)
        m["cell_ptr"] = np.arange(len(m["cell_nodes"]) // 4 + 1, dtype=np.int64) * 4
    elif kind == "periodic_unpaired":
        m["group_kind"] = np.array([mg.PERIODIC, mg.MOVING_WALL], dtype=np.int32)
        m["periodic_shift"] = np.array([[0.37, 0.0], [0.0, 0.0]])
    return m


@pytest.mark.parametrize("kind", ["clockwise", "missing_bface", "extra_bface", "triple_edge", "periodic_unpaired"])
def test_malformed_mesh_rejected(kind):
    with pytest.raises(F.FvlbmError) as e:
        F.Mesh(_broken(kind))
    assert e.value.status == -2, str(e.value)
    with pytest.raises(ValueError):
        O.Geometry(_broken(kind))


def test_invalid_arguments():
    L = F.lib()
    out = ctypes.c_void_p()
    assert L.fvlbm_mesh_create(0, None, 0, None, None, 0, None, None, 0, None, None, 0, ctypes.byref(out)) == -1
    assert b"empty" in L.fvlbm_last_error()
    m = mg.cavity(n=4)
    M = F.Mesh(m)
    size = ctypes.c_size_t()
    assert L.fvlbm_state_bytes(M.handle, 7, 0, ctypes.byref(size)) == -1
    # a laminar FP64 state needs O(n) bytes: at least f, three stage buffers and the gradients
    b64 = M.state_bytes("fp64")
    b32 = M.state_bytes("fp32dev")
    assert b64 > (9 * 4 + 16) * 8 * M.n_cells
    assert b32 < b64
    # FP32 storage with FP64 geometry: the FP32 state plus FP64 copies of the streamed geometry
    assert M.state_bytes("fp32dev_geo64") >= b32 + (8 * 4 + 10) * 8 * M.n_cells


def test_wide_halo_backstep_tiles():
    """The mesh of the wide-halo GPU tests: its 256-cell Morton tiles (the order those tests use)
    have at most 256 ring-1 cells (one thread each) but more than 256 cells in ring 1 + ring 2,
    so the ring kernels must loop over the ring-2 cells beyond one per thread."""
    import scipy.sparse as sp
    m = mg.backstep(core=0.3, dx_core=0.6, dx_corner=0.02, y1=1e-3)
    M = F.Mesh(m, order="morton")
    perm = M.permutation()
    n = len(perm)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    G = O.Geometry(m)
    inner = np.nonzero(G.interior)[0]
    A = sp.csr_matrix((np.ones(len(inner)), (inv[G.cell[inner]], inv[G.nbr[inner]])), shape=(n, n))
    r1, ext = [], []
    for t in range((n + 255) // 256):
        cells = np.arange(t * 256, min(n, t * 256 + 256))
        h1 = np.setdiff1d(np.unique(A[cells].indices), cells)
        h2 = np.setdiff1d(np.unique(A[h1].indices), np.concatenate([cells, h1]))
        r1.append(len(h1))
        ext.append(len(h1) + len(h2))
    assert max(r1) <= 256 < max(ext), (max(r1), max(ext))


def _tile_rings(m, order):
    """Ring-1 and ring-1 + ring-2 cell counts of every 256-cell tile of the library's renumbering."""
    import scipy.sparse as sp
    M = F.Mesh(m, order=order)
    perm = M.permutation()
    n = len(perm)
    inv = np.empty(n, np.int64)
    inv[perm] = np.arange(n)
    G = O.Geometry(m)
    inner = np.nonzero(G.interior)[0]
    A = sp.csr_matrix((np.ones(len(inner)), (inv[G.cell[inner]], inv[G.nbr[inner]])), shape=(n, n))
    r1, ext = [], []
    for t in range((n + 255) // 256):
        cells = np.arange(t * 256, min(n, t * 256 + 256))
        h1 = np.setdiff1d(np.unique(A[cells].indices), cells)
        h2 = np.setdiff1d(np.unique(A[h1].indices), np.concatenate([cells, h1]))
        r1.append(len(h1))
        ext.append(len(h1) + len(h2))
    return np.array(r1), np.array(ext)


def test_graph_tiles_are_compact_on_stretched_meshes():
    """The graph-grown tiles (order "tiles") on an O-mesh with thin wall cells (256 x 192 quads, first
    cell 4.5e-6 chord): Morton tiles there are strips whose ring-1 halos exceed one thread per cell;
    graph-grown tiles keep every ring-1 halo within 256 and the mean halo at less than half."""
    m = mg.naca_omesh(n_wall=256, n_normal=192, y1=4.5e-6)
    r1m, extm = _tile_rings(m, "morton")
    r1t, extt = _tile_rings(m, "tiles")
    assert r1m.max() > 256 >= r1t.max(), (r1m.max(), r1t.max())
    assert r1t.mean() < 0.5 * r1m.mean() and extt.mean() < 0.5 * extm.mean(), (r1t.mean(), r1m.mean())
