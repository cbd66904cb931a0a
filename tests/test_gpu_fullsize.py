"""Parity at the benchmark's full size and launch configuration: the 4.0M-cell graded Delaunay
rectangle with SST, the developed-stream initial state, the cell renumbering (graph-grown tiles) and
the sweep variant (ring-tiled) the benchmark times, one and three steps in FP64 and in FP32-deviation storage
(with FP32 or FP64 geometry), against the oracle on sampled cells.

The oracle cannot step four million cells, but one step reaches only six edge rings (measured in
test_submesh_oracle.py, which also checks the method against full oracle runs): for sample cells
in the interior, next to each wall, the inlet, the outlet and in the corners, the oracle steps the
piece of the mesh within 10 rings of them, with the wall distance measured to the whole mesh's
walls, and gives their exact new values.  Gates: FP64 1e-12 of max |f - w rho0| for f, 1e-11 for
k, omega, nu_t (the small-mesh SST gates); FP32-deviation 2e-6 of U for u and 2e-6 relative for
k and omega (the FP32 SST gate after one step)."""
import sys

import numpy as np
import pytest

import bench
from oracle import fvlbm_oracle as O
from paper_1812_00394_amd import meshgen as mg
from tests import submesh as sm

pytestmark = pytest.mark.gpu

U, H, RE = 0.05, 1.0, 3.6e4
NU = U * H / RE
DT = 6.0e-5      # about 0.9 x the advective Courant limit of this mesh (14 tau0)


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def F():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1812_00394_amd import fvlbm
    fvlbm.lib()
    return fvlbm


def _params(extra_group=False):
    gu, gr, gk, gw = [[0, 0], [U, 0], [0, 0]], [1, 1, 1], [0, 1e-6, 0], [0, 1e-2, 0]
    if extra_group:
        gu, gr, gk, gw = gu + [[0, 0]], gr + [1], gk + [1e-6], gw + [1e-2]
    return O.default_params(nu=NU, dt=DT, sst=True, group_u=gu, group_rho=gr, group_k=gk, group_w=gw)


@pytest.fixture(scope="module")
def full(F):
    say("full size: delaunay 2M points, mesh generation")
    m = mg.delaunay_rect(n_points=2_000_000, seed=5)
    n = len(m["cell_ptr"]) - 1
    assert n > 3_900_000
    xc = sm.centroids(m)
    u, k, w = bench.initial_fields(dict(profile="channel", U=U, H=H, k=1e-6, w=1e-2), xc, NU)
    rng = np.random.default_rng(11)
    bottom, inlet, outlet = sm.boundary_cells(m, 0), sm.boundary_cells(m, 1), sm.boundary_cells(m, 2)
    top = bottom[xc[bottom, 1] > 0.5 * H]
    bottom = bottom[xc[bottom, 1] <= 0.5 * H]
    corners = np.intersect1d(np.r_[inlet, outlet], np.r_[bottom, top])
    seeds = np.unique(np.r_[rng.choice(n, 6, replace=False), rng.choice(bottom, 3), rng.choice(top, 2),
                            rng.choice(inlet, 2), rng.choice(outlet, 2), corners[:4]])
    say("library mesh preprocessing")
    M = F.Mesh(m, order="tiles")
    return m, n, u, k, w, seeds, M


def _reference(full, rings, extra, steps=1):
    m, n, u, k, w, seeds, _ = full
    say("oracle on the piece within", rings, "rings of", len(seeds), "sample cells,", steps, "steps")
    piece, cells = sm.cut(m, sm.rings(m, seeds, rings))
    po = O.Oracle(piece, dict(_params(True), **extra), wall_segments=sm.wall_segments(m))
    g0, k0, w0 = po.init_state(np.ones(len(cells)), u[cells, 0], u[cells, 1], k[cells], w[cells])
    g1, k1, w1 = po.run(g0, k0, w0, steps)
    at = np.searchsorted(cells, seeds)
    _, ux, uy, _ = po.macro(g1[:, at])
    return dict(f=g1[:, at], k=k1[at], w=w1[at], nut=po.last_nut[at], ux=ux, uy=uy)


def _check(F, full, ref, extra, expect, steps=1):
    m, n, u, k, w, seeds, M = full
    for precision in ("fp64", "fp32dev", "fp32dev_geo64"):
        say(steps, "steps on the GPU,", precision, extra)
        st = F.State(M, dict(_params(), **extra), precision=precision, rho=np.ones(n), u=u, k=k, omega=w)
        st.timing(True)
        st.step(steps)
        kt = st.timing_read()
        # the benchmark's launch configuration: ring-tiled SST and sweeps
        for name, cnt in expect.items():
            assert kt[name][1] == cnt * steps, kt
        mo = st.moments()
        if precision == "fp64":
            f = st.get_f()[:, seeds]
            scale = np.abs(ref["f"] - O.WT[:, None]).max()
            err = np.abs(f - ref["f"]).max() / scale
            say("fp64 error at the samples: f", err)
            assert err < 1e-12 * steps, err
            for name, got, r in (("k", mo["k"][seeds], ref["k"]), ("omega", mo["omega"][seeds], ref["w"]),
                                 ("nu_t", mo["nu_t"][seeds], ref["nut"])):
                e = np.abs(got - r).max() / np.abs(r).max()
                assert e < 1e-11 * steps, (name, e)
        else:
            du = max(np.abs(mo["u"][seeds, 0] - ref["ux"]).max(), np.abs(mo["u"][seeds, 1] - ref["uy"]).max()) / U
            dk = np.abs(mo["k"][seeds] - ref["k"]).max() / np.abs(ref["k"]).max()
            dw = np.abs(mo["omega"][seeds] - ref["w"]).max() / np.abs(ref["w"]).max()
            say(precision, "errors at the samples: du/U", du, "dk", dk, "dw", dw)
            assert du < 2e-6 * steps and dk < 2e-6 * steps and dw < 2e-6 * steps, (du, dk, dw)
        del st


@pytest.mark.timeout(900)
def test_fullsize_sampled_parity(F, full):
    ref = _reference(full, 10, {})
    _check(F, full, ref, {}, {"sst": 1, "sweep2": 1, "collide1": 0})


@pytest.mark.timeout(900)
def test_fullsize_sampled_parity_three_steps(F, full):
    """Three steps of the benchmark's step at full size: they reach 18 edge rings, so the oracle
    steps the piece within 22 rings of the samples (which tests/test_submesh_oracle.py shows gives
    the full mesh's values bit for bit); the one-step gates times three."""
    ref = _reference(full, 22, {}, steps=3)
    _check(F, full, ref, {}, {"sst": 1, "sweep2": 1, "collide1": 0}, steps=3)


@pytest.mark.timeout(900)
def test_fullsize_sampled_parity_implicit_sst(F, full):
    """The implicit SST variant as the benchmark times it (4 Jacobi sweeps): the three sweeps after
    the system launch widen the SST's reach from 2 to 5 edge rings, so a step reaches 11 and the
    oracle steps the piece within 12 rings of the samples."""
    extra = dict(sst_sweeps=4)
    ref = _reference(full, 12, extra)
    _check(F, full, ref, extra, {"sst": 1, "sst_jacobi": 1, "sweep2": 1, "collide1": 0})


@pytest.mark.timeout(900)
def test_backstep_fullsize_parity(F):
    """The backward-facing step the benchmark times (122,876 hybrid cells, SST, 60 tau0) on the
    whole mesh, which the oracle can step: one step in FP64 and FP32-deviation storage on the ring
    path (its tiles have up to 298 ring-2 cells) against the oracle on every cell, and the FP64
    adjoint of two recorded steps with a checkpoint every step (the next segment recomputed on the
    second stream) against the oracle's complex step along one direction of the initial state."""
    H_CS = 1e-30
    mesh, flow, init, dt_frac = bench.workload("backstep")
    say("backstep full size: library preprocessing and oracle geometry")
    M = F.Mesh(mesh, order="tiles")
    p = O.default_params(**dict(flow, dt=min(flow["dt"], dt_frac * M.max_dt())))
    orc = O.Oracle(mesh, p)
    n = orc.g.n
    assert n == M.n_cells > 120_000
    rng = np.random.default_rng(12)
    x, y = orc.g.xc[:, 0], orc.g.xc[:, 1]
    ux = 0.04 + 0.01 * np.sin(0.5 * x) * np.cos(3 * y) + 0.002 * rng.standard_normal(n)
    uy = 0.004 * np.sin(2 * y) + 0.002 * rng.standard_normal(n)
    rho = 1 + 0.001 * rng.standard_normal(n)
    f0 = O.feq(rho, ux, uy) + 1e-5 * O.WT[:, None] * rng.standard_normal((9, n))
    k0 = 1e-6 * (1 + 0.5 * rng.random(n))
    w0 = 1e-2 * (1 + 0.5 * rng.random(n))
    say("oracle step")
    f1, k1, w1 = orc.step(f0, k0, w0)
    nut1 = orc.last_nut
    for precision in ("fp64", "fp32dev"):
        say("one step on the GPU,", precision)
        st = F.State(M, p, precision=precision, k=k0, omega=w0)
        st.set_state(f0, k0, w0)
        st.timing(True)
        st.step(1)
        kt = st.timing_read()
        st.timing(False)
        assert kt["sst"][1] == 1 and kt["collide1"][1] == 0, kt     # the ring path
        mo = st.moments()
        if precision == "fp64":
            err = np.abs(st.get_f() - f1).max() / np.abs(f1 - O.WT[:, None]).max()
            assert err < 1e-12, err
            for name, got, ref in (("k", mo["k"], k1), ("omega", mo["omega"], w1), ("nu_t", mo["nu_t"], nut1)):
                e = np.abs(got - ref).max() / np.abs(ref).max()
                assert e < 1e-11, (name, e)
        else:
            _, ux1, uy1, _ = orc.macro(f1)
            du = max(np.abs(mo["u"][:, 0] - ux1).max(), np.abs(mo["u"][:, 1] - uy1).max()) / 0.05
            dk = np.abs(mo["k"] - k1).max() / np.abs(k1).max()
            dw = np.abs(mo["omega"] - w1).max() / np.abs(w1).max()
            say("fp32dev errors: du/U", du, "dk", dk, "dw", dw)
            assert du < 2e-6 and dk < 2e-6 and dw < 2e-6, (du, dk, dw)
        del st
    say("FP64 adjoint of two steps against the complex step")
    st = F.State(M, p, precision="fp64", k=k0, omega=w0)
    st.set_state(f0, k0, w0)
    st.record(2, ckpt_every=1)
    lf, lk, lw = rng.standard_normal((9, n)), rng.standard_normal(n) * 1e3, rng.standard_normal(n)
    lf0, lk0, lw0, _ = st.adjoint_state(lf, lk, lw)
    vf = rng.standard_normal((9, n)) * O.WT[:, None] * 1e-3
    vk, vw = rng.standard_normal(n) * 1e-7, rng.standard_normal(n) * 1e-3
    fN, kN, wN = O.Oracle(mesh, p).run(f0 + 1j * H_CS * vf, k0 + 1j * H_CS * vk, w0 + 1j * H_CS * vw, 2)
    rhs = (np.sum(lf * np.imag(fN)) + np.sum(lk * np.imag(kN)) + np.sum(lw * np.imag(wN))) / H_CS
    lhs = np.sum(lf0 * vf) + np.sum(lk0 * vk) + np.sum(lw0 * vw)
    say("adjoint dot product", lhs, rhs)
    assert abs(lhs - rhs) <= 1e-9 * abs(rhs), (lhs, rhs)


@pytest.mark.timeout(900)
def test_airfoil_fullsize_parity(F):
    """The airfoil the benchmark times (512 x 384 O-mesh, 196,608 quads, Re 6e6, 10 degrees, about
    74 tau0, limiter on, developed near-wall start), whole mesh: one step against the oracle on every
    cell in both precisions, and the wall force (fvlbm_forces) against the oracle's in FP64."""
    say("airfoil full size: mesh, library preprocessing, oracle geometry")
    m = mg.naca_omesh()
    M = F.Mesh(m, order="tiles")
    n = M.n_cells
    _, _, wd = M.geometry()
    Uinf, c, Re, alpha = 0.05, 1.0, 6e6, np.deg2rad(10.0)
    nu = Uinf * c / Re
    kinf, winf = 1e-3 * Uinf * Uinf / Re, 5 * Uinf / c
    p = O.default_params(nu=nu, dt=min(180 * 3 * nu, 0.9 * M.max_dt()), sst=True, theta=alpha, limiter=1,
                         group_u=[[0, 0], [Uinf, 0]], group_rho=[1, 1], group_k=[0, kinf], group_w=[0, winf])
    fac = np.minimum(1.0, (wd / 0.01) ** (1 / 7))
    u0 = np.stack([Uinf * np.cos(alpha) * fac, Uinf * np.sin(alpha) * fac], axis=1)
    w0 = np.maximum(winf, 6 * nu / (0.075 * wd ** 2))
    k0 = np.full(n, kinf)
    orc = O.Oracle(m, p)
    f0, k0o, w0o = orc.init_state(np.ones(n), u0[:, 0], u0[:, 1], k0, w0)
    say("oracle step")
    f1, k1, w1 = orc.step(f0, k0o, w0o)
    nut1 = orc.last_nut
    F1, _ = orc.forces(f1, 1)
    for precision in ("fp64", "fp32dev"):
        say("one step on the GPU,", precision)
        st = F.State(M, p, precision=precision, rho=np.ones(n), u=u0, k=k0, omega=w0)
        st.timing(True)
        st.step(1)
        kt = st.timing_read()
        st.timing(False)
        assert kt["sst"][1] == 1 and kt["collide1"][1] == 0, kt     # the ring path
        mo = st.moments()
        if precision == "fp64":
            err = np.abs(st.get_f() - f1).max() / np.abs(f1 - O.WT[:, None]).max()
            assert err < 1e-12, err
            for name, got, ref in (("k", mo["k"], k1), ("omega", mo["omega"], w1), ("nu_t", mo["nu_t"], nut1)):
                e = np.abs(got - ref).max() / np.abs(ref).max()
                assert e < 1e-11, (name, e)
            Fg, _ = st.forces(1)
            assert np.abs(Fg - F1).max() <= 1e-10 * np.abs(F1).max(), (Fg, F1)
        else:
            _, ux1, uy1, _ = orc.macro(f1)
            du = max(np.abs(mo["u"][:, 0] - ux1).max(), np.abs(mo["u"][:, 1] - uy1).max()) / Uinf
            dk = np.abs(mo["k"] - k1).max() / np.abs(k1).max()
            dw = np.abs(mo["omega"] - w1).max() / np.abs(w1).max()
            say("fp32dev errors: du/U", du, "dk", dk, "dw", dw)
            assert du < 2e-6 and dk < 2e-6 and dw < 2e-6, (du, dk, dw)
        del st


def _compare_run(F, M, p, orc, f0, k0, w0, steps, gates, u_ref, label, rho=None, u=None):
    """Both precisions, `steps` steps from (f0, k0, w0) on the ring path, against the oracle's run on
    every cell.  gates: (FP64 f, FP64 k / omega / nu_t, FP32-dev u / u_ref, FP32-dev k / omega)."""
    say(label, "oracle run of", steps, "steps")
    fo, ko, wo = orc.run(f0, k0, w0, steps)
    nuto = orc.last_nut
    _, uxo, uyo, _ = orc.macro(fo)
    for precision in ("fp64", "fp32dev"):
        say(label, steps, "steps on the GPU,", precision)
        st = F.State(M, p, precision=precision, k=k0, omega=w0)
        st.set_state(f0, k0, w0)
        st.step(steps)
        mo = st.moments()
        if precision == "fp64":
            ef = np.abs(st.get_f() - fo).max() / np.abs(fo - O.WT[:, None]).max()
            ek = [np.abs(mo[key] - ref).max() / np.abs(ref).max()
                  for key, ref in (("k", ko), ("omega", wo), ("nu_t", nuto))]
            print(label, "fp64 after", steps, "steps: f", ef, "k, omega, nu_t", ek)
            assert ef < gates[0] and max(ek) < gates[1], (ef, ek)
        else:
            du = max(np.abs(mo["u"][:, 0] - uxo).max(), np.abs(mo["u"][:, 1] - uyo).max()) / u_ref
            dk = np.abs(mo["k"] - ko).max() / np.abs(ko).max()
            dw = np.abs(mo["omega"] - wo).max() / np.abs(wo).max()
            print(label, "fp32dev after", steps, "steps: du/U", du, "dk", dk, "dw", dw)
            assert du < gates[2] and dk < gates[3] and dw < gates[3], (du, dk, dw)
        del st


@pytest.mark.timeout(900)
def test_backstep_ten_steps_whole_mesh(F):
    """The backstep the benchmark times (122,876 cells, SST, 60 tau0), from the seeded developed state
    of test_backstep_fullsize_parity, 10 steps on the ring path against the oracle on every cell, at
    ten times the one-step gates: FP64 1e-11 of max |f - w rho0| and 1e-10 for k, omega, nu_t;
    FP32-deviation 2e-5 of U and 2e-5 relative for k, omega."""
    mesh, flow, init, dt_frac = bench.workload("backstep")
    M = F.Mesh(mesh, order="tiles")
    p = O.default_params(**dict(flow, dt=min(flow["dt"], dt_frac * M.max_dt())))
    orc = O.Oracle(mesh, p)
    n = orc.g.n
    rng = np.random.default_rng(12)
    x, y = orc.g.xc[:, 0], orc.g.xc[:, 1]
    ux = 0.04 + 0.01 * np.sin(0.5 * x) * np.cos(3 * y) + 0.002 * rng.standard_normal(n)
    uy = 0.004 * np.sin(2 * y) + 0.002 * rng.standard_normal(n)
    f0 = O.feq(1 + 0.001 * rng.standard_normal(n), ux, uy) + 1e-5 * O.WT[:, None] * rng.standard_normal((9, n))
    k0 = 1e-6 * (1 + 0.5 * rng.random(n))
    w0 = 1e-2 * (1 + 0.5 * rng.random(n))
    _compare_run(F, M, p, orc, f0, k0, w0, 10, (1e-11, 1e-10, 2e-5, 2e-5), 0.05, "backstep")


@pytest.mark.timeout(900)
def test_airfoil_ten_steps_whole_mesh(F):
    """The airfoil the benchmark times (196,608 quads, Re 6e6, 10 degrees, 74 tau0, limiter r32,
    developed near-wall start), 10 steps on the ring path against the oracle on every cell, at ten
    times the one-step gates (as test_backstep_ten_steps_whole_mesh)."""
    m = mg.naca_omesh()
    M = F.Mesh(m, order="tiles")
    n = M.n_cells
    Uinf, c, Re, alpha = 0.05, 1.0, 6e6, np.deg2rad(10.0)
    nu = Uinf * c / Re
    kinf, winf = 1e-3 * Uinf * Uinf / Re, 5 * Uinf / c
    p = O.default_params(nu=nu, dt=min(180 * 3 * nu, 0.9 * M.max_dt()), sst=True, theta=alpha, limiter=1,
                         group_u=[[0, 0], [Uinf, 0]], group_rho=[1, 1], group_k=[0, kinf], group_w=[0, winf])
    orc = O.Oracle(m, p)
    wd = orc.g.wall_dist
    fac = np.minimum(1.0, (wd / 0.01) ** (1 / 7))
    f0, k0, w0 = orc.init_state(np.ones(n), Uinf * np.cos(alpha) * fac, Uinf * np.sin(alpha) * fac,
                                np.full(n, kinf), np.maximum(winf, 6 * nu / (0.075 * wd ** 2)))
    _compare_run(F, M, p, orc, f0, k0, w0, 10, (1e-11, 1e-10, 2e-5, 2e-5), Uinf, "airfoil")
