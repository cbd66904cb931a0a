"""GPU parity on degenerate meshes: fewer cells than one 256-cell tile (a single partial tile with
no halo), periodic cells that are their own neighbour across every edge or reach their one
neighbour through two different edges, and cells whose every edge is a boundary edge (walls and a
moving lid, inlet / outlet / walls, far field all round).  Against the FP64 oracle (Section 3.1
Eqs. (imexone)-(imextwo) with the SST of Section 2 on each step): the FP64 step on every sweep
variant, a laminar step, FP32-deviation storage at its gate, the adjoint of three recorded steps
against the oracle's complex step, the step's options (limiters, per-stage and implicit SST) and the
explicit scheme."""
import sys

import numpy as np
import pytest

from oracle import fvlbm_oracle as O
from paper_1812_00394_amd import meshgen as mg

pytestmark = pytest.mark.gpu

H = 1e-30   # complex-step increment

CAV = dict(group_u=[[0, 0], [0.05, 0]], group_k=[0, 0], group_w=[0, 0])
DUCT = dict(group_u=[[0.05, 0.01], [0, 0], [0.05, 0.0]], group_rho=[1.0, 1.002, 1.0],
            group_k=[1e-4, 0, 1e-4], group_w=[0.5, 0, 0.5], theta=0.1)
CHAN = dict(group_u=[[0.04, 0], [0, 0], [0, 0]], group_rho=[1.0, 0.999, 1.0], group_k=[1e-4, 0, 0],
            group_w=[0.5, 0, 0], theta=0.1)
OPEN = dict(group_u=[[0.05, 0.01]], group_k=[1e-4], group_w=[0.5], theta=0.1)

CASES = {
    # two triangles; every edge but the diagonal a wall or the lid
    "cavity1": (lambda: mg.cavity(n=1, jitter=0.0), CAV),
    "cavity2": (lambda: mg.cavity(n=2, jitter=0.1, seed=3), CAV),
    # one quad, its own neighbour across all four edges
    "periodic1x1": (lambda: mg.rectangle(1, 1, kind="periodic", split="none"), {}),
    # two quads, each the other's neighbour through two edges and its own through the other two
    "periodic2x1": (lambda: mg.rectangle(2, 1, kind="periodic", split="none"), {}),
    "periodic1x1_tri": (lambda: mg.rectangle(1, 1, kind="periodic", seed=4), {}),
    "duct2x1": (lambda: mg.rectangle(2, 1, kind="duct", split="none"), DUCT),
    # one quad: inlet, outlet and two walls, no interior edge
    "channel1x1": (lambda: mg.rectangle(1, 1, kind="channel", split="none"), CHAN),
    "open1x1_tri": (lambda: mg.rectangle(1, 1, kind="open", seed=5), OPEN),
}


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


def _courant_dt(m, C=0.5):
    G = O.Geometry(m)
    en = np.maximum(O.EX[:, None] * G.nl[:, 0] + O.EY[:, None] * G.nl[:, 1], 0.0)
    out = np.stack([np.bincount(G.cell, weights=en[a], minlength=G.n) for a in range(9)])
    return C / (out / G.area).max()


def _case(name, sst=True, seed=7):
    make, extra = CASES[name]
    m = make()
    dt = _courant_dt(m)
    p = O.default_params(nu=dt / 60, dt=dt, sst=sst, **extra)
    orc = O.Oracle(m, p)
    n = orc.g.n
    rng = np.random.default_rng(seed)
    ux = 0.03 + 0.005 * rng.standard_normal(n)
    uy = 0.005 * rng.standard_normal(n)
    rho = 1 + 0.002 * rng.standard_normal(n)
    f = O.feq(rho, ux, uy) + 1e-5 * O.WT[:, None] * rng.standard_normal((9, n))
    k = 1e-4 * (1 + 0.5 * rng.random(n)) if sst else None
    w = 0.5 * (1 + 0.5 * rng.random(n)) if sst else None
    return m, p, orc, f, k, w


def _rel(a, b, scale):
    return np.abs(a - b).max() / scale


def test_degenerate_meshes_are_below_one_tile(F):
    for name, (make, _) in CASES.items():
        M = F.Mesh(make())
        assert 1 <= M.n_cells <= 8, (name, M.n_cells)


@pytest.mark.parametrize("sweep", ["ring", "pair", "split", "face"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_degenerate_sst_step_parity(F, name, sweep, monkeypatch):
    """FP64 SST steps: 1 step at 1e-12 and 4 more at 1e-11 of max |f - w rho0| (k, omega, nu_t at
    ten times that, relative to their largest value), as on the larger meshes.  The edge loop leaves
    out the edges of a periodic cell that is its own neighbour, whose two half-edges' fluxes cancel."""
    say("degenerate sst step", name, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    m, p, orc, f, k, w = _case(name)
    st = F.State(F.Mesh(m), p, precision="fp64", k=k, omega=w)
    st.set_state(f, k, w)
    fo, ko, wo = f, k, w
    for nsteps, tol in ((1, 1e-12), (4, 1e-11)):
        fo, ko, wo = orc.run(fo, ko, wo, nsteps)
        st.step(nsteps)
        got, mo = st.get_f(), st.moments()
        scale = np.abs(fo - O.WT[:, None]).max()
        assert _rel(got, fo, scale) < tol, ("f", nsteps, _rel(got, fo, scale))
        assert _rel(mo["k"], ko, np.abs(ko).max()) < 10 * tol, ("k", nsteps)
        assert _rel(mo["omega"], wo, np.abs(wo).max()) < 10 * tol, ("omega", nsteps)
        assert _rel(mo["nu_t"], orc.last_nut, np.abs(orc.last_nut).max()) < 10 * tol, ("nu_t", nsteps)


@pytest.mark.parametrize("name", sorted(CASES))
def test_degenerate_laminar_step_parity(F, name):
    """Five laminar FP64 steps (no SST) on the ring sweeps, at 1e-11."""
    say("degenerate laminar step", name)
    m, p, orc, f, _, _ = _case(name, sst=False, seed=8)
    st = F.State(F.Mesh(m), p, precision="fp64")
    st.set_state(f)
    fo = orc.run(f, None, None, 5)[0]
    st.step(5)
    scale = np.abs(fo - O.WT[:, None]).max()
    assert _rel(st.get_f(), fo, scale) < 1e-11


@pytest.mark.parametrize("name", sorted(CASES))
def test_degenerate_fp32dev_step(F, name):
    """One SST step in FP32-deviation storage: velocity within 2e-6 of the flow speed (0.05), k and
    omega within 2e-6 relative, the gates of the larger meshes."""
    say("degenerate fp32dev step", name)
    m, p, orc, f, k, w = _case(name, seed=9)
    f1, k1, w1 = orc.step(f, k, w)
    _, ux, uy, _ = orc.macro(f1)
    st = F.State(F.Mesh(m), p, precision="fp32dev", k=k, omega=w)
    st.set_state(f, k, w)
    st.step(1)
    mo = st.moments()
    du = max(np.abs(mo["u"][:, 0] - ux).max(), np.abs(mo["u"][:, 1] - uy).max()) / 0.05
    dk = _rel(mo["k"], k1, np.abs(k1).max())
    dw = _rel(mo["omega"], w1, np.abs(w1).max())
    assert du < 2e-6 and dk < 2e-6 and dw < 2e-6, (du, dk, dw)


PARAMS = ["theta", "sigma_k1", "sigma_w1", "beta_star", "a1"]


@pytest.mark.parametrize("sweep", ["ring", "split"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_degenerate_adjoint_against_complex_step(F, name, sweep, monkeypatch):
    """Three recorded FP64 SST steps (a checkpoint every 2): the adjoint's dot product with the
    oracle's complex-step derivative along a random direction of (f, k, omega) at 1e-9, and the five
    parameter gradients of lam . final state at 1e-8 (relative to the largest of them where one is
    zero, as theta's is on the meshes without an inflow)."""
    say("degenerate adjoint", name, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    m, p, orc, f0, k0, w0 = _case(name, seed=10)
    n = f0.shape[1]
    N = 3
    st = F.State(F.Mesh(m), p, precision="fp64", k=k0, omega=w0)
    st.set_state(f0, k0, w0)
    st.record(N, ckpt_every=2)
    rng = np.random.default_rng(11)
    lf = rng.standard_normal((9, n))
    lk = rng.standard_normal(n) * 1e3
    lw = rng.standard_normal(n)
    lf0, lk0, lw0, dp = st.adjoint_state(lf, lk, lw)
    vf = rng.standard_normal((9, n)) * O.WT[:, None] * 1e-3
    vk = rng.standard_normal(n) * 1e-5
    vw = rng.standard_normal(n) * 1e-2
    fN, kN, wN = O.Oracle(m, p).run(f0 + 1j * H * vf, k0 + 1j * H * vk, w0 + 1j * H * vw, N)
    rhs = (np.sum(lf * np.imag(fN)) + np.sum(lk * np.imag(kN)) + np.sum(lw * np.imag(wN))) / H
    lhs = np.sum(lf0 * vf) + np.sum(lk0 * vk) + np.sum(lw0 * vw)
    assert abs(lhs - rhs) <= 1e-9 * abs(rhs), (lhs, rhs)
    refs = []
    for key in PARAMS:
        pc = dict(p)
        pc[key] = p[key] + 1j * H
        fN, kN, wN = O.Oracle(m, pc).run(f0.astype(complex), k0.astype(complex), w0.astype(complex), N)
        refs.append((np.sum(lf * np.imag(fN)) + np.sum(lk * np.imag(kN)) + np.sum(lw * np.imag(wN))) / H)
    refs = np.array(refs)
    scale = np.abs(refs).max()
    assert np.all(np.abs(dp[:len(PARAMS)] - refs) <= 1e-8 * np.maximum(np.abs(refs), 1e-6 * scale)), (dp, refs)


VARIANTS = {
    "limiter1": dict(limiter=1),          # face-value clip (reading r32)
    "limiter2": dict(limiter=2),          # gradient limiter (reading r35)
    "implicit4": dict(sst_sweeps=4),      # implicit SST, four Jacobi sweeps (reading r34)
    "per_stage": dict(sst_stages=1),      # SST before each stage (reading r33)
}


@pytest.mark.parametrize("variant", sorted(VARIANTS))
@pytest.mark.parametrize("name", sorted(CASES))
def test_degenerate_variant_step_parity(F, name, variant):
    """The step's options on the ring sweeps: three FP64 SST steps at 1e-11 (k, omega, nu_t at ten
    times that), then the adjoint of two recorded steps against the oracle's complex step (1e-9).
    With the implicit SST a periodic cell that is its own neighbour keeps that coupling on the
    diagonal of the increments' system, as Jacobi with D = diag(A) does."""
    say("degenerate variant", name, variant)
    m, p, orc, f, k, w = _case(name, seed=12)
    p = dict(p, **VARIANTS[variant])
    orc = O.Oracle(m, p)
    st = F.State(F.Mesh(m), p, precision="fp64", k=k, omega=w)
    st.set_state(f, k, w)
    fo, ko, wo = orc.run(f, k, w, 3)
    st.step(3)
    got, mo = st.get_f(), st.moments()
    assert _rel(got, fo, np.abs(fo - O.WT[:, None]).max()) < 1e-11, ("f", _rel(got, fo, np.abs(fo - O.WT[:, None]).max()))
    assert _rel(mo["k"], ko, np.abs(ko).max()) < 1e-10, ("k", _rel(mo["k"], ko, np.abs(ko).max()))
    assert _rel(mo["omega"], wo, np.abs(wo).max()) < 1e-10, ("omega", _rel(mo["omega"], wo, np.abs(wo).max()))
    n = f.shape[1]
    st.set_state(f, k, w)
    st.record(2, ckpt_every=1)
    rng = np.random.default_rng(13)
    lf, lk, lw = rng.standard_normal((9, n)), rng.standard_normal(n) * 1e3, rng.standard_normal(n)
    lf0, lk0, lw0, _ = st.adjoint_state(lf, lk, lw)
    vf = rng.standard_normal((9, n)) * O.WT[:, None] * 1e-3
    vk, vw = rng.standard_normal(n) * 1e-5, rng.standard_normal(n) * 1e-2
    fN, kN, wN = O.Oracle(m, p).run(f + 1j * H * vf, k + 1j * H * vk, w + 1j * H * vw, 2)
    rhs = (np.sum(lf * np.imag(fN)) + np.sum(lk * np.imag(kN)) + np.sum(lw * np.imag(wN))) / H
    lhs = np.sum(lf0 * vf) + np.sum(lk0 * vk) + np.sum(lw0 * vw)
    assert abs(lhs - rhs) <= 1e-9 * abs(rhs), (lhs, rhs)


@pytest.mark.parametrize("sst", [False, True])
@pytest.mark.parametrize("name", sorted(CASES))
def test_degenerate_explicit_step_parity(F, name, sst):
    """The explicit scheme (forward Euler of the semi-discrete equation, Section 3.1) at dt = tau,
    laminar and with the SST: one step at 1e-12, three more at 1e-11."""
    say("degenerate explicit step", name, sst)
    m, p, orc, f, k, w = _case(name, sst=sst, seed=14)
    p = dict(p, nu=p["dt"] / 3)
    orc = O.Oracle(m, p)
    st = F.State(F.Mesh(m), p, precision="fp64", k=k, omega=w)
    st.set_state(f, k, w)
    fo, ko, wo = f, k, w
    for nsteps, tol in ((1, 1e-12), (3, 1e-11)):
        for _ in range(nsteps):
            fo, ko, wo = orc.step_explicit(fo, ko, wo)
        st.step_explicit(nsteps)
        assert _rel(st.get_f(), fo, np.abs(fo - O.WT[:, None]).max()) < tol, (nsteps,)
        if sst:
            assert _rel(st.moments()["omega"], wo, np.abs(wo).max()) < 10 * tol, (nsteps,)
