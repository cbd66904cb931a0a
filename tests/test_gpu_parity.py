"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the same seeded meshes.

Tolerances (FP64 path): relative to max |f - w rho0| (the part of f that carries information),
<= 1e-12 after one step and <= 1e-10 after the full step count; the convection operator alone
<= 1e-12 relative to its largest value.  These are rounding-order differences: the oracle sums the
convection over a cell's edges in a different order and applies Eq. (imextwo) literally, while the
kernels use the algebraically equal f^(3) + dt/3 Ga3 - dt/6 (Ga1 + Ga2) and deviations f - w rho0.
"""
import sys

import numpy as np
import pytest

from oracle import fvlbm_oracle as O
from paper_1812_00394_amd import meshgen as mg

pytestmark = pytest.mark.gpu


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


def rel(a, b, scale):
    return np.abs(a - b).max() / scale


def dev_scale(f, rho0=1.0):
    return np.abs(f - O.WT[:, None] * rho0).max()


MESHES = {
    "cavity": (lambda: mg.cavity(n=16, jitter=0.2, seed=31), dict(group_u=[[0, 0], [0.1, 0]])),
    "periodic": (lambda: mg.rectangle(9, 8, kind="periodic", jitter=0.25, seed=32), dict()),
    "duct": (lambda: mg.rectangle(10, 7, Lx=1.4, kind="duct", jitter=0.25, seed=33),
             dict(group_u=[[0.05, 0.01], [0, 0], [0.05, 0.0]], group_rho=[1.0, 1.002, 1.0])),
    "channel": (lambda: mg.rectangle(12, 6, Lx=2.0, kind="channel", jitter=0.2, seed=34),
                dict(group_u=[[0.04, 0], [0, 0], [0, 0]], group_rho=[1.0, 0.999, 1.0])),
    "naca": (lambda: mg.naca_omesh(n_wall=48, n_normal=16, y1=2e-3, radius=6.0),
             dict(group_u=[[0, 0], [0.05, 0]], theta=0.1)),
}


def courant_dt(m, C=0.5):
    """time step at advective Courant number C: max over cells and directions of
    (dt / A) sum over edges of max(e.n, 0) dl equals C."""
    G = O.Geometry(m)
    en = np.maximum(O.EX[:, None] * G.nl[:, 0] + O.EY[:, None] * G.nl[:, 1], 0.0)
    out = np.stack([np.bincount(G.cell, weights=en[a], minlength=G.n) for a in range(9)])
    return C / (out / G.area).max()


def _random_state(n, rng, amp=0.02):
    rho = 1 + 0.01 * rng.standard_normal(n)
    ux, uy = 0.05 * rng.standard_normal((2, n))
    f = O.feq(rho, ux, uy) + amp * 1e-2 * O.WT[:, None] * rng.standard_normal((9, n))
    return f


@pytest.mark.parametrize("name", sorted(MESHES))
def test_advection_operator_parity(F, name):
    say("advection", name)
    make, extra = MESHES[name]
    m = make()
    p = O.default_params(nu=1e-3, dt=1e-2, **extra)
    orc = O.Oracle(m, p)
    rng = np.random.default_rng(40)
    g = _random_state(orc.g.n, rng)
    ref = orc.advection(g)
    st = F.State(F.Mesh(m), p, precision="fp64")
    got = st.apply_advection(g)
    assert rel(got, ref, np.abs(ref).max()) < 1e-12


@pytest.mark.parametrize("sweep", ["ring", "pair", "tiled", "tiled-grads", "split", "face"])
@pytest.mark.parametrize("name", sorted(MESHES))
def test_laminar_step_parity(F, name, sweep, monkeypatch):
    """Every sweep variant: ring-tiled (both halo rings staged in LDS, stage 1 collision fused),
    tiled with values and gradients in LDS, tiled with gradients only, the two-kernel path, and the
    edge loop with atomics."""
    say("laminar step", name, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    make, extra = MESHES[name]
    m = make()
    dt = courant_dt(m)
    nu = dt / 30
    p = O.default_params(nu=nu, dt=dt, **extra)
    orc = O.Oracle(m, p)
    rng = np.random.default_rng(41)
    f = _random_state(orc.g.n, rng)
    st = F.State(F.Mesh(m), p, precision="fp64")
    st.set_state(f)
    fo = f
    for k, tol in ((1, 1e-12), (4, 1e-11)):
        for _ in range(k):
            fo, _, _ = orc.step(fo)
        st.step(k)
        got = st.get_f()
        assert rel(got, fo, dev_scale(fo)) < tol, (k, rel(got, fo, dev_scale(fo)))


def _c1_params():
    nu = 0.1 / 1000
    return O.default_params(nu=nu, dt=10 * 3 * nu, group_u=[[0, 0], [0.1, 0]])


def test_cavity_full_run_parity(F):
    """Laminar lid-driven cavity, 48x48 jittered triangles (4608 cells), Re 1000, dt = 10 tau,
    500 steps: f, macro fields, totals and residual against the oracle."""
    say("cavity 4608 cells, 500 steps, fp64")
    m = mg.cavity()
    p = _c1_params()
    orc = O.Oracle(m, p)
    n = orc.g.n
    f, _, _ = orc.init_state(np.ones(n), np.zeros(n), np.zeros(n))
    st = F.State(F.Mesh(m), p, precision="fp64", rho=np.ones(n), u=np.zeros((n, 2)))
    f_prev = f
    for _ in range(500):
        f_prev = f
        f, _, _ = orc.step(f)
    res = st.step(500, residual=True)
    got = st.get_f()
    assert rel(got, f, dev_scale(f)) < 1e-10
    mo = st.moments()
    rho, ux, uy, _ = orc.macro(f)
    np.testing.assert_allclose(mo["rho"], rho, rtol=1e-12)
    np.testing.assert_allclose(mo["u"][:, 0], ux, atol=1e-12 * 0.1)
    np.testing.assert_allclose(mo["totals"], orc.totals(f), rtol=1e-12, atol=1e-13)
    _, ux0, uy0, _ = orc.macro(f_prev)
    np.testing.assert_allclose(res, orc.residual(ux0, uy0, ux, uy), rtol=1e-8)
    # mass is conserved in the closed cavity
    assert abs(mo["totals"][0] - 1.0) < 1e-13


def test_cavity_fp32_deviation_error(F):
    """FP32-deviation storage against the FP64 oracle on the cavity after 200 steps: the error in
    velocity stays below 1e-4 of the lid speed (stated gate)."""
    say("cavity fp32dev 200 steps")
    m = mg.cavity()
    p = _c1_params()
    orc = O.Oracle(m, p)
    n = orc.g.n
    f, _, _ = orc.init_state(np.ones(n), np.zeros(n), np.zeros(n))
    f, _, _ = orc.run(f, None, None, 200)
    st = F.State(F.Mesh(m), p, precision="fp32dev", rho=np.ones(n), u=np.zeros((n, 2)))
    st.step(200)
    mo = st.moments()
    _, ux, uy, _ = orc.macro(f)
    err = max(np.abs(mo["u"][:, 0] - ux).max(), np.abs(mo["u"][:, 1] - uy).max()) / 0.1
    print("fp32dev velocity error / U =", err)
    assert err < 1e-4
    assert abs(mo["totals"][0] - 1.0) < 1e-6


def _sst_case(m, extra, seed):
    dt = courant_dt(m)
    nu = dt / 60
    p = O.default_params(nu=nu, dt=dt, sst=True, **extra)
    orc = O.Oracle(m, p)
    n = orc.g.n
    rng = np.random.default_rng(seed)
    x, y = orc.g.xc[:, 0], orc.g.xc[:, 1]
    ux = 0.05 * np.tanh(3 * (y - y.mean())) + 0.005 * rng.standard_normal(n)
    uy = 0.01 * np.sin(2 * x) + 0.005 * rng.standard_normal(n)
    rho = 1 + 0.002 * rng.standard_normal(n)
    f = O.feq(rho, ux, uy) + 1e-5 * O.WT[:, None] * rng.standard_normal((9, n))
    k = 1e-4 * (1 + 0.5 * rng.random(n))
    w = 0.5 * (1 + 0.5 * rng.random(n))
    return orc, p, f, k, w


SST_MESHES = {
    "backstep_coarse": (lambda: mg.backstep(core=0.25, dx_core=0.5, y1=1e-2, dx_corner=0.05, wall_layers=3),
                        dict(group_u=[[0, 0], [0.05, 0], [0, 0]], group_k=[0, 1e-4, 0], group_w=[0, 0.5, 0])),
    "naca": (lambda: mg.naca_omesh(n_wall=48, n_normal=16, y1=2e-3, radius=6.0),
             dict(group_u=[[0, 0], [0.05, 0]], group_k=[0, 1e-4], group_w=[0, 0.5], theta=0.15)),
    "duct": (lambda: mg.rectangle(10, 7, Lx=1.4, kind="duct", jitter=0.25, seed=33),
             dict(group_u=[[0.05, 0.01], [0, 0], [0.05, 0.0]], group_k=[1e-4, 0, 1e-4], group_w=[0.5, 0, 0.5])),
}


@pytest.mark.parametrize("sweep", ["ring", "pair", "split", "face"])
@pytest.mark.parametrize("name", sorted(SST_MESHES))
def test_sst_step_parity(F, name, sweep, monkeypatch):
    """The SST in one ring-tiled launch and as the two-kernel pair (which the edge loop also uses)."""
    say("sst step", name, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    make, extra = SST_MESHES[name]
    m = make()
    orc, p, f, k, w = _sst_case(m, extra, 50)
    st = F.State(F.Mesh(m), p, precision="fp64", k=k, omega=w)
    st.set_state(f, k, w)
    fo, ko, wo = f, k, w
    for nsteps, tol in ((1, 1e-12), (4, 1e-11)):
        fo, ko, wo = orc.run(fo, ko, wo, nsteps)
        st.step(nsteps)
        got = st.get_f()
        mo = st.moments()
        assert rel(got, fo, dev_scale(fo)) < tol, ("f", nsteps, rel(got, fo, dev_scale(fo)))
        assert rel(mo["k"], ko, np.abs(ko).max()) < tol * 10, ("k", nsteps, rel(mo["k"], ko, np.abs(ko).max()))
        assert rel(mo["omega"], wo, np.abs(wo).max()) < tol * 10, ("w", nsteps)
        assert rel(mo["nu_t"], orc.last_nut, np.abs(orc.last_nut).max()) < tol * 10, ("nu_t", nsteps)


@pytest.mark.parametrize("name", sorted(SST_MESHES))
def test_fp32_with_fp64_geometry_step_parity(F, name):
    """FP32-deviation storage whose ring sweeps stream the geometry in FP64 and form normals, midpoint
    offsets and LSQ coefficients in FP64 (precision fp32dev_geo64): one SST step against the oracle
    at the FP32-deviation gates (2e-6 of U for u, 2e-6 relative for k, omega), printed next to the
    FP32-geometry mode's errors on the same case.  The non-ring sweeps refuse it."""
    say("fp32dev with fp64 geometry", name)
    make, extra = SST_MESHES[name]
    m = make()
    orc, p, f, k, w = _sst_case(m, extra, 58)
    f1, k1, w1 = orc.step(f, k, w)
    _, ux, uy, _ = orc.macro(f1)
    M = F.Mesh(m)
    errs = {}
    for precision in ("fp32dev", "fp32dev_geo64"):
        st = F.State(M, p, precision=precision, k=k, omega=w)
        st.set_state(f, k, w)
        st.step(1)
        mo = st.moments()
        du = max(np.abs(mo["u"][:, 0] - ux).max(), np.abs(mo["u"][:, 1] - uy).max()) / 0.05
        errs[precision] = (du, rel(mo["k"], k1, np.abs(k1).max()), rel(mo["omega"], w1, np.abs(w1).max()))
        del st
    print(name, "one-step errors (du/U, dk, dw):", errs)
    assert max(errs["fp32dev_geo64"]) < 2e-6, errs
    with pytest.MonkeyPatch.context() as mp:
        mp.setenv("FVLBM_SWEEP", "split")
        with pytest.raises(F.FvlbmError, match="EINVAL"):
            F.State(M, p, precision="fp32dev_geo64", k=k, omega=w)


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
@pytest.mark.parametrize("sweep", ["ring", "pair", "split"])
@pytest.mark.parametrize("name", ["backstep_coarse", "naca"])
def test_sst_per_stage_step_parity(F, name, sweep, precision, monkeypatch):
    """The SST solved again before the third stage (params.sst = 2, reading r33): the second SST
    launch from k^n, omega^n with the stage-2 macro variables that stage 1 writes, the third stage's
    relaxation time, the step keeping that solve's k, omega, nu_t.  FP64 to the SST gates; FP32-dev
    to 2e-6 of U for u and 2e-6 relative for k, omega after one step."""
    say("sst per-stage step", name, sweep, precision)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    make, extra = SST_MESHES[name]
    m = make()
    orc, p, f, k, w = _sst_case(m, extra, 52)
    p = dict(p, sst_stages=1)
    orc = O.Oracle(m, p)
    st = F.State(F.Mesh(m), p, precision=precision, k=k, omega=w)
    st.set_state(f, k, w)
    once = O.Oracle(m, dict(p, sst_stages=0))
    f1o, k1o, _ = once.step(f, k, w)
    fo, ko, wo = f, k, w
    for nsteps, tol in ((1, 1e-12), (3, 1e-11)):
        fo, ko, wo = orc.run(fo, ko, wo, nsteps)
        st.step(nsteps)
        mo = st.moments()
        if precision == "fp64":
            got = st.get_f()
            assert rel(got, fo, dev_scale(fo)) < tol, ("f", nsteps, rel(got, fo, dev_scale(fo)))
            assert rel(mo["k"], ko, np.abs(ko).max()) < tol * 10, ("k", nsteps)
            assert rel(mo["omega"], wo, np.abs(wo).max()) < tol * 10, ("w", nsteps)
            assert rel(mo["nu_t"], orc.last_nut, np.abs(orc.last_nut).max()) < tol * 10, ("nu_t", nsteps)
        elif nsteps == 1:
            _, ux, uy, _ = orc.macro(fo)
            du = max(np.abs(mo["u"][:, 0] - ux).max(), np.abs(mo["u"][:, 1] - uy).max()) / 0.05
            assert du < 2e-6, du
            assert rel(mo["k"], ko, np.abs(ko).max()) < 2e-6 and rel(mo["omega"], wo, np.abs(wo).max()) < 2e-6
        if nsteps == 1:
            # the variant is active: its k differs from the once-per-step coupling's
            assert rel(ko, k1o, np.abs(k1o).max()) > 1e-9


def test_sst_impulsive_start_parity(F):
    """Uniform stream started impulsively between walls: the positivity bound of the k / omega
    face values and the implicit negative sources are active on both sides."""
    say("sst impulsive start, graded delaunay")
    m = mg.delaunay_rect(n_points=1500, seed=5)
    U, nu = 0.05, 0.05 / 3.6e4
    p = O.default_params(nu=nu, dt=0.9 * courant_dt(m, 1.0), sst=True, group_u=[[0, 0], [U, 0], [0, 0]],
                         group_rho=[1, 1, 1], group_k=[0, 1e-6, 0], group_w=[0, 1e-2, 0])
    orc = O.Oracle(m, p)
    n = orc.g.n
    f, k, w = orc.init_state(np.ones(n), np.full(n, U), np.zeros(n), np.full(n, 1e-6), np.full(n, 1e-2))
    st = F.State(F.Mesh(m), p, precision="fp64", rho=np.ones(n), u=np.tile([U, 0.0], (n, 1)),
                 k=np.full(n, 1e-6), omega=np.full(n, 1e-2))
    for nsteps in (1, 9, 20):
        f, k, w = orc.run(f, k, w, nsteps)
        st.step(nsteps)
        got = st.get_f()
        mo = st.moments()
        assert rel(got, f, dev_scale(f)) < 1e-10, ("f", nsteps, rel(got, f, dev_scale(f)))
        assert rel(mo["k"], k, np.abs(k).max()) < 1e-9, ("k", nsteps, rel(mo["k"], k, np.abs(k).max()))
        assert rel(mo["omega"], w, np.abs(w).max()) < 1e-9, ("w", nsteps)


def test_sst_impulsive_start_fp32_deviation(F):
    """The same impulsive start in FP32-deviation storage against the FP64 oracle: velocity, k and
    omega within 2e-6 after one step and within 1e-4 after 30 steps of this harsh transient
    (relative to U and to their maxima; stated gates)."""
    say("sst impulsive start fp32dev")
    m = mg.delaunay_rect(n_points=1500, seed=5)
    U, nu = 0.05, 0.05 / 3.6e4
    p = O.default_params(nu=nu, dt=0.9 * courant_dt(m, 1.0), sst=True, group_u=[[0, 0], [U, 0], [0, 0]],
                         group_rho=[1, 1, 1], group_k=[0, 1e-6, 0], group_w=[0, 1e-2, 0])
    orc = O.Oracle(m, p)
    n = orc.g.n
    f, k, w = orc.init_state(np.ones(n), np.full(n, U), np.zeros(n), np.full(n, 1e-6), np.full(n, 1e-2))
    st = F.State(F.Mesh(m), p, precision="fp32dev", rho=np.ones(n), u=np.tile([U, 0.0], (n, 1)),
                 k=np.full(n, 1e-6), omega=np.full(n, 1e-2))
    for nsteps, gate_u, gate_kw in ((1, 2e-6, 2e-6), (29, 1e-4, 1e-4)):
        f, k, w = orc.run(f, k, w, nsteps)
        st.step(nsteps)
        mo = st.moments()
        _, ux, uy, _ = orc.macro(f)
        du = max(np.abs(mo["u"][:, 0] - ux).max(), np.abs(mo["u"][:, 1] - uy).max()) / U
        dk = np.abs(mo["k"] - k).max() / np.abs(k).max()
        dw = np.abs(mo["omega"] - w).max() / np.abs(w).max()
        print("fp32dev sst errors after", nsteps, "steps: du/U", du, "dk", dk, "dw", dw)
        assert np.isfinite(mo["totals"]).all()
        assert du < gate_u and dk < gate_kw and dw < gate_kw, (nsteps, du, dk, dw)


def test_forces_parity(F):
    say("forces naca")
    make, extra = SST_MESHES["naca"]
    m = make()
    orc, p, f, k, w = _sst_case(m, dict(extra, jr_group=0, jr_xmin=0.3, eps_tau=1e-6), 51)
    st = F.State(F.Mesh(m), p, precision="fp64", k=k, omega=w)
    st.set_state(f, k, w)
    Fo, JRo = orc.forces(f, 1)
    Fg, JRg = st.forces(1)
    np.testing.assert_allclose(Fg, Fo, rtol=1e-11, atol=1e-16)
    assert abs(JRg - JRo) < 1e-12 * max(1.0, abs(JRo))


def _airfoil_stream_case(alpha):
    """The small O-mesh around the 12 % section in a developed stream at incidence alpha (SST on,
    limiter on, dt half the advective Courant limit)."""
    m = mg.naca_omesh(n_wall=64, n_normal=24, y1=2e-3, radius=5.0)
    U = 0.05
    p = O.default_params(nu=U / 2e3, dt=courant_dt(m), sst=True, theta=alpha, limiter=1,
                         group_u=[[0, 0], [U, 0]], group_k=[0, 1e-3 * U * U / 2e3], group_w=[0, 5 * U])
    orc = O.Oracle(m, p)
    G = orc.g
    fac = np.minimum(1.0, (G.wall_dist / 0.01) ** (1 / 7))
    f, k, w = orc.init_state(np.ones(G.n), U * np.cos(alpha) * fac, U * np.sin(alpha) * fac,
                             np.full(G.n, p["group_k"][1]), np.full(G.n, 5 * U))
    return m, p, orc, f, k, w, U


def test_lift_drag_parity(F):
    """fvlbm_lift_drag against the oracle's lift_drag (Section 4, the NACA0012 lift/drag table).
    (i) the pressure closed form at rest: C_l = cos(alpha) K, C_d = sin(alpha) K, K = 2 delta / (3 U^2);
    (ii) after 3 steps of a developed stream at 10 degrees: FP64 within 1e-11 of the oracle, FP32-dev
    within 1e-3 relative (the stated FP32-dev gate for lift and drag);
    (iii) at zero incidence on the mirror-symmetric mesh: |C_l| <= 1e-11 C_d after 3 steps."""
    alpha = np.deg2rad(10.0)
    m, p, orc, f, k, w, U = _airfoil_stream_case(alpha)
    n = orc.g.n
    say("lift/drag pressure closed form, naca 64x24")
    delta = 0.01
    fr = O.feq(np.where(orc.g.xc[:, 1] < 0, 1 + delta, 1.0), np.zeros(n), np.zeros(n))
    st = F.State(F.Mesh(m), p, precision="fp64", k=k, omega=w)
    st.set_state(fr, k, w)
    K = 2 * delta / (3 * U * U)
    np.testing.assert_allclose(st.lift_drag(1, U), [np.cos(alpha) * K, np.sin(alpha) * K], rtol=1e-12)
    say("lift/drag after 3 steps at 10 degrees, fp64 and fp32dev")
    fo, ko, wo = orc.run(f, k, w, 3)
    ref = orc.lift_drag(fo, 1, U)
    for prec, tol in (("fp64", 1e-11), ("fp32dev", 1e-3)):
        st = F.State(F.Mesh(m), p, precision=prec, k=k, omega=w)
        st.set_state(f, k, w)
        st.step(3)
        got = np.array(st.lift_drag(1, U))
        err = np.abs(got - ref) / np.abs(ref)
        print(prec, "C_l, C_d", got, "oracle", ref, "relative error", err)
        assert (err < tol).all(), (prec, got, ref)
    say("lift/drag at zero incidence, symmetric mesh")
    m0, p0, orc0, f0, k0, w0, _ = _airfoil_stream_case(0.0)
    st = F.State(F.Mesh(m0), p0, precision="fp64", k=k0, omega=w0)
    st.set_state(f0, k0, w0)
    st.step(3)
    cl, cd = st.lift_drag(1, U)
    print("zero incidence: C_l", cl, "C_d", cd)
    assert cd > 0 and abs(cl) <= 1e-11 * cd


# ------------------------------------------------------------------------------------------------
# Optional face-value limiter (params["limiter"] = 1): same parity gates as the plain scheme.
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("limiter", [1, 2])
@pytest.mark.parametrize("name", ["cavity", "duct", "naca"])
def test_limited_advection_operator_parity(F, name, limiter):
    say("limited advection", name, "limiter", limiter)
    make, extra = MESHES[name]
    m = make()
    p = O.default_params(nu=1e-3, dt=1e-2, limiter=limiter, **extra)
    orc = O.Oracle(m, p)
    rng = np.random.default_rng(43)
    g = _random_state(orc.g.n, rng)
    ref = orc.advection(g)
    st = F.State(F.Mesh(m), p, precision="fp64")
    got = st.apply_advection(g)
    assert rel(got, ref, np.abs(ref).max()) < 1e-12


@pytest.mark.parametrize("limiter", [1, 2])
@pytest.mark.parametrize("sweep", ["ring", "pair", "split", "face"])
@pytest.mark.parametrize("name", ["cavity", "channel", "naca"])
def test_limited_laminar_step_parity(F, name, sweep, limiter, monkeypatch):
    say("limited laminar step", name, sweep, "limiter", limiter)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    make, extra = MESHES[name]
    m = make()
    dt = courant_dt(m)
    p = O.default_params(nu=dt / 30, dt=dt, limiter=limiter, **extra)
    orc = O.Oracle(m, p)
    f = _random_state(orc.g.n, np.random.default_rng(44))
    st = F.State(F.Mesh(m), p, precision="fp64")
    st.set_state(f)
    fo = f
    for k, tol in ((1, 1e-12), (4, 1e-11)):
        for _ in range(k):
            fo, _, _ = orc.step(fo)
        st.step(k)
        assert rel(st.get_f(), fo, dev_scale(fo)) < tol


@pytest.mark.parametrize("limiter", [1, 2])
def test_limited_sst_step_parity(F, limiter):
    say("limited sst step, backstep_coarse, limiter", limiter)
    make, extra = SST_MESHES["backstep_coarse"]
    m = make()
    orc, p, f, k, w = _sst_case(m, extra, 52)
    p = dict(p, limiter=limiter)
    orc = O.Oracle(m, p)
    st = F.State(F.Mesh(m), p, precision="fp64", k=k, omega=w)
    st.set_state(f, k, w)
    fo, ko, wo = orc.run(f, k, w, 2)
    st.step(2)
    assert rel(st.get_f(), fo, dev_scale(fo)) < 1e-11
    assert rel(st.moments()["k"], ko, np.abs(ko).max()) < 1e-10


@pytest.mark.timeout(600)
def test_airfoil_full_size_lift_drag_fp32_vs_fp64(F):
    """The airfoil workload at full size: 512 x 384 O-mesh (196,608 quads) around the sharp-trailing-
    edge 12 % section, Re 6e6 on the chord, 10 degrees incidence, u_inf = 0.05, dt = 0.9 of the
    advective Courant limit, a developed near-wall start, limiter on (without it the flow around the
    sharp trailing edge diverges within ~150 steps in either precision), 3000 steps.  Lift and
    drag in FP32-deviation storage agree with FP64 within 1e-4 relative (stated gate)."""
    say("airfoil 196608 quads, 3000 steps, fp64 and fp32dev")
    m = mg.naca_omesh()
    M = F.Mesh(m, order="tiles")     # the benchmark's renumbering
    n = M.n_cells
    _, _, wd = M.geometry()
    U, c, Re, alpha = 0.05, 1.0, 6e6, np.deg2rad(10.0)
    nu = U * c / Re
    kinf, winf = 1e-3 * U * U / Re, 5 * U / c
    p = dict(nu=nu, dt=min(180 * 3 * nu, 0.9 * M.max_dt()), sst=True, theta=alpha, limiter=1,
             group_u=[[0, 0], [U, 0]], group_rho=[1, 1], group_k=[0, kinf], group_w=[0, winf])
    fac = np.minimum(1.0, (wd / 0.01) ** (1 / 7))
    u0 = np.stack([U * np.cos(alpha) * fac, U * np.sin(alpha) * fac], axis=1)
    w0 = np.maximum(winf, 6 * nu / (0.075 * wd ** 2))
    out = {}
    for prec in ("fp64", "fp32dev"):
        st = F.State(M, p, precision=prec, rho=np.ones(n), u=u0, k=np.full(n, kinf), omega=w0)
        st.step(3000)
        out[prec] = st.lift_drag(1, U, c)
        assert np.isfinite(st.moments()["totals"]).all()
        del st
    print("lift, drag after 3000 steps:", out)
    (l64, d64), (l32, d32) = out["fp64"], out["fp32dev"]
    assert abs(l32 - l64) <= 1e-4 * abs(l64) and abs(d32 - d64) <= 1e-4 * abs(d64), out


# ------------------------------------------------------------------------------------------------
# The explicit scheme the IMEX scheme is compared with (forward Euler, dt < 2 tau).
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("sweep", ["ring", "pair"])
@pytest.mark.parametrize("name", ["cavity", "periodic", "naca"])
def test_explicit_step_parity(F, name, sweep, monkeypatch):
    say("explicit step", name, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    make, extra = MESHES[name]
    m = make()
    dt = courant_dt(m)
    p = O.default_params(nu=dt / 3, dt=dt, **extra)      # dt = tau
    orc = O.Oracle(m, p)
    f = _random_state(orc.g.n, np.random.default_rng(45))
    st = F.State(F.Mesh(m), p, precision="fp64")
    st.set_state(f)
    fo = f
    for k, tol in ((1, 1e-12), (4, 1e-11)):
        for _ in range(k):
            fo, _, _ = orc.step_explicit(fo)
        st.step_explicit(k)
        assert rel(st.get_f(), fo, dev_scale(fo)) < tol


@pytest.mark.parametrize("sweep", ["ring", "pair"])
def test_explicit_sst_step_parity(F, sweep, monkeypatch):
    say("explicit sst step, duct", sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    make, extra = SST_MESHES["duct"]
    m = make()
    orc, p, f, k, w = _sst_case(m, extra, 53)
    p = dict(p, nu=p["dt"] / 3)
    orc = O.Oracle(m, p)
    st = F.State(F.Mesh(m), p, precision="fp64", k=k, omega=w)
    st.set_state(f, k, w)
    fo, ko, wo = f, k, w
    for _ in range(2):
        fo, ko, wo = orc.step_explicit(fo, ko, wo)
    st.step_explicit(2)
    assert rel(st.get_f(), fo, dev_scale(fo)) < 1e-11
    assert rel(st.moments()["omega"], wo, np.abs(wo).max()) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
@pytest.mark.parametrize("sweep", ["ring", "pair", "split"])
@pytest.mark.parametrize("name", sorted(SST_MESHES))
def test_sst_implicit_step_parity(F, name, sweep, precision, monkeypatch):
    """The implicit SST variant (params.sst_sweeps = m, reading r34): the system rows written by
    the SST launch (ring or split), then the Jacobi sweeps, for m = 1 (one finishing launch) and
    m = 4 (two increment buffers in turn).  FP64 to the SST gates over 1 and 3 steps; FP32-dev to
    2e-6 of U for u and 2e-6 relative for k, omega after one step."""
    make, extra = SST_MESHES[name]
    m = make()
    _, p0, f, k, w = _sst_case(m, extra, 54)
    point = O.Oracle(m, p0).step(f, k, w)
    for sweeps in (1, 4):
        say("sst implicit step", name, sweep, precision, "sweeps", sweeps)
        monkeypatch.setenv("FVLBM_SWEEP", sweep)
        p = dict(p0, sst_sweeps=sweeps)
        orc = O.Oracle(m, p)
        st = F.State(F.Mesh(m), p, precision=precision, k=k, omega=w)
        st.set_state(f, k, w)
        fo, ko, wo = f, k, w
        for nsteps, tol in ((1, 1e-12), (2, 1e-11)):
            fo, ko, wo = orc.run(fo, ko, wo, nsteps)
            st.step(nsteps)
            mo = st.moments()
            if precision == "fp64":
                got = st.get_f()
                assert rel(got, fo, dev_scale(fo)) < tol, ("f", nsteps, rel(got, fo, dev_scale(fo)))
                assert rel(mo["k"], ko, np.abs(ko).max()) < tol * 10, ("k", nsteps, rel(mo["k"], ko, np.abs(ko).max()))
                assert rel(mo["omega"], wo, np.abs(wo).max()) < tol * 10, ("w", nsteps)
                assert rel(mo["nu_t"], orc.last_nut, np.abs(orc.last_nut).max()) < tol * 10, ("nu_t", nsteps)
            elif nsteps == 1:
                _, ux, uy, _ = orc.macro(fo)
                du = max(np.abs(mo["u"][:, 0] - ux).max(), np.abs(mo["u"][:, 1] - uy).max()) / 0.05
                assert du < 2e-6, du
                assert rel(mo["k"], ko, np.abs(ko).max()) < 2e-6, rel(mo["k"], ko, np.abs(ko).max())
                assert rel(mo["omega"], wo, np.abs(wo).max()) < 2e-6, rel(mo["omega"], wo, np.abs(wo).max())
            if nsteps == 1:
                # the variant is active: its k differs from the point-implicit one's
                assert rel(ko, point[1], np.abs(point[1]).max()) > 1e-9


def test_sst_implicit_per_stage_step_parity(F, monkeypatch):
    """The implicit variant with the per-stage coupling (both SST solves implicit), ring path."""
    say("sst implicit + per-stage, backstep_coarse, ring")
    monkeypatch.setenv("FVLBM_SWEEP", "ring")
    make, extra = SST_MESHES["backstep_coarse"]
    m = make()
    _, p0, f, k, w = _sst_case(m, extra, 55)
    p = dict(p0, sst_sweeps=3, sst_stages=1)
    orc = O.Oracle(m, p)
    st = F.State(F.Mesh(m), p, precision="fp64", k=k, omega=w)
    st.set_state(f, k, w)
    fo, ko, wo = orc.run(f, k, w, 2)
    st.step(2)
    mo = st.moments()
    assert rel(st.get_f(), fo, dev_scale(fo)) < 1e-11
    assert rel(mo["k"], ko, np.abs(ko).max()) < 1e-10
    assert rel(mo["omega"], wo, np.abs(wo).max()) < 1e-10


def _wide_halo_backstep():
    """A backstep (13,196 cells) whose stretched wall cells give Morton tiles with more than 256
    cells in ring 1 and ring 2 together (tests/test_host_library.py checks the count): more than
    one per thread."""
    return mg.backstep(core=0.3, dx_core=0.6, dx_corner=0.02, y1=1e-3)


@pytest.mark.parametrize("sweep", ["ring", "pair"])
@pytest.mark.parametrize("order", ["morton", "tiles"])
def test_wide_halo_ring_step_parity(F, order, sweep, monkeypatch):
    """The ring kernels loop over ring-2 cells beyond one per thread (Morton tiles of this mesh need
    it).  SST steps against the oracle, under Morton tiles and under the graph-grown tiles the
    library uses by default: FP32-dev on the ring path (its LDS fits), FP64 on whichever path fits;
    gates as the SST parity tests (FP64 1e-12 / 1e-11, FP32-dev 2e-6 after one step)."""
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    m = _wide_halo_backstep()
    extra = dict(group_u=[[0, 0], [0.05, 0], [0, 0]], group_k=[0, 1e-4, 0], group_w=[0, 0.5, 0])
    orc, p, f, k, w = _sst_case(m, extra, 56)
    f1, k1, w1 = orc.step(f, k, w)
    nut1 = orc.last_nut
    M = F.Mesh(m, order=order)
    for precision in ("fp64", "fp32dev"):
        say("wide-halo backstep", order, sweep, precision)
        st = F.State(M, p, precision=precision, k=k, omega=w)
        st.set_state(f, k, w)
        st.timing(True)
        st.step(1)
        kt = st.timing_read()
        st.timing(False)
        ring = kt["sst"][1] == 1 and kt["collide1"][1] == 0
        print(precision, "ring path" if ring else "tiled / split path")
        if precision == "fp32dev":
            assert ring, kt
        mo = st.moments()
        if precision == "fp64":
            got = st.get_f()
            assert rel(got, f1, dev_scale(f1)) < 1e-12
            assert rel(mo["k"], k1, np.abs(k1).max()) < 1e-11
            assert rel(mo["omega"], w1, np.abs(w1).max()) < 1e-11
            assert rel(mo["nu_t"], nut1, np.abs(nut1).max()) < 1e-11
        else:
            _, ux, uy, _ = orc.macro(f1)
            du = max(np.abs(mo["u"][:, 0] - ux).max(), np.abs(mo["u"][:, 1] - uy).max()) / 0.05
            print(order, "fp32dev max |du| / U after one step:", du)
            assert du < 2e-6, du
            assert rel(mo["k"], k1, np.abs(k1).max()) < 2e-6 and rel(mo["omega"], w1, np.abs(w1).max()) < 2e-6


@pytest.mark.parametrize("sweep", ["ring", "pair"])
@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_step_is_independent_of_the_tile_layout(F, precision, sweep, monkeypatch):
    """Every cell forms its LSQ coefficients, gradient, face values and update from its own data with
    the same code whether it is a tile cell or a halo cell of another tile, so the ring path's result
    must not depend on how the cells are grouped into tiles: three SST steps under Morton tiles and
    under graph-grown tiles agree to the last bit (f, k, omega in the caller's cell order)."""
    say("tile-layout independence", precision, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    m = _wide_halo_backstep()
    extra = dict(group_u=[[0, 0], [0.05, 0], [0, 0]], group_k=[0, 1e-4, 0], group_w=[0, 0.5, 0])
    orc, p, f, k, w = _sst_case(m, extra, 57)
    out = {}
    for order in ("morton", "tiles"):
        st = F.State(F.Mesh(m, order=order), p, precision=precision, k=k, omega=w)
        st.set_state(f, k, w)
        st.timing(True)
        st.step(3)
        kt = st.timing_read()
        assert kt["sst"][1] == 3 and kt["collide1"][1] == 0, kt      # the ring path
        mo = st.moments()
        out[order] = (st.get_f(), mo["k"], mo["omega"])
        del st
    for a, b in zip(out["morton"], out["tiles"]):
        np.testing.assert_array_equal(a, b)
