"""GPU adjoint: transposed operators and the full discrete adjoint against complex-step derivatives
of the FP64 oracle (h = 1e-30, exact to rounding) and centred finite differences.

Dot-product tests: for the transpose A^T of an operator's Jacobian A at a state, <A^T lam, v> must
equal <lam, A v>, where A v is the oracle's complex-step directional derivative.
"""
import os
import sys

import numpy as np
import pytest

from oracle import fvlbm_oracle as O
from paper_1812_00394_amd import meshgen as mg

pytestmark = pytest.mark.gpu

H = 1e-30
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def check_fp32_gradient(g, ref, res32=None):
    """The FP32-deviation adjoint's gate: normwise, max |g - ref| <= 1e-3 max |ref| over the five
    parameters, and the inflow angle within 1e-3 of its own value.  A componentwise relative gate
    does not fit FP32: the parameter gradients sum lambda . dR/dp over every cell and step with
    cancellation, so a component a thousand times smaller than the largest carries an error of the
    largest's rounding level (measured: 1e-2 relative on sigma_w1 at 1e-3 of the scale, while no
    component's error exceeded 7.4e-4 of the largest in 6 cases).  That error does not follow the
    FP32 resolution of the initial non-equilibrium part (res32, printed): over a 100x range of the
    non-equilibrium amplitude the largest component's error moved between 1.7e-4 and 2.8e-3
    relative with no trend."""
    g, ref = np.asarray(g), np.asarray(ref)
    scale = np.abs(ref).max()
    err = np.abs(g - ref)
    print("fp32dev gradient", g, "reference", ref, "error / max|ref|", err / scale,
          "relative error", err / np.abs(ref), "res32", res32)
    assert err.max() <= 1e-3 * scale, (g, ref)
    assert err[0] <= 1e-3 * abs(ref[0]), (g[0], ref[0])


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


MESHES = {
    "cavity": (lambda: mg.cavity(n=10, jitter=0.2, seed=61), dict(group_u=[[0, 0], [0.1, 0]])),
    "periodic": (lambda: mg.rectangle(7, 6, kind="periodic", jitter=0.25, seed=62), dict()),
    "duct": (lambda: mg.rectangle(9, 6, Lx=1.4, kind="duct", jitter=0.25, seed=63),
             dict(group_u=[[0.05, 0.01], [0, 0], [0.05, 0.0]], group_rho=[1.0, 1.002, 1.0], theta=0.2)),
    "naca": (lambda: mg.naca_omesh(n_wall=32, n_normal=10, y1=2e-3, radius=6.0),
             dict(group_u=[[0, 0], [0.05, 0]], theta=0.1)),
}


def _state(n, rng):
    rho = 1 + 0.01 * rng.standard_normal(n)
    ux, uy = 0.05 * rng.standard_normal((2, n))
    return O.feq(rho, ux, uy) + 2e-4 * O.WT[:, None] * rng.standard_normal((9, n))


@pytest.mark.parametrize("sweep", ["ring", "split"])
@pytest.mark.parametrize("name", sorted(MESHES))
def test_advection_transpose_dot_product(F, name, sweep, monkeypatch):
    """The ring-tiled transposed convection and the three-kernel one (split path)."""
    say("advection transpose", name, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    make, extra = MESHES[name]
    m = make()
    p = O.default_params(nu=1e-3, dt=1e-2, **extra)
    orc = O.Oracle(m, p)
    n = orc.g.n
    rng = np.random.default_rng(70)
    g = _state(n, rng)
    v = rng.standard_normal((9, n)) * O.WT[:, None]
    lam = rng.standard_normal((9, n))
    lam[0] = 0.0                      # the rest direction has no convection term
    Jv = np.imag(orc.advection(g + 1j * H * v)) / H
    st = F.State(F.Mesh(m), p, precision="fp64")
    gbar, dth = st.apply_advection_adjoint(g, lam)
    lhs, rhs = np.sum(gbar * v), np.sum(lam * Jv)
    assert abs(lhs - rhs) <= 1e-11 * max(abs(rhs), np.abs(lam * Jv).sum() * 1e-3), (lhs, rhs)
    # theta
    pc = dict(p, theta=p.get("theta", 0.0) + 1j * H)
    dGa = np.imag(O.Oracle(m, pc).advection(g.astype(complex))) / H
    ref = np.sum(lam * dGa)
    assert abs(dth - ref) <= 1e-10 * max(abs(ref), 1e-12), (dth, ref)


# ------------------------------------------------------------------------------------------------
# Whole-run adjoint (checkpointed reverse of several IMEX steps)
# ------------------------------------------------------------------------------------------------
def _courant_dt(m, C):
    G = O.Geometry(m)
    en = np.maximum(O.EX[:, None] * G.nl[:, 0] + O.EY[:, None] * G.nl[:, 1], 0.0)
    out = np.stack([np.bincount(G.cell, weights=en[a], minlength=G.n) for a in range(9)])
    return C / (out / G.area).max()


RUNS = {
    # name: (mesh, flow extras, sst)
    "duct_laminar": (lambda: mg.rectangle(9, 6, Lx=1.4, kind="duct", jitter=0.25, seed=63),
                     dict(group_u=[[0.05, 0.01], [0, 0], [0.05, 0.0]], group_rho=[1.0, 1.002, 1.0], theta=0.2), False),
    "backstep_sst": (lambda: mg.backstep(core=0.35, dx_core=0.7, y1=1.5e-2, dx_corner=0.08, wall_layers=2),
                     dict(group_u=[[0, 0], [0.05, 0.004], [0, 0]], group_k=[0, 2e-4, 0], group_w=[0, 0.4, 0],
                          theta=0.05, jr_group=0, jr_xmin=0.0, eps_tau=1e-7), True),
    "naca_sst": (lambda: mg.naca_omesh(n_wall=32, n_normal=10, y1=4e-3, radius=5.0),
                 dict(group_u=[[0, 0], [0.05, 0]], group_k=[0, 2e-4], group_w=[0, 0.4], theta=0.12), True),
}


def _run_case(name, seed=80, amp=2e-5):
    make, extra, sst = RUNS[name]
    m = make()
    dt = _courant_dt(m, 0.5)
    p = O.default_params(nu=dt / 40, dt=dt, sst=sst, **extra)
    orc = O.Oracle(m, p)
    n = orc.g.n
    rng = np.random.default_rng(seed)
    x, y = orc.g.xc[:, 0], orc.g.xc[:, 1]
    ux = 0.04 * np.tanh(2 * (y - y.mean())) + 0.004 * rng.standard_normal(n)
    uy = 0.006 * np.sin(2 * x) + 0.004 * rng.standard_normal(n)
    rho = 1 + 0.002 * rng.standard_normal(n)
    f0 = O.feq(rho, ux, uy) + amp * O.WT[:, None] * rng.standard_normal((9, n))
    k0 = 2e-4 * (1 + 0.5 * rng.random(n)) if sst else None
    w0 = 0.4 * (1 + 0.5 * rng.random(n)) if sst else None
    return m, p, orc, f0, k0, w0, sst


def _oracle_final(m, p, f0, k0, w0, N):
    orc = O.Oracle(m, p)
    return orc.run(f0, k0, w0, N)


PARAMS = ["theta", "sigma_k1", "sigma_w1", "beta_star", "a1"]


@pytest.mark.parametrize("sweep", ["ring", "pair", "split", "face"])
@pytest.mark.parametrize("name", sorted(RUNS))
def test_run_adjoint_dot_product_and_params(F, name, sweep, monkeypatch):
    say("run adjoint", name, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    m, p, orc, f0, k0, w0, sst = _run_case(name)
    _check_run_adjoint(F, m, p, f0, k0, w0, sst, 3)


@pytest.mark.parametrize("sweep", ["ring", "split"])
@pytest.mark.parametrize("name", ["backstep_sst", "naca_sst"])
def test_per_stage_sst_adjoint(F, name, sweep, monkeypatch):
    """The adjoint of the per-stage SST coupling (params.sst = 2, reading r33): the second SST solve,
    on the stage-2 macro variables, gives the third stage's tau3 and the step's k, omega; its reverse
    sends the tau3 adjoint of the third stage's solve back through that solve onto f^(2), k^n,
    omega^n, and the first solve's reverse carries the tau adjoint of stages 1 and 2 alone.  Dot
    product of a 3-step recorded run's adjoint (checkpoint every 2) with the oracle's complex step,
    within 1e-9, and the parameter gradients within 1e-8."""
    say("per-stage sst adjoint", name, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    m, p, orc, f0, k0, w0, sst = _run_case(name, seed=83)
    p = dict(p, sst_stages=1)
    # the variant is active: its state differs from the once-per-step coupling's
    a = O.Oracle(m, p).run(f0, k0, w0, 2)[0]
    b = O.Oracle(m, dict(p, sst_stages=0)).run(f0, k0, w0, 2)[0]
    assert np.abs(a - b).max() > 1e-9 * np.abs(a - O.WT[:, None]).max()
    _check_run_adjoint(F, m, p, f0, k0, w0, sst, 3)


@pytest.mark.parametrize("sweep", ["ring", "split"])
@pytest.mark.parametrize("m_sweeps", [1, 5])
@pytest.mark.parametrize("name", ["backstep_sst", "naca_sst"])
def test_implicit_sst_adjoint(F, name, m_sweeps, sweep, monkeypatch):
    """The adjoint of the implicit SST variant (params.sst_sweeps = m, reading r34): the increments'
    system formed again from the recorded closure, m - 1 transposed Jacobi sweeps, the reverse of
    the rows (mass fluxes, diffusion conductances, sinks, sources) onto the macro variables, k^n,
    omega^n, Gamma, s, beta and the parameters.  Dot product of a 3-step recorded run's adjoint
    (checkpoint every 2) with the oracle's complex step, within 1e-9, and the parameter gradients
    within 1e-8."""
    say("implicit sst adjoint", name, m_sweeps, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    m, p, orc, f0, k0, w0, sst = _run_case(name, seed=85)
    p = dict(p, sst_sweeps=m_sweeps)
    # the variant is active: its k differs from the point-implicit update's
    a = O.Oracle(m, p).run(f0, k0, w0, 2)[1]
    b = O.Oracle(m, dict(p, sst_sweeps=0)).run(f0, k0, w0, 2)[1]
    assert np.abs(a - b).max() > 1e-6 * np.abs(a).max()
    _check_run_adjoint(F, m, p, f0, k0, w0, sst, 3)


def test_implicit_sst_adjoint_sweep_limit(F):
    """Recording refuses the implicit variant beyond 16 sweeps (the reverse keeps every sweep's
    increments), before it changes the state."""
    m, p, orc, f0, k0, w0, sst = _run_case("backstep_sst", seed=85)
    st = F.State(F.Mesh(m), dict(p, sst_sweeps=17), precision="fp64", k=k0, omega=w0)
    st.set_state(f0, k0, w0)
    with pytest.raises(F.FvlbmError, match="ESTATE"):
        st.record(2, ckpt_every=2)
    np.testing.assert_array_equal(st.get_f(), f0)


@pytest.mark.parametrize("sweep", ["ring", "split"])
@pytest.mark.parametrize("limiter", [1, 2])
def test_fp32_limited_adjoint(F, limiter, sweep, monkeypatch):
    """The FP32-deviation adjoint through the limiters (face-value clip of r32, gradient limiter of
    r35) on the SST O-mesh: the gradient of lam . final state over 3 recorded steps (checkpoint every
    2) meets the FP32 gate of check_fp32_gradient against the oracle's complex step."""
    say("fp32dev limited adjoint", limiter, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    m, p, orc, f0, k0, w0, sst = _run_case("naca_sst", seed=89)
    p = dict(p, limiter=limiter)
    n = f0.shape[1]
    N = 3
    rng = np.random.default_rng(90)
    lf = rng.standard_normal((9, n))
    lk = rng.standard_normal(n) * 1e3
    lw = rng.standard_normal(n)
    st = F.State(F.Mesh(m), p, precision="fp32dev", k=k0, omega=w0)
    st.set_state(f0, k0, w0)
    st.record(N, ckpt_every=2)
    g = st.adjoint_state(lf, lk, lw)[3]
    ref = []
    for key in PARAMS:
        pc = dict(p)
        pc[key] = p[key] + 1j * H
        fN, kN, wN = _oracle_final(m, pc, f0.astype(complex), k0.astype(complex), w0.astype(complex), N)
        ref.append((np.sum(lf * np.imag(fN)) + np.sum(lk * np.imag(kN)) + np.sum(lw * np.imag(wN))) / H)
    check_fp32_gradient(g, np.asarray(ref))


@pytest.mark.parametrize("name, limiter", [("backstep_sst", 0), ("naca_sst", 0), ("naca_sst", 1)])
def test_fp32_with_fp64_geometry_adjoint(F, name, limiter, monkeypatch):
    """The adjoint of an FP32-deviation state whose ring sweeps form the edge data from FP64 geometry
    (precision fp32dev_geo64): its recorded steps run those kernels, its reverse the FP32-geometry
    transposes.  The gradient of lam . final state over 3 recorded steps (checkpoint every 2) meets
    the FP32 gate of check_fp32_gradient against the oracle's complex step, and stays within that
    gate of the FP32-geometry state's gradient; the recorded run ends at the unrecorded run's state
    (bitwise; with the face-value limiter, whose recorded sweeps also keep the clip states, to FP32
    rounding)."""
    say("fp32dev_geo64 adjoint", name, "limiter", limiter)
    monkeypatch.setenv("FVLBM_SWEEP", "ring")
    m, p, orc, f0, k0, w0, sst = _run_case(name, seed=87)
    p = dict(p, limiter=limiter)
    n = f0.shape[1]
    N = 3
    rng = np.random.default_rng(88)
    lf = rng.standard_normal((9, n))
    lk = rng.standard_normal(n) * 1e3
    lw = rng.standard_normal(n)
    M = F.Mesh(m)
    grads = {}
    for precision in ("fp32dev", "fp32dev_geo64"):
        plain = F.State(M, p, precision=precision, k=k0, omega=w0)
        plain.set_state(f0, k0, w0)
        plain.step(N)
        st = F.State(M, p, precision=precision, k=k0, omega=w0)
        st.set_state(f0, k0, w0)
        st.record(N, ckpt_every=2)
        if limiter == 0:
            np.testing.assert_array_equal(st.get_f(), plain.get_f())
        else:
            # the recording kernels of the clip are other instantiations: FP32 rounding apart
            fp = plain.get_f()
            assert np.abs(st.get_f() - fp).max() <= 1e-6 * np.abs(fp - O.WT[:, None]).max()
        grads[precision] = st.adjoint_state(lf, lk, lw)[3]
        del st, plain
    ref = []
    for key in PARAMS:
        pc = dict(p)
        pc[key] = p[key] + 1j * H
        fN, kN, wN = _oracle_final(m, pc, f0.astype(complex), k0.astype(complex), w0.astype(complex), N)
        ref.append((np.sum(lf * np.imag(fN)) + np.sum(lk * np.imag(kN)) + np.sum(lw * np.imag(wN))) / H)
    ref = np.asarray(ref)
    print("fp32dev", grads["fp32dev"], "fp32dev_geo64", grads["fp32dev_geo64"], "complex step", ref)
    check_fp32_gradient(grads["fp32dev_geo64"], ref)
    check_fp32_gradient(grads["fp32dev_geo64"], grads["fp32dev"])


def _check_run_adjoint(F, m, p, f0, k0, w0, sst, N):
    """Records N steps (checkpoint every 2) and checks the adjoint's dot product with the oracle's
    complex-step derivative along a random direction (1e-9) and the five parameter gradients of
    lam . final state (1e-8)."""
    n = f0.shape[1]
    st = F.State(F.Mesh(m), p, precision="fp64", k=k0, omega=w0)
    st.set_state(f0, k0, w0)
    st.record(N, ckpt_every=2)
    rng = np.random.default_rng(81)
    lf = rng.standard_normal((9, n))
    lk = rng.standard_normal(n) * 1e3 if sst else None
    lw = rng.standard_normal(n) if sst else None
    lf0, lk0, lw0, dp = st.adjoint_state(lf, lk, lw)
    # directional derivative of the final state along a random initial perturbation
    vf = rng.standard_normal((9, n)) * O.WT[:, None] * 1e-3
    vk = rng.standard_normal(n) * 1e-5 if sst else None
    vw = rng.standard_normal(n) * 1e-2 if sst else None
    fN, kN, wN = _oracle_final(m, p, f0 + 1j * H * vf, None if not sst else k0 + 1j * H * vk,
                               None if not sst else w0 + 1j * H * vw, N)
    rhs = np.sum(lf * np.imag(fN)) / H
    lhs = np.sum(lf0 * vf)
    if sst:
        rhs += (np.sum(lk * np.imag(kN)) + np.sum(lw * np.imag(wN))) / H
        lhs += np.sum(lk0 * vk) + np.sum(lw0 * vw)
    assert abs(lhs - rhs) <= 1e-9 * abs(rhs), (lhs, rhs)
    # parameter derivatives of lam . final state
    for i, key in enumerate(PARAMS):
        if not sst and key != "theta":
            assert dp[i] == 0.0
            continue
        pc = dict(p)
        pc[key] = p[key] + 1j * H
        fN, kN, wN = _oracle_final(m, pc, f0.astype(complex), None if not sst else k0.astype(complex),
                                   None if not sst else w0.astype(complex), N)
        ref = np.sum(lf * np.imag(fN)) / H
        if sst:
            ref += (np.sum(lk * np.imag(kN)) + np.sum(lw * np.imag(wN))) / H
        assert abs(dp[i] - ref) <= 1e-8 * max(abs(ref), 1e-30), (key, dp[i], ref)


def test_adjoint_forces_complex_step_fd_and_checkpoints(F):
    """d(F_x, F_y, J_R)/d params over 4 recorded steps: against complex step on the oracle (1e-8),
    against centred differences of the GPU forward (eps = 1e-6 max(|p|, 1); 1e-3 plus the rounding
    floor), and independent of the checkpoint interval (1, 3, 4)."""
    say("adjoint of forces, backstep sst")
    m, p, orc, f0, k0, w0, sst = _run_case("backstep_sst", seed=90)
    N = 4
    seed = np.array([0.7, -1.3, 2.0])

    def J_of(orc_like, f, k, w):
        Fv, JR = orc_like.forces(f, 1)
        return seed[0] * Fv[0] + seed[1] * Fv[1] + seed[2] * JR

    results = []
    for ck in (1, 3, 4):
        st = F.State(F.Mesh(m), p, precision="fp64", k=k0, omega=w0)
        st.set_state(f0, k0, w0)
        st.record(N, ckpt_every=ck)
        results.append(st.adjoint(1, seed))
    for r in results[1:]:
        np.testing.assert_allclose(r, results[0], rtol=1e-12, atol=1e-300)
    dp = results[0]
    for i, key in enumerate(PARAMS):
        pc = dict(p)
        pc[key] = p[key] + 1j * H
        o = O.Oracle(m, pc)
        fN, kN, wN = o.run(f0.astype(complex), k0.astype(complex), w0.astype(complex), N)
        ref = np.imag(J_of(o, fN, kN, wN)) / H
        assert abs(dp[i] - ref) <= 1e-8 * max(abs(ref), 1e-30), (key, dp[i], ref)
        # centred differences of the GPU forward
        eps = 1e-6 * max(abs(p[key]), 1.0)
        Jpm = []
        for sgn in (1, -1):
            pp = dict(p)
            pp[key] = p[key] + sgn * eps
            s2 = F.State(F.Mesh(m), pp, precision="fp64", k=k0, omega=w0)
            s2.set_state(f0, k0, w0)
            s2.step(N)
            Fv, JR = s2.forces(1)
            Jpm.append(seed[0] * Fv[0] + seed[1] * Fv[1] + seed[2] * JR)
        fd = (Jpm[0] - Jpm[1]) / (2 * eps)
        # central differences straddle the kinks of the scheme (bounds, upwind and max / min
        # switches) and lose digits to rounding when the derivative is small: the exact reference
        # is the complex step, the difference quotient a sanity check at 1e-3 plus its rounding floor
        floor = 1e-13 * (abs(Jpm[0]) + abs(Jpm[1])) / eps
        assert abs(dp[i] - fd) <= 1e-3 * abs(ref) + floor, (key, dp[i], fd, floor)


@pytest.mark.parametrize("amp", [2e-6, 2e-5, 2e-4])
def test_autograd_function_and_fp32(F, amp):
    """torch.autograd through FVLBMObjective equals the oracle's complex-step gradient (FP64 to
    1e-8).  The FP32-deviation adjoint meets the gate of check_fp32_gradient, at three amplitudes of
    the initial non-equilibrium part (the resolution estimate res32 spans 100x)."""
    say("autograd objective, backstep sst, non-equilibrium amplitude", amp)
    import torch
    from paper_1812_00394_amd.autograd import FVLBMObjective, Problem, PARAM_NAMES
    m, p, orc, f0, k0, w0, sst = _run_case("backstep_sst", seed=91, amp=amp)
    n = orc.g.n
    N = 3
    w = torch.tensor([0.3, -0.8, 1.5], dtype=torch.float64)
    ref = []
    for key in PARAM_NAMES:
        pc = dict(p)
        pc[key] = p[key] + 1j * H
        o = O.Oracle(m, pc)
        fN, _, _ = o.run(f0.astype(complex), k0.astype(complex), w0.astype(complex), N)
        Fv, JR = o.forces(fN, 1)
        ref.append(np.imag(w[0].item() * Fv[0] + w[1].item() * Fv[1] + w[2].item() * JR) / H)
    ref = np.array(ref)
    rho0, ux0, uy0, _ = orc.macro(f0)
    neq_rms = np.sqrt(np.mean((f0 - O.feq(rho0, ux0, uy0)) ** 2))
    res32 = 2.0 ** -24 * np.abs(f0 - O.WT[:, None] * p["rho0"]).max() / neq_rms
    say("FP32 resolution of the initial non-equilibrium part", res32)
    for precision in ("fp64", "fp32dev"):
        prob = Problem(F.Mesh(m), p, rho=np.ones(n), u=np.zeros((n, 2)), k=k0, omega=w0, n_steps=N,
                       ckpt_every=2, wall_mask=1, precision=precision, f0=f0)
        params = torch.tensor([p[k] for k in PARAM_NAMES], dtype=torch.float64, requires_grad=True)
        J = FVLBMObjective.apply(params, prob)
        (J @ w).backward()
        g = params.grad.numpy()
        if precision == "fp32dev":
            check_fp32_gradient(g, ref, res32)
            continue
        rel = np.abs(g - ref) / np.maximum(np.abs(ref), 1e-30)
        print(precision, "adjoint gradient", g, "relative error", rel)
        scale = np.abs(ref).max()
        assert np.all(np.abs(g - ref) <= 1e-8 * np.maximum(np.abs(ref), 1e-6 * scale)), (precision, g, ref)


@pytest.mark.parametrize("order", ["morton", "tiles"])
def test_wide_halo_ring_adjoint_fp32(F, order):
    """The ring adjoint kernels with ring-2 cells beyond one per thread (the 13,196-cell backstep of
    the forward wide-halo test, FP32-dev on the ring path): the autograd gradient of the force
    objective against the oracle's complex step, to the gate of check_fp32_gradient."""
    say("wide-halo backstep adjoint, fp32dev ring", order)
    import torch
    from paper_1812_00394_amd.autograd import FVLBMObjective, Problem, PARAM_NAMES
    m = mg.backstep(core=0.3, dx_core=0.6, dx_corner=0.02, y1=1e-3)
    dt = _courant_dt(m, 0.5)
    p = O.default_params(nu=dt / 40, dt=dt, sst=True, group_u=[[0, 0], [0.05, 0.004], [0, 0]],
                         group_k=[0, 2e-4, 0], group_w=[0, 0.4, 0], theta=0.05, jr_group=0, jr_xmin=0.0,
                         eps_tau=1e-7)
    orc = O.Oracle(m, p)
    n = orc.g.n
    rng = np.random.default_rng(92)
    x, y = orc.g.xc[:, 0], orc.g.xc[:, 1]
    ux = 0.04 * np.tanh(2 * (y - y.mean())) + 0.004 * rng.standard_normal(n)
    uy = 0.006 * np.sin(2 * x) + 0.004 * rng.standard_normal(n)
    f0 = O.feq(1 + 0.002 * rng.standard_normal(n), ux, uy) + 2e-5 * O.WT[:, None] * rng.standard_normal((9, n))
    k0, w0 = 2e-4 * (1 + 0.5 * rng.random(n)), 0.4 * (1 + 0.5 * rng.random(n))
    M = F.Mesh(m, order=order)        # Morton tiles need the ring-2 loop; graph tiles are the default
    probe = F.State(M, p, precision="fp32dev", k=k0, omega=w0)
    probe.timing(True)
    probe.step(1)
    kt = probe.timing_read()
    assert kt["sst"][1] == 1 and kt["collide1"][1] == 0, kt     # the ring path
    del probe
    N = 3
    wts = torch.tensor([0.3, -0.8, 1.5], dtype=torch.float64)
    ref = []
    for key in PARAM_NAMES:
        pc = dict(p)
        pc[key] = p[key] + 1j * H
        o = O.Oracle(m, pc)
        fN, _, _ = o.run(f0.astype(complex), k0.astype(complex), w0.astype(complex), N)
        Fv, JR = o.forces(fN, 1)
        ref.append(np.imag(wts[0].item() * Fv[0] + wts[1].item() * Fv[1] + wts[2].item() * JR) / H)
    ref = np.array(ref)
    rho0, ux0, uy0, _ = orc.macro(f0)
    neq_rms = np.sqrt(np.mean((f0 - O.feq(rho0, ux0, uy0)) ** 2))
    res32 = 2.0 ** -24 * np.abs(f0 - O.WT[:, None] * p["rho0"]).max() / neq_rms
    prob = Problem(M, p, rho=np.ones(n), u=np.zeros((n, 2)), k=k0, omega=w0, n_steps=N, ckpt_every=2,
                   wall_mask=1, precision="fp32dev", f0=f0)
    params = torch.tensor([p[k] for k in PARAM_NAMES], dtype=torch.float64, requires_grad=True)
    J = FVLBMObjective.apply(params, prob)
    (J @ wts).backward()
    check_fp32_gradient(params.grad.numpy(), ref, res32)


def test_adjoint_single_segment_set_equals_overlapped(F, monkeypatch):
    """Large meshes keep one set of segment buffers and recompute on the caller's stream; small ones
    recompute the next segment on a second stream into a second set.  Forced here on one small mesh
    (FVLBM_ADJ_OVERLAP=0) with three segments: the same adjoint state and parameter gradient to the
    last bit, and the same as a recording without checkpoints."""
    say("adjoint, one segment set vs two, backstep sst")
    m, p, orc, f0, k0, w0, sst = _run_case("backstep_sst", seed=93)
    n = orc.g.n
    rng = np.random.default_rng(94)
    lf, lk, lw = rng.standard_normal((9, n)), rng.standard_normal(n) * 1e3, rng.standard_normal(n)
    M = F.Mesh(m)
    out = {}
    for key, env, ckpt in (("two", "1", 2), ("one", "0", 2), ("whole", "1", 5)):
        monkeypatch.setenv("FVLBM_ADJ_OVERLAP", env)
        st = F.State(M, p, precision="fp64", k=k0, omega=w0)
        st.set_state(f0, k0, w0)
        st.record(5, ckpt_every=ckpt)
        out[key] = st.adjoint_state(lf, lk, lw)
        del st
    for a, b in zip(out["two"], out["one"]):
        np.testing.assert_array_equal(np.asarray(a), np.asarray(b))
    for a, b in zip(out["two"], out["whole"]):
        np.testing.assert_array_equal(np.asarray(a), np.asarray(b))


@pytest.mark.timeout(300)
def test_c4_derivatives_at_full_length(F):
    """The adjoint workload at its stated length: 400 IMEX + SST steps with a checkpoint every 20 on
    the seeded 800-cell piece of the backstep of tests/c4case.py (walls behind the step, far-field cut
    edges so that the inflow angle acts, the step's flow parameters).  d(w . (F_x, F_y, J_R))/d(theta,
    sigma_k1, sigma_w1, beta*, a1) against the oracle's complex step and centred differences stored by
    tests/golden/make_c4_fixture.py:
      FP64: complex step within 1e-8 relative; centred differences within 1e-3 relative plus their
            rounding floor 1e-13 |J| / eps; checkpoint intervals 1, 20 and 400 agree to 1e-12;
      FP32-deviation: the gate of check_fp32_gradient (1e-3 normwise, 1e-3 on theta)."""
    import json
    from tests import c4case as C
    fx = json.load(open(os.path.join(GOLDEN, "c4_piece_400.json")))
    m = C.piece()
    assert C.mesh_sha(m) == fx["mesh_sha256"], "the piece differs from the one the fixture was written for"
    p = dict(fx["params"])
    n = fx["n_cells"]
    rho, ux, uy, noise, k0, w0 = C.initial_fields(m)
    f0 = O.feq(rho, ux, uy) + 1e-5 * O.WT[:, None] * noise
    seed = np.array(fx["functional_weights"])
    cs, fd, eps = np.array(fx["complex_step"]), np.array(fx["central_difference"]), np.array(fx["fd_eps"])
    N = fx["n_steps"]
    say("C4 full length:", n, "cells,", N, "steps")
    M = F.Mesh(m)
    scale = np.abs(cs).max()
    fd_floor = 1e-13 * abs(fx["J"]) / eps
    assert np.all(np.abs(fd - cs) <= 1e-3 * np.abs(cs) + fd_floor), (fd, cs)     # the fixture itself
    g = {}
    for ck in (20, 1, 400):
        st = F.State(M, p, precision="fp64", k=k0, omega=w0)
        st.set_state(f0, k0, w0)
        st.record(N, ckpt_every=ck)
        g[ck] = np.asarray(st.adjoint(1, seed))
        del st
    print("fp64 gradient", g[20], "complex step", cs, "centred differences", fd)
    rel = np.abs(g[20] - cs) / np.maximum(np.abs(cs), 1e-6 * scale)
    print("fp64 relative error against the complex step", rel)
    assert np.all(rel <= 1e-8), rel
    assert np.all(np.abs(g[20] - fd) <= 1e-3 * np.abs(cs) + fd_floor), (g[20], fd)
    for ck in (1, 400):
        assert np.all(np.abs(g[ck] - g[20]) <= 1e-12 * np.maximum(np.abs(g[20]), 1e-6 * scale)), (ck, g[ck], g[20])
    st = F.State(M, p, precision="fp32dev", k=k0, omega=w0)
    st.set_state(f0, k0, w0)
    st.record(N, ckpt_every=20)
    g32 = np.asarray(st.adjoint(1, seed))
    del st
    check_fp32_gradient(g32, cs)




@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_lift_drag_adjoint_against_complex_step(F, precision):
    """d(s . (C_l, C_d))/d(theta, sigma_k1, sigma_w1, beta*, a1) after 3 IMEX + SST steps on a small
    O-mesh around the 12 % section (Section 4's coefficients): theta turns the far-field stream and
    the lift and drag directions, both of which the oracle's complex step carries.  FP64 through the
    autograd wrapper within 1e-8 of the complex step; FP32-deviation through the C ABI to the gate
    of check_fp32_gradient."""
    say("lift/drag adjoint", precision)
    import torch
    from paper_1812_00394_amd.autograd import LiftDragObjective, Problem, PARAM_NAMES
    m, p, orc, f0, k0, w0, sst = _run_case("naca_sst", seed=96)
    n = orc.g.n
    U = 0.05
    N = 3
    s = np.array([0.8, -1.7])
    ref = []
    for key in PARAM_NAMES:
        pc = dict(p)
        pc[key] = p[key] + 1j * H
        o = O.Oracle(m, pc)
        fN, _, _ = o.run(f0.astype(complex), k0.astype(complex), w0.astype(complex), N)
        ref.append(np.imag(s @ o.lift_drag(fN, 1, U)) / H)
    ref = np.array(ref)
    fN, _, _ = orc.run(f0, k0, w0, N)
    cref = orc.lift_drag(fN, 1, U)
    assert abs(ref[0]) > 0 and np.all(ref[1:] != 0), ref
    if precision == "fp64":
        prob = Problem(F.Mesh(m), p, rho=np.ones(n), u=np.zeros((n, 2)), k=k0, omega=w0, n_steps=N, ckpt_every=2,
                       wall_mask=1, precision="fp64", f0=f0)
        params = torch.tensor([p[k] for k in PARAM_NAMES], dtype=torch.float64, requires_grad=True)
        C = LiftDragObjective.apply(params, prob, U)
        np.testing.assert_allclose(C.detach().numpy(), cref, rtol=1e-11)
        (C @ torch.tensor(s)).backward()
        g = params.grad.numpy()
        rel = np.abs(g - ref) / np.abs(ref)
        print("fp64 lift/drag gradient", g, "complex step", ref, "relative error", rel)
        assert np.all(rel <= 1e-8), rel
    else:
        st = F.State(F.Mesh(m), p, precision="fp32dev", k=k0, omega=w0)
        st.set_state(f0, k0, w0)
        st.record(N, ckpt_every=2)
        g, coeffs = st.adjoint_lift_drag(1, U, 1.0, s)
        check_fp32_gradient(g, ref)



@pytest.mark.parametrize("sweep", ["ring", "split", "face"])
@pytest.mark.parametrize("name", ["duct_laminar", "naca_sst"])
def test_gradient_limiter_adjoint_against_complex_step(F, name, sweep, monkeypatch):
    """The adjoint through the gradient limiter of reading r35 (on the two-kernel transposes, whichever
    sweep ran forward): the reverse finds again, from the recorded stage fields, each direction's
    limiting edge and the stencil value that set its bound, and passes the adjoint of psi on to the
    unlimited gradient, that value and the cell's own.  Dot product of a 3-step recorded run's
    adjoint (checkpoint every 2) with the oracle's complex step, within 1e-9, and the parameter
    gradients within 1e-8.  The case must limit: the limited oracle run differs from the unlimited
    one."""
    say("gradient limiter adjoint", name, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    m, p, orc, f0, k0, w0, sst = _run_case(name, seed=99)
    p = dict(p, limiter=2)
    f_lim = O.Oracle(m, p).run(f0, k0, w0, 3)[0]
    f_pln = O.Oracle(m, dict(p, limiter=0)).run(f0, k0, w0, 3)[0]
    change = np.abs(f_lim - f_pln).max() / np.abs(f_pln - O.WT[:, None]).max()
    print("effect of the limiter on the state after 3 steps:", change)
    assert change > 1e-6, change
    _check_run_adjoint(F, m, p, f0, k0, w0, sst, 3)


@pytest.mark.parametrize("sweep", ["ring", "pair", "split", "face"])
@pytest.mark.parametrize("name", ["duct_laminar", "naca_sst"])
def test_limited_adjoint_against_complex_step(F, name, sweep, monkeypatch):
    """The adjoint through the face-value limiter of reading r32: the ring-tiled forward sweeps record
    which edges were clipped and to which cell's value (the two-kernel reverse forms those states again
    from the stage field and its gradient planes), the transposed convection routes each clipped
    edge's adjoint to that value.  Dot product of the adjoint of a 3-step recorded run
    (checkpoint every 2) with the oracle's complex-step derivative along a random direction, within
    1e-9, and the parameter gradient within 1e-8; on the O-mesh the lift/drag adjoint as well.  The
    case must clip: the limited oracle run differs from the unlimited one."""
    say("limited adjoint", name, sweep)
    monkeypatch.setenv("FVLBM_SWEEP", sweep)
    m, p, orc, f0, k0, w0, sst = _run_case(name, seed=97)
    p = dict(p, limiter=1)
    n = orc.g.n
    N = 3
    f_lim, _, _ = O.Oracle(m, p).run(f0, k0, w0, N)
    f_pln, _, _ = O.Oracle(m, dict(p, limiter=0)).run(f0, k0, w0, N)
    change = np.abs(f_lim - f_pln).max() / np.abs(f_pln - O.WT[:, None]).max()
    print("effect of the limiter on the state after", N, "steps:", change)
    assert change > 1e-6, change
    rng = np.random.default_rng(98)
    lf = rng.standard_normal((9, n))
    lk = rng.standard_normal(n) * 1e3 if sst else None
    lw = rng.standard_normal(n) if sst else None
    st = F.State(F.Mesh(m), p, precision="fp64", k=k0, omega=w0)
    st.set_state(f0, k0, w0)
    st.record(N, ckpt_every=2)
    lf0, lk0, lw0, dp = st.adjoint_state(lf, lk, lw)
    vf = rng.standard_normal((9, n)) * O.WT[:, None] * 1e-3
    vk = rng.standard_normal(n) * 1e-5 if sst else None
    vw = rng.standard_normal(n) * 1e-2 if sst else None
    o = O.Oracle(m, p)
    if sst:
        fN, kN, wN = o.run(f0 + 1j * H * vf, k0 + 1j * H * vk, w0 + 1j * H * vw, N)
        rhs = (np.sum(lf * np.imag(fN)) + np.sum(lk * np.imag(kN)) + np.sum(lw * np.imag(wN))) / H
        lhs = np.sum(lf0 * vf) + np.sum(lk0 * vk) + np.sum(lw0 * vw)
    else:
        fN, _, _ = o.run(f0 + 1j * H * vf, None, None, N)
        rhs = np.sum(lf * np.imag(fN)) / H
        lhs = np.sum(lf0 * vf)
    print("dot products", lhs, rhs)
    assert abs(lhs - rhs) <= 1e-9 * abs(rhs), (lhs, rhs)
    # the parameter gradient of lambda . state against the complex step of each parameter
    keys = PARAMS if sst else PARAMS[:1]
    ref = []
    for key in keys:
        pc = dict(p)
        pc[key] = p[key] + 1j * H
        oc = O.Oracle(m, pc)
        fN, kN, wN = oc.run(f0.astype(complex), k0.astype(complex) if sst else None, w0.astype(complex) if sst else None, N)
        v = np.sum(lf * np.imag(fN))
        if sst:
            v += np.sum(lk * np.imag(kN)) + np.sum(lw * np.imag(wN))
        ref.append(v / H)
    ref = np.array(ref)
    scale = np.abs(ref).max()
    print("parameter gradient", dp[:len(keys)], "complex step", ref)
    assert np.all(np.abs(dp[:len(keys)] - ref) <= 1e-8 * np.maximum(np.abs(ref), 1e-6 * scale)), (dp, ref)
    if name == "naca_sst":
        U = 0.05
        s_ = np.array([0.8, -1.7])
        ld_ref = []
        for key in PARAMS:
            pc = dict(p)
            pc[key] = p[key] + 1j * H
            oc = O.Oracle(m, pc)
            fN, _, _ = oc.run(f0.astype(complex), k0.astype(complex), w0.astype(complex), N)
            ld_ref.append(np.imag(s_ @ oc.lift_drag(fN, 1, U)) / H)
        ld_ref = np.array(ld_ref)
        st2 = F.State(F.Mesh(m), p, precision="fp64", k=k0, omega=w0)
        st2.set_state(f0, k0, w0)
        st2.record(N, ckpt_every=2)
        g, _ = st2.adjoint_lift_drag(1, U, 1.0, s_)
        rel = np.abs(g - ld_ref) / np.abs(ld_ref)
        print("limited lift/drag gradient", g, "complex step", ld_ref, "relative error", rel)
        assert np.all(rel <= 1e-8), rel
