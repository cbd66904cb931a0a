"""Failure detection through the C ABI (Step 7 monitors of the Section 3.2 algorithm): a non-finite
value reaches FVLBM_EDIVERGED at the next reduction, a time step far beyond the advective Courant
limit diverges and is reported, a flow at rest has a zero residual, and a state change after
fvlbm_record drops the recording.  No kernel faults: NaN and overflow are ordinary values to the
kernels, and every loop in them has a fixed trip count."""
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


def _cavity():
    return mg.cavity(n=16, jitter=0.2, seed=31)


@pytest.mark.parametrize("prec", ["fp64", "fp32dev"])
def test_nan_in_one_cell_is_reported(F, prec):
    say("NaN in one wall cell", prec)
    m = _cavity()
    M = F.Mesh(m)
    dt = 0.5 * M.max_dt()
    p = O.default_params(nu=dt / 30, dt=dt, group_u=[[0, 0], [0.1, 0]])
    n = M.n_cells
    G = O.Geometry(m)
    f = O.feq(np.ones(n), np.zeros(n), np.zeros(n))
    wall_cell = int(G.cell[G.bidx[0]])
    f[3, wall_cell] = np.nan
    st = F.State(M, p, precision=prec, rho=np.ones(n), u=np.zeros((n, 2)))
    st.set_state(f)
    with pytest.raises(F.FvlbmError, match="EDIVERGED"):
        st.moments()                          # the totals reduce the NaN
    with pytest.raises(F.FvlbmError, match="EDIVERGED"):
        st.forces(0b11)                       # the wall cell's pressure is NaN
    with pytest.raises(F.FvlbmError, match="EDIVERGED"):
        st.step(1, residual=True)


@pytest.mark.parametrize("prec", ["fp64", "fp32dev"])
def test_time_step_beyond_the_courant_limit_diverges(F, prec):
    """dt = 10 times the advective Courant limit (dt / tau = 30): the oracle's run of the same case
    becomes non-finite after 127 steps; run_to_residual must stop with FVLBM_EDIVERGED."""
    say("dt = 10 x Courant limit", prec)
    m = _cavity()
    M = F.Mesh(m)
    dt = 10.0 * M.max_dt()
    p = O.default_params(nu=dt / 90, dt=dt, group_u=[[0, 0], [0.1, 0]])
    n = M.n_cells
    st = F.State(M, p, precision=prec, rho=np.ones(n), u=np.zeros((n, 2)))
    with pytest.raises(F.FvlbmError, match="EDIVERGED"):
        st.run_to_residual(0.0, 3000, check_every=50)


@pytest.mark.parametrize("prec", ["fp64", "fp32dev"])
def test_rest_state_residual_is_zero(F, prec):
    """A closed cavity with its lid at rest and the fluid at rest stays at rest: the residual is the
    absolute norm of the velocity change, exactly 0 (not 0 / 0)."""
    say("rest state residual", prec)
    m = _cavity()
    M = F.Mesh(m)
    dt = 0.5 * M.max_dt()
    p = O.default_params(nu=dt / 30, dt=dt, group_u=[[0, 0], [0, 0]])
    n = M.n_cells
    st = F.State(M, p, precision=prec, rho=np.ones(n), u=np.zeros((n, 2)))
    assert st.step(3, residual=True) == 0.0
    steps, r = st.run_to_residual(1e-12, 10, check_every=5)
    assert steps == 5 and r == 0.0


def test_state_change_after_record_drops_the_recording(F):
    """The adjoint reverses the recorded run from its final state; stepping or replacing the state
    after fvlbm_record makes that tape stale, so the adjoint must refuse (FVLBM_ESTATE) rather than
    seed the gradient at a state the tape does not end at."""
    say("step between record and adjoint")
    m = mg.backstep(core=0.35, dx_core=0.7, y1=1.5e-2, dx_corner=0.08, wall_layers=2)
    M = F.Mesh(m)
    dt = 0.5 * M.max_dt()
    p = O.default_params(nu=dt / 60, dt=dt, sst=True, group_u=[[0, 0], [0.05, 0.0], [0, 0]],
                         group_k=[0, 1e-4, 0], group_w=[0, 0.5, 0])
    n = M.n_cells
    st = F.State(M, p, precision="fp64", rho=np.ones(n), u=np.zeros((n, 2)), k=np.full(n, 1e-4),
                 omega=np.full(n, 0.5))
    st.record(4, ckpt_every=2)
    g1 = np.asarray(st.adjoint(1, [1.0, 0.0, 0.0]))
    g2 = np.asarray(st.adjoint(1, [1.0, 0.0, 0.0]))        # a second adjoint of the same tape
    np.testing.assert_array_equal(g1, g2)
    st.step(1)
    with pytest.raises(F.FvlbmError, match="ESTATE"):
        st.adjoint(1, [1.0, 0.0, 0.0])
    st.record(4, ckpt_every=2)
    st.set_state(st.get_f())
    with pytest.raises(F.FvlbmError, match="ESTATE"):
        st.adjoint(1, [1.0, 0.0, 0.0])
