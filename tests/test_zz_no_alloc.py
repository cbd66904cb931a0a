"""fvlbm_totals_noalloc, the entry point for callers that cannot allocate, against the totals of
fvlbm_moments (the entry point it is a variant of): the same kernels and summation order, so the
same FP64 values to the last bit, on two calls in a row with the second on a smaller state, in both
precisions, through the C ABI."""
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


@pytest.mark.parametrize("precision", ["fp64", "fp32dev"])
def test_totals_noalloc_matches_moments(F, precision):
    import torch
    cases = [("cavity 48x48 (4,608 cells)", mg.cavity(n=48, jitter=0.15, seed=1), [[0, 0], [0.1, 0]]),
             ("duct 9x8 (144 cells)", mg.rectangle(9, 8, Lx=1.4, kind="duct", jitter=0.25, seed=33),
              [[0.05, 0.01], [0, 0], [0.05, 0.0]])]
    out = torch.full((3,), float("nan"), dtype=torch.float64, device="cuda")
    for name, m, gu in cases:
        say("totals_noalloc", precision, name)
        M = F.Mesh(m)
        n = M.n_cells
        dt = 0.5 * M.max_dt()
        p = O.default_params(nu=dt / 30, dt=dt, group_u=gu)
        rng = np.random.default_rng(7)
        st = F.State(M, p, precision=precision, rho=1 + 0.01 * rng.standard_normal(n),
                     u=0.03 * rng.standard_normal((n, 2)))
        st.step(3)
        st.totals_noalloc(out)
        torch.cuda.synchronize()
        got = out.cpu().numpy().copy()
        ref = st.moments()["totals"]
        print(name, precision, "noalloc", got, "moments", ref)
        np.testing.assert_array_equal(got, ref)
        del st
