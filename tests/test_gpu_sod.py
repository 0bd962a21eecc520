"""The HIP path on the Sod shock tube of the 1-D validation runs (Sec. 3.4) at the
paper's resolution (32 elements of 8 subcells, final time 0.2): the same step
sizes as the oracle, the final state against the oracle's and the density
against the exact Riemann solution."""
import numpy as np
import pytest
import torch

from paper_2011_03338_amd import sedg, workloads as W
from tests.parity import DEV, say
from tests.test_oracle_sod import exact_density_means, run_to

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mask,bound", [(0, 3e-3), (1 << 3, 4e-3)])
def test_sod_gpu_matches_oracle_and_exact(mask, bound):
    """mask 0: all levels O(8) -> O(4) -> O(2) -> FV; 1 << 3: single level O(8) -> FV."""
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mesh, u0, info = W.sod_tube(nelem=32, K=8)
    p = W.Params(level_mask=mask)
    dts = []
    u_o = run_to(mesh, p, u0, info["T"], dts)
    s = sedg.Solver(mesh, p)
    ug = torch.from_numpy(u0).to(DEV)
    for dt in dts:
        s.rk_step(ug, 1, dt)
    s.check()
    u_g = ug.cpu().numpy()
    s.close()
    # rounding can tip the indicator at the shock differently over ~200 steps, so the
    # two trajectories agree to a small absolute tolerance, not to the one-step bound
    diff = float(np.max(np.abs(u_g - u_o)))
    rho = u_g[0, 0].mean(axis=0)
    l1 = float(np.mean(np.abs(rho - exact_density_means(mesh.edges(0), info["T"]))))
    say("  sod mask %d %d steps max|gpu-oracle|=%.3e density L1 vs exact=%.3e" % (mask, len(dts), diff, l1))
    assert diff < 1e-3
    assert l1 < bound
