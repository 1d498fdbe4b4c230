"""The allocation-free CG entry point (nfl_cg_solve_noalloc) against the
allocating one (nfl_cg_solve), through the C-ABI.

Both run the same kernels in the same order; only where the work space lives
differs (the library's static device array versus plan-owned buffers), and
how often the host looks at the status.  The spread adds into the grid with
float atomics, whose order varies from run to run, so two solves differ by
FP32 rounding noise only (about 1e-10 relative in u here, far below what the
1e-6 tolerance allows): the solutions must agree to 1e-7 relative, the
iteration counts to one, and both must converge.  Checked on two calls in a
row, the second with a smaller input, so that the static array's left-over
contents from the first call cannot leak into the second.
Also: the size limit and the refused warm-start mode return errors and
write nothing.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _plan(nfl, n, seed):
    import torch
    v, _ = synth.moons_and_roll(n, seed=seed)
    return nfl.plan(torch.as_tensor(v, device="cuda"), 0.04, N=64, m=6, eps_B=0.0), v


def _rhs(n, seed):
    rng = np.random.default_rng(seed)
    f = np.zeros(n)
    lab = rng.choice(n, size=max(2, n // 50), replace=False)
    f[lab] = rng.choice([-1.0, 1.0], size=lab.size)
    return f


@pytest.mark.parametrize("warm", ["zero", "user"])
def test_noalloc_matches_allocating_cg_on_two_calls(nfl, warm):
    import torch
    for n, seed in ((300_000, 3), (20_000, 4)):          # second call: smaller input
        P, _ = _plan(nfl, n, seed)
        f = torch.as_tensor(_rhs(n, seed + 10), device="cuda")
        u0 = None
        if warm == "user":
            u0 = torch.as_tensor(0.3 * _rhs(n, seed + 20), device="cuda")
        ref = P.cg_solve(f, tau=10.0, tol=1e-6, maxit=200, u0=u0)
        u = u0.clone() if u0 is not None else torch.full_like(f, np.nan)
        got = P.cg_solve_noalloc(f, u, tau=10.0, tol=1e-6, maxit=200,
                                 warm=nfl.WARM_USER if u0 is not None else nfl.WARM_ZERO)
        ur, ug = ref["u"].cpu().numpy(), got["u"].cpu().numpy()
        print("n=%d warm=%s: iters %d / %d, relres %.3e / %.3e, max |du| %.3e"
              % (n, warm, ref["iters"], got["iters"], ref["relres"], got["relres"],
                 np.abs(ur - ug).max()))
        assert got["converged"] and ref["converged"]
        assert abs(got["iters"] - ref["iters"]) <= 1
        assert np.all(np.isfinite(ug))
        assert np.abs(ur - ug).max() <= 1e-7 * np.abs(ur).max()
        assert got["relres"] <= 2e-6 and ref["relres"] <= 2e-6
        P.close()


def test_noalloc_limits(nfl):
    import torch
    P, _ = _plan(nfl, 5_000, 5)
    f = torch.as_tensor(_rhs(5_000, 6), device="cuda")
    u = torch.full_like(f, 7.0)
    with pytest.raises(nfl.NFLError) as e:
        P.cg_solve_noalloc(f, u, tau=10.0, warm=nfl.WARM_MLP)
    assert e.value.code == nfl.NFL_ERR_ARG
    assert torch.all(u == 7.0)
    P.close()
    n = nfl.CG_NOALLOC_MAX_N + 1
    P, _ = _plan(nfl, n, 7)
    f = torch.ones(n, dtype=torch.float64, device="cuda")
    u = torch.full_like(f, 7.0)
    with pytest.raises(nfl.NFLError) as e:
        P.cg_solve_noalloc(f, u, tau=10.0)
    assert e.value.code == nfl.NFL_ERR_ARG
    assert torch.all(u == 7.0)
    P.close()
