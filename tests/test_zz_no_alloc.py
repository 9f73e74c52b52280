"""The pressure solve that allocates nothing (pisoc_helm_solve_noalloc),
through the C ABI, against the workspace entry point it varies
(pisoc_helm_solve) and the FP64 oracle's PCG.

Both entry points run the same kernels with the same launch shapes, so the
solution, the iteration count and the residual must be bitwise identical;
against the oracle the bar of the pressure-solve parity tests holds (same
iteration count, solution within 1e-12 of its magnitude).  Two calls in a row,
the second on a smaller grid, check that the shared scratch keeps nothing
from one call to the next that the next would read.
"""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1404_0959_amd.pisoc as P
    P.lib()
    return P


def system(n, seed):
    rng = np.random.default_rng(seed)
    psidt = 50.0 * (1.0 + 0.2 * rng.random((n, n, n)))
    w = 0.01 * (1.0 + 0.2 * rng.random((n, n, n)))
    b = rng.standard_normal((n, n, n))
    return psidt, w, b


def test_noalloc_matches_workspace_solve(P, ora):
    import torch
    d = lambda a: torch.as_tensor(a, device="cuda")
    for n, seed in ((64, 1), (40, 2)):          # the maximum size, then a smaller ragged one
        print(f"noalloc solve n={n} seed={seed}", flush=True)
        psidt, w, b = system(n, seed)
        xa, ita, rela, sta = P.helm_solve_noalloc(d(psidt), d(w), d(b), tol=1e-10, maxit=500)
        xb, itb, relb, stb = P.helm_solve(d(psidt), d(w), d(b), tol=1e-10, maxit=500)
        assert sta == stb == P.OK
        assert ita == itb and rela == relb
        assert torch.equal(xa, xb)
        xo, ito, relo = ora.pcg(psidt, ora.kfaces(w), b, tol=1e-10, maxit=500)
        assert ita == ito, (ita, ito)
        assert np.max(np.abs(xa.cpu().numpy() - xo)) <= 1e-12 * np.max(np.abs(xo))


def test_noalloc_cap_and_start(P):
    """An iteration cap and a start at the solution behave as in the workspace solve."""
    import torch
    d = lambda a: torch.as_tensor(a, device="cuda")
    n = 16
    psidt, w, b = system(n, 3)
    xa, ita, rela, sta = P.helm_solve_noalloc(d(psidt), d(w), d(b), tol=1e-14, maxit=3)
    xb, itb, relb, stb = P.helm_solve(d(psidt), d(w), d(b), tol=1e-14, maxit=3)
    assert sta == stb == P.WARN_NOT_CONVERGED and ita == itb == 3 and torch.equal(xa, xb)
    xs, _, _, _ = P.helm_solve(d(psidt), d(w), d(b), tol=1e-13, maxit=500)
    xa, ita, rela, sta = P.helm_solve_noalloc(d(psidt), d(w), d(b), x0=xs, tol=1e-8)
    assert sta == P.OK and ita == 0


def test_noalloc_rejects_large_grid(P):
    import torch
    n = P.HELM_NOALLOC_MAX_N + 16
    z = torch.zeros((n, n, n), dtype=torch.float64, device="cuda")
    with pytest.raises(P.PisocError) as e:
        P.helm_solve_noalloc(z + 1.0, z + 0.01, z, tol=1e-8)
    assert e.value.status == P.ERR_WORKSPACE
