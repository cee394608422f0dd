"""Limit eps -> 0 on the batched solver (Section 3.2): members with the same grid, time step and
horizon and eps = 0.16, 0.08, 0.04, 0.02 are advanced in one batched context; the distances
||u_eps_k(T) - u_eps_{k+1}(T)|| computed on the GPU must match those of the FP64 oracle, and,
as the paper observes for the regularised families, they shrink as eps -> 0."""
import math

import numpy as np
import pytest

import oracle
from paper_2005_11931_amd import inputs as I

pytestmark = pytest.mark.gpu

EPS = (0.16, 0.08, 0.04, 0.02)


def _family(kind, n=513, T=0.6):
    x, y, X, Y = I.mesh(n, n)
    dx = 2.0 / (n - 1)
    hs = []
    for e in EPS:
        if kind == "jump":
            hs.append(1.0 + 3.0 * I.heaviside_gauss(X, e))
        else:
            hs.append(1.0 + 0.2 * I.gaussian_1d(X, e))
    hmax = max(float(h.max()) for h in hs)
    tau0 = 0.5 * dx / math.sqrt(hmax)
    N = int(math.ceil(T / tau0))
    tau = T / N
    u0 = I.zero_ring(np.exp(-((X - 0.4) ** 2 + Y ** 2) / 0.01))
    return [I.Case(f"{kind}{e}", n, n, -1, 1, -1, 1, tau, N, h, None, u0, np.zeros_like(u0)) for e, h in zip(EPS, hs)]


@pytest.mark.parametrize("kind", ["jump", "delta"])
def test_eps_limit_distances(kind):
    import torch

    from paper_2005_11931_amd import fdw

    fam = _family(kind)
    N = fam[0].nsteps
    print("limit", kind, "N", N, flush=True)
    s = fdw.family_solver(fam, dtype=fdw.FDW_F64)
    s.step(N)
    d_gpu = [s.distance(k, k + 1) for k in range(len(EPS) - 1)]
    s.close()
    ref = [oracle.forward_case(c)["u_cur"] for c in fam]
    dxdy = fam[0].dx * fam[0].dy
    d_ref = [math.sqrt(dxdy * float(np.sum((ref[k] - ref[k + 1]) ** 2))) for k in range(len(EPS) - 1)]
    print(kind, "gpu", d_gpu, "oracle", d_ref, flush=True)
    for a, b in zip(d_gpu, d_ref):
        assert abs(a - b) <= 1e-9 * max(b, 1e-30)
    # the regularised solutions form a Cauchy-like sequence as eps halves
    assert d_ref[0] > d_ref[1] > d_ref[2] > 0
