"""The largest single-GPU workload: 16384^2 FP32 (smooth random bathymetry, depth 0.2-1, plus a
mollified delta ridge with eps = 2 dx), in the launch configuration the library picks by
default.  After a few steps the state is compared with the FP64 oracle on windows around
sampled nodes; over a longer run the discrete energy must stay constant to FP32 accuracy."""
import sys

import numpy as np
import pytest

import oracle
from paper_2005_11931_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bathymetry():
    case = I.bathymetry_case(n=16384, nsteps=10000)
    print("largest: inputs ready", flush=True)
    return case


@pytest.mark.timeout(600)
def test_bathymetry_16384_windows_and_energy(bathymetry):
    import torch

    from paper_2005_11931_amd import fdw

    n = 16384
    case = bathymetry
    s = fdw.solver_for_case(case, dtype=fdw.FDW_F32)
    n0 = 10
    s.step(n0)
    u = s.get_state()[0].cpu().numpy().astype(np.float64)
    rng = np.random.default_rng(7)
    centres = [(n // 2, n // 2), (n // 2, 1), (n - 2, n - 2)] + [tuple(rng.integers(1, n - 1, 2)) for _ in range(4)]
    for cx, cy in case.meta.get("centres", [])[:2]:
        centres.append((int(round((cy + 1) / case.dy)), int(round((cx + 1) / case.dx))))
    W = n0 + 6
    scale = np.abs(case.u0).max()
    for (j, i) in centres:
        j0, j1 = max(0, j - W), min(n, j + W + 1)
        i0, i1 = max(0, i - W), min(n, i + W + 1)
        sub = I.Case("win", i1 - i0, j1 - j0, 0, (i1 - i0 - 1) * case.dx, 0, (j1 - j0 - 1) * case.dy, case.tau, n0,
                     case.h1[j0:j1, i0:i1], None, case.u0[j0:j1, i0:i1], case.u1[j0:j1, i0:i1])
        ref = oracle.forward_case(sub)["u_cur"]
        m = n0 + 1
        a0 = 0 if j0 == 0 else m
        a1 = (j1 - j0) if j1 == n else (j1 - j0 - m)
        b0 = 0 if i0 == 0 else m
        b1 = (i1 - i0) if i1 == n else (i1 - i0 - m)
        got = u[j0 + a0:j0 + a1, i0 + b0:i0 + b1]
        assert np.abs(got - ref[a0:a1, b0:b1]).max() <= 1e-5 * scale, (j, i)
    del u
    e = s.step(600, energy=True)[0].cpu().numpy()
    assert np.all(np.isfinite(e))
    drift = np.abs(e - e[0]).max() / e[0]
    print("largest: energy drift over 600 steps", drift, flush=True)
    assert drift < 1e-4
    s.close()


@pytest.mark.timeout(600)
def test_bathymetry_crop_gradient_vs_oracle(bathymetry):
    """The adjoint workload cut from the largest one (central 4096^2 crop, zero Dirichlet edge,
    64 receivers, seeded trace gradient, checkpoints every 64 steps) at a shortened horizon of
    300 steps: the FP64 GPU gradient against the oracle's FP64 adjoint (1e-9 relative), and the
    FP32 GPU gradient's error against the same oracle gradient, reported and bounded."""
    import torch

    from paper_2005_11931_amd import fdw

    crop = I.bathymetry_crop_case(bathymetry, nsteps=300)
    N = crop.nsteps
    rec = torch.as_tensor(crop.receivers)
    tg = np.random.default_rng(5004).normal(size=(N + 1, len(crop.receivers)))
    print("crop gradient: oracle", flush=True)
    gref = oracle.adjoint(crop.nx, crop.ny, crop.dx, crop.dy, crop.tau, crop.h1, None, crop.u0, crop.u1, N,
                          crop.receivers, tg, ckpt_every=64)
    scale = np.abs(gref).max()
    errs = {}
    for dt, name in ((fdw.FDW_F64, "f64"), (fdw.FDW_F32, "f32")):
        s = fdw.solver_for_case(crop, dtype=dt)
        g = s.adjoint(rec, torch.as_tensor(tg), ckpt_every=64).cpu().numpy()
        s.close()
        errs[name] = (float(np.abs(g - gref).max() / scale), float(np.linalg.norm(g - gref) / np.linalg.norm(gref)))
    print("crop gradient errors (max-abs rel, L2 rel):", errs, flush=True)
    assert errs["f64"][0] <= 1e-9
    assert errs["f32"][0] <= 1e-3
