"""The paper's own experiments at their own resolution, run through the GPU library (FP64) and
compared with the FP64 oracle over the whole horizon, plus the findings the paper states.

  Section 3.1: depth 100 | 10 with a jump at x = 75 (Case 1), + delta(x-70) (Case 2),
     + delta^2(x-70) (Case 3), Friedrichs eps = 0.2, u0 = 40 exp(-(x-40)^2/8), dx = 0.005, T = 5
     (row mode: a 3-row grid with h2 = 0 is the 1D scheme);
  Section 3.2.3: amplitude-100 delta / delta^2, u0 = e/((x-60)^2+e^2), e = 0.5; the second
     wave is one-signed for the jump, two-signed for delta / delta^2, smaller than the main one;
  Section 3.3: the 2D problem on [0,100]^2 with H_eps = h_{0,eps}(x), eps = 0.8, dx = 0.05,
     u0 = 50 exp(-((x-40)^2+(y-50)^2)/8), T = 5.
The time integrator is explicit leapfrog at CFL 0.5, not the paper's implicit schemes.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2005_11931_amd import inputs as I

pytestmark = pytest.mark.gpu


def _gpu(case, flags=0):
    from paper_2005_11931_amd import fdw

    s = fdw.solver_for_case(case, dtype=fdw.FDW_F64, flags=flags, separate_h2=case.h2 is not None)
    e = s.step(case.nsteps, energy=True)[0].cpu().numpy()
    u = s.get_state()[0].cpu().numpy()
    s.close()
    return u, e


@pytest.mark.parametrize("kind", ["jump", "delta", "delta2"])
def test_section_3_1_cases(kind):
    from paper_2005_11931_amd import fdw

    case = I.paper_1d_case(kind)
    print("section 3.1", kind, "steps", case.nsteps, flush=True)
    u, e = _gpu(case, flags=fdw.FDW_ALLOW_ZERO_H)
    ref = oracle.forward_case(case)["u_cur"]
    amp = np.abs(case.u0).max()
    assert np.abs(u - ref).max() <= 1e-12 * amp
    assert np.abs(e - e[0]).max() <= 1e-11 * e[0]
    x = I.node_coords(case.nx, 0.0, 100.0)
    row = u[1]
    # Case 1 (Section 3.1): the wave grows in height reaching the shallow side; at t = 5 the
    # transmitted pulse (amplitude 20 in deep water) is near 75 + 1.5 sqrt(10)
    if kind == "jump":
        trans = row[(x > 76) & (x < 84)].max()
        assert trans > 20.0 * 1.4


@pytest.mark.parametrize("kind", ["jump", "delta", "delta2"])
def test_section_3_2_3_second_wave(kind):
    from paper_2005_11931_amd import fdw

    case = I.paper_1d_case(kind, amp=100.0, u0_kind="lorentz", e=0.5, T=3.0)
    print("section 3.2.3", kind, "steps", case.nsteps, flush=True)
    u, _ = _gpu(case, flags=fdw.FDW_ALLOW_ZERO_H)
    ref = oracle.forward_case(case)["u_cur"]
    # 12k-51k steps: the two sides round in a different order every step, and leapfrog neither
    # damps nor amplifies those differences, so they add up at most linearly in N: a few
    # roundings of the largest value per update and step
    tol = 4.0 * case.nsteps * np.finfo(np.float64).eps * np.abs(case.u0).max()
    err = np.abs(u - ref).max()
    print("max abs", err, "bound", tol, flush=True)
    assert err <= tol
    x = I.node_coords(case.nx, 0.0, 100.0)
    row = u[1]
    incident = np.abs(case.u0).max() / 2.0
    from_line = row[(x > 40) & (x < 57)]
    from_jump = row[(x > 57) & (x < 66)]
    assert 0.2 * incident < from_jump.max() < incident
    if kind == "jump":
        # one-signed: no negative lobe, only the tails of the two pulses
        assert from_line.min() > -1e-6 and from_line.max() < 0.02 * incident
    else:
        assert from_line.max() > 0.05 * incident and from_line.min() < -0.05 * incident
        assert np.abs(from_line).max() < incident


def test_section_3_3_two_dimensional():
    case = I.paper_2d_case()
    print("section 3.3: grid", case.nx, "steps", case.nsteps, flush=True)
    u, e = _gpu(case)
    ref = oracle.forward_case(case)["u_cur"]
    assert np.abs(u - ref).max() <= 1e-12 * 50.0
    assert np.abs(e - e[0]).max() <= 1e-11 * e[0]
