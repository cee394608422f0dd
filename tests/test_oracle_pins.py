"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these tests re-types the oracle's formulas: each compares it with a closed form,
an invariant, a brute-force derivative or a value the paper prints.

  P1 row-mode d'Alembert: with h2 = 0 rows decouple into the 1D scheme; at Courant number 1
     the leapfrog recurrence with the Taylor start is the discrete d'Alembert formula, so the
     solution equals the odd-periodic sampled d'Alembert solution exactly.
  P2 discrete eigenmode: for constant h1 != h2 and dx != dy the separable sine modes are
     eigenvectors of the operator with a known eigenvalue, so u^n = (cos n theta + B sin n theta) mode.
  P3 manufactured solution: observed second-order convergence.
  P4 energy: the discrete analogue of the conservation law of Section 2 (CL-01) is constant
     to roundoff, and E^{1/2} approximates the continuous |u_t|^2 + |h^{1/2} grad u|^2.
  P5 mirror symmetry (bitwise), the reflected second wave of Sections 3.1/3.2.3 (sign
     structure: one-signed for a jump, two-signed for a delta line), and the 1D jump
     reflection / transmission coefficients.
  P6 adjoint gradient against central finite differences, the Taylor remainder, and the
     store-all vs checkpointed modes (bitwise).
  P8 the forward definition evaluated in extended precision (the reference at very small
     time steps): the exact discrete eigenmode at tau = 2e-4 of the stability limit, the
     FP64 oracle where that one is accurate, and row-mode d'Alembert.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2005_11931_amd import inputs as I


# ----------------------------------------------------------------------------- P1


def _dalembert_row(g: np.ndarray, nsteps: int) -> np.ndarray:
    """Sampled d'Alembert solution 1/2 (G(x - n dx) + G(x + n dx)) with G the odd 2(n-1)-periodic
    extension of the node samples g (g[0] = g[-1] = 0), i.e. the zero-Dirichlet wave at Courant 1."""
    n = g.size
    P = 2 * (n - 1)
    ext = np.empty(P)
    ext[:n] = g
    ext[n:] = -g[-2:0:-1]
    k = np.arange(n)
    return 0.5 * (ext[(k - nsteps) % P] + ext[(k + nsteps) % P])


@pytest.mark.parametrize("nsteps", [1, 2, 37, 150, 400])
def test_p1_row_mode_dalembert_exact(nsteps):
    n = 101
    x = I.node_coords(n, 0.0, 1.0)
    c = 1.7
    g = np.exp(-((x - 0.37) / 0.05) ** 2) - 0.5 * np.exp(-((x - 0.71) / 0.03) ** 2)
    g[0] = g[-1] = 0.0
    dx = x[1] - x[0]
    case = I.row_mode_case(x, np.full(n, c * c), g, dx / c, nsteps)
    r = oracle.forward_case(case)
    expect = _dalembert_row(g, nsteps)
    assert np.abs(r["u_cur"][1] - expect).max() < 1e-13
    # rows 0 and 2 are boundary rows
    assert np.all(r["u_cur"][0] == 0) and np.all(r["u_cur"][2] == 0)


def test_p1_row_mode_previous_level():
    n = 64
    x = I.node_coords(n, -1.0, 1.0)
    g = np.exp(-(x / 0.1) ** 2)
    g[0] = g[-1] = 0.0
    dx = x[1] - x[0]
    case = I.row_mode_case(x, np.full(n, 4.0), g, dx / 2.0, 90)
    r = oracle.forward_case(case)
    assert np.abs(r["u_prev"][1] - _dalembert_row(g, 89)).max() < 1e-13


# ----------------------------------------------------------------------------- P2


def _eigen_case(nx, ny, h1c, h2c, k, l, v, cfl=0.9):
    x0, x1, y0, y1 = 0.0, 1.3, -0.5, 0.5
    dx, dy = (x1 - x0) / (nx - 1), (y1 - y0) / (ny - 1)
    i = np.arange(nx)
    j = np.arange(ny)
    mode = np.outer(np.sin(l * math.pi * j / (ny - 1)), np.sin(k * math.pi * i / (nx - 1)))
    mu = -(h1c * 4.0 / dx**2 * math.sin(k * math.pi / (2 * (nx - 1))) ** 2
           + h2c * 4.0 / dy**2 * math.sin(l * math.pi / (2 * (ny - 1))) ** 2)
    lam_max = 4.0 * h1c / dx**2 + 4.0 * h2c / dy**2
    tau = cfl * 2.0 / math.sqrt(lam_max)
    theta = math.acos(1.0 + tau * tau * mu / 2.0)
    return x0, x1, y0, y1, dx, dy, mode, tau, theta


@pytest.mark.parametrize("k,l,v", [(1, 1, 0.0), (3, 2, 0.0), (7, 5, 0.3), (20, 11, -1.1)])
def test_p2_discrete_eigenmode_exact(k, l, v):
    nx, ny = 41, 29
    h1c, h2c = 2.0, 0.7
    x0, x1, y0, y1, dx, dy, mode, tau, theta = _eigen_case(nx, ny, h1c, h2c, k, l, v)
    nsteps = 400
    h1 = np.full((ny, nx), h1c)
    h2 = np.full((ny, nx), h2c)
    u1 = v * mode
    r = oracle.forward(nx, ny, dx, dy, tau, h1, h2, mode, u1, nsteps)
    B = tau * v / math.sin(theta)
    expect = (math.cos(nsteps * theta) + B * math.sin(nsteps * theta)) * mode
    expect_prev = (math.cos((nsteps - 1) * theta) + B * math.sin((nsteps - 1) * theta)) * mode
    scale = max(1.0, abs(B))
    assert np.abs(r["u_cur"] - expect).max() < 1e-11 * scale
    assert np.abs(r["u_prev"] - expect_prev).max() < 1e-11 * scale


def test_p2_apply_is_eigen():
    nx, ny = 17, 23
    x0, x1, y0, y1, dx, dy, mode, tau, theta = _eigen_case(nx, ny, 1.5, 0.25, 2, 3, 0.0)
    hx, hy = oracle.faces(np.full((ny, nx), 1.5), np.full((ny, nx), 0.25))
    Av = oracle.apply(hx, hy, mode, dx, dy)
    mu = -(1.5 * 4 / dx**2 * math.sin(2 * math.pi / (2 * (nx - 1))) ** 2
           + 0.25 * 4 / dy**2 * math.sin(3 * math.pi / (2 * (ny - 1))) ** 2)
    assert np.abs(Av - mu * mode).max() < 1e-10 * abs(mu)


# ----------------------------------------------------------------------------- P8


@pytest.mark.parametrize("k,l,v", [(1, 1, 0.0), (2, 3, 1.3)])
def test_p8_extended_precision_eigenmode_at_tiny_tau(k, l, v):
    """The forward definition evaluated in extended precision, at a time step 2e-4 of the
    stability limit (the regime of the point-singularity workload, tau ~ 1e-7): after 4000
    steps it equals the exact discrete eigenmode (cos n theta + B sin n theta) mode, with
    sin(theta/2) = tau sqrt(-mu)/2 and B = tau v / sin theta, to FP64 rounding of the output,
    while the FP64 three-level recurrence is a thousand times further off (its roundings act
    as velocity kicks and accumulate faster than linearly at such steps)."""
    nx, ny = 41, 29
    h1c, h2c = 2.0, 0.7
    x0, x1, y0, y1, dx, dy, mode, tau, _ = _eigen_case(nx, ny, h1c, h2c, k, l, v, cfl=2e-4)
    mu = -(h1c * 4.0 / dx**2 * math.sin(k * math.pi / (2 * (nx - 1))) ** 2
           + h2c * 4.0 / dy**2 * math.sin(l * math.pi / (2 * (ny - 1))) ** 2)
    theta = 2.0 * math.asin(tau * math.sqrt(-mu) / 2.0)
    N = 4000
    h1 = np.full((ny, nx), h1c)
    h2 = np.full((ny, nx), h2c)
    B = tau * v / math.sin(theta)
    expect = (math.cos(N * theta) + B * math.sin(N * theta)) * mode
    expect_prev = (math.cos((N - 1) * theta) + B * math.sin((N - 1) * theta)) * mode
    r = oracle.forward_ld(nx, ny, dx, dy, tau, h1, h2, mode, v * mode, N)
    err_ld = np.abs(r["u_cur"] - expect).max()
    assert err_ld < 2e-14
    assert np.abs(r["u_prev"] - expect_prev).max() < 2e-14
    r64 = oracle.forward(nx, ny, dx, dy, tau, h1, h2, mode, v * mode, N)
    assert np.abs(r64["u_cur"] - expect).max() > 100 * err_ld


def test_p8_extended_precision_matches_fp64_where_fp64_is_accurate():
    """At an ordinary time step (CFL 0.5) over a few hundred steps the FP64 oracle is accurate;
    the extended-precision evaluation must agree with it to FP64 rounding, traces included."""
    case = I.line_case(n=96, nsteps=300)
    rec = np.array([[10, 48], [70, 20], [48, 48]], dtype=np.int32)
    a = oracle.forward_case(case, receivers=rec)
    b = oracle.forward_case_ld(case, receivers=rec)
    assert np.abs(a["u_cur"] - b["u_cur"]).max() < 1e-14
    assert np.abs(a["u_prev"] - b["u_prev"]).max() < 1e-14
    assert np.abs(a["traces"] - b["traces"]).max() < 1e-14


def test_p8_extended_precision_row_mode_dalembert():
    """Row-mode d'Alembert (h2 = 0, Courant number 1) is exact for the extended evaluation too."""
    n = 101
    x = I.node_coords(n, 0.0, 1.0)
    g = np.exp(-((x - 0.37) / 0.05) ** 2) - 0.5 * np.exp(-((x - 0.71) / 0.03) ** 2)
    g[0] = g[-1] = 0.0
    dx = x[1] - x[0]
    case = I.row_mode_case(x, np.full(n, 1.7 * 1.7), g, dx / 1.7, 137)
    r = oracle.forward_case_ld(case)
    assert np.abs(r["u_cur"][1] - _dalembert_row(g, 137)).max() < 1e-14


# ----------------------------------------------------------------------------- P3


def _mms_error(n, T=0.5):
    """Manufactured u = cos(2t) sin(pi(x+1)/2) sin(pi(y+1)/2), h = 1 + 0.5 exp(-x^2/0.1) on
    [-1,1]^2; forcing f = u_tt - div(h grad u) worked out by hand."""
    x, y, X, Y = I.mesh(n, n)
    dx = 2.0 / (n - 1)
    h = 1.0 + 0.5 * np.exp(-X * X / 0.1)
    hp = 0.5 * np.exp(-X * X / 0.1) * (-2.0 * X / 0.1)
    k = math.pi / 2
    Sx, Sy = np.sin(k * (X + 1)), np.sin(k * (Y + 1))
    Cx = np.cos(k * (X + 1))

    def u(t):
        return math.cos(2 * t) * Sx * Sy

    def f(t):
        ux = math.cos(2 * t) * k * Cx * Sy
        uu = u(t)
        div = hp * ux + h * (-k * k * uu) + h * (-k * k * uu)
        return -4.0 * uu - div

    tau = 0.4 * dx / math.sqrt(1.5)
    N = int(round(T / tau))
    tau = T / N
    hx, hy = oracle.faces(h, h)
    up = I.zero_ring(u(0.0))
    uc = oracle.start(hx, hy, up, np.zeros_like(up), dx, dx, tau, f0=f(0.0))
    for s in range(1, N):
        un = oracle.step(hx, hy, up, uc, dx, dx, tau, f=f(s * tau))
        up, uc = uc, un
    return np.abs(uc - u(N * tau)).max()


@pytest.mark.slow
def test_p3_manufactured_second_order():
    e = [_mms_error(n) for n in (33, 65, 129)]
    orders = [math.log2(e[0] / e[1]), math.log2(e[1] / e[2])]
    for p in orders:
        assert 1.9 < p < 2.1, (e, orders)


# ----------------------------------------------------------------------------- P4


def test_p4_energy_conserved():
    c = I.line_case(n=64, nsteps=1000)
    r = oracle.forward_case(c, want_energy=True)
    E = r["energy"]
    assert E.shape == (1000,)
    assert np.all(E > 0)
    assert np.abs(E - E[0]).max() / E[0] < 1e-12


def test_p4_energy_conserved_anisotropic_with_velocity():
    rng = np.random.default_rng(7)
    nx, ny = 37, 53
    x, y, X, Y = I.mesh(nx, ny)
    h1 = 0.5 + rng.uniform(0, 1, (ny, nx))
    h2 = 0.3 + rng.uniform(0, 2, (ny, nx))
    u0 = I.zero_ring(np.exp(-((X - 0.2) ** 2 + (Y + 0.1) ** 2) / 0.05))
    u1 = I.zero_ring(np.sin(3 * X) * np.cos(2 * Y))
    dx, dy = 2.0 / (nx - 1), 2.0 / (ny - 1)
    tau = 0.45 * min(dx, dy) / math.sqrt(max(h1.max(), h2.max()))
    r = oracle.forward(nx, ny, dx, dy, tau, h1, h2, u0, u1, 700, want_energy=True)
    E = r["energy"]
    assert np.abs(E - E[0]).max() / E[0] < 1e-12


def test_p4_energy_matches_continuous_quantity():
    """E^{1/2} ~ integral of |u_t|^2 + h |grad u|^2 at t = 0 (no factor 1/2, as in CL-01)."""
    errs = []
    for n in (65, 129, 257):
        x, y, X, Y = I.mesh(n, n)
        h = 1.0 + 0.5 * np.exp(-X * X / 0.1)
        a = 0.15
        g = np.exp(-((X - 0.1) ** 2 + Y * Y) / a**2)
        u0 = I.zero_ring(g)
        dx = 2.0 / (n - 1)
        tau = 0.1 * dx
        r = oracle.forward(n, n, dx, dx, tau, h, h, u0, np.zeros_like(u0), 1, want_energy=True)
        # continuous: |grad g|^2 = (4/a^4) g^2 ((x-0.1)^2 + y^2), integrated on a fine quadrature
        m = 2001
        xs = np.linspace(-1, 1, m)
        XX, YY = np.meshgrid(xs, xs)
        gg = np.exp(-((XX - 0.1) ** 2 + YY**2) / a**2)
        hh = 1.0 + 0.5 * np.exp(-XX * XX / 0.1)
        integrand = hh * (4.0 / a**4) * gg * gg * ((XX - 0.1) ** 2 + YY**2)
        exact = np.trapezoid(np.trapezoid(integrand, xs, axis=1), xs)
        errs.append(abs(r["energy"][0] - exact) / exact)
    assert errs[-1] < 2e-3
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


# ----------------------------------------------------------------------------- P5


def test_p5_mirror_symmetry_bitwise_y():
    c = I.line_case(n=96, nsteps=200)  # h depends on x only, u0 even in y
    r = oracle.forward_case(c)
    u = r["u_cur"]
    assert np.array_equal(u, u[::-1, :])
    assert np.abs(u).max() > 1e-3


def test_p5_mirror_symmetry_bitwise_x():
    c = I.line_case(n=96, nsteps=200, centre=(0.0, 0.3))  # h even in x, u0 even in x
    r = oracle.forward_case(c)
    u = r["u_cur"]
    assert np.array_equal(u, u[:, ::-1])


def _reflected_profile(kind, n=257, T=0.95):
    """Difference on y = 0 between the solution with a mollified line singularity on x = 0 and
    the one with h = 1, from a hump at x = 0.5."""
    x, y, X, Y = I.mesh(n, n)
    dx = 2.0 / (n - 1)
    eps = 4 * dx
    if kind == "delta":
        h = 1.0 + 0.2 * I.gaussian_1d(X, eps)
    else:
        h = 1.0 + 3.0 * I.heaviside_gauss(-X, eps)  # deeper (faster) water on the side of the hump
    u0 = I.zero_ring(np.exp(-((X - 0.5) ** 2 + Y**2) / 0.005))
    hmax = float(h.max())
    tau = 0.5 * dx / math.sqrt(hmax)
    N = int(round(T / tau))
    ref = oracle.forward(n, n, dx, dx, tau, np.ones_like(h), np.ones_like(h), u0, np.zeros_like(u0), N)
    sing = oracle.forward(n, n, dx, dx, tau, h, h, u0, np.zeros_like(u0), N)
    j0 = n // 2
    return x, sing["u_cur"][j0] - ref["u_cur"][j0], ref["u_cur"][j0], N * tau


def test_p5_reflected_wave_delta_line_two_signed():
    x, d, ref, t = _reflected_profile("delta")
    right = x > 0.05
    seg = d[right]
    # the reflected wave travels back to x > 0; it is smaller than the incident wave and has
    # both a positive and a negative part (Section 3.2.3)
    assert seg.max() > 1e-3 and seg.min() < -1e-3
    assert np.abs(seg).max() < np.abs(ref).max()
    # it sits near the image-source circle |x - (-0.5)| = t (unit speed in h = 1)
    xpk = x[right][np.argmax(np.abs(seg))]
    assert abs(xpk - (t - 0.5)) < 0.15


@pytest.mark.slow
@pytest.mark.parametrize("kind", ["jump", "delta", "delta2"])
def test_p5_paper_singularity_tests_sign_structure(kind):
    """Section 3.2.3: depth h0 (100 | 10 at x = 75) plus 100 delta(x-70) or 100 delta^2(x-70),
    Friedrichs-mollified with eps = 0.2, u0 = e/((x-60)^2 + e^2) with e = 0.5, u1 = 0.  The
    second (reflected) wave is smaller than the main one; it is one-signed (positive) for the
    discontinuous case and has positive and negative parts for the delta and delta^2 cases.
    At t = 3 the reflection from x = 70 is near x = 50 and the one from x = 75 near x = 60."""
    n = 10001
    x = I.node_coords(n, 0.0, 100.0)
    dx = x[1] - x[0]
    e = 0.5
    g = e / ((x - 60.0) ** 2 + e * e)
    g[0] = g[-1] = 0.0
    h = I.paper_depth_1d(x, 0.2, kind, amp=100.0)
    tau = 0.5 * dx / math.sqrt(h.max())
    N = int(round(3.0 / tau))
    u = oracle.forward_case(I.row_mode_case(x, h, g, tau, N))["u_cur"][1]
    incident = g.max() / 2.0
    from_line = u[(x > 40) & (x < 57)]
    from_jump = u[(x > 57) & (x < 66)]
    # the jump at x = 75 reflects a positive wave in every case (R > 0 from deep to shallow)
    assert 0.2 * incident < from_jump.max() < incident
    assert from_jump.min() > -0.01 * incident
    if kind == "jump":
        assert np.abs(from_line).max() < 0.02 * incident
    else:
        assert from_line.max() > 0.05 * incident and from_line.min() < -0.05 * incident
        assert np.abs(from_line).max() < incident


def test_p5_jump_reflection_transmission_1d():
    """1D plane-pulse through a mollified jump h_in = 4 -> h_out = 1 (row mode):
    R = (sqrt(h_in) - sqrt(h_out))/(sqrt(h_in) + sqrt(h_out)) = 1/3, T = 1 + R = 4/3."""
    n = 4001
    x = I.node_coords(n, -2.0, 2.0)
    dx = x[1] - x[0]
    h = 1.0 + 3.0 * (1.0 - I.heaviside_gauss(x, 2 * dx))
    g = np.exp(-((x + 1.0) ** 2) / 0.01)
    g[0] = g[-1] = 0.0
    tau = 0.5 * dx / 2.0
    N = int(round(0.9 / tau))
    r = oracle.forward_case(I.row_mode_case(x, h, g, tau, N))
    u = r["u_cur"][1]
    refl = u[(x > -1.0) & (x < -0.6)]
    trans = u[(x > 0.2) & (x < 0.6)]
    R = refl.max() / 0.5
    T = trans.max() / 0.5
    assert abs(R - 1 / 3) < 0.01, R
    assert abs(T - 4 / 3) < 0.01, T


def test_p5_paper_case1_height_increases():
    """Section 3.1, Case 1 (h0 = 100 | 10 at x = 75): the wave grows passing into shallow water,
    T = 2 sqrt(100)/(sqrt(100) + sqrt(10)) = 1.52, and a positive reflected wave appears."""
    n = 4001
    x = I.node_coords(n, 0.0, 100.0)
    dx = x[1] - x[0]
    eps = 0.2
    h = I.paper_depth_1d(x, eps, "jump")
    g = 40.0 * np.exp(-((x - 40.0) ** 2) / 8.0)
    g[0] = g[-1] = 0.0
    tau = 0.5 * dx / 10.0
    T_end = 5.0
    N = int(round(T_end / tau))
    r = oracle.forward_case(I.row_mode_case(x, h, g, tau, N))
    u = r["u_cur"][1]
    # right-moving half (amplitude 20) reaches 75 at t = 3.5; at t = 5 the transmitted pulse is
    # near 75 + 1.5 sqrt(10) = 79.7, the reflected one near 75 - 15 = 60
    trans = u[(x > 76) & (x < 84)].max()
    refl = u[(x > 55) & (x < 65)]
    assert abs(trans / 20.0 - 2 * 10 / (10 + math.sqrt(10))) < 0.03
    Rexp = (10 - math.sqrt(10)) / (10 + math.sqrt(10))
    assert abs(refl.max() / 20.0 - Rexp) < 0.03
    assert refl.min() > -0.02 * 20.0


# ----------------------------------------------------------------------------- P6


def _adj_problem(nx=24, ny=20, N=60, seed=11, R=5):
    rng = np.random.default_rng(seed)
    x, y, X, Y = I.mesh(nx, ny)
    dx, dy = 2.0 / (nx - 1), 2.0 / (ny - 1)
    h = 1.0 + 0.5 * np.exp(-X * X / 0.2) + 0.1 * rng.uniform(size=(ny, nx))
    u0 = I.zero_ring(np.exp(-((X - 0.3) ** 2 + Y**2) / 0.08))
    u1 = I.zero_ring(0.3 * np.exp(-((X + 0.2) ** 2 + (Y - 0.1) ** 2) / 0.1))
    tau = 0.5 * min(dx, dy) / math.sqrt(h.max() * 1.3)
    cols = rng.choice(np.arange(1, nx - 1), size=R, replace=False)
    rows = rng.integers(1, ny - 1, size=R)
    rec = np.stack([cols, rows], axis=1).astype(np.int32)
    d = rng.normal(size=(N + 1, R)) * 0.05
    return nx, ny, dx, dy, tau, h, u0, u1, N, rec, d


def _loss(nx, ny, dx, dy, tau, h1, h2, u0, u1, N, rec, d):
    r = oracle.forward(nx, ny, dx, dy, tau, h1, h2, u0, u1, N, receivers=rec)
    return oracle.misfit(r["traces"], d), r["traces"]


def test_p6_adjoint_vs_central_fd():
    nx, ny, dx, dy, tau, h, u0, u1, N, rec, d = _adj_problem()
    J, tr = _loss(nx, ny, dx, dy, tau, h, h, u0, u1, N, rec, d)
    g = oracle.adjoint(nx, ny, dx, dy, tau, h, None, u0, u1, N, rec, 2.0 * (tr - d))
    rng = np.random.default_rng(99)
    for k in range(6):
        v = rng.normal(size=h.shape)
        delta = 1e-5
        Jp, _ = _loss(nx, ny, dx, dy, tau, h + delta * v, h + delta * v, u0, u1, N, rec, d)
        Jm, _ = _loss(nx, ny, dx, dy, tau, h - delta * v, h - delta * v, u0, u1, N, rec, d)
        fd = (Jp - Jm) / (2 * delta)
        ad = float(np.sum(g * v))
        assert abs(fd - ad) <= 1e-6 * abs(fd), (k, fd, ad)


def test_p6_adjoint_separate_h1_h2_vs_fd():
    nx, ny, dx, dy, tau, h, u0, u1, N, rec, d = _adj_problem(seed=5, N=40)
    h2 = 0.8 * h[::-1, :].copy()
    tau = 0.9 * tau
    J, tr = _loss(nx, ny, dx, dy, tau, h, h2, u0, u1, N, rec, d)
    g1, g2 = oracle.adjoint(nx, ny, dx, dy, tau, h, h2, u0, u1, N, rec, 2.0 * (tr - d), separate=True)
    rng = np.random.default_rng(3)
    for which in (1, 2):
        v = rng.normal(size=h.shape)
        delta = 1e-5
        if which == 1:
            Jp, _ = _loss(nx, ny, dx, dy, tau, h + delta * v, h2, u0, u1, N, rec, d)
            Jm, _ = _loss(nx, ny, dx, dy, tau, h - delta * v, h2, u0, u1, N, rec, d)
            ad = float(np.sum(g1 * v))
        else:
            Jp, _ = _loss(nx, ny, dx, dy, tau, h, h2 + delta * v, u0, u1, N, rec, d)
            Jm, _ = _loss(nx, ny, dx, dy, tau, h, h2 - delta * v, u0, u1, N, rec, d)
            ad = float(np.sum(g2 * v))
        fd = (Jp - Jm) / (2 * delta)
        assert abs(fd - ad) <= 1e-6 * abs(fd), (which, fd, ad)


def test_p6_taylor_remainder_second_order():
    nx, ny, dx, dy, tau, h, u0, u1, N, rec, d = _adj_problem(seed=21, N=50)
    J0, tr = _loss(nx, ny, dx, dy, tau, h, h, u0, u1, N, rec, d)
    g = oracle.adjoint(nx, ny, dx, dy, tau, h, None, u0, u1, N, rec, 2.0 * (tr - d))
    v = np.random.default_rng(1).normal(size=h.shape)
    rem = []
    for delta in (1e-2, 5e-3, 2.5e-3):
        Jd, _ = _loss(nx, ny, dx, dy, tau, h + delta * v, h + delta * v, u0, u1, N, rec, d)
        rem.append(abs(Jd - J0 - delta * float(np.sum(g * v))))
    assert 3.5 < rem[0] / rem[1] < 4.5 and 3.5 < rem[1] / rem[2] < 4.5, rem


@pytest.mark.parametrize("N,c", [(60, 7), (60, 20), (61, 61), (64, 16), (1, 4), (2, 1)])
def test_p6_checkpointed_equals_store_all_bitwise(N, c):
    nx, ny, dx, dy, tau, h, u0, u1, _, rec, d = _adj_problem(N=N)
    d = d[: N + 1]
    _, tr = _loss(nx, ny, dx, dy, tau, h, h, u0, u1, N, rec, d)
    tg = 2.0 * (tr - d)
    ga = oracle.adjoint(nx, ny, dx, dy, tau, h, None, u0, u1, N, rec, tg, ckpt_every=0)
    gb = oracle.adjoint(nx, ny, dx, dy, tau, h, None, u0, u1, N, rec, tg, ckpt_every=c)
    assert np.array_equal(ga, gb)
    assert np.abs(ga).max() > 0


def test_p6_single_step_gradient_brute_force():
    """N = 1: J depends on h only through the start step; every nodal derivative by FD."""
    nx, ny, dx, dy, tau, h, u0, u1, _, rec, d = _adj_problem(nx=7, ny=6, N=1, R=3)
    d = d[:2]
    _, tr = _loss(nx, ny, dx, dy, tau, h, h, u0, u1, 1, rec, d)
    g = oracle.adjoint(nx, ny, dx, dy, tau, h, None, u0, u1, 1, rec, 2.0 * (tr - d))
    fd = np.zeros_like(h)
    delta = 1e-6
    for j in range(ny):
        for i in range(nx):
            e = np.zeros_like(h)
            e[j, i] = delta
            Jp, _ = _loss(nx, ny, dx, dy, tau, h + e, h + e, u0, u1, 1, rec, d)
            Jm, _ = _loss(nx, ny, dx, dy, tau, h - e, h - e, u0, u1, 1, rec, d)
            fd[j, i] = (Jp - Jm) / (2 * delta)
    assert np.abs(g - fd).max() <= 1e-7 * np.abs(fd).max()


# ----------------------------------------------------------------------------- P7 (fixtures)


def test_p7_friedrichs_constant_matches_paper():
    # Section 3.1 prints c ~ 2.2523 for c exp(1/(x^2-1)) to have unit integral
    import json
    import os

    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    printed = gold["friedrichs_constant"]["value"]
    c = I.friedrichs_constant()
    assert abs(c - printed) < 0.5 * 10 ** -gold["friedrichs_constant"]["printed_digits"]


def test_p7_mollifier_masses():
    for eps in (0.05, 0.2, 1.0):
        x = I.node_coords(20001, -10.0, 10.0)
        dx = x[1] - x[0]
        assert abs(np.sum(I.gaussian_1d(x, eps)) * dx - 1.0) < 1e-10
        assert abs(np.sum(I.friedrichs(x, eps)) * dx - 1.0) < 1e-6
    x = I.node_coords(801, -1.0, 1.0)
    X, Y = np.meshgrid(x, x)
    dx = x[1] - x[0]
    assert abs(np.sum(I.gaussian_2d(X * X + Y * Y, 0.05)) * dx * dx - 1.0) < 1e-9


def test_p7_symmetric_coordinates_bitwise():
    for n in (3, 4, 255, 256, 8192):
        x = I.node_coords(n, -1.0, 1.0)
        assert np.array_equal(x[::-1], -x)
        assert x[0] == -1.0 and x[-1] == 1.0


# ----------------------------------------------------------------------------- P9
# The implicit factorized scheme of the 2D experiment (Section 3.3; Section 4, Table 1).


@pytest.mark.parametrize("n", [1, 2, 7, 50, 257])
def test_p9_tridiagonal_solver_against_dense_solve(n):
    """The line solver against numpy's dense LU solve on random diagonally dominant systems."""
    rng = np.random.default_rng(n)
    lo, up = rng.normal(size=n), rng.normal(size=n)
    di = np.abs(lo) + np.abs(up) + 0.5 + rng.uniform(size=n)
    rhs = rng.normal(size=n)
    T = np.diag(di) + np.diag(lo[1:], -1) + np.diag(up[:-1], 1)
    x = oracle.tridiag(lo, di, up, rhs)
    assert np.abs(x - np.linalg.solve(T, rhs)).max() <= 1e-13 * max(1.0, np.abs(x).max())


@pytest.mark.parametrize("k,l,v,cfl", [(1, 1, 0.0, 5.0), (2, 3, 1.3, 5.0), (3, 2, 0.4, 0.7)])
def test_p9_adi_discrete_eigenmode(k, l, v, cfl):
    """Constant h1 != h2, dx != dy: the separable sine modes are eigenvectors of both line
    operators, so the implicit scheme acts on a mode's amplitude by the scalar recurrence
    P (a_{n+1} - 2 a_n + a_{n-1}) = -tau^2 (mu_x + mu_y) a_n, P = (1 + s tau^2 mu_x)(1 + s tau^2 mu_y),
    whose solution with the start a_1 = 1 + tau v - tau^2 (mu_x + mu_y)/(2P) is
    a_n = cos n theta + (tau v / sin theta) sin n theta, cos theta = 1 - tau^2 (mu_x + mu_y)/(2P) --
    also at a time step 5x the explicit stability limit (sigma = 1/4)."""
    nx, ny = 41, 29
    h1c, h2c = 2.0, 0.7
    x0, x1, y0, y1, dx, dy, mode, tau, _ = _eigen_case(nx, ny, h1c, h2c, k, l, v, cfl=min(cfl, 0.9))
    tau = tau * cfl / min(cfl, 0.9)
    s = 0.25
    mx = h1c * 4.0 / dx**2 * math.sin(k * math.pi / (2 * (nx - 1))) ** 2
    my = h2c * 4.0 / dy**2 * math.sin(l * math.pi / (2 * (ny - 1))) ** 2
    P = (1 + s * tau * tau * mx) * (1 + s * tau * tau * my)
    theta = math.acos(1.0 - tau * tau * (mx + my) / (2.0 * P))
    N = 300
    r = oracle.adi_forward(nx, ny, dx, dy, tau, s, np.full((ny, nx), h1c), np.full((ny, nx), h2c), mode, v * mode, N)
    B = tau * v / math.sin(theta)
    expect = (math.cos(N * theta) + B * math.sin(N * theta)) * mode
    assert np.abs(r["u_cur"] - expect).max() <= 1e-11 * max(1.0, abs(B))


def test_p9_adi_sigma_zero_is_leapfrog():
    """sigma = 0 turns every line system into the identity: the leapfrog scheme, bit for bit."""
    c = I.line_case(n=64, nsteps=80)
    a = oracle.forward_case(c)["u_cur"]
    b = oracle.adi_forward_case(c, sigma=0.0)["u_cur"]
    assert np.array_equal(a, b)


def _adi_variable_case(n=65, T=0.4):
    x, y, X, Y = I.mesh(n, n)
    h1 = 1.0 + 0.6 * np.exp(-((X - 0.1) ** 2) / 0.05) + 0.2 * Y
    h2 = 0.8 + 0.3 * np.sin(2 * X) * np.cos(Y)
    u0 = I.zero_ring(np.exp(-((X - 0.2) ** 2 + (Y + 0.1) ** 2) / 0.03))
    u1 = I.zero_ring(0.3 * np.exp(-((X + 0.3) ** 2 + Y**2) / 0.05))
    return n, 2.0 / (n - 1), h1, h2, u0, u1, T


def test_p9_adi_second_order_in_time_to_the_leapfrog_limit():
    """Variable h1 != h2: as tau -> 0 at a fixed grid the implicit and the leapfrog schemes
    converge to the same semi-discrete solution, each at second order in tau; their difference
    at tau, tau/2, tau/4 (tau at CFL 0.4) falls by about 4 per halving."""
    n, d, h1, h2, u0, u1, T = _adi_variable_case()
    tau0 = 0.4 * d / math.sqrt(2 * max(h1.max(), h2.max()))
    diffs = []
    for q in (1, 2, 4):
        N = int(round(T / tau0)) * q
        tau = T / N
        a = oracle.adi_forward(n, n, d, d, tau, 0.25, h1, h2, u0, u1, N)["u_cur"]
        b = oracle.forward(n, n, d, d, tau, h1, h2, u0, u1, N)["u_cur"]
        diffs.append(np.abs(a - b).max())
    r1, r2 = diffs[0] / diffs[1], diffs[1] / diffs[2]
    assert 3.5 < r1 < 4.5 and 3.5 < r2 < 4.5, (diffs, r1, r2)


def test_p9_adi_stable_far_beyond_the_explicit_limit():
    """Variable h1 != h2 at 20x the explicit stability limit: the implicit solution stays bounded
    over 400 steps while the leapfrog scheme at the same step blows up."""
    n, d, h1, h2, u0, u1, _ = _adi_variable_case(n=49)
    tau = 20.0 * d / math.sqrt(2 * max(h1.max(), h2.max()))
    a = oracle.adi_forward(n, n, d, d, tau, 0.25, h1, h2, u0, u1, 400)["u_cur"]
    assert np.isfinite(a).all() and np.abs(a).max() < 3.0 * np.abs(u0).max()
    b = oracle.forward(n, n, d, d, tau, h1, h2, u0, u1, 60)["u_cur"]
    assert not np.isfinite(b).all() or np.abs(b).max() > 1e6


def test_p9_adi_line_factors_against_the_operator():
    """The line systems are the factors of the operator: with variable h1 != h2 and a step far
    beyond the explicit limit, w0 = 2 (u^1 - u^0) (u1 = 0) satisfies
    (I - sigma tau^2 L1)(I - sigma tau^2 L2) w0 = tau^2 (L1 + L2) u^0, the factors applied with the
    leapfrog oracle's operator (pinned by P1-P3): L1 with (h1, 0), L2 with (0, h2)."""
    n, d, h1, h2, u0, _, _ = _adi_variable_case(n=41)
    tau = 4.0 * d
    s = 0.25
    w = 2.0 * (oracle.adi_forward(n, n, d, d, tau, s, h1, h2, u0, np.zeros_like(u0), 1)["u_cur"] - u0)
    z = np.zeros_like(h1)
    L1 = lambda f: oracle.apply(*oracle.faces(h1, z), f, d, d)
    L2 = lambda f: oracle.apply(*oracle.faces(z, h2), f, d, d)
    v = w - s * tau * tau * L2(w)
    res = v - s * tau * tau * L1(v) - tau * tau * (L1(u0) + L2(u0))
    assert np.abs(res).max() <= 1e-12 * np.abs(w).max()
