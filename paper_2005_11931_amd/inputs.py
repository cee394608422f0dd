"""Seeded synthetic inputs for the leapfrog wave solver and for its CPU oracle.

This module builds the Cauchy data (grid, coefficient h_eps, u0, u1, tau, number of
steps) and the receiver sets of every workload, in FP64 on the host.  It holds none
of the solver's arithmetic (no difference operator, no time stepping, no energy, no
adjoint); it is the one module that both the GPU path and the oracle are fed from.

Sources in the paper (arXiv 2005.11931):
  * the PDE and the vector-valued coefficient h = (h_1, ..., h_d) with h_j >= c0 > 0:
    Section 2, equation (2.1);
  * regularisation by convolution with psi_eps(x) = eps^{-1} psi(x/eps): Section 2.1
    (very weak solutions) and Section 3.1 (the 1D experiments);
  * the Friedrichs mollifier c*exp(1/(x^2-1)) with c approximately 2.2523:
    Section 3.1;
  * the 1D cases (h0 = 100 | 10 with a jump at x = 75, h0 + delta(x-70),
    h0 + delta^2(x-70)) and u0 = 40 exp(-(x-40)^2/8): Section 3.1;
  * the singularity tests (amplitude 100 delta / delta^2, u0 = e/((x-60)^2+e^2)):
    Section 3.2.3;
  * the 2D problem on [0,100]^2 with zero Dirichlet data, H_eps(x, y) = h_{0,eps}(x),
    u0 = 50 exp(-((x-40)^2+(y-50)^2)/8): Section 3.3.

Readings taken where the paper is silent (each is listed in the design notes):
  * nodes include both boundary nodes, spacing L/(n-1) (Section 3.3 grid);
  * the "Gaussian mollifier of width eps" is exp(-s^2/(2 eps^2)) / (eps sqrt(2 pi));
    its 2D point form divides by 2 pi eps^2 (unit mass in 2D);
  * the mollified Heaviside is 1/2 (1 + erf(x / (eps sqrt 2)));
  * delta^2 is the pointwise square phi_eps^2 (Section 3.1 states this);
  * tau = cfl * dx / sqrt(max over nodes of h), fixed before any perturbation of h.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence, Tuple

import numpy as np

# --------------------------------------------------------------------------------------
# Grids and elementary profiles
# --------------------------------------------------------------------------------------


def node_coords(n: int, lo: float, hi: float) -> np.ndarray:
    """Node coordinates of a uniform grid with n nodes including both ends.

    For a domain symmetric about 0 (lo == -hi) the coordinates are formed as
    ((2i - (n-1)) / (n-1)) * hi so that x[n-1-i] == -x[i] holds bitwise; this is what
    makes mirror-symmetry checks exact.
    """
    if n < 2:
        raise ValueError("need at least two nodes")
    i = np.arange(n, dtype=np.float64)
    if lo == -hi:
        return ((2.0 * i - (n - 1)) / (n - 1)) * hi
    return lo + i * ((hi - lo) / (n - 1))


def gaussian_1d(s: np.ndarray, eps: float) -> np.ndarray:
    """Unit-mass Gaussian mollifier of width eps in one variable."""
    return np.exp(-(s * s) / (2.0 * eps * eps)) / (eps * math.sqrt(2.0 * math.pi))


def gaussian_2d(r2: np.ndarray, eps: float) -> np.ndarray:
    """Unit-mass (in 2D) Gaussian mollifier of width eps, as a function of r^2."""
    return np.exp(-r2 / (2.0 * eps * eps)) / (2.0 * math.pi * eps * eps)


def heaviside_gauss(s: np.ndarray, eps: float) -> np.ndarray:
    """Heaviside step mollified by the unit-mass Gaussian of width eps."""
    from scipy.special import erf

    return 0.5 * (1.0 + erf(s / (eps * math.sqrt(2.0))))


def _friedrichs_unnormalised(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    m = np.abs(x) < 1.0
    out[m] = np.exp(1.0 / (x[m] * x[m] - 1.0))
    return out


def friedrichs_constant() -> float:
    """c such that c * exp(1/(x^2-1)) on |x| < 1 has unit integral (Section 3.1 prints 2.2523)."""
    from scipy.integrate import quad

    mass, _ = quad(lambda t: math.exp(1.0 / (t * t - 1.0)), -1.0, 1.0, epsabs=1e-14, epsrel=1e-14, limit=200)
    return 1.0 / mass


def friedrichs(x: np.ndarray, eps: float = 1.0) -> np.ndarray:
    """Friedrichs mollifier phi_eps(x) = eps^-1 phi(x/eps) of Section 3.1."""
    return friedrichs_constant() * _friedrichs_unnormalised(np.asarray(x) / eps) / eps


def _bump_kernel(s: float) -> float:
    """exp(1/(s^2-1)) on (-1, 1), 0 where s^2 rounds to 1 or beyond."""
    q = s * s - 1.0
    return math.exp(1.0 / q) if q < 0.0 else 0.0


def heaviside_friedrichs(x: np.ndarray, eps: float) -> np.ndarray:
    """Heaviside step convolved with the Friedrichs phi_eps, i.e. the integral of phi_eps up to x."""
    from scipy.integrate import quad

    c = friedrichs_constant()
    x = np.asarray(x, dtype=np.float64)
    out = np.empty_like(x)
    flat_in, flat_out = x.ravel(), out.ravel()
    for k, xv in enumerate(flat_in):
        t = xv / eps
        if t <= -1.0:
            flat_out[k] = 0.0
        elif t >= 1.0:
            flat_out[k] = 1.0
        else:
            v, _ = quad(_bump_kernel, -1.0, t, epsabs=1e-15, epsrel=1e-13, limit=200)
            flat_out[k] = c * v
    return out


def humps(X: np.ndarray, Y: np.ndarray, centres: Sequence[Tuple[float, float]], width: float,
          amp: float = 1.0) -> np.ndarray:
    """Sum of Gaussian humps amp * exp(-|x - c|^2 / width^2)."""
    u = np.zeros(np.broadcast(X, Y).shape, dtype=np.float64)
    for cx, cy in centres:
        u += amp * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (width * width))
    return u


def gaussian_random_field(n: int, ell: float, rng: np.random.Generator, lo: float = -1.0,
                          hi: float = 1.0) -> np.ndarray:
    """Smooth Gaussian random field on an n x n node grid of [lo, hi]^2.

    White N(0,1) noise is convolved (FFT, periodic) with exp(-r^2 / (2 ell^2)) and the
    result is normalised to zero sample mean and unit sample standard deviation.
    """
    noise = rng.standard_normal((n, n))
    d = (hi - lo) / (n - 1)
    k = np.fft.fftfreq(n, d=d) * 2.0 * math.pi
    kx, ky = np.meshgrid(k, k, indexing="xy")
    # Fourier transform of the Gaussian kernel (up to a constant that the normalisation removes)
    kern = np.exp(-0.5 * ell * ell * (kx * kx + ky * ky))
    g = np.real(np.fft.ifft2(np.fft.fft2(noise) * kern))
    g -= g.mean()
    g /= g.std()
    return g


def gaussian_random_field_upsampled(n: int, ell: float, rng: np.random.Generator, coarse: int = 1024) -> np.ndarray:
    """Gaussian random field for very large grids: drawn at coarse^2, cubic-spline zoomed to n^2."""
    from scipy.ndimage import zoom

    g = gaussian_random_field(coarse, ell, rng)
    z = zoom(g, n / coarse, order=3)
    assert z.shape == (n, n)
    z -= z.mean()
    z /= z.std()
    return z


# --------------------------------------------------------------------------------------
# Cauchy data containers
# --------------------------------------------------------------------------------------


@dataclasses.dataclass
class Case:
    """Cauchy data of one regularised problem (Section 2, equation (2.1); Section 3.3 grid).

    Arrays are FP64, row-major [ny][nx] with x varying fastest.  h2 is None when
    h_1 = h_2 = h (the physical tsunami model); the boundary ring of u0 and u1 is
    zero (Dirichlet data of Section 3.3).
    """

    name: str
    nx: int
    ny: int
    x0: float
    x1: float
    y0: float
    y1: float
    tau: float
    nsteps: int
    h1: np.ndarray
    h2: Optional[np.ndarray]
    u0: np.ndarray
    u1: np.ndarray
    receivers: Optional[np.ndarray] = None  # int32 [R][2] = (i, j)
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def dx(self) -> float:
        return (self.x1 - self.x0) / (self.nx - 1)

    @property
    def dy(self) -> float:
        return (self.y1 - self.y0) / (self.ny - 1)

    @property
    def T(self) -> float:
        return self.nsteps * self.tau

    @property
    def interior_updates(self) -> int:
        return (self.nx - 2) * (self.ny - 2) * self.nsteps


def zero_ring(a: np.ndarray) -> np.ndarray:
    a = np.array(a, dtype=np.float64, copy=True)
    a[0, :] = 0.0
    a[-1, :] = 0.0
    a[:, 0] = 0.0
    a[:, -1] = 0.0
    return a


def cfl_tau(dx: float, hmax: float, cfl: float = 0.5) -> float:
    """tau = cfl * dx / sqrt(max h): the "CFL 0.5" step of the workloads."""
    return cfl * dx / math.sqrt(hmax)


def mesh(nx: int, ny: int, lo: float = -1.0, hi: float = 1.0):
    x = node_coords(nx, lo, hi)
    y = node_coords(ny, lo, hi)
    X, Y = np.meshgrid(x, y, indexing="xy")
    return x, y, X, Y


# --------------------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------------------


def line_case(n: int = 256, nsteps: int = 1000, eps: float = 0.05, amp: float = 2.0, cfl: float = 0.5,
              centre=(0.5, 0.0), width2: float = 0.01, name: str = "line") -> Case:
    """2D plain forward solve with a mollified delta line on x = 0.

    h = 1 + amp * phi_eps(x), h_1 = h_2 = h; u0 = exp(-((x-xc)^2 + (y-yc)^2)/width2), u1 = 0;
    domain [-1, 1]^2; tau = cfl dx / sqrt(max h).  The defaults are the 256^2, 1000-step
    FP64 workload with eps = 0.05.
    """
    x, y, X, Y = mesh(n, n)
    h = 1.0 + amp * gaussian_1d(X, eps)
    u0 = zero_ring(np.exp(-((X - centre[0]) ** 2 + (Y - centre[1]) ** 2) / width2))
    dx = 2.0 / (n - 1)
    tau = cfl_tau(dx, float(h.max()), cfl)
    return Case(name, n, n, -1.0, 1.0, -1.0, 1.0, tau, nsteps, h, None, u0, np.zeros_like(u0),
                meta=dict(eps=eps, amp=amp, cfl=cfl, hmax=float(h.max())))


def point_case(n: int = 8192, nsteps: int = 5000, eps_cells: float = 4.0, amp: float = 5.0, cfl: float = 0.5,
               seed: int = 2002, nhumps: int = 4, width: float = 0.02, name: str = "point") -> Case:
    """Single large forward solve with a mollified point singularity at the origin.

    h = 1 + amp * phi^(2)_eps(r) with eps = eps_cells * dx (2D unit-mass Gaussian);
    u0 = sum of nhumps humps exp(-|x - c_k|^2 / width^2), c_k ~ U([-0.8, 0.8]^2) drawn
    with numpy's PCG64 seeded by `seed`; u1 = 0.  Defaults: 8192^2, 5000 steps.
    """
    x, y, X, Y = mesh(n, n)
    dx = 2.0 / (n - 1)
    eps = eps_cells * dx
    h = 1.0 + amp * gaussian_2d(X * X + Y * Y, eps)
    rng = np.random.default_rng(seed)
    centres = rng.uniform(-0.8, 0.8, size=(nhumps, 2))
    u0 = zero_ring(humps(X, Y, centres, width))
    tau = cfl_tau(dx, float(h.max()), cfl)
    return Case(name, n, n, -1.0, 1.0, -1.0, 1.0, tau, nsteps, h, None, u0, np.zeros_like(u0),
                meta=dict(eps=eps, amp=amp, cfl=cfl, seed=seed, centres=centres.tolist(), hmax=float(h.max())))


FAMILY_SIZES = (512, 1024, 2048, 4096)


def family_member(m: int, count: int = 32, nsteps: int = 2000, sizes: Sequence[int] = FAMILY_SIZES,
                  eps_max: float = 0.1, cfl: float = 0.5, base_seed: int = 3000) -> Case:
    """Member m of the batched family of regularisations.

    Size sizes[m % 4]; a mollified delta line h = 1 + 2 phi_eps(x) when floor(m/4) is
    odd, else a mollified jump h = 1 + 3 H_eps(x); eps_m = eps_max^(1 - m/(count-1)) *
    (2 dx_m)^(m/(count-1)), log-spaced from eps_max down to two cells; u0 = 4 humps of
    width 0.05 seeded with base_seed + m; u1 = 0; tau_m = cfl dx_m / sqrt(max h_m).
    """
    n = sizes[m % len(sizes)]
    x, y, X, Y = mesh(n, n)
    dx = 2.0 / (n - 1)
    s = m / (count - 1)
    eps = eps_max ** (1.0 - s) * (2.0 * dx) ** s
    kind = "delta" if (m // 4) % 2 == 1 else "jump"
    if kind == "delta":
        h = 1.0 + 2.0 * gaussian_1d(X, eps)
    else:
        h = 1.0 + 3.0 * heaviside_gauss(X, eps)
    rng = np.random.default_rng(base_seed + m)
    centres = rng.uniform(-0.8, 0.8, size=(4, 2))
    u0 = zero_ring(humps(X, Y, centres, 0.05))
    tau = cfl_tau(dx, float(h.max()), cfl)
    return Case(f"family{m}", n, n, -1.0, 1.0, -1.0, 1.0, tau, nsteps, h, None, u0, np.zeros_like(u0),
                meta=dict(eps=eps, kind=kind, m=m, seed=base_seed + m, hmax=float(h.max())))


def family(count: int = 32, nsteps: int = 2000, sizes: Sequence[int] = FAMILY_SIZES, **kw) -> List[Case]:
    return [family_member(m, count=count, nsteps=nsteps, sizes=sizes, **kw) for m in range(count)]


def receivers_on_row(nx: int, ny: int, y_line: float, count: int, rng: np.random.Generator,
                     xlo: float = -0.9, xhi: float = 0.9, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """count distinct receivers on the node row nearest y = y_line, x ~ U(xlo, xhi) snapped to nodes.

    Returns int32 [count][2] pairs (i, j) (column, row).
    """
    dy = (hi - lo) / (ny - 1)
    dx = (hi - lo) / (nx - 1)
    j = int(round((y_line - lo) / dy))
    cols: List[int] = []
    seen = set()
    while len(cols) < count:
        xv = rng.uniform(xlo, xhi)
        i = int(round((xv - lo) / dx))
        i = min(max(i, 1), nx - 2)
        if i not in seen:
            seen.add(i)
            cols.append(i)
    return np.array([[i, j] for i in cols], dtype=np.int32)


def adjoint_case(n: int = 2048, nsteps: int = 4000, nrecv: int = 64, eps: float = 0.05, cfl: float = 0.5,
                 field_amp: float = 0.1, ell: float = 0.1, y_line: float = 0.3,
                 seeds=(4001, 4002), name: str = "adjoint") -> Tuple[Case, np.ndarray]:
    """Adjoint-gradient workload: a mollified line, a seeded perturbed h_true and receivers.

    h_eps = 1 + 2 phi_eps(x); h_true = h_eps + field_amp * G(ell) (G seeded with seeds[0]);
    tau = cfl dx / sqrt(max(max h_eps, max h_true)) kept fixed; u0 = exp(-((x-0.25)^2 +
    y^2)/0.01); receivers on the row nearest y = y_line (columns seeded with seeds[1]).
    Returns (case at h = h_eps, h_true).
    """
    x, y, X, Y = mesh(n, n)
    dx = 2.0 / (n - 1)
    h_eps = 1.0 + 2.0 * gaussian_1d(X, eps)
    G = gaussian_random_field(n, ell, np.random.default_rng(seeds[0]))
    h_true = h_eps + field_amp * G
    tau = cfl_tau(dx, max(float(h_eps.max()), float(h_true.max())), cfl)
    u0 = zero_ring(np.exp(-((X - 0.25) ** 2 + Y ** 2) / 0.01))
    rec = receivers_on_row(n, n, y_line, nrecv, np.random.default_rng(seeds[1]))
    case = Case(name, n, n, -1.0, 1.0, -1.0, 1.0, tau, nsteps, h_eps, None, u0, np.zeros_like(u0),
                receivers=rec, meta=dict(eps=eps, seeds=list(seeds)))
    return case, h_true


def fd_direction(n: int, k: int, ell: float = 0.1, base_seed: int = 4100) -> np.ndarray:
    """Seeded finite-difference direction v_k = G(ell) / max|G| (seed base_seed + k)."""
    G = gaussian_random_field(n, ell, np.random.default_rng(base_seed + k))
    return G / np.abs(G).max()


def bathymetry_case(n: int = 16384, nsteps: int = 10000, cfl: float = 0.5, seeds=(5001, 5002),
                    ridge_amp: float = 2.0, ridge_cells: float = 2.0, name: str = "bathymetry") -> Case:
    """Largest forward solve: smooth random depth in [0.2, 1] plus a mollified delta ridge on x = 0.

    b = 0.2 + 0.8 (G - min G)/(max G - min G) with G a correlation-length-0.1 field;
    h = b + ridge_amp * phi_eps(x), eps = ridge_cells * dx; u0 = 4 humps of width 0.02.
    """
    x, y, X, Y = mesh(n, n)
    dx = 2.0 / (n - 1)
    rng = np.random.default_rng(seeds[0])
    G = gaussian_random_field_upsampled(n, 0.1, rng) if n > 2048 else gaussian_random_field(n, 0.1, rng)
    b = 0.2 + 0.8 * (G - G.min()) / (G.max() - G.min())
    eps = ridge_cells * dx
    h = b + ridge_amp * gaussian_1d(X, eps)
    centres = np.random.default_rng(seeds[1]).uniform(-0.8, 0.8, size=(4, 2))
    u0 = zero_ring(humps(X, Y, centres, 0.02))
    tau = cfl_tau(dx, float(h.max()), cfl)
    return Case(name, n, n, -1.0, 1.0, -1.0, 1.0, tau, nsteps, h, None, u0, np.zeros_like(u0),
                meta=dict(eps=eps, seeds=list(seeds), hmax=float(h.max()), centres=centres.tolist()))


def bathymetry_crop_case(full: Case, first: int = 6144, n: int = 4096, nsteps: int = 4000, nrecv: int = 64,
                         y_line: float = 0.075, seed: int = 5003, hump_x: float = -0.05,
                         name: str = "bathymetry_crop") -> Case:
    """Adjoint workload cut from the largest one: nodes first .. first+n-1 on both axes of the
    16384^2 bathymetry case (same spacing, same tau), zero Dirichlet data on the crop's edge,
    nsteps steps, nrecv distinct receivers on the crop row nearest y = y_line (columns seeded).
    The ridge sets tau (about 1e-6), so in 4000 steps the waves of the parent case's humps
    travel a few hundredths at most; a hump of width 0.02 at (hump_x, y_line) is added so that
    the receivers record a signal.
    """
    sl = slice(first, first + n)
    x0 = full.x0 + first * full.dx
    x1 = full.x0 + (first + n - 1) * full.dx
    y0 = full.y0 + first * full.dy
    y1 = full.y0 + (first + n - 1) * full.dy
    h = np.ascontiguousarray(full.h1[sl, sl])
    dy = full.dy
    X, Y = np.meshgrid(x0 + full.dx * np.arange(n), y0 + dy * np.arange(n), indexing="xy")
    j = int(round((y_line - y0) / dy))
    u0 = zero_ring(np.ascontiguousarray(full.u0[sl, sl]) + humps(X, Y, [(hump_x, y0 + j * dy)], 0.02))
    del X, Y
    rng = np.random.default_rng(seed)
    cols: List[int] = []
    seen = set()
    while len(cols) < nrecv:
        i = int(rng.integers(1, n - 1))
        if i not in seen:
            seen.add(i)
            cols.append(i)
    rec = np.array([[i, j] for i in cols], dtype=np.int32)
    return Case(name, n, n, x0, x1, y0, y1, full.tau, nsteps, h, None, u0, np.zeros_like(u0), receivers=rec,
                meta=dict(first=first, seed=seed, parent=full.name))


# --------------------------------------------------------------------------------------
# The paper's own experiments (Sections 3.1 - 3.3), on the leapfrog grid
# --------------------------------------------------------------------------------------


def paper_depth_1d(x: np.ndarray, eps: float, kind: str = "jump", amp: float = 1.0) -> np.ndarray:
    """Regularised 1D depth of Section 3.1: h0 = 100 on [0, 75), 10 on [75, 100], convolved with
    the Friedrichs phi_eps, plus amp*phi_eps(x-70) (kind 'delta') or amp*phi_eps(x-70)^2
    (kind 'delta2')."""
    # h0 * phi_eps = 10 + 90 * (1 - H_eps(x - 75))
    h = 10.0 + 90.0 * (1.0 - heaviside_friedrichs(x - 75.0, eps))
    if kind == "delta":
        h = h + amp * friedrichs(x - 70.0, eps)
    elif kind == "delta2":
        h = h + amp * friedrichs(x - 70.0, eps) ** 2
    elif kind != "jump":
        raise ValueError(kind)
    return h


def row_mode_case(x: np.ndarray, h: np.ndarray, u0: np.ndarray, tau: float, nsteps: int, name: str = "row") -> Case:
    """Embed a 1D problem on nodes x (both ends included, zero Dirichlet) as the single
    interior row of a 3-row grid with h_2 = 0, so that rows decouple into the 1D scheme."""
    n = x.size
    H1 = np.zeros((3, n))
    H1[:, :] = h[None, :]
    H2 = np.zeros((3, n))
    U0 = np.zeros((3, n))
    U0[1, :] = u0
    U0 = zero_ring(U0)
    dy = 1.0
    return Case(name, n, 3, float(x[0]), float(x[-1]), 0.0, 2.0 * dy, tau, nsteps, H1, H2, U0, np.zeros_like(U0))


def paper_1d_case(kind: str = "jump", eps: float = 0.2, dx: float = 0.005, T: float = 5.0, amp: float = 1.0,
                  u0_kind: str = "gauss", e: float = 0.5, cfl: float = 0.5) -> Case:
    """Section 3.1 / 3.2.3 in row mode: (0, 100) with spacing dx, the regularised depth of
    paper_depth_1d, u0 = 40 exp(-(x-40)^2/8) ("gauss", Section 3.1) or e/((x-60)^2+e^2)
    ("lorentz", Section 3.2.3), u1 = 0, tau = cfl dx / sqrt(max h), horizon T."""
    n = int(round(100.0 / dx)) + 1
    x = node_coords(n, 0.0, 100.0)
    h = paper_depth_1d(x, eps, kind, amp=amp)
    if u0_kind == "gauss":
        g = 40.0 * np.exp(-((x - 40.0) ** 2) / 8.0)
    else:
        g = e / ((x - 60.0) ** 2 + e * e)
    g[0] = g[-1] = 0.0
    tau0 = cfl * (x[1] - x[0]) / math.sqrt(float(h.max()))
    N = int(math.ceil(T / tau0))
    c = row_mode_case(x, h, g, T / N, N, name=f"paper1d-{kind}")
    c.meta.update(kind=kind, eps=eps, amp=amp, u0=u0_kind, e=e)
    return c


def paper_2d_case(eps: float = 0.8, dx: float = 0.05, T: float = 5.0, cfl: float = 0.5) -> Case:
    """Section 3.3: [0, 100]^2, H_eps(x, y) = h_{0,eps}(x) (100 | 10 at x = 75, Friedrichs
    mollified), u0 = 50 exp(-((x-40)^2 + (y-50)^2)/8), u1 = 0, zero Dirichlet data,
    tau = cfl dx / sqrt(max h) (the paper's own implicit run uses dt = 0.5)."""
    n = int(round(100.0 / dx)) + 1
    x = node_coords(n, 0.0, 100.0)
    hx = paper_depth_1d(x, eps, "jump")
    H = np.broadcast_to(hx[None, :], (n, n)).copy()
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = zero_ring(50.0 * np.exp(-((X - 40.0) ** 2 + (Y - 50.0) ** 2) / 8.0))
    tau0 = cfl * dx / math.sqrt(float(hx.max()))
    N = int(math.ceil(T / tau0))
    return Case("paper2d", n, n, 0.0, 100.0, 0.0, 100.0, T / N, N, H, None, u0, np.zeros_like(u0),
                meta=dict(eps=eps))



def consistency_family(n: int = 513, eps_list: Sequence[float] = (0.08, 0.04, 0.02, 0.01, 0.005),
                       sigma: float = 0.1, amp: float = 1.0, centre=(0.3, 0.0), s0: float = 0.05,
                       T: float = 0.5, cfl: float = 0.5) -> List[Case]:
    """Consistency with the classical solution (Section 2.3, Theorem 2.6): a smooth positive
    depth h = 1 + amp exp(-|x|^2 / (2 sigma^2)) (in W^{1,inf}) and a smooth u0 = exp(-|x - c|^2 /
    (2 s0^2)), each convolved with the 2D unit-mass Gaussian mollifier of width eps.  Both
    convolutions have closed forms (Gaussian widths add in quadrature):
        h_eps  = 1 + amp sigma^2 / (sigma^2 + eps^2) exp(-|x|^2 / (2 (sigma^2 + eps^2))),
        u0_eps = s0^2 / (s0^2 + eps^2) exp(-|x - c|^2 / (2 (s0^2 + eps^2))).
    Returns the classical problem (eps = 0, first) followed by one member per eps, all on the
    same n x n grid of [-1, 1]^2 with one common tau (CFL 0.5 for the largest depth) and
    horizon T; u1 = 0.
    """
    x, y, X, Y = mesh(n, n)
    dx = 2.0 / (n - 1)
    r2 = X * X + Y * Y
    c2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2
    out = []
    for eps in (0.0,) + tuple(eps_list):
        sh = sigma * sigma + eps * eps
        su = s0 * s0 + eps * eps
        h = 1.0 + amp * (sigma * sigma / sh) * np.exp(-r2 / (2.0 * sh))
        u0 = zero_ring((s0 * s0 / su) * np.exp(-c2 / (2.0 * su)))
        out.append((eps, h, u0))
    hmax = max(float(h.max()) for _, h, _ in out)
    tau0 = cfl_tau(dx, hmax, cfl)
    N = int(math.ceil(T / tau0))
    tau = T / N
    return [Case(f"consistency{eps}", n, n, -1.0, 1.0, -1.0, 1.0, tau, N, h, None, u0, np.zeros_like(u0),
                 meta=dict(eps=eps, sigma=sigma, amp=amp, s0=s0)) for eps, h, u0 in out]


def paper_case1_eps_sweep(eps_list: Sequence[float] = (0.8, 0.5, 0.2, 0.1, 0.05, 0.02), dx: float = 0.005,
                          T: float = 5.0) -> List[Case]:
    """Section 3.1, Case 1 (depth 100 | 10 with a jump at x = 75, Friedrichs-mollified) at the
    regularisation widths the paper compares at t = 5, in row mode; all members share dx and
    tau (the depth lies in [10, 100] for every eps)."""
    return [paper_1d_case("jump", eps=e, dx=dx, T=T) for e in eps_list]


def paper_table1_case(n: int, dt: float = 0.05, T: float = 5.0, eps: float = 0.8) -> Case:
    """The workload of the paper's GPU timings (Section 4, Table 1): the Section 3.3 problem on an
    n x n node grid of [0, 100]^2 (dx = dy = 100/(n-1)), H_eps = h_{0,eps}(x), u0 = 50 exp(-((x-40)^2
    + (y-50)^2)/8), u1 = 0, time step dt = 0.05 and T = 5 (100 steps), as the table states."""
    x = node_coords(n, 0.0, 100.0)
    hx = paper_depth_1d(x, eps, "jump")
    H = np.broadcast_to(hx[None, :], (n, n)).copy()
    X, Y = np.meshgrid(x, x, indexing="xy")
    u0 = zero_ring(50.0 * np.exp(-((X - 40.0) ** 2 + (Y - 50.0) ** 2) / 8.0))
    N = int(round(T / dt))
    return Case(f"table1-{n}", n, n, 0.0, 100.0, 0.0, 100.0, T / N, N, H, None, u0, np.zeros_like(u0),
                meta=dict(eps=eps, dt=dt))
