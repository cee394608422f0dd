"""The pins must catch plausible mistakes in the oracle.

Each case below plants one mistake (a dropped term, a wrong sign or index, a transposed
operand) in a temporary copy of the oracle source, compiles it with gcc, and runs a fast
subset of the pins against it; at least one pin must fail.  The real oracle passes all of
them (last case).  CPU only: nothing here touches the GPU.
"""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
from paper_2005_11931_amd import inputs as I

SRC = os.path.join(os.path.dirname(oracle.__file__), "fdw_oracle.c")

MUTANTS = {
    "start_drops_half": ("0.5 * (tau * tau) * acc", "(tau * tau) * acc"),
    "start_drops_velocity": ("AT(u0, j, i) + tau * AT(u1, j, i)", "AT(u0, j, i)"),
    "step_sign_of_previous": ("2.0 * AT(u_cur, j, i) - AT(u_prev, j, i)", "2.0 * AT(u_cur, j, i) - AT(u_cur, j, i)"),
    "apply_east_face_from_hy": ("AT(hx, j, i) * (AT(v, j, i + 1) - c)", "AT(hy, j, i) * (AT(v, j, i + 1) - c)"),
    "apply_west_face_index": ("AT(hx, j, i - 1) * (AT(v, j, i - 1) - c)", "AT(hx, j, i) * (AT(v, j, i - 1) - c)"),
    "apply_dx_dy_swapped": ("(east + west) / (dx * dx) + (north + south) / (dy * dy)",
                            "(east + west) / (dy * dy) + (north + south) / (dx * dx)"),
    "faces_hy_from_h1": ("0.5 * (AT(h2, j, i) + AT(h2, j + 1, i))", "0.5 * (AT(h1, j, i) + AT(h1, j + 1, i))"),
    "energy_potential_wrong_scale": ("K + X / (dx * dx) + Y / (dy * dy)", "K + X / (dx * dy) + Y / (dy * dy)"),
    "energy_kinetic_unscaled": ("double v = (AT(u_np1, j, i) - AT(u_n, j, i)) / tau;",
                                "double v = (AT(u_np1, j, i) - AT(u_n, j, i));"),
    "adjoint_start_weight": ("(k == 0) ? 0.5 * tt : tt", "tt"),
    "adjoint_grad_sign": ("w * (AT(lam, j, i) - AT(lam, j, i + 1))", "w * (AT(lam, j, i + 1) - AT(lam, j, i))"),
    "adjoint_drops_second_level": ("2.0 * AT(lam_next, j, i) - AT(lam_next2, j, i)", "2.0 * AT(lam_next, j, i)"),
    "adjoint_nodal_half": ("double g1 = 0.5 * (", "double g1 = 1.0 * ("),
    "adjoint_y_grad_index": ("(AT(u, j + 1, i) - AT(u, j, i)) / (dy * dy)", "(AT(u, j + 1, i) - AT(u, j - 1 + (j == 0), i)) / (dy * dy)"),
    # the extended-precision evaluation of the forward definition
    "ld_start_drops_half": ("0.5L * tt * AT(scr, j, i)", "tt * AT(scr, j, i)"),
    "ld_start_drops_velocity": ("T * (ld_t)AT(u1, j, i)", "0.0L * (ld_t)AT(u1, j, i)"),
    "ld_step_previous_level": ("2.0L * AT(cur, j, i) - AT(prev, j, i)", "2.0L * AT(cur, j, i) - AT(cur, j, i)"),
    "ld_apply_dx_dy_swapped": ("(east + west) / dx2 + (north + south) / dy2", "(east + west) / dy2 + (north + south) / dx2"),
    "ld_faces_hy_from_h1": ("0.5L * ((ld_t)AT(h2, j, i) + (ld_t)AT(h2, j + 1, i))",
                            "0.5L * ((ld_t)AT(h1, j, i) + (ld_t)AT(h1, j + 1, i))"),
    # the implicit factorized scheme and its line solver
    "adi_start_drops_half": ("tau * AT(u1, j, i) + 0.5 * AT(w, j, i)", "tau * AT(u1, j, i) + AT(w, j, i)"),
    "adi_offdiag_sign": ("up[k] = -gx * AT(hx, j, i);", "up[k] = gx * AT(hx, j, i);"),
    "adi_y_face_index": ("lo[k] = -gy * AT(hy, jj - 1, i);", "lo[k] = -gy * AT(hy, jj, i);"),
    "adi_x_uses_gy": ("di[k] = 1.0 + gx * (AT(hx, j, i - 1) + AT(hx, j, i));",
                      "di[k] = 1.0 + gy * (AT(hx, j, i - 1) + AT(hx, j, i));"),
    "thomas_elimination": ("const double m = di[k] - lo[k] * cp[k - 1];", "const double m = di[k] - up[k] * cp[k - 1];"),
    "thomas_back_substitution": ("x[k] = dp[k] - cp[k] * x[k + 1];", "x[k] = dp[k] + cp[k] * x[k + 1];"),
}


def _build_variant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor not found: {name}"
    mutated = src.replace(old, new)
    d = tmp_path / name
    d.mkdir()
    (d / "fdw_oracle.c").write_text(mutated)
    (d / "fdw_oracle.h").write_text(open(SRC.replace(".c", ".h")).read())
    so = d / "libmut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    str(d / "fdw_oracle.c"), "-o", str(so), "-lm"], check=True)
    return str(so)


def _pins_pass() -> dict:
    """Fast pins (each a few ms); returns name -> passed."""
    out = {}
    # P1 d'Alembert in row mode
    n = 61
    x = I.node_coords(n, 0.0, 1.0)
    g = np.exp(-((x - 0.4) / 0.07) ** 2)
    g[0] = g[-1] = 0.0
    dx = x[1] - x[0]
    try:
        r = oracle.forward_case(I.row_mode_case(x, np.full(n, 2.25), g, dx / 1.5, 45))
        P = 2 * (n - 1)
        ext = np.concatenate([g, -g[-2:0:-1]])
        k = np.arange(n)
        expect = 0.5 * (ext[(k - 45) % P] + ext[(k + 45) % P])
        out["p1"] = bool(np.abs(r["u_cur"][1] - expect).max() < 1e-12)
    except Exception:
        out["p1"] = False
    # P2 anisotropic eigenmode with initial velocity
    nx, ny = 21, 15
    X0, X1, Y0, Y1 = 0.0, 1.3, -0.5, 0.5
    ddx, ddy = (X1 - X0) / (nx - 1), (Y1 - Y0) / (ny - 1)
    kk, ll, v = 3, 2, 0.4
    mode = np.outer(np.sin(ll * math.pi * np.arange(ny) / (ny - 1)), np.sin(kk * math.pi * np.arange(nx) / (nx - 1)))
    h1c, h2c = 2.0, 0.7
    mu = -(h1c * 4 / ddx**2 * math.sin(kk * math.pi / (2 * (nx - 1))) ** 2
           + h2c * 4 / ddy**2 * math.sin(ll * math.pi / (2 * (ny - 1))) ** 2)
    tau = 0.8 * 2.0 / math.sqrt(4 * h1c / ddx**2 + 4 * h2c / ddy**2)
    th = math.acos(1 + tau * tau * mu / 2)
    try:
        r = oracle.forward(nx, ny, ddx, ddy, tau, np.full((ny, nx), h1c), np.full((ny, nx), h2c), mode, v * mode, 50,
                           want_energy=True)
        B = tau * v / math.sin(th)
        expect = (math.cos(50 * th) + B * math.sin(50 * th)) * mode
        out["p2"] = bool(np.abs(r["u_cur"] - expect).max() < 1e-10)
        # P4: for a single mode the energy is known in closed form:
        # E = |mode|^2 dx dy [ ((a1 - a0)/tau)^2 - mu a1 a0 ]
        a = [math.cos(s * th) + B * math.sin(s * th) for s in range(51)]
        msq = float(np.sum(mode * mode))
        e_exact = [ddx * ddy * msq * (((a[s + 1] - a[s]) / tau) ** 2 - mu * a[s + 1] * a[s]) for s in range(50)]
        out["p4"] = bool(np.abs(r["energy"] - np.array(e_exact)).max() < 1e-9 * abs(e_exact[0]))
    except Exception:
        out["p2"] = False
        out["p4"] = False
    # P8 the extended-precision forward: the same anisotropic eigenmode with velocity at a tiny
    # time step (sin(theta/2) = tau sqrt(-mu)/2)
    try:
        tau8 = 2e-4 * 2.0 / math.sqrt(4 * h1c / ddx**2 + 4 * h2c / ddy**2)
        th8 = 2.0 * math.asin(tau8 * math.sqrt(-mu) / 2.0)
        r8 = oracle.forward_ld(nx, ny, ddx, ddy, tau8, np.full((ny, nx), h1c), np.full((ny, nx), h2c), mode,
                               v * mode, 1500)
        B8 = tau8 * v / math.sin(th8)
        expect8 = (math.cos(1500 * th8) + B8 * math.sin(1500 * th8)) * mode
        out["p8"] = bool(np.abs(r8["u_cur"] - expect8).max() < 1e-13)
    except Exception:
        out["p8"] = False
    # P9 the implicit scheme: anisotropic eigenmode with velocity beyond the explicit limit, the
    # line solver against a dense solve, and the leapfrog limit at small tau with variable h1, h2
    try:
        s9 = 0.25
        tau9 = 3.0 * 2.0 / math.sqrt(4 * h1c / ddx**2 + 4 * h2c / ddy**2)
        mx9 = h1c * 4 / ddx**2 * math.sin(kk * math.pi / (2 * (nx - 1))) ** 2
        my9 = h2c * 4 / ddy**2 * math.sin(ll * math.pi / (2 * (ny - 1))) ** 2
        P9 = (1 + s9 * tau9 * tau9 * mx9) * (1 + s9 * tau9 * tau9 * my9)
        th9 = math.acos(1.0 - tau9 * tau9 * (mx9 + my9) / (2.0 * P9))
        r9 = oracle.adi_forward(nx, ny, ddx, ddy, tau9, s9, np.full((ny, nx), h1c), np.full((ny, nx), h2c), mode,
                                v * mode, 60)
        e9 = (math.cos(60 * th9) + tau9 * v / math.sin(th9) * math.sin(60 * th9)) * mode
        ok9 = bool(np.abs(r9["u_cur"] - e9).max() < 1e-10)
        rng9 = np.random.default_rng(9)
        lo9, up9 = rng9.normal(size=9), rng9.normal(size=9)
        di9 = np.abs(lo9) + np.abs(up9) + 1.0
        b9 = rng9.normal(size=9)
        T9 = np.diag(di9) + np.diag(lo9[1:], -1) + np.diag(up9[:-1], 1)
        ok9 = ok9 and bool(np.abs(oracle.tridiag(lo9, di9, up9, b9) - np.linalg.solve(T9, b9)).max() < 1e-12)
        n9 = 25
        xx9, yy9, X9, Y9 = I.mesh(n9, n9)
        d9 = 2.0 / (n9 - 1)
        g1 = 1.0 + 0.6 * np.exp(-((X9 - 0.1) ** 2) / 0.05) + 0.2 * Y9
        g2 = 0.8 + 0.3 * np.sin(2 * X9) * np.cos(Y9)
        w0 = I.zero_ring(np.exp(-((X9 - 0.2) ** 2 + (Y9 + 0.1) ** 2) / 0.03))
        # one start step: w0 = 2 (u^1 - u^0) solves (I - s t^2 L1)(I - s t^2 L2) w0 = t^2 A u^0; the factors
        # are applied with the (separately pinned) leapfrog operator, L1 from (h1, 0), L2 from (0, h2)
        t9 = 3.0 * d9
        w9 = 2.0 * (oracle.adi_forward(n9, n9, d9, d9, t9, 0.25, g1, g2, w0, np.zeros_like(w0), 1)["u_cur"] - w0)
        z0 = np.zeros_like(g1)
        L1 = lambda f: oracle.apply(*oracle.faces(g1, z0), f, d9, d9)
        L2 = lambda f: oracle.apply(*oracle.faces(z0, g2), f, d9, d9)
        v9 = w9 - 0.25 * t9 * t9 * L2(w9)
        res9 = v9 - 0.25 * t9 * t9 * L1(v9) - t9 * t9 * (L1(w0) + L2(w0))
        ok9 = ok9 and bool(np.abs(res9).max() < 1e-11 * np.abs(w9).max())
        out["p9"] = ok9
    except Exception:
        out["p9"] = False
    # P6 adjoint vs central FD, h1 != h2
    rng = np.random.default_rng(2)
    nx, ny, N = 12, 10, 20
    xx, yy, X, Y = I.mesh(nx, ny)
    ddx, ddy = 2.0 / (nx - 1), 2.0 / (ny - 1)
    h1 = 1.0 + 0.3 * rng.uniform(size=(ny, nx))
    h2 = 0.7 + 0.3 * rng.uniform(size=(ny, nx))
    u0 = I.zero_ring(np.exp(-((X - 0.2) ** 2 + Y**2) / 0.1))
    u1 = I.zero_ring(0.2 * np.exp(-(X**2 + (Y - 0.2) ** 2) / 0.1))
    tau = 0.4 * min(ddx, ddy) / math.sqrt(1.3)
    rec = np.array([[3, 4], [8, 2], [5, 7]], dtype=np.int32)
    dd = rng.normal(size=(N + 1, 3)) * 0.05

    def loss(a, b):
        rr = oracle.forward(nx, ny, ddx, ddy, tau, a, b, u0, u1, N, receivers=rec)
        return oracle.misfit(rr["traces"], dd), rr["traces"]

    try:
        J, tr = loss(h1, h2)
        g1, g2 = oracle.adjoint(nx, ny, ddx, ddy, tau, h1, h2, u0, u1, N, rec, 2 * (tr - dd), separate=True)
        ok = True
        for which in (1, 2):
            vv = rng.normal(size=h1.shape)
            e = 1e-6
            if which == 1:
                fd = (loss(h1 + e * vv, h2)[0] - loss(h1 - e * vv, h2)[0]) / (2 * e)
                ad = float(np.sum(g1 * vv))
            else:
                fd = (loss(h1, h2 + e * vv)[0] - loss(h1, h2 - e * vv)[0]) / (2 * e)
                ad = float(np.sum(g2 * vv))
            ok = ok and abs(fd - ad) <= 1e-6 * abs(fd)
        out["p6"] = bool(ok)
    except Exception:
        out["p6"] = False
    return out


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(tmp_path, name):
    old, new = MUTANTS[name]
    so = _build_variant(tmp_path, name, old, new)
    saved = oracle._lib
    try:
        oracle._lib = None
        real = oracle._LIB
        oracle._LIB = so
        # _load() rebuilds when the .so is older than the source; point it at the mutant only
        os.utime(so, None)
        res = _pins_pass()
    finally:
        oracle._LIB = real
        oracle._lib = saved
    assert not all(res.values()), f"mutant {name} passed every pin: {res}"


def test_real_oracle_passes_fast_pins():
    res = _pins_pass()
    assert all(res.values()), res
