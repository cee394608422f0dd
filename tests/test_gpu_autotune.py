"""The autotuner (fdw_autotune): it picks a supported (time block, segment rows, lane columns)
configuration for a batched context, caches it under the context's key, and the results it
leads to equal those of the default configuration bit for bit (the launch configuration never
changes the arithmetic)."""
import os

import numpy as np
import pytest

from paper_2005_11931_amd import inputs as I

pytestmark = pytest.mark.gpu


def _cases():
    out = []
    for k, (nx, ny) in enumerate([(300, 200), (512, 384), (257, 257)]):
        rng = np.random.default_rng(700 + k)
        x, y, X, Y = I.mesh(nx, ny)
        h = 1.0 + 2.0 * I.gaussian_1d(X, 0.05) + 0.2 * rng.uniform(size=(ny, nx))
        u0 = I.zero_ring(np.exp(-((X - 0.3) ** 2 + (Y + 0.1) ** 2) / 0.01))
        dx, dy = 2.0 / (nx - 1), 2.0 / (ny - 1)
        tau = 0.45 / np.sqrt(h.max() * (1 / dx**2 + 1 / dy**2))
        out.append(I.Case(f"tune{k}", nx, ny, -1, 1, -1, 1, tau, 200, h, None, u0, np.zeros_like(u0)))
    # one time step for all members (the family advances in lock-step)
    tau = min(c.tau for c in out)
    return [I.Case(**{**c.__dict__, "tau": tau}) for c in out]


@pytest.mark.parametrize("dtype_name", ["f32", "f64"])
def test_autotune_choice_cache_and_bitwise_results(tmp_path, dtype_name):
    import torch

    from paper_2005_11931_amd import fdw

    dt = fdw.FDW_F32 if dtype_name == "f32" else fdw.FDW_F64
    cases = _cases()
    cache = tmp_path / "tune.txt"
    os.environ["FDW_AUTOTUNE_CACHE"] = str(cache)
    try:
        print("autotune", dtype_name, flush=True)
        s = fdw.family_solver(cases, dtype=dt)
        K, S, C = s.autotune(steps=32)
        assert (K, S, C) == (s.config(fdw.FDW_CFG_TIME_BLOCK), s.config(fdw.FDW_CFG_SEGMENT_ROWS),
                             s.config(fdw.FDW_CFG_LANE_COLUMNS))
        if dt == fdw.FDW_F32:
            assert (C == 2 and 1 <= K <= 8) or (C == 4 and 1 <= K <= 6)
        else:
            assert (C == 2 and 1 <= K <= 4) or (C == 1 and 1 <= K <= 8)
        assert S in (8, 16, 32, 48, 64, 96, 128)
        assert all(s.steps_taken(m) == 0 for m in range(len(cases)))
        text = cache.read_text()
        P = s.config(fdw.FDW_CFG_STREAM_POLICY)
        assert P in (0, 3)
        assert text.count("|") == 1 and text.strip().endswith(f"{K} {S} {C} {P}")
        e = s.step(150, energy=True).cpu().numpy()
        tuned = [s.get_state(m)[0].cpu().numpy() for m in range(len(cases))]
        s.close()
        # a second context of the same shape takes the cached choice
        s2 = fdw.family_solver(cases, dtype=dt)
        assert s2.autotune(steps=32) == (K, S, C)
        s2.close()
        assert cache.read_text() == text
        # the default configuration gives the same numbers, bit for bit
        s3 = fdw.family_solver(cases, dtype=dt)
        e3 = s3.step(150, energy=True).cpu().numpy()
        for m in range(len(cases)):
            assert np.array_equal(tuned[m], s3.get_state(m)[0].cpu().numpy()), m
        tol = 1e-13 if dt == fdw.FDW_F64 else 1e-6
        assert np.abs(e - e3).max() <= tol * np.abs(e3).max()
        s3.close()
    finally:
        del os.environ["FDW_AUTOTUNE_CACHE"]


@pytest.mark.parametrize("batch_mode", [0, 1])
def test_autotune_in_graph_and_persistent_modes(tmp_path, batch_mode):
    """Tuning under the context's own launch mode (hipGraph replay, and the persistent launch,
    which takes time blocks 1, 2, 4, 8 only): the choice is cached under a key that names the
    mode, and the tuned solve equals the default one bit for bit."""
    from paper_2005_11931_amd import fdw

    cases = _cases()
    cache = tmp_path / "tune.txt"
    os.environ["FDW_AUTOTUNE_CACHE"] = str(cache)
    try:
        print("autotune graph, batch mode", batch_mode, flush=True)
        s = fdw.family_solver(cases, dtype=fdw.FDW_F32)
        s.configure(fdw.FDW_CFG_USE_GRAPH, 1)
        s.configure(fdw.FDW_CFG_BATCH_MODE, batch_mode)
        K, S, C = s.autotune(steps=32)
        if batch_mode == 1:
            assert K in (1, 2, 4, 8)
        assert s.config(fdw.FDW_CFG_USE_GRAPH) == 1 and s.config(fdw.FDW_CFG_BATCH_MODE) == batch_mode
        assert f" g1b{batch_mode}|" in cache.read_text()
        s.step(150)
        tuned = [s.get_state(m)[0].cpu().numpy() for m in range(len(cases))]
        s.close()
        s3 = fdw.family_solver(cases, dtype=fdw.FDW_F32)
        s3.step(150)
        for m in range(len(cases)):
            assert np.array_equal(tuned[m], s3.get_state(m)[0].cpu().numpy()), m
        s3.close()
    finally:
        del os.environ["FDW_AUTOTUNE_CACHE"]


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_autotune_adjoint(tmp_path, dtype_name):
    """Tuning the reverse sweep (time block, lane columns, rows per item) on a recorded forward
    run: a supported choice is applied and cached, and the gradient it gives agrees with the
    default configuration's (the time block groups the FP64 gradient sums differently, so to
    rounding: 1e-12 relative in FP64)."""
    import torch

    from paper_2005_11931_amd import fdw

    dt = fdw.FDW_F64 if dtype_name == "f64" else fdw.FDW_F32
    case, _ = I.adjoint_case(n=384, nsteps=300, nrecv=16)
    rec = torch.as_tensor(case.receivers)
    tg = torch.as_tensor(np.random.default_rng(9).normal(size=(case.nsteps + 1, 16)))
    cache = tmp_path / "tune.txt"
    os.environ["FDW_AUTOTUNE_CACHE"] = str(cache)
    try:
        print("autotune adjoint", dtype_name, flush=True)
        s0 = fdw.solver_for_case(case, dtype=dt)
        g0 = s0.adjoint(rec, tg, ckpt_every=64).cpu().numpy()
        s0.close()
        s = fdw.solver_for_case(case, dtype=dt)
        s.record_checkpoints(64)
        s.step(case.nsteps)
        K, S, C = s.autotune_adjoint(rec, tg, ckpt_every=64)
        assert (K, S, C) == (s.config(fdw.FDW_CFG_ADJ_TIME_BLOCK), s.config(fdw.FDW_CFG_ADJ_SEGMENT_ROWS),
                             s.config(fdw.FDW_CFG_ADJ_LANE_COLUMNS))
        narrow = 1 if dt == fdw.FDW_F64 else 2
        assert (C == narrow and 2 <= K <= 6) or (C == 2 * narrow and 2 <= K <= 4)
        assert " adj m0 " in cache.read_text()
        g = s.adjoint(rec, tg, ckpt_every=64).cpu().numpy()
        s.close()
        tol = 1e-12 if dt == fdw.FDW_F64 else 1e-4
        assert np.abs(g - g0).max() <= tol * np.abs(g0).max()
    finally:
        del os.environ["FDW_AUTOTUNE_CACHE"]


def test_autotune_stream_policy_on_a_grid_beyond_the_cache(tmp_path):
    """A float grid whose working set exceeds the last-level cache (2 x 256 MiB): the tuner also
    times the non-temporal-stores / cacheable-loads policy, caches its choice with the triple,
    and a second context takes both from the cache; the tuned solve equals the default one bit
    for bit."""
    from paper_2005_11931_amd import fdw

    n = 6144  # 5 planes x 6144^2 x 4 B = 755 MB
    x, y, X, Y = I.mesh(n, n)
    h = 1.0 + 0.5 * np.exp(-(X**2 + Y**2) / 0.05)
    u0 = I.zero_ring(np.exp(-((X - 0.2) ** 2 + Y**2) / 0.01))
    dx = 2.0 / (n - 1)
    tau = 0.45 / np.sqrt(h.max() * 2 / dx**2)
    case = I.Case("big", n, n, -1, 1, -1, 1, tau, 64, h, None, u0, np.zeros_like(u0))
    cache = tmp_path / "tune.txt"
    os.environ["FDW_AUTOTUNE_CACHE"] = str(cache)
    try:
        print("autotune stream policy", flush=True)
        s = fdw.solver_for_case(case, dtype=fdw.FDW_F32)
        K, S, C = s.autotune(steps=16)
        P = s.config(fdw.FDW_CFG_STREAM_POLICY)
        assert P in (0, 3)
        assert cache.read_text().strip().endswith(f"{K} {S} {C} {P}")
        s.step(40)
        tuned = s.get_state()[0].cpu().numpy()
        s.close()
        s2 = fdw.solver_for_case(case, dtype=fdw.FDW_F32)
        assert s2.autotune(steps=16) == (K, S, C) and s2.config(fdw.FDW_CFG_STREAM_POLICY) == P
        s2.close()
        s3 = fdw.solver_for_case(case, dtype=fdw.FDW_F32)
        s3.step(40)
        assert np.array_equal(tuned, s3.get_state()[0].cpu().numpy())
        s3.close()
    finally:
        del os.environ["FDW_AUTOTUNE_CACHE"]
