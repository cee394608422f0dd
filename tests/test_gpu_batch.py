"""Batched family of regularisations: one launch per time block over all members, and
one persistent cooperative launch per step_n call.  Each member must equal its own
single-member solve bit for bit, and the oracle within the FP64 / FP32 bars."""
import sys

import numpy as np
import pytest

import oracle
from paper_2005_11931_amd import inputs as I

pytestmark = pytest.mark.gpu


def _fdw():
    from paper_2005_11931_amd import fdw

    return fdw


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _small_family(count=6, nsteps=90, sizes=(67, 131, 200)):
    return I.family(count=count, nsteps=nsteps, sizes=sizes)


def _states(s):
    return [tuple(t.cpu().numpy() for t in s.get_state(m)[:2]) for m in range(s.count)]


def _single(case, dtype, n, K=0, energy=False):
    fdw = _fdw()
    s = fdw.solver_for_case(case, dtype=dtype)
    if K:
        s.configure(fdw.FDW_CFG_TIME_BLOCK, K)
    e = s.step(n, energy=energy)
    u, du, _ = s.get_state()
    out = (u.cpu().numpy(), du.cpu().numpy(), None if e is None else e[0].cpu().numpy())
    s.close()
    return out


@pytest.mark.parametrize("dtype_name", ["f32", "f64"])
def test_batched_equals_single_and_oracle(dtype_name):
    fdw = _fdw()
    dt = fdw.FDW_F32 if dtype_name == "f32" else fdw.FDW_F64
    fam = _small_family()
    N = fam[0].nsteps
    _say("batched", dtype_name)
    # K = 8 ends in a shorter time block whose decomposition has a different wave count (the
    # grouped energy finalisation of the earlier blocks must use theirs)
    for K in (1, 3, 4, 8):
        s = fdw.family_solver(fam, dtype=dt)
        s.configure(fdw.FDW_CFG_TIME_BLOCK, K)
        E = s.step(N, energy=True).cpu().numpy()
        st = _states(s)
        s.close()
        for m, case in enumerate(fam):
            u1, du1, e1 = _single(case, dt, N, K=K, energy=True)
            assert np.array_equal(st[m][0], u1) and np.array_equal(st[m][1], du1), (K, m)
            assert np.abs(E[m] - e1).max() <= (1e-13 if dt == fdw.FDW_F64 else 1e-7) * abs(e1[0])
            ref = oracle.forward_case(case, want_energy=True)
            if dt == fdw.FDW_F64:
                assert np.abs(st[m][0] - ref["u_cur"]).max() <= 1e-12
                assert np.abs(E[m] - ref["energy"]).max() <= 1e-12 * ref["energy"][0]
            else:
                assert np.abs(st[m][0] - ref["u_cur"]).max() <= 1e-5 * np.abs(ref["u_cur"]).max()


@pytest.mark.parametrize("dtype_name", ["f32", "f64"])
def test_persistent_equals_per_block_launches(dtype_name):
    fdw = _fdw()
    dt = fdw.FDW_F32 if dtype_name == "f32" else fdw.FDW_F64
    fam = _small_family(count=8, nsteps=203)
    _say("persistent", dtype_name)
    for K in (1, 2, 4):
        a = fdw.family_solver(fam, dtype=dt)
        a.configure(fdw.FDW_CFG_TIME_BLOCK, K)
        a.step(203)
        sa = _states(a)
        a.close()
        b = fdw.family_solver(fam, dtype=dt)
        b.configure(fdw.FDW_CFG_TIME_BLOCK, K)
        b.configure(fdw.FDW_CFG_BATCH_MODE, 1)
        b.step(1)
        b.step(150)
        b.step(52)
        sb = _states(b)
        b.close()
        for m in range(len(fam)):
            assert np.array_equal(sa[m][0], sb[m][0]) and np.array_equal(sa[m][1], sb[m][1]), (K, m)


def test_member_reset_mid_run():
    """A member returned to step 0 restarts (start step) while the others continue."""
    fdw = _fdw()
    fam = _small_family(count=3, nsteps=100)
    _say("reset mid-run")
    s = fdw.family_solver(fam, dtype=fdw.FDW_F64)
    s.step(30)
    s.reset(1)
    s.step(40)
    assert [s.steps_taken(m) for m in range(3)] == [70, 40, 70]
    st = _states(s)
    s.close()
    for m, n in ((0, 70), (1, 40), (2, 70)):
        ref = oracle.forward_case(fam[m], nsteps=n)["u_cur"]
        assert np.abs(st[m][0] - ref).max() <= 1e-12, m


def test_full_family_launch_configuration():
    """The 32-member family (512^2 .. 4096^2, FP32) in the benchmark's launch configuration:
    after 24 steps every member equals its single-member solve bit for bit; the smallest
    members are also run for the full 2000 steps against the oracle."""
    import torch

    fdw = _fdw()
    fam = I.family()
    _say("full family")
    s = fdw.family_solver(fam, dtype=fdw.FDW_F32)
    s.configure(fdw.FDW_CFG_BATCH_MODE, 1)
    s.step(24)
    st = _states(s)
    s.close()
    torch.cuda.empty_cache()
    for m, case in enumerate(fam):
        u1, du1, _ = _single(case, fdw.FDW_F32, 24)
        assert np.array_equal(st[m][0], u1) and np.array_equal(st[m][1], du1), m
    for m in (0, 28):  # 512^2 jump member, 512^2 smallest-eps delta member
        case = fam[m]
        u, _, _ = _single(case, fdw.FDW_F32, case.nsteps)
        ref = oracle.forward_case(case)["u_cur"]
        rel = np.abs(u - ref).max() / np.abs(ref).max()
        _say("member", m, "fp32 rel", rel)
        assert rel <= 1e-5


@pytest.mark.parametrize("dtype_name", ["f32", "f64"])
@pytest.mark.parametrize("graph", [0, 1])
def test_persistent_with_energy_vs_oracle(dtype_name, graph):
    """The persistent launch with the per-step energy summed inside it, plain and replayed from a
    hipGraph, member by member against the oracle: states (FP64 max-abs 1e-12, FP32 1e-5
    relative) and every energy (FP64 1e-12 relative, FP32 1e-5 relative); the state equals the
    per-time-block launches bit for bit and the energies agree with theirs to rounding.  Two
    calls of 1 + 150 + 52 steps: the start step, a call that spans the in-kernel energy sums,
    and one with a tail; the graph is replayed for a second solve from step 0."""
    fdw = _fdw()
    dt = fdw.FDW_F32 if dtype_name == "f32" else fdw.FDW_F64
    fam = _small_family(count=8, nsteps=203)
    _say("persistent + energy vs oracle", dtype_name, "graph", graph)
    a = fdw.family_solver(fam, dtype=dt)
    Ea = a.step(203, energy=True).cpu().numpy()
    sa = _states(a)
    a.close()
    b = fdw.family_solver(fam, dtype=dt)
    b.configure(fdw.FDW_CFG_BATCH_MODE, 1)
    b.configure(fdw.FDW_CFG_USE_GRAPH, graph)
    for rep in range(2 if graph else 1):
        for m in range(len(fam)):
            b.reset(m)
        E = np.concatenate([b.step(k, energy=True).cpu().numpy() for k in (1, 150, 52)], axis=1)
        sb = _states(b)
        for m, case in enumerate(fam):
            assert np.array_equal(sa[m][0], sb[m][0]) and np.array_equal(sa[m][1], sb[m][1]), (rep, m)
            assert np.abs(E[m] - Ea[m]).max() <= (1e-13 if dt == fdw.FDW_F64 else 1e-6) * abs(Ea[m][0]), (rep, m)
            ref = oracle.forward_case(case, want_energy=True)
            if dt == fdw.FDW_F64:
                assert np.abs(sb[m][0] - ref["u_cur"]).max() <= 1e-12
                assert np.abs(E[m] - ref["energy"]).max() <= 1e-12 * ref["energy"][0]
            else:
                assert np.abs(sb[m][0] - ref["u_cur"]).max() <= 1e-5 * np.abs(ref["u_cur"]).max()
                assert np.abs(E[m] - ref["energy"]).max() <= 1e-5 * ref["energy"][0]
    b.close()


def test_persistent_barrier_timeout_is_reported():
    """The persistent launch's barrier error word is read back after the call: the host marks it
    (test hook; no kernel waits on it) and the call returns FDW_ESYNC; the next call is clean."""
    fdw = _fdw()
    fam = _small_family(count=4, nsteps=60)
    s = fdw.family_solver(fam, dtype=fdw.FDW_F32)
    s.configure(fdw.FDW_CFG_BATCH_MODE, 1)
    s.step(1)
    s.configure(fdw.FDW_CFG_TEST_BARRIER_FLAG, 1)
    with pytest.raises(fdw.FdwError) as e:
        s.step(16)
    assert e.value.status == fdw.FDW_ESYNC
    assert s.config(fdw.FDW_CFG_TEST_BARRIER_FLAG) == 0
    s.step(16)
    s.close()


@pytest.mark.parametrize("batch_mode", [0, 1])
def test_mixed_storage_family_vs_oracle(batch_mode):
    """A family whose two smallest-eps members are stored in FP64 and the others in FP32 (one
    launch sequence per storage type), with energies: every member against the oracle at its
    own storage type's bar, the FP64 members equal to their single-member FP64 solves bit for
    bit, energies in the family's row of each member, per-member state, traces and adjoint
    routed to the right type, and the FP32-vs-FP64 distance refused."""
    import torch

    fdw = _fdw()
    fam = _small_family(count=6, nsteps=120)
    dts = [fdw.FDW_F32] * 4 + [fdw.FDW_F64] * 2
    _say("mixed family, batch mode", batch_mode)
    s = fdw.family_solver(fam, dtype=dts)
    s.configure(fdw.FDW_CFG_BATCH_MODE, batch_mode)
    E = s.step(120, energy=True).cpu().numpy()
    st = _states(s)
    for m, case in enumerate(fam):
        ref = oracle.forward_case(case, want_energy=True)
        if dts[m] == fdw.FDW_F64:
            assert st[m][0].dtype == np.float64
            u1, du1, e1 = _single(case, fdw.FDW_F64, 120, energy=True)
            assert np.array_equal(st[m][0], u1) and np.array_equal(st[m][1], du1), m
            assert np.abs(st[m][0] - ref["u_cur"]).max() <= 1e-12
            assert np.abs(E[m] - ref["energy"]).max() <= 1e-12 * ref["energy"][0]
        else:
            assert st[m][0].dtype == np.float32
            assert np.abs(st[m][0] - ref["u_cur"]).max() <= 1e-5 * np.abs(ref["u_cur"]).max()
            assert np.abs(E[m] - ref["energy"]).max() <= 1e-5 * ref["energy"][0]
    hosts = s.energy()
    assert all(abs(hosts[m] - E[m][-1]) <= 1e-6 * abs(E[m][-1]) for m in range(len(fam)))
    assert [s.steps_taken(m) for m in range(len(fam))] == [120] * len(fam)
    with pytest.raises(fdw.FdwError) as e:
        s.distance(0, 5)
    assert e.value.status == fdw.FDW_ENOTSUP
    # adjoint of an FP64 member of the mixed family against the oracle
    case = fam[5]
    # receivers at and beside the largest initial displacement (where the traces carry signal)
    jm, im = np.unravel_index(np.argmax(np.abs(case.u0)), case.u0.shape)
    rec = np.array([[im, jm], [im + 3, jm], [im, jm - 4]], dtype=np.int32)
    N = case.nsteps
    tg = np.random.default_rng(5).normal(size=(N + 1, 3))
    g = s.adjoint(torch.as_tensor(rec), torch.as_tensor(tg), ckpt_every=16, member=5).cpu().numpy()
    gref = oracle.adjoint(case.nx, case.ny, case.dx, case.dy, case.tau, case.h1, None, case.u0, case.u1, N, rec, tg,
                          ckpt_every=16)
    assert np.linalg.norm(g - gref) <= 1e-9 * np.linalg.norm(gref)
    s.close()
