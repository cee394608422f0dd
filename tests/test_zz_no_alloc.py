"""fdw_misfit_noalloc (no context, no workspace, no device allocation) against fdw_misfit on
the same arrays, through the C-ABI: two calls in a row, the second with a smaller input, in
FP32 and FP64 trace storage; the size limits are rejected on the host."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("dtype_name", ["f64", "f32"])
def test_misfit_noalloc_matches_context_misfit(dtype_name):
    import torch

    from paper_2005_11931_amd import fdw
    from paper_2005_11931_amd import inputs as I

    dt = fdw.FDW_F64 if dtype_name == "f64" else fdw.FDW_F32
    td = fdw.torch_dtype(dt)
    case = I.line_case(n=64, nsteps=10)
    s = fdw.solver_for_case(case, dtype=dt)  # a context, only for the reference fdw_misfit
    rng = np.random.default_rng(11)
    for rows, R in ((4001, 64), (301, 7)):  # the second call is smaller than the first
        _say("noalloc misfit", dtype_name, rows, R)
        tr = torch.as_tensor(rng.normal(size=(rows, R)), dtype=td, device="cuda")
        d = torch.as_tensor(rng.normal(size=(rows, R)), dtype=torch.float64, device="cuda")
        J_ref, g_ref = s.misfit(tr, d)
        J = torch.empty((), dtype=torch.float64, device="cuda")
        g = torch.full((rows, R), float("nan"), dtype=torch.float64, device="cuda")
        fdw.misfit_noalloc(tr, d, J, g)
        torch.cuda.synchronize()
        assert J.item() == J_ref.item()
        assert torch.equal(g, g_ref)
        # against the definition in FP64 on the host
        e = tr.double().cpu().numpy() - d.cpu().numpy()
        assert abs(J.item() - float(np.sum(e * e))) <= 1e-12 * float(np.sum(e * e))
        # without the adjoint source
        J2 = torch.empty((), dtype=torch.float64, device="cuda")
        fdw.misfit_noalloc(tr, d, J2, None)
        torch.cuda.synchronize()
        assert J2.item() == J_ref.item()
    s.close()


def test_misfit_noalloc_rejects_sizes_beyond_the_limits():
    import ctypes

    from paper_2005_11931_amd import fdw

    lib = fdw.lib()
    dummy = ctypes.c_void_p(1)  # never dereferenced: the size checks come first
    st = lib.fdw_misfit_noalloc(fdw.FDW_F64, dummy, dummy, 10, 16385, dummy, None, None)
    assert st == fdw.FDW_EINVAL and b"16384" in lib.fdw_noalloc_last_error()
    st = lib.fdw_misfit_noalloc(fdw.FDW_F64, dummy, dummy, 2**31, 4, dummy, None, None)
    assert st == fdw.FDW_EINVAL
    st = lib.fdw_misfit_noalloc(7, dummy, dummy, 10, 4, dummy, None, None)
    assert st == fdw.FDW_EINVAL
