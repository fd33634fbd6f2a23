"""The entry point that allocates nothing (rfd_integrate_oneshot_noalloc)
against rfd_integrate_oneshot, through the C ABI: two calls in a row on one
plan, the second with a smaller cloud and field, each bitwise equal to the
allocating entry point's result on a fresh plan (same kernels, same split of
the cloud), and both within the FP32 / BF16 bars of the oracle; the limits are
refused before any launch. Runs alone in a fresh process or after every other
GPU test."""
import ctypes as C

import numpy as np
import pytest

from oracle import rfd_oracle as o
from paper_2302_00942_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16": 2e-3}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2302_00942_amd import rfd
    rfd.lib()
    return torch


def _noalloc(torch, plan, X, F):
    """Calls the C entry point directly (ctypes), on torch's current stream."""
    from paper_2302_00942_amd import rfd
    out = torch.full_like(F, float("nan"))
    st = torch.cuda.current_stream().cuda_stream
    s = rfd.lib().rfd_integrate_oneshot_noalloc(plan.handle, X.data_ptr(), X.shape[0], F.data_ptr(), F.stride(0),
                                                F.shape[1], out.data_ptr(), out.stride(0), C.c_void_p(st))
    assert s == rfd.OK, rfd.status_string(s)
    return out


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("m,d1,d2", [(64, 16, 3), (128, 40, 9), (256, 32, 20), (256, 16, 1)])
def test_noalloc_matches_oneshot_twice(torch_cuda, prec, m, d1, d2):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    eps, lam, seed = 0.05, -0.5, 3
    calls = [(wl.torus(65536, 1), wl.field(65536, d1, 2)), (wl.sphere(3001, 4), wl.field(3001, d2, 5))]
    plan = rfd.Plan(m, eps, lam, seed, precision=prec)
    for X, F in calls:
        Xd = torch.from_numpy(X).cuda()
        Fd = torch.from_numpy(F).cuda()
        got = _noalloc(torch, plan, Xd, Fd)
        ref_plan = rfd.Plan(m, eps, lam, seed, precision=prec)
        ref = ref_plan.oneshot(Xd, Fd)
        torch.cuda.synchronize()
        assert plan.check() == rfd.OK and ref_plan.check() == rfd.OK
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(g, r), (prec, m, X.shape[0], F.shape[1], float(np.abs(g - r).max()))
        if X.shape[0] <= 3001:
            e = o.relf(g, o.rfd_integrate(X, F, eps, lam, m, seed))
            print(f"noalloc m={m} N={X.shape[0]} d={F.shape[1]} {prec}: relF={e:.3e}")
            assert e <= TOL[prec]
        ref_plan.close()
    plan.close()


def test_noalloc_leaves_the_resident_plan_alone(torch_cuda):
    """A resident plan's integrate gives the same bits before and after a
    no-alloc call on another cloud with the same plan."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    plan = rfd.Plan(128, 0.05, -0.5, 7, precision="bf16")
    X = torch.from_numpy(wl.ellipsoid(20000, 1)).cuda()
    F = torch.from_numpy(wl.field(20000, 5, 2)).cuda()
    plan.features(X)
    a = plan.integrate(F).cpu().numpy()
    _noalloc(torch, plan, torch.from_numpy(wl.sphere(5000, 3)).cuda(), torch.from_numpy(wl.field(5000, 7, 4)).cuda())
    assert plan.points == 20000
    b = plan.integrate(F).cpu().numpy()
    assert np.array_equal(a, b)
    assert plan.check() == rfd.OK


def test_noalloc_refuses_beyond_its_limits(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    plan = rfd.Plan(256, 0.05, -0.5, 0)
    X = torch.zeros((65537, 3), device="cuda")
    F = torch.zeros((65537, 4), device="cuda")
    out = torch.empty_like(F)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    L = rfd.lib()
    s = L.rfd_integrate_oneshot_noalloc(plan.handle, X.data_ptr(), 65537, F.data_ptr(), 4, 4, out.data_ptr(), 4, st)
    assert s == rfd.OUT_OF_BUDGET
    F33 = torch.zeros((100, 33), device="cuda")
    o33 = torch.empty_like(F33)
    s = L.rfd_integrate_oneshot_noalloc(plan.handle, X.data_ptr(), 100, F33.data_ptr(), 33, 33, o33.data_ptr(), 33, st)
    assert s == rfd.OUT_OF_BUDGET
    s = L.rfd_integrate_oneshot_noalloc(plan.handle, X.data_ptr(), 100, F.data_ptr(), 4, 4, None, 4, st)
    assert s == rfd.INVALID_ARG
