"""A plan whose device memory is a caller's tensor (rfd_plan_create_in):
same bits as a plan that allocates its own buffers, no device allocation by
the library after creation, and calls beyond the arena's sizing refused
before any launch."""
import numpy as np
import pytest

from oracle import rfd_oracle as o
from paper_2302_00942_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2302_00942_amd import rfd
    rfd.lib()
    return torch


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("m,n,d", [(256, 200_000, 16), (128, 30_001, 40), (64, 5000, 3)])
def test_arena_plan_matches_own_plan(torch_cuda, prec, m, n, d):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    X = torch.from_numpy(wl.torus(n, 2)).cuda()
    F = torch.from_numpy(wl.field(n, d, 3)).cuda()
    before = torch.cuda.memory_allocated()
    ap = rfd.Plan.in_arena(m, 0.03, -0.5, N_max=n, d_max=d, seed=4, precision=prec)
    nbytes = rfd.workspace_size(m, 0.03, n, d, seed=4, precision=prec)
    assert torch.cuda.memory_allocated() - before >= nbytes  # torch holds the plan's memory
    own = rfd.Plan(m, 0.03, -0.5, 4, precision=prec)
    a = ap.oneshot(X, F).cpu().numpy()
    b = own.oneshot(X, F).cpu().numpy()
    assert ap.check() == rfd.OK and np.array_equal(a, b)
    # resident use and a smaller cloud in the same arena
    assert np.array_equal(ap.integrate(F).cpu().numpy(), own.integrate(F).cpu().numpy())
    Xs, Fs = X[: n // 3].contiguous(), F[: n // 3].contiguous()
    assert np.array_equal(ap.oneshot(Xs, Fs).cpu().numpy(), own.oneshot(Xs, Fs).cpu().numpy())
    if n <= 5000:
        ref = o.rfd_integrate(wl.torus(n, 2)[: n // 3], wl.field(n, d, 3)[: n // 3], 0.03, -0.5, m, 4)
        assert o.relf(ap.oneshot(Xs, Fs).cpu().numpy(), ref) <= {"fp32": 1e-5, "bf16": 2e-3}[prec]


def test_arena_plan_refuses_beyond_its_sizing(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    ap = rfd.Plan.in_arena(128, 0.05, -0.5, N_max=1000, d_max=16, seed=1)
    X = torch.from_numpy(wl.sphere(1001, 1)).cuda()
    F = torch.zeros((1001, 4), device="cuda")
    with pytest.raises(rfd.RfdError) as e:
        ap.oneshot(X, F)
    assert e.value.status == rfd.OUT_OF_BUDGET
    with pytest.raises(rfd.RfdError) as e:
        ap.features(X)
    assert e.value.status == rfd.OUT_OF_BUDGET
    X1 = X[:1000].contiguous()
    ap.features(X1)
    with pytest.raises(rfd.RfdError) as e:
        ap.integrate(torch.zeros((1000, 1024), device="cuda"))  # wider slices than the sizing
    assert e.value.status == rfd.OUT_OF_BUDGET
    out = ap.integrate(torch.ones((1000, 16), device="cuda"))
    assert ap.check() == rfd.OK and torch.isfinite(out).all()
    # too small an arena
    arena = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    import ctypes as C
    p, _ = rfd.make_params(256, 0.05, -0.5)
    h = C.c_void_p()
    s = rfd.lib().rfd_plan_create_in(C.byref(p), (arena.data_ptr() + 255) & ~255, 1 << 19, 1000, 16, C.byref(h))
    assert s == rfd.OUT_OF_BUDGET
