"""FP64 precision of the device phi_1 (Sec. 2.4: the m x m core exponential,
the one step of the path computed in FP64).

The end-to-end parity tests see phi_1 only through out, where an FP32 phi_1
would pass. Here the device's own core M (rfd_plan_core) is handed to the
oracle's phi_1 (dense Pade [13/13] on the augmented matrix, scaling and
squaring, FP64), and the device results are held to a bar that only FP64
arithmetic meets:

* S = lambda phi_1(lambda M) (the full form, resident plans);
* G = lambda phi_1(lambda M) H (the action form of one-shot calls with at
  most 32 channels), with H the device's own FP64 B^T F (rfd_plan_action).

Bar: relative Frobenius error <= 1e-11. The device's Taylor-23 scheme and the
oracle's Pade scheme, both in FP64, differ by at most ~2e-14 on these cores
(FP64 NumPy emulation of the device scheme), while the same scheme in FP32
is off by 5e-7 ... 7e-6 (the 1M-point core: 2.3e-6)."""
import numpy as np
import pytest

from oracle import rfd_oracle as o
from paper_2302_00942_amd import workloads as wl

pytestmark = pytest.mark.gpu

BAR = 1e-11


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2302_00942_amd import rfd
    rfd.lib()
    return torch


def _check_core(plan, lam, label):
    M, S, s = plan.core()
    ref = lam * o.phi1(lam * M)
    e = o.relf(S, ref)
    print(f"[{label}] s={s} ||lam M||_1={np.abs(lam * M).sum(0).max():.4g} relF(S)={e:.3e}")
    assert np.all(np.isfinite(S))
    assert e <= BAR, (label, e)
    return M


CASES = [  # (surface, N, m, eps, lam)
    ("sphere", 2000, 64, 0.1, -0.5),
    ("torus", 5003, 128, 0.05, -0.5),
    ("ellipsoid", 300, 128, 0.05, -0.5),   # N < m: singular core
    ("torus", 20000, 256, 0.05, -0.5),
    ("sphere", 4000, 30, 0.1, -1.0),       # m padded to 64
    ("sphere", 3000, 64, 0.05, 0.02),      # lambda > 0
]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}{c[1]}_m{c[2]}" for c in CASES])
def test_full_form_s_is_fp64(torch_cuda, case, prec):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    kind, N, m, eps, lam = case
    X = wl.surface(kind, N, 5)
    plan = rfd.Plan(m, eps, lam, 3, precision=prec)
    plan.features(torch.from_numpy(X).cuda())
    assert plan.check() == rfd.OK
    _check_core(plan, lam, f"S {kind} N={N} m={m} {prec}")


@pytest.mark.parametrize("d", [1, 3, 16, 32])
@pytest.mark.parametrize("case", CASES[:4], ids=[f"{c[0]}{c[1]}_m{c[2]}" for c in CASES[:4]])
def test_action_form_g_is_fp64(torch_cuda, case, d):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    kind, N, m, eps, lam = case
    X = wl.surface(kind, N, 6)
    F = wl.field(N, d, 7)
    plan = rfd.Plan(m, eps, lam, 4, precision="bf16")
    plan.oneshot(torch.from_numpy(X).cuda(), torch.from_numpy(F).cuda())
    assert plan.check() == rfd.OK
    H, G = plan.action()
    assert H.shape == (m, d) and G.shape == (m, d)
    M, _, _ = plan.core()  # forms S (the action form left it stale); M is unchanged
    ref = lam * (o.phi1(lam * M) @ H)
    e = o.relf(G, ref)
    print(f"[G {kind} N={N} m={m} d={d}] relF(G)={e:.3e}")
    assert e <= BAR, e
    # H is B^T F of the device's BF16 features against the oracle's FP64 ones
    om, w = plan.export()
    Phi, _ = o.features(X, om, w)
    assert o.relf(H, Phi.T @ F.astype(np.float64)) < 2e-2


def test_headline_core_is_fp64(torch_cuda):
    """The 1M-point torus (m = 256, d = 16, BF16, the benchmark's one-shot
    call): ||lambda M||_1 ~ 1.6e4 and 13 squarings. Both the action-form G of
    the one-shot call and the full-form S are held to the FP64 bar."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    c = wl.large_torus()
    plan = rfd.Plan(c.m, c.eps, c.lam, c.seed, precision="bf16")
    plan.oneshot(torch.from_numpy(c.X).cuda(), torch.from_numpy(c.F).cuda())
    assert plan.check() == rfd.OK
    H, G = plan.action()
    M = _check_core(plan, c.lam, "S torus N=1e6 m=256")
    e = o.relf(G, c.lam * (o.phi1(c.lam * M) @ H))
    print(f"[G torus N=1e6 m=256 d=16] relF(G)={e:.3e}")
    assert e <= BAR, e


def test_action_export_needs_an_action_call(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    plan = rfd.Plan(64, 0.1, -0.5, 0)
    plan.features(torch.from_numpy(wl.sphere(500, 1)).cuda())
    with pytest.raises(rfd.RfdError) as e:
        plan.action()
    assert e.value.status == rfd.NOT_READY
