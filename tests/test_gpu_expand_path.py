"""The two arithmetic paths of the expansion out = F + A G' for fields of at
most four channels (Sec. 2.4, the A (G) step with m d small): the matrix
cores (F and G' enter as BF16 hi + lo pairs in BF16 mode, FP32 MFMA in FP32
mode) and FP32 FMAs, one thread per point (k_expand_valu). Both are held to
the oracle's bars; a batch takes each cloud's path from the same table entry
as the single-cloud entry points, so it stays bitwise equal to them; the
autotuner times both paths and records the faster."""
import numpy as np
import pytest

from oracle import rfd_oracle as o
from paper_2302_00942_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16": 2e-3}
MFMA, VALU = 1, 2


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2302_00942_amd import rfd
    rfd.lib()
    return torch


def _force(rfd, M, prec, d, path):
    rfd.tune_import(f"3 {M} {1 if prec == 'bf16' else 0} 1 {d} {path}\n")


def _padded(m):
    return 64 if m <= 64 else (128 if m <= 128 else 256)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("m,n", [(64, 5003), (128, 3001), (256, 2049), (30, 777)])
def test_both_paths_match_the_oracle(torch_cuda, prec, m, n):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    X = wl.ellipsoid(n, 3)
    try:
        for d in (1, 2, 3, 4):
            F = wl.field(n, d, 10 + d)
            ref = o.rfd_integrate(X, F, 0.05, -0.5, m, 2)
            outs = {}
            for path in (MFMA, VALU):
                _force(rfd, _padded(m), prec, d, path)
                plan = rfd.Plan(m, 0.05, -0.5, 2, precision=prec)
                Xd, Fd = torch.from_numpy(X).cuda(), torch.from_numpy(F).cuda()
                one = plan.oneshot(Xd, Fd).cpu().numpy()
                res = plan.integrate(Fd).cpu().numpy()  # resident: the same expansion path
                assert plan.check() == rfd.OK
                outs[path] = one
                e = o.relf(one, ref)
                print(f"m={m} N={n} d={d} {prec} path={'mfma' if path == MFMA else 'fma'}: relF={e:.3e}")
                assert e <= TOL[prec]
                assert o.relf(res, ref) <= TOL[prec]
            # two roundings of one result
            assert o.relf(outs[VALU], outs[MFMA]) <= TOL[prec]
    finally:
        rfd.tune_reset()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_follows_the_single_cloud_path(torch_cuda, prec):
    """Mixed widths in one batch, with the FMA path forced on for d = 3 and
    the rule's choice elsewhere: every cloud equals its one-shot result
    bitwise."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    clouds = wl.uneven_batch(count=6, d=3, m=128, seed=8, lo=1500, hi=9000)
    widths = [3, 1, 16, 4, 2, 40]
    Fs_np = [wl.field(c.n, dd, 70 + i) for i, (c, dd) in enumerate(zip(clouds, widths))]
    try:
        for forced in (None, VALU, MFMA):
            rfd.tune_reset()
            if forced is not None:
                _force(rfd, 128, prec, 3, forced)
            plans = [rfd.Plan(c.m, c.eps, c.lam, c.seed, precision=prec) for c in clouds]
            Xs = [torch.from_numpy(c.X).cuda() for c in clouds]
            Fs = [torch.from_numpy(F).cuda() for F in Fs_np]
            outs = [torch.empty_like(F) for F in Fs]
            rfd.Batch(plans, Xs, Fs, outs).launch()
            torch.cuda.synchronize()
            for c, X, F, out in zip(clouds, Xs, Fs, outs):
                alone = rfd.Plan(c.m, c.eps, c.lam, c.seed, precision=prec).oneshot(X, F)
                assert np.array_equal(alone.cpu().numpy(), out.cpu().numpy()), (forced, prec, F.shape[1])
    finally:
        rfd.tune_reset()


def test_autotune_records_an_expansion_path(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    rfd.tune_reset()
    try:
        c = wl.plain_sphere(n=200_000, d=3, m=128, seed=5)
        for prec in ("fp32", "bf16"):
            plan = rfd.Plan(c.m, c.eps, c.lam, c.seed, precision=prec)
            plan.features(torch.from_numpy(c.X).cuda())
            Fd = torch.from_numpy(c.F).cuda()
            out = torch.empty_like(Fd)
            plan.autotune(Fd, out, reps=3)
            after = plan.integrate(Fd).cpu().numpy()
            assert np.array_equal(out.cpu().numpy(), after)
        rows = [ln.split() for ln in rfd.tune_export().splitlines()]
        paths = [r for r in rows if r[0] == "3"]
        print("expansion paths:", paths)
        assert len(paths) == 2 and all(r[1] == "128" and r[4] == "3" and r[5] in ("1", "2") for r in paths)
    finally:
        rfd.tune_reset()
