"""GPU: batched integration of many uneven clouds (one launch per stage,
hipGraph replay) against the per-cloud entry point and the CPU oracle."""
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


def _clouds(count, d, m, seed, lo=1000, hi=20000):
    return wl.uneven_batch(count=count, d=d, m=m, seed=seed, lo=lo, hi=hi)


def _single(torch, c, prec, d=None):
    from paper_2302_00942_amd import rfd
    plan = rfd.Plan(c.m, c.eps, c.lam, c.seed, precision=prec)
    out = plan.oneshot(torch.from_numpy(c.X).cuda(), torch.from_numpy(c.F).cuda())
    assert plan.check() == rfd.OK
    return out.cpu().numpy()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_equals_per_cloud_bitwise(torch_cuda, prec):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    clouds = _clouds(24, 3, 128, 5)
    plans = [rfd.Plan(c.m, c.eps, c.lam, c.seed, precision=prec) for c in clouds]
    Xs = [torch.from_numpy(c.X).cuda() for c in clouds]
    Fs = [torch.from_numpy(c.F).cuda() for c in clouds]
    outs = [torch.empty_like(F) for F in Fs]
    b = rfd.Batch(plans, Xs, Fs, outs)
    b.launch()
    torch.cuda.synchronize()
    for p in plans:
        assert p.check() == rfd.OK
    for i, c in enumerate(clouds):
        got = outs[i].cpu().numpy()
        ref = _single(torch, c, prec)
        assert np.array_equal(got, ref), (i, c.n, np.abs(got - ref).max())
    # and against the oracle for a few
    tol = {"fp32": 1e-5, "bf16": 2e-3}[prec]
    for i in (0, 7, 23):
        c = clouds[i]
        e = o.relf(outs[i].cpu().numpy(), o.rfd_integrate(c.X, c.F, c.eps, c.lam, c.m, c.seed))
        print(f"batch cloud {i} N={c.n} {prec}: relF={e:.3e}")
        assert e <= tol
    b.close()


def test_batch_graph_replay_matches_eager(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    clouds = _clouds(16, 3, 64, 9)
    plans = [rfd.Plan(c.m, c.eps, c.lam, c.seed, precision="bf16") for c in clouds]
    Xs = [torch.from_numpy(c.X).cuda() for c in clouds]
    Fs = [torch.from_numpy(c.F).cuda() for c in clouds]
    outs = [torch.empty_like(F) for F in Fs]
    s = torch.cuda.Stream()
    b = rfd.Batch(plans, Xs, Fs, outs)
    results = []
    for it in range(4):  # eager, capture + replay, replay, replay
        for o_ in outs:
            o_.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            b.launch(stream=s)
        s.synchronize()
        results.append([o_.cpu().numpy() for o_ in outs])
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda")
        junk.mul_(2.0).sum().item()
    for it in range(1, 4):
        for a, r in zip(results[0], results[it]):
            assert np.array_equal(a, r), it
    b.close()


def test_batch_mixed_field_widths(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    clouds = _clouds(6, 3, 128, 13)
    widths = [3, 16, 1, 9, 16, 5]
    Fs_np = [wl.field(c.n, dd, 100 + i) for i, (c, dd) in enumerate(zip(clouds, widths))]
    plans = [rfd.Plan(c.m, c.eps, c.lam, c.seed, precision="fp32") for c in clouds]
    Xs = [torch.from_numpy(c.X).cuda() for c in clouds]
    Fs = [torch.from_numpy(F).cuda() for F in Fs_np]
    outs = [torch.empty_like(F) for F in Fs]
    rfd.Batch(plans, Xs, Fs, outs).launch()
    torch.cuda.synchronize()
    for c, F, out in zip(clouds, Fs_np, outs):
        e = o.relf(out.cpu().numpy(), o.rfd_integrate(c.X, F, c.eps, c.lam, c.m, c.seed))
        assert e <= 1e-5, e


def test_batch_rejects_mixed_m(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    cs = _clouds(2, 3, 64, 1)
    plans = [rfd.Plan(64, 0.05, -0.5, 0), rfd.Plan(128, 0.05, -0.5, 0)]
    Xs = [torch.from_numpy(c.X).cuda() for c in cs]
    Fs = [torch.from_numpy(c.F).cuda() for c in cs]
    with pytest.raises(rfd.RfdError) as e:
        rfd.Batch(plans, Xs, Fs, [torch.empty_like(F) for F in Fs])
    assert e.value.status == rfd.INVALID_ARG


def test_uneven_batch_512_clouds(torch_cuda):
    """512 clouds, N log-uniform in [1k, 64k], sphere/torus/ellipsoid, m=128,
    d=3, BF16: sampled clouds against the oracle."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    clouds = wl.uneven_batch()
    plans = [rfd.Plan(c.m, c.eps, c.lam, c.seed, precision="bf16") for c in clouds]
    Xs = [torch.from_numpy(c.X).cuda() for c in clouds]
    Fs = [torch.from_numpy(c.F).cuda() for c in clouds]
    outs = [torch.empty_like(F) for F in Fs]
    b = rfd.Batch(plans, Xs, Fs, outs)
    b.launch()
    torch.cuda.synchronize()
    assert all(p.check() == rfd.OK for p in plans)
    sizes = np.array([c.n for c in clouds])
    for i in (int(np.argmin(sizes)), int(np.argmax(sizes)), 100, 301):
        c = clouds[i]
        e = o.relf(outs[i].cpu().numpy(), o.rfd_integrate(c.X, c.F, c.eps, c.lam, c.m, c.seed))
        print(f"512-batch cloud {i} N={c.n}: relF={e:.3e}")
        assert e <= 2e-3
    b.close()


def test_batch_tune_keeps_results(torch_cuda):
    """Tuning the batched expansion geometry changes no bit of the outputs;
    the graph recorded after tuning replays the same results."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    rfd.tune_reset()
    clouds = wl.uneven_batch(count=40, seed=4)
    plans = [rfd.Plan(c.m, c.eps, c.lam, c.seed, precision="bf16") for c in clouds]
    Xs = [torch.from_numpy(c.X).cuda() for c in clouds]
    Fs = [torch.from_numpy(c.F).cuda() for c in clouds]
    outs = [torch.empty_like(F) for F in Fs]
    b = rfd.Batch(plans, Xs, Fs, outs)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b.launch(st)
    st.synchronize()
    ref = [o_.cpu().numpy() for o_ in outs]
    for o_ in outs:
        o_.fill_(float("nan"))
    torch.cuda.synchronize()
    tpi = b.tune(reps=2, stream=st)
    st.synchronize()
    print(f"tuned tiles per item: {tpi}")
    assert all(np.array_equal(r, o_.cpu().numpy()) for r, o_ in zip(ref, outs))
    for _ in range(3):  # record after tuning, then replays
        for o_ in outs:
            o_.fill_(float("nan"))
        torch.cuda.synchronize()
        with torch.cuda.stream(st):
            b.launch(st)
        st.synchronize()
        assert all(np.array_equal(r, o_.cpu().numpy()) for r, o_ in zip(ref, outs))
    b.close()
    rfd.tune_reset()


def test_batch_mixed_widths_bitwise_equal_alone(torch_cuda):
    """A batch whose fields straddle the action-form width (<= 32 channels:
    phi_1 applied to the field block; wider: S and G = S H) takes, cloud by
    cloud, the same path as the one-shot entry point: bitwise equal alone."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    clouds = _clouds(5, 3, 128, 21)
    widths = [3, 40, 32, 33, 1]
    Fs_np = [wl.field(c.n, dd, 200 + i) for i, (c, dd) in enumerate(zip(clouds, widths))]
    for prec in ("fp32", "bf16"):
        plans = [rfd.Plan(c.m, c.eps, c.lam, c.seed, precision=prec) for c in clouds]
        Xs = [torch.from_numpy(c.X).cuda() for c in clouds]
        Fs = [torch.from_numpy(F).cuda() for F in Fs_np]
        outs = [torch.empty_like(F) for F in Fs]
        rfd.Batch(plans, Xs, Fs, outs).launch()
        torch.cuda.synchronize()
        for c, X, F, out in zip(clouds, Xs, Fs, outs):
            alone = rfd.Plan(c.m, c.eps, c.lam, c.seed, precision=prec).oneshot(X, F)
            assert np.array_equal(alone.cpu().numpy(), out.cpu().numpy()), (prec, F.shape[1])
        # resident use after the batch forms S where the batch did not
        F2 = torch.from_numpy(wl.field(clouds[0].n, 4, 9)).cuda()
        fresh = rfd.Plan(clouds[0].m, clouds[0].eps, clouds[0].lam, clouds[0].seed, precision=prec)
        fresh.features(Xs[0])
        assert np.array_equal(plans[0].integrate(F2).cpu().numpy(), fresh.integrate(F2).cpu().numpy())


@pytest.mark.parametrize("m", [64, 256])
def test_batch_schedules_bitwise_equal_alone(torch_cuda, m):
    """The per-cloud phi_1 kernel stages its tiles differently by m (one K
    block per tile, streamed, for m <= 128; 32-wide pipelined blocks at
    m = 256) and the single-cloud kernel differently again (128-wide blocks);
    the products are summed in one fixed order, so every cloud of a batch
    equals its one-shot result bitwise, in action form (d <= 32) and with
    the full core (d > 32; a batch at m = 256 takes fields of at most 32
    channels, the width of its fused first pass)."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    clouds = _clouds(6, 3, m, 41, lo=1500, hi=12000)
    widths = [3, 40, 16, 33, 1, 64] if m <= 128 else [3, 32, 16, 20, 1, 31]
    Fs_np = [wl.field(c.n, dd, 300 + i) for i, (c, dd) in enumerate(zip(clouds, widths))]
    for prec in ("fp32", "bf16"):
        plans = [rfd.Plan(c.m, c.eps, c.lam, c.seed, precision=prec) for c in clouds]
        Xs = [torch.from_numpy(c.X).cuda() for c in clouds]
        Fs = [torch.from_numpy(F).cuda() for F in Fs_np]
        outs = [torch.empty_like(F) for F in Fs]
        rfd.Batch(plans, Xs, Fs, outs).launch()
        torch.cuda.synchronize()
        assert all(p.check() == rfd.OK for p in plans)
        for c, X, F, out in zip(clouds, Xs, Fs, outs):
            alone = rfd.Plan(c.m, c.eps, c.lam, c.seed, precision=prec).oneshot(X, F)
            assert np.array_equal(alone.cpu().numpy(), out.cpu().numpy()), (m, prec, F.shape[1])
        c, F = clouds[1], Fs_np[1]
        e = o.relf(outs[1].cpu().numpy(), o.rfd_integrate(c.X, F, c.eps, c.lam, c.m, c.seed))
        assert e <= {"fp32": 1e-5, "bf16": 2e-3}[prec], e


@pytest.mark.parametrize("d", [16, 32, 64])
def test_batch_in_place_equals_per_cloud(torch_cuda, d):
    """out may be F itself. Each cloud spans several expansion work items (64
    tiles of 16 points each) and ends in a ragged tile; a tile handled by two
    work items would, in place, carry the correction twice. Full 16-channel
    blocks (d = 16, 32, 64) take the expansion's interior-tile loop."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    clouds = _clouds(6, d, 128, 11, lo=3000, hi=9000)
    assert all(c.n % 16 for c in clouds) and all(c.n > 2 * 64 * 16 for c in clouds)
    plans = [rfd.Plan(c.m, c.eps, c.lam, c.seed, precision="bf16") for c in clouds]
    Xs = [torch.from_numpy(c.X).cuda() for c in clouds]
    Fs = [torch.from_numpy(c.F).cuda() for c in clouds]
    b = rfd.Batch(plans, Xs, Fs, Fs)
    b.launch()
    torch.cuda.synchronize()
    for p in plans:
        assert p.check() == rfd.OK
    for i, c in enumerate(clouds):
        got = Fs[i].cpu().numpy()
        ref = _single(torch, c, "bf16")
        assert np.array_equal(got, ref), (i, c.n, np.abs(got - ref).max())
    b.close()
