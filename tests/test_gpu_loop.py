"""GPU parity of repeated application: the row-scaled integrate and the
alternating loop v <- s_k . exp(lambda_k A_k B_k^T) v (App. D, Alg. 1 shape)
against the CPU FP64 oracle, and the hipGraph replay of the loop against its
eager launch (bitwise)."""
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


def make_plans(torch, clouds, prec):
    from paper_2302_00942_amd import rfd
    plans = []
    for c in clouds:
        p = rfd.Plan(c.m, c.eps, c.lam, c.seed, precision=prec)
        p.features(torch.from_numpy(c.X).cuda())
        plans.append(p)
    assert all(p.check() == rfd.OK for p in plans)
    return plans


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_integrate_scaled_matches_oracle(torch_cuda, prec):
    torch = torch_cuda
    c = wl.plain_sphere(n=6001, d=7, m=128, seed=3)
    s0, _ = wl.scaling_vectors(c.n, 5)
    plan = make_plans(torch, [c], prec)[0]
    out = plan.integrate_scaled(torch.from_numpy(c.F).cuda(), torch.from_numpy(s0).cuda()).cpu().numpy()
    ref = s0.astype(np.float64)[:, None] * o.rfd_integrate(c.X, c.F, c.eps, c.lam, c.m, c.seed)
    e = o.relf(out, ref)
    print(f"scaled integrate {prec}: relF={e:.3e}")
    assert e <= TOL[prec]
    # scale = None is the plain integrate, bitwise
    a = plan.integrate_scaled(torch.from_numpy(c.F).cuda(), None).cpu().numpy()
    b = plan.integrate(torch.from_numpy(c.F).cuda()).cpu().numpy()
    assert np.array_equal(a, b)


def loop_reference(clouds, v0, scales, iters, plans):
    oms, ws = zip(*[p.export() for p in plans])
    return o.repeated_apply([c.X for c in clouds], v0, scales, [c.lam for c in clouds], iters, oms, ws)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("d", [1, 32])
def test_loop_graph_replay_and_oracle(torch_cuda, prec, d):
    """Small pair of clouds, 12 iterations: eager launch vs graph replay
    bitwise, and the result vs the oracle's loop, held to the one-result bar:
    the diffusion operators are contractions for lambda <= 0, so errors of
    earlier steps are damped rather than compounded."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    clouds = wl.sinkhorn_pair(n=5000, d=d, m=128, seed=7)
    s0, s1 = wl.scaling_vectors(5000, 9)
    plans = make_plans(torch, clouds, prec)
    v0 = torch.from_numpy(clouds[0].F).cuda()
    v = v0.clone()
    sd = [torch.from_numpy(s0).cuda(), torch.from_numpy(s1).cuda()]
    iters = 12
    loop = rfd.Loop(plans, sd, v, iters)
    st = torch.cuda.Stream()
    results = []
    junk = torch.randn(1 << 20, device="cuda")
    for it in range(4):  # eager, capture + replay, replay, replay
        with torch.cuda.stream(st):
            v.copy_(v0)
            loop.launch(st)
        st.synchronize()
        results.append(v.cpu().numpy())
        junk.mul_(1.0001)  # unrelated device work between replays
        torch.cuda.synchronize()
    for r in results[1:]:
        assert np.array_equal(r, results[0])
    ref = loop_reference(clouds, clouds[0].F, (s0, s1), iters, plans)
    e = o.relf(results[0], ref)
    print(f"loop d={d} {prec} x{iters}: relF={e:.3e}")
    assert e <= TOL[prec]
    assert all(p.check() == rfd.OK for p in plans)
    loop.close()


def test_loop_equals_stepwise_integrate(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    clouds = wl.sinkhorn_pair(n=3000, d=5, m=64, seed=1)
    s0, s1 = wl.scaling_vectors(3000, 2)
    plans = make_plans(torch, clouds, "bf16")
    sd = [torch.from_numpy(s0).cuda(), torch.from_numpy(s1).cuda()]
    v = torch.from_numpy(clouds[0].F).cuda()
    w = v.clone()
    rfd.Loop(plans, sd, v, 5).launch()
    for t in range(5):
        plans[t % 2].integrate_scaled(w, sd[t % 2], out=w)
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), w.cpu().numpy())


def test_loop_argument_errors(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    a = rfd.Plan(64, 0.1, -0.5, 0)
    b = rfd.Plan(64, 0.1, -0.5, 1)
    v = torch.zeros((100, 2), device="cuda")
    with pytest.raises(rfd.RfdError) as e:
        rfd.Loop([a], None, v, 3)  # features not computed
    assert e.value.status == rfd.NOT_READY
    a.features(torch.from_numpy(wl.sphere(100, 0)).cuda())
    b.features(torch.from_numpy(wl.sphere(120, 1)).cuda())
    with pytest.raises(ValueError):
        rfd.Loop([a, b], None, v, 3)  # unequal cloud sizes: v cannot match both
    with pytest.raises(rfd.RfdError) as e:
        rfd.Loop([a], None, v, 0)
    assert e.value.status == rfd.INVALID_ARG


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_repeated_application_full_size(torch_cuda, prec):
    """The repeated-application workload at its full size: sphere and deformed
    torus of 100,000 points, m = 128, 100 alternating iterations, d = 32,
    graph-replayed, against the oracle's loop."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    n, iters = 100_000, 100
    clouds = wl.sinkhorn_pair(n=n, d=32, m=128, seed=0)
    s0, s1 = wl.scaling_vectors(n, 1)
    plans = make_plans(torch, clouds, prec)
    v0 = torch.from_numpy(clouds[0].F).cuda()
    v = v0.clone()
    sd = [torch.from_numpy(s0).cuda(), torch.from_numpy(s1).cuda()]
    loop = rfd.Loop(plans, sd, v, iters)
    st = torch.cuda.Stream()
    outs = []
    for _ in range(3):
        with torch.cuda.stream(st):
            v.copy_(v0)
            loop.launch(st)
        st.synchronize()
        outs.append(v.cpu().numpy())
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])
    ref = loop_reference(clouds, clouds[0].F, (s0, s1), iters, plans)
    e = o.relf(outs[0], ref)
    print(f"repeated application N=1e5 d=32 {prec} x{iters}: relF={e:.3e}")
    assert e <= TOL[prec]
    loop.close()


def test_loop_after_same_size_action_form_oneshot(torch_cuda):
    """A one-shot call of at most 32 channels on a loop's plan, with a new
    cloud of the same size, applies phi_1 in action form and leaves S and T
    stale; the next loop launch forms them for the new cloud first, so the
    loop matches the oracle on the new cloud."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    n, iters = 3000, 6
    clouds = wl.sinkhorn_pair(n=n, d=4, m=64, seed=11)
    s0, s1 = wl.scaling_vectors(n, 12)
    plans = make_plans(torch, clouds, "fp32")
    sd = [torch.from_numpy(s0).cuda(), torch.from_numpy(s1).cuda()]
    v0 = torch.from_numpy(clouds[0].F).cuda()
    v = v0.clone()
    loop = rfd.Loop(plans, sd, v, iters)
    loop.launch()
    torch.cuda.synchronize()
    Xnew = wl.ellipsoid(n, 13)
    Fnew = torch.from_numpy(wl.field(n, 8, 14)).cuda()
    plans[0].oneshot(torch.from_numpy(Xnew).cuda(), Fnew)  # action form (8 <= 32 channels)
    v.copy_(v0)
    loop.launch()
    torch.cuda.synchronize()
    oms, ws = zip(*[p.export() for p in plans])
    ref = o.repeated_apply([Xnew, clouds[1].X], clouds[0].F, (s0, s1), [clouds[0].lam, clouds[1].lam], iters, oms,
                           ws)
    e = o.relf(v.cpu().numpy(), ref)
    print(f"loop after an action-form one-shot on a new cloud: relF={e:.3e}")
    assert e <= TOL["fp32"]
    assert all(p.check() == rfd.OK for p in plans)
    loop.close()


def test_loop_rows_must_match_the_clouds(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    a = rfd.Plan(64, 0.1, -0.5, 0)
    a.features(torch.from_numpy(wl.sphere(100, 0)).cuda())
    with pytest.raises(ValueError):
        rfd.Loop([a], None, torch.zeros((99, 2), device="cuda"), 3)
