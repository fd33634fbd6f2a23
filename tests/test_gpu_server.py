"""GPU tests of the serving loop: every request's result is the same alone and
in a mix of concurrent requests (bitwise: the split of each cloud depends only
on its own N), equals the standalone one-shot entry point, and meets the
oracle bars; resident features are reused; the HBM budget is respected by
eviction; per-request errors stay with their request."""
import threading

import numpy as np
import pytest

from oracle import rfd_oracle as o
from paper_2302_00942_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16": 2e-3}
GiB = 1 << 30


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2302_00942_amd import rfd
    rfd.lib()
    return torch


def request_set(count, seed, lo=2000, hi=60000):
    reqs = wl.poisson_requests(count, 1000.0, seed, lo=lo, hi=hi)
    out = []
    for i, q in enumerate(reqs):
        X = wl.surface(q["surface"], q["n"], q["seed"])
        F = wl.field(q["n"], q["d"], q["seed"] + 1)
        out.append(dict(X=X, F=F, m=q["m"], seed=q["seed"] % 1000, prec="bf16" if i % 2 else "fp32"))
    return out


def to_dev(torch, reqs):
    for q in reqs:
        q["Xd"] = torch.from_numpy(q["X"]).cuda()
        q["Fd"] = torch.from_numpy(q["F"]).cuda()
    return reqs


def run_server(torch, reqs, burst, budget=8 * GiB, inflight=8):
    from paper_2302_00942_amd import rfd
    srv = rfd.Server(budget, inflight)
    outs = [torch.full_like(q["Fd"], float("nan")) for q in reqs]
    stats = []
    if burst:
        tickets = [srv.submit(q["Xd"], q["Fd"], o_, q["m"], 0.05, -0.5, q["seed"], q["prec"])
                   for q, o_ in zip(reqs, outs)]
        res = [srv.wait(t) for t in tickets]
    else:
        res = []
        for q, o_ in zip(reqs, outs):
            t = srv.submit(q["Xd"], q["Fd"], o_, q["m"], 0.05, -0.5, q["seed"], q["prec"])
            res.append(srv.wait(t))
    stats.append(srv.stats())
    srv.close()
    return [x.cpu().numpy() for x in outs], res, stats


def test_alone_equals_mix_equals_oneshot(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    reqs = to_dev(torch, request_set(16, 3))
    alone, ra, _ = run_server(torch, reqs, burst=False)
    mix, rm, st = run_server(torch, reqs, burst=True)
    assert all(r[0] == rfd.OK for r in ra + rm)
    for i, q in enumerate(reqs):
        assert np.array_equal(alone[i], mix[i]), i
        plan = rfd.Plan(q["m"], 0.05, -0.5, q["seed"], precision=q["prec"])
        ref = plan.oneshot(q["Xd"], q["Fd"]).cpu().numpy()
        assert np.array_equal(ref, mix[i]), i
        plan.close()
    # overlap: in the burst, some request was admitted before an earlier one finished
    t_start = [r[2] for r in rm]
    t_done = [r[3] for r in rm]
    assert any(t_start[j] < t_done[j - 1] for j in range(1, len(rm)))
    for i in (0, 5, 11):  # oracle bar on a few requests
        q = reqs[i]
        ref = o.rfd_integrate(q["X"], q["F"], 0.05, -0.5, q["m"], q["seed"])
        e = o.relf(mix[i], ref)
        print(f"served request {i} N={len(q['X'])} d={q['F'].shape[1]} m={q['m']} {q['prec']}: relF={e:.3e}")
        assert e <= TOL[q["prec"]]


def test_resident_features_are_reused(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    c = wl.plain_sphere(n=30000, d=16, m=128, seed=1)
    X = torch.from_numpy(c.X).cuda()
    F1 = torch.from_numpy(c.F).cuda()
    F2 = torch.from_numpy(wl.field(c.n, 16, 99)).cuda()
    srv = rfd.Server(4 * GiB, 4)
    o1, o2 = torch.empty_like(F1), torch.empty_like(F2)
    t1 = srv.submit(X, F1, o1, c.m, c.eps, c.lam, c.seed, "bf16", cloud_key=42)
    t2 = srv.submit(X, F2, o2, c.m, c.eps, c.lam, c.seed, "bf16", cloud_key=42)
    assert srv.wait(t1)[0] == rfd.OK and srv.wait(t2)[0] == rfd.OK
    assert srv.stats()["plans"] == 1
    plan = rfd.Plan(c.m, c.eps, c.lam, c.seed, precision="bf16")
    assert np.array_equal(plan.oneshot(X, F1).cpu().numpy(), o1.cpu().numpy())  # first request: one-shot
    res = rfd.Plan(c.m, c.eps, c.lam, c.seed, precision="bf16")
    res.features(X)
    assert np.array_equal(res.integrate(F2).cpu().numpy(), o2.cpu().numpy())  # resident: integrate only
    # another cloud without a key gets its own plan while the budget allows
    # (the resident features of cloud 42 are kept) ...
    Y = torch.from_numpy(wl.torus(20000, 5)).cuda()
    G = torch.from_numpy(wl.field(20000, 3, 6)).cuda()
    o3 = torch.empty_like(G)
    assert srv.wait(srv.submit(Y, G, o3, c.m, c.eps, c.lam, c.seed, "bf16"))[0] == rfd.OK
    assert srv.stats()["plans"] == 2
    assert np.array_equal(plan.oneshot(Y, G).cpu().numpy(), o3.cpu().numpy())
    # ... and a further keyless cloud reuses that idle keyless plan's buffers
    Z = torch.from_numpy(wl.ellipsoid(15000, 7)).cuda()
    H = torch.from_numpy(wl.field(15000, 5, 8)).cuda()
    o4 = torch.empty_like(H)
    assert srv.wait(srv.submit(Z, H, o4, c.m, c.eps, c.lam, c.seed, "bf16"))[0] == rfd.OK
    assert srv.stats()["plans"] == 2
    assert np.array_equal(plan.oneshot(Z, H).cpu().numpy(), o4.cpu().numpy())
    # cloud 42 is still resident: a third field on it runs the integrate passes only
    o5 = torch.empty_like(F1)
    assert srv.wait(srv.submit(X, F1, o5, c.m, c.eps, c.lam, c.seed, "bf16", cloud_key=42))[0] == rfd.OK
    assert srv.stats()["plans"] == 2
    assert np.array_equal(res.integrate(F1).cpu().numpy(), o5.cpu().numpy())
    srv.close()


def test_budget_eviction_and_out_of_budget(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    reqs = to_dev(torch, request_set(10, 11, lo=2000, hi=20000))
    for q in reqs:
        q["m"] = 256  # large fixed plan footprint (about 15 MB each)
    budget = 48 << 20  # room for about three such plans
    srv = rfd.Server(budget, 4)
    outs = [torch.empty_like(q["Fd"]) for q in reqs]
    tickets = [srv.submit(q["Xd"], q["Fd"], o_, 256, 0.05, -0.5, 1000 + i, q["prec"])
               for i, (q, o_) in enumerate(zip(reqs, outs))]
    assert all(srv.wait(t)[0] == rfd.OK for t in tickets)
    st = srv.stats()
    assert st["device_bytes"] <= budget and st["plans"] <= 3, st
    for i in (0, 9):
        q = reqs[i]
        plan = rfd.Plan(256, 0.05, -0.5, 1000 + i, precision=q["prec"])
        assert np.array_equal(plan.oneshot(q["Xd"], q["Fd"]).cpu().numpy(), outs[i].cpu().numpy())
    big = torch.zeros((3_000_000, 3), device="cuda")
    with pytest.raises(rfd.RfdError) as e:
        srv.submit(big, big, torch.empty_like(big), 256, 0.05, -0.5)
    assert e.value.status == rfd.OUT_OF_BUDGET
    srv.close()


def test_errors_stay_with_their_request(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    c = wl.plain_sphere(n=5000, d=4, m=64, seed=2)
    X = torch.from_numpy(c.X).cuda()
    F = torch.from_numpy(c.F).cuda()
    Fbad = F.clone()
    Fbad[123, 2] = float("nan")
    srv = rfd.Server(GiB, 4)
    outs = [torch.empty_like(F) for _ in range(3)]
    t_bad = srv.submit(X, Fbad, outs[0], 64, c.eps, c.lam, c.seed)
    t_range = srv.submit(X, F, outs[1], 64, c.eps, 5.0, c.seed)  # growing kernel beyond the FP64 range
    t_ok = srv.submit(X, F, outs[2], 64, c.eps, c.lam, c.seed)
    assert srv.wait(t_bad)[0] == rfd.NONFINITE
    assert srv.wait(t_range)[0] == rfd.RANGE
    assert srv.wait(t_ok)[0] == rfd.OK
    plan = rfd.Plan(64, c.eps, c.lam, c.seed)
    assert np.array_equal(plan.oneshot(X, F).cpu().numpy(), outs[2].cpu().numpy())
    with pytest.raises(rfd.RfdError):
        srv.wait(t_ok)  # already collected
    # a zero timeout on fresh large work reports NOT_READY or the result; the ticket stays valid
    Y = torch.from_numpy(wl.torus(200000, 1)).cuda()
    G = torch.from_numpy(wl.field(200000, 64, 2)).cuda()
    oy = torch.empty_like(G)
    t = srv.submit(Y, G, oy, 256, 0.05, -0.5, 3)
    first = srv.wait(t, 0.0)[0]
    assert first in (rfd.NOT_READY, rfd.OK)
    if first == rfd.NOT_READY:
        assert srv.wait(t)[0] == rfd.OK
    srv.close()


def test_concurrent_submitters(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    reqs = to_dev(torch, request_set(12, 21, lo=2000, hi=30000))
    ref, _, _ = run_server(torch, reqs, burst=False)
    srv = rfd.Server(8 * GiB, 8)
    outs = [torch.full_like(q["Fd"], float("nan")) for q in reqs]
    torch.cuda.synchronize()
    status = [None] * len(reqs)

    def client(k):
        for i in range(k, len(reqs), 4):
            q = reqs[i]
            t = srv.submit(q["Xd"], q["Fd"], outs[i], q["m"], 0.05, -0.5, q["seed"], q["prec"])
            status[i] = srv.wait(t)[0]

    th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    assert all(s == rfd.OK for s in status)
    for i in range(len(reqs)):
        assert np.array_equal(ref[i], outs[i].cpu().numpy()), i
    srv.close()
