"""GPU: points in D != 3 dimensions (the graph-classification appendix: node
features as points of R^D, the kernel's eigenvalues as the graph's signature).
The D-dimensional Gram pass (k_gram_nd) gives the core M = B^T A, and from it
the spectrum of exp(lambda A B^T), against the oracle's D-dimensional
features and kernel_spectrum.

Bars: M to the integrator's relative bar (FP32 1e-5, BF16 2e-3); each
eigenvalue to |lambda| max(1, max spectrum) ||M||_F times that bar (Weyl's
inequality, as for 3-D points). Entry points that apply the kernel to a field
refuse a D != 3 plan."""
import math

import numpy as np
import pytest

from oracle import rfd_oracle as o
from paper_2302_00942_amd import workloads as wl

pytestmark = pytest.mark.gpu

BAR = {"fp32": 1e-5, "bf16": 2e-3}
SHAPE = {"ball": o.BALL_L2, "box": o.BOX_LINF}


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2302_00942_amd import rfd
    rfd.lib()
    return torch


def _eps(D):
    return 0.15 * math.sqrt(2.0 * D)  # about the spread between a cluster's nodes


def _oracle_M(X, eps, m, seed, shape):
    om, w = o.frequencies_and_weights(m, eps, seed, SHAPE[shape], dim=X.shape[1])
    Phi, sg = o.features(X, om, w)
    return Phi.T @ (Phi * sg)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("D,m,n,shape", [(1, 64, 3001, "ball"), (2, 128, 2500, "ball"), (5, 64, 700, "box"),
                                         (7, 256, 300, "ball"), (16, 128, 1500, "ball"), (64, 64, 500, "ball"),
                                         (37, 250, 90, "box"), (4, 128, 64, "ball")])
def test_core_and_spectrum_match_oracle(torch_cuda, D, m, n, shape, prec):
    """Every padded feature count, N above, below and equal to the chunk
    size with ragged tails, ball and box, D from 1 to 64."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    X = wl.node_features(n, D, 10 + D)
    eps, lam = _eps(D), -0.3
    plan = rfd.Plan(m, eps, lam, 3, shape=shape, precision=prec, dim=D)
    om, w = plan.export()
    om_ref, w_ref = o.frequencies_and_weights(m, eps, 3, SHAPE[shape], dim=D)
    assert om.shape == (m // 2, D) and np.array_equal(om, om_ref)
    plan.features(torch.from_numpy(X).cuda(), sync=True)
    M, _, _ = plan.core()
    Mref = _oracle_M(X, eps, m, 3, shape)
    eM = o.relf(M, Mref)
    ref = o.kernel_spectrum(X, eps, lam, m, 3, SHAPE[shape])
    lo = plan.spectrum(n, "smallest").cpu().numpy()
    hi = plan.spectrum(min(n, 10), "largest").cpu().numpy()
    assert plan.check() == rfd.OK
    tol = abs(lam) * max(1.0, float(ref.max())) * float(np.linalg.norm(Mref)) * BAR[prec]
    err = max(np.abs(lo - ref).max(), np.abs(hi - ref[::-1][: len(hi)]).max())
    print(f"D={D} m={m} N={n} {shape} {prec}: relF(M)={eM:.2e} spectrum err {err:.2e} (bar {tol:.2e})")
    assert eM <= BAR[prec]
    assert err <= tol


def test_batch_spectrum_mixes_dimensions(torch_cuda):
    """One batched spectrum launch over plans of several dimensions and
    feature counts equals the single-plan calls bitwise."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    plans = []
    for i, (D, m, n) in enumerate([(3, 64, 200), (8, 128, 120), (1, 64, 90), (64, 256, 40), (20, 128, 300)]):
        p = rfd.Plan(m, _eps(D), -0.2, 7 + i, dim=D)
        X = wl.node_features(n, D, 40 + i) if D != 3 else wl.sphere(n, 40 + i)
        p.features(torch.from_numpy(X).cuda())
        plans.append((p, n))
    k = 8
    for which in ("smallest", "largest"):
        got = rfd.spectrum_batch([p for p, _ in plans], k, which)
        for (p, n), g in zip(plans, got):
            assert np.array_equal(g.cpu().numpy(), p.spectrum(k, which).cpu().numpy())


def test_graph_set_top_eigenvalues(torch_cuda):
    """A synthetic graph-classification set (node counts log-uniform in
    [10, 300], 16-dimensional node features): the 10 largest eigenvalues of
    each graph's kernel, in one batched launch, against the oracle."""
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    graphs = wl.graph_batch(48, 16, 3)
    eps, lam, m = _eps(16), -0.3, 64
    plans = []
    for i, X in enumerate(graphs):
        p = rfd.Plan(m, eps, lam, 100 + i, dim=16)
        p.features(torch.from_numpy(X).cuda())
        plans.append(p)
    k = 10
    got = rfd.spectrum_batch(plans, k, "largest")
    for i, (X, g) in enumerate(zip(graphs, got)):
        ref = o.kernel_spectrum(X, eps, lam, m, 100 + i)[::-1][:k]
        kk = min(k, X.shape[0])
        tol = abs(lam) * max(1.0, float(ref.max())) * float(np.linalg.norm(_oracle_M(X, eps, m, 100 + i, "ball"))) * 1e-5
        assert np.abs(g.cpu().numpy()[:kk] - ref[:kk]).max() <= tol, i


def test_field_entry_points_refuse_other_dimensions(torch_cuda):
    torch = torch_cuda
    from paper_2302_00942_amd import rfd
    X5 = torch.from_numpy(wl.node_features(500, 5, 1)).cuda()
    X3 = torch.from_numpy(wl.sphere(500, 1)).cuda()
    F = torch.from_numpy(wl.field(500, 3, 1)).cuda()
    plan = rfd.Plan(64, _eps(5), -0.3, 1, dim=5)
    plan.features(X5)
    out = torch.empty_like(F)
    with pytest.raises(rfd.RfdError) as e:
        plan.integrate(F)
    assert e.value.status == rfd.INVALID_ARG
    with pytest.raises(rfd.RfdError) as e:
        plan.oneshot(X3, F)
    assert e.value.status == rfd.INVALID_ARG
    with pytest.raises(rfd.RfdError) as e:
        plan.autotune(F, out, reps=1)
    assert e.value.status == rfd.INVALID_ARG
    with pytest.raises(rfd.RfdError) as e:
        rfd.Batch([plan], [X3], [F], [out]).launch()
    assert e.value.status == rfd.INVALID_ARG
    with pytest.raises(ValueError):
        plan.features(X3)  # three columns for a 5-dimensional plan
    assert plan.check() == rfd.OK
