"""CPU checks of the C ABI: the library loads, exports every declared symbol,
rejects bad parameters, and its host-side sampler and weights agree with the
oracle's independent implementation. No compute call needs a GPU here."""
import ctypes as C

import numpy as np
import pytest

from oracle import rfd_oracle as o
from paper_2302_00942_amd import rfd


def test_library_exports_every_declared_symbol():
    L = rfd.lib()
    names = rfd.declared_symbols()
    assert "rfd_plan_create" in names and "rfd_submit" in names and len(names) >= 15
    for n in names:
        assert hasattr(L, n), n


@pytest.mark.parametrize("m,eps,seed", [(64, 0.1, 0), (256, 0.02, 0), (128, 0.05, 12345), (30, 0.01, 7)])
def test_sampler_matches_oracle_bitwise(m, eps, seed):
    om, w = rfd.frequencies(m, eps, seed)
    om_ref, w_ref = o.frequencies_and_weights(m, eps, seed)
    assert om.dtype == np.float32 and np.array_equal(om, om_ref)
    assert np.allclose(w, w_ref, rtol=1e-12, atol=0)


def test_box_sampler_and_weights_match_oracle():
    om, w = rfd.frequencies(64, 0.05, 3, shape="box")
    om_ref, w_ref = o.frequencies_and_weights(64, 0.05, 3, shape=o.BOX_LINF)
    assert np.array_equal(om, om_ref)
    assert np.allclose(w, w_ref, rtol=1e-12, atol=0)


def test_custom_sigma_radius_signed_weights_match_oracle():
    om, w = rfd.frequencies(64, 0.1, 5, sigma=10.0, radius=30.0)
    om_ref, w_ref = o.frequencies_and_weights(64, 0.1, 5, sigma=10.0, radius=30.0)
    assert np.array_equal(om, om_ref)
    assert np.any(w < 0)
    assert np.allclose(w, w_ref, rtol=1e-11, atol=1e-14 * np.abs(w_ref).max())


@pytest.mark.parametrize("D", [1, 2, 4, 5, 8, 17, 64])
@pytest.mark.parametrize("shape", ["ball", "box"])
def test_sampler_in_d_dimensions_matches_oracle(D, shape):
    """Points in D dimensions: the host sampler draws the oracle's frequencies
    bit for bit (D normals per candidate, the squared norm summed in order, its
    own first Bessel zero for the preset radius) and its weights (its own
    Bessel function and incomplete gamma) agree to rounding."""
    sh = o.BALL_L2 if shape == "ball" else o.BOX_LINF
    om, w = rfd.frequencies(96, 0.2, 21, shape=shape, dim=D)
    om_ref, w_ref = o.frequencies_and_weights(96, 0.2, 21, sh, dim=D)
    assert om.shape == (48, D) and np.array_equal(om, om_ref)
    assert np.all(w_ref > 0)  # the preset keeps every weight positive
    assert np.allclose(w, w_ref, rtol=1e-11, atol=0)
    # explicit law reaching past the main lobe (signed weights), scaled with D
    R = 2.5 * o.preset(0.2, sh, dim=D)[1]
    sig = R / np.sqrt(D + 6.0)
    om, w = rfd.frequencies(64, 0.2, 4, shape=shape, sigma=sig, radius=R, dim=D)
    om_ref, w_ref = o.frequencies_and_weights(64, 0.2, 4, sh, sigma=sig, radius=R, dim=D)
    assert np.array_equal(om, om_ref)
    assert np.allclose(w, w_ref, rtol=1e-9, atol=1e-12 * np.abs(w_ref).max())


def test_sampler_refuses_a_law_that_accepts_nothing():
    """A truncation that keeps almost no mass (64-D Gaussian cut at 3 sigma):
    both samplers give up instead of looping."""
    p, _ = rfd.make_params(32, 0.2, -0.5, 1, sigma=4.0, radius=12.0, dim=64)
    om = np.zeros((16, 64), dtype=np.float32)
    w = np.zeros(16)
    assert rfd.lib().rfd_params_frequencies(C.byref(p), om.ctypes.data, w.ctypes.data) == rfd.INVALID_ARG


def test_dim_zero_means_three_and_bad_dims_are_rejected():
    om0, w0 = rfd.frequencies(32, 0.1, 2, dim=0)
    om3, w3 = rfd.frequencies(32, 0.1, 2, dim=3)
    assert np.array_equal(om0, om3) and np.array_equal(w0, w3)
    for D in (-1, 65, 1000):
        p, _ = rfd.make_params(32, 0.1, -0.5, 2, dim=D)
        om = np.zeros((16, 1000), dtype=np.float32)
        w = np.zeros(16)
        assert rfd.lib().rfd_params_frequencies(C.byref(p), om.ctypes.data, w.ctypes.data) == rfd.INVALID_ARG


@pytest.mark.parametrize("kw", [dict(m=63), dict(m=0), dict(m=258), dict(eps=0.0), dict(eps=-1.0),
                                dict(lam=float("nan")), dict(sigma=1.0), dict(radius=2.0), dict(shape=5),
                                dict(precision=7)])
def test_invalid_params_are_rejected_before_any_device_work(kw):
    base = dict(m=64, eps=0.1, lam=-0.5, seed=0, shape="ball", precision="fp32", sigma=0.0, radius=0.0)
    base.update(kw)
    p, _ = rfd.make_params(base["m"], base["eps"], base["lam"], base["seed"], "ball", "fp32",
                           base["sigma"], base["radius"])
    if "shape" in kw:
        p.shape = kw["shape"]
    if "precision" in kw:
        p.precision = kw["precision"]
    f = max(base["m"], 2) // 2 + 1
    om = np.zeros((f, 3), dtype=np.float32)
    w = np.zeros(f)
    assert rfd.lib().rfd_params_frequencies(C.byref(p), om.ctypes.data, w.ctypes.data) == rfd.INVALID_ARG
    h = C.c_void_p()
    assert rfd.lib().rfd_plan_create(C.byref(p), C.byref(h)) == rfd.INVALID_ARG
    assert not h.value


def test_null_arguments():
    L = rfd.lib()
    assert L.rfd_plan_create(None, None) == rfd.INVALID_ARG
    assert L.rfd_features(None, None, 0, None) == rfd.INVALID_ARG
    assert L.rfd_integrate(None, None, 0, 0, None, 0, None) == rfd.INVALID_ARG
    assert L.rfd_plan_check(None, None) == rfd.INVALID_ARG
    L.rfd_plan_destroy(None)
    assert rfd.status_string(rfd.NONFINITE).startswith("non-finite")


def test_server_loop_and_batch_argument_checks():
    """Argument checks that return before any device call."""
    L = rfd.lib()
    h = C.c_void_p()
    assert L.rfd_server_create(0, 4, C.byref(h)) == rfd.INVALID_ARG
    assert L.rfd_server_create(1 << 30, 0, C.byref(h)) == rfd.INVALID_ARG
    assert L.rfd_server_create(1 << 30, 65, C.byref(h)) == rfd.INVALID_ARG
    assert L.rfd_server_create(1 << 30, 4, None) == rfd.INVALID_ARG
    assert L.rfd_submit(None, None, None) == rfd.INVALID_ARG
    assert L.rfd_wait(None, 1, 0.0, None) == rfd.INVALID_ARG
    assert L.rfd_server_stats(None, None, None, None, None) == rfd.INVALID_ARG
    L.rfd_server_destroy(None)
    assert L.rfd_loop_create(None, None, 1, None, 1, 1, 1, C.byref(h)) == rfd.INVALID_ARG
    assert L.rfd_loop_launch(None, None) == rfd.INVALID_ARG
    L.rfd_loop_destroy(None)
    assert L.rfd_batch_create(None, None, None, None, None, None, None, None, 0, C.byref(h)) == rfd.INVALID_ARG
    assert L.rfd_batch_launch(None, None) == rfd.INVALID_ARG
    assert L.rfd_integrate_scaled(None, None, 0, 0, None, 0, None, None) == rfd.INVALID_ARG


def test_tuning_table_text_round_trip():
    """The launch-geometry table (host only): import validates the whole text,
    export lists the entries, reset clears them."""
    rfd.tune_reset()
    assert rfd.tune_export() == ""
    rfd.tune_import("0 256 1 1 20 8\n1 128 1 1 23 32\n")
    txt = rfd.tune_export()
    assert txt.splitlines() == ["0 256 1 1 20 8", "1 128 1 1 23 32"]
    for bad in ("0 256 1 1 20\n", "9 256 1 1 20 8\n", "0 100 1 1 20 8\n", "0 256 1 3 20 8\n",
                "0 256 1 1 20 0\n", "0 256 1 1 20 8\nxyz\n"):
        with pytest.raises(rfd.RfdError) as e:
            rfd.tune_import(bad)
        assert e.value.status == rfd.INVALID_ARG
    assert rfd.tune_export() == txt  # rejected imports change nothing
    rfd.tune_import(txt.replace(" 8\n", " 4\n"))
    assert rfd.tune_export().splitlines()[0] == "0 256 1 1 20 4"
    rfd.tune_reset()
    assert rfd.tune_export() == ""


def _taylor_theta(q: int, nmax: int = 120) -> float:
    """Largest theta with sum_n |h_n| theta^(n-1) <= 2^-53, where
    h(x) = log(e^{-x} T_q(x)) = sum_{n>q} h_n x^n is the backward-error series
    of the degree-q Taylor polynomial T_q of exp (exact rationals)."""
    import math
    from fractions import Fraction as Fr
    em = [Fr((-1) ** k, math.factorial(k)) for k in range(nmax + 1)]
    r = [sum(em[i] * Fr(1, math.factorial(n - i)) for i in range(n + 1) if n - i <= q) for n in range(nmax + 1)]
    r[0] -= 1  # r = e^{-x} T_q(x) - 1, starts at x^{q+1}
    h = [Fr(0)] * (nmax + 1)
    rp, k = r[:], 1
    while any(rp) and k <= nmax // (q + 1) + 1:  # log(1 + r) = r - r^2/2 + ...
        for n in range(nmax + 1):
            h[n] += Fr((-1) ** (k + 1), k) * rp[n]
        nxt = [Fr(0)] * (nmax + 1)
        for i, a in enumerate(rp):
            if a:
                for j in range(nmax + 1 - i):
                    if r[j]:
                        nxt[i + j] += a * r[j]
        rp, k = nxt, k + 1
    ht = [abs(float(v)) for v in h]
    f = lambda th: sum(c * th ** n for n, c in enumerate(ht)) / th
    lo, hi = 1e-3, 20.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if f(mid) <= 2.0 ** -53 else (lo, mid)
    return lo


def test_taylor_scaling_threshold():
    """The phi_1 kernel picks s from ||lambda M||_1 / theta_23 with
    theta_23 = 2.014710780944616 (its degree-23 Taylor evaluation). Pinned by
    recomputing the threshold from the backward-error series, and the method
    itself by reproducing the published degree-18 value theta_18 = 1.09
    (Al-Mohy & Higham's Taylor thresholds for double precision)."""
    assert abs(_taylor_theta(23) - 2.014710780944616) < 1e-9
    assert abs(_taylor_theta(18) - 1.09) < 5e-3


def test_plan_row_check_runs_on_the_host():
    """Plan._rows refuses F and out whose row count differs from the plan's
    cloud before anything reaches the library (host logic; no GPU)."""
    class FakePlan(rfd.Plan):
        points = 500

        def __init__(self):
            pass

    class T:
        def __init__(self, rows):
            self.shape = (rows, 3)

    p = FakePlan()
    p._rows(T(500), T(500))
    for F, out in ((T(499), T(499)), (T(500), T(499)), (T(501), T(501))):
        with pytest.raises(ValueError):
            p._rows(F, out)


def test_workspace_size_query_is_host_only_and_monotone():
    """rfd_plan_workspace_size needs no device: the bytes grow with the cloud
    and the field width, and invalid sizes are refused."""
    small = rfd.workspace_size(256, 0.02, 1000, 16)
    assert small > 0 and small % 256 == 0
    assert rfd.workspace_size(256, 0.02, 1_000_000, 16) > small
    assert rfd.workspace_size(256, 0.02, 1000, 64) >= small
    assert rfd.workspace_size(64, 0.02, 1000, 16) < small
    # the point copy alone is 12 bytes per point
    assert rfd.workspace_size(64, 0.1, 200_000, 3) - rfd.workspace_size(64, 0.1, 100_000, 3) >= 12 * 100_000
    for bad in ((-1, 16), (10, -1), (10, 1025)):
        with pytest.raises(rfd.RfdError):
            rfd.workspace_size(64, 0.1, *bad)
