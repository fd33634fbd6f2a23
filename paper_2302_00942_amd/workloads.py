"""Seeded synthetic inputs: point clouds on surfaces and random fields.

The paper evaluates RFD on mesh vertex clouds (Thingi10K meshes of a few
thousand to 1.5M vertices, vertex normals and velocities with d=3, Sec. 3 and
App. C; distributions with d=1 for the Wasserstein experiments, App. D). Those
meshes are not available, so these generators stand in for them: points drawn
area-uniformly on a sphere, a torus, an ellipsoid and a deformed torus, plus
i.i.d. N(0,1) fields. Everything is drawn with numpy's PCG64 generator from a
stated seed, in float64, and cast once to float32.

This module holds no arithmetic of the integrator itself. Both the GPU path
(through the tests and the benchmark) and the CPU oracle read their inputs
from here.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field as _dc_field

import numpy as np

SURFACES = ("sphere", "torus", "ellipsoid")


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def sphere(n: int, seed: int, radius: float = 1.0) -> np.ndarray:
    """Uniform on the sphere: normalised N(0, I3) draws."""
    g = _rng(seed)
    p = g.standard_normal((n, 3))
    nrm = np.linalg.norm(p, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    return (radius * p / nrm).astype(np.float32)


def torus(n: int, seed: int, R: float = 1.0, r: float = 0.3, jitter: float = 0.0,
          deform: bool = False) -> np.ndarray:
    """Area-uniform on the torus by rejection on the angle v.

    The area element of the torus is r (R + r cos v) du dv, so (u, v) uniform
    is accepted with probability (R + r cos v) / (R + r). With ``deform`` the
    tube radius becomes r (1 + 0.25 sin 3u) and z is lifted by 0.2 sin 2u (the
    sampling density is that of the undeformed torus). ``jitter`` adds
    N(0, jitter^2) noise to each coordinate.
    """
    g = _rng(seed)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        k = max(2 * (n - out.shape[0]), 1024)
        u = g.uniform(0.0, 2 * math.pi, k)
        v = g.uniform(0.0, 2 * math.pi, k)
        acc = g.uniform(0.0, 1.0, k) < (R + r * np.cos(v)) / (R + r)
        u, v = u[acc], v[acc]
        rr = r * (1.0 + 0.25 * np.sin(3 * u)) if deform else r
        x = (R + rr * np.cos(v)) * np.cos(u)
        y = (R + rr * np.cos(v)) * np.sin(u)
        z = rr * np.sin(v) + (0.2 * np.sin(2 * u) if deform else 0.0)
        out = np.concatenate([out, np.stack([x, y, z], axis=1)])
    out = out[:n]
    if jitter > 0:
        out = out + g.normal(0.0, jitter, out.shape)
    return out.astype(np.float32)


def ellipsoid(n: int, seed: int, axes=(1.0, 0.6, 0.3)) -> np.ndarray:
    """Area-uniform on the ellipsoid with semi-axes a >= b >= c.

    Points p uniform on the unit sphere map to (a px, b py, c pz); the area
    stretch of that map is sqrt((bc px)^2 + (ac py)^2 + (ab pz)^2), whose
    maximum is ab, so p is accepted with probability stretch / (ab).
    """
    a, b, c = axes
    g = _rng(seed)
    out = np.empty((0, 3))
    while out.shape[0] < n:
        k = max(2 * (n - out.shape[0]), 1024)
        p = g.standard_normal((k, 3))
        p /= np.linalg.norm(p, axis=1, keepdims=True)
        stretch = np.sqrt((b * c * p[:, 0]) ** 2 + (a * c * p[:, 1]) ** 2 + (a * b * p[:, 2]) ** 2)
        acc = g.uniform(0.0, 1.0, k) < stretch / (a * b)
        q = p[acc] * np.array([a, b, c])
        out = np.concatenate([out, q])
    return out[:n].astype(np.float32)


def surface(kind: str, n: int, seed: int) -> np.ndarray:
    if kind == "sphere":
        return sphere(n, seed)
    if kind == "torus":
        return torus(n, seed)
    if kind == "ellipsoid":
        return ellipsoid(n, seed)
    if kind == "deformed_torus":
        return torus(n, seed, deform=True)
    raise ValueError(f"unknown surface {kind!r}")


def field(n: int, d: int, seed: int) -> np.ndarray:
    """F in R^{n x d}, i.i.d. N(0, 1), drawn in float64 and cast to float32."""
    return _rng(seed).standard_normal((n, d)).astype(np.float32)


@dataclass
class Cloud:
    """One integration problem: points X (n x 3), field F (n x d) and the
    integrator's parameters."""
    X: np.ndarray
    F: np.ndarray
    eps: float
    lam: float
    m: int
    seed: int
    surface: str = ""
    extra: dict = _dc_field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.X.shape[0])

    @property
    def d(self) -> int:
        return int(self.F.shape[1])


def plain_sphere(n: int = 2000, d: int = 3, m: int = 64, seed: int = 0) -> Cloud:
    """N points uniform on the unit sphere, eps=0.1, lambda=-0.5, m=64, d=3."""
    return Cloud(sphere(n, seed), field(n, d, seed + 1), eps=0.1, lam=-0.5, m=m, seed=seed,
                 surface="sphere")


def large_torus(n: int = 1_000_000, d: int = 16, m: int = 256, seed: int = 0) -> Cloud:
    """One large cloud: torus R=1, r=0.3 plus N(0, 0.01^2) jitter; eps=0.02,
    lambda=-1, m=256, d=16."""
    return Cloud(torus(n, seed, jitter=0.01), field(n, d, seed + 1), eps=0.02, lam=-1.0, m=m,
                 seed=seed, surface="torus")


def batch_sizes(count: int = 512, lo: int = 1000, hi: int = 65536, seed: int = 0) -> np.ndarray:
    """Cloud sizes N = floor(exp(U(ln lo, ln hi)))."""
    g = _rng(seed)
    return np.floor(np.exp(g.uniform(math.log(lo), math.log(hi), count))).astype(np.int64)


def uneven_batch(count: int = 512, d: int = 3, m: int = 128, seed: int = 0,
                 lo: int = 1000, hi: int = 65536) -> list[Cloud]:
    """Many clouds of log-uniform size on sphere / torus / ellipsoid by index
    mod 3; eps=0.05, lambda=-0.5, m=128, d=3."""
    sizes = batch_sizes(count, lo, hi, seed)
    out = []
    for i, n in enumerate(sizes):
        kind = SURFACES[i % 3]
        s = seed * 100003 + 17 * i + 1
        out.append(Cloud(surface(kind, int(n), s), field(int(n), d, s + 7), eps=0.05, lam=-0.5,
                         m=m, seed=s, surface=kind))
    return out


def sinkhorn_pair(n: int = 100_000, d: int = 1, m: int = 128, seed: int = 0) -> list[Cloud]:
    """Two clouds for repeated application: a sphere and a deformed torus of n
    points each, eps=0.05, lambda=-0.5, m=128; F holds d start vectors."""
    return [
        Cloud(sphere(n, seed), field(n, d, seed + 1), eps=0.05, lam=-0.5, m=m, seed=seed,
              surface="sphere"),
        Cloud(torus(n, seed + 2, deform=True), field(n, d, seed + 3), eps=0.05, lam=-0.5, m=m,
              seed=seed + 2, surface="deformed_torus"),
    ]


def scaling_vectors(n: int, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Two positive scaling vectors s0, s1 ~ U[0.9, 1.1] for the alternating
    repeated-application loop."""
    g = _rng(seed)
    return (g.uniform(0.9, 1.1, n).astype(np.float32), g.uniform(0.9, 1.1, n).astype(np.float32))


def box_cloud(n: int, seed: int) -> np.ndarray:
    """Uniform in the unit cube: a random 3-D distribution of the kind the
    Gromov-Wasserstein experiments (App. "Ablation Studies for Gromov
    Wasserstein experiments") run on."""
    return _rng(seed).uniform(0.0, 1.0, (n, 3)).astype(np.float32)


def coupling(n: int, m: int, seed: int) -> np.ndarray:
    """A dense positive coupling T (n x m) with total mass 1: the product of
    two random marginals, each entry perturbed by a factor U[0.5, 1.5]."""
    g = _rng(seed)
    a = g.uniform(0.5, 1.5, n)
    b = g.uniform(0.5, 1.5, m)
    T = np.outer(a, b) * g.uniform(0.5, 1.5, (n, m))
    return (T / T.sum()).astype(np.float32)


def gw_pair(n: int = 3000, m: int = 3000, seed: int = 0, feats: int = 16):
    """Source and target clouds of a Gromov-Wasserstein problem (uniform in the
    unit cube and on a sphere of radius 0.5 about the cube's centre) with the
    RFD parameters of the paper's GW experiments (m = 16 features, eps = 0.3,
    lambda = -0.2) and a dense coupling T (n x m). The clouds carry no field."""
    Xc = box_cloud(n, seed)
    Xd = (0.5 + sphere(m, seed + 1, radius=0.5)).astype(np.float32)
    c = Cloud(Xc, np.zeros((n, 0), np.float32), eps=0.3, lam=-0.2, m=feats, seed=seed, surface="box")
    d = Cloud(Xd, np.zeros((m, 0), np.float32), eps=0.3, lam=-0.2, m=feats, seed=seed + 1, surface="sphere")
    return c, d, coupling(n, m, seed + 2)


def poisson_requests(count: int, qps: float, seed: int, lo: int = 2000, hi: int = 200_000,
                     ds=(3, 16, 64), ms=(64, 128, 256)) -> list[dict]:
    """Request stream for the serving loop: exponential inter-arrival gaps at
    the given rate, log-uniform N, a random surface, d and m drawn uniformly."""
    g = _rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += g.exponential(1.0 / qps)
        n = int(math.floor(math.exp(g.uniform(math.log(lo), math.log(hi)))))
        out.append(dict(t=t, n=n, surface=SURFACES[int(g.integers(0, 3))], d=int(g.choice(ds)),
                        m=int(g.choice(ms)), seed=int(g.integers(0, 2**31 - 1))))
    return out


# Mesh sizes of the paper's barycenter table (Table 2: alien, duck, land, octocat).
BARYCENTER_SIZES = (5212, 9862, 14738, 18944)


@dataclass
class BaryProblem:
    """k input distributions on a cloud for the Wasserstein-barycenter loop,
    with the paper's settings (App. D, "Details on Hyper-parameters"):
    eps = 0.01, lambda = 0.5, m = 30 features, k = 3, alpha = 1/3; the
    frequency law is the truncated Gaussian sigma = 1, R = 3."""
    X: np.ndarray        # n x 3 float32
    a: np.ndarray        # n float32: area weights (area-uniform samples: 1/n each)
    mus: np.ndarray      # n x k float32: distribution i in column i, a . mu_i = 1
    eps: float = 0.01
    lam: float = 0.5
    m: int = 30
    seed: int = 3
    sigma: float = 1.0
    radius: float = 3.0
    alpha: tuple = (1 / 3, 1 / 3, 1 / 3)


def barycenter_problem(n: int, surface_kind: str = "sphere", seed: int = 0, k: int = 3,
                       width: float = 0.3, background: float = 1e-2) -> BaryProblem:
    """Each input has its mass around a distinct centre point of the cloud (a
    Gaussian bump of the given width in 3-D distance) over a small uniform
    background (so every entry is positive), normalised to a . mu = 1."""
    X = surface(surface_kind, n, seed)
    g = _rng(seed + 1000)
    centres = X[g.choice(n, k, replace=False)].astype(np.float64)
    a = np.full(n, 1.0 / n)
    cols = []
    for c in centres:
        b = np.exp(-np.sum((X.astype(np.float64) - c) ** 2, axis=1) / (2.0 * width * width))
        b = b + background * b.max()
        cols.append(b / (a @ b))
    return BaryProblem(X=X, a=a.astype(np.float32), mus=np.stack(cols, axis=1).astype(np.float32))


# ------------------------------------------------------------------ node features in D dimensions
def node_features(n: int, dim: int, seed: int, clusters: int = 4, spread: float = 0.15) -> np.ndarray:
    """n points of R^dim standing in for a graph's node-feature vectors (the
    graph-classification appendix treats them as a point set): a few cluster
    centres uniform in the unit cube (node kinds) and Gaussian spread around
    them, float32 n x dim."""
    g = _rng(seed)
    centres = g.uniform(0.0, 1.0, (clusters, dim))
    which = g.integers(0, clusters, n)
    return (centres[which] + spread * g.normal(size=(n, dim))).astype(np.float32)


def graph_batch(count: int = 1024, dim: int = 16, seed: int = 0, lo: int = 10, hi: int = 300):
    """Synthetic stand-in for a graph-classification set: `count` graphs with
    node counts log-uniform in [lo, hi] (the appendix's datasets average 14 to
    284 nodes) and node features in R^dim, each a node_features cloud."""
    g = _rng(seed)
    sizes = np.floor(np.exp(g.uniform(math.log(lo), math.log(hi + 1), count))).astype(np.int64)
    return [node_features(int(n), dim, seed * 100003 + i) for i, n in enumerate(sizes)]
