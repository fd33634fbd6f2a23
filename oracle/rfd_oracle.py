"""CPU oracle for the RFDiffusion (RFD) graph-field integrator.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this module; only the tests, the smoke check and the benchmark's CPU
baseline leg use it. It shares no code with the GPU library: it has its own
frequency sampler, its own weights, its own matrix exponential and its own
phi_1, all in float64 with numpy (a library matmul and a dense linear solve
serve as steps; nothing is blocked, fused or reordered).

What it computes (paper Sec. 2.4, "RFDiffusion"):

* Graph-field integration i(v) = sum_w K(w, v) F(w) (Eq. 1) with the graph
  diffusion kernel K = exp(lambda W_G) (Eq. 3), W_G(i, j) = f(n_i - n_j) and
  f(z) = 1[||z|| <= eps] for the epsilon-NN graph (Eq. "w").
* W_G is replaced by a Monte-Carlo random-feature estimate A B^T: f is
  written as the inverse Fourier transform of tau, frequencies omega_k are
  drawn from a truncated Gaussian P with pdf p, and each contributes with the
  importance weight tau/p (Sec. 2.4; the real-part estimator of the Lemma 2.5
  proof, App. A.4).
* exp(lambda A B^T) F is applied in low-rank form (Sec. 2.4, the displayed
  identity and the bracket order of the GFI formula that follows it). The
  identity is used in the phi_1 form F + A (lambda phi_1(lambda B^T A)) (B^T F)
  with phi_1(X) = sum_k X^k / (k+1)!, which needs no inverse of B^T A.

Readings where the paper is silent or garbled (each is listed with its reason
in the design notes of the repository):

* m counts real feature columns: f = m/2 frequencies, each giving a cos and a
  sin column, so the real part of the complex estimator is exact.
* Feature scale c_k = sqrt(|w_k| / f) with w_k = tau(omega_k)/p(omega_k); the
  sign s_k = sgn(w_k) goes on A only (A = Phi diag(s, s), B = Phi).
* P is N(0, sigma^2 I3) truncated by rejection to the L2 ball of radius R
  (L-infinity ball for the box shape). Default "main-lobe" preset:
  R = r0/eps with r0 the first zero of tau_ball in units of 1/eps, sigma = R/3,
  which keeps every weight non-negative.
* tau of the L2 ball indicator in 3-D is the spherical-Bessel form
  (sin u - u cos u) / (2 pi^2 r^3), u = 2 pi eps r; the paper's L1 formula is
  read as the transform of the L-infinity box, prod_i sin(2 pi eps w_i)/(pi w_i).
* Points in D dimensions (the graph-classification appendix: node features as
  vectors in R^D): tau of the D-ball is eps^(D/2) J_{D/2}(2 pi eps r) / r^(D/2)
  (Sec. 2.4: a Bessel function of order tied to the dimension), the box
  transform is the same product over D coordinates, P is N(0, sigma^2 I_D)
  truncated to the D-ball (chi_D mass, the regularised incomplete gamma
  function) or D-box, and the main-lobe ball radius is the first zero of
  J_{D/2} over 2 pi eps. D = 3 keeps the closed forms above.
* Self-loops: W_ii = 1 (f(0) = 1).
* Random stream: SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) from the seed,
  53-bit uniforms, Box-Muller with both outputs used in order, 3 normals per
  candidate frequency, rejection in float64, then rounding to float32.
* phi_1 and exp: Pade [13/13] with scaling and squaring (Higham 2005), phi_1
  through the augmented matrix [[Y, I], [0, 0]] (Al-Mohy & Higham 2011), and
  phi_1(2Y) = phi_1(Y) (e^Y + I) / 2 to undo the scaling.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
from scipy import optimize as _opt
from scipy import special as _sp

# First positive root of tan(u) = u, i.e. of sin(u) - u cos(u): the first zero
# of the 3-D ball transform's numerator. r0 = U0 / (2 pi) is that zero in
# frequency units for eps = 1.
U0 = 4.493409457909064
R0 = U0 / (2.0 * math.pi)

# Largest 1-norm for which the [13/13] Pade approximant of exp meets double
# precision backward error (Higham 2005, SIAM J. Matrix Anal. Appl. 26(4),
# Table 2.3).
THETA13 = 5.371920351148152

BALL_L2 = 0
BOX_LINF = 1

# Rejection sampling gives up after this many candidates (per frequency, plus
# a fixed allowance): a law whose truncation keeps almost no mass is refused.
MAX_CANDIDATES_PER_FREQUENCY = 10000
MAX_CANDIDATES_EXTRA = 1000000

_MASK64 = (1 << 64) - 1


# --------------------------------------------------------------------------
# Random stream: SplitMix64 and Box-Muller.
# --------------------------------------------------------------------------
def splitmix64(seed: int):
    """SplitMix64 (Steele, Lea & Flood 2014): a Weyl sequence with increment
    0x9E3779B97F4A7C15 passed through the variant-13 mixing function."""
    state = seed & _MASK64
    while True:
        state = (state + 0x9E3779B97F4A7C15) & _MASK64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        yield z ^ (z >> 31)


def gaussian_stream(seed: int):
    """Standard normals by Box-Muller on pairs of 53-bit uniforms:
    u1 in (0, 1], u2 in [0, 1); r = sqrt(-2 ln u1); yields r cos(2 pi u2)
    then r sin(2 pi u2). Scalar glibc math through Python's math module."""
    g = splitmix64(seed)
    twopi = 2.0 * math.pi
    while True:
        a = next(g)
        b = next(g)
        u1 = ((a >> 11) + 1) * (1.0 / 9007199254740992.0)
        u2 = (b >> 11) * (1.0 / 9007199254740992.0)
        r = math.sqrt(-2.0 * math.log(u1))
        t = twopi * u2
        yield r * math.cos(t)
        yield r * math.sin(t)


def bessel_first_zero(nu: float) -> float:
    """First positive zero j_{nu,1} of the Bessel function J_nu (nu >= 1/2):
    bracketed between nu and nu + 2 sqrt(nu + 1) + 3 (the zero lies above nu)
    and found by Brent's method on scipy's J_nu."""
    a = max(nu, 1e-3)
    b = nu + 2.0 * math.sqrt(nu + 1.0) + 3.0
    # step up from a until J_nu changes sign (its first sign change is j_{nu,1})
    xs = np.linspace(a, b, 400)
    v = _sp.jv(nu, xs)
    i = int(np.nonzero(np.sign(v[1:]) != np.sign(v[:-1]))[0][0])
    return float(_opt.brentq(lambda x: _sp.jv(nu, x), xs[i], xs[i + 1], xtol=1e-15, rtol=8.9e-16, maxiter=200))


def ball_radius_unit(dim: int) -> float:
    """r0 of the D-ball: the first zero of its transform in units of 1/eps,
    j_{D/2,1} / (2 pi); the 3-D constant R0 for D = 3."""
    return R0 if dim == 3 else bessel_first_zero(0.5 * dim) / (2.0 * math.pi)


def preset(eps: float, shape: int = BALL_L2, sigma: float = 0.0, radius: float = 0.0, dim: int = 3):
    """(sigma, R) of the truncated Gaussian. sigma = R = 0 selects the
    main-lobe preset: ball R = r0/eps, box R = 1/(2 eps); sigma = R/3 in 3-D,
    R / sqrt(D + 6) in D dimensions (the same for D = 3; the D-dimensional
    Gaussian's mass sits near radius sigma sqrt(D), which stays inside R)."""
    if sigma > 0.0 and radius > 0.0:
        return float(sigma), float(radius)
    if sigma != 0.0 or radius != 0.0:
        raise ValueError("sigma and radius must both be set or both be 0")
    R = (ball_radius_unit(dim) / eps) if shape == BALL_L2 else (0.5 / eps)
    return (R / 3.0 if dim == 3 else R / math.sqrt(dim + 6.0)), R


def sample_frequencies(f: int, eps: float, seed: int, shape: int = BALL_L2,
                       sigma: float = 0.0, radius: float = 0.0, dim: int = 3) -> np.ndarray:
    """f frequencies omega_k ~ N(0, sigma^2 I_D) truncated to ||omega|| <= R
    (L2 for the ball, L-infinity for the box) by rejection, as float32
    (f x D). Sec. 2.4: omega_1..omega_m i.i.d. from P, P a truncated Gaussian.
    A candidate takes the next D normals of the stream in order; the squared
    norm is summed left to right."""
    if dim < 1:
        raise ValueError("dim must be >= 1")
    sig, R = preset(eps, shape, sigma, radius, dim)
    g = gaussian_stream(seed)
    out = np.empty((f, dim), dtype=np.float32)
    k = 0
    tries = 0
    while k < f:
        tries += 1
        if tries > MAX_CANDIDATES_PER_FREQUENCY * f + MAX_CANDIDATES_EXTRA:
            raise ValueError("the truncated frequency law accepts too few candidates")
        cand = [sig * next(g) for _ in range(dim)]
        if shape == BALL_L2:
            r2 = cand[0] * cand[0]
            for c in cand[1:]:
                r2 = r2 + c * c
            ok = r2 <= R * R
        else:
            ok = max(abs(c) for c in cand) <= R
        if ok:
            out[k] = cand
            k += 1
    return out


# --------------------------------------------------------------------------
# Importance weights w = tau / p.
# --------------------------------------------------------------------------
def tau_ball(omega: np.ndarray, eps: float) -> np.ndarray:
    """Fourier transform of 1[||z||_2 <= eps] in 3-D with the convention
    f(z) = int exp(2 pi i w.z) tau(w) dw: (sin u - u cos u) / (2 pi^2 r^3),
    r = ||w||, u = 2 pi eps r; its Taylor series near u = 0."""
    om = np.asarray(omega, dtype=np.float64)
    r = np.sqrt(np.sum(om * om, axis=-1))
    u = 2.0 * math.pi * eps * r
    vol = 4.0 * math.pi * eps ** 3 / 3.0
    small = u < 1e-2
    out = np.empty_like(r)
    us = u[small]
    out[small] = vol * (1.0 - us * us / 10.0 + us ** 4 / 280.0)
    ub, rb = u[~small], r[~small]
    out[~small] = (np.sin(ub) - ub * np.cos(ub)) / (2.0 * math.pi ** 2 * rb ** 3)
    return out


def tau_ball_nd(omega: np.ndarray, eps: float) -> np.ndarray:
    """Fourier transform of 1[||z||_2 <= eps] in D = omega.shape[-1]
    dimensions, same convention: eps^(D/2) J_{D/2}(2 pi eps r) / r^(D/2);
    at r = 0 the ball's volume pi^(D/2) eps^D / Gamma(D/2 + 1) (the limit of
    J_nu(u) ~ (u/2)^nu / Gamma(nu + 1)), and its two-term series for small u."""
    om = np.asarray(omega, dtype=np.float64)
    D = om.shape[-1]
    nu = 0.5 * D
    r = np.sqrt(np.sum(om * om, axis=-1))
    u = 2.0 * math.pi * eps * r
    vol = math.pi ** nu * eps ** D / math.gamma(nu + 1.0)
    small = u < 1e-4
    out = np.empty_like(r)
    us = u[small]
    out[small] = vol * (1.0 - us * us / (4.0 * (nu + 1.0)))
    ub, rb = u[~small], r[~small]
    out[~small] = eps ** nu * _sp.jv(nu, ub) / rb ** nu
    return out


def tau_box(omega: np.ndarray, eps: float) -> np.ndarray:
    """Fourier transform of prod_i 1[|z_i| <= eps]: prod_i sin(2 pi eps w_i)/(pi w_i)
    = prod_i 2 eps sinc(2 eps w_i) with sinc(t) = sin(pi t)/(pi t)."""
    om = np.asarray(omega, dtype=np.float64)
    return np.prod(2.0 * eps * np.sinc(2.0 * eps * om), axis=-1)


def truncation_mass(t: float, shape: int = BALL_L2, dim: int = 3) -> float:
    """P(N(0, I_D) lies in the ball of radius t): the chi_D CDF, the
    regularised lower incomplete gamma P(D/2, t^2/2); for D = 3 the closed form
    erf(t/sqrt2) - sqrt(2/pi) t exp(-t^2/2). For the box, erf(t/sqrt2)^D."""
    if shape == BALL_L2:
        if dim == 3:
            return math.erf(t / math.sqrt(2.0)) - math.sqrt(2.0 / math.pi) * t * math.exp(-t * t / 2.0)
        return float(_sp.gammainc(0.5 * dim, 0.5 * t * t))
    return math.erf(t / math.sqrt(2.0)) ** dim


def pdf(omega: np.ndarray, sigma: float, R: float, shape: int = BALL_L2) -> np.ndarray:
    """Density of N(0, sigma^2 I_D) truncated to the radius-R ball (or box),
    D = omega.shape[-1]."""
    om = np.asarray(omega, dtype=np.float64)
    D = om.shape[-1]
    r2 = np.sum(om * om, axis=-1)
    C = truncation_mass(R / sigma, shape, D)
    return (2.0 * math.pi * sigma * sigma) ** (-0.5 * D) * np.exp(-r2 / (2.0 * sigma * sigma)) / C


def weights(omega: np.ndarray, eps: float, shape: int = BALL_L2, sigma: float = 0.0,
            radius: float = 0.0) -> np.ndarray:
    """w_k = tau(omega_k) / p(omega_k) at the float32 frequencies (Sec. 2.4:
    nu_k^2 = tau/p); the dimension is that of the frequencies."""
    D = np.asarray(omega).shape[-1]
    sig, R = preset(eps, shape, sigma, radius, D)
    if shape == BALL_L2:
        tau = tau_ball(omega, eps) if D == 3 else tau_ball_nd(omega, eps)
    else:
        tau = tau_box(omega, eps)
    return tau / pdf(omega, sig, R, shape)


# --------------------------------------------------------------------------
# Features and the low-rank factors.
# --------------------------------------------------------------------------
def features(X: np.ndarray, omega: np.ndarray, w: np.ndarray):
    """Real feature matrix Phi (N x m) and column signs (m,).

    Phi_i = [c_k cos(2 pi omega_k . x_i)]_k || [c_k sin(2 pi omega_k . x_i)]_k,
    c_k = sqrt(|w_k| / f). With s = [sgn w, sgn w], A = Phi diag(s) and B = Phi
    give (A B^T)_ij = (1/f) sum_k w_k cos(2 pi omega_k . (x_i - x_j)), the
    real-part estimator of the Lemma 2.5 proof (App. A.4)."""
    Xd = np.asarray(X, dtype=np.float32).astype(np.float64)
    Om = np.asarray(omega, dtype=np.float32).astype(np.float64)
    f = Om.shape[0]
    theta = Xd @ Om.T  # N x f, revolutions
    c = np.sqrt(np.abs(w) / f)
    Phi = np.concatenate([c * np.cos(2.0 * math.pi * theta), c * np.sin(2.0 * math.pi * theta)], axis=1)
    sg = np.where(np.asarray(w) < 0.0, -1.0, 1.0)
    return Phi, np.concatenate([sg, sg])


# --------------------------------------------------------------------------
# Matrix exponential and phi_1 (Pade [13/13], scaling and squaring).
# --------------------------------------------------------------------------
def pade13_coefficients() -> np.ndarray:
    """b_k = (2q - k)! q! / ((2q)! k! (q - k)!) for q = 13: numerator of the
    [q/q] Pade approximant of e^x; the denominator is the same with x -> -x."""
    q = 13
    fa = math.factorial
    return np.array([float(Fraction(fa(2 * q - k) * fa(q), fa(2 * q) * fa(k) * fa(q - k)))
                     for k in range(q + 1)])


def pade13(A: np.ndarray) -> np.ndarray:
    """r13(A) = q13(A)^{-1} p13(A) with plain powers of A."""
    b = pade13_coefficients()
    n = A.shape[0]
    P = np.zeros((n, n))
    Q = np.zeros((n, n))
    Ak = np.eye(n)
    for k in range(14):
        if k > 0:
            Ak = Ak @ A
        P += b[k] * Ak
        Q += ((-1.0) ** k) * b[k] * Ak
    return np.linalg.solve(Q, P)


def scaling_power(A: np.ndarray) -> int:
    """s = max(0, ceil(log2(||A||_1 / theta13)))."""
    nrm = np.max(np.sum(np.abs(A), axis=0)) if A.size else 0.0
    if nrm <= THETA13:
        return 0
    return max(0, int(math.ceil(math.log2(nrm / THETA13))))


def expm(A: np.ndarray) -> np.ndarray:
    """exp(A) by scaling and squaring: e^A = (r13(A / 2^s))^(2^s)."""
    A = np.asarray(A, dtype=np.float64)
    s = scaling_power(A)
    E = pade13(A / (2.0 ** s))
    for _ in range(s):
        E = E @ E
    return E


def phi1_and_exp(X: np.ndarray):
    """(phi_1(X), e^X) for a square X.

    Y = X / 2^s; the exponential of the augmented 2n x 2n matrix
    Z = [[Y, I], [0, 0]] is [[e^Y, phi_1(Y)], [0, I]], so one dense Pade
    approximant of Z gives both blocks. Then s times:
    phi_1 <- phi_1 (e^Y + I) / 2 and e^Y <- e^Y e^Y, by phi_1(2Y) = phi_1(Y)(e^Y + I)/2."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    s = scaling_power(X)
    Y = X / (2.0 ** s)
    Z = np.zeros((2 * n, 2 * n))
    Z[:n, :n] = Y
    Z[:n, n:] = np.eye(n)
    R = pade13(Z)
    E = R[:n, :n].copy()
    P = R[:n, n:].copy()
    I = np.eye(n)
    for _ in range(s):
        P = 0.5 * (P @ (E + I))
        E = E @ E
    return P, E


def phi1(X: np.ndarray) -> np.ndarray:
    return phi1_and_exp(X)[0]


# --------------------------------------------------------------------------
# The integrator.
# --------------------------------------------------------------------------
def lowrank_apply(A: np.ndarray, B: np.ndarray, F: np.ndarray, lam: float):
    """exp(lam A B^T) F = F + A (lam phi_1(lam B^T A)) (B^T F): the low-rank
    identity of Sec. 2.4 in phi_1 form, in the paper's bracket order
    (B^T F first, then the m x m core, then A). Returns out and the pieces."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    Fd = np.asarray(F, dtype=np.float64)
    M = B.T @ A
    H = B.T @ Fd
    S = lam * phi1(lam * M)
    G = S @ H
    out = Fd + A @ G
    return out, dict(M=M, H=H, S=S, G=G)


def frequencies_and_weights(m: int, eps: float, seed: int, shape: int = BALL_L2,
                            sigma: float = 0.0, radius: float = 0.0, dim: int = 3):
    if m <= 0 or m % 2:
        raise ValueError("m must be a positive even number")
    f = m // 2
    om = sample_frequencies(f, eps, seed, shape, sigma, radius, dim)
    return om, weights(om, eps, shape, sigma, radius)


def rfd_integrate(X, F, eps: float, lam: float, m: int, seed: int, shape: int = BALL_L2,
                  sigma: float = 0.0, radius: float = 0.0, return_parts: bool = False):
    """One-shot RFD: sample features, build A and B, apply exp(lam A B^T) to F."""
    om, w = frequencies_and_weights(m, eps, seed, shape, sigma, radius)
    Phi, sg = features(X, om, w)
    out, parts = lowrank_apply(Phi * sg, Phi, F, lam)
    if return_parts:
        parts.update(omega=om, w=w, Phi=Phi, sign=sg)
        return out, parts
    return out


def what_hat(X, omega, w) -> np.ndarray:
    """Dense N x N estimate A B^T (tiny N only)."""
    Phi, sg = features(X, omega, w)
    return (Phi * sg) @ Phi.T


def dense_adjacency(X, eps: float, shape: int = BALL_L2, self_loops: bool = True) -> np.ndarray:
    """W_ij = 1[||x_i - x_j|| <= eps] (Eq. "w"), compared in float64 from the
    float32 points, boundary inclusive; W_ii = 1 unless self_loops is False."""
    Xd = np.asarray(X, dtype=np.float32).astype(np.float64)
    D = Xd[:, None, :] - Xd[None, :, :]
    if shape == BALL_L2:
        W = (np.sum(D * D, axis=-1) <= eps * eps).astype(np.float64)
    else:
        W = (np.max(np.abs(D), axis=-1) <= eps).astype(np.float64)
    if not self_loops:
        np.fill_diagonal(W, 0.0)
    return W


def dense_integrate(X, F, eps: float, lam: float, shape: int = BALL_L2,
                    self_loops: bool = True) -> np.ndarray:
    """Brute-force GFI (Sec. 1): materialise K = exp(lam W) and multiply."""
    W = dense_adjacency(X, eps, shape, self_loops)
    return expm(lam * W) @ np.asarray(F, dtype=np.float64)


def repeated_apply(clouds, v0, scales, lam_list, iters: int, omegas, ws):
    """v_{t+1} = s_{t mod 2} * K_{t mod 2}(v_t) for two clouds of equal size,
    each K_c = exp(lam_c A_c B_c^T) with fixed features (a Sinkhorn-style
    alternating loop, App. D Alg. 1 shape)."""
    v = np.asarray(v0, dtype=np.float64)
    ops = []
    for X, om, w, lam in zip(clouds, omegas, ws, lam_list):
        Phi, sg = features(X, om, w)
        A = Phi * sg
        S = lam * phi1(lam * (Phi.T @ A))
        ops.append((A, Phi, S))
    for t in range(iters):
        A, B, S = ops[t % 2]
        v = np.asarray(scales[t % 2], dtype=np.float64)[:, None] * (v + A @ (S @ (B.T @ v)))
    return v


def wasserstein_barycenter(apply_K, mus, a, alpha, iters: int, floor=None, return_state: bool = False):
    """Entropic Wasserstein barycenter by the scaling iteration of App. D
    (Alg. 1, "Fast Computation of Wasserstein Barycenter"), with the kernel
    entering only through its action apply_K (an FM: here the RFD operator).

    mus: k input distributions (each N,), a: area weights (N,), alpha: k
    weights. Starting from v^i = w^i = 1, each of `iters` iterations does, for
    i = 1..k,
        w^i = mu^i / K(a v^i),   d^i = v^i K(a w^i),   mu = mu * (d^i)^alpha_i,
    and then v^i = v^i mu / d^i for every i.

    Reading: mu restarts from the all-ones vector at the start of every
    iteration, so mu = prod_i (d^i)^alpha_i, the weighted geometric mean of
    the current marginals (the listing initialises mu once; without the
    restart the update would multiply the barycenter into mu at every
    iteration and have no fixed point).

    floor (optional safeguard, not in the listing): a factor rho >= 0 by which
    every output y = K(x) of the two kernel actions is replaced by
    max(y, rho x) elementwise. With rho = 1 this is the lower bound
    exp(lambda W) x >= x that the exact kernel satisfies for lambda >= 0 and a
    non-negative W, which the random-feature estimate can violate (its values
    can be negative). Returns mu, or (mu, v, d, floored count) with
    return_state."""
    mus = [np.asarray(m_, dtype=np.float64) for m_ in mus]
    a = np.asarray(a, dtype=np.float64)
    k = len(mus)
    N = a.shape[0]
    v = [np.ones(N) for _ in range(k)]
    d = [np.ones(N) for _ in range(k)]
    mu = np.ones(N)
    floored = 0

    def K(x):
        nonlocal floored
        y = np.asarray(apply_K(x), dtype=np.float64)
        if floor is None:
            return y
        lo = floor * x
        floored += int(np.sum(y < lo))
        return np.maximum(y, lo)

    for _ in range(iters):
        mu = np.ones(N)
        for i in range(k):
            w = mus[i] / K(a * v[i])
            d[i] = v[i] * K(a * w)
            mu = mu * d[i] ** alpha[i]
        for i in range(k):
            v[i] = v[i] * mu / d[i]
    if return_state:
        return mu, v, d, floored
    return mu


def rfd_operator(X, eps: float, lam: float, m: int, seed: int, shape: int = BALL_L2,
                 sigma: float = 0.0, radius: float = 0.0):
    """x -> exp(lam A B^T) x on the cloud X with the frequencies of `seed`
    (frequency law as in sample_frequencies), by the low-rank identity
    (Sec. 2.4): x + A (lam phi_1(lam B^T A)) (B^T x)."""
    om, w = frequencies_and_weights(m, eps, seed, shape, sigma, radius)
    Phi, sg = features(X, om, w)
    A = Phi * sg
    S = lam * phi1(lam * (Phi.T @ A))

    def apply(x):
        x = np.asarray(x, dtype=np.float64)
        return x + A @ (S @ (Phi.T @ x))

    return apply


def gw_terms(apply_C, apply_D, T):
    """The three terms of the Gromov-Wasserstein loss matrix for the Euclidean
    loss (App. "Fast Computation of Tensor Products", Alg. 2): with p = T 1
    and q = T^T 1,
        v1 = C^2 p, v2 = D^2 q, w3 = C T D^T,
    where C^2 p (the Hadamard square of C applied to p) is taken as
    diag(C (C diag(p))^T) (the Hadamard-square subsection before Alg. 2) and
    D likewise, and C T D^T as (D (C T)^T)^T (Alg. 2, step 3); C and D enter
    only through their actions (apply_C on n-row, apply_D on m-row blocks)."""
    T = np.asarray(T, dtype=np.float64)
    p = T.sum(axis=1)
    q = T.sum(axis=0)
    v1 = np.diag(apply_C(apply_C(np.diag(p)).T)).copy()
    v2 = np.diag(apply_D(apply_D(np.diag(q)).T)).copy()
    w3 = apply_D(apply_C(T).T).T
    return v1, v2, w3


def gw_loss(apply_C, apply_D, T):
    """L = v1 1^T + 1 v2^T - 2 w3 (Alg. 2, its returned value) from gw_terms."""
    v1, v2, w3 = gw_terms(apply_C, apply_D, T)
    return v1[:, None] + v2[None, :] - 2.0 * w3


def kernel_spectrum(X, eps: float, lam: float, m: int, seed: int, shape: int = BALL_L2,
                    sigma: float = 0.0, radius: float = 0.0):
    """All N eigenvalues, ascending, of the RFD kernel matrix exp(lam A B^T)
    through the low-rank factors, as the classification experiments use them
    (Sec. 3, point-cloud classification; the graph-classification appendix):
    det(t I_N - A B^T) = t^(N-m) det(t I_m - B^T A), so A B^T has the m
    eigenvalues mu_i of B^T A and N - m zeros when N >= m, and for N < m the
    eigenvalues of B^T A less m - N of its zero ones (those of smallest |mu|);
    exp(lam A B^T) has exp(lam mu) for each. Points may have any dimension D
    (the frequencies take the points' dimension)."""
    D = np.asarray(X).shape[1]
    om, w = frequencies_and_weights(m, eps, seed, shape, sigma, radius, D)
    Phi, sg = features(X, om, w)
    M = Phi.T @ (Phi * sg)  # B^T A
    mu = np.linalg.eigvals(M).real
    N = np.asarray(X).shape[0]
    if N >= m:
        mu = np.concatenate([mu, np.zeros(N - m)])
    else:
        mu = mu[np.argsort(np.abs(mu), kind="stable")[m - N:]]
    return np.sort(np.exp(lam * mu))


def relf(a, b) -> float:
    """Relative Frobenius error ||a - b|| / ||b||."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))
