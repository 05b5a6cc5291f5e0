"""Pins of the oracle's scheme, eq. (21) with the memory modes of eqs. (22), (24):
gamma = 1 is classical FTCS diffusion (a sparse-matrix textbook scheme), gamma = 2 is the
classical leapfrog scheme of the wave equation, a discrete sine mode is an eigenvector
(the PDE reduces to a scalar recursion), the scalar recursion converges to Mittag-Leffler
relaxation at first order (sub- and superdiffusion), the GL weights reproduce the
closed-form fractional derivative (and integral) of t^p, and the degenerate memory
settings reproduce full memory bit for bit.  1D, 2D and 3D grids."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy import special

import oracle
from paper_1004_5128_amd import workloads as W


def lap_matrix(p):
    def d2(n):
        return sp.diags([np.ones(n - 1), -2 * np.ones(n), np.ones(n - 1)], [-1, 0, 1])
    if p["ndim"] == 1:
        return d2(p["nx"]).tocsr()
    L2 = sp.kron(sp.identity(p["ny"]), d2(p["nx"])) + sp.kron(d2(p["ny"]), sp.identity(p["nx"]))
    if p["ndim"] == 2:
        return L2.tocsr()
    # 3D, x fastest then y then z: the 2D operator on every z layer plus the z coupling
    return (sp.kron(sp.identity(p["nz"]), L2) +
            sp.kron(d2(p["nz"]), sp.identity(p["nx"] * p["ny"]))).tocsr()


def ftcs(p, u0, n):
    """Classical forward-time centred-space diffusion with an explicit reaction term."""
    L = lap_matrix(p)
    r = p["alpha"] * p["dt"] / p["dx"] ** 2
    u = u0.copy()
    for _ in range(n):
        if p["rxn"] == "linear":
            f = -p["rate"] * u
        elif p["rxn"] == "fisher":
            f = p["rate"] * u * (1 - u)
        else:
            f = 0.0
        u = u + p["dt"] * f + r * (L @ u)
    return u


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("ndim,rxn", [(1, "none"), (2, "linear"), (2, "fisher"), (3, "fisher")])
def test_gamma_one_is_ftcs(ndim, rxn):
    p = W.problem(ndim, 24 if ndim < 3 else 11, 1.0, 0.7, 0.2 if ndim < 3 else 0.1, rxn=rxn,
                  rate=0.3)
    u0 = W.gaussian(p, 11) + 0.2
    n = 300
    got = oracle.run(p, W.memory("full"), u0, n)
    assert rel(got, ftcs(p, u0, n)) < 1e-13


MEMS = [W.memory("full"), W.memory("short", L=7), W.memory("adaptive", a=2),
        W.memory("adaptive", a=3, rule="literal"), W.memory("adaptive", a=4)]


@pytest.mark.parametrize("mem", MEMS, ids=lambda m: "%s-%s-%d" % (m["mode"], m["rule"], m["a"]))
@pytest.mark.parametrize("ndim,pq", [(1, (1, 1, 1)), (1, (5, 1, 1)), (2, (1, 1, 1)),
                                     (2, (2, 3, 1)), (3, (1, 1, 1)), (3, (2, 1, 3))])
def test_sine_mode_is_an_eigenvector(mem, ndim, pq):
    p = W.problem(ndim, 15 if ndim < 3 else 7, 0.7, 1.0, 0.08 if ndim < 3 else 0.05,
                  rxn="linear", rate=0.5)
    n = 250
    phi = W.sine_mode(p, pq[0], pq[1], mode_s=pq[2])
    U = oracle.run(p, mem, 0.8 * phi, n, store_all=True)
    v = oracle.mode_run(p, mem, pq[0], pq[1], 0.8, n, s=pq[2])
    err = np.abs(U - np.outer(v, phi)).max()
    assert err < 1e-13 * np.abs(U).max()


def mittag_leffler(gamma, z):
    """E_gamma(-z): erfcx at gamma = 1/2 (exact identity), power series otherwise."""
    if gamma == 0.5:
        return special.erfcx(z)
    j = np.arange(0, 120)
    return float(np.sum((-z) ** j / special.gamma(gamma * j + 1)))


@pytest.mark.parametrize("gamma,T", [(0.5, 0.01), (0.8, 0.05), (0.65, 0.03),
                                     (1.3, 0.2), (1.7, 0.3), (2.0, 0.4)])
def test_mode_recursion_converges_to_mittag_leffler(gamma, T):
    # du/dt = alpha D^(1-gamma) Lap u on one eigenmode is Caputo relaxation
    # d^gamma v/dt^gamma = -alpha lam v, solved by v(t) = E_gamma(-alpha lam t^gamma);
    # the explicit GL scheme is first order in dt.  For 1 < gamma <= 2, D^(1-gamma) is the
    # fractional integral of order gamma - 1 and the same holds with v'(0) = 0 (at gamma = 2,
    # E_2(-z) = cos(sqrt(z))).
    nx = 7
    dx = 1.0 / (nx + 1)
    lam = 4 * np.sin(np.pi / (2 * (nx + 1))) ** 2 / dx ** 2
    exact = mittag_leffler(gamma, lam * T ** gamma)
    errs = []
    for n in (500, 1000, 2000, 4000):
        p = W.problem(1, nx, gamma, 1.0, None, dt=T / n)
        v = oracle.mode_run(p, W.memory("full"), 1, 1, 1.0, n)
        errs.append(abs(v[-1] - exact))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((ratios > 1.7) & (ratios < 2.3)), (errs, ratios)
    assert errs[-1] < 5e-3 * exact


def test_cfg1_mode_matches_mittag_leffler():
    # 1D, 128 points, gamma = 1/2, r = 0.2, 2000 steps, u0 = sin(pi x).
    w = W.cfg1()
    p = w["problem"]
    u = oracle.run(p, w["memory"], w["u0"], w["nsteps"])
    lam = 4 * np.sin(np.pi / (2 * (p["nx"] + 1))) ** 2 / p["dx"] ** 2
    T = w["nsteps"] * p["dt"]
    amp = special.erfcx(p["alpha"] * lam * np.sqrt(T))
    assert rel(u, amp * w["u0"]) < 2e-6


@pytest.mark.parametrize("gamma", [0.3, 0.5, 0.8, 1.3, 1.7])
@pytest.mark.parametrize("q", [1, 2, 3])
def test_gl_weights_reproduce_derivative_of_power(gamma, q):
    # h^-nu sum_{m=0}^{k} psi(gamma,m) f(t - m h) -> D^nu t^q = Gamma(q+1)/Gamma(q+1-nu) t^(q-nu),
    # nu = 1 - gamma, with first-order convergence in h (eqs. 5, 7); for gamma > 1, nu < 0
    # and the same sum is the GL fractional integral of order -nu.
    nu = 1.0 - gamma
    exact = special.gamma(q + 1) / special.gamma(q + 1 - nu)
    errs = []
    for k in (200, 400, 800, 1600):
        h = 1.0 / k
        ps = oracle.psi(gamma, k)
        f = ((k - np.arange(k + 1)) * h) ** q
        errs.append(abs(h ** (-nu) * np.sum(ps * f) - exact))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all((ratios > 1.8) & (ratios < 2.2)), (errs, ratios)


def test_short_memory_zero_window_closed_form():
    # L = 0 keeps only psi(0) delta[k]: the mode decays as (1 - r lam - dt rate)^k.
    p = W.problem(2, 12, 0.6, 1.0, 0.1, rxn="linear", rate=0.4)
    n = 100
    mem = W.memory("short", L=0)
    phi = W.sine_mode(p, 3, 2)
    r = oracle.r_of(p)
    lam = 4 * np.sin(3 * np.pi / 26) ** 2 + 4 * np.sin(2 * np.pi / 26) ** 2
    g = 1 - r * lam - p["dt"] * p["rate"]
    v = oracle.mode_run(p, mem, 3, 2, 1.0, n)
    np.testing.assert_allclose(v, g ** np.arange(n + 1), rtol=1e-12)
    u = oracle.run(p, mem, phi, n)
    assert rel(u, g ** n * phi) < 1e-12


def test_degenerate_memory_modes_are_bitwise_full():
    p = W.problem(2, 10, 0.75, 1.0, 0.1, rxn="fisher", rate=1.0)
    u0 = W.uniform_field(p, 3)
    n = 120
    full = oracle.run(p, W.memory("full"), u0, n)
    for mem in (W.memory("short", L=n), W.memory("short", L=10 * n), W.memory("adaptive", a=n),
                W.memory("adaptive", a=3, rule="unit_stride")):
        assert np.array_equal(oracle.run(p, mem, u0, n), full), mem


def test_linearity_zero_and_symmetry():
    p = W.problem(2, 14, 0.7, 1.0, 0.1, rxn="linear", rate=0.2)
    n = 100
    mem = W.memory("adaptive", a=2)
    u1, u2 = W.gaussian(p, 1), W.uniform_field(p, 2)
    lhs = oracle.run(p, mem, 2.0 * u1 - 3.0 * u2, n)
    rhs = 2.0 * oracle.run(p, mem, u1, n) - 3.0 * oracle.run(p, mem, u2, n)
    assert rel(lhs, rhs) < 1e-13
    assert np.all(oracle.run(p, mem, np.zeros_like(u1), n) == 0.0)
    g = W.gaussian(p, 0, noise=0.0)       # centred and noise-free: mirror symmetric
    u = oracle.run(p, mem, g, n).reshape(14, 14)
    assert np.abs(u - u[:, ::-1]).max() < 1e-15 * np.abs(u).max() + 1e-300
    assert np.abs(u - u[::-1, :]).max() < 1e-14 * np.abs(u).max()
    assert np.abs(u - u.T).max() < 1e-14 * np.abs(u).max()


@pytest.mark.parametrize("gamma", [0.3, 0.6, 0.9])
def test_stability_bound(gamma):
    # The scheme is stable iff r * lam_max <= 2^gamma (z-transform of eq. 21 at z = -1 with
    # sum psi z^m = (1-z)^(1-gamma)); lam_max -> 4 ndim: the bound r 4 ndim <= 2^gamma.
    nx = 31
    lam_max = 4 * np.sin(nx * np.pi / (2 * (nx + 1))) ** 2
    for factor, bounded in ((0.97, True), (1.03, False)):
        r = factor * 2 ** gamma / lam_max
        p = W.problem(1, nx, gamma, 1.0, r)
        v = oracle.mode_run(p, W.memory("full"), nx, 1, 1.0, 3000)
        assert (np.abs(v).max() <= 1.0 + 1e-12) == bounded, factor


def test_history_sum_against_closed_form_weights(golden_dir):
    # S = sum_t c psi(m) H[k-m] for a seeded FP32 history, with weights from the Gamma
    # function closed form and the hand-derived a = 3, k = 20 schedule.
    rng = np.random.default_rng(7)
    k, P = 20, 33
    H = rng.standard_normal((k + 1, P)).astype(np.float32)
    gamma = 0.65
    ms = [0, 1, 2, 3, 5, 8, 12, 17, 20]
    cs = [1, 1, 1, 1, 3, 3, 5, 5, 1]
    m = np.arange(k + 1, dtype=np.float64)
    w = np.ones(k + 1)
    w[1:] = -np.exp(special.gammaln(m[1:] - 1 + gamma) - special.gammaln(m[1:] + 1)
                    - special.gammaln(gamma - 1))
    ref = sum(c * w[mm] * H[k - mm].astype(np.float64) for mm, c in zip(ms, cs))
    got = oracle.history_sum(gamma, W.memory("adaptive", a=3), k, H)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)
    full = oracle.history_sum(gamma, W.memory("full"), k, np.ones((k + 1, 4), np.float32))
    ref_full = np.exp(special.gammaln(k + gamma) - special.gammaln(gamma) - special.gammaln(k + 1))
    np.testing.assert_allclose(full, ref_full, rtol=1e-12)


@pytest.mark.parametrize("gamma", [1.2, 1.4, 1.8, 2.0])
def test_stability_bound_superdiffusion(gamma):
    # The same bound r lam_max <= 2^gamma for 1 < gamma <= 2: on |z| = 1 the characteristic
    # equation z (1 - 1/z)^gamma = -r lam has its only real positive solution at z = -1.  The
    # amplitude may overshoot 1 (the solutions oscillate), so bounded means below 10.
    nx = 31
    lam_max = 4 * np.sin(nx * np.pi / (2 * (nx + 1))) ** 2
    for factor, bounded in ((0.97, True), (1.03, False)):
        r = factor * 2 ** gamma / lam_max
        p = W.problem(1, nx, gamma, 1.0, r)
        with np.errstate(over="ignore", invalid="ignore"):
            v = oracle.mode_run(p, W.memory("full"), nx, 1, 1.0, 3000)
            grown = not np.all(np.abs(v) < 10.0)
        assert grown != bounded, (factor, np.abs(v).max())


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_gamma_two_is_leapfrog_wave(ndim):
    # psi(2, m) = 1: u[k+1] - u[k] = r sum_{j<=k} delta[j], so u[k+1] - 2 u[k] + u[k-1] =
    # r delta[k], the explicit central-difference wave scheme, started with u[1] = u[0] +
    # r delta[0] (no reaction).
    p = W.problem(ndim, 24 if ndim < 3 else 9, 2.0, 1.0, 0.9 / ndim)
    u0 = W.gaussian(p, 12)
    n = 200
    L = lap_matrix(p)
    r = p["alpha"] * p["dt"] ** 2 / p["dx"] ** 2
    prev, cur = u0, u0 + r * (L @ u0)
    for _ in range(n - 1):
        prev, cur = cur, 2 * cur - prev + r * (L @ cur)
    got = oracle.run(p, W.memory("full"), u0, n)
    assert rel(got, cur) < 1e-11


def test_gamma_two_mode_closed_form():
    # On one sine mode the leapfrog recursion v[k+1] = (2 - r lam) v[k] - v[k-1], v[1] =
    # (1 - r lam) v[0], has v[k] = cos((k + 1/2) theta) / cos(theta / 2) with
    # cos(theta) = 1 - r lam / 2.
    p = W.problem(2, 13, 2.0, 1.0, 0.45)
    r = oracle.r_of(p)
    lam = 4 * np.sin(3 * np.pi / 28) ** 2 + 4 * np.sin(5 * np.pi / 28) ** 2
    theta = np.arccos(1 - r * lam / 2)
    k = np.arange(1001)
    v = oracle.mode_run(p, W.memory("full"), 3, 5, 1.0, 1000)
    np.testing.assert_allclose(v, np.cos((k + 0.5) * theta) / np.cos(theta / 2), rtol=0,
                               atol=1e-9)


@pytest.mark.parametrize("ndim,shape", [(2, (13, 6, 1)), (3, (9, 7, 5))])
def test_non_square_grids_are_ftcs_at_gamma_one(ndim, shape):
    # Unequal sides catch an axis length or stride taken from the wrong side.
    p = W.problem(ndim, shape[0], 1.0, 1.0, 0.1, rxn="linear", rate=0.2)
    p.update(ny=shape[1], nz=shape[2])
    rng = np.random.default_rng(21)
    u0 = rng.uniform(0, 1, size=W.npoints(p))
    n = 120
    assert rel(oracle.run(p, W.memory("full"), u0, n), ftcs(p, u0, n)) < 1e-13
