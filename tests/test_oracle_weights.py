"""Pins of the oracle's GL weights psi(gamma, m) and d psi / d gamma against closed
forms, exact values and finite differences (Sec. 2.1, eqs. 8-12)."""
import os

import numpy as np
import pytest
from scipy import special

import oracle

GAMMAS = [0.3, 0.5, 0.6, 0.7, 0.8, 0.95]
# superdiffusion: the same weights for 1 < gamma < 2 (the recurrence holds for any gamma)
SUPER = [1.2, 1.5, 1.8]


def psi_closed_form(gamma, n):
    """(-1)^m binom(1-gamma, m) = Gamma(m-1+gamma) / (Gamma(gamma-1) Gamma(m+1)) via lgamma."""
    m = np.arange(n + 1, dtype=np.float64)
    out = np.empty(n + 1)
    out[0] = 1.0
    mm = m[1:]
    logmag = special.gammaln(mm - 1 + gamma) - special.gammaln(gamma - 1) - special.gammaln(mm + 1)
    sign = special.gammasgn(mm - 1 + gamma) * special.gammasgn(gamma - 1)
    out[1:] = sign * np.exp(logmag)
    return out


@pytest.mark.parametrize("gamma", GAMMAS + SUPER)
def test_psi_matches_gamma_function_closed_form(gamma):
    n = 50000
    ps = oracle.psi(gamma, n)
    ref = psi_closed_form(gamma, n)
    rel = np.abs(ps - ref) / np.abs(ref)
    assert rel.max() < 1e-9


@pytest.mark.parametrize("gamma", GAMMAS + SUPER)
def test_psi_small_m_matches_scipy_binomial(gamma):
    n = 30
    m = np.arange(n + 1)
    ref = (-1.0) ** m * special.binom(1.0 - gamma, m)
    np.testing.assert_allclose(oracle.psi(gamma, n), ref, rtol=1e-13, atol=0)


def test_psi_exact_values_at_gamma_half(golden_dir):
    rows = np.loadtxt(os.path.join(golden_dir, "psi_gamma_half.txt"))
    ps = oracle.psi(0.5, int(rows[-1, 0]))
    assert np.array_equal(ps[rows[:, 0].astype(int)], rows[:, 1])


@pytest.mark.parametrize("gamma", GAMMAS + SUPER)
def test_psi_partial_sums_closed_form(gamma):
    # sum_{j<=k} psi(j) is the k-th coefficient of (1-z)^(1-gamma)/(1-z) = (1-z)^(-gamma),
    # i.e. Gamma(k+gamma) / (Gamma(gamma) Gamma(k+1)).
    n = 50000
    cs = np.cumsum(oracle.psi(gamma, n))
    k = np.arange(n + 1, dtype=np.float64)
    ref = np.exp(special.gammaln(k + gamma) - special.gammaln(gamma) - special.gammaln(k + 1))
    assert (np.abs(cs - ref) / ref).max() < 1e-9


@pytest.mark.parametrize("gamma", GAMMAS + SUPER)
def test_psi_generating_function(gamma):
    # sum_m psi(gamma, m) z^m = (1 - z)^(1 - gamma) for |z| < 1.
    for z in (-0.5, 0.3, 0.5):
        ps = oracle.psi(gamma, 200)
        val = np.sum(ps * z ** np.arange(201))
        assert abs(val - (1 - z) ** (1 - gamma)) < 1e-14


@pytest.mark.parametrize("gamma", GAMMAS)
def test_psi_signs_and_decay(gamma):
    ps = oracle.psi(gamma, 5000)
    assert ps[0] == 1.0
    assert np.all(ps[1:] < 0)
    assert np.all(np.diff(np.abs(ps[1:])) < 0)   # |psi| decreases for m >= 1
    # asymptotics psi(m) ~ m^(gamma-2) / Gamma(gamma-1)
    m = 5000.0
    assert abs(ps[-1] / (m ** (gamma - 2) / special.gamma(gamma - 1)) - 1) < 2e-3


def test_psi_gamma_one_is_classical_diffusion():
    ps = oracle.psi(1.0, 1000)
    assert ps[0] == 1.0 and np.all(ps[1:] == 0.0)


@pytest.mark.parametrize("gamma", GAMMAS + SUPER)
def test_dpsi_digamma_closed_form(gamma):
    # d/dgamma of prod_{i=1}^m (i-2+gamma)/i = psi * (digamma(m-1+gamma) - digamma(gamma-1))
    n = 20000
    ps = oracle.psi(gamma, n)
    dps = oracle.dpsi(gamma, n)
    m = np.arange(1, n + 1, dtype=np.float64)
    ref = ps[1:] * (special.digamma(m - 1 + gamma) - special.digamma(gamma - 1))
    assert dps[0] == 0.0
    # (d psi(2)/d gamma = gamma - 1/2 vanishes at gamma = 1/2: an absolute floor covers it)
    assert np.all(np.abs(dps[1:] - ref) <= 1e-10 * np.abs(ref) + 1e-16)


@pytest.mark.parametrize("gamma", GAMMAS + SUPER)
def test_dpsi_central_difference(gamma):
    n, h = 3000, 1e-5
    fd = (oracle.psi(gamma + h, n) - oracle.psi(gamma - h, n)) / (2 * h)
    dps = oracle.dpsi(gamma, n)
    assert np.abs(fd - dps).max() / np.abs(dps).max() < 1e-8


def test_dpsi_at_gamma_one_is_harmonic():
    dps = oracle.dpsi(1.0, 10000)
    m = np.arange(1, 10001, dtype=np.float64)
    assert dps[0] == 0.0
    np.testing.assert_allclose(dps[1:], 1.0 / m, rtol=1e-12, atol=0)


@pytest.mark.parametrize("gamma", SUPER)
def test_psi_superdiffusion_signs_and_decay(gamma):
    # 1 - gamma < 0: (-1)^m binom(1 - gamma, m) = binom(gamma - 2 + m, m) > 0, decreasing in m,
    # with the same asymptotics m^(gamma-2) / Gamma(gamma-1) and a divergent sum.
    ps = oracle.psi(gamma, 5000)
    assert ps[0] == 1.0
    assert np.all(ps[1:] > 0)
    assert np.all(np.diff(ps) < 0)
    m = 5000.0
    assert abs(ps[-1] / (m ** (gamma - 2) / special.gamma(gamma - 1)) - 1) < 2e-3


def test_psi_gamma_two_is_all_ones():
    # binom(-1, m) (-1)^m = 1; d psi / d gamma = psi * sum_{i<=m} 1/(i-2+gamma) = H_m at gamma 2
    ps = oracle.psi(2.0, 1000)
    assert np.all(ps == 1.0)
    dps = oracle.dpsi(2.0, 1000)
    m = np.arange(1, 1001, dtype=np.float64)
    np.testing.assert_allclose(dps[1:], np.cumsum(1.0 / m), rtol=1e-12, atol=0)
