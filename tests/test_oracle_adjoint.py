"""Pins of the oracle's FP64 adjoint (gradient of 0.5||u[n] - target||^2 with respect
to u0, alpha, gamma and the reaction rate, dt and dx fixed) against central finite
differences of the oracle's own forward loss, for every memory mode."""
import numpy as np
import pytest

import oracle
from paper_1004_5128_amd import workloads as W


def loss(p, mem, u0, n, target):
    u = oracle.run(p, mem, u0, n)
    return 0.5 * float(np.sum((u - target) ** 2))


CASES = [
    (2, "linear", W.memory("full"), 0.7),
    (2, "fisher", W.memory("full"), 0.7),
    (1, "linear", W.memory("short", L=6), 0.7),
    (2, "linear", W.memory("adaptive", a=2), 0.7),
    (2, "fisher", W.memory("adaptive", a=3, rule="literal"), 0.7),
    (3, "fisher", W.memory("full"), 0.7),
    (2, "linear", W.memory("full"), 1.5),
    (1, "linear", W.memory("adaptive", a=2), 2.0),
]


@pytest.mark.parametrize("ndim,rxn,mem,gamma", CASES,
                         ids=lambda c: str(c) if not isinstance(c, dict) else c["mode"] + c["rule"])
def test_adjoint_matches_central_differences(ndim, rxn, mem, gamma):
    p = W.problem(ndim, 7, gamma, 1.0, 0.05, rxn=rxn, rate=0.3)
    n = 60
    u0 = W.gaussian(p, 4) * 0.5 + 0.1
    tp = dict(p, gamma=gamma - 0.05, alpha=1.2)
    target = oracle.run(tp, mem, u0, n)
    L, du0, dpar = oracle.adjoint(p, mem, u0, n, target)
    # the same P squared errors summed in two orders (sequential in C, pairwise in numpy)
    assert abs(L - loss(p, mem, u0, n, target)) <= 1e-13 * L

    for idx, key in enumerate(("alpha", "gamma", "rate")):
        h = 1e-5 * p[key]
        lp = loss(dict(p, **{key: p[key] + h}), mem, u0, n, target)
        lm = loss(dict(p, **{key: p[key] - h}), mem, u0, n, target)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - dpar[idx]) <= 1e-7 * abs(dpar[idx]) + 1e-14, (key, fd, dpar[idx])

    v = np.random.default_rng(44).standard_normal(u0.size)
    v /= np.linalg.norm(v)
    h = 1e-5
    fd = (loss(p, mem, u0 + h * v, n, target) - loss(p, mem, u0 - h * v, n, target)) / (2 * h)
    dd = float(du0 @ v)
    assert abs(fd - dd) <= 1e-7 * np.abs(du0).sum() * 1e-0 + 1e-14, (fd, dd)


def test_adjoint_of_linear_problem_is_the_transpose():
    # For f linear the run is u[n] = M u0 with M linear; the adjoint at target 0 returns
    # dL/du0 = M^T M u0, so <dL/du0, w> = <M u0, M w> for every w.
    p = W.problem(2, 6, 0.6, 1.0, 0.08, rxn="linear", rate=0.2)
    mem = W.memory("adaptive", a=2)
    n = 40
    rng = np.random.default_rng(3)
    u0, w = rng.standard_normal(36), rng.standard_normal(36)
    _, du0, _ = oracle.adjoint(p, mem, u0, n, np.zeros(36))
    Mu, Mw = oracle.run(p, mem, u0, n), oracle.run(p, mem, w, n)
    assert abs(du0 @ w - Mu @ Mw) < 1e-13 * abs(Mu @ Mw) + 1e-15
