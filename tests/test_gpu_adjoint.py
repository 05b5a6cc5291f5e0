"""The GPU adjoint sweep (gl_adjoint) against the FP64 oracle's adjoint, against central
finite differences of the GPU forward, checkpointed against single-segment recomputation
(bitwise), and through torch.autograd.  Tolerance vs FD: 1e-4."""
import numpy as np
import pytest
import torch

import oracle
from paper_1004_5128_amd import workloads as W
from gpu_util import gl, gpu_run, print_case, rel_l2

pytestmark = pytest.mark.gpu

TOL_FD = 1e-4


def gpu_adjoint(p, mem, u0, n, target, sum_path="gemv", ckpt_every=0, block_B=0):
    G = gl()
    with G.Solver(p, mem, torch.as_tensor(u0), max_steps=n, sum_path=sum_path,
                  ckpt_every=ckpt_every, block_B=block_B) as s:
        uT = s.step(n)
        tgt = torch.as_tensor(target).cuda()
        du0, dpar = s.adjoint(uT - tgt)
        loss = 0.5 * float(torch.sum((uT - tgt) ** 2))
        return loss, du0.cpu().numpy(), dpar[0].cpu().numpy()


CASES = [("linear", W.memory("full"), "gemv"), ("fisher", W.memory("full"), "gemv"),
         ("linear", W.memory("short", L=9), "gemv"), ("fisher", W.memory("full"), "toeplitz"),
         ("none", W.memory("full"), "toeplitz"), ("linear", W.memory("short", L=70), "toeplitz"),
         ("linear", W.memory("adaptive", a=2), "gemv"),
         ("fisher", W.memory("adaptive", a=3, rule="literal"), "gemv"),
         ("none", W.memory("adaptive", a=5), "gemv")]


@pytest.mark.parametrize("rxn,mem,path", CASES,
                         ids=["lin-full-gemv", "fisher-full-gemv", "lin-short-gemv",
                              "fisher-full-toeplitz", "none-full-toeplitz", "lin-short-toeplitz",
                              "lin-adaptive2-gemv", "fisher-adaptive3-literal-gemv",
                              "none-adaptive5-gemv"])
def test_adjoint_matches_oracle(rxn, mem, path):
    p = W.problem(2, 14, 0.7, 1.0, 0.05, rxn=rxn, rate=0.3)
    n = 300
    u0 = 0.5 * W.gaussian(p, 4) + 0.1
    target = oracle.run(dict(p, gamma=0.65, alpha=1.2), mem, u0, n)
    print_case("adjoint vs oracle", rxn, mem["mode"], path)
    L, du0, dpar = gpu_adjoint(p, mem, u0, n, target, sum_path=path, ckpt_every=64, block_B=64)
    Lr, du0r, dparr = oracle.adjoint(p, mem, u0, n, target)
    tol = 1e-7 if path == "gemv" else 1e-4
    assert abs(L - Lr) <= tol * Lr
    assert rel_l2(du0, du0r) <= tol
    assert np.all(np.abs(dpar - dparr) <= tol * np.abs(dparr) + 1e-12 * np.abs(dparr).max()), (dpar, dparr)


@pytest.mark.parametrize("path", ["gemv", "toeplitz"])
def test_checkpointed_equals_single_segment(path):
    p = W.problem(2, 20, 0.6, 1.0, 0.05, rxn="fisher", rate=1.0)
    n = 257
    u0 = W.uniform_field(p, 3)
    target = np.zeros_like(u0)
    print_case("checkpoints", path)
    a = gpu_adjoint(p, W.memory("full"), u0, n, target, sum_path=path, ckpt_every=10, block_B=32)
    b = gpu_adjoint(p, W.memory("full"), u0, n, target, sum_path=path, ckpt_every=n, block_B=32)
    assert a[0] == b[0]
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def test_adjoint_needs_a_run():
    G = gl()
    p = W.problem(2, 8, 0.7, 1.0, 0.05)
    u0 = torch.as_tensor(W.gaussian(p, 0)).cuda()
    for mem in (W.memory("full"), W.memory("adaptive", a=2)):
        with G.Solver(p, mem, u0, max_steps=10) as s:
            with pytest.raises(G.GLError) as e:
                s.adjoint(u0)
            assert e.value.status == G.GL_ESTATE


def test_adaptive_adjoint_after_longer_runs_matches_oracle():
    # the transposed schedule depends on the run length: gradients after 150 steps, then after
    # continuing to 420 (a longer transpose), then after a reset and 90 steps, each against
    # the oracle's adjoint of that run
    p = W.problem(2, 15, 0.6, 1.0, 0.08, rxn="linear", rate=0.4)
    mem = W.memory("adaptive", a=2)
    u0 = 0.5 * W.gaussian(p, 7) + 0.1
    G = gl()
    print_case("adaptive adjoint, several lengths")
    with G.Solver(p, mem, torch.as_tensor(u0), max_steps=420, ckpt_every=50) as s:
        for n, fresh in ((150, False), (420, False), (90, True)):
            if fresh:
                s.reset(torch.as_tensor(u0))
            uT = s.step(n - s.k)
            target = oracle.run(dict(p, gamma=0.55), mem, u0, n)
            du0, dpar = s.adjoint(uT - torch.as_tensor(target).cuda())
            Lr, du0r, dparr = oracle.adjoint(p, mem, u0, n, target)
            assert rel_l2(du0.cpu().numpy(), du0r) <= 1e-7, n
            assert np.all(np.abs(dpar[0].cpu().numpy() - dparr) <= 1e-7 * np.abs(dparr)), n


def _loss(p, mem, u0, n, target, path):
    u = gpu_run(p, mem, u0, n, sum_path=path)
    return 0.5 * float(np.sum((u - target) ** 2))


@pytest.mark.parametrize("path", ["gemv", "toeplitz"])
def test_cfg4_full_size_adjoint_vs_finite_differences(path):
    # 128^2, gamma 0.7, alpha 1, f = -0.2 u, 5000 steps, checkpoints every 500 steps; the
    # target is the same run at gamma 0.65, alpha 1.2.
    w = W.cfg4()
    p, mem, u0, n = w["problem"], w["memory"], w["u0"], w["nsteps"]
    print_case(w["name"], path)
    target = gpu_run(w["target_problem"], mem, u0, n, sum_path=path)
    L, du0, dpar = gpu_adjoint(p, mem, u0, n, target, sum_path=path, ckpt_every=w["ckpt_every"])
    # dL/drate is small (the run spans t = n dt = 6.5e-5, so the decay term barely acts): a
    # step of 1e-4 rate moves L by ~1e-9 relative, below the forward's rounding noise (BF16
    # products on the blocked path).  L depends on the rate through exp(-rate t), so the
    # central difference's error is ~(h t)^2 / 6 relative: a step of half the rate is exact
    # to ~1e-10 and keeps the difference far above the noise.
    # On the blocked path the forward carries BF16-product rounding (rel-L2 ~1e-9 per run),
    # which a 1e-4 step in alpha or gamma turns into ~1e-4 of FD noise; a 1e-3 step keeps the
    # truncation error (~h^2 ln(dt)^2 / 6, ~3e-5 for gamma) and the noise below 1e-4.
    big = 1e-3 if path == "toeplitz" else 1e-4
    for i, (key, rel) in enumerate((("alpha", big), ("gamma", big), ("rate", 0.5))):
        h = rel * p[key]
        fd = (_loss(dict(p, **{key: p[key] + h}), mem, u0, n, target, path) -
              _loss(dict(p, **{key: p[key] - h}), mem, u0, n, target, path)) / (2 * h)
        assert abs(fd - dpar[i]) <= TOL_FD * abs(fd), (key, fd, dpar[i])
    # f is linear, so L is exactly quadratic in u0 and the central difference is exact for any
    # step: a large one keeps the difference far above the forward's rounding noise
    v = w["direction"]
    h = 0.1
    fd = (_loss(p, mem, u0 + h * v, n, target, path) - _loss(p, mem, u0 - h * v, n, target, path)) / (2 * h)
    assert abs(fd - du0 @ v) <= TOL_FD * abs(fd), (fd, du0 @ v)
    if path == "toeplitz":
        # and it is the plain path's gradient up to the forward's rounding
        _, du0g, dparg = gpu_adjoint(p, mem, u0, n, target, sum_path="gemv",
                                     ckpt_every=w["ckpt_every"])
        assert rel_l2(du0, du0g) <= 1e-5
        assert np.all(np.abs(dpar - dparg) <= 1e-5 * np.abs(dparg)), (dpar, dparg)


def test_autograd_function_matches_gl_adjoint():
    from paper_1004_5128_amd.autograd import gl_solve
    p = W.problem(2, 16, 0.7, 1.0, 0.05, rxn="linear", rate=0.2)
    n = 200
    mem = W.memory("full")
    u0 = torch.as_tensor(W.gaussian(p, 4)).cuda().requires_grad_(True)
    alpha = torch.tensor(1.0, dtype=torch.float64, requires_grad=True)
    gamma = torch.tensor(0.7, dtype=torch.float64, requires_grad=True)
    rate = torch.tensor(0.2, dtype=torch.float64, requires_grad=True)
    target = torch.as_tensor(oracle.run(dict(p, gamma=0.65, alpha=1.2), mem, W.gaussian(p, 4), n)).cuda()
    print_case("autograd")
    uT = gl_solve(u0, alpha, gamma, rate, p, mem, n, ckpt_every=50)
    loss = 0.5 * torch.sum((uT - target) ** 2)
    loss.backward()
    Lr, du0r, dparr = oracle.adjoint(p, mem, W.gaussian(p, 4), n, target.cpu().numpy())
    assert rel_l2(u0.grad.cpu().numpy(), du0r) <= 1e-7
    got = np.array([alpha.grad.item(), gamma.grad.item(), rate.grad.item()])
    assert np.all(np.abs(got - dparr) <= 1e-7 * np.abs(dparr)), (got, dparr)
