"""gl_autotune: the launch shapes it picks are among its candidates, it leaves the context at
step 0 with its initial fields, and runs after it still match the FP64 oracle (plain path
<= 1e-6, blocked path <= 1e-5, adjoint <= 1e-7), alone and in an ensemble."""
import numpy as np
import pytest
import torch

import oracle
from paper_1004_5128_amd import workloads as W
from gpu_util import gl, print_case, rel_l2

pytestmark = pytest.mark.gpu

GEMV_TARGETS = (256, 512, 1024, 2048, 4096)


@pytest.mark.parametrize("mem", [W.memory("full"), W.memory("adaptive", a=3)],
                         ids=["full", "adaptive3"])
def test_plain_path_autotune(mem):
    p = W.problem(2, 64, 0.7, 1.0, 0.1, rxn="linear", rate=0.2)
    u0 = W.gaussian(p, 50)
    n = 800
    G = gl()
    print_case("autotune plain", mem["mode"])
    with G.Solver(p, mem, torch.as_tensor(u0), max_steps=n) as s:
        g, w = s.autotune()
        assert g in GEMV_TARGETS and w in (1, 2, 4)
        assert s.k == 0 and np.array_equal(s.state().cpu().numpy(), u0)
        got = s.step(n).cpu().numpy()
    assert rel_l2(got, oracle.run(p, mem, u0, n)) <= 1e-6


@pytest.mark.parametrize("side,B", [(96, 256), (40, 128), (256, 256)])
def test_blocked_path_autotune(side, B):
    p = W.problem(2, side, 0.6, 0.5, 0.1, rxn="fisher", rate=1.0)
    u0 = W.uniform_field(p, 51)
    n = 1100 if side < 256 else 600
    G = gl()
    print_case("autotune blocked", side, B)
    with G.Solver(p, W.memory("full"), torch.as_tensor(u0), max_steps=n, sum_path="toeplitz",
                  block_B=B) as s:
        g, w = s.autotune()
        assert g in GEMV_TARGETS and w in (1, 2, 4)
        assert s.k == 0 and np.array_equal(s.state().cpu().numpy(), u0)
        got = s.step(n).cpu().numpy()
        # a reset run gives the same bits as the first run after tuning
        s.reset(torch.as_tensor(u0))
        again = s.step(n).cpu().numpy()
    assert np.array_equal(got, again)
    assert rel_l2(got, oracle.run(p, W.memory("full"), u0, n)) <= 1e-5


def test_autotune_state_errors():
    G = gl()
    p = W.problem(2, 16, 0.7, 1.0, 0.1)
    u0 = torch.as_tensor(W.gaussian(p, 52))
    with G.Solver(p, W.memory("full"), u0, max_steps=50) as s:
        with pytest.raises(G.GLError) as e:
            s.autotune(what=4)
        assert e.value.status == G.GL_EINVAL
        s.step(3)
        with pytest.raises(G.GLError) as e:
            s.autotune()
        assert e.value.status == G.GL_ESTATE
        s.reset(u0)
        s.autotune(what=G.GL_TUNE_GEMV)


def test_ensemble_and_adjoint_after_autotune():
    probs = [W.problem(2, 48, 0.5, 1.0, 0.1, rxn="linear", rate=0.3),
             W.problem(2, 20, 0.85, 0.8, 0.1, rxn="fisher", rate=0.6),
             W.problem(1, 500, 0.6, 1.0, 0.2)]
    u0s = [W.gaussian(probs[0], 53), W.uniform_field(probs[1], 54), W.sine_mode(probs[2], 2)]
    mem = W.memory("adaptive", a=2)
    n = 300
    G = gl()
    print_case("autotune ensemble + adjoint")
    u0 = np.concatenate(u0s)
    # targets at gamma + 0.05 with the same dt, dx: r = alpha dt^gamma / dx^2 shrinks (dt < 1),
    # so the target runs stay inside the stability bound
    targets = [oracle.run(dict(p, gamma=p["gamma"] + 0.05), mem, q, n) for p, q in zip(probs, u0s)]
    with G.Solver(probs, mem, torch.as_tensor(u0), max_steps=n, ckpt_every=40) as s:
        s.autotune()
        uT = s.step(n)
        du0, dpar = s.adjoint(uT - torch.as_tensor(np.concatenate(targets)).cuda())
        uT, du0, dpar = uT.cpu().numpy(), du0.cpu().numpy(), dpar.cpu().numpy()
    off = 0
    for i, (p, q) in enumerate(zip(probs, u0s)):
        P = W.npoints(p)
        assert rel_l2(uT[off:off + P], oracle.run(p, mem, q, n)) <= 1e-6
        _, du0r, dparr = oracle.adjoint(p, mem, q, n, targets[i])
        assert rel_l2(du0[off:off + P], du0r) <= 1e-7
        assert np.all(np.abs(dpar[i] - dparr) <= 1e-7 * np.abs(dparr)), (dpar[i], dparr)
        off += P


def test_blocked_autotune_on_a_large_3d_grid():
    # 64 x 64 x 32 = 131072 points: the default block length is 512 rows, whose product
    # targets half as many workgroups per CU; tuning, state and parity as above
    p = W.problem(3, 64, 0.7, 1.0, 0.05, rxn="linear", rate=0.2)
    p["nz"] = 32
    u0 = W.gaussian(p, 55)
    n = 1100
    G = gl()
    print_case("autotune blocked 3D", W.npoints(p))
    with G.Solver(p, W.memory("full"), torch.as_tensor(u0), max_steps=n,
                  sum_path="toeplitz") as s:
        g, w = s.autotune()
        assert g in GEMV_TARGETS and w in (1, 2, 4)
        assert s.k == 0 and np.array_equal(s.state().cpu().numpy(), u0)
        got = s.step(n).cpu().numpy()
    assert rel_l2(got, oracle.run(p, W.memory("full"), u0, n)) <= 1e-5


@pytest.mark.parametrize("path", ["gemv", "toeplitz"])
def test_autotune_on_a_one_step_context(path):
    # the candidates run at step max_steps / 2 = 0: one history row and checkpoints every
    # step; the context then takes its one step and matches the oracle
    p = W.problem(2, 12, 0.7, 1.0, 0.1)
    u0 = W.gaussian(p, 56)
    G = gl()
    with G.Solver(p, W.memory("full"), torch.as_tensor(u0), max_steps=1, ckpt_every=1,
                  sum_path=path) as s:
        s.autotune()
        got = s.step(1).cpu().numpy()
    assert rel_l2(got, oracle.run(p, W.memory("full"), u0, 1)) <= 1e-12
