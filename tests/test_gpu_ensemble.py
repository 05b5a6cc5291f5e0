"""The batched ensemble: 64 independent 2D problems of uneven sizes and different gamma,
alpha and decay rate, adaptive memory (a = 4, partition reading), 10000 steps, in one
context (one batched GEMV launch and one batched update launch per step).  Every member
starts as a discrete sine mode with a linear reaction, so the oracle's scalar recursion
gives each member's exact result.  The ensemble gives each member a share of the GEMV
workgroup target in proportion to its size; with that same target a solo run of the
member is bit-identical to it."""
import time

import numpy as np
import pytest
import torch

import oracle
from paper_1004_5128_amd import workloads as W
from gpu_util import gemv_groups, gl, gpu_run, member_groups, print_case, rel_l2

pytestmark = pytest.mark.gpu

TOL_PLAIN = 1e-6


def test_cfg5_ensemble_full_size():
    w = W.cfg5()
    probs, mem, n = w["problems"], w["memory"], w["nsteps"]
    sizes = [W.npoints(p) for p in probs]
    print_case(w["name"], len(probs), "problems", sum(sizes), "points", n, "steps")
    G = gl()
    u0 = torch.as_tensor(np.concatenate(w["u0s"]))
    with G.Solver(probs, mem, u0, max_steps=n) as s:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = s.step(n)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        macs = sum(sizes) * sum(s.schedule_terms(k) for k in range(n))
        print_case("ensemble solve %.3f s, %.3g history MACs/s" % (secs, macs / secs))
        out = out.cpu().numpy()
    off = 0
    worst = 0.0
    members = []
    for i, (p, (a, b)) in enumerate(zip(probs, w["modes"])):
        v = oracle.mode_run(p, mem, a, b, 1.0, n)
        got = out[off:off + sizes[i]]
        err = rel_l2(got, v[-1] * w["u0s"][i])
        worst = max(worst, err)
        assert err <= TOL_PLAIN, (i, p["nx"], err)
        members.append((off, sizes[i]))
        off += sizes[i]
    print_case("worst member rel-L2", worst)
    # members are bit-identical to their solo runs (smallest, a middle and the largest side)
    order = np.argsort([p["nx"] for p in probs], kind="stable")
    for i in (int(order[0]), int(order[len(order) // 2]), int(order[-1])):
        print_case("solo", i, probs[i]["nx"])
        o, sz = members[i]
        with gemv_groups(member_groups(sz, sum(sizes))):
            solo = gpu_run(probs[i], mem, w["u0s"][i], n)
        assert np.array_equal(solo, out[o:o + sz]), i


def test_small_ensemble_mixed_reactions_each_memory_mode():
    probs = [W.problem(2, 33, 0.35, 1.7, 0.1, rxn="linear", rate=0.45),
             W.problem(2, 65, 0.9, 0.6, 0.1, rxn="fisher", rate=1.0),
             W.problem(1, 500, 0.5, 1.0, 0.2),
             W.problem(2, 7, 0.6, 1.0, 0.1, rxn="linear", rate=0.1)]
    u0s = [W.gaussian(probs[0], 1), W.uniform_field(probs[1], 2), W.sine_mode(probs[2], 3),
           W.uniform_field(probs[3], 4)]
    n = 600
    for mem in (W.memory("full"), W.memory("short", L=50), W.memory("adaptive", a=3),
                W.memory("adaptive", a=2, rule="literal")):
        print_case("small ensemble", mem)
        G = gl()
        with G.Solver(probs, mem, torch.as_tensor(np.concatenate(u0s)), max_steps=n) as s:
            out = s.step(n).cpu().numpy()
        off = 0
        total = sum(W.npoints(p) for p in probs)
        for p, u0 in zip(probs, u0s):
            P = W.npoints(p)
            with gemv_groups(member_groups(P, total)):
                assert np.array_equal(out[off:off + P], gpu_run(p, mem, u0, n))
            assert rel_l2(out[off:off + P], oracle.run(p, mem, u0, n)) <= TOL_PLAIN
            off += P
