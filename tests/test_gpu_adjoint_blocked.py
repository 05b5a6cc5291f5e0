"""The blocked path's reverse sweep: several reverse steps per launch on the in-block tiles,
with the mu rows since a sub-block's start summed point by point and the dot products of a
segment formed in one launch.  Against the FP64 oracle's adjoint on ragged 1D, 2D and 3D
grids, short windows narrower than a launch, one blocking level, superdiffusion and an
ensemble (tolerance 1e-5, the blocked forward's, 1e-4 for superdiffusion); and bit for bit against itself under every
grouping of the reverse steps into launches and checkpoint segments."""
import numpy as np
import pytest
import torch

import oracle
from paper_1004_5128_amd import workloads as W
from gpu_util import env, gl, print_case, rel_l2

pytestmark = pytest.mark.gpu

TOL_MFMA = 1e-5


def shaped(ndim, shape, gamma, r, rxn="none", rate=0.0):
    p = W.problem(ndim, shape[0], gamma, 1.0, r, rxn=rxn, rate=rate)
    if ndim >= 2:
        p["ny"] = shape[1]
    if ndim == 3:
        p["nz"] = shape[2]
    return p


def blocked_adjoint(probs, mem, u0, n, targets, ckpt_every, block_B):
    G = gl()
    with G.Solver(probs, mem, torch.as_tensor(u0), max_steps=n, sum_path="toeplitz",
                  ckpt_every=ckpt_every, block_B=block_B) as s:
        uT = s.step(n)
        tgt = torch.as_tensor(targets).cuda()
        du0, dpar = s.adjoint(uT - tgt)
        loss = 0.5 * float(torch.sum((uT - tgt) ** 2))
        return loss, du0.cpu().numpy(), dpar.cpu().numpy()


def param_bound(p, dparr, tol):
    """Allowed |error| of {dL/dalpha, dL/dgamma, dL/drate}: tol relative to each, except that
    dL/dgamma = r ln(dt) <lam, S> + r <lam, G> (the first term is ln(dt) alpha dL/dalpha) is
    held relative to the sum of its two terms' sizes, which cancel in places (by ~30 in the
    superdiffusive case); a floor of 1e-12 of the largest component (dL/drate is exactly 0
    without a reaction)."""
    t1 = np.log(p["dt"]) * p["alpha"] * dparr[0]
    scale = np.abs(dparr).astype(np.float64)
    scale[1] = abs(t1) + abs(dparr[1] - t1)
    return tol * scale + 1e-12 * np.abs(dparr).max()


def target_of(p, mem, u0, n):
    # the same run at gamma + 0.05 and alpha 0.6 alpha with the same dt and dx: r shrinks
    # (dt < 1), so the target stays inside the stability bound.  The target is far enough from
    # u[n] (a residual of 4 to 26 % of |u0|) that the blocked forward's rounding, relative to
    # the largest state, stays small against it also where the state has decayed a hundredfold
    # (superdiffusion)
    return oracle.run(dict(p, gamma=p["gamma"] + 0.05, alpha=0.6 * p["alpha"]), mem, u0, n)


# The superdiffusive case decays a hundredfold in 300 steps, so the forward's BF16-product
# rounding (relative to the largest state) reaches ~1e-5 of u[n]: its bar is the 1e-4 of the
# other blocked-adjoint tests.
CASES = [
    ("1d-ragged", (1, (300, 1, 1)), 0.6, 0.2, "fisher", W.memory("full"), 64, None, TOL_MFMA),
    ("2d-ragged-short3", (2, (21, 19, 1)), 0.8, 0.1, "linear", W.memory("short", L=3), 64, None,
     TOL_MFMA),
    ("2d-one-level", (2, (20, 20, 1)), 0.7, 0.1, "none", W.memory("full"), 128, 0, TOL_MFMA),
    ("3d-ragged-short40", (3, (9, 7, 6)), 0.7, 0.05, "linear", W.memory("short", L=40), 64, None,
     TOL_MFMA),
    ("2d-super1.5", (2, (18, 18, 1)), 1.5, 0.1, "none", W.memory("full"), 64, None, 1e-4),
]


@pytest.mark.parametrize("name,geom,gamma,r,rxn,mem,B,sub,tol", CASES, ids=[c[0] for c in CASES])
def test_blocked_adjoint_matches_oracle(name, geom, gamma, r, rxn, mem, B, sub, tol):
    ndim, shape = geom
    p = shaped(ndim, shape, gamma, r, rxn=rxn, rate=0.4)
    n = 300
    u0 = 0.5 * W.uniform_field(p, 71) + 0.1
    target = target_of(p, mem, u0, n)
    print_case("blocked adjoint", name)
    if sub is None:
        L, du0, dpar = blocked_adjoint(p, mem, u0, n, target, 50, B)
    else:
        with env("GL_SUBBLOCK", sub):
            L, du0, dpar = blocked_adjoint(p, mem, u0, n, target, 50, B)
    Lr, du0r, dparr = oracle.adjoint(p, mem, u0, n, target)
    e_u0 = rel_l2(du0, du0r)
    print("[err]", name, abs(L - Lr) / Lr, e_u0, np.abs(dpar[0] - dparr), dparr, flush=True)
    assert abs(L - Lr) <= tol * Lr
    assert e_u0 <= tol
    assert np.all(np.abs(dpar[0] - dparr) <= param_bound(p, dparr, tol)), (dpar[0], dparr)


def test_blocked_adjoint_of_an_ensemble():
    # two 2D members and a 1D member swept one after the other through the same buffers
    probs = [shaped(2, (17, 23), 0.55, 0.1, "linear", 0.3), shaped(2, (32, 16), 0.9, 0.1),
             shaped(1, (700,), 0.7, 0.2, "fisher", 0.5)]
    u0s = [W.gaussian(probs[0], 72), W.uniform_field(probs[1], 73), W.sine_mode(probs[2], 2)]
    mem = W.memory("full")
    n = 260
    targets = [target_of(p, mem, q, n) for p, q in zip(probs, u0s)]
    print_case("blocked adjoint ensemble")
    _, du0, dpar = blocked_adjoint(probs, mem, np.concatenate(u0s), n, np.concatenate(targets),
                                   40, 64)
    off = 0
    for i, (p, q) in enumerate(zip(probs, u0s)):
        P = W.npoints(p)
        _, du0r, dparr = oracle.adjoint(p, mem, q, n, targets[i])
        assert rel_l2(du0[off:off + P], du0r) <= TOL_MFMA
        assert np.all(np.abs(dpar[i] - dparr) <= param_bound(p, dparr, TOL_MFMA)), \
            (i, dpar[i], dparr)
        off += P


@pytest.mark.parametrize("ndim", [2, 3])
def test_blocked_adjoint_does_not_depend_on_grouping(ndim):
    # reverse steps per launch (1 .. 8, 2 at most in 3D) and checkpoint segments that cut
    # sub-blocks anywhere give the same bits: each chain runs in the same order
    p = shaped(ndim, (23, 21, 5), 0.75, 0.1 if ndim == 2 else 0.05, "fisher", 0.6)
    mem = W.memory("full")
    n = 211
    u0 = W.uniform_field(p, 74, 0.0, 0.5)
    target = np.zeros_like(u0)
    print_case("blocked adjoint grouping", ndim)
    outs = []
    # (n, 2): every launch takes two steps, the instantiation that once rounded differently
    for C, fuse in [(n, 8), (10, 8), (7, 3), (33, 1), (64, 5), (1, 2), (n, 2)]:
        with env("GL_FUSE", fuse):
            outs.append(blocked_adjoint(p, mem, u0, n, target, C, 64))
    for o in outs[1:]:
        assert o[0] == outs[0][0]
        assert np.array_equal(o[1], outs[0][1]) and np.array_equal(o[2], outs[0][2])
