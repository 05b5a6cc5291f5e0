"""Helpers shared by the GPU tests: run a workload through libgl and compare."""
import contextlib
import os

import numpy as np
import torch


def gl():
    from paper_1004_5128_amd import gl as _gl
    return _gl


def gpu_run(problem, memory, u0, nsteps, sum_path="gemv", block_B=0, max_steps=None, **kw):
    """u[nsteps] from libgl (numpy float64)."""
    G = gl()
    with G.Solver(problem, memory, torch.as_tensor(np.asarray(u0, np.float64)),
                  max_steps=max_steps or max(nsteps, 1), sum_path=sum_path, block_B=block_B,
                  **kw) as s:
        out = s.step(nsteps)
        torch.cuda.synchronize()
        return out.cpu().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def print_case(*args):
    print("[case]", *args, flush=True)


GEMV_GROUPS = 1024   # the library's default workgroup target of the history GEMV


def member_groups(P, P_total, groups=GEMV_GROUPS):
    """The GEMV workgroup target an ensemble gives a member of P points (its size share)."""
    return max(1, (groups * P + P_total - 1) // P_total)


@contextlib.contextmanager
def gemv_groups(value):
    """Run a solo problem with the split target an ensemble member gets (GL_GEMV_GROUPS)."""
    old = os.environ.get("GL_GEMV_GROUPS")
    os.environ["GL_GEMV_GROUPS"] = str(value)
    try:
        yield
    finally:
        if old is None:
            del os.environ["GL_GEMV_GROUPS"]
        else:
            os.environ["GL_GEMV_GROUPS"] = old


@contextlib.contextmanager
def env(name, value):
    """Set an environment variable the library reads when a solver is created."""
    old = os.environ.get(name)
    os.environ[name] = str(value)
    try:
        yield
    finally:
        if old is None:
            del os.environ[name]
        else:
            os.environ[name] = old
