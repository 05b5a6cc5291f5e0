"""Helpers shared by the GPU tests: run a workload through libgl and compare."""
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
