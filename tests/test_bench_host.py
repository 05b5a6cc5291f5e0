"""Host logic of bench.py, without a GPU: the launch plan it models for the in-block kernel,
the decomposition of every history MAC of a blocked solve into the block product, the
sub-block product and the in-block sums (each term counted once), the sine-mode projection
behind its parity figures, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1004_5128_amd import workloads as W  # noqa: E402


@pytest.fixture
def knobs(monkeypatch):
    def set_(fuse=None, sub=None):
        for name, v in (("GL_FUSE", fuse), ("GL_SUBBLOCK", sub)):
            if v is None:
                monkeypatch.delenv(name, raising=False)
            else:
                monkeypatch.setenv(name, str(v))
    return set_


@pytest.mark.parametrize("n,B,ndim,fuse,sub", [(700, 64, 2, None, None), (20000, 256, 2, None, None),
                                              (333, 32, 1, 3, None), (600, 512, 3, None, None),
                                              (257, 128, 2, 5, 0), (1000, 256, 2, 8, 64)])
def test_block_launches_cover_each_step_once(knobs, n, B, ndim, fuse, sub):
    knobs(fuse, sub)
    B2 = bench.sub_block(B)
    span = B2 or B
    limit = bench.fuse(ndim)
    assert limit == min(fuse or 8, 2 if ndim == 3 else 8)
    k = 0
    for start, s in bench.block_launches(n, B, ndim):
        assert start == k and 1 <= s <= limit
        # a launch never crosses a sub-block (or, with one level, a block)
        assert start // span == (start + s - 1) // span
        k += s
    assert k == n


@pytest.mark.parametrize("n,B,sub", [(1024, 256, None), (2048, 512, None), (768, 64, None),
                                     (512, 128, 0)])
def test_blocked_work_counts_every_history_term_once(knobs, n, B, sub):
    # full memory: step k sums k history rows (m >= 1).  On the blocked path the rows before
    # the block come from the block product, the block's rows before the sub-block from the
    # sub-block product, the rest from the in-block kernel.  With n a multiple of B the
    # products' MACs (flops / 6 per point) plus the in-block rows give sum_k k exactly.
    knobs(None, sub)
    P = 7
    terms = [k + 1 for k in range(n)]
    work = bench.algorithmic_work("toeplitz", P, n, B, terms)
    B2 = bench.sub_block(B)
    product = work["toeplitz"][1] / (6 * P)
    subblock = work.get("subblock", ("mfma", 0))[1] / (6 * P)
    inblock = sum(k % (B2 or B) for k in range(n))
    assert product + subblock + inblock == n * (n - 1) // 2
    # the plain path reads each of those rows once: 4 bytes per point and term
    assert work["hist_gemv"][1] == 4 * P * n * (n - 1) // 2


@pytest.mark.parametrize("ndim,shape,modes", [(2, (23, 17, 1), bench.MODES),
                                              (3, (9, 11, 7), bench.MODES3)])
def test_modal_projection_picks_out_each_sine_mode(ndim, shape, modes):
    # the discrete sine modes are orthogonal on the interior grid: the projection of mode j
    # is 1 at j and 0 at every other mode, so the bench's modal errors compare like with like
    p = W.problem(ndim, shape[0], 0.7, 1.0, 0.1)
    p["ny"] = shape[1]
    if ndim == 3:
        p["nz"] = shape[2]
    for j, m in enumerate(modes):
        u = W.sine_mode(p, m[0], m[1], 1.0, m[2] if ndim == 3 else 1)
        c = bench.modal(u, p, modes)
        expect = np.zeros(len(modes))
        expect[j] = 1.0
        np.testing.assert_allclose(c, expect, atol=1e-12)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
