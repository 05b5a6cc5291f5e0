"""Benchmark of the GL history-sum hot path on one MI355X.

Workload: 2D 256 x 256 grid, gamma 0.8, alpha 1, f = -0.1 u, Gaussian bump
sigma 0.1 plus seeded uniform noise (seed 2), r = 0.1, 20000 steps, full
memory.  One benchmark step is one whole solve (restart from u0, 20000 time
steps, each summing every stored state), with the inputs resident in device
memory.  The metric is history MACs/s: one MAC is one (weight x stored state)
term of a history sum, counted once per grid point.

Two history-sum paths are timed: the plain path (every step reads its
history rows once, FP32 loads, FP64 accumulation) and the blocked Toeplitz
path (blocks of B steps take the sum over the states before the block as
one BF16 hi/lo x 3 matrix product); the headline value is the last path.

Prints one JSON line.  Also reports, for each history-sum path, the relative
L2 error against the FP64 oracle on an 800-step prefix of the same workload,
the mode-by-mode error at full length (the workload is linear, so single
sine modes are sampled outputs the oracle computes exactly), the per-kernel
durations from HIP events, and the oracle's own throughput on the host.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 matrix, TFLOP/s
PREFIX_MACS = 4.72e10   # oracle sample: the first steps of the workload, about this many MACs


def default_block(P):
    """The library's block length for block_B = 0 (gl_problem docs): 512 rows from 131072
    points, else 256."""
    return 512 if P >= 131072 else 256


def grid_of(p):
    return [p["nx"], p["ny"]] + ([p["nz"]] if p["ndim"] == 3 else [])


def prefix_steps(P):
    """Steps of the oracle's prefix run for P points: 1200 at 256^2, 600 at 64^3."""
    return max(100, int(round(np.sqrt(2 * PREFIX_MACS / P) / 100)) * 100)


WORKLOADS = ("2d_256", "superdiffusion_2d", "diffusion_3d", "fisher_512", "ensemble64")
WORKLOAD_NAMES = {
    "2d_256": "2d_256x256_gamma0.8_alpha1_linear0.1_gaussian_r0.1_20000steps_full",
    "superdiffusion_2d": "2d_256x256_gamma1.5_alpha1_none_gaussian_r0.1_20000steps_full",
    "diffusion_3d": "3d_64x64x64_gamma0.8_alpha1_linear0.1_gaussian_r0.05_20000steps_full",
    "fisher_512": "2d_512x512_gamma0.6_alpha0.5_fisher1_uniform0.1_r0.1_50000steps_full",
    "ensemble64": "ensemble_64x2d_sides64-384_gamma0.3-0.95_linear_sine_r0.1_10000steps_adaptive_a4"}
ENSEMBLE_CPU_STEPS = 320   # oracle sample: every member's first 320 steps (about 4e10 MACs)
MODES = [(1, 1), (1, 3), (3, 1), (3, 3), (1, 5), (5, 5)]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


MODES3 = [(1, 1, 1), (1, 1, 3), (3, 1, 1), (1, 3, 3), (3, 3, 3)]


def modal(u, p, modes):
    """Sine-mode coefficients of a 2D or 3D field (discrete sine transform at the modes)."""
    from paper_1004_5128_amd import workloads as W
    x, y = W.coords(p["nx"]), W.coords(p["ny"])
    if p["ndim"] == 3:
        z = W.coords(p["nz"])
        U = np.asarray(u).reshape(p["nz"], p["ny"], p["nx"])
        return np.array([8.0 / ((p["nx"] + 1) * (p["ny"] + 1) * (p["nz"] + 1)) *
                         np.einsum("k,j,i,kji->", np.sin(c * np.pi * z), np.sin(b * np.pi * y),
                                   np.sin(a * np.pi * x), U) for a, b, c in modes])
    U = np.asarray(u).reshape(p["ny"], p["nx"])
    return np.array([4.0 / ((p["nx"] + 1) * (p["ny"] + 1)) *
                     (np.sin(b * np.pi * y) @ U @ np.sin(a * np.pi * x)) for a, b in modes])


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain device copy of known size, for scaling the HBM traffic counters."""
    import torch
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    log("copy calibration: %d x %d bytes read + written" % (reps, nbytes))


def source_sha(kernel):
    """SHA-256 of the HIP source holding a kernel (traffic counters are tied to it)."""
    import hashlib
    path = os.path.join(ROOT, "paper_1004_5128_amd", "csrc", KERNEL_SOURCES[kernel])
    return hashlib.sha256(open(path, "rb").read()).hexdigest()[:16]


KERNEL_SOURCES = {"hist_gemv": "gl_kernels.hip", "update": "gl_kernels.hip",
                  "toeplitz": "gl_toeplitz.hip", "old_reduce": "gl_toeplitz.hip",
                  "subblock": "gl_toeplitz.hip", "sub_reduce": "gl_toeplitz.hip",
                  "triangle": "gl_block.hip"}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.txt")


def measured_traffic():
    """{kernel: HBM bytes / algorithmic bytes} from the committed counter summary, for
    kernels whose source is unchanged since the counters were taken."""
    out = {}
    if not os.path.exists(TRAFFIC_FILE):
        return out
    for line in open(TRAFFIC_FILE):
        if line.startswith("kernel="):
            kv = dict(tok.split("=", 1) for tok in line.split())
            if kv.get("source_sha") == source_sha(kv["kernel"]):
                out[kv["kernel"]] = float(kv["traffic_over_algorithmic"])
    return out


def rocprof_name(kernel, B, B2):
    """The bench's name of a libgl kernel in a rocprofv3 record (the Toeplitz product kernel
    is the block product for B output rows and the sub-block product for B2), or None."""
    k = kernel.replace("void ", "")
    if k.startswith("gl::hist_gemv_kernel") or k.startswith("gl::hist_gemv_batched_kernel"):
        return "hist_gemv"
    if k.startswith("gl::update_kernel") or k.startswith("gl::update_batched_kernel"):
        return "update"
    if k.startswith("gl::toeplitz_gemm_kernel<%d>" % B):
        return "toeplitz"
    if B2 and k.startswith("gl::toeplitz_gemm_kernel<%d>" % B2):
        return "subblock"
    if k.startswith("gl::old_reduce_kernel"):
        return "old_reduce"
    if k.startswith("gl::block_steps_kernel"):
        return "triangle"
    return None


# solves of each path in a --profile-steps run: the timed solve and the profiled one
PROFILE_SOLVES = 2


def summarize_counters(fetch_csv, write_csv, work, B):
    """Lines of the traffic summary from two rocprofv3 counter CSVs (FETCH_SIZE, WRITE_SIZE, KiB
    per dispatch) of a --profile-steps run with --copy-calibration; `work` is that run's
    algorithmic work.  Each counter is scaled by what it reads for the 1 GiB device copy."""
    import collections
    import csv

    def per_kernel(path, counter):
        vals, copies = collections.defaultdict(list), []
        for row in csv.DictReader(open(path)):
            if row["Counter_Name"] != counter:
                continue
            v = float(row["Counter_Value"])
            if "copyBuffer" in row["Kernel_Name"] and int(row["Grid_Size"]) >= 131072:
                copies.append(v)
            name = rocprof_name(row["Kernel_Name"], B, sub_block(B))
            if name:
                vals[name].append(v)
        return vals, copies

    fetch, fcopy = per_kernel(fetch_csv, "FETCH_SIZE")
    write, wcopy = per_kernel(write_csv, "WRITE_SIZE")
    gib_kib = float(1 << 20)
    ff, wf = (sum(fcopy) / len(fcopy)) / gib_kib, (sum(wcopy) / len(wcopy)) / gib_kib
    lines = ["# copy calibration: a 1 GiB device copy reads FETCH_SIZE %.4f GiB, WRITE_SIZE %.4f GiB"
             % (ff, wf)]
    for name in sorted(fetch):
        n = len(fetch[name])
        hbm = (sum(fetch[name]) / n / ff + sum(write[name]) / len(write[name]) / wf) * 1024
        kind, w = work.get(name + "_bytes", work.get(name, (None, None)))
        if kind != "hbm":
            continue
        # `work` covers one solve; the counted launches span PROFILE_SOLVES solves
        alg = w * PROFILE_SOLVES / n
        lines.append("kernel=%s source_sha=%s launches=%d fetch_kib_per_launch=%.1f "
                     "write_kib_per_launch=%.1f hbm_bytes_per_launch=%.0f "
                     "algorithmic_bytes_per_launch=%.0f traffic_over_algorithmic=%.4f"
                     % (name, source_sha(name), n, sum(fetch[name]) / n,
                        sum(write[name]) / len(write[name]), hbm, alg, hbm / alg))
    return lines


def sub_block(B):
    """The library's sub-block length for block length B (GL_SUBBLOCK, default 32; 0: none)."""
    B2 = int(os.environ.get("GL_SUBBLOCK", "32"))
    return B2 if 0 < B2 < B and B % B2 == 0 else 0


def compute_units():
    """Compute units of GPU 0 (MI355X: 256 when summarizing counters without a GPU)."""
    import torch
    if torch.cuda.is_available():
        return torch.cuda.get_device_properties(0).multi_processor_count
    return 256


def toeplitz_chunks(rows, BM, P):
    """Chunks of a Toeplitz product over `rows` history rows, as the library cuts it: rows of
    GL_TOEPLITZ_KCHUNK if set, else the fewest chunks whose workgroups (128-point column
    tiles x chunks) fill the GPU, two per CU (one for the 512-row block)."""
    v = os.environ.get("GL_TOEPLITZ_KCHUNK")
    if v:
        kc = max(128, int(v) // 128 * 128)
    else:
        tiles = -(-P // 128)
        ncu = compute_units()
        target = ncu * (1 if BM >= 512 else 2)
        n = max(1, min(-(-target // tiles), -(-rows // 128)))
        kc = -(-(-(-max(rows, 1) // n)) // 128) * 128
    return -(-rows // kc) if rows > 0 else 0


def fuse(ndim=2):
    """In-block steps per launch (GL_FUSE, default 8; at most 2 on 3D grids)."""
    v = os.environ.get("GL_FUSE")
    f = min(8, max(1, int(v))) if v else 8
    return min(f, 2) if ndim == 3 else f


def block_launches(n, B, ndim=2):
    """(first step, steps) of each in-block launch of an n-step run, as the library groups them:
    at most fuse() steps, never across a sub-block (a block with one level)."""
    B2 = sub_block(B)
    out, k = [], 0
    while k < n:
        left = B2 - (k % B) % B2 if B2 else B - k % B
        s = max(1, min(fuse(ndim), n - k, left))
        out.append((k, s))
        k += s
    return out


def algorithmic_work(path, P, n, B, terms, ndim=2):
    """Algorithmic work of each kernel over one solve of n steps (see the design notes):
     hist_gemv:  every history row of terms m >= 1 read once, 4 bytes per point
     update:     u[k] read, u[k+1] and the FP32 history row k written (20 bytes per point)
     toeplitz:   6 flops (three BF16 products) per (block row, history row, point); its HBM
                 side: history rows read once, then FP32 chunk products written, or the FP64
                 sums themselves when the rows fit one chunk
     triangle:   one in-block launch of s steps: the sub-block's rows before the launch (4
                 bytes each), u read and written once, s history rows written, the s rows of
                 the block sums read (8 bytes) once any exist
     subblock:   the product over a block's rows before a sub-block (as toeplitz), its FP64
                 sums written, the block sums of its rows read as their base
     old_reduce, sub_reduce: the FP32 chunk products read, the FP64 sums written (only
                 for products of more than one chunk)"""
    work = {"hist_gemv": ("hbm", 4 * P * sum(t - 1 for t in terms)),
            "update": ("hbm", 20 * P * n)}
    if path == "toeplitz":
        blocks = range(B, n, B)
        B2 = sub_block(B)
        chunks = lambda rows, BM=B: toeplitz_chunks(rows, BM, P)
        work["toeplitz"] = ("mfma", 6 * B * P * sum(blocks))
        work["toeplitz_bytes"] = ("hbm", P * sum(4 * k0 + (8 * B if chunks(k0) == 1 else
                                                           4 * B * chunks(k0)) for k0 in blocks))
        tri = 0
        for k, s in block_launches(n, B, ndim):
            b = k % B
            b2 = b % B2 if B2 else b
            has_pre = k >= B or b - b2 > 0
            tri += 4 * b2 + 16 + 4 * s + (8 * s if has_pre else 0)
        work["triangle"] = ("hbm", P * tri)
        multi = [k0 for k0 in blocks if chunks(k0) > 1]
        if multi:
            work["old_reduce"] = ("hbm", B * P * sum(4 * chunks(k0) + 8 for k0 in multi))
        if B2:
            # sub-block products: rows k0 .. k1-1 for every sub-block start k1 > k0 (< n)
            starts = [k1 for k1 in range(B2, n, B2) if k1 % B]
            work["subblock"] = ("mfma", 6 * B2 * P * sum(k1 % B for k1 in starts))
            base = lambda k1: 8 * B2 if k1 >= B else 0   # block sums read as the base
            work["subblock_bytes"] = ("hbm", P * sum(
                4 * (k1 % B) + (8 * B2 + base(k1) if chunks(k1 % B, B2) == 1 else
                                4 * B2 * chunks(k1 % B, B2)) for k1 in starts))
            multi2 = [k1 for k1 in starts if chunks(k1 % B, B2) > 1]
            if multi2:
                work["sub_reduce"] = ("hbm", P * sum(B2 * (4 * chunks(k1 % B, B2) + 8) + base(k1)
                                                     for k1 in multi2))
    return work


def run_path(path, w, steps, warmup, block_B, prefix=True, nsteps=None):
    """One history-sum path on workload w: `steps` timed solves after `warmup`, one solve
    with per-kernel events, and (prefix) the state after the oracle's prefix length."""
    import torch
    from paper_1004_5128_amd import gl
    p = w["problem"]
    n = nsteps or w["nsteps"]
    P = gl.npoints(p)
    u0 = torch.as_tensor(w["u0"], dtype=torch.float64).cuda()
    s = gl.Solver(p, w["memory"], u0, max_steps=n, sum_path=path, block_B=block_B)
    B = block_B or default_block(P)
    terms = [s.schedule_terms(k) for k in range(n)]
    macs = P * sum(terms)
    work = algorithmic_work(path, P, n, B, terms, p["ndim"])
    def solve():
        # long runs advance in pieces with a progress line each (calls split anywhere give
        # the same results)
        piece = n if n <= 20000 else 10000
        for k in range(0, n, piece):
            s.advance(min(piece, n - k))
            if piece < n:
                log(path, "step", min(k + piece, n), "of", n)

    for i in range(warmup):
        log(path, "warmup", i)
        s.reset(u0)
        solve()
    torch.cuda.synchronize()
    log(path, "timed", steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        s.reset(u0)
        solve()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    uT = s.state().cpu().numpy()
    # per-kernel durations: one more solve with HIP events stamped at each kernel's start
    # and end (kernels launched one by one, so no graph replay in this solve)
    log(path, "profiled solve")
    s.set_profiling(True)
    s.reset(u0)
    solve()
    torch.cuda.synchronize()
    prof = s.profile()
    s.set_profiling(False)
    u_prefix = None
    if prefix:   # prefix run for the oracle comparison
        s.reset(u0)
        s.advance(prefix_steps(P))
        u_prefix = s.state().cpu().numpy()
    s.close()
    ms = (t1 - t0) * 1e3 / steps
    return {"ms_per_step": ms, "macs": macs, "work": work, "prof": prof, "uT": uT,
            "u_prefix": u_prefix, "steps": 1}


MODE_RUNS = (("short_L1000", "gemv", {"mode": "short", "L": 1000}),
             ("short_L1000_blocked", "toeplitz", {"mode": "short", "L": 1000}),
             ("adaptive_a2", "gemv", {"mode": "adaptive", "a": 2}),
             ("adaptive_a4", "gemv", {"mode": "adaptive", "a": 4}),
             ("adaptive_a10", "gemv", {"mode": "adaptive", "a": 10}))


def run_memory_modes(w, u_full, oracle_modes):
    """The same workload under short memory (L = 1000 steps; plain and blocked paths) and
    adaptive memory (a = 2, 4, 10, partition reading; plain path): time per solve (one warmup,
    one timed, then one more after gl_autotune), history MACs/s and, on the plain path,
    algorithmic GB/s, the rel-L2
    difference from the full-memory result (the paper's error of a memory mode) and, with the
    oracle, the largest sine-mode error against the oracle's recursion for that mode."""
    import torch
    from paper_1004_5128_amd import gl, workloads as W
    p, n = w["problem"], w["nsteps"]
    P = W.npoints(p)
    u0 = torch.as_tensor(w["u0"], dtype=torch.float64).cuda()
    out = {}
    for name, path, spec in MODE_RUNS:
        mem = W.memory(spec["mode"], **{k: v for k, v in spec.items() if k != "mode"})
        log("memory mode", name)
        with gl.Solver(p, mem, u0, max_steps=n, sum_path=path) as s:
            terms = sum(s.schedule_terms(k) for k in range(n))
            s.advance(n)
            torch.cuda.synchronize()
            s.reset(u0)
            t0 = time.perf_counter()
            s.advance(n)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            uT = s.state().cpu().numpy()
            # the same solve after gl_autotune picked the launch shapes for this schedule
            s.reset(u0)
            tuned = s.autotune()
            s.reset(u0)
            t0 = time.perf_counter()
            s.advance(n)
            torch.cuda.synchronize()
            dt_tuned = time.perf_counter() - t0
        d = {"path": path, "ms_per_solve": dt * 1e3, "history_macs_per_solve": P * terms,
             "history_macs_per_s": P * terms / dt,
             "ms_per_solve_autotuned": dt_tuned * 1e3,
             "autotuned": {"gemv_groups": tuned[0], "product_chunk_wgs": tuned[1]},
             "rel_l2_vs_full_memory": float(np.linalg.norm(uT - u_full) / np.linalg.norm(u_full))}
        if path == "gemv":
            d["algorithmic_gbs"] = 4 * P * (terms - n) / dt / 1e9
        if oracle_modes is not None:
            import oracle
            c0 = modal(w["u0"], p, MODES)
            ref = np.array([c0[i] * oracle.mode_run(p, mem, a, b, 1.0, n)[-1]
                            for i, (a, b) in enumerate(MODES)])
            cg = modal(uT, p, MODES)
            d["modal_err_vs_oracle"] = float(np.abs(cg - ref).max() / np.abs(ref).max())
        out[name] = d
    return out


def roofline_of(kind, work_per_solve, launches_per_solve, ms_per_solve):
    """Achieved rate of one kernel: algorithmic work per launch / average launch time."""
    per_launch = work_per_solve / launches_per_solve
    avg_s = ms_per_solve / launches_per_solve * 1e-3
    if kind == "mfma":
        achieved = per_launch / avg_s / 1e12
        return {"bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / BF16_PEAK_TFLOPS, "traffic": None,
                "algorithmic_flops_per_launch": per_launch, "avg_launch_us": avg_s * 1e6}
    achieved = per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": None,
            "algorithmic_bytes_per_launch": per_launch, "avg_launch_us": avg_s * 1e6}


def probe_product(k, reps=3):
    """The block product alone: gl_history_sum at step k (B = 256, so the product covers the
    k0 = k - k % 256 rows before the block, plus a short GEMV) over a synthetic FP32 history
    of 65536 points, timed `reps` times; for counter collection on the product kernel."""
    import torch
    from paper_1004_5128_amd import gl, workloads as W
    P = 65536
    gen = torch.Generator(device="cuda").manual_seed(5)
    H = torch.rand((k + 1, P), dtype=torch.float32, device="cuda", generator=gen) * 0.1
    p = W.problem(1, P, 0.8, 1.0, 0.05)
    out = []
    with gl.Solver(p, W.memory("full"), np.zeros(P), max_steps=k, sum_path="toeplitz") as s:
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.history_sum(k, H)
            torch.cuda.synchronize()
            out.append((time.perf_counter() - t0) * 1e3)
    print(json.dumps({"probe": "toeplitz product", "k": k, "points": P, "ms": out}), flush=True)


def paper_fig3(reps=2):
    """The short- vs adaptive-memory comparison of Sec. 3.2 (the experiment of its Fig. 3) on
    the GPU's plain path: for each of four gamma values, full memory and short (L) and
    adaptive (a) memory sweeps, each with its history terms, GPU time per run (best of
    `reps`, after one warmup) and its error relative to full memory.  At 400 points a run is
    bound by its 3000 launches, so the term count is the cost to read the trade-off by."""
    import torch
    from paper_1004_5128_amd import gl, workloads as W
    out = {}
    for gamma in (0.5, 0.75, 0.9, 0.95):
        w = W.paper_fig3(gamma)
        p, n = w["problem"], w["nsteps"]
        u0 = torch.as_tensor(w["u0"], dtype=torch.float64).cuda()
        rows, full = [], None
        mems = ([("full", 0, W.memory("full"))] +
                [("short", L, W.memory("short", L=L)) for L in (10, 25, 50, 100, 200, 400, 800)] +
                [("adaptive", a, W.memory("adaptive", a=a)) for a in (2, 3, 4, 6, 10, 20)])
        for mode, par, mem in mems:
            with gl.Solver(p, mem, u0, max_steps=n) as s:
                terms = sum(s.schedule_terms(k) for k in range(n))
                s.advance(n)
                best = None
                for _ in range(reps):
                    s.reset(u0)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    s.advance(n)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    best = dt if best is None else min(best, dt)
                uT = s.state().cpu().numpy()
            if full is None:
                full = uT
            rows.append({"mode": mode, "param": par, "history_terms": terms,
                         "gpu_ms": best * 1e3,
                         "error_vs_full_pct": 100 * float(np.linalg.norm(uT - full) /
                                                          np.linalg.norm(full))})
        out["gamma_%g" % gamma] = rows
    print(json.dumps({"probe": "paper fig3 (short vs adaptive memory)", "results": out}),
          flush=True)


def run_adjoint_leg():
    """The adjoint workload (2D 128^2, gamma 0.7, alpha 1, f = -0.2 u, 5000 steps, checkpoints
    every 500 steps; target: the same run at gamma 0.65, alpha 1.2) on both paths: forward
    and gl_adjoint times (one warmup each), and the directional derivative <dL/du0, v>
    against a central difference of the GPU loss (exact for a quadratic loss of a linear
    scheme, step 0.1)."""
    import torch
    from paper_1004_5128_amd import gl, workloads as W
    w = W.cfg4()
    p, mem, n = w["problem"], w["memory"], w["nsteps"]
    u0 = torch.as_tensor(w["u0"]).cuda()
    v = torch.as_tensor(w["direction"]).cuda()
    out = {}
    for path in ("gemv", "toeplitz"):
        log("adjoint", path)
        with gl.Solver(w["target_problem"], mem, u0, max_steps=n, sum_path=path) as s:
            target = s.step(n).clone()

        def loss(x):
            with gl.Solver(p, mem, x, max_steps=n, sum_path=path) as s2:
                return 0.5 * float(torch.sum((s2.step(n) - target) ** 2))

        with gl.Solver(p, mem, u0, max_steps=n, sum_path=path,
                       ckpt_every=w["ckpt_every"]) as s:
            times = []
            for _ in range(2):   # the first of each is the warmup
                s.reset(u0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                uT = s.step(n)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                du0, dpar = s.adjoint(uT - target)
                torch.cuda.synchronize()
                t2 = time.perf_counter()
                times.append((t1 - t0, t2 - t1))
        fd = (loss(u0 + 0.1 * v) - loss(u0 - 0.1 * v)) / 0.2
        out[path] = {"forward_ms": times[-1][0] * 1e3, "adjoint_ms": times[-1][1] * 1e3,
                     "adjoint_over_forward": times[-1][1] / times[-1][0],
                     "directional_derivative_rel_err_vs_fd":
                         abs(float(du0 @ v) - fd) / abs(fd)}
    return out


def run_extra_workloads(block_B, with_oracle):
    """Superdiffusion (2D 256^2, gamma 1.5) and a 3D grid (64^3, 7-point stencil), 20000 steps
    each, full memory, on the blocked path: time per solve (one warmup, one timed), history
    MACs/s, the dominant kernel's roofline from a profiled solve and, with the oracle, the
    largest error of a few sine-mode coefficients at the last step against the oracle's mode
    recursion, relative to the largest initial coefficient (the scale of the history terms)."""
    from paper_1004_5128_amd import workloads as W
    out = {}
    for w, modes in ((W.superdiffusion_2d(), MODES), (W.diffusion_3d(), MODES3)):
        p, n = w["problem"], w["nsteps"]
        log("workload", w["name"])
        r = run_path("toeplitz", w, 1, 1, block_B, prefix=False)
        d = {"ms_per_solve": r["ms_per_step"], "history_macs_per_solve": r["macs"],
             "value": r["macs"] / (r["ms_per_step"] / 1e3), "unit": "history MACs/s",
             "grid": grid_of(p),
             "gamma": p["gamma"], "time_steps": n}
        kern = {}
        for name, (cnt, ms) in r["prof"].items():
            if cnt:
                kern[name] = {"launches": cnt, "ms_per_solve": ms, "avg_us": ms * 1e3 / cnt}
                if name in r["work"]:
                    kind, work = r["work"][name]
                    kern[name]["roofline"] = roofline_of(kind, work, cnt, ms)
        d["kernels"] = kern
        if with_oracle:
            import oracle
            c0 = modal(w["u0"], p, modes)
            ref = np.array([c0[i] * oracle.mode_run(p, w["memory"], m[0], m[1], 1.0, n,
                                                    s=m[2] if len(m) > 2 else 1)[-1]
                            for i, m in enumerate(modes)])
            d["modal_err_vs_oracle_full_length"] = float(
                np.abs(modal(r["uT"], p, modes) - ref).max() / np.abs(c0).max())
        out[w["name"]] = d
    return out


def run_ensemble(args):
    """The batched ensemble: 64 2D problems (sides 64 .. 384, 3 489 792 points), gamma, alpha
    and reaction rate drawn per member, sine-mode initial states, adaptive memory (a = 4),
    10 000 steps on the plain path, where each step is one batched GEMV and one batched update
    launch over all members.  Prints the contract's line: history MACs/s of the timed solves,
    the GEMV's roofline from a profiled solve, each member against the oracle's sine-mode
    recursion over the full length and against the oracle's run over a prefix, and the
    oracle's own rate on that prefix (every member, ENSEMBLE_CPU_STEPS steps)."""
    import torch
    from paper_1004_5128_amd import gl, workloads as W
    w = W.cfg5()
    probs, mem, n = w["problems"], w["memory"], w["nsteps"]
    sizes = [W.npoints(p) for p in probs]
    P = sum(sizes)
    u0 = torch.as_tensor(np.concatenate(w["u0s"]), dtype=torch.float64).cuda()
    s = gl.Solver(probs, mem, u0, max_steps=n)
    terms = [s.schedule_terms(k) for k in range(n)]   # the schedule depends on k only
    macs = P * sum(terms)
    work = {"hist_gemv": ("hbm", 4 * P * sum(t - 1 for t in terms)),
            "update": ("hbm", 20 * P * n)}
    for i in range(args.warmup):
        log("ensemble warmup", i)
        s.reset(u0)
        s.advance(n)
    torch.cuda.synchronize()
    log("ensemble timed", args.steps)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.reset(u0)
        s.advance(n)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    uT = s.state().cpu().numpy()
    log("ensemble profiled solve")
    s.set_profiling(True)
    s.reset(u0)
    s.advance(n)
    torch.cuda.synchronize()
    prof = s.profile()
    s.set_profiling(False)
    n_cpu = min(ENSEMBLE_CPU_STEPS, n)
    s.reset(u0)
    s.advance(n_cpu)
    u_pre = s.state().cpu().numpy()
    s.close()
    kernels = {}
    for name, (cnt, kms) in prof.items():
        if cnt:
            kd = {"launches": cnt, "ms_per_solve": kms, "avg_us": kms * 1e3 / cnt}
            if name in work:
                kd["roofline"] = roofline_of(work[name][0], work[name][1], cnt, kms)
            kernels[name] = kd
    roofline = dict(kernels["hist_gemv"]["roofline"], kernel="hist_gemv")
    d = {"ms_per_step": ms, "value": macs / (ms / 1e3), "kernels": kernels,
         "traffic_note": "no counter run on this workload: traffic is null"}
    cpu = None
    if not args.no_cpu:
        import oracle
        log("oracle: every member,", n_cpu, "steps, and the sine-mode recursions")
        worst_pre = worst_mode = 0.0
        t_cpu = 0.0
        off = 0
        for i, (p, (a, b)) in enumerate(zip(probs, w["modes"])):
            t1 = time.perf_counter()
            ref = oracle.run(p, mem, w["u0s"][i], n_cpu)
            t_cpu += time.perf_counter() - t1
            got = u_pre[off:off + sizes[i]]
            worst_pre = max(worst_pre, float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
            v = oracle.mode_run(p, mem, a, b, 1.0, n)[-1] * w["u0s"][i]
            got = uT[off:off + sizes[i]]
            worst_mode = max(worst_mode, float(np.linalg.norm(got - v) / np.linalg.norm(v)))
            off += sizes[i]
        d["worst_member_rel_l2_vs_oracle_prefix"] = worst_pre
        d["worst_member_rel_l2_vs_oracle_mode_full_length"] = worst_mode
        macs_cpu = P * sum(terms[:n_cpu])
        cpu = {"value": macs_cpu / t_cpu, "unit": "history MACs/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "first %d of the %d steps of every member of the same ensemble (%.3g "
                         "MACs, %.1f s)" % (n_cpu, n, macs_cpu, t_cpu)}
    line = {
        "metric": "history MACs/s + rel-L2 vs FP64 oracle; plain FP32 sum vs blocked MFMA sum",
        "value": macs / (ms / 1e3), "unit": "history MACs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 history, f64 accumulate", "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES["ensemble64"], "problems": len(probs),
                   "points": P, "time_steps": n, "memory": "adaptive a=4",
                   "history_macs_per_solve": macs, "path": "gemv"},
        "paths": {"gemv": d},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


def probe_hipblaslt(reps=10):
    """Vendor BF16 GEMMs (torch.matmul -> hipBLASLt) on the same GPU for comparison: square
    4096..16384 and the block product's shape (256 x 19968) x (19968 x 65536)."""
    import torch
    res = {}
    for m, kk, n in ((4096, 4096, 4096), (8192, 8192, 8192), (16384, 16384, 16384),
                     (256, 19968, 65536)):
        a = torch.randn(m, kk, dtype=torch.bfloat16, device="cuda")
        b = torch.randn(kk, n, dtype=torch.bfloat16, device="cuda")
        for _ in range(2):
            c = a @ b
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            c = a @ b
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        res["%dx%dx%d" % (m, kk, n)] = {"ms": dt * 1e3, "tflops": 2 * m * kk * n / dt / 1e12}
        del a, b, c
    print(json.dumps({"probe": "hipblaslt bf16", "gemms": res}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--paths", default="gemv,toeplitz",
                    help="history-sum paths to time; the last one is the headline value")
    ap.add_argument("--block-B", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle legs")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the short / adaptive memory runs of the same workload")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the superdiffusion and 3D workloads")
    ap.add_argument("--workload", choices=WORKLOADS, default="2d_256",
                    help="the headline workload (default: 2D 256^2, gamma 0.8); the others run "
                         "without the memory-mode and extra-workload legs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a 1 GiB device copy (reference for traffic counters)")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="short run for counter collection: one solve of this many steps per "
                         "path, no warmup, no oracle")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="print the traffic summary lines from the counter CSVs of a "
                         "--profile-steps run of the given --paths (no GPU)")
    ap.add_argument("--probe-product", type=int, default=0, metavar="K",
                    help="time the block product alone at step K (for counter collection)")
    ap.add_argument("--probe-hipblaslt", action="store_true",
                    help="time vendor BF16 GEMMs (torch.matmul) for comparison")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the adjoint leg and print its JSON (for kernel traces)")
    ap.add_argument("--paper-fig3", action="store_true",
                    help="the paper's short vs adaptive memory comparison (Sec. 3.2)")
    args = ap.parse_args()
    if args.paper_fig3:
        import torch
        torch.cuda.set_device(0)
        paper_fig3()
        return
    if args.probe_product or args.probe_hipblaslt:
        import torch
        torch.cuda.set_device(0)
        if args.probe_product:
            probe_product(args.probe_product)
        if args.probe_hipblaslt:
            probe_hipblaslt()
        return
    if args.summarize_counters:
        from paper_1004_5128_amd import workloads as W
        w = W.cfg2()
        n = args.profile_steps or w["nsteps"]
        for path in [x for x in args.paths.split(",") if x]:
            work = algorithmic_work(path, W.npoints(w["problem"]), n,
                                    args.block_B or default_block(W.npoints(w["problem"])),
                                    [k + 1 for k in range(n)])
            print("\n".join(summarize_counters(*args.summarize_counters, work,
                                                args.block_B or
                                                default_block(W.npoints(w["problem"])))))
        return
    if args.gpus != 1:
        print("bench.py: measures one GPU only (the solver runs on a single "
              "MI355X); --gpus %d is not supported" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.adjoint_only:
        print(json.dumps({"adjoint_128x128_5000steps": run_adjoint_leg()}), flush=True)
        return
    if args.workload == "ensemble64":
        run_ensemble(args)
        return

    import torch
    from paper_1004_5128_amd import workloads as W
    torch.cuda.set_device(0)
    w = {"2d_256": W.cfg2, "superdiffusion_2d": W.superdiffusion_2d,
         "diffusion_3d": W.diffusion_3d, "fisher_512": W.cfg3}[args.workload]()
    p, n = w["problem"], w["nsteps"]
    P = W.npoints(p)
    modes = MODES3 if p["ndim"] == 3 else MODES
    if args.workload != "2d_256":
        args.no_modes = args.no_extra = True
    n_pre = prefix_steps(P)

    if args.copy_calibration:
        copy_calibration()
    paths = [x for x in args.paths.split(",") if x]
    if args.profile_steps:
        args.no_cpu, args.steps, args.warmup = True, 1, 0
    res = {path: run_path(path, w, args.steps, args.warmup, args.block_B, prefix=not args.no_cpu,
                          nsteps=args.profile_steps or None)
           for path in paths}
    primary = paths[-1]

    out_paths = {}
    # the counters were taken on the 256^2 workload (its kernels and launch shapes); other
    # workloads report traffic as null rather than that ratio
    traffic = measured_traffic() if args.workload == "2d_256" else {}
    oracle_prefix = oracle_modal = None
    cpu = None
    if not args.no_cpu:
        import oracle
        log("oracle prefix", n_pre, "steps on", oracle.num_threads(), "threads")
        t0 = time.perf_counter()
        oracle_prefix = oracle.run(p, w["memory"], w["u0"], n_pre)
        t_cpu = time.perf_counter() - t0
        macs_cpu = P * n_pre * (n_pre + 1) // 2
        cpu = {"value": macs_cpu / t_cpu, "unit": "history MACs/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "first %d of the %d steps of the same %s workload (%.3g MACs, "
                         "%.1f s)" % (n_pre, n, "x".join(str(v) for v in grid_of(p)), macs_cpu,
                                      t_cpu)}
        if p["rxn"] != "fisher":   # sine modes evolve alone only under a linear reaction
            c0 = modal(w["u0"], p, modes)
            oracle_modal = np.array([c0[i] * oracle.mode_run(p, w["memory"], m[0], m[1], 1.0, n,
                                                             s=m[2] if len(m) > 2 else 1)[-1]
                                     for i, m in enumerate(modes)])

    for path, r in res.items():
        d = {"ms_per_step": r["ms_per_step"], "value": r["macs"] / (r["ms_per_step"] / 1e3)}
        d["kernel_timing"] = ("one extra solve after the timed ones, each kernel launched on its "
                              "own with HIP events stamped at its start and end")
        for name, (cnt, ms) in r["prof"].items():
            if cnt:
                kd = {"launches": cnt // r["steps"], "ms_per_solve": ms / r["steps"],
                      "avg_us": ms * 1e3 / cnt}
                if name in r["work"]:
                    kind, work = r["work"][name]
                    kd["roofline"] = roofline_of(kind, work, cnt / r["steps"], ms / r["steps"])
                    # algorithmic HBM bytes per launch (for MFMA kernels: their memory side)
                    hbm = r["work"].get(name + "_bytes", (None, work if kind == "hbm" else None))[1]
                    if hbm is not None:
                        kd["roofline"]["algorithmic_bytes_per_launch"] = hbm * r["steps"] / cnt
                        if name in traffic:
                            kd["roofline"]["traffic"] = traffic[name] * hbm * r["steps"] / cnt
                d.setdefault("kernels", {})[name] = kd
        if oracle_prefix is not None:
            d["rel_l2_vs_oracle_prefix"] = float(np.linalg.norm(r["u_prefix"] - oracle_prefix) /
                                                 np.linalg.norm(oracle_prefix))
            if oracle_modal is not None:
                cg = modal(r["uT"], p, modes)
                d["modal_err_vs_oracle_full_length"] = float(np.abs(cg - oracle_modal).max() /
                                                             np.abs(oracle_modal).max())
        out_paths[path] = d

    if not args.no_modes and not args.profile_steps:
        full = res.get("gemv", res[primary])
        out_paths["memory_modes"] = run_memory_modes(
            w, full["uT"], None if args.no_cpu else True)
        out_paths["memory_modes"]["full"] = {
            "path": "gemv" if "gemv" in res else primary,
            "ms_per_solve": full["ms_per_step"], "history_macs_per_solve": full["macs"]}

    if not args.no_extra and not args.profile_steps:
        out_paths["workloads"] = run_extra_workloads(args.block_B, not args.no_cpu)
        out_paths["adjoint_128x128_5000steps"] = run_adjoint_leg()

    r = res[primary]
    # the dominant kernel of the headline path (largest share of the solve's time)
    kern = out_paths[primary].get("kernels", {})
    dom = max((k for k in kern if "roofline" in kern[k]), key=lambda k: kern[k]["ms_per_solve"],
              default=None)
    roofline = dict(kern[dom]["roofline"], kernel=dom) if dom else None
    if len(res) > 1 and "gemv" in res and "toeplitz" in res:
        out_paths["toeplitz_speedup_over_gemv"] = (res["gemv"]["ms_per_step"] /
                                                   res["toeplitz"]["ms_per_step"])
    value = r["macs"] / (r["ms_per_step"] / 1e3)
    line = {
        "metric": "history MACs/s + rel-L2 vs FP64 oracle; plain FP32 sum vs blocked MFMA sum",
        "value": value, "unit": "history MACs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16x3 mfma (f32 acc) + f64" if primary == "toeplitz" else "f32 history, f64 accumulate",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_NAMES[args.workload],
                   "grid": grid_of(p), "time_steps": args.profile_steps or n,
                   "memory": "full",
                   "history_macs_per_solve": r["macs"], "path": primary},
        "paths": out_paths,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
