"""Seeded synthetic workloads for the GL fractional reaction-diffusion solver.

This module only builds inputs: problem parameters, memory settings and
initial fields, as plain dicts and numpy arrays.  It holds none of the
method's arithmetic, and it is the only code that both the GPU path and the
FP64 oracle use.  Every random draw comes from ``numpy.random.default_rng``
seeded with the value stated per workload, drawn in the order written.

Conventions (shared by both sides):
  * the domain is the unit interval / square / cube with N interior points
    per side and zero values outside (zero Dirichlet edge); dx = 1 / (N + 1)
    and the interior point j sits at x_j = (j + 1) dx;
  * a field is stored as u[l * nx + j] (x1 index j fastest), in 3D as
    u[(n * ny + l) * nx + j];
  * dt is chosen from a target r = alpha dt^gamma / dx^2, i.e.
    dt = (r dx^2 / alpha)^(1 / gamma);
  * problem dict keys: ndim, nx, ny, nz, dx, dt, gamma, alpha, rxn
    ("none" | "linear" | "fisher"), rate (f = -rate u or rate u (1 - u));
  * memory dict keys: mode ("full" | "short" | "adaptive"), L (window in
    steps), a (adaptive base), rule ("partition" | "literal" | "unit_stride").
"""
import numpy as np

SIDES_CFG5 = (64, 128, 192, 256, 384)


def dt_for_r(r, dx, alpha, gamma):
    """Time step giving alpha dt^gamma / dx^2 = r."""
    return float((r * dx * dx / alpha) ** (1.0 / gamma))


def problem(ndim, n, gamma, alpha, r, rxn="none", rate=0.0, dt=None, dx=None):
    """A problem on n interior points per side of the unit interval/square/cube."""
    dx = 1.0 / (n + 1) if dx is None else float(dx)
    dt = dt_for_r(r, dx, alpha, gamma) if dt is None else float(dt)
    return {"ndim": int(ndim), "nx": int(n), "ny": int(n) if ndim >= 2 else 1,
            "nz": int(n) if ndim == 3 else 1, "dx": dx,
            "dt": dt, "gamma": float(gamma), "alpha": float(alpha), "rxn": rxn,
            "rate": float(rate)}


def memory(mode="full", L=0, a=2, rule="partition"):
    return {"mode": mode, "L": int(L), "a": int(a), "rule": rule}


def npoints(p):
    return (p["nx"] * (p["ny"] if p["ndim"] >= 2 else 1) *
            (p.get("nz", 1) if p["ndim"] == 3 else 1))


def coords(n):
    """Interior coordinates x_j = (j + 1) / (n + 1), j = 0..n-1."""
    return np.arange(1, n + 1, dtype=np.float64) / (n + 1)


def sine_mode(p, mode_p, mode_q=1, amplitude=1.0, mode_s=1):
    """amplitude * sin(p pi x) sin(q pi y) [sin(s pi z)] on the interior grid (1D:
    sin(p pi x))."""
    x = coords(p["nx"])
    fx = np.sin(mode_p * np.pi * x)
    if p["ndim"] == 1:
        return amplitude * fx
    y = coords(p["ny"])
    fy = np.sin(mode_q * np.pi * y)
    f2 = np.outer(fy, fx).reshape(-1)
    if p["ndim"] == 2:
        return amplitude * f2
    fz = np.sin(mode_s * np.pi * coords(p["nz"]))
    return amplitude * np.outer(fz, f2).reshape(-1)


def gaussian(p, seed, sigma=0.1, centre=(0.5, 0.5, 0.5), noise=1e-3):
    """exp(-|x - c|^2 / (2 sigma^2)) plus seeded uniform noise in [-noise, noise]."""
    rng = np.random.default_rng(seed)
    x = coords(p["nx"])
    if p["ndim"] == 1:
        g = np.exp(-((x - centre[0]) ** 2) / (2 * sigma * sigma))
        return g + rng.uniform(-noise, noise, size=p["nx"])
    y = coords(p["ny"])
    if p["ndim"] == 2:
        g = np.exp(-((x[None, :] - centre[0]) ** 2 + (y[:, None] - centre[1]) ** 2)
                   / (2 * sigma * sigma))
        return (g + rng.uniform(-noise, noise, size=(p["ny"], p["nx"]))).reshape(-1)
    z = coords(p["nz"])
    g = np.exp(-((x[None, None, :] - centre[0]) ** 2 + (y[None, :, None] - centre[1]) ** 2
                 + (z[:, None, None] - centre[2]) ** 2) / (2 * sigma * sigma))
    return (g + rng.uniform(-noise, noise, size=(p["nz"], p["ny"], p["nx"]))).reshape(-1)


def uniform_field(p, seed, lo=0.0, hi=0.1):
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=npoints(p))


# ------------------------------------------------------------- named workloads

def cfg1():
    """1D, 128 points, gamma 0.5, alpha 1, f = 0, u0 = sin(pi x), r = 0.2, 2000 steps, full."""
    p = problem(1, 128, 0.5, 1.0, 0.2)
    return {"name": "1d_n128_g0.5_full", "problem": p, "memory": memory("full"),
            "u0": sine_mode(p, 1), "nsteps": 2000}


def cfg2(mode="full", L=1000, a=2, rule="partition", n=256, nsteps=20000):
    """2D 256^2, gamma 0.8, alpha 1, f = -0.1 u, Gaussian sigma 0.1 + U(+-1e-3) (seed 2),
    r = 0.1, 20000 steps; full / short L / adaptive a."""
    p = problem(2, n, 0.8, 1.0, 0.1, rxn="linear", rate=0.1)
    return {"name": "2d_n%d_g0.8_%s" % (n, mode), "problem": p,
            "memory": memory(mode, L=L, a=a, rule=rule), "u0": gaussian(p, 2),
            "nsteps": nsteps}


def cfg3(n=512, nsteps=50000):
    """2D 512^2, gamma 0.6, alpha 0.5, Fisher-KPP f = u(1-u), u0 ~ U[0, 0.1] (seed 3),
    r = 0.1, 50000 steps, full."""
    p = problem(2, n, 0.6, 0.5, 0.1, rxn="fisher", rate=1.0)
    return {"name": "2d_n%d_g0.6_fisher_full" % n, "problem": p, "memory": memory("full"),
            "u0": uniform_field(p, 3), "nsteps": nsteps}


def cfg4(n=128, nsteps=5000):
    """Adjoint case: 2D 128^2, gamma 0.7, alpha 1, f = -0.2 u, Gaussian (seed 4), r = 0.05,
    5000 steps; the target comes from the same dt, dx, u0 and rate at gamma 0.65,
    alpha 1.2.  Also a seeded unit direction (seed 44) for directional derivatives."""
    p = problem(2, n, 0.7, 1.0, 0.05, rxn="linear", rate=0.2)
    target_p = dict(p, gamma=0.65, alpha=1.2)
    u0 = gaussian(p, 4)
    v = np.random.default_rng(44).standard_normal(npoints(p))
    v /= np.linalg.norm(v)
    return {"name": "2d_n%d_g0.7_adjoint" % n, "problem": p, "target_problem": target_p,
            "memory": memory("full"), "u0": u0, "direction": v, "nsteps": nsteps,
            "ckpt_every": 500}


def cfg5(nprob=64, nsteps=10000, a=4):
    """Ensemble of 64 2D problems (seed 5): side from {64,128,192,256,384}, gamma in
    U[0.3, 0.95], alpha in U[0.5, 2], f = -k u with k in U[0, 0.5], sine mode (p, q) in
    {1..4}^2; r = 0.1; adaptive memory a = 4 (partition reading); 10000 steps."""
    rng = np.random.default_rng(5)
    sides = rng.choice(np.array(SIDES_CFG5), size=nprob)
    gammas = rng.uniform(0.3, 0.95, size=nprob)
    alphas = rng.uniform(0.5, 2.0, size=nprob)
    ks = rng.uniform(0.0, 0.5, size=nprob)
    pq = rng.integers(1, 5, size=(nprob, 2))
    probs, u0s = [], []
    for i in range(nprob):
        p = problem(2, int(sides[i]), float(gammas[i]), float(alphas[i]), 0.1, rxn="linear",
                    rate=float(ks[i]))
        probs.append(p)
        u0s.append(sine_mode(p, int(pq[i, 0]), int(pq[i, 1])))
    return {"name": "ensemble64_adaptive_a%d" % a, "problems": probs, "modes": pq.tolist(),
            "memory": memory("adaptive", a=a), "u0s": u0s, "nsteps": nsteps}


def paper_fig1(gamma):
    """Sec. 3.1 example: 100x100 grid, point source U[50,50] = 0.1 with its four neighbours
    0.05, zero edge, alpha 1, no reaction, dt 0.5, dx 5, run to t = 100 (200 steps)."""
    p = problem(2, 100, gamma, 1.0, None, dt=0.5, dx=5.0)
    u0 = np.zeros((100, 100))
    u0[50, 50] = 0.1
    u0[51, 50] = u0[49, 50] = u0[50, 51] = u0[50, 49] = 0.05
    return {"name": "paper_fig1_g%g" % gamma, "problem": p, "memory": memory("full"),
            "u0": u0.reshape(-1), "nsteps": 200}


def paper_fig3(gamma, mem=None):
    """Sec. 3.2 comparison: 20x20 grid, U[10,10] = 10, alpha 1, no reaction, dt 1, dx 10,
    run to t = 1500 (1500 steps)."""
    p = problem(2, 20, gamma, 1.0, None, dt=1.0, dx=10.0)
    u0 = np.zeros((20, 20))
    u0[10, 10] = 10.0
    return {"name": "paper_fig3_g%g" % gamma, "problem": p,
            "memory": mem or memory("full"), "u0": u0.reshape(-1), "nsteps": 1500}


def superdiffusion_2d(n=256, nsteps=20000, gamma=1.5):
    """Superdiffusion (gamma in (1, 2]): 2D 256^2, gamma 1.5, alpha 1, no reaction,
    Gaussian sigma 0.1 + U(+-1e-3) (seed 6), r = 0.1, 20000 steps, full memory."""
    p = problem(2, n, gamma, 1.0, 0.1)
    return {"name": "2d_n%d_g%g_super_full" % (n, gamma), "problem": p,
            "memory": memory("full"), "u0": gaussian(p, 6), "nsteps": nsteps}


def diffusion_3d(n=64, nsteps=20000):
    """3D 64^3 (7-point stencil), gamma 0.8, alpha 1, f = -0.1 u, Gaussian sigma 0.1 +
    U(+-1e-3) (seed 7), r = 0.05, 20000 steps, full memory."""
    p = problem(3, n, 0.8, 1.0, 0.05, rxn="linear", rate=0.1)
    return {"name": "3d_n%d_g0.8_full" % n, "problem": p, "memory": memory("full"),
            "u0": gaussian(p, 7), "nsteps": nsteps}
