"""MI355X-native explicit Grunwald-Letnikov fractional reaction-diffusion solver.

The hot path (GL weights, memory schedules, history sums, stencil update,
adjoint) runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/gl.h`` (``libgl.so``).  ``paper_1004_5128_amd.gl`` is its Python
binding; importing this package loads nothing.
"""
__all__ = ["gl", "workloads"]
