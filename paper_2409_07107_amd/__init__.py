"""MI355X-native differentiable contact-dynamics step (arXiv 2409.07107).

The step, its full Jacobian and its vector-Jacobian product run as HIP
kernels for gfx950 behind the C ABI declared in include/dsim.h; `dsim` is the
Python binding (argument marshalling only) and `scenes` the seeded synthetic
workload generator.  Importing the package loads nothing: the binding loads
the shared library on first use and raises if it has not been built.
"""
__all__ = ["dsim", "scenes"]
