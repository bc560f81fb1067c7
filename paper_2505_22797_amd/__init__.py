"""MI355X (gfx950) library for the model operator of trajectory-independent,
model-based Magnetic Particle Imaging: A (convolution with the Langevin
Jacobian kernel, sampling along the trajectory, contraction with the velocity),
its exact transpose and the gradient/denoise iteration.

`mpik` is the thin ctypes binding of the C ABI in include/mpik.h; `synth`
holds the seeded synthetic inputs.  Importing the package loads nothing; the
binding loads libmpik.so on first use and raises if it is missing.
"""
__all__ = ["mpik", "synth", "build"]
