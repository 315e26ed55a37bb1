"""MI355X (gfx950) library for the hot path of the hybrid Monte Carlo method of
Zhang, Bartel & Lusk (arXiv:1009.0457): checkerboard Potts sweeps with a local
constant-traction elastic zone solve per trial flip and a global explicit stress refresh.

Submodules: ``hmc`` (binding of the C ABI in include/hmc.h), ``synth`` (seeded synthetic
inputs), ``build`` (hipcc build of libhmc.so).  Importing the package loads nothing.
"""
