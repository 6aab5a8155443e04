"""craneplan for MI355X: the GPU stochastic path optimizer of a forestry crane.

The package holds the HIP kernels and C-ABI library (``csrc/``), the ctypes
binding (``craneplan``) and the seeded synthetic-input generator (``synth``).
Importing the package loads nothing; ``paper_2503_14160_amd.craneplan`` loads
the native library on first use and raises if it is missing.
"""
