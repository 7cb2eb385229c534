"""Colour-coding tree subgraph counting on AMD MI355X (gfx950).

The counting runs in libsc (HIP kernels behind the C ABI of include/sc.h);
``sc`` is its ctypes binding and ``inputs`` holds the seeded synthetic
graph and template generators.
"""
__all__ = ["sc", "inputs"]
