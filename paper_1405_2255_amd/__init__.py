"""MI355X-native fast multipole method for collisional stellar dynamics
(Dehnen 2014): unsoftened 1/r potential and acceleration of all N particles,
computed by hand-written HIP kernels for gfx950 behind a C ABI (libfmm.so).

The Python side is argument marshalling only; see ``fmm`` for the binding.
"""
__all__ = ["fmm", "workloads"]
