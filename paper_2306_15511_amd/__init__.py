"""MI355X-native constrained-realization solver (HEALPix SHT + PCG) for the
joint CMB sky / C_l Gibbs step of Eskilt et al. 2023 (arXiv:2306.15511).

The compute library is ``libcrsht.so`` (HIP, gfx950), C ABI in
``include/crsht.h``; ``paper_2306_15511_amd.crsht`` is its Python binding and
``paper_2306_15511_amd.build`` compiles it.
"""
__all__ = ["crsht", "build"]
