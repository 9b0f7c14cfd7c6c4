"""Boxcar single-pulse search (Adamek & Armour, arXiv:1910.08324) for AMD MI355X (gfx950).

The search runs in libspd.so (hand-written HIP kernels behind the C ABI in include/spd.h);
`paper_1910_08324_amd.spd` is its Python binding.
"""
__all__ = ["spd"]
