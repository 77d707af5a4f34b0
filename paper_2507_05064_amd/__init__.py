"""MI355X (gfx950) implementation of the VIF Gaussian-process approximation
hot path (arXiv 2507.05064): HIP kernels behind the C ABI of include/vif.h,
with a thin ctypes binding in ``paper_2507_05064_amd.vif``."""
