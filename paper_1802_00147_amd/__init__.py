"""MI355X (gfx950) library for batched, manifold-corrected FP64 integration of
spinning compact binaries and fast-Lyapunov-indicator phase-space scans
(arXiv:1802.00147).  The C ABI is include/pn.h; `pn` is its Python binding;
`workloads` generates the seeded synthetic scan inputs."""
__all__ = ["pn", "workloads", "build"]
