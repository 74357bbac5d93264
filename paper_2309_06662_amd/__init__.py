"""MI355X-native split-explicit hydrostatic ocean step (HIP kernels behind a C ABI)."""
__all__ = ["inputs"]
