"""Batched frequency-domain compact-binary log-likelihood on AMD Instinct MI355X (gfx950).

The compute lives in libgwlike.so (HIP kernels behind the C ABI of include/gwlike.h);
`gwlike` is its Python binding and `synth` the seeded input generator.
"""
__all__ = ["gwlike", "synth"]
