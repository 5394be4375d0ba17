"""MI355X-native GLS solves for mixed-model GWAS (Eq. 1 of the paper).

The compute path lives in the HIP library ``libgwas.so`` built from ``csrc/``;
``binding`` is a thin ctypes layer over its C ABI.  Importing this package does
not load the library; ``binding.load()`` does, and raises if it is missing.
"""

__all__ = ["binding", "synth"]
