"""GLASS-style batched small dense linear algebra for MI355X (gfx950).

The HIP library and its C-ABI live in ``csrc/``; ``glass`` is the thin ctypes
binding.  Importing the package loads nothing; ``from paper_2609_28179_amd
import glass`` loads the built library and fails loudly when it is missing.
"""
__all__ = ["glass", "inputs"]
