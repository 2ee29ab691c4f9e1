"""Partitioned quantum-circuit tensor-network contraction on MI355X (gfx950).

Importing the package loads nothing native; `paper_2507_20667_amd.lib` loads
the C-ABI library.
"""
__version__ = "0.1.0"
