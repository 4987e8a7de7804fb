"""All-pairs LCS similarity stage of FAMSA (arXiv 1603.06958) for gfx950.

Importing the package loads nothing; ``paper_1603_06958_amd.binding`` loads
the HIP library and fails loudly when it is missing.
"""
__version__ = "0.1.0"
