"""Dynamic Frontier PageRank on MI355X (gfx950).

``dfpr`` is the ctypes binding of libdfpr (include/dfpr.h); ``inputs``
draws seeded synthetic graphs and batches; ``build`` compiles the library.
"""
__all__ = ["dfpr", "inputs", "build"]
