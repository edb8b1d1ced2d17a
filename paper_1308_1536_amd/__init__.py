"""MI355X-native multiprecision determinant, leading determinants and
last-column minors (Gaussian elimination without pivoting; Beliakov &
Matiyasevich).  The compute path is the C-ABI library ``libmpdet.so``
(hand-written HIP for gfx950); ``binding`` is a thin ctypes layer over it.

Importing the package loads nothing; ``binding.lib()`` loads the library and
fails loudly if it has not been built.
"""
__all__ = ["inputs", "binding"]
