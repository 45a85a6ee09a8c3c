"""MI355X-native incremental maintenance of matrix-power views (LINVIEW
IncrExp, arXiv 1403.6968) behind the C ABI of liblinview.

    from paper_1403_6968_amd import linview
    view = linview.View(A, k=16)          # A: float32/float64 device tensor
    view.update(U, V)                     # Delta A = U V^T
    P16 = view.read(16)
"""

from . import linview  # noqa: F401

__all__ = ["linview"]
