"""MI355X (gfx950) implementation of the filtered Paterson-Stockmeyer
evaluation of sparse matrix power series (arXiv 2208.05683, Section 3 and
Algorithm 2 with a fixed entry threshold).

The computation lives in ``libfps.so`` (hand-written HIP kernels behind the C
ABI of ``include/fps.h``); ``binding`` marshals arguments to it and ``api``
adds a small torch-facing convenience layer.  Importing ``binding`` or ``api``
fails loudly if the library has not been built.
"""

__all__ = ["api", "binding", "build"]
