"""thx: fast polynomial basis conversion on AMD MI355X (gfx950).

Computes beta = A alpha for the conversion matrices of Townsend, Webb & Olver,
"Fast polynomial transforms based on Toeplitz and Hankel matrices"
(arXiv:1604.07486), written A = D1 (T o H) D2 with a pivoted-Cholesky low-rank
Hankel part and FFT-based Toeplitz products.  All arithmetic runs in the HIP
library libthx.so (C ABI in include/thx.h); this package only marshals
arguments (see ``paper_1604_07486_amd.binding``).  The binding is imported
lazily so that ``paper_1604_07486_amd.inputs`` works without the library.
"""
import importlib

__all__ = ["binding", "inputs"]


def __getattr__(name):
    if name in ("binding", "inputs"):
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
