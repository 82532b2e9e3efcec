"""MI355X (gfx950) context-enhanced similarity join: the tensor-join hot path
behind a C ABI (``include/ejoin.h``), with a thin ctypes binding in
``paper_2312_01476_amd.ejoin``.  Importing the package loads nothing; the HIP
library is loaded on first use and its absence is an error."""
__all__ = ["ejoin", "datagen"]
