"""FP64 CPU oracle for the similarity join (test infrastructure only).

Nothing in the GPU library imports this package; only the test suite, the smoke
check and the bench's CPU-baseline leg do.  See ``ejoin_oracle.c`` for the
canonical similarity rule and ``exact.py`` for the exact-rational brute force
that pins it.
"""
