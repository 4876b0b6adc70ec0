"""Numerical entanglement of integer streams on MI355X (gfx950).

Implements the method of Anam & Andreopoulos, "Failure Mitigation in Linear,
Sesquilinear and Bijective Operations On Integer Data Streams Via Numerical
Entanglement" (IOLTS 2015): M >= 3 integer streams are entangled pairwise
(eq. (14)-(15)), an LSB operation runs on each entangled stream
independently (eq. (9)), and every output is recovered from any M-1 of the
entangled outputs with additions and arithmetic shifts (eq. (16)-(19)).

All arithmetic runs in the HIP library ``libne`` (C-ABI, ``include/ne.h``);
``ne`` is its thin ctypes binding. Importing this package loads nothing;
``paper_1509_03838_amd.ne`` loads the library on first use and raises if it
is missing.
"""
__all__ = ["ne", "workloads"]
