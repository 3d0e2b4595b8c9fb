"""CPU oracle for frequency-response evaluation -- TEST INFRASTRUCTURE ONLY.

Nothing in the product path may import, call or execute this package: only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark use
it.  It shares no code with the GPU library (no kernels, headers, helpers or
constants); the only thing both sides see is the seeded input generator,
which holds none of the method's arithmetic.

What it computes (all plain, slow and in float64 unless stated):

* ``freqresp``           the definition G(jw) = C (jw I - A)^{-1} B + D, one
                         dense LU with partial pivoting per frequency
                         (LAPACK zgesv through numpy.linalg.solve);
* ``freqresp_at``        the same definition at arbitrary complex points s
                         (off the imaginary axis, or z = exp(j theta) for a
                         discrete-time model); ``freqresp_at_extended`` with
                         the extended-precision refinement;
* ``derivative_at``      dG/ds = -C (s I - A)^{-2} B by two dense solves;
                         ``derivative_at_extended`` with both refined;
* ``freqresp_extended``  the same solve followed by iterative refinement whose
                         residual and iterate are held in extended precision
                         (x87 80-bit ``clongdouble``); the oracle of record for
                         ill-conditioned points;
* ``freqresp_descriptor`` G(s) = C (s E - A)^{-1} B + D of a descriptor
                         system (E possibly singular), dense LU per point;
                         ``freqresp_descriptor_extended`` with the refinement;
* ``cond2``              2-norm condition number of jw I - A per frequency;
* ``rel_err``            the per-frequency relative Frobenius error metric;
* ``exact.freqresp_exact``  exact rational evaluation for tiny systems;
* ``peaks.peaks_bruteforce``  resonance peaks and the H-infinity norm by a
                         dense grid and derivative-free golden-section search;
* ``hessenberg.hessenberg`` unblocked Householder reduction to upper
                         Hessenberg form with Q^T B and C Q;
* ``imdp``               robust value iteration for interval MDPs (the
                         paper's own method: its Eq. 2, with the inner
                         problem of Eq. 3 solved by sequential
                         O-maximization as its section 4 describes).

The mathematical problem: for a continuous-time LTI system
x' = A x + B u, y = C x + D u, the transfer matrix evaluated on the imaginary
axis s = jw is G(jw) = C (jw I - A)^{-1} B + D (any linear-systems text, e.g.
Kailath, *Linear Systems*, 1980, ch. 2).  The paper this project follows is
silent on this problem; every function here cites the textbook or published
method it restates instead.
"""
from .freqresp import (freqresp, freqresp_extended, freqresp_at, freqresp_at_extended, derivative_at,
                       derivative_at_extended, cond2, rel_err, rel_err_max, freqresp_descriptor,
                       freqresp_descriptor_extended)
from . import exact, hessenberg, imdp, peaks

__all__ = [
    "freqresp",
    "freqresp_extended",
    "freqresp_at",
    "freqresp_at_extended",
    "derivative_at",
    "derivative_at_extended",
    "cond2",
    "rel_err",
    "rel_err_max",
    "freqresp_descriptor",
    "freqresp_descriptor_extended",
    "exact",
    "hessenberg",
    "peaks",
    "imdp",
]
