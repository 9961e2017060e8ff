"""Reference oracle for the decomposed fractional stiffness operator (TEST INFRASTRUCTURE).

This package is a plain, slow, FP64 CPU implementation of what the library
computes, written from the paper (Lei, Turkiyyah, Knio, "Finite element
discretizations for variable-order fractional diffusion problems").  It exists
only to check the HIP path: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
library (``paper_2302_02863_amd``); both read inputs from ``fpde_inputs``.

Modules
-------
rules      Gauss-Legendre rules and the per-element (collapsed) rule, Sec. 5.2/6.1.
fields     P1 fields, the kernel gamma(x,y)=a(x,y)/|x-y|^{d+s(x)+s(y)} (Sec. 2).
singular   touching element pairs (Sec. 4, eqs. e:int-v-2, e:int-e, e:int-i-2) and
           the 1D analogue derived the same way.
assembly   exact dense assembly by definition (eq. e:l-stiff) and the three-way
           split A = B + K + M (eqs. e:decomp, e:b, e:k, e:m, e:tgt-sum).
h2         KD cluster tree, admissibility, Chebyshev interpolation; the
           H2-consistent K~ (Sec. 5) and the point-collocation density (Sec. 6.2),
           evaluated entrywise with directly computed (non-nested) bases.
exterior   analytic density beyond the auxiliary ball (eq. e:rho).
solve      dense Cholesky and textbook CG solves of the Galerkin system (O8).

Parity status of every function is listed in its module header.
"""
