"""Independent CPU oracle for stencil composition (test infrastructure only).

This package is the plain, slow, obviously-correct reference that the GPU
library is checked against. It shares no code with the HIP library: it has
its own exact rational stencil algebra (``oracle.rational``) and its own
naive FP64 loops in C (``oracle/oracle.c``, loaded by ``oracle.capi``).

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import it. The product path never calls it.

Paper basis (Mishra, Salac, Knepley, "On the order of accuracy for finite
difference approximations of partial differential equations using stencil
composition"):

* stencil Taylor series and validity rules: Sec. 2.1, eq. (CompactNotation),
  Definition (StencilRules);
* composition C = B(A): Sec. 2.2, eq. (C=B(A));
* re-targeting and the order lemma: Sec. 2.2.2, eq. (Retarget),
  eq. (AccuracyComposition), Lemma (Accuracy), Proposition (CoeffAccuracy);
* multi-dimensional composition: Sec. 2.3;
* biharmonic BVP: Sec. 3.3; Cahn-Hilliard: Sec. 4.

Functions whose results are not pinned by an independent check say
"parity unpinned" in their docstring.
"""
