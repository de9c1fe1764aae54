"""CPU FP64 oracle for the spectral-element in situ extraction path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
module; only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may call it.  It shares no code, table or constant with the
HIP library: every quantity here (GLL nodes, differentiation matrix,
marching-cubes case table) is recomputed from its definition.

What the path computes, and where it comes from
-----------------------------------------------
The paper (section 1, Introduction) places the data in a spectral-element
(SEM) solver and (section 3, DataAdaptor subsection) says the snapshots live
in GPU memory and use the Nek data model; it does not spell out the analysis
itself.  The extraction steps are therefore written from their standard
definitions:

* GLL nodes, weights and the collocation derivative matrix -- Deville,
  Fischer & Mund, *High-Order Methods for Incompressible Fluid Flow* (2002),
  chapter 2 (module ``gll``).
* Tensor-product reference derivatives, isoparametric Jacobian, chain rule
  (same book, chapter 4) and the Q-criterion of Hunt, Wray & Moin (1988)
  plus vorticity magnitude (module ``sem``).
* Marching cubes of Lorensen & Cline (1987) with a case table generated from
  a face-consistent rule, stream compaction by exclusive prefix sum
  (module ``mc``).

All floating point is FP64 unless a function says otherwise (the FP32
classification of ``mc`` compares in FP32 so that an integer decision is
taken in the same precision as the FP32 kernel).
"""

from . import gll, sem, mc  # noqa: F401

__all__ = ["gll", "sem", "mc"]
