"""FP64 CPU oracle for the semi-coherent time-frequency statistic.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only the test-suite, the smoke
check and the CPU-baseline timing leg of the benchmark use it.

Two tiers (plain, slow, obviously correct; float64 throughout):

* O1, the definition (``oracle.o1``): each template is synthesised in the time
  domain (TaylorT3 phase, rigid-orbit single-link responses with explicit
  light-time delays, TDI X/Y/Z -> A/E), every tranche is transformed by a
  direct DFT, and the per-segment inner products are summed.
* O2, the method (``oracle.o2``): per tranche, the template's spectrum is the
  Fresnel-kernel form of Eq. (fresnel-ft) with the paper's two Fresnel
  branches, multiplied by the TDI transfer function evaluated once per
  tranche (Eq. (tdi2)), on the N_F = 21 bins around the track frequency;
  tranche sums are combined into segments (Eqs. (inner-segment-tf),
  (inner-tranche-tf)) and into the statistic of Eq. (Upsilon-seg).
  Its gradient is torch autograd of the same float64 code.
* ``oracle.cpu`` builds ``o2_cpu.c``, a plain scalar C version of O2 (OpenMP
  over templates) used to time the oracle on host cores and to evaluate
  large parity samples.

Readings of the paper that the oracle fixes are listed in each module's
docstring.
"""
