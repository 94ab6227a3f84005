"""CPU FP64 oracle for the lattice Green's function solve.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU-baseline
leg of the benchmark, never by the product path.

  lgf.py         G by the Bessel integral (Appendix A) + A^q far away; exact direct sum
  asymptotic.py  A^q derived from Eq. lgf1 with exact rationals (Sec. 2.1)
  flgf.py        the FLGF method step by step (Sec. 3.1), numpy FFT as the primitive
  lgf_oracle.c   the C parts (quadrature, Bessel recurrence, direct sum, A^q evaluation)
"""
