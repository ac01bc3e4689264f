"""CPU FP64 oracle for the strongly coupled immersed-boundary step (Nair & Goza).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, dense NumPy rendering of
what the method computes, written from the paper and kept independent of the HIP
library: it shares no code, tables or helpers with ``paper_2103_06415_amd``, and
neither side imports the other.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it; the product path never does.

Everything is float64.  Sine transforms are dense matrix products (no FFT), small
linear systems use ``numpy.linalg.solve``, and every operator has a direct
definition that can be checked against the paper by eye:

* ``grid``        curl C, its transpose, the 5-point Laplacian C^T C, the
                  rotational-form nonlinear term (Sec. 2.2, Appendix A eq. (A.1)).
* ``dst``         DST-I diagonalisation of C^T C and the solve with C^T A C
                  (Sec. 3.2.1, eqs. (30)-(31)).
* ``delta``       discrete delta kernels and the interpolation E / regularisation
                  E^T (Sec. 3.1, eq. (24)).
* ``multidomain`` nested-level boundary rings and coarsification (Sec. 5, far-field
                  treatment by nested grids).
* ``structure``   Newmark torsional body and corotational beam (Appendix A,
                  eqs. (A.4)-(A.5), (A.10)-(A.13)).
* ``subdomain``   sub-domain operator E0, hat interpolation P, B and the drop
                  filter (Sec. 3.1-3.2, eqs. (25)-(29), (34)-(35)).
* ``step``        one time step: predictor, FSI iteration on the Schur system,
                  corrector (eqs. (16)-(20) and (36)-(40); Algorithms 1 and 2).

Readings of passages the paper leaves open are listed in each module's header.
"""
