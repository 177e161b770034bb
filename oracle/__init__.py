"""Plain FP64 CPU oracle for the ASMG-preconditioned CG solve (TEST INFRASTRUCTURE ONLY).

This package is the independent reference that the HIP path is checked against.
Only the tests, the smoke check in ``__graft_entry__`` and the ``cpu_baseline``
leg of ``bench.py`` may import it. The product library never calls into it, and
the two share no code. The only shared module is ``workloads``, which holds the
seeded input generators and none of the method's arithmetic.

Paper: Grasedyck, Wang, Xu, "A Nearly Optimal Multigrid Method for General
Unstructured Grids" (arXiv:1410.2153). Each module cites the section, equation
or algorithm it follows:

* ``fem``       P1 stiffness matrix of the model problem (Section 2, eq. (2)).
* ``cluster``   barycenters, regular box tree, cluster tree (Section 3.1) and
                closure (Section 3.2), in two independent forms.
* ``auxgrid``   conforming nested auxiliary triangulations (Section 3.3) and
                Dirichlet auxiliary grids (Section 3.4).
* ``auxops``    auxiliary stiffness matrices A_l and prolongations P_l
                (Section 4.1, Algorithm 2, Section 5.1).
* ``transfer``  Scott-Zhang quasi-interpolation Pi between the auxiliary and
                the original space (Section 4.1).
* ``colour``    the multicolour ordering used for Gauss-Seidel.
* ``asmg``      Gauss-Seidel smoother (Section 4.1), V-cycle (Algorithm 2) and
                the multiplicative auxiliary space preconditioner (Algorithm 1,
                eq. (fasp2)).
* ``pcg``       preconditioned CG (Section 5.2), including the FP32-preconditioner
                variant.
* ``adjoint``   gradient of a least-squares loss w.r.t. per-element log-coefficients.
* ``hierarchy`` glue: builds every setup object for one mesh.

Parity status of every function is listed in the module headers; a function
without an independent pin says "parity unpinned".
"""
