"""FP64 CPU oracle for one contact-dynamics time step and its derivatives.

TEST INFRASTRUCTURE ONLY.  This package is imported by `tests/`, by the
`smoke()` check of the entry module and by the `cpu_baseline` leg of the
benchmark, never by the library: the HIP path shares no code with it.

It is plain and slow on purpose:
  * rigid-body dynamics by the textbook recursive Newton-Euler algorithm in
    body coordinates (`rbd`), the mass matrix as the columns of inverse
    dynamics with respect to the acceleration, contact Jacobians as the
    velocity map of the contact points;
  * the frictional-contact NCP (Section II.B, eq. NCP) by block Gauss-Seidel
    with exact per-contact solves, then Newton on the mode-fixed equations,
    then a check of every condition (`ncp`);
  * the step derivative (Section III, eq. FD_grads and the mode equations
    of Section III.B) as the implicit-function theorem applied to the raw
    mode-fixed system, with forward-mode automatic differentiation of the
    plain definitions and a min-norm least-squares solve (`derivative`);
  * the paper's reduced system of Appendix B formed densely, as a
    structural cross-check, and central finite differences.

Derivatives in q are taken along the tangent perturbation q (+) dq: a revolute
angle adds dq, a free flyer composes its placement with Exp(dq) on the right
(dq = body-frame linear and angular parts).

Parity status: every function here is pinned by `tests/test_oracle_*.py`
against closed forms, invariants, brute force or finite differences; the
pins are listed in the module docstrings.
"""
