"""FP64 CPU oracle for the relativistic lattice Boltzmann time step of
Gabbana, Mendoza, Succi, Tripiccione, "Towards a unified lattice kinetic
scheme for relativistic hydrodynamics" (arXiv:1703.04605).

This package is TEST INFRASTRUCTURE.  It is a plain, slow, obviously correct
implementation of what the GPU library computes, written directly from the
paper in float64 (mpmath at 40+ digits for init-time quantities).  Only the
test suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  It shares no code, table or constant with the
GPU library in ``paper_1703_04605_amd``; neither side imports the other.

Modules
-------
groups       velocity-group table of Appendix C (full-symmetric sets)
special      modified Bessel functions K_n (scipy / mpmath, black boxes)
polynomials  second-order orthonormal polynomials of Appendix A
projections  projection coefficients a^(k) = b^(k)/T_R (eq. mj-projection-coefficients)
quadrature   weights of the prescribed-abscissa quadrature (Sec. III.C-D)
eos          Karsch equation of state and its inversion (eq. relativistic-eos)
landau       Landau-Lifshitz frame by eigen-decomposition (Sec. II.A)
lattice      the discrete model: populations, equilibrium, collision, streaming
mlp          float64 reference of the learned Landau-frame guess (not in the paper)
"""
