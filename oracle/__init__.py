"""CPU oracle for the EFPI / PIC-burst hot path — TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, obviously correct FP64 implementation of what the
GPU path computes, written from the paper (Cazeaux & Hesthaven, "Projective
multiscale time-integration for electrostatic particle-in-cell methods",
arXiv:1610.01071) and nothing else.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product package
``paper_1610_01071_amd`` never imports, links or calls anything here, and this
package never imports the product package: the two share no code.

Modules
-------
pic      fine-scale solver: fixed-point CIC deposit, Poisson-Boltzmann Newton,
         field, gather, leapfrog push, energy diagnostic (Sec. 2.2, eqs. 2.4-2.5,
         3.14-3.16).
efpi     coarse representation and the projective cycle: co-evolving restriction
         (App. B), Haar scaling coefficients (App. A), least-squares slope and
         projection (eqs. 3.17-3.18), quiet-start lift (App. C), the macro step
         (Sec. 3.1) and the ensemble mean.
kinetic  fine solver with kinetic electrons (two-species leapfrog, linear
         Poisson, eq. 2.2), Boltzmann-equilibrium electron loading at lift
         (eqs. 3.15-3.16, App. C) and the macro step with kinetic electrons.
phase    phase-space coarse variables (Sec. 3.3, App. A, App. C): phase-space
         histogram, full weighting and midpoint interpolation (eqs. 3.7-3.8), the
         order-4 Coiflet filter from its defining conditions, the periodized
         wavelet transform, the CDF repair and inverse-CDF quiet start, and the
         macro step on phase-space coefficients.
nn       1D-convolution surrogate for the coarse time derivative: forward,
         hand-derived backward and Adam, FP64.
metrics  the relative L2 error of eq. 4.2.

Every function states the passage it follows.  Functions whose result has no
independent pin say "parity unpinned" in their docstring; the tests under
``tests/test_oracle_*.py`` pin the rest against closed forms, invariants, brute
force and library routines.
"""
