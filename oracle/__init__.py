"""CPU oracle for the staggered RHMC hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 (numpy + mpmath) implementation of what the GPU path
computes, written from the paper (Gupta & Majumdar, arXiv:1710.09178):

* ``lattice``  -- site address and checkerboard parity (Sec. 2, Sec. 3.2)
* ``su3``      -- Lie-algebra coordinates, matrix exponential, reunitarisation
* ``dirac``    -- staggered operator M = 2m + D, its even-odd blocks and the
                  half-lattice operator (M^dag M)_ee (Sec. 3.2)
* ``solvers``  -- CG and the multi-shift CG used for the rational functions (Sec. 4)
* ``rational`` -- minimax rational approximation of x^p and its partial
                  fractions (eq. ratapprx, Appendix)
* ``gauge``    -- plaquette action (eq. pfact, second term) and its force
* ``fermion``  -- pseudofermion action (eq. pfact, first term) and its force
* ``hmc``      -- heat bath, leapfrog molecular dynamics and Metropolis (Sec. 3.1)
* ``philox``   -- Philox4x32-10 counter-based generator and Box-Muller
* ``surrogate``-- reference for the learned force model (not in the paper)

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it and it
never calls the GPU library; the two share only the seeded input generators of
``synth``.
"""
