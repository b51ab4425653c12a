"""Plain, slow, obviously-correct FP64 CPU oracle for Multi-Frequency WaveHoltz.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this
package: only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code with the HIP library (no
kernels, headers, tables or helpers) and it never imports that library.

Modules
-------
plan      time-step recipe, modified frequencies, quadrature weights, filter
          coefficients, the N_f x N_f matrix B, beta_d / mu_d, least-squares
          filter optimisation (Section 5, Algorithm 2; Section 6).
fd        the discrete operator L_h (order 2/4, Dirichlet), its sparse matrix,
          sparse direct and DST-I Helmholtz solves (Section 6, eq.
          discreteHelmholtz).
mfwh      one MFWH application (Algorithm 1 with the discrete scheme of
          Section 6), fixed-point iteration and restarted GMRES (Section 7),
          plain or with deflated restarting.
krylov    GMRES with deflated restarting (Morgan 2002) on a generic operator.
checks    error / residual measures of Section 8 and leapfrog energy.
cnn       FP64 reference for the warm-start convolutional network.

Parity notes: every function here is pinned by a ``-m "not gpu"`` test
against something other than itself (printed paper values, closed forms,
library routines on special cases, invariants); functions without such a
pin say "parity unpinned" in their docstring.
"""
