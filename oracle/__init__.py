"""FP64 CPU oracle for the analytic-pulse particle-in-cell step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP path (no kernels, headers, helpers, tables or constant generators); the
two sides meet only at the seeded input generator, which holds none of the
method's arithmetic.

The oracle is written to be read against the paper (Weichman et al.,
"Analytic pulse technique for computational electromagnetics"):

* ``units``     -- normalised units, time step rule and the Yee dispersion
                   constants of Sec. II.A, Eqs. (10)-(14).
* ``pulses``    -- the analytic vacuum fields E1, B1: pulsed plane wave
                   (Eqs. (15), (17)), paraxial Gaussian (Eqs. (20)-(23) and
                   the secondary components of Sec. III.A), Laguerre-Gaussian
                   modes, flying focus (Eqs. (24)-(26), Sec. III.C) and the
                   nonparaxial Gaussian.
* ``pic``       -- the modified PIC loop of Fig. 1: gather of the internal
                   fields E2, B2, sum with E1, B1, relativistic Boris push,
                   move, charge-conserving (Esirkepov) deposition and the Yee
                   update of E2, B2 only (Eqs. (4), (7)-(9)).
* ``diag``      -- FP64 diagnostics: charge density, continuity residual,
                   energies and moments.
* ``grad``      -- forward-mode reference gradients of particle observables
                   with respect to pulse parameters.

Everything is FP64 (complex128 where the paper writes analytic signals).
"""
