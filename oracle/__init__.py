"""CPU FP64 oracle for the Local Exponential Method (LEM) hot path.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The GPU product
path never calls, links or falls back to anything here, and nothing here
imports the GPU package: the two share no code.  Inputs come from the seeded
generators in ``lem_inputs`` (which hold none of the method's arithmetic).

Everything is plain NumPy/SciPy in float64, written for a reader to check
against the paper (L. Bonaventura, "Local Exponential Methods: a domain
decomposition approach to exponential time integration of PDEs"):

  operator.py   the semi-discrete operator A of the model problem (eq. (2)
                discretized as in eq. (3)); centered finite differences as in
                section 4.1, conservative flux form as in section 4.3 (ibv2d)
  partition.py  the overlapping decomposition M_i = D_i u B_i of section 3
  halo.py       a provable restatement of the off-diagonal decay bound
                (Theorem 1, section 2) used to size the buffers B_i
  expm.py       Pade [13/13] scaling and squaring (the dense local exponential
                computation the paper names in sections 3 and 4)
  krylov.py     Arnoldi/Krylov action of the exponential (section 4.3)
  lem.py        one LEM step: local problems (4), update (5), core overwrite
                (step 3 of section 3), with exact local exponentials
  globalexp.py  the global exponential exp(dt A) u (the D=1 reference),
                via the discrete Fourier symbol for periodic constant
                coefficients, dense expm or the Krylov action otherwise
  phi.py        phi_1 and the exponential-Euler form of update (5)
  rosenbrock.py exponential Rosenbrock-Euler LEM for Burgers (sections 3, 4.2)
                with a Jacobian frozen between refreshes
  schrodinger.py LEM for the 1D Schroedinger equation with a harmonic
                potential (section 4.1), complex local exponentials
  metrics.py    relative l2 / l-infinity errors
"""
from . import operator, partition, halo, expm, krylov, lem, globalexp, phi, metrics, rosenbrock, schrodinger  # noqa: F401
