"""FP64 CPU oracle for the SRBE constant-potential step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, table or
constant generator with the HIP library under ``paper_2509_24742_amd/``; the two
meet only on seeded synthetic inputs.

The oracle is a plain, slow, obviously-correct transcription of the method of
Gao, Zhou, Zhang & Xu, "Symmetry-preserving random batch Ewald method for
constant-potential simulation of electrochemical systems" (arXiv 2509.24742):

* ``ewald``   -- the Ewald decomposition with the zero-padded slab correction
                 (Sec. 2, Eqs. (12)-(19)), full reciprocal sums, the electrode
                 matrix A, the vector b, forces and energy;
* ``cp``      -- the constant-potential charge solve (Sec. 2, Eqs. (9)-(11));
* ``srbe``    -- the SRBE estimators for a given sample of Fourier modes
                 (Sec. 3, Eqs. (24)-(27)) and the energy they imply;
* ``langevin`` -- the Euler-Maruyama step of the Langevin thermostat (Sec. 3)
                 with reflecting walls (a reading) and Philox normal deviates;
* ``sampler`` -- the Metropolis sampler of Sec. 3 (Eqs. (28)-(29)) driven by
                 ``philox``, a counter-based generator written from its published
                 definition;
* ``virial``  -- the electrostatic virial (pressure) tensor of the complete energy
                 and its SRBE estimate (a reading: the paper gives none);
* ``ewald2d`` -- the exact quasi-2D Ewald sum (Eq. (14), k_z integral done in
                 closed form) and brute-force 2-D image sums, used only as pins.

Units are the caller's: every Coulomb term is multiplied by ``coulomb_k``
(1.43996454784 eV nm / e^2 for nm, e, V, eV).

Readings of places where the paper is silent or inconsistent are listed in the
functions that take them; each one is pinned by a test in ``tests/``.
"""

from . import philox, ewald, cp, srbe, sampler, ewald2d, virial  # noqa: F401
