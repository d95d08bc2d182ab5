"""Plain FP64 CPU oracle for the staggered FFT phase-field fracture solve.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the HIP path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it; the product package never does, and nothing here imports the
product package.  The two share no code.

Method source: Andrews & Pastewka, "Crack-path selection in phase-field models
for brittle fracture" (arXiv:2203.16467).  Each function cites the section,
equation or algorithm it follows.  Where the paper is silent or garbled the
reading taken is stated in the docstring (same reading on the GPU side).

Representation choices that differ on purpose from the GPU path:
  * tensors are full 2x2 symmetric matrices, shape (ny, nx, 2, 2), with the
    inner product A:B = sum_ij A_ij B_ij;
  * the constitutive split uses ``numpy.linalg.eigh`` eigen-decompositions,
    and the spectral tangent is written in the eigenbasis;
  * transforms are full complex ``numpy.fft.fft2`` / ``ifft2``.

Modules
  spectral      -- grid wavevectors, compatibility projection, collocation
                   Laplacian (Sec. 3.1, 3.1.1, 3.1.2)
  constitutive  -- energy densities, splits, stresses, tangent (Sec. 2.1)
  mechanics     -- Fourier-Galerkin Newton + CG (Sec. 3.1.1)
  phasefield    -- F_phi, J, bound-constrained CG (Sec. 3.1.2, Alg. 1)
  evolution     -- alternating minimisation load step, energies (Sec. 3.2.1,
                   Alg. 2)
"""

from . import spectral, constitutive, mechanics, phasefield, evolution  # noqa: F401
from .evolution import Problem  # noqa: F401
