"""Plain CPU FP64 oracle for the ensemble Fourier-Chebyshev DNS step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
C ABI or its Python binding) may import, call or link anything in this
package.  It is used by ``tests/``, by ``__graft_entry__.smoke()`` and by the
``cpu_baseline`` leg of ``bench.py``.  It shares no code with the HIP path.

The oracle follows the paper (arXiv 2306.12739, "vectorized Navier-Stokes
ensemble DNS") step by step, in the paper's order and notation:

* ``cheb``        -- Chebyshev-Gauss-Lobatto nodes and collocation derivative
                     matrices, including the clamped fourth-derivative operator
                     (Sec. 2, discussion after Eq. (Dv_F)).
* ``spectral``    -- x-z Fourier transforms with 3/2 zero padding (Sec. 3.2,
                     2/3-rule dealiasing).
* ``operators``   -- pre-inverted Crank-Nicolson operators per (kx, kz) pair
                     (Sec. 3.2, Eqs. (CN1)-(CN4), Listings 1 and 3).
* ``step``        -- one CN/RK3 time step of the whole ensemble (Sec. 3.1),
                     with the paper's advective nonlinear term or, as an
                     alternative discretization, its rotational form.
* ``diagnostics`` -- energy, dissipation, power input, flux, one-point
                     statistics (Sec. 4, one-point statistics paragraph).
* ``s3t``         -- approximate S3T ensemble (Sec. 4): members sharing one
                     streamwise-mean flow, quasi-linear perturbations,
                     additive (Lap v, eta) forcing.
* ``optimal``     -- optimal disturbances of a frozen streamwise-mean flow by
                     forward-adjoint iteration with Gram-Schmidt (App. B).
* ``sno``         -- learned spin-up (not in the paper): channel form of a
                     state and back to an admissible state, a spectral neural
                     operator with its gradient, AdamW.

Every function here is written for clarity, not speed: library primitives
(numpy FFTs, ``numpy.linalg.solve``, matrix products) are the only building
blocks, with no blocking, fusion or reordering beyond what the paper states.
"""

from .cheb import (nodes, diff_matrix, dirichlet_d2, clamped_matrices,
                   clenshaw_curtis_weights)
from .spectral import SpectralGrid
from .operators import ModeOperators, MeanOperators
from .step import OracleDNS
from .s3t import OracleS3T
from . import diagnostics
from . import sno
from . import optimal

__all__ = [
    "nodes", "diff_matrix", "dirichlet_d2", "clamped_matrices",
    "clenshaw_curtis_weights", "SpectralGrid", "ModeOperators",
    "MeanOperators", "OracleDNS", "OracleS3T", "diagnostics", "sno", "optimal",
]
