"""Reference oracle for the space-time sparse-grid combination technique.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, double-precision CPU
implementation of what the GPU library computes, written directly from the
paper (Ferrari, Moiola, Perinati, Perugia, "A space-time sparse-grid method
for the wave equation").  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it.  It shares no code with the
HIP path (``paper_2606_09688_amd``) and never imports it.

Every step follows the paper's definitions with library primitives (sparse
matrix products, SuperLU, Gauss-Legendre nodes) and nothing else:

* ``levels``  - combination index set and signs, eq. (19), Fig. 1.
* ``basis``   - clamped quadratic C^1 B-splines in time (Sec. 2.2, Rem. 1,
                Sec. 3.2 with p_t = 2, r_t = 1) and P1/Q1 hats in space.
* ``space``   - spatial mass and c^2-weighted stiffness matrices (eq. 9).
* ``timemat`` - the time matrices A_{j_t}, B_{j_t} of Prop. 1 (eq. 30) and
                the load factors of eq. (9), weighted by e^{-t/T}.
* ``method``  - one Galerkin solve per component (eq. 9), the signed
                combination (eq. 19) plus the lift by u0 (Sec. 2.1), its
                adjoint, and the full-grid solve P_{J,J}.

Readings of points the paper leaves open (level convention, how nodal data
are turned into functions, quadrature) are stated in the docstring of the
function that uses them.
"""

from . import levels, basis, space, timemat, method  # noqa: F401
from .method import Problem  # noqa: F401
