"""CPU oracle for the C0 interior-penalty biharmonic solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this
package; only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It is a plain, slow,
float64 implementation written from the paper's definitions (explicit
quadrature of the bilinear form, dense LU per vertex patch, Algorithm 1,
flexible GMRES) and shares no code with the HIP path.
"""

from .c0ip_oracle import *  # noqa: F401,F403
