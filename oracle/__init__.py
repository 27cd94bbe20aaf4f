"""FP64 CPU oracle for the tensor-train S_N step-then-truncate method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this
package: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with
the HIP library; both read inputs from the ``workloads`` package.

Two independent forms (paper: arXiv 2503.18056, "Thermal Radiation
Transport with Tensor Trains"):

* ``full``     -- the plain definition: a dense intensity array
                  I[N_s, N_theta, N_phi] stepped by the explicit upwind
                  finite-volume formula (Sec. 3.1, eqs. lhs and upwind) and
                  the backward-Euler absorption/emission split (Sec. 3.2,
                  eqs. couple_a / couple_b and the energy-conserving
                  temperature update).  This is the paper's "traditional
                  S_N" baseline rebuilt.
* ``tt``       -- the same step in tensor-train form (Sec. 4): explicit
                  concatenated cores (Sec. 4.1 Addition) rounded with the
                  Gram-SVD truncation (App. A, Algorithm 1 and A.2).
* ``rounding`` -- Gram-SVD, TT-SVD (App. A.1) and dense-SVD rounding,
                  plus the rank/clip/cluster/gauge rules.
* ``adjoint``  -- discrete adjoint of the full-grid step for the
                  detector-energy loss, and finite differences.
* ``metrics``  -- compression factor (Sec. 5.1), reconstruction and
                  relative Frobenius differences of TTs.

Everything is float64.  Where the paper is silent the readings listed in
the project's design notes are used; each is restated in the docstring of
the function that applies it.
"""
from . import quadrature, full, material, rounding, tt, adjoint, metrics  # noqa: F401
from .setup import Setup  # noqa: F401
