"""Plain FP64 CPU oracle of the VIP method (test infrastructure only).

Used only by the tests, the smoke entry point and the CPU-baseline leg of the
benchmark, to check the HIP library.  It shares no code with the library: it
reads the same input arrays (node set, boundary table, fields) and computes
every result on its own, in NumPy/SciPy, following the paper's definitions.

Modules: `mls` (shape functions, Section 3), `operators` (VIP operators,
Section 4), `step` (fractional step, eqs. 12-15), `forces` (body force by traction,
Section 5.4), `krylov` (timing-mode
solvers), `exact` (closed-form solutions).
"""
from . import exact, forces, krylov, mls, operators, step  # noqa: F401
