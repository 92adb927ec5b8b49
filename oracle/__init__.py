"""CPU oracle for SGTP planning (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The planner itself never calls it.  See ``sgtp_ref.c`` for
what is computed and which paper passages each function follows.
"""

from .ref import build, load, Oracle  # noqa: F401
