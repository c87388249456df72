"""FP64 CPU oracle for the distributed-MIMO hot path (test infrastructure only).

Only the tests, the smoke check and the CPU baseline leg of the benchmark may
import this package.  The library itself never does, and the package shares no
code with the HIP path.
"""
from . import dmimo_oracle, brute, dberror  # noqa: F401
