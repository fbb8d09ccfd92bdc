"""FP64 CPU oracle for the GW hot path (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the product library never imports, links or calls it.
"""
from . import gw  # noqa: F401
