"""FP64 CPU oracle for the APH predistorter -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import this
package.  It shares no code with the GPU library (``paper_1612_09001_amd``) and
never imports it.
"""
from .oracle import (  # noqa: F401
    Oracle, forward, forward_at, backward, ls_normal, threads, build, lib_path,
)
from . import brute  # noqa: F401
from . import pa  # noqa: F401,E402
from . import ila  # noqa: F401,E402
