"""FP64 CPU oracle for the RBM variational-Monte-Carlo hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py``.  It shares no
code with the HIP library and the product never imports it.

Pin status (what fixes each function independently of itself) is listed in
``tests/test_oracle_pins.py``; every function here has at least one pin.
"""
from . import core  # noqa: F401
