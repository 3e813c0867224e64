"""FP64 CPU oracle for the WPCD hot path.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py, never by the product package.  See wpcd.py.
"""
from .wpcd import *  # noqa: F401,F403
