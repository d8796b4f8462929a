"""FP64 CPU oracle for the hybrid LB/EPD step -- test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import it.  The GPU library never calls it and shares no code with it.
"""
from . import epdlb_oracle  # noqa: F401
