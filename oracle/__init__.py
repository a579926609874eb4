"""CPU oracle of the EVIS event path.  Test infrastructure only: imported by
tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py."""
from . import evis_oracle  # noqa: F401
