"""FP64 CPU oracle for the thermal pseudopotential D3Q19 lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check of
__graft_entry__ and by the CPU-baseline leg of bench.py, never by the
product package.  It shares no code with the HIP library.

Pins (the tests that fix it independently of itself) are listed in the test
modules tests/test_oracle_*.py; functions without such a pin are marked
"parity unpinned" in their docstrings.
"""
from . import eos, lbm  # noqa: F401
