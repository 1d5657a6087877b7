"""CPU fp64 oracle for the implicit Discrete Elastic Rods step.

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
cpu_baseline leg of bench.py.  The product path (the HIP library and its Python
binding) never imports or calls anything in this package.
"""
from . import der  # noqa: F401
