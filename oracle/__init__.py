"""CPU oracle for CCSD linear response — test infrastructure only.

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
import this package.  The GPU library never calls it.
"""
