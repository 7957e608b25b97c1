"""CPU oracle for aggregate batches over joins: TEST INFRASTRUCTURE ONLY.

May be imported only by tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``; the engine never calls it.
"""
from .oracle import Result, brute_force, build, evaluate  # noqa: F401
