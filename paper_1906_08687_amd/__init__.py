"""MI355X (gfx950) engine for batches of group-by aggregates over acyclic joins.

The compiled library ``liblmfao.so`` holds the planner, the executor and every
HIP kernel; ``lmfao`` is its ctypes binding.
"""
