"""FP64 CPU oracle for the VLBM grid-refinement method -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product library never does.
"""
