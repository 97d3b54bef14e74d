"""FP64 CPU oracle of the sheared-suspension LBM + DEM step.

TEST INFRASTRUCTURE ONLY: used by ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py``.  The GPU library never imports it.
"""
