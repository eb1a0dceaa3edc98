"""CPU oracle for the PIMI sweep.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py``; never by the product path.  It
shares no code with the HIP library.
"""
