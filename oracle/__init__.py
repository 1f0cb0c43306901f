"""FP64 CPU oracle of DLMPC-ADMM and its brute-force certifiers.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py``; never by the library or its Python binding.
"""
