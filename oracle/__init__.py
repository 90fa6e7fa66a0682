"""ORACLE — test infrastructure only.

A plain, slow, FP64 CPU implementation of the Cholesky-decomposition
Sigma(2) quasi-particle method (arXiv:0912.1459), written from the paper and
sharing no code with the HIP library.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.
"""
