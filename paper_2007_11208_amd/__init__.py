"""MI355X-native adaptive solver of A x = b (Sanderson & Curtin, arXiv 2007.11208).

The solver itself lives in the HIP library ``libada.so`` (built from ``csrc/``);
:mod:`paper_2007_11208_amd.ada` is its thin ctypes binding. Importing this
package does not load the library; ``ada`` loads it on first use and raises if
it is missing.
"""
__all__ = ["ada", "workloads"]
