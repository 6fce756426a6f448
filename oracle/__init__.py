"""FP64 CPU oracle of the coupled LB/FD step (arXiv:2304.05657).

TEST INFRASTRUCTURE ONLY.  The oracle is a plain, slow, obviously correct
restatement of the method in C (``lbfd_oracle.c``) with a ctypes wrapper.
Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it.  It shares no code with the GPU library.
"""
from .oracle import Oracle, build, lib_path, single  # noqa: F401
