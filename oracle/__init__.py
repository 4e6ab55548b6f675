"""Plain FP64 CPU oracle for approximate coefficient-domain matching pursuit.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2202_12380_amd``) and never imports it.

* ``oracle.core`` - ctypes wrapper around ``mp_oracle.c`` (DGT, cross-kernels,
  the MP loop with real-atom pairs, synthesis).
* ``oracle.textbook`` - numpy textbook MP that recomputes every inner product
  in the signal domain; usable only for tiny signals.
"""
