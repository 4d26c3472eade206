"""Plain CPU reference implementations (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP
library in ``paper_2303_14119_amd`` and never imports it.

* ``oracle.solver``  -- FP64 C solver (``oracle.c``) behind ctypes.
* ``oracle.theory``  -- the single-particle SEEA prediction (Eq 19-20).
* ``oracle.mlp``     -- FP64 numpy MLP forward/backward and AdamW.
* ``oracle.warm``    -- enclosed-charge profile and warm-start state.
"""
