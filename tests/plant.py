"""Planted mistakes in the oracle (CPU only).

`planted(old, new)` compiles a copy of oracle/ctu_oracle.c in which the one
occurrence of `old` is replaced by `new`, and routes the oracle's Python
front end to that copy for the duration of the block.  Pin tests use it to
show that a plausible mistake in the oracle fails the pin."""
import contextlib
import ctypes
import os
import subprocess
import tempfile

import oracle as O


@contextlib.contextmanager
def planted(old, new):
    src = open(O.SRC).read()
    assert src.count(old) == 1, f"plant site must occur exactly once: {old!r}"
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "planted.c")
        so = os.path.join(d, "libplanted.so")
        with open(c, "w") as f:
            f.write(src.replace(old, new))
        subprocess.check_call(["gcc", "-O1", "-std=c99", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
                               "-fPIC", "-shared", "-o", so, c, "-lm"])
        saved = O.lib()
        O._lib = O.configure(ctypes.CDLL(so))
        try:
            yield
        finally:
            O._lib = saved
