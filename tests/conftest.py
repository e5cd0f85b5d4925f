import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

_C_FLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"]


def _ensure_host_libs():
    """Compile the generator and the oracle if nothing is built yet."""
    jobs = [("gen/libafmm_gen.so", ["-fopenmp", "gen/afmm_gen.c", "-lm"]),
            ("oracle/liboracle.so", ["oracle/afmm_oracle.c"])]
    for out, args in jobs:
        if not os.path.exists(os.path.join(ROOT, out)):
            src = [a for a in args if a.endswith(".c")]
            other = [a for a in args if not a.endswith(".c")]
            subprocess.run(["gcc", *_C_FLAGS, *[o for o in other if o != "-lm"], "-o", out,
                            *src, "-lm"], check=True, cwd=ROOT)


_ensure_host_libs()


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
