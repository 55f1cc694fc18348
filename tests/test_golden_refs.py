"""The stored oracle reference outputs (tests/golden/*.npz, written by
tests/golden/make_refs.py) are what the oracle and the input generator
produce now: the digests of the initial and final ghosted states match a
fresh run, and the stored interior, dt and c_h sequences are bitwise the
fresh run's."""
import os
import sys

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))

import make_refs as M  # noqa: E402


@pytest.mark.parametrize("name", sorted(M.REFS))
def test_stored_reference_is_the_oracle_output(name):
    r = M.REFS[name]
    z = np.load(M.path(name))
    U0, U, dts, chs = M.run_chain(r)
    assert str(z["sha_initial"]) == M.digest(U0)
    assert str(z["sha_final"]) == M.digest(U)
    n, ng = r["n"], M.NG
    assert np.array_equal(z["interior"], U[:, ng:ng + n, ng:ng + n, ng:ng + n])
    assert np.array_equal(z["dt"], dts) and np.array_equal(z["ch"], chs)
    assert len(dts) == r["steps"]


def test_step_params_are_the_oracle_values():
    """the stored benchmark step parameters hold every workload, and C1's
    ten-step dt / c_h chain is bitwise the oracle's (the 3D workloads' rates
    over 192^3-256^3 states take minutes on the host: make_refs.py writes
    them the same way)"""
    import json

    d = json.load(open(M.STEP_PARAMS))
    assert set(d) == {"C1", "C2", "C4", "C5"} and set(d["C4"]) == set(M.C4_VARIANTS)
    assert d["C1"] == M.step_params_c1()
    for leg in ("C2", "C5"):
        assert d[leg]["dt"] > 0 and d[leg]["ch"] > 0
