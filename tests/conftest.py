import functools
import os
import sys

import numpy as np
import pytest

ROOT = os.path.abspath(os.path.join(os.path.dirname(__file__), ".."))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (run through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU test")


@functools.lru_cache(maxsize=None)
def c1_system():
    import synth

    return synth.config_system("c1_parity_32")


@functools.lru_cache(maxsize=None)
def c1_ground_state():
    """Oracle ground state of the 32^3 parity molecule (stored input fixture)."""
    d = np.load(os.path.join(GOLDEN, "c1_ground_state.npz"))
    s = c1_system()
    assert str(d["digest"]) == s.digest(), "fixture was made for a different molecule"
    return d["psi"], d["eps"]


@functools.lru_cache(maxsize=None)
def c1_model():
    import oracle

    psi, _ = c1_ground_state()
    return oracle.Model(c1_system(), psi)


@functools.lru_cache(maxsize=None)
def c1_oracle_run(n_steps=200, h_thrs=1e-12, axis=0):
    import oracle
    import synth

    rp = synth.config_run("c1_parity_32", n_steps=n_steps, h_thrs=h_thrs, axis=axis)
    return oracle.run(c1_model(), rp)
