"""Writes c1_ground_state.npz: the self-consistent ground-state orbitals of the
32^3 parity molecule, computed by the oracle's ground-state solver.  They are an
input of the time step (Algorithm 1 starts from ground-state orbitals), shared
by the oracle and the GPU path.  Run from the repository root:

    python tests/golden/make_c1_ground_state.py
"""

import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))

import synth  # noqa: E402
from oracle.ground_state import ground_state  # noqa: E402


def main():
    s = synth.config_system("c1_parity_32")
    t = time.time()
    gs = ground_state(s, tol_rho=1e-11, tol_res=1e-10, verbose=True)
    print(f"done in {time.time() - t:.0f} s, scf {gs['scf_iters']}, rho err {gs['rho_err']:.2e}, "
          f"residual {gs['res']:.2e}")
    out = os.path.join(os.path.dirname(__file__), "c1_ground_state.npz")
    np.savez_compressed(out, psi=gs["psi"], eps=gs["eps"], rho_err=gs["rho_err"], res=gs["res"],
                        digest=np.array(s.digest()))


if __name__ == "__main__":
    main()
