"""Write the FP64 oracle's results for the full 512^2 forward + adjoint
workload (Nt = 2000, 256 ring sensors, lossy, PML 20) to fwdadj512_oracle.npz.

Calls only the oracle and the seeded input generators:
  data  = H_a p0                    p0 = the workload's 5 blobs (seed 1822)
  dobs  = H_a p1 + 1% noise         p1 = blobs of seed 1823, noise seed 1824
  grad  = H_a^* (data - dobs)       gradient of 0.5 ||H_a p0 - dobs||^2
The arrays are stored rounded to float32 (their relative rounding, ~6e-8, is
far below the 1e-4 parity bar).  Run from the repository root:
    python tests/golden/make_fwdadj512.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import qpat_inputs as qi  # noqa: E402
from oracle import kspace as K  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fwdadj512_oracle.npz")


def main():
    cfg = qi.config("fwdadj512")
    prm, c0, rho0, p0 = cfg["params"], cfg["c0"], cfg["rho0"], cfg["p0"]
    ops = K.Operators(prm, c0, rho0)
    t = time.time()
    data = K.forward(prm, c0, rho0, p0, ops=ops)
    print(f"forward p0 {time.time() - t:.0f} s", flush=True)
    p1 = qi.blobs(512, 512, 1823, radius_cells=110)
    d1 = K.forward(prm, c0, rho0, p1, ops=ops)
    dobs = d1 + 0.01 * np.sqrt(np.mean(d1 ** 2)) * qi.gaussian_field(d1.shape, 1824)
    print(f"forward p1 {time.time() - t:.0f} s", flush=True)
    grad = K.adjoint(prm, c0, rho0, data - dobs, ops=ops)
    print(f"adjoint {time.time() - t:.0f} s", flush=True)
    np.savez_compressed(OUT, data=data.astype(np.float32), dobs=dobs.astype(np.float32),
                        grad=grad.astype(np.float32))
    print("wrote", OUT)


if __name__ == "__main__":
    main()
