"""Write the FP64 oracle's phi at the end of the long FP32-accuracy cases.

Runs only the oracle (oracle/): the 256^2 slotted-disk turn (8000 steps) and
the 512^2 single vortex to maximum stretch and back (12 800 steps), from the
seeded inputs of paper_2007_07760_amd.inputs, and stores phi rounded to FP32
(a relative rounding of 3e-8, far below the 1e-5 L2 the FP32 runs are held
to) in oracle_phi_fields.npz beside this script.  The 512^2 run takes several
minutes on a few cores, which is why it is stored rather than rerun by the
GPU tests.

    python tests/golden/make_oracle_fields.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2007_07760_amd import inputs as I  # noqa: E402

CASES = (("c2", 8000), ("c3_512", 12800))


def main() -> None:
    out = {}
    for name, steps in CASES:
        w = I.workload(name)
        p = oracle.Params(w["nx"], w["ny"], w["mobility"], w["width"], w["cfl"], w["recon"],
                          w["vel_kind"], w["vel_param"])
        s = oracle.State(p, w["phi0"]).run(steps)
        out[f"{name}_{steps}"] = s.phi().astype(np.float32)
        print(f"{name}: {steps} steps, mass {s.mass():.15e}", flush=True)
    np.savez_compressed(os.path.join(HERE, "oracle_phi_fields.npz"), **out)


if __name__ == "__main__":
    main()
