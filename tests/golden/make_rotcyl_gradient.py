"""Write rotcyl_512x256_gradient.json: the FP64 oracle's gradient of the window-mean
drag of the spinning cylinder (512 x 256 cells, D = 32 at (128, 128), Re = 200,
xi seeded in [0, 2), 400 steps, mean C_D over steps 200..399, A_ref = 2R) with
respect to (xi, R), by complex step with the time-step schedule of the real run
frozen.  Calls only the oracle and the seeded input generators.

    python tests/golden/make_rotcyl_gradient.py   (about 40 minutes on one core)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import wlsynth  # noqa: E402
from oracle import adjoint as OA  # noqa: E402

STEPS, WINDOW = 400, 200


def main():
    w = wlsynth.rotating_cylinder_2d()
    xi, R = wlsynth.rotcyl_xi0(0), float(w.body.radius)
    t0 = time.time()
    J, gx, gR, dts = OA.gradient(w, xi, R, STEPS, WINDOW)
    out = {"workload": w.name, "xi": xi, "R": R, "steps": STEPS, "window_start": WINDOW, "tol": 1e-12,
           "J": J, "dJ_dxi": gx, "dJ_dR": gR, "dt_schedule": dts,
           "method": "complex step (h = 1e-30) of the FP64 oracle, time steps frozen",
           "seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "rotcyl_512x256_gradient.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("J", "dJ_dxi", "dJ_dR", "seconds")}))


if __name__ == "__main__":
    main()
