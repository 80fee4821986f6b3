"""Write the oracle's energy history of the thermal 128 x 128 box (16 ppc,
1 keV, FP64, 1000 steps) to energy_uniform_1000.json.

Calls only the oracle and the seeded workload generator.  The FP32 HIP run
is compared against this history: its energy drift over the same steps must
agree with the oracle's own drift (the explicit scheme heats this
under-resolved plasma by itself) within 1e-3 of the initial energy.

    python tests/golden/make_energy_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1511_03878_amd import workloads as W  # noqa: E402


def main(nsteps=1000):
    wl = W.to_float32_state(W.uniform_2d())
    s = oracle.Sim(wl["grid"])
    s.set_particles(wl["x"], wl["u"], wl["w"])
    U, K = [], []
    for k in range(nsteps):
        s.step(1)
        u, kk = s.energy()
        U.append(u)
        K.append(kk)
        if k % 100 == 0:
            print(k, u + kk, flush=True)
    out = {
        "source": "oracle (FP64) on the FP32-rounded thermal 128x128 box, 16 ppc, 1 keV, "
                  "dx = 0.1 c/omega_p, dt = 0.95 of the Yee limit; written by "
                  "tests/golden/make_energy_golden.py",
        "nsteps": nsteps, "U": U, "K": K,
    }
    with open(os.path.join(HERE, "energy_uniform_1000.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
