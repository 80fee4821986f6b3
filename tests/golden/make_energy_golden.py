"""Write the oracle's energy history of the thermal 128 x 128 box (16 ppc,
1 keV, FP64, 1000 steps) to energy_uniform_1000.json, and with --order 6 the
same box under the sixth-order field solver (dt at 0.95 of its stability
limit) to energy_uniform_1000_order6.json.

Calls only the oracle and the seeded workload generator.  The FP32 HIP run
is compared against this history: its energy drift over the same steps must
agree with the oracle's own drift (the explicit scheme heats this
under-resolved plasma by itself) within 1e-3 of the initial energy.

    python tests/golden/make_energy_golden.py [--order 6]
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1511_03878_amd import workloads as W  # noqa: E402


S6 = 75 / 64 + 25 / 384 + 3 / 640  # sum of |c_m| of the sixth-order stencil


def main(nsteps=1000, order=2):
    if order == 6:
        wl = W.to_float32_state(W.uniform_2d(cfl=0.95 / S6))
    else:
        wl = W.to_float32_state(W.uniform_2d())
    s = oracle.Sim(wl["grid"])
    if order == 6:
        s.set_maxwell_order(6)
    s.set_particles(wl["x"], wl["u"], wl["w"])
    U, K = [], []
    for k in range(nsteps):
        s.step(1)
        u, kk = s.energy()
        U.append(u)
        K.append(kk)
        if k % 100 == 0:
            print(k, u + kk, flush=True)
    solver = ("the sixth-order solver, dt = 0.95 of its stability limit" if order == 6
              else "dt = 0.95 of the Yee limit")
    out = {
        "source": "oracle (FP64) on the FP32-rounded thermal 128x128 box, 16 ppc, 1 keV, "
                  f"dx = 0.1 c/omega_p, {solver}; written by tests/golden/make_energy_golden.py",
        "nsteps": nsteps, "U": U, "K": K,
    }
    name = "energy_uniform_1000_order6.json" if order == 6 else "energy_uniform_1000.json"
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main(order=6 if "--order" in sys.argv and sys.argv[sys.argv.index("--order") + 1] == "6" else 2)
