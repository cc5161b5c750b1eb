"""Write the golden response tensors under tests/golden/ with the CPU oracle only.

Configurations (seeded generators, three dipole perturbations):
* alpha_o10v80.json:  o = 10, v = 80, seed 1, z = 0 and z = 0.08 + 0.004i;
* alpha_o16v120.json: o = 16, v = 120, seed 2 (the damped-spectrum size),
  z = 0 + 0.005i and z = 0.5 + 0.005i (both ends of the spectrum).
The response solves use preconditioned GMRES (scipy) on the oracle's Jacobian
transforms; the values are <<X_p; X_q>>_z as complex numbers (real, imag).

Run:  python tests/golden/make_golden.py [o10v80|o16v120]
(several minutes for o10v80, about an hour for o16v120 on a CPU)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from gen import synth as s  # noqa: E402
from oracle import cclr_ref as O  # noqa: E402

CONFIGS = {
    "o10v80": (10, 80, 1, (0.0, 0.08 + 0.004j)),
    "o16v120": (16, 120, 2, (0.005j, 0.5 + 0.005j)),
}


def main(name):
    o, v, seed, zs = CONFIGS[name]
    pb = s.Problem(o, v, seed)
    inst = s.instance(pb)
    H = O.Hamiltonian(o, v, inst["f"].numpy(), {k: x.numpy() for k, x in inst["V"].items()})
    cc = O.CCLR(H, inst["t1"].numpy(), inst["t2"].numpy())
    Xs = [s.dipole(pb, k).numpy() for k in range(3)]
    t0 = time.time()
    cc.solve_lambda("gmres")
    print(f"lambda: done at {time.time() - t0:.0f} s", flush=True)
    out = {"o": o, "v": v, "seed": seed, "perturbations": "dipole k=0,1,2", "method": "oracle GMRES", "values": {}}
    for z in zs:
        a = cc.response(Xs, z, method="gmres")
        out["values"][repr(complex(z))] = [[[x.real, x.imag] for x in row] for row in a]
        print(f"z={z}: done at {time.time() - t0:.0f} s", flush=True)
    with open(os.path.join(HERE, f"alpha_{name}.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "o10v80")
