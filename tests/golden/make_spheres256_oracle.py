"""Writes spheres256_oracle.json: the CPU oracle's permeability, mass and
momentum on the full 256^3 random sphere pack (porosity 0.4, radius U[4,12),
seed 2, periodic; FP64 quasi-compressible LBGK, tau 0.7, uniform g_x = 1e-6,
rho0 = 1, from rest) after a fixed number of steps.

Only the oracle and the seeded geometry generator are used (no GPU code):

    python tests/golden/make_spheres256_oracle.py [--steps N]

Permeability follows the Darcy reading k = nu * q / g_x with the superficial
flux q = sum_fluid rho u_x / (rho0 * N_box) over the whole box (the
porosity convention of Section 4.6); the sums are numpy pairwise sums over the
oracle's FP64 fields.  About 0.5 s per step on 8 host threads (2.6 GB per
lattice).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from oracle import tiles_ref  # noqa: E402
from paper_1611_02445_amd import inputs  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "spheres256_oracle.json")
TAU, G, SEED = 0.7, 1e-6, 2


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=400)
    args = ap.parse_args()
    solid, n_sph = inputs.sphere_pack((256, 256, 256), 0.4, 4.0, 12.0, seed=SEED)
    sp = tiles_ref.pad(solid, 7)
    f = O.init(sp)
    t0 = time.time()
    f = O.run(f, sp, TAU, args.steps, force=[G, 0.0, 0.0], periodic=7)
    dt = time.time() - t0
    s = O.sums(f, sp, force=[G, 0.0, 0.0])
    k = O.permeability(f, sp, TAU, G, force=[G, 0.0, 0.0])
    out = {
        "source": "CPU FP64 oracle (oracle/lbm_oracle.c) written by tests/golden/make_spheres256_oracle.py",
        "workload": "256^3 periodic random sphere pack, porosity 0.4, radius U[4,12), seed 2; "
                    "quasi-compressible LBGK, tau 0.7, g_x 1e-6, rho0 1, from rest",
        "spheres": int(n_sph),
        "steps": args.steps,
        "tau": TAU, "g_x": G,
        "n_fluid": int(s[4]),
        "permeability": float(k),
        "mass": float(s[0]),
        "momentum": [float(s[1]), float(s[2]), float(s[3])],
        "oracle_threads": O.num_threads(),
        "oracle_seconds": round(dt, 1),
    }
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=2)
        fh.write("\n")
    print(json.dumps(out))


if __name__ == "__main__":
    main()
