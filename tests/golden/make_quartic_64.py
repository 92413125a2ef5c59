"""Write ``quartic_64.json``: oracle statistics of the block order parameter
of the 64^3 critical-point workload (a = 0, b = 0.1, kappa = 0.1, kT = 1e-4,
tau = 1), which the GPU statistics are tested against.

Observables (Sec. II B): the box means m_L of the order parameter phi =
(rho - rho0)/rho0 over the boxes of edge L_b = 32, 16, 8, 4, 2, 1 (Eq. (mL)),
their second and fourth moments (Eqs. (ML), (chiL)) and the Binder ratio
U = 1 - <m^4> / (3 <m^2>^2).  Run shape of the workload: 20000 steps, the
first 3500 discarded, a sample every 10 steps (1650 samples), statistics
from 15 consecutive batches of 110 samples.

Only the oracle (``oracle/``) steps the model here; the seeds and parameters
come from ``workloads``.  Usage: ``python tests/golden/make_quartic_64.py
[seed_index ...] [--out PATH]`` (about 8 minutes per seed on 16 host
threads); runs already in PATH are kept, so the seeds can be run one call at a
time.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import workloads  # noqa: E402
from oracle import moments  # noqa: E402

L = 64
STEPS, DISCARD, EVERY, NBINS = 20000, 3500, 10, 15
LEVELS = (32, 16, 8, 4, 2, 1)
SEEDS = (workloads.SEED + 64, workloads.SEED + 65)
OUT = os.path.join(HERE, "quartic_64.json")


def run(seed):
    sim = oracle.Sim(L, seed, **workloads.MODEL)
    t0 = time.time()
    m2 = {Lb: [] for Lb in LEVELS}
    m4 = {Lb: [] for Lb in LEVELS}
    while sim.t < STEPS:
        sim.step(EVERY)
        if sim.t % 1000 == 0:
            print(f"seed {seed}: step {sim.t} ({time.time() - t0:.0f} s)", flush=True)
        if sim.t <= DISCARD:
            continue
        phi = moments.order_parameter(sim.rho())
        for Lb in LEVELS:
            m, _ = moments.block_values(phi, L, Lb)
            m2[Lb].append(float(np.mean(m ** 2)))
            m4[Lb].append(float(np.mean(m ** 4)))
    n = len(m2[LEVELS[0]])
    assert n == (STEPS - DISCARD) // EVERY and n % NBINS == 0
    out = {}
    for Lb in LEVELS:
        b2 = np.array(m2[Lb]).reshape(NBINS, -1).mean(axis=1)
        b4 = np.array(m4[Lb]).reshape(NBINS, -1).mean(axis=1)
        out[str(Lb)] = {"m2_batches": b2.tolist(), "m4_batches": b4.tolist()}
    return out


def main(argv):
    out = OUT
    if "--out" in argv:
        i = argv.index("--out")
        out = argv[i + 1]
        argv = argv[:i] + argv[i + 2:]
    which = [SEEDS[int(a)] for a in argv] or list(SEEDS)
    data = {
        "what": "oracle batch means of <m_L^2> and <m_L^4> (box means of phi, Sec. II B Eq. (mL))",
        "L": L, "params": workloads.MODEL, "steps": STEPS, "discard": DISCARD, "sample_every": EVERY,
        "nbins": NBINS, "levels": list(LEVELS), "seeds": list(SEEDS), "runs": {},
    }
    if os.path.exists(out):
        with open(out) as fh:
            data["runs"] = json.load(fh)["runs"]
    for seed in which:
        data["runs"][str(seed)] = run(seed)
        with open(out, "w") as fh:
            json.dump(data, fh, indent=1)
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
