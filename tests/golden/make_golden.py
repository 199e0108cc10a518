"""Write oracle reference values for the large hardware-efficient-ansatz cases.

Calls only ``oracle`` and ``synth``: the seeded inputs are regenerated here and
on the device side from the same seeds, so only the oracle's outputs are
stored (with a digest of the inputs that produced them).  Usage:

    python tests/golden/make_golden.py 12 16 20 24     # qubit counts

Each case: hardware-efficient ansatz with L = n layers (RY, RZ on every wire,
CNOT ladder), 500 random Pauli strings of weight <= 4, parameters U(-pi, pi),
one energy and the full adjoint gradient.
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def case_inputs(n):
    spec = synth.hea_circuit(n, n)
    ham = synth.random_pauli_sum(n, 500, seed=synth.MASTER_SEED + n)
    theta = synth.uniform_thetas(spec.n_params, 1, seed=synth.MASTER_SEED + n)[0]
    return spec, ham, theta


def main(ns, threads):
    oracle.set_threads(threads)
    for n in ns:
        spec, ham, theta = case_inputs(n)
        t0 = time.time()
        e, g = oracle.energy_grad(spec, ham, theta, "adjoint")
        dt = time.time() - t0
        out = {"n": n, "layers": n, "terms": 500, "seed": synth.MASTER_SEED + n,
               "ham_digest": ham.digest(), "circuit_key": spec.shape_key(),
               "energy": e, "grad": g.tolist(), "oracle_seconds": dt, "oracle_threads": threads}
        path = os.path.join(HERE, f"hea_n{n}.json")
        with open(path, "w") as f:
            json.dump(out, f)
        print(f"n={n}: E={e:.15f} |g|={np.linalg.norm(g):.6f} ({dt:.1f} s) -> {path}", flush=True)


if __name__ == "__main__":
    ns = [int(a) for a in sys.argv[1:]] or [12, 16, 20]
    main(ns, threads=int(os.environ.get("ORACLE_THREADS", "8")))
