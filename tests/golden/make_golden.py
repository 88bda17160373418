"""Write stored expected values for the parity tests.  Calls only the oracle.

    python tests/golden/make_golden.py C1 [n_steps]

Stores, for the named workload, the moments (n_e, mean energy, k_i) every 100
steps (every 10 for n_steps <= 100) and the final state, in
``tests/golden/<name>_oracle_<n_steps>.npz`` together with a hash of the inputs.
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle                      # noqa: E402
import workloads                   # noqa: E402
from oracle import semi_implicit as S   # noqa: E402


def config_hash(cfg):
    def enc(o):
        if isinstance(o, np.ndarray):
            return o.tolist()
        raise TypeError(type(o))
    return hashlib.sha256(json.dumps(cfg, default=enc, sort_keys=True).encode()).hexdigest()[:16]


def main():
    name = sys.argv[1]
    cfg = workloads.config(name)
    n_steps = int(sys.argv[2]) if len(sys.argv) > 2 else cfg["n_steps"]
    every = 10 if n_steps <= 100 else 100
    ops = oracle.build_operators(cfg)
    F = S.initial_state(ops, workloads.density_profile(ops.xhat, cfg["ic"]["ne_peak"]), cfg["ic"]["Te_eV"])
    mom = [S.moments(ops, F)]
    t0 = time.time()
    for n in range(n_steps):
        F = S.step(ops, F, n * ops.dt)
        if (n + 1) % every == 0:
            mom.append(S.moments(ops, F))
            print(f"step {n + 1}/{n_steps}  {time.time() - t0:.0f}s  ne_max {mom[-1][0].max():.4e}", flush=True)
    out = os.path.join(ROOT, "tests", "golden", f"{name.lower()}_oracle_{n_steps}.npz")
    np.savez_compressed(out, moments=np.array(mom), F=F, every=every, n_steps=n_steps,
                        config_hash=config_hash(cfg))
    print("wrote", out)


if __name__ == "__main__":
    main()
