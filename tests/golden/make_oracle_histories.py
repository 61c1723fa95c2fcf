"""Write the FP64 oracle's per-step history for the large workloads.

Runs only the CPU oracle (oracle/) on the seeded inputs of
paper_1108_1954_amd.inputs and stores, per step n, the oracle's
[KE^n, W_E^n, P^{n+1/2}, K^{n+1/2}] rows as text.  The GPU tests compare the
engine's field-energy history with these files.

    python tests/golden/make_oracle_histories.py warm_two_stream   # ~20 min, one core
    python tests/golden/make_oracle_histories.py maxwellian        # ~4 h, one core
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_1108_1954_amd import inputs as I  # noqa: E402

CASES = {
    # Warm two-stream: L=2.053*64, Ng=4096, Np=2^26, dt=0.1, 1000 steps
    "warm_two_stream": lambda: I.warm_two_stream_large(),
    # Warm Maxwellian: L=64 pi, Ng=8192, Np=2^28, dt=0.05, 2000 steps
    "maxwellian": lambda: I.warm_maxwellian_large(),
}


def main(name):
    spec = CASES[name]()
    t = time.time()
    x, v = spec.particles()
    print(f"{name}: generated {spec.np_} particles in {time.time() - t:.0f} s", flush=True)
    p = O.params(spec.L, spec.ng, spec.np_, dt=spec.dt, qm=spec.qm, rho0=spec.rho0)
    t = time.time()
    out = O.run(p, x, v, spec.nsteps, mode=O.DEPOSIT_PLAIN)
    print(f"{name}: {spec.nsteps} steps in {time.time() - t:.0f} s", flush=True)
    path = os.path.join(HERE, f"oracle_history_{name}.txt")
    header = (f"FP64 oracle history, {spec.name}: L={spec.L!r} ng={spec.ng} np={spec.np_} dt={spec.dt} "
              f"steps={spec.nsteps}, plain FP64 deposit.\n"
              "Written by tests/golden/make_oracle_histories.py (oracle only).\n"
              "columns: KE^n  W_E^n  P^{n+1/2}  K^{n+1/2}")
    np.savetxt(path, out["hist"], fmt="%.17g", header=header)
    print("wrote", path, flush=True)


if __name__ == "__main__":
    main(sys.argv[1])
