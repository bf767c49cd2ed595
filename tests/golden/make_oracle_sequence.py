"""Write the oracle's eigenvalues for every step of a synthetic SCF sequence
(the constructed pencil of the input generator, perturbed step by step) to a
JSON fixture, so that GPU tests at sizes where the oracle takes minutes per
solve can compare every step without re-running it.

Calls only the oracle (oracle/) and the seeded input generator.  Usage:
    python tests/golden/make_oracle_sequence.py N STEPS [SEED]
writes tests/golden/oracle_seq_n{N}_nev{NEV}_steps{STEPS}_seed{SEED}.json
(nev = round(0.1 N), the clustered construction of the n = 8192 sequence
scaled to N, eps_k = 5e-3 * 0.6^k).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import oracle  # noqa: E402
from paper_1007_4400_amd import synth  # noqa: E402


def fixture_path(n, nev, steps, seed):
    return os.path.join(HERE, f"oracle_seq_n{n}_nev{nev}_steps{steps}_seed{seed}.json")


def main():
    n, steps = int(sys.argv[1]), int(sys.argv[2])
    seed = int(sys.argv[3]) if len(sys.argv) > 3 else 0
    wl = synth.scaled(synth.LARGE, n, steps=steps)
    out = {"recipe": f"synth.scaled(synth.LARGE, {n}, steps={steps}), synth.sequence(wl, {seed}); "
                     "oracle.solve(A_k, B, nev) for every step k",
           "n": n, "nev": wl.nev, "steps": steps, "seed": seed, "eps0": wl.eps0, "decay": wl.decay,
           "eigenvalues": [], "oracle_seconds": []}
    for k, (A, B) in enumerate(synth.sequence(wl, seed)):
        t = time.perf_counter()
        lam, _ = oracle.solve(A, B, wl.nev)
        out["oracle_seconds"].append(round(time.perf_counter() - t, 1))
        out["eigenvalues"].append([float(x) for x in lam])
        print(f"step {k}: {out['oracle_seconds'][-1]} s", flush=True)
    with open(fixture_path(n, wl.nev, steps, seed), "w") as f:
        json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
