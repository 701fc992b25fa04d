"""Writes life_16384_torus_seed3.txt: the CPU oracle's result for the full-size Game
of Life workload (16384 x 16384 torus, live-cell density 0.3 from seed 3, live
count checked every generation, stop when it is unchanged at 10 consecutive checks
or at 2000 generations).

Only the oracle is called (B3/S23 of Fig. 1 with the stable-count condition); the
stored values are its stop generation, its final live count, the SHA-256 of its
final grid (row-major, one byte per cell, 0 or 1) and the live count after every
generation. Run:  python tests/golden/make_life_golden.py  (about 20 minutes on
8 cores).
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_1609_04567_amd import inputs as I  # noqa: E402

N, SEED, GENS, WINDOW = 16384, 3, 2000, 10
OUT = os.path.join(HERE, "life_16384_torus_seed3.txt")


def main() -> None:
    t0 = time.time()
    a = I.life_input(N, seed=SEED)
    o, r = O.life_run(a, bc=O.BC_TORUS, stable_window=WINDOW, max_iter=GENS, trace_cap=GENS)
    digest = hashlib.sha256(o.tobytes()).hexdigest()
    with open(OUT, "w") as fh:
        fh.write(f"# Game of Life B3/S23 on a {N} x {N} torus, density 0.3 from seed {SEED}; live "
                 f"count every generation; stop when unchanged at {WINDOW} consecutive checks or at "
                 f"{GENS} generations.\n")
        fh.write("# Written by tests/golden/make_life_golden.py from the CPU oracle "
                 f"({O.threads()} threads, {time.time() - t0:.0f} s).\n")
        fh.write(f"rows {N}\ncols {N}\nn {r.n}\nconverged {int(r.converged)}\ncount {r.count}\n")
        fh.write(f"sha256 {digest}\n")
        fh.write("trajectory\n")
        for c in r.trace:
            fh.write(f"{int(c)}\n")
    print(f"n={r.n} count={r.count} sha256={digest} ({time.time() - t0:.0f} s)")


if __name__ == "__main__":
    main()
