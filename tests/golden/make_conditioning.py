"""Write conditioning_spreads.json: the float64 oracle's own spread under
float32-level rounding of its intensity input, for the one-iteration cases of
the small workload.  The GPU parity test scales its bar with these values and
checks that they reproduce.  Calls only the oracle (through tests/_cases.py)
and the seeded input generators.

Usage: python tests/golden/make_conditioning.py"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from _cases import SMALL_ONE_ITER_CASES, small_one_iter_spread  # noqa: E402


def main():
    out = {}
    for alg, B, upd in SMALL_ONE_ITER_CASES:
        sO, sP = small_one_iter_spread(alg, B, upd)
        out[f"{alg}-{B}-{upd}"] = {"spread_object": sO, "spread_probe": sP,
                                   "bar_object": max(1e-5, 100 * sO), "bar_probe": max(1e-5, 100 * sP)}
    with open(os.path.join(HERE, "conditioning_spreads.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
