"""Write annulus_localisation_case.json: the initial state of one particle of
the annular-passage workload (48x24x48 elements, N_geo=6, 1e7 particles, seed
1004) whose second stage segment is not traced under reference-space
localisation (Sec. 3.2.3) and ends in a neighbour element where Newton on the
previous element's map diverges.  The values are the seeded input generator's
draws; nothing here runs the GPU library or the oracle.

    python tests/golden/make_annulus_localisation_case.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

from paper_2211_05458_amd import workloads as W  # noqa: E402

INDEX = 9471980


def main():
    w = W.config4(n_particles=10_000_000)
    case = {"source": "workloads.config4(n_particles=10_000_000), particle %d" % INDEX,
            "x": w.x[INDEX].tolist(), "v": w.v[INDEX].tolist(), "d": float(w.d[INDEX]),
            "elem_hint": int(w.elem_hint[INDEX])}
    with open(os.path.join(HERE, "annulus_localisation_case.json"), "w") as f:
        json.dump(case, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
