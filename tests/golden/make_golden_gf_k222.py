"""Write full-size G(K, w) parity values for tests/test_gpu_fullsize_gf.py.

Calls only the CPU oracle and the seeded input generator.  For the Si-like
2x2x2 system (4 + 26 spin orbitals per cell) at K = Gamma and K = 5, the orbitals
ORBS (every one for IP at Gamma), and the frequencies WIDX of its 64-point grid on
[-1, 1] Ha (spread over the grid: inside and across the IP band, in the gap, and at
the lower EA band edge), it stores G+ and G- from the oracle's own restarted GMRES at tol
1e-13 (a diagonal preconditioner damped by PETA Ha, which changes only the
iteration count), with each solve's final true relative residual.

    python tests/golden/make_golden_gf_k222.py [part [K]]    # hours on 8 cores

With K, only that momentum is solved and its points replace those of the same K in
the part's file (the others are kept).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from paper_2208_07478_amd import synth  # noqa: E402
from oracle import eom, solve  # noqa: E402

PRESET = "si_k222"
KS = (0, 5)
# grid indices of the 64-point grid on [-1, 1]: IP at eight (including the hard removal
# continuum at -0.905 Ha), EA at four up to the lower band edge (inside the EA continuum,
# 0.65 Ha, the oracle's GMRES needs thousands of steps per solve: out of this script's budget)
WIDX = {"ip": (3, 12, 21, 29, 33, 38, 44, 52), "ea": (3, 21, 33, 44)}
# orbitals per (part, K): IP all of them at Gamma and a spread of occupied and virtual ones at
# K = 5; EA (an oracle EA product costs seconds) two occupied and four virtual orbitals at
# Gamma, one of each and a high virtual at K = 5
ORBS = {("ip", 0): range(30), ("ip", 5): (0, 3, 4, 10, 20, 29), ("ea", 0): (0, 3, 4, 10, 20, 29),
        ("ea", 5): (1, 6, 25)}
PETA = 0.25
TOL = 1e-13


def main():
    parts = sys.argv[1:2] or ["ip", "ea"]
    only_k = int(sys.argv[2]) if len(sys.argv) > 2 else None
    t0 = time.time()
    s = synth.preset_system(PRESET)
    grid, eta = synth.preset_query(PRESET)
    E = eom.EOMSystem(s)
    print(f"oracle built in {time.time() - t0:.0f} s", flush=True)
    for part in parts:
        ws = grid[list(WIDX[part])]
        path = os.path.join(HERE, f"si_k222_gf_{part}.json")
        out = {"preset": PRESET, "part": part, "eta": eta, "tol": TOL, "precond_eta": PETA, "widx": list(WIDX[part]),
               "omega": ws.tolist(), "points": []}
        if only_k is not None and os.path.exists(path):
            with open(path) as f:
                out["points"] = [q for q in json.load(f)["points"] if q["K"] != only_k]
        sM, sE = solve.shift_sign(part)
        for K in KS if only_k is None else (only_k,):
            d = E.pack(part, K, E.diag(part, K))
            for p in ORBS[(part, K)]:
                b = E.pack(part, K, E.b_vector(part, K, p))
                e = E.pack(part, K, E.e_vector(part, K, p))
                for w in ws:
                    dinv = 1.0 / (w + 1j * sE * PETA + sM * d)
                    x, it, res = solve.gmres(solve.shifted_operator(E, part, K, w, eta), b, dinv=dinv, tol=TOL,
                                             restart=200, maxiter=20000)
                    g = complex(e @ x)
                    out["points"].append({"K": K, "p": p, "w": float(w), "g": [g.real, g.imag], "res": res,
                                          "iterations": it})
                    print(part, K, p, f"{w:+.4f}", it, f"{res:.1e}", f"{time.time() - t0:.0f} s", flush=True)
                with open(path, "w") as f:
                    json.dump(out, f)


if __name__ == "__main__":
    main()
