"""Write the full-size oracle samples used by tests/test_gpu_fullsize.py.

Calls only the CPU oracle (oracle/) and the seeded input generator.  For the
Si-like 2x2x2 system (4 + 26 spin orbitals per cell) it stores:
  * sigma(x) of seeded random antisymmetric vectors at K = 0 and K = 5, on a
    seeded sample of entries (plus every 1h / 1p entry), for IP and EA;
  * b and e vectors of a few orbitals on the same entries;
  * G+ and G- at a few (K, p, w) points from the oracle's own GMRES (tol 1e-12).

    python tests/golden/make_golden.py      # ~3 minutes on 8 cores
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
NVEC = 120          # sigma batch width of the bench's step (30 orbitals x 4 frequencies)
VEC_IDS = (0, 57, 119)
NSAMPLE = 400
KS = (0, 5)


def sample_index(n, n1, seed):
    rng = np.random.default_rng(seed)
    idx = np.unique(np.concatenate([np.arange(n1), rng.choice(np.arange(n1, n), NSAMPLE, replace=False)]))
    return idx


def cpack(a):
    a = np.asarray(a)
    return [a.real.tolist(), a.imag.tolist()]


def main():
    t0 = time.time()
    s = synth.preset_system(PRESET)
    omega, eta = synth.preset_query(PRESET)
    E = eom.EOMSystem(s)
    print(f"oracle built in {time.time() - t0:.0f} s", flush=True)
    out = {"preset": PRESET, "nvec": NVEC, "vec_ids": list(VEC_IDS), "sigma": [], "vectors": [], "gf": []}
    for part in ("ip", "ea"):
        n1 = s.nocc if part == "ip" else s.nvir
        for K in KS:
            seed = 1000 + 10 * K + (1 if part == "ea" else 0)
            X = synth.random_eom_vectors(s.kmesh, s.nocc, s.nvir, part, K, NVEC, seed=seed)
            assert np.allclose(E.unpack(part, K, E.pack(part, K, X[0])), X[0])  # antisymmetric input
            idx = sample_index(E.size(part), n1, seed)
            for v in VEC_IDS:
                y = E.sigma(part, K, X[v])
                out["sigma"].append({"part": part, "K": K, "seed": seed, "vec": v, "idx": idx.tolist(),
                                     "scale": float(np.abs(y).max()), "val": cpack(y[idx])})
            for p in (0, 3, 4, 29):
                b = E.b_vector(part, K, p)
                e = E.e_vector(part, K, p)
                out["vectors"].append({"part": part, "K": K, "p": p, "idx": idx.tolist(),
                                       "b": cpack(b[idx]), "e": cpack(e[idx])})
            print(part, K, f"{time.time() - t0:.0f} s", flush=True)
    # G at a few points where the oracle's GMRES converges quickly
    for part, K, p, w in (("ip", 0, 0, 0.5), ("ip", 0, 10, 0.5), ("ea", 0, 3, -0.5), ("ea", 5, 29, -0.5)):
        sM, sE = solve.shift_sign(part)
        b = E.pack(part, K, E.b_vector(part, K, p))
        e = E.pack(part, K, E.e_vector(part, K, p))
        d = E.pack(part, K, E.diag(part, K))
        dinv = 1.0 / (w + 1j * sE * eta + sM * d)
        x, it, res = solve.gmres(solve.shifted_operator(E, part, K, w, eta), b, dinv=dinv, tol=1e-12, restart=100)
        out["gf"].append({"part": part, "K": K, "p": p, "w": w, "eta": eta, "g": cpack(e @ x), "res": res,
                          "iterations": it})
        print("gf", part, K, p, w, it, res, f"{time.time() - t0:.0f} s", flush=True)
    with open(os.path.join(HERE, "si_k222_oracle_samples.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
