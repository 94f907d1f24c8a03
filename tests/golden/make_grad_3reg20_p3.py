"""Writes grad_3reg20_p3.json: per-sample d log p(x) / d theta of QAOA p=3
MaxCut on a seeded 20-node random 3-regular graph, for 64 bitstrings drawn
by the oracle's Algorithm 1, computed two ways by the CPU oracle only:
forward-mode derivatives of the complex128 state vector (the score-function
gradient's per-sample term, d log p = 2 Re(conj(a) da) / |a|^2) and central
finite differences of log p in FP64 (h = 1e-4).

Run from the repository root:  python tests/golden/make_grad_3reg20_p3.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import instances as I  # noqa: E402
from oracle import gradient as GR  # noqa: E402
from oracle import sampler as S  # noqa: E402

N_SAMPLES = 64


def main():
    c, _, seed = I.workload_grad3reg64(20)
    bits = S.sample_ideal(c, N_SAMPLES, seed)
    idx = S.basis_index(bits)
    score = GR.score(c, idx)
    fd = GR.score_fd(c, idx, h=1e-4)
    out = {
        "source": "oracle/gradient.py score (forward mode) and score_fd (central differences, h = 1e-4); "
                  "bitstrings from oracle/sampler.py sample_ideal",
        "workload": "instances.workload_grad3reg64(20): QAOA p=3 MaxCut, random 3-regular n=20",
        "seed": int(seed),
        "bits": [[int(b) for b in row] for row in bits],
        "score": score.tolist(),
        "score_fd": fd.tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grad_3reg20_p3.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
