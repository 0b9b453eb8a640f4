"""Writes split_4096_b256.json, the oracle's reference for the end-to-end
tests of the split-precision paths at a size whose thin products run on the
128 x 128 GEMM tiles (tests/test_gpu_split_oracle.py).

Workload: A = X diag(sigma) Y^T, 4096 x 4096, sigma_j = exp(-j/512) planted
between Haar factors (seed 0), G from seed 1, b = 256, q = 1, the first three
steps (k_stop = 768).  Stored: diag(T)(0:768) and ||T(k:, k:)||_F for
k = 256, 512, 768 from the oracle, and the same after a seeded relative
perturbation A o (1 + delta E) at delta = 2^-24 (FP32's unit roundoff) and
2^-16 (the BF16x3 split's representation error), so that a test can take
its tolerance from the oracle's own response.  Only oracle/ and the seeded
input generators are called.

Usage: python tests/golden/make_split_golden.py   (a few minutes on 8 cores)
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import randutv_ref as ref  # noqa: E402
from paper_1703_00998_amd import workloads as wl  # noqa: E402

M = N = 4096
B, Q, KSTOP = 256, 1, 768
PERTURB_SEED = 7


def sigma():
    return np.exp(-np.arange(1, N + 1, dtype=np.float64) / 512.0)


def inputs():
    A = wl.planted(M, N, sigma(), seed=0)
    G = wl.gaussian_g(M, N, B, seed=1)
    return A, G


def summary(A, G):
    _, T, _, k = ref.randutv(A, B, Q, G, form_u=False, form_v=False, k_stop=KSTOP)
    assert k == KSTOP
    diag = np.diagonal(T)[:KSTOP].tolist()
    tails = [float(np.linalg.norm(T[k:, k:])) for k in (256, 512, 768)]
    return diag, tails


def main():
    A, G = inputs()
    out = {"workload": "4096x4096, sigma_j=exp(-j/512) planted (seed 0), G seed 1, b=256, q=1, "
                       "k_stop=768",
           "citation": "Figure 'The algorithm randUTV' (Section 5.2), run by the FP64 oracle",
           "A_fro": float(np.linalg.norm(A)), "A_00": float(A[0, 0]),
           "A_last": float(A[-1, -1])}
    out["diag"], out["tails"] = summary(A, G)
    E = np.random.default_rng(PERTURB_SEED).standard_normal(A.shape)
    for name, delta in (("fp32", 2.0 ** -24), ("bf16", 2.0 ** -16)):
        Ap = np.asfortranarray(A * (1.0 + delta * E))
        d, t = summary(Ap, G)
        out[f"perturbed_{name}"] = {"delta": delta, "seed": PERTURB_SEED, "diag": d, "tails": t}
        print(name, "done", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "split_4096_b256.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path)


if __name__ == "__main__":
    main()
