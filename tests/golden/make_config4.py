"""Writes config4_krylov_k128_p32_v8_seed11.json: the FP64 oracle's solve of the 16384 x 16384
workload (sigma_i = i^-1/2, reflector-product unitaries, workloads.config4) by the block Krylov
scheme (Alg. 4, Sec. 5) with k = 128, p = 32, a budget of 8 views and sketch seed 11.

Calls only oracle/ and workloads/.  The run takes about half an hour on 8 cores and needs about
25 GB of host memory, so the GPU tests read its stored result instead of running it:
  - sha256: hash of the FP32 planes of A (the GPU side regenerates A and checks the hash first);
  - nA2: ||A||_F^2 of those FP32 values, in FP64;
  - S: the k singular values; pass_err: the oracle's per-view estimates (the last one is the
    error ||A - U diag(S) V^H||_F / ||A||_F of its result, an exact identity in FP64);
  - samples: entries (i, j) of A_hat = U diag(S) V^H at seeded random positions, four planes.

Usage: python tests/golden/make_config4.py [output.json]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
import workloads as W  # noqa: E402

N, K, P, V, SEED = 16384, 128, 32, 8, 11
NSAMPLES, SAMPLE_SEED = 4096, 2025


def sample_entries(U, S, Vm, rows, cols):
    """A_hat[i, j] = sum_t U[i, t] S_t conj(V[j, t]) (quaternion products, eq. (1))."""
    a = U[:, rows, :] * S[None, None, :]                 # (4, N, k)
    b = Vm[:, cols, :].copy()
    b[1:] *= -1.0                                        # conj
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    out = np.stack([
        aw * bw - ax * bx - ay * by - az * bz,
        aw * bx + ax * bw + ay * bz - az * by,
        aw * by - ax * bz + ay * bw + az * bx,
        aw * bz + ax * by - ay * bx + az * bw,
    ])
    return out.sum(axis=2)


def main(path):
    t0 = time.time()
    A32, sigma = W.config4()
    sha = hashlib.sha256(A32.tobytes()).hexdigest()
    print(f"A built in {time.time() - t0:.1f} s, sha256 {sha}", flush=True)
    A = A32.astype(np.float64)
    del A32
    nA2 = float(np.sum(A * A))
    t1 = time.time()
    U, S, Vm, e = O.qlra(A, K, P, V, O.BLOCK_KRYLOV, SEED)
    print(f"oracle solve {time.time() - t1:.1f} s; e = {e.tolist()}", flush=True)
    del A
    rng = np.random.default_rng(SAMPLE_SEED)
    rows = rng.integers(0, N, NSAMPLES)
    cols = rng.integers(0, N, NSAMPLES)
    ah = sample_entries(U, S, Vm, rows, cols)
    rec = {
        "workload": "16384 x 16384 dense quaternion, sigma_i = i^-1/2, reflector-product unitaries "
                    "(workloads.config4, data seed 4)",
        "scheme": "block Krylov (Alg. 4)", "k": K, "p": P, "v": V, "seed": SEED,
        "sha256": sha, "nA2": nA2,
        "S": S.tolist(), "pass_err": [None if np.isnan(x) else float(x) for x in e],
        "sample_seed": SAMPLE_SEED, "rows": rows.tolist(), "cols": cols.tolist(),
        "ahat": ah.tolist(),
        "oracle_seconds": time.time() - t1,
    }
    with open(path + ".tmp", "w") as f:
        json.dump(rec, f)
    os.replace(path + ".tmp", path)
    print(f"wrote {path}", flush=True)


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(here, "config4_krylov_k128_p32_v8_seed11.json"))
