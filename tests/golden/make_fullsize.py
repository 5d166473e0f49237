#!/usr/bin/env python3
"""Write the full-size oracle fixtures ``fullsize_*.json`` (CPU only).

The full-size workloads (2D 1024^2 at p = 4 and p = 3, 3D 256^3 at p = 4)
take the CPU oracle from tens of seconds to minutes per solve, too long to
repeat inside a GPU test.  This script runs the oracle's plain FP64 PSD loop
(Sec. 2.2 with the preconditioner of Sec. 5.3 and the exact line search of
Sec. 6.1) once per workload and stores what the GPU tests compare against:

  * the iteration count at ||f - N_h[u]||_inf <= 1e-10 from u0 = 0 and the
    per-update history (alpha_k, ||r_k||_inf);
  * the converged iterate at 1024 seeded sample cells (plus the cell of the
    largest |u|), its max-norm, mean and root-mean-square;
  * the iterate after exactly three updates at the same cells;
  * a rounding scale of the residual, max|u| + s max|div_h(...)| +
    s eps^2 max|Delta_h^2 u|, from which the tests bound the rounding noise
    of alpha_k.

Only ``oracle`` and the seeded input generators are called.  Usage:
    python tests/golden/make_fullsize.py [c2_p4 c2_p3 c3]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import psd_inputs  # noqa: E402

NSAMPLE = 1024
SAMPLE_SEED = 1607_777


def workloads():
    return {
        "c2_p4": psd_inputs.config2(4.0),
        "c2_p3": psd_inputs.config2(3.0),
        "c3": psd_inputs.config3(),
    }


def sample_cells(N: int, u: np.ndarray, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    idx = rng.choice(N, size=NSAMPLE, replace=False)
    idx = np.union1d(idx, [int(np.argmax(np.abs(u.ravel())))])
    return idx.astype(np.int64)


def run(name: str, w) -> dict:
    O = oracle.Problem(w.dim, w.n, w.L, p=w.p, s=w.s, eps=w.eps)
    t0 = time.time()
    ref = O.solve(w.f, tol=1e-10, max_iter=500, history=True)
    t1 = time.time()
    k3 = O.solve(w.f, tol=0.0, max_iter=3)
    t2 = time.time()
    u = ref["u"]
    idx = sample_cells(u.size, u, SAMPLE_SEED)
    scale = (np.abs(u).max() + w.s * np.abs(O.plap(u)).max()
             + w.s * w.eps ** 2 * np.abs(O.lap(O.lap(u))).max())
    fl = lambda a: [float(x) for x in a]
    return {
        "workload": w.name,
        "problem": {"dim": w.dim, "n": w.n, "L": w.L, "p": w.p, "s": w.s, "eps": w.eps},
        "generator": "psd_inputs." + ("config2(%g)" % w.p if w.dim == 2 else "config3()"),
        "tol": 1e-10,
        "iters": int(ref["iters"]),
        "res0_inf": float(np.abs(w.f).max()),
        "alpha": fl(ref["hist"][:, 0]),
        "res_inf": fl(ref["hist"][:, 1]),
        "rounding_scale": float(scale),
        "sample_idx": [int(i) for i in idx],
        "u_final": {"samples": fl(u.ravel()[idx]), "absmax": float(np.abs(u).max()),
                    "mean": float(u.mean()), "rms": float(np.sqrt(np.mean(u * u)))},
        "u_k3": {"samples": fl(k3["u"].ravel()[idx]), "absmax": float(np.abs(k3["u"]).max())},
        "oracle_seconds": {"solve": round(t1 - t0, 1), "three_updates": round(t2 - t1, 1)},
    }


def main(argv):
    names = argv or list(workloads())
    ws = workloads()
    for name in names:
        print(f"oracle: {name}", flush=True)
        rec = run(name, ws[name])
        path = os.path.join(HERE, f"fullsize_{name}.json")
        with open(path, "w") as fh:
            json.dump(rec, fh, indent=0)
        print(f"  iters {rec['iters']}  {rec['oracle_seconds']}  -> {path}", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
