"""Write ``served_grad_57529f_128.json``: expected values for one served gradient
request of the served workload's kind at its large end (57 529 faces of a seeded
ellipsoid union with deleted faces, 128^3 voxel centres, sigmoid k = 50 MSE against a
seeded solid ellipsoid), computed by the FP64 oracle alone:

  * W at every voxel centre (Section 2.2, Eq. 5, 7, 8), from which
  * the loss and dL/dW (mean over the voxels of (sigmoid(k (W - 1/2)) - target)^2), and
  * dL/dT = sum_q dL/dW_q dW_q/dv for 64 seeded faces (the chain rule of the solid angle);
  * W at 512 seeded voxels, as a forward check.

Run from the repository root: ``python tests/golden/make_served_grad.py`` (about 15
minutes on 8 cores; the oracle's cost is 1.2e11 point-face pairs).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from wn_inputs.configs import Request  # noqa: E402

MESH_SEED = 11
FACES = 60000
RES = 128
N_FACES_CHECKED = 64
N_VOXELS_CHECKED = 512
SAMPLE_SEED = 300


def main():
    req = Request(0, 0.0, FACES, RES, True, MESH_SEED)
    w = req.build()
    V64 = np.asarray(w.V, np.float32).astype(np.float64)   # the device sees FP32 vertices
    Q = oracle.grid_points(w.grid)
    t0 = time.time()
    W = oracle.winding(V64, w.F, Q)
    t1 = time.time()
    loss, dLdW = oracle.sigmoid_mse(W, w.target, w.tau, w.k)
    rng = np.random.default_rng(SAMPLE_SEED)
    fs = np.sort(rng.choice(len(w.F), N_FACES_CHECKED, replace=False))
    T, _ = oracle.grad(V64, w.F[fs], Q, dLdW)
    qs = np.sort(rng.choice(len(Q), N_VOXELS_CHECKED, replace=False))
    guard = oracle.guard_mask(V64, w.F, Q[qs])
    out = {
        "what": "oracle values for one served gradient request (see make_served_grad.py)",
        "request": {"faces_requested": FACES, "res": RES, "mesh_seed": MESH_SEED, "wants_grad": True},
        "n_vertices": int(len(w.V)),
        "n_faces": int(len(w.F)),
        "tau": float(w.tau),
        "k": float(w.k),
        "loss": float(loss),
        "faces": [int(f) for f in fs],
        "dLdT": np.asarray(T, np.float64).reshape(len(fs), 9).tolist(),
        "voxels": [int(q) for q in qs],
        "W": [float(x) for x in W[qs]],
        "guard": [bool(g) for g in guard],
        "oracle_seconds": t1 - t0,
        "threads": oracle.max_threads(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"served_grad_{len(w.F)}f_{RES}.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(path, f"W in {t1 - t0:.0f} s, loss {loss:.6g}")


if __name__ == "__main__":
    main()
