"""Write the digest of the oracle's result on the 3D workload at a 20^3 grid.

    python tests/golden/make_lap3d_digest.py

The 3D 7-point Laplacian with the seeded random long-range perturbation
(seed 3, scaled to ||Z||_1 = 1.5), cosine series m = 24, PS block s = 5,
tau = 1e-12, on a 20 x 20 x 20 grid (n = 8000).  Its powers fill in to dense
rows, so the oracle needs several minutes of CPU time; the GPU test compares
the HIP result with the stored digest instead of recomputing it.  Only the
oracle computes the stored values.

The digest is SHA-256 over the canonical CSR's bytes: row pointers (int64),
columns (int32), values (float64), all little-endian, in that order.
"""

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

OUT = os.path.join(HERE, "lap3d_side20_cos_m24_s5.json")


def csr_digest(row_ptr, col, val) -> str:
    import numpy as np

    h = hashlib.sha256()
    h.update(np.ascontiguousarray(row_ptr, dtype="<i8").tobytes())
    h.update(np.ascontiguousarray(col, dtype="<i4").tobytes())
    h.update(np.ascontiguousarray(val, dtype="<f8").tobytes())
    return h.hexdigest()


def main():
    import numpy as np

    import oracle as O
    from fps_inputs import generators as G

    cfg = G.config3(side=20)
    t0 = time.time()
    F, st = O.filtered_ps(cfg["Z"], cfg["coeffs"], cfg["m"], cfg["s"], cfg["tau"])
    rec = {
        "workload": "lap3d_perturbed side=20 seed=3 norm1=1.5, cos m=24, s=5, tau=1e-12",
        "n": int(F.n),
        "nnz": int(F.nnz),
        "sha256": csr_digest(F.row_ptr, F.col, F.val),
        "fro_norm": float(np.sqrt(np.sum(F.val * F.val))),
        "products": int(sum(x["products"] for x in st)),
        "stage_nnz": [int(x["nnz_kept"]) for x in st],
        "oracle_seconds": round(time.time() - t0, 1),
    }
    with open(OUT, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
