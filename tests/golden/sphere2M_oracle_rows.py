"""Writes sphere2M_oracle_rows.json: 1,000 rows of the dense Galerkin products
G x and K x on the 2,097,152-triangle unit sphere, computed by the oracle only.

Mesh: octahedron with every face split 512 x 512, vertices projected to the
unit sphere; x ~ N(0,1) from seeds 501 (G, one entry per triangle) and 502
(K, one per vertex); rows drawn without replacement with seed 503; near-field
quadrature order 6 (the order of Table 1 for this size).  Every pair of
triangles is integrated by the regularised rule, so a row costs about ten
seconds of one core.

    python tests/golden/sphere2M_oracle_rows.py [threads]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
import synth  # noqa: E402

NROWS, Q = 1000, 6


def main():
    oracle.build(force=False)
    if len(sys.argv) > 1:
        oracle.set_threads(int(sys.argv[1]))
    v, t = synth.octa_sphere(512)
    rows = np.sort(np.random.default_rng(503).choice(len(t), NROWS, replace=False))
    out = {"mesh": "octa_sphere(512)", "q_near": Q, "rows_seed": 503, "rows": rows.tolist()}
    for name, fn, seed, n in (("G", oracle.slp_rows, 501, len(t)), ("K", oracle.dlp_rows, 502, len(v))):
        x = synth.random_vector(n, seed)
        vals = []
        t0 = time.time()
        for b in range(0, NROWS, 50):
            vals.extend(fn(v, t, Q, rows[b:b + 50], x).tolist())
            print("%s rows %d/%d (%.0f s)" % (name, b + 50, NROWS, time.time() - t0), flush=True)
        out[name] = {"x_seed": seed, "y": vals}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere2M_oracle_rows.json"), "w") as fh:
        json.dump(out, fh)


if __name__ == "__main__":
    main()
