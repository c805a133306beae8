"""Run the 3D oracle on the paper's model 2 at k2 = 1 (run by hand; minutes).

Model 2 (section 6.1) is the unit cube with 64^3 fine cells in 8^3 coarse blocks; at
k2 = 1 its permeability is 1 everywhere.  With eta 0.2, K_i^+ = K_i + 2, one pre- and
one post-smoothing and the tolerance 10, the model-2 tables print Dim 1857 for the
three coarse spaces and Cond 3.0 (GMsFEM) / 3.1 (RT0, MsFEM), at a residual reduction
of 1e7.  This writes the oracle's Dim, iteration counts and Lanczos Cond (at that
reduction and converged) to tests/golden/oracle3d_model2_homogeneous.json.  Only the
oracle is called.

    python tests/golden/make_model2_homogeneous.py
"""
import json
import os
import sys
import time
import warnings

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.grid3d import Grid3D  # noqa: E402
from oracle.solver3d import OracleSolver3D  # noqa: E402

if __name__ == "__main__":
    warnings.filterwarnings("ignore")
    t0 = time.time()
    g = Grid3D(64, 64, 64, 8, 8, 8)
    o = OracleSolver3D(g, np.ones(g.nc), 10.0)
    print(f"setup {time.time() - t0:.0f} s, Dim {o.dim}, counts {np.unique(o.counts)}", flush=True)
    F = np.zeros(g.nc)
    F[0], F[-1] = 1.0, -1.0  # a source and a sink in opposite corner cells
    r7 = o.solve(F, rtol=1e-7, maxit=200)
    print(f"reduction 1e7: {r7['iters']} iterations, Cond {r7['cond']:.4f}", flush=True)
    r14 = o.solve(F, rtol=1e-13, maxit=400)
    print(f"rtol 1e-13: {r14['iters']} iterations, Cond {r14['cond']:.4f}", flush=True)
    out = {"_source": "3D oracle on the paper's model 2 at k2 = 1 (permeability 1): 64^3 cells, 8^3 blocks, "
                      "eta 0.2, overlap 2, one pre- and one post-smoothing, tolerance 10, corner source and sink",
           "dim": o.dim, "counts": sorted(set(int(c) for c in o.counts)), "eig_first": [float(x) for x in o.eigs[0][:4]],
           "iters_1e7": r7["iters"], "cond_1e7": r7["cond"], "iters_1e13": r14["iters"], "cond_1e13": r14["cond"],
           "seconds": time.time() - t0}
    with open(os.path.join(HERE, "oracle3d_model2_homogeneous.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)
