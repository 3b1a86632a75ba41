"""Writes c1_3d_osem_2epochs.npz: the FP64 oracle's image of the 3D non-TOF
brain-sized workload (128x128x71, 252 views x 344 radial x 2204 planes,
25 subsets, 1e7 counts) after one OSEM epoch from x = 1 and two epochs of
preconditioned SVRG (Algorithm 1 with the clipped step of eq. (sgm);
stepsize 1 / (1 + 0.02 k / n), preconditioner at iterations 0 and n, subset
orders from the seeded generator of the inputs).  Only oracle/ computes; synth/
supplies the seeded inputs.  Run from the repository root:

    python tests/golden/make_c1_osem_2epochs.py

(about 30 minutes on 8 cores).  The GPU test compares its own OSEM + 2 epochs
against this image (relative L2 <= 1e-4).
"""

import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import recon  # noqa: E402
from synth import configs, data  # noqa: E402

EPOCHS = 2
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_3d_osem_2epochs.npz")


def main():
    cfg = configs.get("c1_3d")
    n = cfg["n_subsets"]
    t0 = time.time()
    d = data.make_dataset(cfg)
    beta = configs.beta_value(cfg)
    prob0 = recon.Problem(cfg, d["y"], d["r"], d["mult"], beta=beta, gamma=2.0, eps=1.0, alpha=1.0, delta=1.0)
    print(f"problem ready in {time.time() - t0:.0f} s", flush=True)
    x0 = recon.osem_epoch(prob0, np.ones(prob0.shape))
    m0 = float(x0.max())
    print(f"OSEM done at {time.time() - t0:.0f} s, max {m0:.9g}", flush=True)
    prob = recon.Problem(cfg, d["y"], d["r"], d["mult"], beta=beta, gamma=2.0, eps=1e-3 * m0, alpha=1.0,
                         delta=1e-3 * m0)
    prob._sens_i = prob0._sens_i
    del prob0
    orders = data.subset_orders(cfg, EPOCHS)

    def progress(e, x):
        print(f"epoch {e} done at {time.time() - t0:.0f} s", flush=True)

    x = recon.svrg(prob, x0, EPOCHS, recon.order_rule(orders), recon.stepsize_vanishing(1.0, 0.02, n),
                   recon.pc_update_iters(n), callback=progress)
    np.savez_compressed(OUT, x=x.astype(np.float32), x_osem_max=np.float64(m0), beta=np.float64(beta),
                        orders=np.asarray(orders, np.int32), epochs=np.int32(EPOCHS))
    print(f"wrote {OUT} at {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
