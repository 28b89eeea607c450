"""Write the oracle's state of the 1D two-soliton workload after its full length.

The 1D two-soliton scattering workload (L = 16384, eps = 0.1, g = (1, c1, 0.5) with the
spin coupling c1 = -0.5 or +0.5, interleaved split, seeded initial field from
`qlg_inputs.two_solitons_1d_L16384`) is run for 20000 steps by the FP64 CPU oracle alone;
psi = a + b after 2000 and after 20000 steps is stored (arrays `psi_2000`, `psi_20000`,
complex128, shape (5, 16384)), together with the parameters used, in
`two_solitons_L16384_oracle_psi.npz` (c1 = -0.5) or
`two_solitons_L16384_c1_plus05_oracle_psi.npz` (c1 = +0.5).

Usage (from the repository root; about 20 minutes on 8 CPU threads per coupling):

    python tests/golden/make_two_solitons_reference.py [--c1 -0.5|0.5]
"""
import argparse
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import qlg_inputs as qi  # noqa: E402
from oracle import qlg_oracle as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = {-0.5: os.path.join(HERE, "two_solitons_L16384_oracle_psi.npz"),
       0.5: os.path.join(HERE, "two_solitons_L16384_c1_plus05_oracle_psi.npz")}
SAVE_AT = (2000, 20000)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--c1", type=float, default=-0.5, choices=sorted(OUT))
    c1 = ap.parse_args().c1
    w = qi.two_solitons_1d_L16384(c1=c1)
    assert w.nsteps == SAVE_AT[-1]
    p = torch.from_numpy(np.ascontiguousarray(w.psi[0])).to(torch.complex128)
    a, b = O.encode(p)
    saved = {}
    t0 = time.time()
    done = 0
    with torch.no_grad():
        for target in SAVE_AT:
            while done < target:
                k = min(500, target - done)
                a, b = O.run(a, b, k, w.eps, w.g, 1, "interleaved")
                done += k
                print("step %d (%.0f s)" % (done, time.time() - t0), flush=True)
            saved["psi_%d" % target] = (a + b).numpy()
    np.savez_compressed(OUT[c1], L=w.nx[0], eps=w.eps, g=np.array(w.g), steps=np.array(SAVE_AT), **saved)
    print("wrote", OUT[c1])


if __name__ == "__main__":
    main()
