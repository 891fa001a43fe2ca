"""Write the expected values of the n = 2048 convection-diffusion parity test.

Y = T G for the first four Dirichlet vectors of the n = 2048 configuration (seed 4004), computed by
the oracle's sparse direct solve of the whole interior system (Section 3.1's Schur complement
applied through one sparse LU; no nested dissection), for the seeded coefficient fields of that
configuration (seeds 4001-4003).  Calls only `oracle` and the seeded input module; takes about
three minutes on eight cores.

    python tests/golden/make_cfg4_columns.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import sparse_apply  # noqa: E402

COLS = 4
OUT = os.path.join(HERE, "cfg4_convdiff_Y4.npy")


def main():
    P = W.config("cfg4", "convdiff")
    G = np.asfortranarray(P.G()[:, :COLS])
    Y = sparse_apply(P.n, G, P.b, P.c, P.d)
    np.save(OUT, np.ascontiguousarray(Y))
    print(f"wrote {OUT}: {Y.shape}")


if __name__ == "__main__":
    main()
