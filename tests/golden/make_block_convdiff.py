"""Writes block_convdiff_100.npz: the oracle's block-Krylov result for the
100^3 convection-diffusion system with 16 generators as one block (k = 30
block steps, 200 steps of 1e-4, 5 outputs).  Only oracle/ computes; the
system comes from the seeded generators in workloads/.  The oracle takes
a few minutes here, which is why the result is stored.

    python tests/golden/make_block_convdiff.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import block as OB  # noqa: E402


def problem():
    return W.conv_diff3d(100, 100, 100, ngen=16, gen_len=1000, o=5, k=30, steps=200, dt=1e-4)


def main():
    prob = problem()
    ref = OB.block_verify(prob, p=16)
    res = ref["blocks"][0]
    p, m = res.p, res.H.shape[0]
    # H is block upper Hessenberg: keep its diagonal and sub-diagonal blocks
    diag = np.stack([res.H[i:i + p, i:i + p] for i in range(0, m, p)])
    sub = np.stack([res.H[i + p:i + 2 * p, i:i + p] for i in range(0, m - p, p)])
    v = ref["verdict"]
    np.savez_compressed(os.path.join(HERE, "block_convdiff_100.npz"), basis=ref["basis"], h_diag=diag,
                        h_sub=sub, k_eff=np.int64(res.k_eff), first_step=np.int64(v["first_step"]),
                        row=np.int64(v["row"]))


if __name__ == "__main__":
    main()
