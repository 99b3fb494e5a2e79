"""Write the stored expected values of the GPU parity tests.

Calls only the CPU oracle (oracle/) on the seeded workloads; run from the
repository root:  python tests/golden/make_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2204_14242_amd import workloads as W  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def main():
    oracle.build()
    t = time.time()
    k, hw, sp = W.stencil_plain()
    res, rank = oracle.estimate(k, hw, sp)
    np.savez(os.path.join(HERE, "stencil_plain_256.npz"), results=res, rank=rank)
    print(f"stencil_plain_256: {len(res)} configs in {time.time() - t:.1f} s")


if __name__ == "__main__":
    main()
