"""Write the golden fixtures of this folder.  Calls only the CPU oracle.

omega_seed1_r0-63_c0-4.txt : Omega(seed=1)[0:64, 0:5] as FP32 hex bit patterns,
    the generated operand of the small single-block workload (2048 x 5 block,
    seed 1), i.e. GenRandom of Alg. 1 under the Philox reading of Sec. 6.3.
omega_seed2026_offsets.txt : entries at large and unaligned global offsets.
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
import oracle  # noqa: E402

POINTS = [(0, 0), (1, 0), (2, 1), (3, 7), (4093, 4), (4096 * 7 + 1, 2), (1 << 20, 63),
          ((1 << 32) + 5, 1), ((1 << 34) + 3, 1023)]


def main():
    om = oracle.omega_block(1, 0, 64, 0, 5)
    with open(os.path.join(HERE, "omega_seed1_r0-63_c0-4.txt"), "w") as f:
        f.write("# Omega(seed=1) rows 0..63, cols 0..4, FP32 bit patterns (row per line)\n")
        for row in om.view(np.uint32):
            f.write(" ".join(f"{int(v):08x}" for v in row) + "\n")
    with open(os.path.join(HERE, "omega_seed2026_offsets.txt"), "w") as f:
        f.write("# row col fp32-bits of Omega(seed=2026)(row, col)\n")
        for r, c in POINTS:
            v = np.float32(oracle.omega_value(2026, r, c)).view(np.uint32)
            f.write(f"{r} {c} {int(v):08x}\n")


if __name__ == "__main__":
    main()
