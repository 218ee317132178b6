"""Write the frozen generator draws under tests/golden/ (calls only the oracle).

    python tests/golden/make_golden.py

omega_seed09094061_n6_l7.txt   6 x 7 Gaussian test matrix, seed 0x09094061, stream 0
srft_seed09094061_n32_l8.txt   row 0: the 32 SRFT signs; row 1: the 8 sampled
                               coordinates (padded with -1) for seed 0x09094061
"""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import philox  # noqa: E402


def main():
    seed = 0x09094061
    om = philox.gaussian_omega(6, 7, seed=seed, stream=0)
    np.savetxt(os.path.join(HERE, "omega_seed09094061_n6_l7.txt"), om, fmt="%.17g")
    d = philox.srft_signs(32, seed=seed, stream=0)
    R = philox.srft_sample(32, 8, seed=seed, stream=0)
    row = -np.ones(32)
    row[:8] = R
    np.savetxt(os.path.join(HERE, "srft_seed09094061_n32_l8.txt"), np.stack([d, row]), fmt="%.17g")


if __name__ == "__main__":
    main()
