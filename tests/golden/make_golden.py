"""Writes the stored expected values under tests/golden/.  Calls only oracle/.

    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402


def main():
    P = O.rademacher_probes(12345, 3, 5, 300)
    np.savetxt(os.path.join(HERE, "probes_seed12345_t3_K5_D300.txt"), P, fmt="%d",
               header="Rademacher probes of the oracle: seed 12345, EM iteration t=3, K=5, D=300 "
                      "(rows j, columns k).  Written by tests/golden/make_golden.py.")


if __name__ == "__main__":
    main()
