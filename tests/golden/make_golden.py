"""Write the regression fixtures under tests/golden/ from the FP64 oracle only.

df_weights_A1.0_dz0.1.txt: quadrature weights of the frequency-shift integral
(Eq. 3 of the paper, Giessibl's formula) for a peak-to-peak amplitude of 1 A
and 0.1 A height steps, j = -5..5 (physical offset j*dz).
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as orc  # noqa: E402


def main():
    w = orc.df_weights(1.0, 0.1)
    np.savetxt(os.path.join(HERE, "df_weights_A1.0_dz0.1.txt"), w, fmt="%.17e",
               header="Eq. 3 (Giessibl) piecewise-linear weights, A=1.0 A, dz=0.1 A, j=-5..5")


if __name__ == "__main__":
    main()
