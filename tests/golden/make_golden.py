"""Write c1_oracle.npz from the oracle alone (run from the repository root)."""

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from synth import crystal_for  # noqa: E402
from oracle.pipeline import epsinv_crystal  # noqa: E402
from oracle.epsinv import crystal_qpg  # noqa: E402


def main():
    cr = crystal_for("c1")
    E, chi = epsinv_crystal(cr)
    np.savez_compressed(os.path.join(HERE, "c1_oracle.npz"), epsinv=E, chi0=chi,
                        omegas=cr.omegas, qpg=crystal_qpg(cr))


if __name__ == "__main__":
    main()
