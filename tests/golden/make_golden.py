"""Writes the stored expected values under tests/golden/ from the oracle only.

Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import render  # noqa: E402


def main():
    here = os.path.dirname(os.path.abspath(__file__))
    m = render.render_one([1.0, 0.6, 0.0, 0.0, 0.0, 0.0], 53, 0.2, 0.7)
    out = {
        "description": "||m||_2 of a unit-flux exponential, hlr 0.6 arcsec, Gaussian PSF "
                       "FWHM 0.7 arcsec, 0.2 arcsec/px, centred on 53x53 (oracle renderer); "
                       "used to map the SNR range to a flux range (SNR definition: "
                       "Section 2 footnote).",
        "unit_flux_norm_median": float(np.sqrt(np.sum(m * m))),
        "exponential_hlr_over_r0": render.ETA_EXP,
    }
    with open(os.path.join(here, "unit_flux_norm.json"), "w") as f:
        json.dump(out, f, indent=2)
        f.write("\n")


if __name__ == "__main__":
    main()
