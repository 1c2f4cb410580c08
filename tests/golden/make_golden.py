"""Write small_field_checksums.json from the FP64 oracle only (no GPU code involved)."""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import gwsgen  # noqa: E402
import oracle  # noqa: E402


def main():
    scene, grid = gwsgen.workload("small")
    u = oracle.forward(scene, grid)[0]
    picks = [(0, 0), (128, 128), (17, 200), (255, 3), (90, 61)]
    out = {
        "workload": "64 Gaussians, 256x256, 8 um, 520 nm, seed 1001 (gwsgen.workload('small'))",
        "norm_l2": float(np.linalg.norm(u)),
        "sum": [float(u.sum().real), float(u.sum().imag)],
        "pixels": {"%d,%d" % p: [float(u[p].real), float(u[p].imag)] for p in picks},
    }
    with open(os.path.join(HERE, "small_field_checksums.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
