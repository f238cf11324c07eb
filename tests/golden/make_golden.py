"""Write the oracle regression fixture c1_oracle.json.

The paper prints no worked numerical example, so this fixture records what the
FP64 oracle computes on the seeded C1 workload (64x64 image, 32x32 source,
15x15 PSF, one ray per pixel; the observed image is the oracle's own model at
the true parameters plus the seeded noise).  It calls only the oracle and the
seeded input generator.  A later change to the oracle's arithmetic that moves
these numbers must name the passage of the paper that justifies it.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

from oracle import rtu_oracle as O  # noqa: E402
from paper_2606_30620_amd import synth  # noqa: E402


def c1_with_mock_image():
    """C1 inputs whose observed image is the oracle model at the truth + noise."""
    p = synth.make_problem("C1")
    r = O.loss_grad_problem(p, 0, want_grad=False)
    p.image = (r["model"].detach().numpy() + p.noise.astype(np.float64)).astype(np.float32)
    return p


def main():
    p = c1_with_mock_image()
    # evaluate at a perturbed point so the gradient is not ~0
    p.lens[0] = (p.lens[0].astype(np.float64) + np.array([0.01, 0.005, -0.004, 0.003, -0.002, 0.001, 0.002])).astype(np.float32)
    r = O.loss_grad_problem(p, 0)
    out = {
        "workload": "C1 (64x64, 32x32 source, 15x15 PSF, ss=1), lens perturbed by "
                    "[0.01,0.005,-0.004,0.003,-0.002,0.001,0.002]",
        "loss": float(r["loss"]),
        "chi2_mask": float(r["chi2_mask"]),
        "grad_lens": r["grad_lens"].tolist(),
        "grad_ps": r["grad_ps"].tolist(),
        "grad_latent_sum": float(r["grad_latent"].sum()),
        "grad_latent_l2": float(torch.linalg.norm(r["grad_latent"])),
        "status": int(r["status"]),
    }
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_oracle.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
