"""Write the stored oracle results used by the GPU full-run parity tests.

Calls only the FP64 oracle (``oracle/``) and the seeded input generators; no
value here comes from the HIP library.

    python tests/golden/make_golden.py blobs64      # ~1 min
    python tests/golden/make_golden.py tissue160    # ~25 min
    python tests/golden/make_golden.py microscopy128  # ~3 min

Each output ``<name>_oracle.npz`` holds the per-iteration loss history, the
final displacement sampled on a strided grid (``field_stride``), the final
singularity fraction and, for labelled workloads, the Dice overlap of the
nearest-neighbour warped labels.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2404_01249_amd import synth  # noqa: E402

STRIDES = {"blobs64": 2, "tissue160": 4, "microscopy128": 2}


def main(name):
    p = synth.load(name)
    P = O.Params(eta=0.5, sigma_grad=1.0, sigma_warp=0.5, window=p.window)
    t0 = time.time()

    def cb(level, i, d, m, v, L, ex):
        if i % 25 == 0:
            print(f"level {level} iter {i} loss {L:.6f} ({time.time() - t0:.0f} s)", flush=True)

    d, losses, t = O.register(p.fixed, p.moving, p.scales, p.iters, P, callback=cb)
    s = STRIDES[name]
    out = dict(losses=np.asarray(losses, np.float64), field=d[:, ::s, ::s, ::s].astype(np.float32),
               field_stride=np.int64(s), singular=np.float64(O.singular_fraction(d)),
               eta=np.float64(P.eta), sigma_grad=np.float64(P.sigma_grad),
               sigma_warp=np.float64(P.sigma_warp), window=np.int64(P.window),
               scales=np.asarray(p.scales, np.float64), iters=np.asarray(p.iters, np.int64))
    if p.fixed_labels is not None:
        warped = O.warp_labels_nearest(p.moving_labels, d)
        out["dice"] = np.float64(O.dice(warped, p.fixed_labels, range(4)))
        out["dice_identity"] = np.float64(O.dice(p.moving_labels, p.fixed_labels, range(4)))
    np.savez_compressed(os.path.join(HERE, f"{name}_oracle.npz"), **out)
    print(f"wrote {name}_oracle.npz in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["blobs64"]:
        main(n)
