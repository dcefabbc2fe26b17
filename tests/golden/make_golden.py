"""Write the stored filling-rate sequences of the test suite from the CPU oracle only.

* fr_blob128.json: the 128x128 blob image (seed 1), 16384 pixels;
* fr_config4.json: 8 images of the 256-image batch of synth.config4 (sides
  24..96, seed 3): the largest and 7 more spread over the size range.

These runs take minutes on the CPU, so their source sequences are stored once.
Inputs come from ``synth``, the values from ``oracle``; nothing here touches
the GPU library.  Usage: python tests/golden/make_golden.py [blob128] [config4]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def blob128():
    img = synth.config2()
    t = time.time()
    fr = oracle.filling_rate(img, conn=4)
    out = {
        "cite": "Section 3.4, algorithm filling, on the 128x128 blob image of synth.config2 (4-neighbours, d_+)",
        "generator": "tests/golden/make_golden.py (oracle only)",
        "sha256": synth.sha256(img),
        "n_prop": fr.n_prop,
        "centroid": fr.centroid,
        "oracle_seconds": round(time.time() - t, 1),
        "filled_last": int(fr.filled[-1]),
        "sequence": fr.sequence.tolist(),
    }
    with open(os.path.join(HERE, "fr_blob128.json"), "w") as f:
        json.dump(out, f)
    print("blob128", out["n_prop"], out["oracle_seconds"])


def config4_picks(images):
    """The largest image of the batch and 7 more at evenly spaced size ranks."""
    by_size = sorted(range(len(images)), key=lambda b: (-images[b].size, b))
    ranks = [0] + [round(k * (len(images) - 1) / 7) for k in range(1, 8)]
    return [by_size[r] for r in ranks]


def config4():
    images = synth.config4()
    picks = config4_picks(images)
    recs = []
    t0 = time.time()
    for b in picks:
        img = images[b]
        t = time.time()
        fr = oracle.filling_rate(img, conn=4)
        recs.append({"index": b, "shape": list(img.shape), "sha256": synth.sha256(img), "n_prop": fr.n_prop,
                     "centroid": fr.centroid, "filled_last": int(fr.filled[-1]),
                     "oracle_seconds": round(time.time() - t, 1), "sequence": fr.sequence.tolist()})
        print("config4 image", b, img.shape, fr.n_prop, recs[-1]["oracle_seconds"], flush=True)
    out = {
        "cite": "Section 3.4, algorithm filling, on images of the batch synth.config4 (4-neighbours, d_+)",
        "generator": "tests/golden/make_golden.py (oracle only)",
        "oracle_seconds": round(time.time() - t0, 1),
        "images": recs,
    }
    with open(os.path.join(HERE, "fr_config4.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    which = sys.argv[1:] or ["blob128", "config4"]
    if "blob128" in which:
        blob128()
    if "config4" in which:
        config4()
