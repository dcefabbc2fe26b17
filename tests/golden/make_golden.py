"""Write tests/golden/fr_blob128.json from the CPU oracle only.

The filling-rate run on the 128x128 blob image (seed 1) takes minutes on the
CPU, so its source sequence is stored once.  Inputs come from ``synth``, the
values from ``oracle``; nothing here touches the GPU library.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
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
    print(out["n_prop"], out["oracle_seconds"])


if __name__ == "__main__":
    main()
