"""Write tests/golden/oracle_tiny.json: digests of the CPU oracle's renders of
the tiny configuration.  Calls only the oracle and the seeded scene generator,
so a change of these digests means the oracle's arithmetic (or the scene
generator) changed; such a change must name the paper passage that justifies it.
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2310_07182_amd import scenes  # noqa: E402

CASES = [
    dict(mode="incoherent", tile=(4, 4), k=2, seed=2310071820),
    dict(mode="reuse", tile=(4, 4), k=2, seed=2310071820),
    dict(mode="reuse", tile=(8, 8), k=8, seed=7),
    dict(mode="sorted", tile=(4, 4), k=2, seed=2310071820),
]


def digests():
    sc = oracle.OracleScene(scenes.tiny())
    out = []
    for c in CASES:
        r = sc.render(64, 64, 1, 2, **c)
        h = hashlib.sha256()
        for key in ("radiance", "hit_prim", "hit_t"):
            h.update(r[key].tobytes())
        out.append(dict(case=dict(c, tile=list(c["tile"])), sha256=h.hexdigest(),
                        rays_per_bounce=[int(v) for v in r["rays_per_bounce"]],
                        mean_radiance=[float(v) for v in r["radiance"].mean(axis=(0, 1))]))
    return out


if __name__ == "__main__":
    with open(os.path.join(HERE, "oracle_tiny.json"), "w") as f:
        json.dump(dict(config="tiny 64x64, 1 spp, 2 bounces", cases=digests()), f, indent=1)
    print("wrote oracle_tiny.json")
