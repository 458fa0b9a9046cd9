"""Write tests/golden/full_configs.json: oracle schedules and plan counters on the
full-size meson_ring and baryon_mix workloads (structure only, FP64 sizes).

Calls only the oracle (and the seeded generators).  The Tree schedule of the
meson workload takes about half a minute in pure Python, hence the stored file.
Run: python tests/golden/make_full_configs.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from synth import workloads as W  # noqa: E402
from oracle import dag as OD, planner as OP, schedules as OS  # noqa: E402

KEYS = ("peak_resident", "n_evict", "n_h2d", "h2d_bytes", "n_d2h", "d2h_bytes", "n_steps")


def main():
    out = {}
    for name in ("meson_ring", "baryon_mix"):
        wl = W.config(name, with_data=False)
        d = OD.build(wl.leaves, wl.graphs)
        if wl.budget_rule == "quarter_input_peak_live":
            budget = OS.memsim(d, OS.input_order(d))["peak_live"] // 4
        else:
            budget = wl.budget_bytes
        entry = {"budget": budget, "policies": {}}
        for policy in ("input", "sibling", "tree"):
            order = OS.schedule(d, policy)
            sim = OS.memsim(d, order)
            g = {"order_sha256": hashlib.sha256(np.asarray(order, dtype=np.int64).tobytes()).hexdigest(),
                 "peak_post": sim["peak_post"], "peak_live": sim["peak_live"], "plans": {}}
            for mode in ("per_contraction", "waves"):
                res = OP.plan(d, order, budget=budget, batched=(mode == "waves"))
                g["plans"][mode] = {k: res[k] for k in KEYS}
            entry["policies"][policy] = g
            print(name, policy, g["peak_post"], g["plans"]["waves"], flush=True)
        out[name] = entry
    with open(os.path.join(HERE, "full_configs.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
