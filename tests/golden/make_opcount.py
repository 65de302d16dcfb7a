"""Writes tests/golden/opcount.json: algorithmic FP64 operations per cell of one RK2
stage (spatial operator + update) for each named workload, counted by running the CPU
oracle with an operation-counting scalar type on the workload's initial state
(+ - * / sqrt pow count one each; comparisons are free).

The count is intensive (per cell), so each workload is evaluated on a slice with its
own vertical resolution and physics and a reduced r/theta extent.  Calls only oracle/.

    python tests/golden/make_opcount.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_2207_04252_amd import synth  # noqa: E402


def main():
    out = {}
    for name, cfg in synth.CONFIGS.items():
        nr = min(cfg.nr, 64)
        nth = min(cfg.nth, 64)
        sl = cfg.scaled(nr, nth, cfg.nz, name=f"{name}@slice")
        ops = oracle.count_ops(sl, synth.noise(sl) if sl.noise_amp else None)
        out[name] = {"ops_per_cell_stage": ops, "slice": [nr, nth, cfg.nz],
                     "fields": cfg.n_fields}
        print(name, ops, flush=True)
    with open(os.path.join(HERE, "opcount.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
