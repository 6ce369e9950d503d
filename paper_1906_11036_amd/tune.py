"""Run the library's launch autotuner on the benchmark workloads and store the
picks in tuning.json (read by bench.py, so timed and profiled runs launch one
fixed configuration).

    python -m paper_1906_11036_amd.tune [--workloads batch256,gaussian_hill_4096]
                                        [--storages f32,f64,f16neq,bf16neq]
"""
from __future__ import annotations

import argparse
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
TUNING = os.path.join(HERE, "tuning.json")


def load() -> dict:
    if os.path.exists(TUNING):
        with open(TUNING) as fh:
            return json.load(fh)
    return {}


def lookup(workload: str, storage: str):
    """The stored launch (rows_per_wave, waves_per_block, schedule, xcd_remap) or None."""
    entry = load().get(workload, {}).get(storage)
    return tuple(entry["launch"]) if entry else None


def main():
    import torch

    import paper_1906_11036_amd as dg
    from paper_1906_11036_amd import workloads as W

    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="batch256,gaussian_hill_4096")
    ap.add_argument("--storages", default="f32,f64,f16neq,bf16neq")
    ap.add_argument("--trials", type=int, default=8)
    ap.add_argument("--out", default=TUNING)
    args = ap.parse_args()
    table = load()
    for wl in args.workloads.split(","):
        probs = W.batch_problems() if wl == "batch256" else [W.workload(wl)]
        for st in args.storages.split(","):
            b = dg.Batch(probs, storage=st)
            b.set_all_phi()
            b.step(4)
            b.autotune(args.trials)
            inf = b.info(0)
            launch = [inf["rows_per_wave"], inf["waves_per_block"], inf["schedule"], inf["xcd_remap"]]
            b.step(4)
            ms = b.time_steps(32) / 32
            table.setdefault(wl, {})[st] = {"launch": launch, "ms_per_step": round(ms, 5)}
            print(wl, st, launch, f"{ms:.4f} ms/step", flush=True)
            del b
            torch.cuda.empty_cache()
    with open(args.out, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    print("wrote", args.out)


if __name__ == "__main__":
    main()
