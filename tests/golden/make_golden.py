"""Write the stored expected probe waveforms used by the GPU parity tests.

Every value here is computed by the FP64 oracle (oracle/) from the seeded
inputs of paper_2207_06908_amd.scenarios; nothing comes from the GPU path.

    python tests/golden/make_golden.py [config2_full|config2_small|config3_subset|all] [--threads N]
"""
import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import orc  # noqa: E402
from paper_2207_06908_amd import scenarios as S  # noqa: E402

CONFIG3_SUBSET = list(range(0, 256, 16))  # 16 grids of the 256-grid sweep


def _save(name, sc_list, outs):
    data = {}
    for sc, out in zip(sc_list, outs):
        for pname, w in out.items():
            data[f"{sc.name}/{pname}"] = w
    path = os.path.join(HERE, name + ".npz")
    np.savez_compressed(path, **data)
    print("wrote", path, len(data), "waveforms", flush=True)


def run(sc):
    t = time.time()
    out = orc.run_scenario(sc, S.apply)
    print(f"{sc.name}: {sc.cells} cells x {sc.n_steps} steps in {time.time() - t:.1f} s", flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", default="all", nargs="?")
    ap.add_argument("--threads", type=int, default=os.cpu_count())
    a = ap.parse_args()
    orc.build(force=False)
    orc.set_threads(a.threads)
    if a.which in ("config2_small", "all"):
        sc = S.config2_small()
        _save("config2_small", [sc], [run(sc)])
    if a.which in ("config3_subset", "all"):
        grids = S.config3()
        sub = [grids[g] for g in CONFIG3_SUBSET]
        _save("config3_subset", sub, [run(g) for g in sub])
    if a.which in ("config2_full", "all"):
        sc = S.config2()
        _save("config2_full", [sc], [run(sc)])


if __name__ == "__main__":
    main()
