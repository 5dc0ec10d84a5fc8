"""Build and time compile-time shapes of the FP32 pair sweep.

Each shape is the library compiled with other values of the macros
HAWKES_KT (target rows per lane), HAWKES_UJ_GRAD / HAWKES_UJ (unroll of the
source loop in the loglik+gradient sweep / the loglik-only sweeps),
HAWKES_GS (FP32 terms per FP64 fold) and HAWKES_WAVES_PER_EU (register
budget), into paper_2407_11349_amd/_variants/.  Every shape is timed with the
library's own HIP-event hook on the 1e6-event, 1200-day workload (FP32
log-likelihood + gradient, and the FP32 skip mode), for several group counts
of the symmetric sweep and for the row sweep; its result is compared with the
first shape's and with the stored FP64 oracle value of that workload.

    python -m paper_2407_11349_amd.tune_shapes build [shape ...]
    python -m paper_2407_11349_amd.tune_shapes time [--n N] [shape ...]
"""

from __future__ import annotations

import argparse
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

from .build import CSRC, HIPCC_FLAGS, ROOT, SOURCES, hipcc

OUT = Path(__file__).resolve().parent / "_variants"

# name -> macro definitions
SHAPES = {
    "kt2": {"HAWKES_KT": 2},
    "kt2_uj1": {"HAWKES_KT": 2, "HAWKES_UJ_GRAD": 1},
    "kt2_uj2": {"HAWKES_KT": 2, "HAWKES_UJ_GRAD": 2},
    "kt2_uj8": {"HAWKES_KT": 2, "HAWKES_UJ_GRAD": 8},
    "kt2_w3": {"HAWKES_KT": 2, "HAWKES_WAVES_PER_EU": 3},
    "kt1": {"HAWKES_KT": 1},
    "kt4": {"HAWKES_KT": 4},
}

# how whole-set FP32 calls are swept: ("sym", groups) or ("rows", target workgroups)
MODES = [("sym", 160), ("sym", 200), ("sym", 256), ("sym", 320), ("sym", 384), ("rows", 32768)]


def _build_one(name: str) -> str:
    OUT.mkdir(exist_ok=True)
    defs = [f"-D{k}={v}" for k, v in SHAPES[name].items()]
    out = OUT / f"libhawkes_{name}.so"
    cmd = [hipcc(), *HIPCC_FLAGS, *defs, "-I", str(ROOT / "include"), "-I", str(CSRC),
           *[str(CSRC / s) for s in SOURCES], "-o", str(out), "-Rpass-analysis=kernel-resource-usage"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {name}:\n{res.stderr}")
    # register use and occupancy of the gradient sweep
    lines = res.stderr.splitlines()
    info = []
    for i, line in enumerate(lines):
        if "Function Name" in line and "k_pair_f32ILb1ELb0" in line:
            for l2 in lines[i + 1:i + 14]:
                m = re.search(r"remark:\s+(.*?)\s*\[-Rpass", l2)
                if m and m.group(1).split(":")[0] in ("VGPRs", "ScratchSize [bytes/lane]", "Occupancy [waves/SIMD]"):
                    info.append(m.group(1))
            break
    return f"{name}: " + ", ".join(i.strip() for i in info)


def build(names) -> None:
    with ThreadPoolExecutor(max_workers=4) as pool:
        for line in pool.map(_build_one, names):
            print(line, flush=True)


def time_shapes(names, n: int) -> None:
    import numpy as np
    import torch

    sys.path.insert(0, str(ROOT))
    import synth
    from . import _lib
    from . import likelihood as hk

    ev = synth.generate(synth.N1M, n=n)
    th = synth.theta_default()
    dev = hk.DeviceEvents.from_arrays(ev.t, ev.x, ev.y, ev.s)
    ref = None
    gold = None
    gpath = ROOT / "tests" / "golden" / "oracle_values.json"
    if n == 1_000_000 and gpath.exists():
        import json

        gold = json.load(open(gpath)).get("n1m")
    for name in names:
        _lib._lib = None
        lib = _lib.load(OUT / f"libhawkes_{name}.so")
        hk.set_timing(True)
        ws = hk.Workspace(n, "fp32")  # the skip mode uses the same layout
        for mode, size in MODES:
            if mode == "sym":
                lib.hawkes_tune_symmetric_groups(size)
            else:
                lib.hawkes_tune_symmetric_groups(0)
                lib.hawkes_tune_target_workgroups(size)
            ms = []
            for _ in range(3):
                ll, g = hk.loglik_grad(dev, th, "fp32", ws=ws)
                torch.cuda.synchronize()
                ms.append(hk.last_pair_kernel_ms())
            llv, gv = float(ll.item()), g.cpu().numpy()
            ref = ref or (llv, gv)
            dl = abs(llv - ref[0]) / abs(ref[0])
            dg = float(np.max(np.abs(gv - ref[1]) / np.abs(ref[1])))
            hk.loglik_grad(dev, th, "fp32_skip", ws=ws)
            torch.cuda.synchronize()
            skip_ms = hk.last_pair_kernel_ms()
            if gold is not None:
                el = abs(llv - gold["loglik"]) / abs(gold["loglik"])
                eg = float(np.max(np.abs(gv - np.array(gold["grad"])) / np.abs(np.array(gold["grad"]))))
                err = f" {el:.1e} | {eg:.1e} |"
            else:
                err = " - | - |"
            print(f"| {name} | {mode} {size} | {min(ms):.1f} | {skip_ms:.1f} | {dl:.1e} | {dg:.1e} |{err}", flush=True)
        del ws
        hk.set_timing(False)
        lib.hawkes_tune_target_workgroups(32768)
        lib.hawkes_tune_symmetric_groups(_lib.SYM_GROUPS_DEFAULT)


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["build", "time"])
    ap.add_argument("shapes", nargs="*")
    ap.add_argument("--n", type=int, default=1_000_000)
    a = ap.parse_args()
    names = a.shapes or list(SHAPES)
    for s in names:
        if s not in SHAPES:
            raise SystemExit(f"unknown shape {s}; known: {', '.join(SHAPES)}")
    if a.what == "build":
        build(names)
    else:
        print("| shape | sweep | FP32 ms (best of 3) | FP32 skip ms | loglik rel diff | grad rel diff "
              "| loglik rel err vs oracle | grad rel err vs oracle |")
        print("|---|---|---|---|---|---|---|---|")
        time_shapes(names, a.n)


if __name__ == "__main__":
    main()
