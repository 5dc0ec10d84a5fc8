"""Builds the test-only HIP probes of tests/csrc (gfx950, the library's hipcc flags) in-tree:
libexp2_probe.so, the device check of the FP32 exp2 bias that the FP32 sweep corrects for."""

from __future__ import annotations

import os
import subprocess
from pathlib import Path

HERE = Path(__file__).resolve().parent
PROBES = {"libexp2_probe.so": "exp2_probe.hip"}


def build_probes() -> list[Path]:
    from paper_2407_11349_amd.build import HIPCC_FLAGS, hipcc

    out = []
    for lib, src in PROBES.items():
        dst = HERE / lib
        tmp = dst.with_name(dst.name + ".tmp%d" % os.getpid())
        res = subprocess.run([hipcc(), *HIPCC_FLAGS, str(HERE / src), "-o", str(tmp)], capture_output=True,
                             text=True)
        if res.returncode != 0:
            raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
        os.replace(tmp, dst)
        out.append(dst)
    return out


if __name__ == "__main__":
    print(build_probes())
