"""Builds the sanitizer drivers of tests/csrc (CPU only):

* sanitize_oracle: the FP64 oracle (oracle/hawkes_oracle.c) with AddressSanitizer and
  UndefinedBehaviorSanitizer (gcc), driven by sanitize_oracle.c;
* sanitize_abi: the HIP library with the sanitizers on its host code only (each -fsanitize=
  follows -Xarch_host; device code is built as usual), driven by sanitize_abi.cpp through the
  host-side validation of every C-ABI entry point.
"""

from __future__ import annotations

import os
import subprocess
from pathlib import Path

HERE = Path(__file__).resolve().parent
ROOT = HERE.parent.parent
SAN = ["address", "undefined"]


def _run(cmd):
    res = subprocess.run([str(c) for c in cmd], capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(map(str, cmd)) + "\n" + res.stdout + res.stderr)


def build_sanitized() -> list[Path]:
    from paper_2407_11349_amd.build import SOURCES, hipcc

    ora = HERE / "sanitize_oracle"
    _run(["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
          *[f"-fsanitize={s}" for s in SAN], HERE / "sanitize_oracle.c", ROOT / "oracle" / "hawkes_oracle.c",
          "-lm", "-o", ora])
    abi = HERE / "sanitize_abi"
    host_san = []
    for s in SAN:
        host_san += ["-Xarch_host", f"-fsanitize={s}"]
    csrc = ROOT / "paper_2407_11349_amd" / "csrc"
    _run([hipcc(), "-O1", "-g", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", *host_san, "-Xarch_host", "-fno-sanitize-recover=all", "-I", ROOT / "include",
          "-I", csrc, HERE / "sanitize_abi.cpp", *[csrc / s for s in SOURCES], "-o", abi])
    return [ora, abi]


if __name__ == "__main__":
    print(build_sanitized())
