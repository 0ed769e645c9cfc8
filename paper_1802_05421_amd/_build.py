"""Build step for libcaddelag.so (gfx950 only) - compiles csrc/*.hip with hipcc."""

from __future__ import annotations

import glob
import json
import os
import re
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libcaddelag.so")
# per-kernel register, scratch and LDS use of the last build (compiler remarks)
RESOURCES = os.path.join(PKG, "libcaddelag.resources.json")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # no packed FP32 arithmetic anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


_REMARK = re.compile(r"remark:\s+(Function Name|VGPRs|AGPRs|ScratchSize \[bytes/lane\]|"
                     r"Dynamic Stack|Occupancy \[waves/SIMD\]|SGPRs Spill|VGPRs Spill|"
                     r"LDS Size \[bytes/block\]): (\S+) \[-Rpass-analysis=kernel-resource-usage\]")
_KEYS = {"VGPRs": "vgpr", "AGPRs": "agpr", "ScratchSize [bytes/lane]": "scratch",
         "Dynamic Stack": "dynamic_stack", "Occupancy [waves/SIMD]": "occupancy",
         "SGPRs Spill": "sgpr_spill", "VGPRs Spill": "vgpr_spill", "LDS Size [bytes/block]": "lds"}


def parse_resources(text: str) -> dict:
    """{kernel symbol: {vgpr, agpr, scratch, dynamic_stack, occupancy, ...}}
    from the compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for m in _REMARK.finditer(text):
        key, val = m.group(1), m.group(2)
        if key == "Function Name":
            cur = out.setdefault(val, {})
        elif cur is not None:
            cur[_KEYS[key]] = (val == "True") if key == "Dynamic Stack" else int(val)
    return out


def build(verbose: bool = False) -> str:
    """Compile the library in-tree; always recompiles.  Also writes the
    kernels' resource use (registers, scratch, LDS, occupancy) next to it."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, *FLAGS, "-Rpass-analysis=kernel-resource-usage",
           "-I" + os.path.join(ROOT, "include"), "-o", tmp, *sources()]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    text = proc.stdout + proc.stderr
    msgs = [ln for ln in text.splitlines()
            if "packed-fp32-ops' is not a recognized feature" not in ln
            and "kernel-resource-usage" not in ln and not re.match(r"^\s*(\d+ \|.*|\|\s*\^?)$", ln)]
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    with open(RESOURCES + ".tmp", "w") as f:
        json.dump(parse_resources(text), f, indent=1, sort_keys=True)
    os.replace(RESOURCES + ".tmp", RESOURCES)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
