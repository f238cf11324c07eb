"""Host build of the library's kernels and runtime for bounds checking.

The HIP sources are compiled as host C++ against hip/hip_runtime.h of this
folder, an emulation of the device environment they use (workgroups as
threads with real barriers, wave operations through a per-wave exchange), with
AddressSanitizer.  Every device allocation, and every buffer carved out of a
plan's pool, is followed by a poisoned red zone as large as itself, so an
out-of-bounds access of any kernel is reported with its source line.  The
copies of the sources get three mechanical substitutions: dynamic LDS arrays
take the launch's buffer, carved buffers get their red zones, and the header
path.  Host code only: nothing here runs on a GPU."""
from __future__ import annotations

import hashlib
import os
import re
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2606_30620_amd", "csrc")
HEADER = os.path.join(ROOT, "include", "rtu.h")
OUT = os.path.join(HERE, "_build")
CXX = "/opt/rocm/llvm/bin/clang++"
FLAGS = ["-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address", "-pthread", "-w"]


def available() -> bool:
    return os.path.exists(CXX)


def _prepared_sources():
    out = {}
    for f in sorted(os.listdir(CSRC)):
        if not (f.endswith(".hip") or f.endswith(".h")):
            continue
        s = open(os.path.join(CSRC, f)).read()
        s = re.sub(r"extern __shared__ __align__\(16\) ([\w ]+?) (\w+)\[\];", r"\1* \2 = (\1*)emu_dyn_lds();", s)
        if f == "rtu_runtime.hip":
            old = "    off += count * sizeof(T);\n    return p;"
            assert old in s, "the pool carving changed: update the red-zone substitution"
            s = s.replace(old, "    off += count * sizeof(T);\n    off = emu_guard(base, (char*)p, count * sizeof(T), off);\n"
                               "    return p;")
            s = s.replace('#include "rtu_internal.h"',
                          '#include "rtu_internal.h"\nsize_t emu_guard(char* base, char* p, size_t n, size_t off);', 1)
        out[f] = s.replace('#include "../../include/rtu.h"', '#include "rtu.h"')
    out["rtu.h"] = open(HEADER).read()
    return out


def build() -> str:
    """Compile (when any input changed) and return the path of the emulation program."""
    srcs = _prepared_sources()
    own = {f: open(os.path.join(HERE, f)).read() for f in ("emu.cpp", "driver.cpp", os.path.join("hip", "hip_runtime.h"))}
    h = hashlib.sha256()
    for k in sorted(srcs):
        h.update(k.encode() + srcs[k].encode())
    for k in sorted(own):
        h.update(k.encode() + own[k].encode())
    h.update(" ".join(FLAGS).encode())
    tag = h.hexdigest()[:16]
    exe = os.path.join(OUT, f"driver_{tag}")
    if os.path.exists(exe):
        return exe
    if os.path.isdir(OUT):
        shutil.rmtree(OUT)
    src_dir = os.path.join(OUT, "src")
    os.makedirs(src_dir)
    for k, v in srcs.items():
        open(os.path.join(src_dir, k), "w").write(v)
    inc = ["-I" + HERE, "-I" + src_dir]
    units = [(os.path.join(src_dir, f), ["-x", "c++"]) for f in
             ("rtu_kernels.hip", "rtu_runtime.hip", "rtu_fit.hip", "rtu_fleet.hip")]
    units += [(os.path.join(HERE, "emu.cpp"), []), (os.path.join(HERE, "driver.cpp"), [])]

    def compile_one(u):
        src, lang = u
        obj = os.path.join(OUT, os.path.basename(src) + ".o")
        subprocess.run([CXX] + FLAGS + inc + lang + ["-c", src, "-o", obj], check=True)
        return obj

    with ThreadPoolExecutor(max_workers=6) as ex:
        objs = list(ex.map(compile_one, units))
    subprocess.run([CXX, "-fsanitize=address", "-pthread"] + objs + ["-o", exe], check=True)
    return exe
