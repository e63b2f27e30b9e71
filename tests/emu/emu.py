"""Build and run libsfft in the host emulation (test infrastructure).

The library's own sources -- kernels, ABI and autotuner -- are compiled for the
host with g++ against tests/emu/hip/hip_runtime.h instead of the HIP
runtime, together with emu_runtime.cpp (work-group threads, checked barriers,
the matrix instruction's wavefront exchange) and emu_driver.cpp, under
AddressSanitizer + UndefinedBehaviorSanitizer ("asan") or ThreadSanitizer
("tsan").  The only change to a source on its way in is the declaration of the
dynamic LDS array, which becomes the emulator's per-work-group heap block, and
the FP32 4-vector type, spelled as GCC spells it.
"""
from __future__ import annotations

import os
import re
import shutil
import struct
import subprocess
import tempfile

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_1606_07407_amd", "csrc")
BUILD = os.path.join(ROOT, "_build", "emu")
SOURCES = ["sfft_kernels.hip", "sfft_mlp.hip", "sfft_abi.cpp", "sfft_tune.cpp"]
SANITIZE = {
    "asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
             "-fno-omit-frame-pointer"],
    "tsan": ["-fsanitize=thread"],
}
LDS_DECL = re.compile(r"extern\s+__shared__\s+__align__\(\d+\)\s+char\s+lds\[\];")


def compiler() -> str:
    """g++: its ThreadSanitizer keeps exact happens-before for the 257 threads of a
    work-group run (the LLVM runtime here recycles its thread slots past 255 and then
    misses races)."""
    return os.environ.get("EMU_CXX", "g++")


def _sources_stamp() -> str:
    import hashlib
    h = hashlib.sha256()
    for d, files in ((CSRC, sorted(os.listdir(CSRC))),
                     (HERE, ["emu_runtime.cpp", "emu_driver.cpp", "planted.cpp", "emu.py",
                             "hip/hip_runtime.h"])):
        for f in files:
            path = os.path.join(d, f)
            if os.path.isfile(path):
                h.update(f.encode())
                h.update(open(path, "rb").read())
    h.update(open(os.path.join(ROOT, "include", "sfft.h"), "rb").read())
    return h.hexdigest()[:16]


def build(kind: str) -> str:
    """Compile the driver for one sanitizer; returns the executable's path (cached by a
    hash of every source it is built from)."""
    exe = os.path.join(BUILD, f"emu_driver_{kind}_{_sources_stamp()}")
    if os.path.exists(exe):
        return exe
    os.makedirs(BUILD, exist_ok=True)
    # a private directory per build: parallel test workers may build at the same time
    src_dir = tempfile.mkdtemp(prefix=f"src_{kind}_", dir=BUILD)
    units = []
    for f in sorted(os.listdir(CSRC)):      # headers too: the build includes these copies
        if not f.endswith((".hpp", ".h")):
            continue
        text = open(os.path.join(CSRC, f)).read().replace("ext_vector_type(4)", "vector_size(16)")
        with open(os.path.join(src_dir, f), "w") as fh:
            fh.write(text)
    for f in SOURCES:
        text = open(os.path.join(CSRC, f)).read()
        text, n = LDS_DECL.subn("char* lds = ::emu::dyn_lds();", text)
        text = text.replace("ext_vector_type(4)", "vector_size(16)")  # GCC's spelling
        out = os.path.join(src_dir, f + ".cpp")
        with open(out, "w") as fh:
            fh.write(text)
        units.append(out)
    units += [os.path.join(HERE, "emu_runtime.cpp"), os.path.join(HERE, "emu_driver.cpp")]
    # ThreadSanitizer at -O0: optimised code may load a shared value speculatively on a
    # path that the source does not take (`tid == 0 && st.x == 0` read by every thread),
    # which the sanitizer, instrumenting the optimised code, would report as a race
    opt = "-O0" if kind == "tsan" else "-O1"
    flags = ["-std=c++17", opt, "-g", "-pthread", "-x", "c++", "-I", HERE, "-I", src_dir,
             "-I", os.path.join(ROOT, "include"), "-Wno-attributes",
             "-Wno-unknown-pragmas", *SANITIZE[kind]]
    objs = []
    for u in units:
        o = os.path.join(src_dir, os.path.basename(u) + f".{kind}.o")
        r = subprocess.run([compiler(), *flags, "-c", u, "-o", o], capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(f"emulator build failed on {u}:\n{r.stderr[-4000:]}")
        objs.append(o)
    tmp = os.path.join(src_dir, "emu_driver")
    r = subprocess.run([compiler(), "-pthread", *SANITIZE[kind], "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"emulator link failed:\n{r.stderr[-4000:]}")
    os.replace(tmp, exe)
    shutil.rmtree(src_dir, ignore_errors=True)
    return exe


def build_planted(kind: str) -> str:
    """The deliberate-defect program (planted.cpp) under one sanitizer."""
    exe = os.path.join(BUILD, f"planted_{kind}_{_sources_stamp()}")
    if os.path.exists(exe):
        return exe
    os.makedirs(BUILD, exist_ok=True)
    work = tempfile.mkdtemp(prefix=f"planted_{kind}_", dir=BUILD)
    flags = ["-std=c++17", "-O1", "-g", "-pthread", "-x", "c++", "-I", HERE,
             "-Wno-attributes", "-Wno-unknown-pragmas", *SANITIZE[kind]]
    objs = []
    for u in ("planted.cpp", "emu_runtime.cpp"):
        o = os.path.join(work, f"{u}.{kind}.o")
        r = subprocess.run([compiler(), *flags, "-c", os.path.join(HERE, u), "-o", o],
                           capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(f"build failed on {u}:\n{r.stderr[-3000:]}")
        objs.append(o)
    tmp = os.path.join(work, "planted")
    r = subprocess.run([compiler(), "-pthread", *SANITIZE[kind], "-o", tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"link failed:\n{r.stderr[-3000:]}")
    os.replace(tmp, exe)
    shutil.rmtree(work, ignore_errors=True)
    return exe


def run_planted(kind: str, mode: str, timeout: float = 120.0):
    """(return code, stderr) of one deliberate defect."""
    e = dict(os.environ)
    e.update({"ASAN_OPTIONS": "detect_leaks=0", "TSAN_OPTIONS": "halt_on_error=1",
              "EMU_BARRIER_TIMEOUT_S": "3"})
    r = subprocess.run([build_planted(kind), mode], capture_output=True, text=True,
                       timeout=timeout, env=e)
    return r.returncode, r.stderr


def _params_bytes(params) -> bytes:
    c = params.to_c()
    import ctypes
    return ctypes.string_at(ctypes.addressof(c), ctypes.sizeof(c)), ctypes.sizeof(c)


def run(kind: str, params, pb, max_batch: int | None = None, entry: int = 0,
        timeout: float = 900.0, env=None, dft_x=None) -> dict:
    """Recover planted batch pb with plan parameters params (an sfft.Params) in the
    emulation; returns the outputs as numpy arrays plus the sanitizer's stderr.
    entry = 2 runs sfft_dft on the complex rows of dft_x instead (pb only fills
    the input format) and returns them transformed under "dft"."""
    exe = build(kind)
    raw, size = _params_bytes(params)
    blocks = [] if params.blocks is None else [int(v) for v in params.blocks]
    order = [] if params.order is None else [int(v) for v in params.order]
    B = pb.B
    mb = max_batch or B
    c = np.asarray(pb.coeffs, np.complex128)
    buf = bytearray()
    buf += struct.pack("<qq", 0x73666674656D75, size) + raw
    buf += struct.pack("<i", len(blocks)) + np.asarray(blocks, np.int32).tobytes()
    buf += struct.pack("<i", len(order)) + np.asarray(order, np.int32).tobytes()
    buf += struct.pack("<iii", B, mb, entry)
    buf += np.asarray(pb.mode_off, np.int64).tobytes()
    buf += np.ascontiguousarray(pb.freqs, np.int64).tobytes()
    buf += np.ascontiguousarray(np.stack([c.real, c.imag], -1), np.float64).tobytes()
    buf += np.asarray(pb.k, np.int32).tobytes()
    buf += np.asarray(pb.sigma, np.float64).tobytes()
    buf += struct.pack("<Q", int(pb.seed) & 0xFFFFFFFFFFFFFFFF)
    if entry == 2:
        x = np.asarray(dft_x, np.complex128)
        buf += struct.pack("<ii", x.shape[1], x.shape[0])
        buf += np.ascontiguousarray(np.stack([x.real, x.imag], -1), np.float64).tobytes()
    with tempfile.TemporaryDirectory() as td:
        fin, fout = os.path.join(td, "in.bin"), os.path.join(td, "out.bin")
        open(fin, "wb").write(bytes(buf))
        e = dict(os.environ)
        e.update({"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
                  "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
                  "TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1"})
        if env:
            e.update(env)
        r = subprocess.run([exe, fin, fout], capture_output=True, text=True, timeout=timeout,
                           env=e)
        if r.returncode != 0:
            raise RuntimeError(f"emulated run failed ({r.returncode}):\n{r.stderr[-6000:]}")
        data = open(fout, "rb").read()
    out = {"stderr": r.stderr}
    off = 0

    def take(dtype, n):
        nonlocal off
        a = np.frombuffer(data, dtype=dtype, count=n, offset=off).copy()
        off += a.nbytes
        return a

    out["plan_status"] = int(take(np.int32, 1)[0])
    if out["plan_status"] != 0:
        return out
    out["call_status"] = int(take(np.int32, 1)[0])
    if entry == 2:
        cnt, p = np.asarray(dft_x).shape
        xo = take(np.float64, 2 * cnt * p).reshape(cnt, p, 2)
        out["dft"] = xo[..., 0] + 1j * xo[..., 1]
        return out
    km, d, R = params.k_max, params.d, params.max_rounds
    out["freqs"] = take(np.int64, B * km * d).reshape(B, km, d)
    co = take(np.float64, B * km * 2).reshape(B, km, 2)
    out["coeffs"] = co[..., 0] + 1j * co[..., 1]
    out["k_found"] = take(np.int32, B)
    out["status"] = take(np.int32, B)
    out["rounds"] = take(np.int32, B)
    out["samples"] = take(np.int64, B)
    out["trace"] = take(np.int32, B * R * 8).reshape(B, R, 8)
    return out
