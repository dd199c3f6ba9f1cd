"""LDS read bandwidth of the chip, measured (the ceiling the sweep kernels'
LDS traffic is compared with): a probe kernel streams 16-byte LDS reads in
every workgroup and the launch is timed with HIP events.

usage: python3 lds_bandwidth.py --build    (here, once: hipcc for gfx950)
       python3 lds_bandwidth.py            (on the GPU; from the repository root)
"""
import ctypes
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lds_probe.hip")
LIB = os.path.join(HERE, "_build", "liblds_probe.so")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def build() -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    subprocess.run(["hipcc", *FLAGS, "-o", LIB, SRC], check=True, cwd="/tmp")
    return LIB


def main():
    if "--build" in sys.argv:
        print(build())
        return
    if not os.path.exists(LIB):
        raise SystemExit(f"{LIB} is not built; run python3 lds_bandwidth.py --build first")
    lib = ctypes.CDLL(LIB)
    lib.lds_probe_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.lds_probe_run.restype = ctypes.c_int
    threads, iters, reps = 256, 4096, 20
    for blocks in (256 * 8, 256 * 32):
        ms = ctypes.c_double()
        rc = lib.lds_probe_run(blocks, iters, reps, ctypes.byref(ms))
        if rc != 0:
            raise SystemExit(f"probe failed: HIP error {rc}")
        nbytes = blocks * threads * iters * 16
        print(f"workgroups {blocks}: {nbytes / (ms.value * 1e-3) / 1e12:.2f} TB/s of LDS reads "
              f"({ms.value:.3f} ms per launch, {nbytes / 2**30:.1f} GiB)", flush=True)


if __name__ == "__main__":
    main()
