"""Build the HIP library libdr.so for gfx950 (hipcc), in-tree.

Objects go to _build/ at the repository root; the shared library lands next to
this file so that it travels with the source tree.
"""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build")
LIB_PATH = os.path.join(PKG, "libdr.so")
PROBE_PATH = os.path.join(PKG, "libdr_probe.so")  # benchmark's streaming reference
ARCH = os.environ.get("PYTORCH_ROCM_ARCH", "gfx950").split(";")[0] or "gfx950"

# -ffp-contract=off: FP64 geometry must not be contracted into FMAs (bin
# indices are exact results of a fixed operation order).  Packed FP32 ops are
# disabled for all device code.
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", f"-I{INCLUDE}", f"-I{CSRC}"]
DEVICE = ["-x", "hip", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops"]
SOURCES = [("dr_tiles_rows.hip", True), ("dr_tiles_rows_add.hip", True),
           ("dr_tiles_batch.hip", True), ("dr_tiles_batch_add.hip", True),
           ("dr_kernels.hip", True), ("dr_pixels.hip", True), ("dr_select.hip", True),
           ("dr_noalloc.hip", True),
           ("dr_runtime.cpp", False),
           ("dr_list.cpp", False), ("dr_serve.cpp", False), ("dr_sched.cpp", False)]


def _compile(src: str, device: bool) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = ["hipcc", *COMMON, *(DEVICE if device else []), "-c", os.path.join(CSRC, src), "-o", obj]
    subprocess.run(cmd, check=True, stderr=subprocess.PIPE, stdout=subprocess.PIPE)
    return obj


# HDF5 file layer (libdr_h5.so): built when an HDF5 installation is found
HDF5_ROOT = os.environ.get("DR_HDF5_ROOT", "/opt/conda")
H5_LIB_PATH = os.path.join(PKG, "libdr_h5.so")


def hdf5_available() -> bool:
    return os.path.exists(os.path.join(HDF5_ROOT, "include", "hdf5.h")) and \
        os.path.exists(os.path.join(HDF5_ROOT, "lib", "libhdf5.so"))


def build_h5(verbose: bool = False) -> str:
    """g++ build of the HDF5 layer against HDF5_ROOT (rpath to its lib/)."""
    if not hdf5_available():
        if verbose:
            print("HDF5 not found under", HDF5_ROOT, "- libdr_h5.so not built")
        return ""
    lib = os.path.join(HDF5_ROOT, "lib")
    tmp = H5_LIB_PATH + ".tmp"
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-Wall", f"-I{INCLUDE}",
           f"-I{os.path.join(HDF5_ROOT, 'include')}", os.path.join(CSRC, "dr_h5.cpp"), "-o", tmp,
           f"-L{lib}", "-lhdf5", f"-Wl,-rpath,{lib}", "-lpthread"]
    r = subprocess.run(cmd, stderr=subprocess.PIPE, stdout=subprocess.PIPE)
    if r.returncode != 0:
        raise RuntimeError("g++ failed for dr_h5.cpp:\n" + r.stderr.decode(errors="replace"))
    os.replace(tmp, H5_LIB_PATH)
    if verbose:
        print("built", H5_LIB_PATH)
    return H5_LIB_PATH


def build_probe(verbose: bool = False) -> str:
    """hipcc build of libdr_probe.so, the benchmark's streaming reference kernel."""
    tmp = PROBE_PATH + ".tmp"
    cmd = ["hipcc", *COMMON, *DEVICE, "-shared", os.path.join(CSRC, "dr_probe.hip"), "-o", tmp]
    r = subprocess.run(cmd, stderr=subprocess.PIPE, stdout=subprocess.PIPE)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for dr_probe.hip:\n" + r.stderr.decode(errors="replace"))
    os.replace(tmp, PROBE_PATH)
    if verbose:
        print("built", PROBE_PATH)
    return PROBE_PATH


C_CONSUMER_SRC = os.path.join(ROOT, "tests", "c", "abi_consumer.c")
C_CONSUMER = os.path.join(ROOT, "tests", "c", "abi_consumer")


def build_c_consumer(verbose: bool = False) -> str:
    """gcc build of the plain-C test caller of the ABI (links libdr.so by rpath)."""
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", f"-I{INCLUDE}", f"-I{os.path.join(rocm, 'include')}",
           "-D__HIP_PLATFORM_AMD__", C_CONSUMER_SRC, "-o", C_CONSUMER + ".tmp", f"-L{PKG}", "-ldr",
           "-Wl,-rpath,$ORIGIN/../../paper_2201_13309_amd", f"-L{os.path.join(rocm, 'lib')}",
           "-lamdhip64", f"-Wl,-rpath,{os.path.join(rocm, 'lib')}", "-lm"]
    r = subprocess.run(cmd, stderr=subprocess.PIPE, stdout=subprocess.PIPE)
    if r.returncode != 0:
        raise RuntimeError("gcc failed for abi_consumer.c:\n" + r.stderr.decode(errors="replace"))
    os.replace(C_CONSUMER + ".tmp", C_CONSUMER)
    if verbose:
        print("built", C_CONSUMER)
    return C_CONSUMER


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with ThreadPoolExecutor(len(SOURCES) + 1) as ex:
        probe = ex.submit(build_probe, verbose)
        futs = [ex.submit(_compile, s, d) for s, d in SOURCES]
        objs = []
        for f in futs:
            try:
                objs.append(f.result())
            except subprocess.CalledProcessError as e:
                raise RuntimeError("hipcc failed:\n" + e.stderr.decode(errors="replace")) from e
    tmp = LIB_PATH + ".tmp"
    link = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread"]
    r = subprocess.run(link, stderr=subprocess.PIPE, stdout=subprocess.PIPE)
    if r.returncode != 0:
        raise RuntimeError("hipcc link failed:\n" + r.stderr.decode(errors="replace"))
    os.replace(tmp, LIB_PATH)
    if verbose:
        print("built", LIB_PATH)
    probe.result()
    build_h5(verbose)
    build_c_consumer(verbose)
    return LIB_PATH


if __name__ == "__main__":
    build(verbose=True)
