"""Build step of the HIP library: compiles csrc/*.hip and csrc/*.cpp for gfx950
into an in-tree shared library ``libchem.so`` (explicit hipcc, no JIT cache)."""
from __future__ import annotations

import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libchem.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
ARCH = "gfx950"

HIPCC_FLAGS = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
               # no packed FP32 instructions anywhere in the device code
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-I", INCLUDE, "-Wall"]


# The one-thread-per-cell integrators keep a whole cell's state per lane.
# Machine-level loop-invariant code motion hoists every FP64 constant of the
# mechanism (and every per-element slot address) out of the cell loop into
# registers, which then spill to scratch (about 1 KB per lane); without it
# the kernels need no scratch at all.
NO_MACHINE_LICM = ["-mllvm", "-disable-machine-licm"]


def per_file_flags(src: str) -> list:
    name = os.path.basename(src)
    if name.startswith("gen_") or name == "chem_kernels.hip":
        return NO_MACHINE_LICM
    return []


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def specialised_mechanisms(outdir: str) -> dict:
    """Mechanisms that get compiled-in specialised kernels: the standard
    9-species synthetic mechanism and the 9-species stand-in with real
    mechanism features (one thread per cell holds its state), plus any .mech
    files listed in CHEM_EXTRA_MECHS (colon-separated paths)."""
    sys.path.insert(0, os.path.dirname(HERE))
    from chemgen.mechanism import standard_mechanism
    os.makedirs(outdir, exist_ok=True)
    paths = {}
    for name in ("M9", "H2R"):
        p = os.path.join(outdir, f"{name}.mech")
        standard_mechanism(name).write(p)
        paths[name] = p
    for i, extra in enumerate(filter(None, os.environ.get("CHEM_EXTRA_MECHS", "").split(":"))):
        paths[f"X{i}"] = extra
    return paths


def build(verbose: bool = False) -> str:
    """Generate the specialised sources, compile everything, link libchem.so
    (always rebuilds)."""
    from . import codegen
    objdir = os.path.join(HERE, "_build")
    gendir = os.path.join(objdir, "gen")
    os.makedirs(objdir, exist_ok=True)
    gen_sources = codegen.write_generated(specialised_mechanisms(gendir), gendir)
    jobs = []
    for src in sources() + gen_sources:
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        cmd = ["hipcc", *HIPCC_FLAGS, *per_file_flags(src), "-I", CSRC, "-x", "hip", "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((src, obj, cmd))
    # one compiler process per source file, at most one per host core
    width = max(1, min(len(jobs), os.cpu_count() or 1, 16))
    with concurrent.futures.ThreadPoolExecutor(width) as pool:
        runs = list(pool.map(lambda j: subprocess.run(j[2], stderr=subprocess.PIPE, text=True), jobs))
    for (src, _, _), r in zip(jobs, runs):
        if r.returncode != 0:
            sys.stderr.write(r.stderr)
            raise RuntimeError(f"hipcc failed on {src}")
    objs = [obj for _, obj, _ in jobs]
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    from paper_2312_13513_amd import _build as b
    print(b.build(verbose="-v" in sys.argv))
