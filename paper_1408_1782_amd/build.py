"""Build the HIP library libqb.so for gfx950 in-tree (hipcc, no JIT)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqb.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("QB_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed FP32 instructions (v_pk_*_f32): every FP32 op is issued unpacked
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{os.path.join(ROOT, 'include')}",
]


BUILD = os.path.join(HERE, "_build")


def _units():
    """qb_lib.hip (host code, ABI, small kernels) and the qb_tiles_*.hip
    units (the FFT kernels of every tile shape), compiled separately."""
    names = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    return [os.path.join(CSRC, f) for f in names]


def build(verbose=False, extra=None, jobs=None):
    """Compile every unit to an object in parallel, then link libqb.so;
    returns its path.  Raises CalledProcessError on failure."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(BUILD, exist_ok=True)
    units = _units()
    objs = [os.path.join(BUILD, os.path.basename(u)[:-4] + ".o") for u in units]
    compile_flags = [f for f in FLAGS if f != "-shared"]
    cmds = [[HIPCC] + compile_flags + (extra or []) + ["-c", u, "-o", o] for u, o in zip(units, objs)]
    if verbose:
        for c in cmds:
            print(" ".join(c), flush=True)
    jobs = jobs or min(len(cmds), max(1, os.cpu_count() or 1), 16)

    def run(c):
        return subprocess.run(c, capture_output=True, text=True)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(run, cmds))
    for c, r in zip(cmds, results):
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise subprocess.CalledProcessError(r.returncode, c)
    tmp = LIB + ".tmp"
    link = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
    print(LIB)
