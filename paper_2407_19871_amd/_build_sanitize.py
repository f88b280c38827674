"""Address- and undefined-behaviour-sanitizer build of liblocpir's host code
(the device code is compiled as usual) into a directory of the caller's
choosing, for the CPU tests: load it with LOCPIR_LIB=<dir>/liblocpir.so,
LOCPIR_NO_TORCH=1 and the sanitizer runtime preloaded
(oracle.build.sanitizer_runtime())."""
import concurrent.futures
import os
import subprocess

from ._build import ARCH, CSRC, HIP_FLAGS, SOURCES

# sanitizers for the host compilation only
SAN_HOST = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined".split()


def build(outdir: str, verbose: bool = False) -> str:
    os.makedirs(outdir, exist_ok=True)
    flags = [f for f in HIP_FLAGS if f not in ("-O3",)] + ["-O1", "-g", "-fno-omit-frame-pointer", *SAN_HOST]

    def one(src):
        obj = os.path.join(outdir, src + ".o")
        cmd = ["hipcc", *flags, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True, capture_output=not verbose)
        return obj

    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(one, SOURCES))
    out = os.path.join(outdir, "liblocpir.so")
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *SAN_HOST, "-shared-libasan", "-o", out, *objs,
           "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, capture_output=not verbose)
    return out
