"""Build the HIP library libirs.so for gfx950 (in-tree).

Every translation unit under csrc/ is compiled by hipcc into _build/ and
linked into paper_2204_10871_amd/libirs.so.  Packed FP32 instructions are
disabled (-packed-fp32-ops) and fma contraction is limited to single
expressions (-ffp-contract=on).
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libirs.so")
ARCH = os.environ.get("IRS_OFFLOAD_ARCH", "gfx950")


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          # contract a*b+c into an fma only within one source expression (decided
          # in the front end), so every kernel instantiation rounds alike
          "-ffp-contract=on",
          f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          # every atomic here is issued by one lane or to lane-varying
          # addresses; the compiler's wave-level combining of atomics only
          # adds instructions around them
          "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
          "-I", os.path.join(HERE, "..", "include")]


def sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _compile(src):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [_hipcc()] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    return obj, warn


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(_compile, srcs))
    objs = [o for o, _ in results]
    if verbose:
        for (o, w) in results:
            if w:
                print(w, file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


# AddressSanitizer and UndefinedBehaviorSanitizer for the host pass only (the
# sanitizers are not for device code here), every report fatal
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def build_host_sanitized(out_dir: str) -> str:
    """A copy of the library, out_dir/libirs_san.so, whose host sources (the
    geometry, the C ABI's argument checks and plan management, the batch
    front end) are compiled with SAN_HOST; the HIP sources' objects are the
    regular ones from build().  A process that loads it must preload
    asan_runtime().  Returns the library's path."""
    if not all(os.path.exists(os.path.join(BUILD, s + ".o")) for s in sources()):
        build()
    os.makedirs(out_dir, exist_ok=True)
    objs = []
    for s in sources():
        if s.endswith(".cpp"):
            obj = os.path.join(out_dir, s + ".san.o")
            cmd = [_hipcc()] + [f for f in COMMON if f != "-O3"] + ["-O1", "-g"] + SAN_HOST + \
                  ["-c", os.path.join(CSRC, s), "-o", obj]
            r = subprocess.run(cmd, capture_output=True, text=True)
            if r.returncode != 0:
                raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
            objs.append(obj)
        else:
            objs.append(os.path.join(BUILD, s + ".o"))
    lib = os.path.join(out_dir, "libirs_san.so")
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", lib] + SAN_HOST + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return lib


def asan_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (it carries the
    UndefinedBehaviorSanitizer handlers too)."""
    r = subprocess.run([_hipcc(), "-print-resource-dir"], capture_output=True, text=True,
                       check=True)
    base = r.stdout.strip().splitlines()[-1]
    for rel in ("lib/linux/libclang_rt.asan-x86_64.so",
                "lib/x86_64-unknown-linux-gnu/libclang_rt.asan.so"):
        path = os.path.join(base, rel)
        if os.path.exists(path):
            return path
    raise RuntimeError(f"no AddressSanitizer runtime under {base}")


if __name__ == "__main__":
    print(build(verbose=True))
