"""Build synth/libsynth.so (the device input generator) for gfx950."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libsynth.so")
SRC = os.path.join(HERE, "gmm.hip")


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-x", "hip", "--offload-arch=gfx950", "-O3",
           "-std=c++17", "-fPIC", "-shared", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", SRC, "-o", tmp]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
