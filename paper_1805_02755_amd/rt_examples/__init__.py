"""Example payloads supplied at run time: HIP sources for the GPU (compiled
by the engine with hipRTC) and their host versions in C (escape_host.c,
built here with gcc on first use)."""
import ctypes as C
import os
import struct
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
_host = None


def source(name: str) -> str:
    with open(os.path.join(HERE, name)) as f:
        return f.read()


def host_lib():
    """Builds escape_host.c (host versions of the example payloads) once per process."""
    global _host
    if _host is None:
        out = os.path.join(tempfile.mkdtemp(prefix="rt_host_"), "librt_host.so")
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared", "-o", out,
                        os.path.join(HERE, "escape_host.c"), "-lm"], check=True, capture_output=True)
        _host = C.CDLL(out)
    return _host


def host_fn(name: str) -> int:
    """Address of a host version, for Engine.program_source(host=...)."""
    return C.cast(getattr(host_lib(), name), C.c_void_p).value


def escape_scalars(w, x0, y0, dx, dy, max_iter) -> bytes:
    """Scalar block of escape.hiprtc: x0, y0, dx, dy (float32), w, max_iter (uint32)."""
    return struct.pack("<4f2I", x0, y0, dx, dy, w, max_iter)
