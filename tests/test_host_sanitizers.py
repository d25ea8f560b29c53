"""The host runtime and the C ABI under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; no GPU needed).

capi.cpp is compiled with the sanitizers on its host pass and linked with the
other objects of the normal build into a separate library, which a child
Python process loads (with the sanitizer runtime preloaded) to drive every
entry point that does its work on the host: parameter checks, the projection
for many shapes, the size queries, and the argument errors of the calls that
would launch work.  Any sanitizer report aborts the child and fails the test."""
import os
import subprocess
import sys
import tempfile

import pytest

from tests.conftest import ROOT

CSRC = os.path.join(ROOT, "paper_2412_03301_amd", "csrc")
OBJ = os.path.join(CSRC, "_obj")

CHILD = r'''
import ctypes as C, sys
L = C.CDLL(sys.argv[1])
class Params(C.Structure):
    _fields_ = [("dim", C.c_uint32), ("code_bits", C.c_uint32), ("fan_in", C.c_uint32), ("wta_k", C.c_uint32),
                ("access_lists", C.c_uint32), ("min_count", C.c_uint32), ("top_t", C.c_uint32),
                ("flags", C.c_uint32), ("seed", C.c_uint64)]
L.bvs_last_error.restype = C.c_char_p
p = Params()
L.bvs_params_default(C.byref(p))
assert L.bvs_params_check(C.byref(p)) == -6
for d, Lb, s, k in [(128, 1024, 8, 32), (384, 4096, 16, 64), (768, 4096, 16, 64), (17, 256, 17, 3),
                    (1024, 2048, 32, 100), (1, 256, 1, 1)]:
    p.dim, p.code_bits, p.fan_in, p.wta_k, p.top_t = d, Lb, s, k, 100
    assert L.bvs_params_check(C.byref(p)) == 0, (d, Lb, s, k, L.bvs_last_error())
    out = (C.c_uint16 * (Lb * s))()
    for seed in (0, 1, 2**64 - 1):
        p.seed = seed
        assert L.bvs_projection(C.byref(p), out) == 0
        assert all(int(out[j * s + i]) < d for j in range(0, Lb, 97) for i in range(s))
    nb = C.c_uint64(0)
    assert L.bvs_index_bytes(C.byref(p), 1000, 50000, C.byref(nb)) == 0 and nb.value > 0
    assert L.bvs_build_workspace_bytes(C.byref(p), 1000, 50000, C.byref(nb)) == 0
for field, bad in [("dim", 0), ("code_bits", 1000), ("fan_in", 0), ("wta_k", 0), ("access_lists", 9),
                   ("min_count", 256), ("top_t", 0), ("flags", 1)]:
    q = Params.from_buffer_copy(p)
    setattr(q, field, bad)
    assert L.bvs_params_check(C.byref(q)) != 0 and L.bvs_last_error()
nb = C.c_uint64(0)
off = (C.c_uint64 * 4)(0, 3, 2, 5)           # not increasing
assert L.bvs_build_index(C.byref(p), C.c_void_p(16), off, 3, None, 0, None, 0, None, C.byref(C.c_void_p())) != 0
assert L.bvs_search(None, None, None, 1, 10, None, 0, None, None, None, None) == -1
assert L.bvs_search_metric(None, 9, None, None, 1, 10, None, 0, None, None, None, None) == -1
assert L.bvs_bruteforce_metric(None, -3, None, None, 1, 10, None, 0, None, None, None, None) == -1
assert L.bvs_search_full(None, None, None, 1, 10, None, 0, None, None, None, None) == -1
assert L.bvs_search_noalloc(None, None, None, 1, 10, None, None, None, None) == -1
assert L.bvs_index_set_search_params(None, 3, 1, 100) == -1
assert L.bvs_index_set_first_layer(None, 1) == -1
assert L.bvs_codes_bytes(None, C.byref(nb)) == -1 and L.bvs_lists_workspace_bytes(None, C.byref(nb)) == -1
assert L.bvs_mlp_weight_count(768, 1024, 4096, C.byref(nb)) == 0 and nb.value == 768 * 1024 + 1024 + 4096 * 1024 + 4096
for k in range(20):
    L.bvs_stage_name(k)
print("sanitized host calls ok")
'''


def _asan_runtime():
    out = subprocess.run(["/opt/rocm/llvm/bin/clang", "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True).stdout.strip()
    return out if out and os.path.exists(out) else None


@pytest.mark.slow
def test_host_runtime_under_asan_and_ubsan():
    rt = _asan_runtime()
    objs = [os.path.join(OBJ, f) for f in sorted(os.listdir(OBJ))] if os.path.isdir(OBJ) else []
    if not rt or not objs:
        pytest.skip("no sanitizer runtime or no objects of a normal build")
    objs = [o for o in objs if not o.endswith("capi.o") and o.endswith(".o")]
    with tempfile.TemporaryDirectory() as tmp:
        san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
        capi = os.path.join(tmp, "capi.o")
        cc = ["/opt/rocm/bin/hipcc", "-xhip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", f"-I{os.path.join(ROOT, 'include')}",
              f"-I{CSRC}", *san, "-c", os.path.join(CSRC, "capi.cpp"), "-o", capi]
        r = subprocess.run(cc, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        lib = os.path.join(tmp, "libbvs_san.so")
        ld = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan", *san, capi, *objs,
              "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib", "-o", lib]
        r = subprocess.run(ld, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([sys.executable, "-c", CHILD, lib], capture_output=True, text=True, env=env, timeout=300)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
        assert "sanitized host calls ok" in r.stdout
