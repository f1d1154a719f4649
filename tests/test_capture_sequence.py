"""Host-only check of the stream, event, copy and graph calls the library
makes, against a recording stand-in of the HIP runtime
(tests/capture_check/hip_record.cpp).  The library's sources are compiled for
the host only (no device code) with the graph execution of fbt_batch_eval
built in, and linked against the stand-in instead of the runtime; the driver
(tests/capture_check/driver.cpp) runs the graph execution (captures, replays,
re-captures), the worker execution, and the single-context entry points in
every precision.  The stand-in reports every broken rule of stream capture
and every copy outside its allocation; the self-test first shows that it
detects each kind.

This is the check of the graph execution's capture sequence: it finds the
sequence legal (every forked stream joined back into the origin, every waited
event recorded inside the capture, no allocation, creation or host wait
during the capture, only pinned host memory in captured copies, every copy in
bounds, staging buffers outliving the graph), so the host crash of the
graph execution on the GPU is not explained by the order or kinds of these
calls, and the path stays switched off in the product build.
"""
import os
import re
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2601_11437_amd", "csrc")
CHECK = os.path.join(HERE, "capture_check")
SOURCES = ["fbt_kernels.hip", "fbt_engine.hip", "fbt_fit.cpp", "fbt_batch.cpp", "fbt_round.hip",
           "fbt_plan.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ROCM_INC = "/opt/rocm/include"

pytestmark = pytest.mark.skipif(not (os.path.exists(HIPCC) and shutil.which("g++")),
                                reason="hipcc or g++ not available")


def _run(cmd, cwd=None):
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=cwd)
    if r.returncode != 0:
        raise RuntimeError("failed: %s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return r


@pytest.fixture(scope="module")
def built(tmp_path_factory):
    out = tmp_path_factory.mktemp("capture_check")
    procs = []
    objs = []
    for src in SOURCES:
        obj = str(out / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen(
            [HIPCC, "--offload-host-only", "-O1", "-std=c++17", "-fPIC", "-DFBT_GRAPH_EXEC=1",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-c", os.path.join(CSRC, src),
             "-o", obj], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        so, se = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("host-only compile failed:\n%s%s" % (so, se))
    gxx = ["g++", "-O1", "-std=c++17", "-Wno-unused-result", "-D__HIP_PLATFORM_AMD__",
           "-I", ROCM_INC, "-I", os.path.join(ROOT, "include")]
    for name in ("hip_record", "driver", "selftest"):
        _run(gxx + ["-c", os.path.join(CHECK, name + ".cpp"), "-o", str(out / (name + ".o"))])
    # the host objects name their (absent) device images: empty stand-ins
    syms = set()
    for obj in objs:
        syms |= set(re.findall(r"__hip_fatbin\w*", _run(["nm", "-u", obj]).stdout))
    stub = out / "fatbin_stub.c"
    stub.write_text("".join("char %s[1];\n" % s for s in sorted(syms)))
    _run(["gcc", "-c", str(stub), "-o", str(out / "fatbin_stub.o")])
    rec = str(out / "hip_record.o")
    _run(["g++", "-o", str(out / "check"), str(out / "driver.o"), rec] + objs +
         [str(out / "fatbin_stub.o"), "-lpthread"])
    _run(["g++", "-o", str(out / "selftest"), str(out / "selftest.o"), rec, "-lpthread"])
    return out


def test_recorder_detects_each_rule(built):
    r = subprocess.run([str(built / "selftest")], capture_output=True, text=True, timeout=60)
    sys.stdout.write(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr


def test_library_capture_sequence_is_legal(built):
    r = subprocess.run([str(built / "check")], capture_output=True, text=True, timeout=300)
    sys.stdout.write(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    m = re.search(r"batch graph: (\d+) captures, (\d+) graph launches", r.stdout)
    assert m and int(m.group(1)) == 3 and int(m.group(2)) == 5
    # the persistent round's graph: captured for the first modes, replayed,
    # captured again for new modes
    m = re.search(r"persistent round graph: (\d+) captures, (\d+) graph launches", r.stdout)
    assert m and int(m.group(1)) == 2 and int(m.group(2)) == 3
    assert "no violations" in r.stdout
