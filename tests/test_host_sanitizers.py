"""The host code of the library (plan builder, work decomposition, launch
sequences, Hermitian eigensolver) under the address and undefined-behaviour
sanitizers: plan.cpp and eigh.cpp are compiled with g++ (host only, no GPU
code) together with a small driver (tests/native/sanitize_driver.cpp) that
builds the plans of every small problem, of the configs c0-c2 and c4, of a
batch of c3 instances and of invalid descriptors, describes their work
blocks, and solves random Hermitian matrices.  Any sanitizer report fails
the run; the external determinant counts must equal the library's."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import pytest

import synth.problems as SP

from helpers import SMALL, problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2608_11529_amd", "csrc")


def records(M):
    out = []
    names = list(SMALL) + ["c0", "c1", "c2", "c4"]
    for nm in names:
        out.append(([M.desc_of_problem(problem(nm))], nm))
    out.append(([M.desc_of_problem(SP.batched_instance(s)) for s in range(8)], "c3[0:8]"))
    bad = M.desc_of_problem(problem("s_das"))
    bad.n_act_elec = 40                       # more electrons than active spinors
    out.append(([bad], "bad-electrons"))
    wide = M.desc_of_problem(SP.small("wide", 1, 0, 2, [40, 30], 2, 4, [(4, 1.0)]))   # 70 active spinors
    out.append(([wide], "bad-width"))
    return out


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_plan_and_eigh_under_sanitizers():
    import paper_2608_11529_amd as M
    recs = records(M)
    tmp = tempfile.mkdtemp(prefix="mrpt2_san_")
    try:
        exe = os.path.join(tmp, "driver")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
               "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "eigh.cpp"),
               os.path.join(ROOT, "tests", "native", "sanitize_driver.cpp"), "-o", exe]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        blob = os.path.join(tmp, "descs.bin")
        with open(blob, "wb") as f:
            for descs, _ in recs:
                f.write(ctypes.c_int32(len(descs)))
                for d in descs:
                    f.write(bytes(d))
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([exe, blob], capture_output=True, text=True, env=env, timeout=900)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
        lines = [ln.split() for ln in r.stdout.splitlines() if ln.startswith("plan")]
        assert lines and r.stdout.rstrip().endswith("eigh ok")
        assert len(lines) == len(recs)
        for (descs, name), ln in zip(recs, lines):
            status = int(ln[1])
            if name.startswith("bad"):
                assert status != 0, name
                continue
            assert status == 0, name
            plan = M.Plan(descs)
            assert [int(x) for x in ln[2:]] == [plan.info(i).n_ext for i in range(len(descs))], name
    finally:
        shutil.rmtree(tmp, ignore_errors=True)
