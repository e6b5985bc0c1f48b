"""The library's device-independent host logic built with the compiler's
sanitizers and exercised on the CPU: the branch-and-bound core
(csrc/bnb_core.hpp, with the oracle as node solver) under AddressSanitizer and
UndefinedBehaviorSanitizer, and the server's admission logic
(csrc/serve_core.hpp, driven by worker and producer threads) under
ThreadSanitizer and under AddressSanitizer + UndefinedBehaviorSanitizer.  A
sanitizer report makes the program exit non-zero."""
import json
import os
import subprocess

import numpy as np
import pytest

from paper_2602_04551_amd import datagen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
# verify_asan_link_order=0: the environment may preload a library ahead of the
# sanitizer runtime, which the runtime otherwise refuses
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
           UBSAN_OPTIONS="halt_on_error=1", TSAN_OPTIONS="halt_on_error=1")


def build(src, out, flags, libs=()):
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", *flags, os.path.join(HOST, src), "-o", out,
                           "-lpthread", *libs])
    return out


@pytest.fixture(scope="module")
def bnb_asan(orc, tmp_path_factory):
    odir = os.path.join(ROOT, "oracle")
    return build("bnb_core_check.cpp", str(tmp_path_factory.mktemp("san") / "bnb_core_asan"), ASAN,
                 [f"-L{odir}", "-loracle", f"-Wl,-rpath,{odir}"])


@pytest.mark.parametrize("K,policy", [(1, 1), (8, 0)])
def test_bnb_core_under_address_and_ub_sanitizers(orc, bnb_asan, tmp_path, K, policy):
    inst = datagen.make_instance(35, 11, rho=0.5, k=3, snr=2.0, seed=1, lambda0=0.02, lambda2=0.01)
    fn = str(tmp_path / "inst.bin")
    with open(fn, "wb") as f:
        np.array([inst.n, inst.p], np.int64).tofile(f)
        np.array([inst.lambda0, inst.lambda2, inst.M], np.float64).tofile(f)
        np.asfortranarray(inst.X).T.ravel().tofile(f)
        inst.y.astype(np.float64).tofile(f)
    r = subprocess.run([bnb_asan, fn, str(K), str(policy), "1e-7", "20000"], capture_output=True, text=True,
                       timeout=600, env=ENV)
    assert r.returncode == 0, r.stderr[-3000:]
    res = json.loads(r.stdout.splitlines()[-1])
    ref = orc.Oracle.from_instance(inst).bnb(tol_node=1e-7, max_iter=5000, max_iter_root=20000)
    assert res["certified"] == pytest.approx(ref["certified"], rel=1e-12)
    assert res["slots_in_use"] == 0


@pytest.mark.parametrize("flags", [["-fsanitize=thread"], ASAN], ids=["tsan", "asan_ubsan"])
def test_admission_logic_under_sanitizers(tmp_path, flags):
    exe = build("serve_core_check.cpp", str(tmp_path / "serve_core_check"), flags)
    r = subprocess.run([exe, "300", "4"], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    res = json.loads(r.stdout.splitlines()[-1])
    assert res["violations"] == 0 and res["ran"] + res["cancelled"] == 300 and res["max_running"] <= 4
