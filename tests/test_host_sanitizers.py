"""The host code of the library under AddressSanitizer and UndefinedBehaviorSanitizer,
and under ThreadSanitizer with several contexts planning at once.

The planner, the distribution planner, the batcher's validation and the C ABI's
error paths are rebuilt with host-side instrumentation (the device code is
the ordinary build's objects) and linked into ``sanitize_driver.cpp``, which
plans a set of networks on a host-only context (every execution order and
chunk size, every step query, distribution over 2, 4 and 8 devices) and feeds
the ABI malformed inputs.  Any out-of-bounds access, use after free, leak or
undefined operation ends the driver with a report.  The ThreadSanitizer build
runs the same planning in four threads, each on a context of its own
(independent contexts share no mutable state).  Both builds end with a
serving run on a host-only context: four threads submit requests and batcher
rows, poll and wait while the server's six worker threads admit and complete
them (unexecuted, as a host-only server does), a batcher is destroyed with
rows queued, and every call that would change a plan under the workers is
refused.  No GPU is used.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2606_01852_amd import build as pkg_build
from workloads import configs
from workloads.circuits import circuit_network_batched
from workloads.grids import random_grid_network
from workloads.paths import greedy_path, greedy_slice, random_greedy_path

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_SOURCES = ["api", "planner", "executor", "serve", "autotune", "distplan"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
TSAN = ["-Xarch_host", "-fsanitize=thread"]

pytestmark = pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not installed")


def _kernel_objects():
    """The device-code objects of the ordinary build, recompiled when a
    source or a shared header is newer than its object."""
    srcs = [s for s in pkg_build.sources() if s.endswith(".hip")]
    headers = [os.path.join(pkg_build.CSRC, f) for f in os.listdir(pkg_build.CSRC) if f.endswith(".hpp")]
    newest_header = max(os.path.getmtime(h) for h in headers)
    os.makedirs(pkg_build.BUILD, exist_ok=True)
    stale = []
    for s in srcs:
        obj = os.path.join(pkg_build.BUILD, os.path.basename(s) + ".o")
        if not os.path.exists(obj) or os.path.getmtime(obj) < max(os.path.getmtime(s), newest_header):
            stale.append(s)
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(pkg_build._compile, stale))
    return [os.path.join(pkg_build.BUILD, os.path.basename(s) + ".o") for s in srcs]


def _hipcc(args):
    r = subprocess.run(["hipcc"] + args, capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        raise RuntimeError("hipcc " + " ".join(args) + "\n" + r.stderr)


def _build_driver(out, san):
    common = ["-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={pkg_build.ARCH}",
              "-I", os.path.join(ROOT, "include")] + pkg_build.DEVICE_FLAGS + san
    jobs = [(os.path.join(pkg_build.CSRC, f + ".cpp"), str(out / (f + ".o"))) for f in HOST_SOURCES]
    jobs.append((os.path.join(ROOT, "tests", "sanitize_driver.cpp"), str(out / "driver.o")))
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        list(ex.map(lambda j: _hipcc(common + ["-c", j[0], "-o", j[1]]), jobs))
    exe = str(out / "sanitize_driver")
    _hipcc([f"--offload-arch={pkg_build.ARCH}"] + san + [j[1] for j in jobs] + _kernel_objects() + ["-o", exe])
    return exe


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    return _build_driver(tmp_path_factory.mktemp("san"), SAN)


def _write_net(path, net, pairs, sliced=(), batch_label=-1, batch_leaves=()):
    words = [len(net.labels)]
    for lab in net.labels:
        words += [len(lab), *lab]
    words += [len(net.extents), *[int(e) for e in net.extents]]
    words += [len(net.open), *net.open]
    pairs = np.asarray(pairs, dtype=np.int64).reshape(-1, 2)
    words += [len(pairs), *pairs.ravel().tolist()]
    words += [len(sliced), *sliced]
    words += [batch_label, len(batch_leaves), *batch_leaves]
    path.write_text(" ".join(str(int(w)) for w in words) + "\n")
    return str(path)


def _networks(out):
    files = []
    net, p = configs.circuit12()
    files.append(_write_net(out / "circuit12.txt", net, p.pairs))
    net, p = configs.circuit12(open_qubits=(0, 5, 11))
    files.append(_write_net(out / "circuit12_open.txt", net, p.pairs))
    net, p = configs.grid8()
    files.append(_write_net(out / "grid8.txt", net, p.pairs))
    net, p = configs.circuit40()
    files.append(_write_net(out / "circuit40.txt", net, p.pairs, p.sliced))
    net, p = configs.pair30()
    files.append(_write_net(out / "pair30.txt", net, p.pairs))
    net, p = configs.pair_batch(batch=8, scale=4)
    files.append(_write_net(out / "pair_batch.txt", net, p.pairs))
    for seed in range(4):
        net = random_grid_network(3 + seed % 2, 4, 2 + seed % 3, seed=300 + seed)
        p = random_greedy_path(net, seed=seed)
        sl = greedy_slice(net, p.pairs, n_sliced=seed)
        files.append(_write_net(out / f"grid_random{seed}.txt", net, p.pairs, sl))
    circ = configs.circuit12_circuit()
    bits = np.zeros((16, circ.n_qubits), dtype=np.int64)
    net = circuit_network_batched(circ, bits)
    beta = net.open[0]
    carriers = [t for t, lab in enumerate(net.labels) if beta in lab]
    files.append(_write_net(out / "circuit12_batched.txt", net, greedy_path(net).pairs, (), beta, carriers))
    return files


def test_host_code_is_clean_under_asan_and_ubsan(driver, tmp_path):
    files = _networks(tmp_path)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "halt_on_error=1:abort_on_error=0:detect_leaks=1:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([driver] + files, capture_output=True, text=True, timeout=600, env=env)
    report = r.stdout[-4000:] + r.stderr[-8000:]
    assert r.returncode == 0, report
    assert "runtime error" not in r.stderr, report
    assert r.stdout.count("ok ") == len(files) + 2, report


def test_concurrent_contexts_are_race_free_under_tsan(tmp_path_factory, tmp_path):
    exe = _build_driver(tmp_path_factory.mktemp("tsan"), TSAN)
    files = _networks(tmp_path)
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1:exitcode=23"
    r = subprocess.run([exe, "--threads", "4"] + files, capture_output=True, text=True, timeout=600, env=env)
    report = r.stdout[-2000:] + r.stderr[-8000:]
    assert r.returncode == 0, report
    assert "ThreadSanitizer" not in r.stderr, report
    assert r.stdout.count("ok ") == 4 * len(files) + 1, report
