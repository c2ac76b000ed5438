"""The library's host runtime on the CPU, under AddressSanitizer and UndefinedBehaviorSanitizer
(and, for the scenarios whose emulated kernel runs in worker threads, ThreadSanitizer).

`paper_2104_10073_amd/csrc/zmc_host.hip` is compiled as ordinary C++ against a
CPU emulation of the HIP runtime (`tests/hipemu/`: "device" memory in host
memory, in-order synchronous streams, every kernel replaced by a host routine
with the kernel's effect on the buffers the host reads back) and driven
through its C ABI by `tests/hipemu/emu_scenarios.cpp`: admission and queueing,
launches of a few tiles under every scheduling policy, graphs, promotion,
parameter grids, abort, error paths, the plain paths, two contexts, the tuning
cache, the resident engine (its kernel emulated by worker threads that follow
the kernel's protocol: relaunch after idling, record-arena recycling, abort,
destroy while running), checkpoint and resume between launch and resident
contexts (damaged snapshots, queued restored requests), cancellation of single
requests, seeded scripts that interleave submissions, snapshots, restores and
cancels in a launch and a resident context (also with one HIP call failing
in each run), logging, the packing's hypot and atan2, and a sweep that fails every checked HIP call of a workload
in turn (MC_FAULT_HIP) and requires each request to come back either with
exactly its results or with an error -- never MC_OK with wrong values, never a
hang, no leak.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "hipemu")
SCENARIOS = ["basic", "many_launches", "admission", "grid", "abort", "errors", "plain", "two_contexts",
             "fault_sweep", "autotune_cache", "resident_basic", "resident_relaunch", "resident_flush",
             "resident_abort", "log_levels", "snapshot", "pack_math", "cancel", "interleave",
             "interleave_faults"]


# scenarios whose emulated kernel runs in worker threads beside the host runtime
THREADED = ["resident_basic", "resident_relaunch", "resident_flush", "resident_abort", "snapshot", "cancel",
            "interleave", "interleave_faults"]


def _build(tmp_path_factory, name, sanitize):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ is not available")
    exe = str(tmp_path_factory.mktemp("hipemu") / name)
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer"] + sanitize + ["-Wall",
           "-I" + os.path.join(EMU, "include"), "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_2104_10073_amd", "csrc"), "-I" + EMU,
           "-x", "c++", os.path.join(ROOT, "paper_2104_10073_amd", "csrc", "zmc_host.hip"),
           "-x", "none", os.path.join(EMU, "hipemu.cpp"), os.path.join(EMU, "emu_scenarios.cpp"),
           "-o", exe, "-lpthread"]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    assert proc.returncode == 0, proc.stderr[-4000:]
    return exe


@pytest.fixture(scope="module")
def emu_binary(tmp_path_factory):
    return _build(tmp_path_factory, "emu_scenarios", ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])


@pytest.fixture(scope="module")
def emu_tsan_binary(tmp_path_factory):
    return _build(tmp_path_factory, "emu_scenarios_tsan", ["-fsanitize=thread"])


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_host_runtime_scenario(emu_binary, scenario):
    env = dict(os.environ)
    env.pop("MC_FAULT_HIP", None)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    proc = subprocess.run([emu_binary, scenario], capture_output=True, text=True, env=env, timeout=600)
    assert proc.returncode == 0, (proc.stdout[-2000:], proc.stderr[-6000:])
    assert f"ok {scenario}" in proc.stdout
    if scenario == "fault_sweep":
        print(proc.stdout)


@pytest.mark.parametrize("scenario", THREADED)
def test_host_runtime_threads(emu_tsan_binary, scenario):
    """The threaded scenarios under ThreadSanitizer: no data race between the
    host runtime and the emulated resident kernel's workgroups (ring entries,
    acknowledgements, control and exit words, done words and result slots)."""
    env = dict(os.environ)
    env.pop("MC_FAULT_HIP", None)
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    proc = subprocess.run([emu_tsan_binary, scenario], capture_output=True, text=True, env=env, timeout=600)
    assert proc.returncode == 0, (proc.stdout[-2000:], proc.stderr[-6000:])
    assert f"ok {scenario}" in proc.stdout
    assert "ThreadSanitizer" not in proc.stderr
