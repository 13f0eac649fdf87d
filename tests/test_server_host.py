"""The continuous-batching server's host code (scheduler, staging, arena) on a
stand-in runtime on the CPU, built with AddressSanitizer and
UndefinedBehaviorSanitizer (tests/host_sched): serving traces are replayed
saturated, paced, under a tight memory budget, with cancellations and in the
one-job-per-launch mode, and every access the stand-in kernels model (from
each kernel's own indexing) must fall inside memory that is live and was
allocated before the launch was enqueued.  One planted lifetime mistake in a
copy of the scheduler shows that the replay detects such errors."""
import concurrent.futures as cf
import os
import subprocess

import pytest

from paper_2511_22094_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2511_22094_amd", "csrc")
HS = os.path.join(ROOT, "tests", "host_sched")
CXX = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address,undefined"]
FLAGS = ["-x", "hip", "--offload-host-only", "-std=c++17", "-O1", "-g", "-fPIC",
         "-fno-omit-frame-pointer", "-DGC_HOST_HARNESS", "-D__HIP_PLATFORM_AMD__",
         "-I", os.path.join(ROOT, "include"), "-Wno-unused-command-line-argument", *SAN]
SOURCES = [os.path.join(CSRC, f) for f in
           ("gc_server.cpp", "gc_capi.cpp", "gc_timing.cpp", "gc_variants.cpp")] + \
          [os.path.join(HS, f) for f in ("fake_hip.cpp", "stub_kernels.cpp", "replay.cpp")]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")

pytestmark = pytest.mark.skipif(not os.path.exists(CXX), reason="ROCm clang++ not available")


def _compile(src, out):
    r = subprocess.run([CXX, *FLAGS, "-c", src, "-o", out], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


def _link(objs, exe):
    r = subprocess.run([CXX, *SAN, "-o", exe, *objs, "-lpthread"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    return exe


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("host_sched")
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(lambda s: _compile(s, str(d / (os.path.basename(s) + ".o"))), SOURCES))
    exe = _link(objs, str(d / "replay"))
    for name, nj, vr, mi in (("trace64", 64, (1e3, 1e5), (1000, 4000)),
                             ("trace256", 256, (1e3, 1e6), (1000, 10000)),
                             ("trace256small", 256, (1e2, 1e4), (1000, 10000))):
        with open(d / f"{name}.txt", "w") as f:
            for j in synth.serving_trace(3, nj, 20.0, vr, mi, (200, 500)):
                f.write(f"{j.arrival_s:.6f} {j.model} {j.kind} {j.n_vox} {j.seed} "
                        f"{j.n_chains} {j.n_iter} {j.burnin} {j.thin} {int(j.tv)}\n")
    return d, exe, objs


def _replay(exe, trace, *opts, delay=100, timeout=600, extra_env=None):
    env = dict(ENV, HH_DELAY_US=str(delay), **(extra_env or {}))
    r = subprocess.run([exe, str(trace), *opts], capture_output=True, text=True, env=env,
                       timeout=timeout)
    return r.returncode, r.stdout + r.stderr


CASES = [
    ("saturated", "trace64", ("--saturated",), 100, None),
    ("saturated_slow_gpu", "trace64", ("--saturated", "--chunk", "64"), 1000, None),
    ("saturated_cancels", "trace64", ("--saturated", "--cancel", "3", "--cancel-delay", "300",
                                      "60"), 300, None),
    ("tight_budget", "trace64", ("--saturated", "--budget", str(200 << 20)), 300, None),
    ("few_slots", "trace64", ("--saturated", "--slots", "4"), 100, None),
    ("baseline", "trace64", ("--saturated", "--baseline"), 100, None),
    ("paced_cancels", "trace64", ("--scale", "0.05", "--cancel", "4", "--chunk", "100"), 100,
     None),
    ("full_trace_saturated", "trace256", ("--saturated",), 100, None),
    # a launch that fails: the jobs of that round fail once their earlier
    # rounds have drained, every other job completes
    ("failed_mh_launch", "trace64", ("--saturated", "--expect-failures"), 300,
     {"HH_FAIL_LAUNCH": "mh_chunk:7"}),
    ("failed_fit_step_launch", "trace64", ("--saturated", "--expect-failures"), 300,
     {"HH_FAIL_LAUNCH": "fit_step:60"}),
]


@pytest.mark.parametrize("name,trace,opts,delay,env", CASES, ids=[c[0] for c in CASES])
def test_replay_has_no_out_of_lifetime_access(harness, name, trace, opts, delay, env):
    d, exe, _ = harness
    rc, out = _replay(exe, d / f"{trace}.txt", *opts, delay=delay, extra_env=env)
    assert rc == 0, out[-6000:]
    assert "violations 0" in out, out[-6000:]


def _planted(d, objs, tag, old, new):
    """The replay built with a copy of the scheduler in which `old` reads `new`."""
    src = open(os.path.join(CSRC, "gc_server.cpp")).read()
    assert old in src
    bad = src.replace(old, new)
    bad = bad.replace('#include "gc_runtime.hpp"', f'#include "{CSRC}/gc_runtime.hpp"')
    bad = bad.replace('#include "gc_timing.hpp"', f'#include "{CSRC}/gc_timing.hpp"')
    p = d / f"gc_server_{tag}.cpp"
    p.write_text(bad)
    obj = _compile(str(p), str(d / f"gc_server_{tag}.o"))
    others = [o for o in objs if not os.path.basename(o).startswith("gc_server.cpp")]
    return _link([obj, *others], str(d / f"replay_{tag}"))


def test_replay_detects_a_planted_lifetime_mistake(harness):
    """A copy of the scheduler that returns a round's descriptor block to the
    arena as soon as the round is enqueued (not when its event completes)."""
    d, _, objs = harness
    exe = _planted(d, objs, "early_round_release",
                   "            (void)hipEventRecord(rec.ev, S->compute);\n"
                   "            inflight.push_back(std::move(rec));",
                   "            (void)hipEventRecord(rec.ev, S->compute);\n"
                   "            S->arena.free(rec.dev);\n"
                   "            rec.dev = nullptr;\n"
                   "            inflight.push_back(std::move(rec));")
    rc, out = _replay(exe, d / "trace64.txt", "--saturated", delay=300)
    # the released block is either still free when a stub reads it, or
    # already handed to a later allocation: both are reported
    early = ("freed arena memory", "allocation made after the launch was enqueued")
    assert rc != 0 and "VIOLATION" in out and any(e in out for e in early), out[-3000:]


def test_replay_shows_failed_round_must_wait_for_earlier_rounds(harness):
    """The failure path as the server first had it: the jobs of a failed round
    released at once, while their earlier rounds may still run.  Their blocks
    then return to the arena under queued work that reads them -- with memory
    handed to the next jobs, kernels reading reused descriptors and arrays.
    The replay shows those accesses; the present failure path (see the
    failed-launch cases above) shows none."""
    d, _, objs = harness
    exe = _planted(d, objs, "immediate_failure",
                   "                for (Job* J : active) {\n"
                   "                    J->cancel = true;\n"
                   "                    J->fail_status = rc;\n"
                   "                    J->err = msg;\n"
                   "                }",
                   "                for (Job* J : active) {\n"
                   "                    J->cancel = true;\n"
                   "                    J->fail_status = rc;\n"
                   "                    J->err = msg;\n"
                   "                    if (!J->finishing) complete_job(S, J, rc);\n"
                   "                }")
    rc, out = _replay(exe, d / "trace64.txt", "--saturated", "--expect-failures", delay=1000,
                      extra_env={"HH_FAIL_LAUNCH": "mh_chunk:7"})
    assert rc != 0 and "VIOLATION" in out, out[-3000:]


def test_replay_detects_lanes_not_joined_into_the_round(harness):
    """A copy of the scheduler whose round event does not wait for the launch
    lanes: the event can complete while groups still run on the lanes, and
    the descriptors and arrays it guards go back to the arena under them."""
    d, _, objs = harness
    exe = _planted(d, objs, "unjoined_lanes",
                   "                (void)hipStreamWaitEvent(S->compute, S->lane_end[k], 0);",
                   "                (void)S->lane_end[k];")
    rc, out = _replay(exe, d / "trace64.txt", "--saturated", delay=300)
    assert rc != 0 and "VIOLATION" in out, out[-3000:]


def _peak(out):
    import re
    m = re.search(r"resident \d+ \(peak (\d+)\)", out)
    assert m, out[-2000:]
    return int(m.group(1))


def test_default_admission_takes_many_small_jobs_and_few_large(harness):
    """With the default slot count, a saturated trace of small jobs keeps more
    than 64 jobs resident (they hold too few lanes to fill the GPU), an
    explicit slot count stays a hard limit, and a trace of large jobs stays
    at 64."""
    d, exe, _ = harness
    rc, out = _replay(exe, d / "trace256small.txt", "--saturated", delay=20)
    assert rc == 0 and "violations 0" in out, out[-6000:]
    assert _peak(out) > 64, out[-2000:]
    rc, out = _replay(exe, d / "trace256small.txt", "--saturated", "--slots", "64", delay=20)
    assert rc == 0 and "violations 0" in out, out[-6000:]
    assert _peak(out) <= 64, out[-2000:]
    rc, out = _replay(exe, d / "trace256.txt", "--saturated", delay=20)
    assert rc == 0 and "violations 0" in out, out[-6000:]
    assert _peak(out) <= 64, out[-2000:]
