"""The serving scheduler's policy on the CPU (no GPU): dr_sched.cpp driven by
a simulated executor with a fake clock (tests/c/sched_sim.cpp), built with
AddressSanitizer and UndefinedBehaviorSanitizer.  Scenarios: Poisson mix,
budget refusal and FIFO queueing, the output counted in the footprint, slot
exhaustion, a small request beside a full-frame copy, out-of-order
completion, failures of copies (enqueue and device), allocations and epochs
(launch and device).  Planted mistakes in a copy of the policy must each fail
a scenario."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2201_13309_amd", "csrc")
SIM = os.path.join(ROOT, "tests", "c", "sched_sim.cpp")
FLAGS = ["-std=c++17", "-O1", "-g", "-Wall", "-Wextra", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
         f"-I{os.path.join(ROOT, 'include')}"]


@pytest.fixture(scope="module")
def sim_obj(tmp_path_factory):
    """The simulated executor and scenarios, compiled once."""
    tmp = tmp_path_factory.mktemp("sim")
    obj = tmp / "sched_sim.o"
    subprocess.run(["g++", *FLAGS, f"-I{CSRC}", "-c", SIM, "-o", str(obj)], check=True,
                   capture_output=True)
    return obj


def _build(tmp, sched_src, sim_obj):
    exe = tmp / "sched_sim"
    subprocess.run(["g++", *FLAGS, f"-I{CSRC}", str(sched_src), str(sim_obj), "-o", str(exe)],
                   check=True, capture_output=True)
    return exe


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)


def test_scheduler_scenarios(tmp_path, sim_obj):
    exe = _build(tmp_path, os.path.join(CSRC, "dr_sched.cpp"), sim_obj)
    r = _run(exe)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.count(" ok") == 10


MUTANTS = [
    ("release_before_drained", "const bool drained = r->copies.empty() && r->epochs_open == 0;",
     "const bool drained = r->failing || (r->copies.empty() && r->epochs_open == 0);"),
    ("fail_everyone_on_launch_error", "for (Req* r : reqs) fail(r, st);",
     "for (Req* r : active_) fail(r, st);"),
    ("admit_over_budget", "if (c_.in_use + r->footprint > budget_) break;",
     "if (c_.in_use > budget_) break;"),
    ("largest_copy_first", "if (!best || left < best_left) {", "if (!best || left > best_left) {"),
    ("finish_before_last_rows", "if (r->rows_ready == r->ny) {  // every row launched",
     "if (r->rows_ready > 0) {  // every row launched"),
    ("no_epoch_limit", "if (epochs_in_flight() >= kEpochsInFlight) return false;",
     "if (epochs_in_flight() > kEpochSlots) return false;"),
    ("copy_slot_not_returned", "            copies_in_flight_--;\n",
     "            if (q == kDone) copies_in_flight_--;\n"),
    ("ready_before_copy_done", "if (q == kDone && !r->failing) r->rows_ready = r->copies.front().second;",
     "if (!r->failing) r->rows_ready = r->rows_copied;"),
]


@pytest.mark.parametrize("name,orig,repl", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_scheduler_mutant_is_caught(tmp_path, sim_obj, name, orig, repl):
    text = open(os.path.join(CSRC, "dr_sched.cpp")).read()
    assert orig in text, f"mutation site for {name} not found"
    src = tmp_path / "dr_sched.cpp"
    src.write_text(text.replace(orig, repl))
    exe = _build(tmp_path, src, sim_obj)
    r = _run(exe)
    assert r.returncode != 0 and "FAIL" in r.stdout, (name, r.stdout)
