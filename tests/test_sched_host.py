"""The server's admission and failure logic (paper_2407_14783_amd/csrc/batcher.h) on the host, against a fake
backend that steps a host table of env states (tests/sched_fake_backend.cpp), fails batches at random
after their step has run, and takes host-forced faults.

Checks: every request completes exactly once; no two batches in flight share an env slot; no batch
exceeds its arena; each completed request's results and the final table equal a serial run of the
completed requests in arrival order (so a retried batch changes nothing); requests of a batch that
fails on every attempt fail and leave their slots as they were.
"""
import json
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def fake(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sched") / "sched_fake_backend")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-I", os.path.join(ROOT, "paper_2407_14783_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sched_fake_backend.cpp"), "-o", exe])

    def run(seed, n, fail_prob, inject, attempts):
        out = subprocess.run([exe, str(seed), str(n), str(fail_prob), str(inject), str(attempts)], capture_output=True,
                             text=True, timeout=120)
        assert out.returncode == 0, out.stderr
        return json.loads(out.stdout)
    return run


def _invariants(r):
    assert r["unfinished"] == 0 and r["completed_more_than_once"] == 0
    assert r["ok"] + r["failed"] == r["requests"]
    assert r["overlap_violations"] == 0 and r["budget_violations"] == 0
    assert r["wrong_results"] == 0 and r["state_mismatch"] == 0


def test_scheduler_without_failures(fake):
    r = fake(1, 3000, 0.0, 0, 3)
    _invariants(r)
    assert r["ok"] == 3000 and r["failed_batches"] == 0 and r["requeued"] == 0
    assert r["max_batch"] > 8          # requests of distinct slots share batches


def test_scheduler_requeues_after_backend_errors(fake):
    r = fake(2, 3000, 0.1, 25, 6)
    _invariants(r)
    assert r["failed_batches"] == r["random_failures"] + 25
    assert r["requeued"] > 0 and r["ok"] > 2900


def test_injected_faults_change_no_result(fake):
    clean = fake(3, 2000, 0.0, 0, 3)
    faulty = fake(3, 2000, 0.0, 60, 100)
    _invariants(clean)
    _invariants(faulty)
    assert faulty["ok"] == 2000 and faulty["failed_batches"] == 60


def test_requests_fail_after_max_attempts_and_leave_slots_restored(fake):
    r = fake(4, 300, 1.0, 0, 2)
    _invariants(r)            # the serial reference has no completed request: the table must be untouched
    assert r["ok"] == 0 and r["failed"] == 300
