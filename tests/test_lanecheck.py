"""Stream-ordering checks of the library's launch sequences, on the CPU.

The library's own object files are linked against a host-only stand-in for
the HIP runtime (tests/lanecheck/hip_stub.cpp) that turns every launch,
copy, event record and wait, capture and graph launch into a node of a
dependency graph and checks the rules listed at the top of that file: every
side stream forked in a call or a capture is joined back to the caller's
stream before the call returns or the capture ends, captured waits are on
events recorded in the same capture, no work escapes an active capture, no
synchronisation inside one, no wait cycle between side streams of one
capture, no use of destroyed graphs, streams or events.

Every entry point runs three times in a row per caller stream (direct,
captured, replayed), at sizes with and without the low-degree sub-plan, in
every precision mode, in workspace slices, as ragged batches, past both
graph-cache bounds and with the kernel trace on."""
import json
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
LC = os.path.join(HERE, "lanecheck")
sys.path.insert(0, LC)


@pytest.fixture(scope="module")
def built():
    import build as lbuild

    try:
        lbuild.build()
    except FileNotFoundError as e:
        pytest.skip(str(e))
    return lbuild


def _run(script, *args):
    # a fresh process: the library's HIP references must bind to the
    # stand-in, not to a HIP runtime another module may have loaded
    r = subprocess.run([sys.executable, os.path.join(LC, script), *args], capture_output=True, text=True,
                       timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    return json.loads(r.stdout.strip().splitlines()[-1])


def test_checker_names_each_planted_mistake(built):
    out = _run("planted.py")
    expect = {
        "correct fork and join in a capture": None,
        "side stream not joined before the capture ends": "capture-unjoined",
        "capture waits on an event recorded outside it": "capture-foreign-wait",
        "capture waits on an event never recorded": "capture-foreign-wait",
        "work on a stream outside the active capture": "escape",
        "synchronisation inside a capture": "sync-in-capture",
        "two side streams wait on each other in a capture": "capture-wait-cycle",
        "wait outside any capture on an event recorded in one": "stale-capture-wait",
        "direct call joins its side stream": None,
        "direct call leaves side-stream work unjoined": "call-unjoined",
        "graph launched after it was destroyed": "dead-handle",
        "event recorded after it was destroyed": "dead-handle",
    }
    assert set(out) == set(expect)
    for name, rule in expect.items():
        rules = {v.split(":")[0] for v in out[name]}
        if rule is None:
            assert not rules, (name, out[name])
        else:
            assert rules == {rule}, (name, out[name])


def test_library_stream_orderings(built):
    out = _run("run_check.py")
    assert out["errors"] == []
    assert out["violation_count"] == 0, out["violations"]
    # the sequences did run direct, captured and replayed
    assert out["calls"] > 3000 and out["launches"] > 10000
    assert out["captures"] > 1000 and out["graph_launches"] > 1500
    assert out["event_waits"] > 1000
    # the ragged batch's grid query
    assert out["batch_grid"]["before_ok"] and out["batch_grid"]["after_ok"], out["batch_grid"]
    assert out["batch_grid"]["bad_status"] == [-1, -1, -1, -1, -2]
    # the allocation-free forward allocates, frees, creates and synchronises
    # nothing, and neither captures nor records nor waits on events
    assert len(out["noalloc"]) == 4
    for case, r in out["noalloc"].items():
        assert r["launches"] > 0, case
        assert r["resources"] == [0, 0, 0, 0, 0], case
        assert r["captures_graphs_records_waits"] == [0, 0, 0, 0], case
