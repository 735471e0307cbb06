"""Planted ordering mistakes, each driven straight into the HIP stand-in:
the checker must name the rule each one breaks (and find nothing in the
correct sequence).  Prints {scenario: [violation messages]} as JSON."""
import ctypes
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)
import build as lbuild  # noqa: E402


def main():
    S = ctypes.CDLL(lbuild.STUB, mode=ctypes.RTLD_GLOBAL)
    vp = ctypes.c_void_p
    S.stub_violation.restype = ctypes.c_char_p
    S.stub_call_end.argtypes = [vp]
    for f in ("hipEventRecord", "hipStreamWaitEvent", "hipStreamBeginCapture", "hipStreamEndCapture",
              "hipGraphInstantiate", "hipGraphLaunch", "hipGraphExecDestroy", "hipStreamSynchronize",
              "hipEventDestroy"):
        getattr(S, f).restype = ctypes.c_int
    S.hipStreamWaitEvent.argtypes = [vp, vp, ctypes.c_uint]
    S.hipEventRecord.argtypes = [vp, vp]
    S.hipStreamBeginCapture.argtypes = [vp, ctypes.c_int]
    S.hipStreamEndCapture.argtypes = [vp, ctypes.POINTER(vp)]
    S.hipGraphInstantiate.argtypes = [ctypes.POINTER(vp), vp, vp, vp, ctypes.c_size_t]
    S.hipGraphLaunch.argtypes = [vp, vp]
    S.hipGraphExecDestroy.argtypes = [vp]
    S.hipStreamSynchronize.argtypes = [vp]
    S.hipEventDestroy.argtypes = [vp]

    class dim(ctypes.Structure):
        _fields_ = [("x", ctypes.c_uint), ("y", ctypes.c_uint), ("z", ctypes.c_uint)]

    S.hipLaunchKernel.argtypes = [vp, dim, dim, vp, ctypes.c_size_t, vp]

    def stream():
        s = vp()
        S.hipStreamCreateWithFlags(ctypes.byref(s), 1)
        return s

    def event():
        e = vp()
        S.hipEventCreateWithFlags(ctypes.byref(e), 2)
        return e

    def kernel(s):
        S.hipLaunchKernel(None, dim(1, 1, 1), dim(64, 1, 1), None, 0, s)

    def fork(a, b, e):
        S.hipEventRecord(e, a)
        S.hipStreamWaitEvent(b, e, 0)

    out = {}

    def scenario(name, fn):
        S.stub_reset_violations()
        fn()
        out[name] = [S.stub_violation(i).decode() for i in range(S.stub_violation_count())]

    def capture(body):
        o, a, b = stream(), stream(), stream()
        e = [event() for _ in range(4)]
        S.hipStreamBeginCapture(o, 2)
        body(o, a, b, e)
        g = vp()
        S.hipStreamEndCapture(o, ctypes.byref(g))
        return g

    def correct(o, a, b, e):
        fork(o, a, e[0])
        kernel(a)
        fork(o, b, e[1])
        kernel(b)
        kernel(o)
        fork(a, o, e[2])
        fork(b, o, e[3])
        kernel(o)

    def unjoined(o, a, b, e):
        fork(o, a, e[0])
        kernel(a)
        kernel(o)

    def foreign(o, a, b, e):
        S.hipStreamWaitEvent(o, pre, 0)
        kernel(o)

    def never(o, a, b, e):
        S.hipStreamWaitEvent(o, e[3], 0)
        kernel(o)

    def escape(o, a, b, e):
        kernel(o)
        kernel(a)

    def sync(o, a, b, e):
        kernel(o)
        S.hipStreamSynchronize(o)

    def cycle(o, a, b, e):
        fork(o, a, e[0])
        fork(o, b, e[1])
        kernel(a)
        fork(a, b, e[2])
        kernel(b)
        fork(b, a, e[3])
        kernel(a)
        j = event()
        fork(a, o, j)

    pre = event()
    outside = stream()
    S.hipEventRecord(pre, outside)
    scenario("correct fork and join in a capture", lambda: capture(correct))
    scenario("side stream not joined before the capture ends", lambda: capture(unjoined))
    scenario("capture waits on an event recorded outside it", lambda: capture(foreign))
    scenario("capture waits on an event never recorded", lambda: capture(never))
    scenario("work on a stream outside the active capture", lambda: capture(escape))
    scenario("synchronisation inside a capture", lambda: capture(sync))
    scenario("two side streams wait on each other in a capture", lambda: capture(cycle))

    def stale():
        ev = []

        def body(o, a, b, e):
            fork(o, a, e[0])
            kernel(a)
            fork(a, o, e[1])
            ev.append(e[1])

        capture(body)
        s = stream()
        S.hipStreamWaitEvent(s, ev[0], 0)

    scenario("wait outside any capture on an event recorded in one", stale)

    def call_unjoined():
        u, side, e = stream(), stream(), event()
        S.stub_call_begin()
        fork(u, side, e)
        kernel(side)
        kernel(u)
        S.stub_call_end(u)

    def call_joined():
        u, side, e, e2 = stream(), stream(), event(), event()
        S.stub_call_begin()
        fork(u, side, e)
        kernel(side)
        kernel(u)
        fork(side, u, e2)
        S.stub_call_end(u)

    scenario("direct call joins its side stream", call_joined)
    scenario("direct call leaves side-stream work unjoined", call_unjoined)

    def dead_exec():
        g = capture(correct)
        x = vp()
        S.hipGraphInstantiate(ctypes.byref(x), g, None, None, 0)
        s = stream()
        S.hipGraphLaunch(x, s)
        S.hipGraphExecDestroy(x)
        S.hipGraphLaunch(x, s)

    def dead_event():
        e, s = event(), stream()
        S.hipEventDestroy(e)
        S.hipEventRecord(e, s)

    scenario("graph launched after it was destroyed", dead_exec)
    scenario("event recorded after it was destroyed", dead_event)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
