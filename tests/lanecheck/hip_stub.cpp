// Host-only stand-in for the HIP runtime, used to check the library's stream
// orderings on the CPU (test infrastructure; no device is touched).
//
// The library's object files are linked against this file instead of the
// HIP runtime.  Memory calls work on host memory, kernel launches do not run
// (the library never reads device data back on the host, so its control
// flow is the same as on a GPU), and every operation that orders work --
// kernel launches, async copies, event records and waits, stream capture,
// graph launches -- becomes a node of a dependency graph.  The checker then
// applies these rules:
//
//   capture-unjoined   at hipStreamEndCapture, every node captured on any
//                      stream must be an ancestor of the origin stream's
//                      last node (each side stream forked into the capture
//                      was joined back);
//   capture-foreign-wait  a stream in a capture waits only on events
//                      recorded in that same capture (an event recorded
//                      outside it, or in an earlier capture, or never
//                      recorded, gives no dependency inside the graph);
//   stale-capture-wait a stream outside any capture waits on an event whose
//                      last record was inside a capture;
//   escape             while a capture is active, work is enqueued on a
//                      stream that is not part of it (it would run at once,
//                      outside the graph);
//   sync-in-capture    a synchronising call while a capture is active;
//   capture-wait-cycle inside one capture, the relation "stream A waited on
//                      an event recorded on stream B", taken over the streams
//                      other than the origin (A is not the origin), has a
//                      cycle (a side stream that waits on a second side
//                      stream which, in the same capture, waits on the first,
//                      possibly through others);
//   call-unjoined      (checked at stub_call_end) work enqueued during one
//                      library call on any stream other than the caller's is
//                      not an ancestor of the caller's stream's last node
//                      (work that a later hipDeviceSynchronize in the call
//                      waited for has completed and is exempt);
//   dead-handle        a graph executable, stream or event is used after it
//                      was destroyed, or a pointer is freed that is not a
//                      live allocation.
#include <hip/hip_runtime_api.h>
#include <sys/mman.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <set>
#include <string>
#include <vector>

namespace {

struct Node {
    std::string what;
    int stream;
    std::vector<int> deps;
    int capture;  // capture id (0: not captured)
};

struct Stream {
    int last = -1;       // last node in stream order
    int capture = 0;     // active capture this stream belongs to
    int pre_last = -1;   // last node before it joined the capture
};

struct Event {
    int node = -1;
    int capture = 0;  // capture id of the last record (0: outside any capture)
    int stream = 0;   // stream of the last record
    bool recorded = false;
};

struct Capture {
    int origin = 0;
    bool active = false;
    std::vector<int> nodes;
    std::set<int> streams;
    std::set<std::pair<int, int>> waits;  // (recording stream, waiting side stream)
};

// does the wait relation of C have a cycle?
bool wait_cycle(const Capture& C) {
    std::map<int, std::vector<int>> adj;
    for (auto& e : C.waits) adj[e.first].push_back(e.second);
    std::map<int, int> color;  // 0 new, 1 on the path, 2 done
    bool cyc = false;
    std::function<void(int)> dfs = [&](int v) {
        color[v] = 1;
        for (int u : adj[v]) {
            if (color[u] == 1) cyc = true;
            else if (color[u] == 0) dfs(u);
        }
        color[v] = 2;
    };
    for (auto& kv : adj)
        if (color[kv.first] == 0) dfs(kv.first);
    return cyc;
}

struct State {
    std::vector<Node> nodes;
    std::map<int, Stream> streams;  // stream id -> state (0 = the null stream)
    std::map<int, Event> events;
    std::map<int, Capture> captures;
    std::map<const void*, std::string> kernels;
    std::map<void*, size_t> allocs;
    std::set<int> live_execs, dead_execs, dead_streams, dead_events;
    std::map<int, int> exec_of_graph;
    std::vector<std::string> violations;
    int next_id = 1;
    int call_first_node = 0;
    int done_upto = 0;  // nodes below this had completed at a device synchronisation
    long n_launch = 0, n_capture = 0, n_graph_launch = 0, n_record = 0, n_wait = 0;
    long n_side_to_side = 0;  // captured waits of one side stream on another's record
    long n_alloc = 0, n_free = 0, n_stream_create = 0, n_event_create = 0, n_sync = 0;
    std::map<const void*, size_t> vars;        // registered device variables: size
    std::map<const void*, void*> var_addr;     // their stand-in device addresses
};

State& st() {
    static State s;
    return s;
}

// handles are small heap cells holding an id
template <class H>
H make_handle(int id) {
    int* p = new int(id);
    return reinterpret_cast<H>(p);
}
template <class H>
int id_of(H h) {
    return h ? *reinterpret_cast<int*>(h) : 0;
}

void violate(const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    st().violations.emplace_back(buf);
}

int active_capture() {
    for (auto& kv : st().captures)
        if (kv.second.active) return kv.first;
    return 0;
}

// A node of work on stream s with extra dependencies.
int add_node(int s, const std::string& what, std::vector<int> extra = {}) {
    State& S = st();
    if (S.dead_streams.count(s)) violate("dead-handle: %s enqueued on destroyed stream %d", what.c_str(), s);
    Stream& ss = S.streams[s];
    const int ac = active_capture();
    if (ac && ss.capture != ac)
        violate("escape: %s enqueued on stream %d outside the active capture %d", what.c_str(), s, ac);
    Node n{what, s, std::move(extra), ss.capture};
    if (ss.last >= 0) n.deps.push_back(ss.last);
    const int id = (int)S.nodes.size();
    S.nodes.push_back(n);
    ss.last = id;
    if (ss.capture) S.captures[ss.capture].nodes.push_back(id);
    return id;
}

// is a an ancestor of (or equal to) b?
bool reaches(int a, int b) {
    if (a < 0) return true;
    if (b < 0) return false;
    State& S = st();
    std::vector<int> stack{b};
    std::vector<char> seen(S.nodes.size(), 0);
    while (!stack.empty()) {
        int x = stack.back();
        stack.pop_back();
        if (x == a) return true;
        if (x < a || seen[x]) continue;  // ids grow along every edge
        seen[x] = 1;
        for (int d : S.nodes[x].deps) stack.push_back(d);
    }
    return false;
}

void sync_point(const char* what, int s) {
    ++st().n_sync;
    const int ac = active_capture();
    if (ac && (s < 0 || st().streams[s].capture == ac))
        violate("sync-in-capture: %s during capture %d", what, ac);
}

}  // namespace

extern "C" {

// ---------------------------------------------------------------- checker --
void stub_reset_violations() { st().violations.clear(); }
int stub_violation_count() { return (int)st().violations.size(); }
// the i-th violation message ("" past the end)
const char* stub_violation(int i) {
    static std::string out;
    out = (i >= 0 && i < (int)st().violations.size()) ? st().violations[i] : std::string();
    return out.c_str();
}
void stub_call_begin() { st().call_first_node = (int)st().nodes.size(); }
// Every node added since stub_call_begin on a stream other than `user` must
// be an ancestor of the user stream's last node.
int stub_call_end(hipStream_t user) {
    State& S = st();
    const int u = id_of(user);
    const int last = S.streams[u].last;
    int bad = 0;
    for (int i = S.call_first_node; i < (int)S.nodes.size(); ++i) {
        const Node& n = S.nodes[i];
        if (n.stream == u || n.capture || i < S.done_upto) continue;
        if (!reaches(i, last)) {
            violate("call-unjoined: %s on stream %d (node %d) is not ordered before the caller's stream %d",
                    n.what.c_str(), n.stream, i, u);
            ++bad;
        }
    }
    return bad;
}
// resource counters: allocations, frees, streams and events created,
// synchronising calls
void stub_resource_counts(long* out) {
    State& S = st();
    out[0] = S.n_alloc;
    out[1] = S.n_free;
    out[2] = S.n_stream_create;
    out[3] = S.n_event_create;
    out[4] = S.n_sync;
}
// counters: launches, captures, graph launches, event records, waits, and
// waits inside a capture of one side stream on an event recorded on another
// (not an error; a topology that is not a plain fork from and join to the
// origin stream)
void stub_counts(long* out) {
    State& S = st();
    out[5] = S.n_side_to_side;
    out[0] = S.n_launch;
    out[1] = S.n_capture;
    out[2] = S.n_graph_launch;
    out[3] = S.n_record;
    out[4] = S.n_wait;
}

// ------------------------------------------------------- registration ----
void** __hipRegisterFatBinary(const void*) {
    static void* mod = nullptr;
    return &mod;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) { st().vars[var] = size; }
hipError_t hipGetSymbolAddress(void** p, const void* symbol) {
    State& S = st();
    auto it = S.vars.find(symbol);
    if (!p || it == S.vars.end()) return hipErrorInvalidSymbol;
    auto a = S.var_addr.find(symbol);
    if (a == S.var_addr.end()) {
        void* q = mmap(nullptr, it->second, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
        if (q == MAP_FAILED) return hipErrorOutOfMemory;
        a = S.var_addr.emplace(symbol, q).first;
    }
    *p = a->second;
    return hipSuccess;
}
void __hipRegisterFunction(void**, const void* hostFunction, char*, const char* deviceName, unsigned int, uint3*,
                           uint3*, dim3*, dim3*, int*) {
    st().kernels[hostFunction] = deviceName ? deviceName : "?";
}

static thread_local hipStream_t g_cfg_stream = nullptr;
hipError_t __hipPushCallConfiguration(dim3, dim3, size_t, hipStream_t stream) {
    g_cfg_stream = stream;
    return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* g, dim3* b, size_t* shm, hipStream_t* stream) {
    if (g) *g = dim3(1, 1, 1);
    if (b) *b = dim3(1, 1, 1);
    if (shm) *shm = 0;
    if (stream) *stream = g_cfg_stream;
    return hipSuccess;
}

static std::string kname(const void* f) {
    auto it = st().kernels.find(f);
    return it == st().kernels.end() ? std::string("kernel?") : it->second;
}

hipError_t hipLaunchKernel(const void* f, dim3, dim3, void**, size_t, hipStream_t stream) {
    ++st().n_launch;
    add_node(id_of(stream), kname(f));
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s);

hipError_t hipExtLaunchKernel(const void* f, dim3 g, dim3 b, void** args, size_t shm, hipStream_t stream,
                              hipEvent_t start, hipEvent_t stop, int) {
    if (start) (void)hipEventRecord(start, stream);
    (void)hipLaunchKernel(f, g, b, args, shm, stream);
    if (stop) (void)hipEventRecord(stop, stream);
    return hipSuccess;
}

hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipGetDevice(int* d) {
    if (d) *d = 0;
    return hipSuccess;
}

// ---------------------------------------------------------------- memory --
hipError_t hipMalloc(void** p, size_t bytes) {
    if (!p) return hipErrorInvalidValue;
    ++st().n_alloc;
    size_t n = bytes ? bytes : 1;
    void* q = mmap(nullptr, n, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (q == MAP_FAILED) return hipErrorOutOfMemory;
    st().allocs[q] = n;
    *p = q;
    return hipSuccess;
}
hipError_t hipFree(void* p) {
    if (!p) return hipSuccess;
    ++st().n_free;
    sync_point("hipFree", -1);
    auto it = st().allocs.find(p);
    if (it == st().allocs.end()) {
        violate("dead-handle: hipFree of %p, not a live allocation", p);
        return hipErrorInvalidValue;
    }
    munmap(p, it->second);
    st().allocs.erase(it);
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t bytes, hipMemcpyKind) {
    sync_point("hipMemcpy", -1);
    std::memmove(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* dst, const void* src, size_t bytes, hipMemcpyKind, hipStream_t s) {
    // host memory stands in for device memory, so an ordered copy is a no-op
    // here as far as values go; it is a node of the stream like a kernel
    (void)dst;
    (void)src;
    (void)bytes;
    add_node(id_of(s), "memcpyAsync");
    return hipSuccess;
}

// ------------------------------------------------------- streams, events --
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
    ++st().n_stream_create;
    const int id = st().next_id++;
    st().streams[id] = Stream();
    *s = make_handle<hipStream_t>(id);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    const int sid = id_of(s);
    if (!st().dead_streams.insert(sid).second) violate("dead-handle: stream %d destroyed twice", sid);
    if (st().streams[sid].capture) violate("dead-handle: stream %d destroyed during a capture", sid);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    sync_point("hipStreamSynchronize", id_of(s));
    return hipSuccess;
}
hipError_t hipDeviceSynchronize() {
    sync_point("hipDeviceSynchronize", -1);
    // every node enqueued outside a capture so far has completed
    if (!active_capture()) st().done_upto = (int)st().nodes.size();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
    ++st().n_event_create;
    const int id = st().next_id++;
    st().events[id] = Event();
    *e = make_handle<hipEvent_t>(id);
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventDestroy(hipEvent_t e) {
    const int eid = id_of(e);
    if (!st().dead_events.insert(eid).second) violate("dead-handle: event %d destroyed twice", eid);
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t e) {
    (void)e;
    sync_point("hipEventSynchronize", -1);
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
    if (ms) *ms = 1.0f;
    return hipSuccess;
}

hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    State& S = st();
    ++S.n_record;
    const int sid = id_of(s);
    if (S.dead_events.count(id_of(e))) violate("dead-handle: destroyed event %d recorded", id_of(e));
    const int n = add_node(sid, "record");
    Event& ev = S.events[id_of(e)];
    ev.node = n;
    ev.recorded = true;
    ev.capture = S.streams[sid].capture;
    ev.stream = sid;
    return hipSuccess;
}

hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
    State& S = st();
    ++S.n_wait;
    const int sid = id_of(s), eid = id_of(e);
    if (S.dead_events.count(eid)) violate("dead-handle: stream %d waits on destroyed event %d", sid, eid);
    Event& ev = S.events[eid];
    Stream& ss = S.streams[sid];
    if (ev.capture) {
        Capture& C = S.captures[ev.capture];
        if (!C.active) {
            violate(ss.capture ? "capture-foreign-wait: stream %d waits on event %d recorded in ended capture %d"
                               : "stale-capture-wait: stream %d waits on event %d last recorded in capture %d",
                    sid, eid, ev.capture);
            return hipSuccess;
        }
        if (ss.capture == 0) {  // the stream joins the capture
            ss.capture = ev.capture;
            ss.pre_last = ss.last;
            ss.last = -1;
            C.streams.insert(sid);
        } else if (ss.capture != ev.capture) {
            violate("capture-foreign-wait: stream %d in capture %d waits on an event of capture %d", sid, ss.capture,
                    ev.capture);
            return hipSuccess;
        }
        if (sid != C.origin && ev.stream != C.origin) ++S.n_side_to_side;
        if (sid != C.origin) C.waits.insert({ev.stream, sid});
        add_node(sid, "wait", {ev.node});
        return hipSuccess;
    }
    if (ss.capture) {
        violate("capture-foreign-wait: stream %d in capture %d waits on event %d %s", sid, ss.capture, eid,
                ev.recorded ? "recorded outside the capture" : "that was never recorded");
        return hipSuccess;
    }
    if (ev.recorded) add_node(sid, "wait", {ev.node});
    return hipSuccess;
}

// ---------------------------------------------------------------- capture --
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    State& S = st();
    const int sid = id_of(s);
    if (sid == 0) return hipErrorStreamCaptureUnsupported;
    Stream& ss = S.streams[sid];
    if (ss.capture) return hipErrorIllegalState;
    const int cid = S.next_id++;
    Capture& C = S.captures[cid];
    C.origin = sid;
    C.active = true;
    C.streams.insert(sid);
    ss.capture = cid;
    ss.pre_last = ss.last;
    ss.last = -1;
    ++S.n_capture;
    return hipSuccess;
}

hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    State& S = st();
    const int sid = id_of(s);
    const int cid = S.streams[sid].capture;
    if (!cid || S.captures[cid].origin != sid) return hipErrorIllegalState;
    Capture& C = S.captures[cid];
    const int last = S.streams[sid].last;
    bool unjoined = false;
    for (int n : C.nodes)
        if (!reaches(n, last)) {
            violate("capture-unjoined: %s on stream %d (node %d) is not joined to the origin stream %d at the end of "
                    "capture %d",
                    S.nodes[n].what.c_str(), S.nodes[n].stream, n, sid, cid);
            unjoined = true;
        }
    if (wait_cycle(C)) {
        std::string rel;
        for (auto& e : C.waits) rel += " " + std::to_string(e.first) + "->" + std::to_string(e.second);
        violate("capture-wait-cycle: the waits between side streams of capture %d form a cycle (record->wait:%s)",
                cid, rel.c_str());
    }
    for (int t : C.streams) {
        Stream& ts = S.streams[t];
        ts.capture = 0;
        ts.last = ts.pre_last;
    }
    C.active = false;
    if (g) *g = make_handle<hipGraph_t>(cid);
    return unjoined ? hipErrorStreamCaptureUnjoined : hipSuccess;
}

hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    State& S = st();
    const int xid = S.next_id++;
    S.live_execs.insert(xid);
    S.exec_of_graph[xid] = id_of(g);
    *x = make_handle<hipGraphExec_t>(xid);
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    State& S = st();
    const int xid = id_of(x);
    if (!S.live_execs.erase(xid)) violate("dead-handle: graph executable %d destroyed twice", xid);
    S.dead_execs.insert(xid);
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
    State& S = st();
    const int xid = id_of(x);
    if (!S.live_execs.count(xid)) violate("dead-handle: graph executable %d launched after it was destroyed", xid);
    ++S.n_graph_launch;
    add_node(id_of(s), "graph");
    return hipSuccess;
}

}  // extern "C"
