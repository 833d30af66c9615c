// A CPU stand-in for the HIP runtime calls librr makes, for testing the library's host logic
// under AddressSanitizer / UBSan without a GPU.  It is test infrastructure only: the library
// itself always links the real runtime.
//
// Memory is host memory and kernels do nothing.  Streams, events, graphs and executable graphs
// are heap objects whose every use reads them, so that the sanitizer reports any use of a
// destroyed one; re-recording or waiting on an event whose last record was on a destroyed stream
// is reported the same way.  Capture follows the CUDA rules: a stream joins a capture by
// waiting on an event recorded in it, the capture ends on every joined stream, and a wait during
// a capture on an event recorded outside it, or in an earlier capture, counts as a violation.
// Counters (captures, allocations, frees) let a driver check the host logic's bookkeeping.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>

namespace {
constexpr unsigned kStreamMagic = 0x5757u, kEventMagic = 0xE7E7u, kGraphMagic = 0x6A6Au, kExecMagic = 0xECECu;
struct MStream {
    unsigned magic = kStreamMagic;
    int capturing = 0;   // id of the capture the stream belongs to, 0 = none
};
struct MEvent {
    unsigned magic = kEventMagic;
    MStream* last = nullptr;   // stream of the last record
    int capture = 0;           // capture id of the last record (0 = outside a capture)
};
struct MGraph {
    unsigned magic = kGraphMagic;
};
struct MExec {
    unsigned magic = kExecMagic;
};

// function-local statics: module constructors of the library may run before this file's
std::set<MStream*>& streams() {
    static std::set<MStream*> s;
    return s;
}
std::map<const void*, void*>& vars() {
    static std::map<const void*, void*> m;
    return m;
}
int g_capture = 0, g_next_capture = 0;
long g_violations = 0, g_captures = 0, g_mallocs = 0, g_frees = 0;
dim3 g_grid, g_block;
size_t g_shmem = 0;
hipStream_t g_stream = nullptr;

void violation(const char* what) {
    std::fprintf(stderr, "MOCK VIOLATION: %s\n", what);
    ++g_violations;
}
MStream* stream_of(hipStream_t s, const char* who) {
    if (!s) return nullptr;   // the null stream
    MStream* m = reinterpret_cast<MStream*>(s);
    if (m->magic != kStreamMagic) violation(who);
    return m;
}
MEvent* event_of(hipEvent_t e, const char* who) {
    MEvent* m = reinterpret_cast<MEvent*>(e);
    if (!m || m->magic != kEventMagic) violation(who);
    return m;
}
}  // namespace

extern "C" {
long mock_violations() { return g_violations; }
long mock_captures() { return g_captures; }
long mock_mallocs() { return g_mallocs; }
long mock_frees() { return g_frees; }

void** __hipRegisterFatBinary(const void*) {
    static void* h = nullptr;
    return &h;
}
void __hipUnregisterFatBinary(void**) {}
void __hipRegisterFunction(void**, const void*, char*, const char*, unsigned int, void*, void*, void*, void*, int*) {}
void __hipRegisterVar(void**, void* var, char*, char*, int, size_t size, int, int) {
    vars()[var] = std::calloc(1, size ? size : 1);
}
hipError_t __hipPushCallConfiguration(dim3 grid, dim3 block, size_t shmem, hipStream_t stream) {
    g_grid = grid;
    g_block = block;
    g_shmem = shmem;
    g_stream = stream;
    return hipSuccess;
}
hipError_t __hipPopCallConfiguration(dim3* grid, dim3* block, size_t* shmem, hipStream_t* stream) {
    *grid = g_grid;
    *block = g_block;
    *shmem = g_shmem;
    *stream = g_stream;
    return hipSuccess;
}
}

hipError_t hipLaunchKernel(const void*, dim3 grid, dim3 block, void**, size_t, hipStream_t stream) {
    stream_of(stream, "kernel launch on a destroyed stream");
    if (grid.x == 0 || grid.y == 0 || grid.z == 0 || block.x == 0 || block.x * block.y * block.z > 1024)
        violation("kernel launch with an empty grid or an oversized workgroup");
    return hipSuccess;
}
hipError_t hipMalloc(void** p, size_t n) {
    if (g_capture) violation("allocation during a capture");
    ++g_mallocs;
    *p = std::calloc(1, n ? n : 1);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
    if (g_capture) violation("free during a capture");
    if (p) ++g_frees;
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind kind) {
    if (g_capture) violation("synchronous copy during a capture");
    std::memmove(d, s, n);
    // RR_MOCK_FLAGS_SET: device-to-host copies come back with every 32-bit word 1, so that
    // the batched call's per-pool states report an overflow and every pool takes the
    // single-pool path (the batched call's state read is the library's only synchronous
    // device-to-host copy)
    if (kind == hipMemcpyDeviceToHost && std::getenv("RR_MOCK_FLAGS_SET")) {
        uint32_t* w = static_cast<uint32_t*>(d);
        for (size_t i = 0; i < n / 4; ++i) w[i] = 1u;
    }
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t st) {
    stream_of(st, "copy on a destroyed stream");
    std::memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t st) {
    stream_of(st, "memset on a destroyed stream");
    std::memset(d, v, n);
    return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int* v, hipDeviceAttribute_t, int) {
    *v = 256;
    return hipSuccess;
}
hipError_t hipDeviceSynchronize() {
    if (g_capture) violation("device synchronisation during a capture");
    return hipSuccess;
}
hipError_t hipGetLastError() { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "mock runtime error"; }
hipError_t hipFuncGetAttributes(hipFuncAttributes* a, const void*) {
    std::memset(a, 0, sizeof(*a));
    a->numRegs = 128;
    return hipSuccess;
}
hipError_t hipFuncSetAttribute(const void*, hipFuncAttribute, int) { return hipSuccess; }
hipError_t hipGetSymbolAddress(void** p, const void* sym) {
    auto it = vars().find(sym);
    if (it == vars().end()) return hipErrorInvalidSymbol;
    *p = it->second;
    return hipSuccess;
}

hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
    MStream* m = new MStream();
    streams().insert(m);
    *s = reinterpret_cast<hipStream_t>(m);
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
    MStream* m = stream_of(s, "destroying a destroyed stream");
    if (m->capturing) violation("destroying a stream during a capture");
    streams().erase(m);
    delete m;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t s) {
    MStream* m = stream_of(s, "synchronising a destroyed stream");
    if (m && m->capturing) violation("synchronising a capturing stream");
    return hipSuccess;
}
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned int) {
    MStream* ms = stream_of(s, "wait on a destroyed stream");
    MEvent* me = event_of(e, "wait on a destroyed event");
    if (me->last) stream_of(reinterpret_cast<hipStream_t>(me->last), "wait on an event of a destroyed stream");
    if (me->capture) {
        if (me->capture != g_capture) violation("wait on an event recorded in an earlier capture");
        else if (ms) ms->capturing = g_capture;   // the stream joins the capture
    } else if (ms && ms->capturing) {
        violation("capturing stream waits on an event recorded outside the capture");
    }
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) {
    *e = reinterpret_cast<hipEvent_t>(new MEvent());
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete event_of(e, "destroying a destroyed event");
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
    MEvent* me = event_of(e, "recording a destroyed event");
    MStream* ms = stream_of(s, "recording on a destroyed stream");
    if (me->last) stream_of(reinterpret_cast<hipStream_t>(me->last), "re-recording an event of a destroyed stream");
    me->last = ms;
    me->capture = ms ? ms->capturing : 0;
    return hipSuccess;
}
hipError_t hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    event_of(a, "timing a destroyed event");
    event_of(b, "timing a destroyed event");
    *ms = 1.0f;
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode) {
    MStream* m = stream_of(s, "capture on a destroyed stream");
    if (!m || g_capture) {
        violation("capture begun on the null stream or inside another capture");
        return hipErrorIllegalState;
    }
    g_capture = ++g_next_capture;
    m->capturing = g_capture;
    ++g_captures;
    return hipSuccess;
}
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t* g) {
    MStream* m = stream_of(s, "ending a capture on a destroyed stream");
    if (!m || m->capturing != g_capture || !g_capture) violation("capture ended on a stream that did not begin it");
    for (MStream* x : streams())
        if (x->capturing == g_capture) x->capturing = 0;   // the capture ends on every joined stream
    g_capture = 0;
    *g = reinterpret_cast<hipGraph_t>(new MGraph());
    return hipSuccess;
}
hipError_t hipGraphInstantiate(hipGraphExec_t* x, hipGraph_t g, hipGraphNode_t*, char*, size_t) {
    if (reinterpret_cast<MGraph*>(g)->magic != kGraphMagic) violation("instantiating a destroyed graph");
    *x = reinterpret_cast<hipGraphExec_t>(new MExec());
    return hipSuccess;
}
hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t s) {
    stream_of(s, "graph launch on a destroyed stream");
    if (reinterpret_cast<MExec*>(x)->magic != kExecMagic) violation("launching a destroyed graph");
    return hipSuccess;
}
hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
    MExec* m = reinterpret_cast<MExec*>(x);
    if (m->magic != kExecMagic) violation("destroying a destroyed graph");
    delete m;
    return hipSuccess;
}
hipError_t hipGraphDestroy(hipGraph_t g) {
    MGraph* m = reinterpret_cast<MGraph*>(g);
    if (m->magic != kGraphMagic) violation("destroying a destroyed graph");
    delete m;
    return hipSuccess;
}
