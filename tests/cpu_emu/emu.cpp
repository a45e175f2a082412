// CPU emulation of HIP kernel execution and runtime calls (TEST INFRASTRUCTURE).
//
// One fiber per GPU thread, scheduled cooperatively on the calling OS thread.  A wave
// intrinsic is a two-phase rendezvous of the live lanes of a wave (deposit, then read); a
// __syncthreads() waits for every live thread of the block.  Any lane reaching a different
// intrinsic (by source line) than its wave-mates is reported as divergent use, and a round in
// which no fiber can make progress is reported as a deadlock; both abort the process.
#include "hip/hip_runtime.h"

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <mutex>
#include <random>
#include <set>
#include <cstdio>
#include <cstdlib>
#include <vector>

#if defined(__SANITIZE_ADDRESS__)
#define EMU_ASAN 1
#elif defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#endif
#endif
#ifdef EMU_ASAN
#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>
#endif

namespace evsim {
// Dynamic shared memory ("extern __shared__ float smem[]") of the block that is running.  The
// initializer is not a constant, so the compiler emits this variable's TLS init function: g++
// calls that function unconditionally from function templates that declare the array `extern`,
// and without a definition the call would jump to address 0.
static float zero_value() { return 0.0f; }
thread_local float smem[1 << 16] = {zero_value()};
}

// Minimal x86-64 (System V) stack switch: saves the callee-saved registers and the SSE/x87
// control words on the current stack, stores the stack pointer to *save, loads `next` and pops
// the same frame from it.  No signal-mask system call (unlike swapcontext).
extern "C" void emu_ctx_switch(void** save, void* next);
asm(R"(
    .text
    .globl emu_ctx_switch
    .type emu_ctx_switch, @function
emu_ctx_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    subq $8, %rsp
    stmxcsr (%rsp)
    fnstcw 4(%rsp)
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    ldmxcsr (%rsp)
    fldcw 4(%rsp)
    addq $8, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size emu_ctx_switch, .-emu_ctx_switch
)");

namespace {

constexpr size_t kStack = 512 * 1024;

struct Fiber {
    void* sp;          // saved stack pointer while switched out
    emu_uint3 tid;
    int wave;
    bool done;
};

struct Wave {
    int state;        // 0 collecting, 1 draining
    int arrived, departed;
    int op, line;
    uint64_t gen;
    uint64_t vals[64];
    int args[64];
    bool present[64];
    int live;
};

struct Block {
    std::vector<Fiber> fibers;
    std::vector<Wave> waves;
    int live = 0;
    int bar_arrived = 0;
    int bar_line = -1;
    uint64_t bar_gen = 0;
    void* sched_sp = nullptr;
    int cur = -1;
    const std::function<void()>* body = nullptr;
    uint64_t progress = 0;
    const char* name = "";
};

Block B;
const void* g_main_bottom = nullptr;   // the scheduler's (process) stack, for the sanitizer
size_t g_main_size = 0;
emu_uint3 g_block{0, 0, 0};
dim3 g_bdim, g_gdim;
std::vector<char*> g_stacks;
hipError_t g_last = hipSuccess;

[[noreturn]] void die(const char* what) {
    fprintf(stderr, "[cpu-emu] %s in kernel %s, block (%u,%u,%u)\n", what, B.name, g_block.x,
            g_block.y, g_block.z);
    fflush(stderr);
    abort();
}

void switch_to(void** save, void* next, const void* stack_bottom, size_t size) {
#ifdef EMU_ASAN
    void* fake = nullptr;
    __sanitizer_start_switch_fiber(&fake, stack_bottom, size);
    emu_ctx_switch(save, next);
    __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#else
    (void)stack_bottom;
    (void)size;
    emu_ctx_switch(save, next);
#endif
}

void yield_fiber() {
    Fiber& f = B.fibers[B.cur];
    // back to the scheduler, which runs on the process stack
    switch_to(&f.sp, B.sched_sp, g_main_bottom, g_main_size);
}

void wave_try_complete(Wave& w) {
    if (w.state == 0 && w.arrived > 0 && w.arrived == w.live) {
        w.state = 1;
        w.departed = 0;
        w.gen++;
        B.progress++;
    }
}

void barrier_try_release() {
    if (B.bar_arrived > 0 && B.bar_arrived == B.live) {
        B.bar_arrived = 0;
        B.bar_line = -1;
        B.bar_gen++;
        B.progress++;
    }
}

[[noreturn]] void trampoline() {
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &g_main_bottom, &g_main_size);
#endif
    (*B.body)();
    Fiber& f = B.fibers[B.cur];
    f.done = true;
    B.live--;
    Wave& w = B.waves[f.wave];
    w.live--;
    B.progress++;
    wave_try_complete(w);
    barrier_try_release();
#ifdef EMU_ASAN
    __sanitizer_start_switch_fiber(nullptr, g_main_bottom, g_main_size);
#endif
    void* dead = nullptr;
    emu_ctx_switch(&dead, B.sched_sp);   // never resumed
    abort();
}

// Initial frame of a fiber: what emu_ctx_switch pops, then the entry address as return address
// and a fake return address of the entry function (so rsp is 8 mod 16 at its first instruction).
void* initial_sp(char* stack) {
#ifdef EMU_ASAN
    // the stack is reused across blocks: drop the frame poisoning of the previous fiber
    __asan_unpoison_memory_region(stack, kStack);
#endif
    uint64_t top = ((uint64_t)(stack + kStack)) & ~(uint64_t)15;
    uint64_t* sp = (uint64_t*)top;
    *--sp = 0;                          // fake return address of trampoline
    *--sp = (uint64_t)&trampoline;      // popped by ret
    for (int r = 0; r < 6; ++r) *--sp = 0;   // rbp rbx r12 r13 r14 r15
    // default x86-64 SysV control words: MXCSR 0x1F80 (round to nearest, all exceptions
    // masked, no flush-to-zero), x87 control word 0x037F
    *--sp = (uint64_t)0x1F80u | ((uint64_t)0x037Fu << 32);
    return sp;
}

void run_block(int n, const std::function<void()>& body, const char* name) {
    B.fibers.assign(n, Fiber());
    B.waves.assign((n + 63) / 64, Wave());
    for (auto& w : B.waves) memset(&w, 0, sizeof(Wave));
    B.live = n;
    B.bar_arrived = 0;
    B.bar_line = -1;
    B.bar_gen = 0;
    B.body = &body;
    B.name = name;
    while ((int)g_stacks.size() < n) g_stacks.push_back((char*)malloc(kStack));
    for (int i = 0; i < n; ++i) {
        Fiber& f = B.fibers[i];
        f.tid = emu_uint3{(unsigned)i, 0u, 0u};
        f.wave = i / 64;
        f.done = false;
        B.waves[f.wave].live++;
        f.sp = initial_sp(g_stacks[i]);
    }
    while (B.live > 0) {
        const uint64_t before = B.progress;
        for (int i = 0; i < n; ++i) {
            if (B.fibers[i].done) continue;
            B.cur = i;
            switch_to(&B.sched_sp, B.fibers[i].sp, g_stacks[i], kStack);
        }
        if (B.live > 0 && B.progress == before) die("deadlock (no fiber can progress)");
    }
    B.cur = -1;
}

}  // namespace

const emu_uint3& emu_thread_idx() { return B.fibers[B.cur].tid; }
const emu_uint3& emu_block_idx() { return g_block; }
const dim3& emu_block_dim() { return g_bdim; }
const dim3& emu_grid_dim() { return g_gdim; }

void emu_syncthreads(int line) {
    if (B.bar_arrived == 0) B.bar_line = line;
    else if (B.bar_line != line) die("__syncthreads reached from different lines");
    const uint64_t gen = B.bar_gen;
    B.bar_arrived++;
    B.progress++;
    barrier_try_release();
    while (B.bar_gen == gen) yield_fiber();
}

uint64_t emu_wave_exchange(int op, uint64_t value, int arg, int line) {
    Fiber& f = B.fibers[B.cur];
    Wave& w = B.waves[f.wave];
    const int lane = (int)(f.tid.x & 63u);
    while (w.state == 1) yield_fiber();
    if (w.arrived == 0) {
        w.op = op;
        w.line = line;
    } else if (w.op != op || w.line != line) {
        die("divergent wave intrinsic (lanes at different calls)");
    }
    w.vals[lane] = value;
    w.args[lane] = arg;
    w.present[lane] = true;
    w.arrived++;
    B.progress++;
    const uint64_t gen = w.gen;
    wave_try_complete(w);
    while (w.gen == gen) yield_fiber();
    uint64_t r = 0;
    if (op == EMU_SHFL) {
        const int src = arg & 63;
        r = w.present[src] ? w.vals[src] : value;
    } else if (op == EMU_SHFL_UP) {
        const int src = lane - arg;
        r = (src >= 0 && w.present[src]) ? w.vals[src] : value;
    } else if (op == EMU_SHFL_DOWN) {
        const int src = lane + arg;
        r = (src < 64 && w.present[src]) ? w.vals[src] : value;
    } else {
        for (int l = 0; l < 64; ++l)
            if (w.present[l] && w.vals[l]) r |= 1ull << l;
    }
    w.departed++;
    B.progress++;
    if (w.departed == w.arrived) {
        w.state = 0;
        w.arrived = 0;
        memset(w.present, 0, sizeof(w.present));
    }
    return r;
}

// Execution options (emu_set_execution): shuffled block order when the seed is not zero.
static uint64_t g_shuffle_seed = getenv("EMU_SHUFFLE") ? strtoull(getenv("EMU_SHUFFLE"), 0, 10) : 0;
static uint64_t g_launches = 0;

void emu_run_grid(dim3 grid, dim3 block, size_t shmem, const std::function<void()>& body,
                  const char* name) {
    if (shmem > sizeof(evsim::smem)) die("dynamic shared memory request too large");
    if (getenv("EMU_TRACE"))
        fprintf(stderr, "emu: launch %s grid %u block %u shmem %zu\n", name, grid.x, block.x,
                shmem);
    if (block.y != 1 || block.z != 1 || block.x == 0 || block.x > 1024) die("unsupported block");
    g_gdim = grid;
    g_bdim = block;
    const uint64_t n = (uint64_t)grid.x * grid.y * grid.z;
    if (g_shuffle_seed == 0) {
        for (unsigned bz = 0; bz < grid.z; ++bz)
            for (unsigned by = 0; by < grid.y; ++by)
                for (unsigned bx = 0; bx < grid.x; ++bx) {
                    g_block = emu_uint3{bx, by, bz};
                    run_block((int)block.x, body, name);
                }
        return;
    }
    // blocks in a seeded random order (the device promises no order between blocks)
    std::vector<uint64_t> order(n);
    for (uint64_t i = 0; i < n; ++i) order[i] = i;
    std::mt19937_64 rng(g_shuffle_seed + 0x9e3779b97f4a7c15ull * ++g_launches);
    std::shuffle(order.begin(), order.end(), rng);
    for (uint64_t i : order) {
        g_block = emu_uint3{(unsigned)(i % grid.x), (unsigned)((i / grid.x) % grid.y),
                            (unsigned)(i / ((uint64_t)grid.x * grid.y))};
        run_block((int)block.x, body, name);
    }
}

// ---- runtime API ------------------------------------------------------------------------------
//
// By default every call runs its work at once.  With deferred execution (emu_set_execution, or
// EMU_DEFERRED=1 in the environment) kernels, memsets and copies that involve only device or
// pinned memory are queued per stream and run only when a synchronisation needs them: a stream
// or event synchronisation, a wait on an event, and the calls that HIP documents as synchronous
// (hipFree and hipHostFree synchronise the device; a copy to or from pageable host memory
// completes before it returns, after the work queued before it on its stream).  Code that reads a
// result before synchronising, or frees or regrows a buffer that queued work still uses, then
// reads stale data or trips the sanitizer, as it could on the device.
struct emu_event_t;
struct EmuOp {
    int kind;                    // 0 work, 1 event record, 2 wait for an event record
    std::function<void()> fn;
    emu_event_t* ev;
    uint64_t seq;                // the record's sequence number
    struct emu_stream_t* where;  // wait: the stream holding that record
};
struct emu_stream_t {
    std::deque<EmuOp> q;
};
struct emu_event_t {
    std::chrono::steady_clock::time_point t;
    uint64_t recorded = 0, completed = 0;
    emu_stream_t* where = nullptr;
};

static bool g_deferred = getenv("EMU_DEFERRED") && atoi(getenv("EMU_DEFERRED")) != 0;
static std::recursive_mutex g_exec_mu;      // queues and execution (one host thread at a time)
static emu_stream_t g_null_stream;
static std::set<emu_stream_t*> g_streams = {&g_null_stream};

static emu_stream_t* stream_of(hipStream_t s) { return s ? s : &g_null_stream; }

static void drain_event(emu_event_t* e, uint64_t target, emu_stream_t* where);

// Runs the head of a stream's queue (a wait first runs what it waits for).
static void step_head(emu_stream_t* s) {
    EmuOp op = std::move(s->q.front());
    s->q.pop_front();
    if (op.kind == 2) {
        if (op.ev->completed < op.seq) drain_event(op.ev, op.seq, op.where);
        return;
    }
    if (op.kind == 1) {
        if (op.ev->completed < op.seq) op.ev->completed = op.seq;
        op.ev->t = std::chrono::steady_clock::now();
        return;
    }
    op.fn();
}

static void drain(emu_stream_t* s) {
    while (!s->q.empty()) step_head(s);
}

static void drain_event(emu_event_t* e, uint64_t target, emu_stream_t* where) {
    while (e->completed < target) {
        if (!where || where->q.empty()) die("wait for an event record that is not queued");
        step_head(where);
    }
}

static void drain_all() {
    for (bool any = true; any;) {
        any = false;
        for (emu_stream_t* s : g_streams)
            if (!s->q.empty()) {
                step_head(s);
                any = true;
            }
    }
}

extern "C" void emu_set_execution(int deferred, unsigned long long shuffle_seed) {
    std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
    drain_all();
    g_deferred = deferred != 0;
    g_shuffle_seed = shuffle_seed;
}

void emu_submit(hipStream_t s, std::function<void()> op) {
    std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
    if (!g_deferred) {
        op();
        return;
    }
    stream_of(s)->q.push_back(EmuOp{0, std::move(op), nullptr, 0, nullptr});
}

// Pinned host allocations (hipHostMalloc), which hipPointerGetAttributes reports as host memory
// the device can read; other host memory is pageable unless emu_host_memory_pinned(1) says that
// all of it is (so that tests can route host inputs through either path).
static std::mutex g_pinned_mu;
static std::map<uintptr_t, size_t> g_pinned;
static std::map<uintptr_t, size_t> g_device;   // hipMalloc allocations
static bool g_all_pinned = false;
extern "C" void emu_host_memory_pinned(int on) { g_all_pinned = on != 0; }

static bool in_map(const std::map<uintptr_t, size_t>& m, const void* p) {
    auto it = m.upper_bound((uintptr_t)p);
    if (it == m.begin()) return false;
    --it;
    return (uintptr_t)p < it->first + it->second;
}

// Memory that HIP copies synchronously: host memory that is not pinned.  Anything that is not a
// device or pinned allocation of this emulation counts as host memory, except __device__
// variables, which tests reach only through the library.  (emu_host_memory_pinned changes only
// what hipPointerGetAttributes reports, not how copies of host buffers behave.)
static bool pageable(const void* p) {
    std::lock_guard<std::mutex> lock(g_pinned_mu);
    return !in_map(g_device, p) && !in_map(g_pinned, p);
}

// Failure injection for tests of error handling: once armed with emu_fail_alloc_after(k), the
// device allocation after k more successful ones fails (then the countdown is off again).
static long g_fail_countdown = -1;
static long g_allocs = 0;
static std::vector<size_t> g_alloc_sizes;   // sizes of the device allocations since the reset
extern "C" void emu_fail_alloc_after(long k) { g_fail_countdown = k; }
extern "C" long emu_alloc_count(void) { return g_allocs; }
extern "C" void emu_reset_alloc_log(void) { g_alloc_sizes.clear(); }
// Copies up to cap logged sizes to out; returns how many are logged.
extern "C" size_t emu_alloc_log(size_t* out, size_t cap) {
    for (size_t i = 0; i < g_alloc_sizes.size() && i < cap; ++i) out[i] = g_alloc_sizes[i];
    return g_alloc_sizes.size();
}

hipError_t emu_hipMalloc(void** p, size_t n) {
    if (g_fail_countdown == 0) {
        g_fail_countdown = -1;
        *p = nullptr;
        return hipErrorOutOfMemory;
    }
    if (g_fail_countdown > 0) --g_fail_countdown;
    *p = malloc(n ? n : 1);
    if (!*p) return hipErrorOutOfMemory;
    memset(*p, 0xA5, n);   // device memory starts as garbage
    ++g_allocs;
    g_alloc_sizes.push_back(n);
    std::lock_guard<std::mutex> lock(g_pinned_mu);
    g_device[(uintptr_t)*p] = n ? n : 1;
    return hipSuccess;
}
hipError_t emu_hipFree(void* p) {
    {
        std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
        drain_all();   // hipFree synchronises the device
    }
    {
        std::lock_guard<std::mutex> lock(g_pinned_mu);
        g_device.erase((uintptr_t)p);
    }
    free(p);
    return hipSuccess;
}
hipError_t emu_hipHostMalloc(void** p, size_t n, unsigned) {
    *p = malloc(n ? n : 1);
    if (!*p) return hipErrorOutOfMemory;
    std::lock_guard<std::mutex> lock(g_pinned_mu);
    g_pinned[(uintptr_t)*p] = n ? n : 1;
    return hipSuccess;
}
hipError_t emu_hipPointerGetAttributes(hipPointerAttribute_t* a, const void* p) {
    memset(a, 0, sizeof(*a));
    bool pinned = g_all_pinned, device = false;
    {
        std::lock_guard<std::mutex> lock(g_pinned_mu);
        pinned = pinned || in_map(g_pinned, p);
        device = in_map(g_device, p);
    }
    if (device) {
        a->type = hipMemoryTypeDevice;
        a->devicePointer = const_cast<void*>(p);
        return hipSuccess;
    }
    if (!pinned) return hipErrorInvalidValue;
    a->type = hipMemoryTypeHost;
    a->devicePointer = const_cast<void*>(p);
    a->hostPointer = const_cast<void*>(p);
    return hipSuccess;
}
hipError_t emu_hipHostFree(void* p) {
    {
        std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
        drain_all();   // hipHostFree synchronises the device
    }
    {
        std::lock_guard<std::mutex> lock(g_pinned_mu);
        g_pinned.erase((uintptr_t)p);
    }
    free(p);
    return hipSuccess;
}
hipError_t emu_hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
    std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
    drain(&g_null_stream);
    if (n) memmove(dst, src, n);
    return hipSuccess;
}
// ---- stream capture
struct emu_graph_t {
    std::vector<std::function<void()>> ops;
};
static thread_local emu_graph_t* g_capture = nullptr;
bool emu_capturing() { return g_capture != nullptr; }
void emu_record(std::function<void()> op) { g_capture->ops.push_back(std::move(op)); }
hipError_t emu_hipStreamBeginCapture(hipStream_t, int) {
    if (g_capture) return hipErrorInvalidValue;
    g_capture = new emu_graph_t();
    return hipSuccess;
}
hipError_t emu_hipStreamEndCapture(hipStream_t, hipGraph_t* g) {
    if (!g_capture) return hipErrorInvalidValue;
    *g = g_capture;
    g_capture = nullptr;
    return hipSuccess;
}
hipError_t emu_hipGraphInstantiate(hipGraphExec_t* e, hipGraph_t g, hipGraphNode_t*, char*,
                                   size_t) {
    *e = new emu_graph_t(*g);   // an executable graph is a copy of the recorded ops
    return hipSuccess;
}
hipError_t emu_hipGraphLaunch(hipGraphExec_t e, hipStream_t s) {
    if (g_capture) return hipErrorInvalidValue;
    for (auto& op : e->ops) emu_submit(s, op);
    return hipSuccess;
}
hipError_t emu_hipGraphDestroy(hipGraph_t g) {
    delete g;
    return hipSuccess;
}
hipError_t emu_hipGraphExecDestroy(hipGraphExec_t e) {
    delete e;
    return hipSuccess;
}

// A copy that HIP performs synchronously (pageable host memory on either side) runs now, after
// the work queued before it on its stream; any other copy is queued.
static hipError_t copy_on_stream(bool sync, hipStream_t s, std::function<void()> op) {
    std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
    if (sync && g_deferred) {
        drain(stream_of(s));
        op();
        return hipSuccess;
    }
    emu_submit(s, std::move(op));
    return hipSuccess;
}
hipError_t emu_hipMemcpyAsync(void* dst, const void* src, size_t n, hipMemcpyKind, hipStream_t s) {
    auto op = [=]() {
        if (n) memmove(dst, src, n);
    };
    if (g_capture) {
        emu_record(op);
        return hipSuccess;
    }
    return copy_on_stream(n && (pageable(dst) || pageable(src)), s, op);
}
hipError_t emu_hipMemcpy2DAsync(void* dst, size_t dpitch, const void* src, size_t spitch,
                                size_t width, size_t height, hipMemcpyKind, hipStream_t s) {
    if (width > dpitch || width > spitch) return hipErrorInvalidValue;
    auto op = [=]() {
        for (size_t r = 0; r < height; ++r)
            memmove((char*)dst + r * dpitch, (const char*)src + r * spitch, width);
    };
    if (g_capture) {
        emu_record(op);
        return hipSuccess;
    }
    return copy_on_stream(height && width && (pageable(dst) || pageable(src)), s, op);
}
hipError_t emu_hipMemsetAsync(void* p, int v, size_t n, hipStream_t s) {
    auto op = [=]() { memset(p, v, n); };
    if (g_capture) {
        emu_record(op);
        return hipSuccess;
    }
    emu_submit(s, op);
    return hipSuccess;
}
hipError_t emu_hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
    *s = new emu_stream_t();
    g_streams.insert(*s);
    return hipSuccess;
}
hipError_t emu_hipStreamSynchronize(hipStream_t s) {
    if (g_capture) return hipErrorInvalidValue;   // not allowed while capturing
    std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
    drain(stream_of(s));
    return hipSuccess;
}
hipError_t emu_hipStreamDestroy(hipStream_t s) {
    std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
    drain(s);   // queued work completes before the stream's resources go
    g_streams.erase(s);
    delete s;
    return hipSuccess;
}
hipError_t emu_hipEventCreate(hipEvent_t* e) {
    *e = new emu_event_t();
    return hipSuccess;
}
hipError_t emu_hipEventCreateWithFlags(hipEvent_t* e, unsigned) { return emu_hipEventCreate(e); }
hipError_t emu_hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
    if (g_capture) return hipErrorInvalidValue;
    std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
    if (!g_deferred || e->recorded == 0) return hipSuccess;   // nothing to wait for
    stream_of(s)->q.push_back(EmuOp{2, nullptr, e, e->recorded, e->where});
    return hipSuccess;
}
hipError_t emu_hipEventRecord(hipEvent_t e, hipStream_t s) {
    std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
    const uint64_t seq = ++e->recorded;
    e->where = stream_of(s);
    if (!g_deferred) {
        e->completed = seq;
        e->t = std::chrono::steady_clock::now();
        return hipSuccess;
    }
    e->where->q.push_back(EmuOp{1, nullptr, e, seq, nullptr});
    return hipSuccess;
}
hipError_t emu_hipEventSynchronize(hipEvent_t e) {
    std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
    drain_event(e, e->recorded, e->where);
    return hipSuccess;
}
hipError_t emu_hipEventElapsedTime(float* ms, hipEvent_t a, hipEvent_t b) {
    std::lock_guard<std::recursive_mutex> lock(g_exec_mu);
    if (a->completed < a->recorded || b->completed < b->recorded) return hipErrorInvalidValue;
    *ms = std::chrono::duration<float, std::milli>(b->t - a->t).count();
    return hipSuccess;
}
hipError_t emu_hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t emu_hipGetLastError() {
    hipError_t e = g_last;
    g_last = hipSuccess;
    return e;
}
hipError_t emu_hipGetDevice(int* dev) {
    *dev = 0;
    return hipSuccess;
}
hipError_t emu_hipGetDeviceProperties(hipDeviceProp_t* p, int) {
    snprintf(p->gcnArchName, sizeof(p->gcnArchName), "cpu-emulation");
    return hipSuccess;
}
hipError_t emu_hipGetSymbolAddress(void** p, const void* symbol) {
    *p = const_cast<void*>(symbol);
    return hipSuccess;
}
const char* emu_hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "error"; }
