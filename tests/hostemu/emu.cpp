// Fiber scheduler and checks of the host emulation (see emu.h).
#include "emu.h"
#include "texel.h"

#include <setjmp.h>
#include <stdarg.h>
#include <time.h>
#include <ucontext.h>

#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#include <sanitizer/common_interface_defs.h>
#endif
#endif

EmuDim emu_block_idx, emu_block_dim, emu_grid_dim;

void emu_fail(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    fprintf(stderr, "EMU ERROR: ");
    vfprintf(stderr, fmt, ap);
    fprintf(stderr, "\n");
    va_end(ap);
    fflush(stderr);
    abort();
}

namespace {

constexpr size_t kStack = 512 * 1024;
constexpr int kWave = 64;

enum State { RUNNING, AT_BARRIER, AT_WAVE_OP, DONE };

struct Fiber {
    ucontext_t start;        // entry context (used once per launch of the work item)
    jmp_buf jb;              // where the fiber resumes
    bool started = false;
    char* stack = nullptr;
    EmuDim tid;
    int lin = 0;
    State state = DONE;
    const char* site = nullptr;
    EmuOp op = EMU_BALLOT;
    uint64_t a = 0, b = 0, result = 0;
    int param = 0;
};

std::vector<Fiber*> g_fib;   // (stable addresses: parked fibers keep pointers to themselves)
jmp_buf g_sched;             // the scheduler's resume point
Fiber* g_cur = nullptr;
void (*g_body)(void*) = nullptr;
void* g_ctx = nullptr;
int g_nthreads = 0;
unsigned long long g_barrier_gen = 0;

// Switches use _setjmp / _longjmp (no signal-mask system calls); makecontext
// only sets up each fiber's first entry.

void yield_to_scheduler();

// A fiber is entered once per process and then runs one work item per
// resumption: the body of the current launch, then it parks as DONE.
void fiber_entry() {
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, nullptr, nullptr);
#endif
    for (;;) {
        g_body(g_ctx);
        g_cur->state = DONE;
        yield_to_scheduler();
    }
}

void yield_to_scheduler() {
    Fiber* f = g_cur;
#ifdef EMU_ASAN
    void* fake = nullptr;
    __sanitizer_start_switch_fiber(&fake, nullptr, 0);
#endif
    if (!_setjmp(f->jb)) _longjmp(g_sched, 1);
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
    g_cur = f;
}

void run_fiber(Fiber& f) {
    g_cur = &f;
#ifdef EMU_ASAN
    void* fake = nullptr;
    __sanitizer_start_switch_fiber(&fake, f.stack, kStack);
#endif
    if (!_setjmp(g_sched)) {
        if (!f.started) {
            f.started = true;
            setcontext(&f.start);
        }
        _longjmp(f.jb, 1);
    }
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
}

int src_lane(EmuOp op, int lane, int param) {
    switch (op) {
        case EMU_SHFL_XOR:
            return lane ^ param;
        case EMU_DPP:
            if (param == 0x140) return (lane & ~15) | (15 - (lane & 15));   // row_mirror
            if (param == 0x141) return (lane & ~7) | (7 - (lane & 7));      // row_half_mirror
            if (param < 0x100) return (lane & ~3) | ((param >> (2 * (lane & 3))) & 3);   // quad_perm
            emu_fail("unsupported DPP control 0x%x", param);
        default:
            return lane;
    }
}

// Complete the wave op of wave w if every live lane of it has arrived.
bool try_complete_wave(int w) {
    const int lo = w * kWave, hi = std::min(g_nthreads, lo + kWave);
    int first = -1;
    for (int i = lo; i < hi; ++i) {
        const Fiber& f = *g_fib[i];
        if (f.state == DONE) continue;
        if (f.state != AT_WAVE_OP) return false;
        if (first < 0) first = i;
    }
    if (first < 0) return false;
    const Fiber& f0 = *g_fib[first];
    for (int i = lo; i < hi; ++i) {
        const Fiber& f = *g_fib[i];
        if (f.state == DONE) continue;
        if (f.op != f0.op || strcmp(f.site, f0.site) != 0 || (f.op == EMU_READLANE && f.param != f0.param) ||
            (f.op != EMU_READLANE && f.op != EMU_SHFL_XOR && f.param != f0.param))
            emu_fail("wave %d (block %u): lanes at different cross-lane operations (%s vs %s)", w, emu_block_idx.x,
                     f.site, f0.site);
    }
    auto live = [&](int l) { return l >= 0 && lo + l < hi && g_fib[lo + l]->state != DONE; };
    uint64_t ballot = 0;
    if (f0.op == EMU_BALLOT)
        for (int i = lo; i < hi; ++i)
            if (g_fib[i]->state != DONE && g_fib[i]->a) ballot |= 1ull << (i - lo);
    for (int i = lo; i < hi; ++i) {
        Fiber& f = *g_fib[i];
        if (f.state == DONE) continue;
        const int lane = i - lo;
        switch (f.op) {
            case EMU_BALLOT:
                f.result = ballot;
                break;
            case EMU_READLANE:
                if (!live(f.param)) emu_fail("readlane of lane %d, which is not active (%s)", f.param, f.site);
                f.result = g_fib[lo + f.param]->a;
                break;
            case EMU_SHFL_XOR:
            case EMU_DPP: {
                const int s = src_lane(f.op, lane, f.param);
                if (!live(s)) emu_fail("lane %d reads lane %d, which is not active (%s)", lane, s, f.site);
                f.result = g_fib[lo + s]->a;
                break;
            }
            case EMU_PL16: {
                const int row = lane >> 4;
                uint32_t na, nb;
                if (row & 1) {
                    if (!live(lane - 16)) emu_fail("permlane16 swap with an inactive lane");
                    na = (uint32_t)g_fib[i - 16]->b;
                    nb = (uint32_t)f.b;
                } else {
                    if (!live(lane + 16)) emu_fail("permlane16 swap with an inactive lane");
                    na = (uint32_t)f.a;
                    nb = (uint32_t)g_fib[i + 16]->a;
                }
                f.result = (uint64_t)na | ((uint64_t)nb << 32);
                break;
            }
            case EMU_PL32: {
                uint32_t na, nb;
                if (lane >= 32) {
                    if (!live(lane - 32)) emu_fail("permlane32 swap with an inactive lane");
                    na = (uint32_t)g_fib[i - 32]->b;
                    nb = (uint32_t)f.b;
                } else {
                    if (!live(lane + 32)) emu_fail("permlane32 swap with an inactive lane");
                    na = (uint32_t)f.a;
                    nb = (uint32_t)g_fib[i + 32]->a;
                }
                f.result = (uint64_t)na | ((uint64_t)nb << 32);
                break;
            }
        }
    }
    for (int i = lo; i < hi; ++i)
        if (g_fib[i]->state == AT_WAVE_OP) g_fib[i]->state = RUNNING;
    return true;
}

bool try_complete_barrier() {
    int waiting = 0, live = 0;
    for (int i = 0; i < g_nthreads; ++i) {
        if (g_fib[i]->state == DONE) continue;
        ++live;
        if (g_fib[i]->state == AT_BARRIER) ++waiting;
        else return false;
    }
    if (live == 0 || waiting != live) return false;
    const char* site = nullptr;
    for (int i = 0; i < g_nthreads; ++i)
        if (g_fib[i]->state == AT_BARRIER) {
            if (!site) site = g_fib[i]->site;
            else if (strcmp(site, g_fib[i]->site) != 0)
                emu_fail("work items of block %u wait at different barriers (%s, %s)", emu_block_idx.x, site,
                         g_fib[i]->site);
            g_fib[i]->state = RUNNING;
        }
    ++g_barrier_gen;
    return true;
}

}  // namespace

EmuDim emu_thread_idx() { return g_cur->tid; }

void emu_shutdown() {
    for (Fiber* f : g_fib) {
        free(f->stack);
        delete f;
    }
    g_fib.clear();
}

void emu_syncthreads(const char* site) {
    g_cur->state = AT_BARRIER;
    g_cur->site = site;
    yield_to_scheduler();
}

uint64_t emu_wave_op(EmuOp op, const char* site, uint64_t a, uint64_t b, int param) {
    Fiber* f = g_cur;
    f->state = AT_WAVE_OP;
    f->op = op;
    f->site = site;
    f->a = a;
    f->b = b;
    f->param = param;
    yield_to_scheduler();
    return g_cur->result;
}

void emu_run_grid(dim3 grid, dim3 block, void (*body)(void*), void* ctx) {
    static const bool trace = getenv("VCT_EMU_TRACE") != nullptr;
    struct timespec t0;
    clock_gettime(CLOCK_MONOTONIC, &t0);
    struct Report {
        bool on;
        dim3 g, b;
        timespec t0;
        ~Report() {
            if (!on) return;
            timespec t1;
            clock_gettime(CLOCK_MONOTONIC, &t1);
            fprintf(stderr, "launch %ux%ux%u x %u: %.3f s\n", g.x, g.y, g.z, b.x * b.y * b.z,
                    (t1.tv_sec - t0.tv_sec) + 1e-9 * (t1.tv_nsec - t0.tv_nsec));
        }
    } report{trace, grid, block, t0};
    const int n = (int)(block.x * block.y * block.z);
    if (n <= 0 || n > 1024) emu_fail("workgroup of %d work items", n);
    while ((int)g_fib.size() < n) g_fib.push_back(new Fiber());
    for (int i = 0; i < n; ++i) {
        Fiber& f = *g_fib[i];
        if (f.stack) continue;
        f.stack = static_cast<char*>(malloc(kStack));
        f.started = false;
        getcontext(&f.start);
        f.start.uc_stack.ss_sp = f.stack;
        f.start.uc_stack.ss_size = kStack;
        f.start.uc_link = nullptr;
        makecontext(&f.start, fiber_entry, 0);
    }
    g_body = body;
    g_ctx = ctx;
    g_nthreads = n;
    emu_grid_dim = {grid.x, grid.y, grid.z};
    emu_block_dim = {block.x, block.y, block.z};
    for (unsigned bz = 0; bz < grid.z; ++bz)
        for (unsigned by = 0; by < grid.y; ++by)
            for (unsigned bx = 0; bx < grid.x; ++bx) {
                emu_block_idx = {bx, by, bz};
                for (int i = 0; i < n; ++i) {
                    Fiber& f = *g_fib[i];
                    f.lin = i;
                    f.tid = {(unsigned)i % block.x, ((unsigned)i / block.x) % block.y, (unsigned)i / (block.x * block.y)};
                    f.state = RUNNING;
                }
                for (;;) {
                    bool ran = false, alive = false;
                    for (int i = 0; i < n; ++i) {
                        if (g_fib[i]->state == RUNNING) {
                            run_fiber(*g_fib[i]);
                            ran = true;
                        }
                        if (g_fib[i]->state != DONE) alive = true;
                    }
                    if (!alive) break;
                    bool progress = ran;
                    for (int w = 0; w * kWave < n; ++w) progress |= try_complete_wave(w);
                    progress |= try_complete_barrier();
                    if (!progress) emu_fail("block %u: work items wait on each other (deadlock)", bx);
                }
            }
}

// ---------------------------------------------------------------------------
// memory: registered allocations, index bounds, buffer-resource loads
// ---------------------------------------------------------------------------
namespace {
struct Alloc {
    uintptr_t lo, hi;
    const char* name;
};
std::vector<Alloc> g_allocs;
uint64_t g_texel_limit = ~0ull, g_acc_limit = ~0ull;

void check_span(uintptr_t p, size_t n, const char* what) {
    for (const Alloc& a : g_allocs)
        if (p >= a.lo && p + n <= a.hi) return;
    emu_fail("%s reads %zu bytes at %p, outside every registered allocation", what, n, (void*)p);
}

struct Rsrc {
    uintptr_t base;
    uint32_t stride, records;
};
Rsrc decode(vct_v4i r) {
    Rsrc o;
    o.base = (uintptr_t)((uint64_t)(uint32_t)r.x | ((uint64_t)((uint32_t)r.y & 0xffffu) << 32));
    o.stride = ((uint32_t)r.y >> 16) & 0x3fffu;
    o.records = (uint32_t)r.z;
    return o;
}

// raw (byte-offset) load of n dwords: each dword past the range reads zero
template <int N>
void raw_load(vct_v4i rsrc, uint32_t off, int32_t* out, const char* what) {
    const Rsrc r = decode(rsrc);
    if (r.stride != 0) emu_fail("%s: raw load through a resource with stride %u", what, r.stride);
    if (off >= 0x80000000u) emu_fail("%s: byte offset %u would be negative as a 32-bit offset", what, off);
    for (int d = 0; d < N; ++d) {
        const uint64_t o = (uint64_t)off + 4u * d;
        if (o + 4 > r.records) {
            out[d] = 0;
            continue;
        }
        check_span(r.base + o, 4, what);
        memcpy(&out[d], (const void*)(r.base + o), 4);
    }
}

template <int N>
void struct_load(vct_v4i rsrc, int32_t vindex, int32_t voffset, int32_t* out, const char* what) {
    const Rsrc r = decode(rsrc);
    const uint32_t idx = (uint32_t)vindex;
    if (r.stride == 0) emu_fail("%s: structured load through a resource with stride 0", what);
    if ((uint64_t)idx * r.stride >= (1ull << 32))
        emu_fail("%s: record %u x %u bytes passes the 32-bit byte offset of a structured load", what, idx, r.stride);
    if ((uint32_t)voffset + 4u * N > r.stride) emu_fail("%s: %d dwords at offset %d exceed the record", what, N, voffset);
    if (idx >= r.records) {
        for (int d = 0; d < N; ++d) out[d] = 0;
        return;
    }
    const uintptr_t p = r.base + (uint64_t)idx * r.stride + (uint32_t)voffset;
    check_span(p, 4u * N, what);
    memcpy(out, (const void*)p, 4u * N);
}
}  // namespace

void emu_register(const void* p, size_t n, const char* name) { g_allocs.push_back({(uintptr_t)p, (uintptr_t)p + n, name}); }
void emu_clear_allocations() { g_allocs.clear(); }
void emu_set_limits(uint64_t texels, uint64_t acc) {
    g_texel_limit = texels;
    g_acc_limit = acc;
}

void emu_check_texel(uint64_t idx, const char* site) {
    if (idx >= g_texel_limit) emu_fail("texel index %llu >= %llu (%s)", (unsigned long long)idx,
                                       (unsigned long long)g_texel_limit, site);
}
void emu_check_acc(uint64_t idx, const char* site) {
    if (idx >= g_acc_limit) emu_fail("accumulator texel %llu >= %llu (%s)", (unsigned long long)idx,
                                     (unsigned long long)g_acc_limit, site);
}

vct_v4i vct_raw_load_v4i32(vct_v4i rsrc, int32_t voffset, int32_t soffset, int32_t) {
    vct_v4i v;
    int32_t o[4];
    raw_load<4>(rsrc, (uint32_t)voffset + (uint32_t)soffset, o, "raw dwordx4");
    v.x = o[0], v.y = o[1], v.z = o[2], v.w = o[3];
    return v;
}
vct_v2i vct_raw_load_v2i32(vct_v4i rsrc, int32_t voffset, int32_t soffset, int32_t) {
    vct_v2i v;
    int32_t o[2];
    raw_load<2>(rsrc, (uint32_t)voffset + (uint32_t)soffset, o, "raw dwordx2");
    v.x = o[0], v.y = o[1];
    return v;
}
vct_v4f vct_struct_load_v4f32(vct_v4i rsrc, int32_t vindex, int32_t voffset, int32_t, int32_t) {
    int32_t o[4];
    struct_load<4>(rsrc, vindex, voffset, o, "structured dwordx4");
    vct_v4f v;
    memcpy(&v, o, 16);
    return v;
}
vct_v2i vct_struct_load_v2i32(vct_v4i rsrc, int32_t vindex, int32_t voffset, int32_t, int32_t) {
    int32_t o[2];
    struct_load<2>(rsrc, vindex, voffset, o, "structured dwordx2");
    vct_v2i v;
    v.x = o[0], v.y = o[1];
    return v;
}
vct_v4i vct_scalar_load_v4i32(vct_v4i rsrc, int32_t offset, int32_t) {
    vct_v4i v;
    int32_t o[4];
    raw_load<4>(rsrc, (uint32_t)offset, o, "scalar dwordx4");
    v.x = o[0], v.y = o[1], v.z = o[2], v.w = o[3];
    return v;
}
vct_v2i vct_scalar_load_v2i32(vct_v4i rsrc, int32_t offset, int32_t) {
    vct_v2i v;
    int32_t o[2];
    raw_load<2>(rsrc, (uint32_t)offset, o, "scalar dwordx2");
    v.x = o[0], v.y = o[1];
    return v;
}

// ---------------------------------------------------------------------------
// the few HIP runtime calls the library's host code makes
// ---------------------------------------------------------------------------
extern "C" {
hipError_t hipGetDevice(int* device) {
    *device = 0;
    return hipSuccess;
}
hipError_t hipStreamGetDevice(hipStream_t, hipDevice_t* device) {
    *device = 0;
    return hipSuccess;
}
// (the library's device arrays are host arrays here)
hipError_t hipGetSymbolAddress(void** ptr, const void* symbol) {
    *ptr = const_cast<void*>(symbol);
    return hipSuccess;
}
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipPeekAtLastError(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "emulated"; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
}
