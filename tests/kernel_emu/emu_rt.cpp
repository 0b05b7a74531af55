// Runtime of the host kernel emulation: fibers for GPU threads (a minimal
// x86-64 stack switch) with block and wavefront barriers, the raw buffer
// loads/stores of the step kernels (descriptor base + offsets, checked
// against the descriptor's range), and the HIP host API on host memory.
// Graph capture reports "not supported"; callers run with graphs off.
#include <sanitizer/common_interface_defs.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <string>
#include <vector>

#include "hip/hip_runtime.h"

namespace {

constexpr size_t kStack = 256 * 1024;

extern "C" void emu_swap(void **save_sp, void *new_sp);
asm(R"(
.text
.globl emu_swap
.type emu_swap,@function
emu_swap:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
)");

struct Fiber {
    void *sp = nullptr;
    EmuCtx ctx;
    bool done = false;
    int wait = 0;          // 0 none, 1 block barrier, 2 wave barrier
    uint64_t wait_gen = 0;
    char *stack = nullptr;
};

struct Block {
    std::vector<Fiber> f;
    int live = 0;
    int arrived = 0;
    uint64_t gen = 0;
    int wlive[64] = {}, warrived[64] = {};
    uint64_t wgen[64] = {};
    double xchg[64][64];
};

void *g_sched_sp = nullptr;
Fiber *g_cur = nullptr;
Block *g_blk = nullptr;
void (*g_entry)(void *) = nullptr;
void *g_arg = nullptr;
std::vector<char *> g_stacks;
std::vector<char> g_dyn;
void *g_fake_stack = nullptr;
const void *g_sched_bottom = nullptr;
size_t g_sched_size = 0;
std::map<std::string, long> g_launches;

void to_sched()
{
    __sanitizer_start_switch_fiber(&g_fake_stack, g_sched_bottom, g_sched_size);
    emu_swap(&g_cur->sp, g_sched_sp);
    __sanitizer_finish_switch_fiber(g_fake_stack, nullptr, nullptr);
}

void trampoline()
{
    // entered by the first switch into this fiber
    __sanitizer_finish_switch_fiber(nullptr, &g_sched_bottom, &g_sched_size);
    g_entry(g_arg);
    Fiber *me = g_cur;
    me->done = true;
    Block &b = *g_blk;
    b.live--;
    const int w = int(me->ctx.tid.x / 64);
    b.wlive[w]--;
    if (b.live > 0 && b.arrived == b.live) {
        b.arrived = 0;
        b.gen++;
    }
    if (b.wlive[w] > 0 && b.warrived[w] == b.wlive[w]) {
        b.warrived[w] = 0;
        b.wgen[w]++;
    }
    __sanitizer_start_switch_fiber(nullptr, g_sched_bottom, g_sched_size);
    void *dead = nullptr;
    emu_swap(&dead, g_sched_sp);
    __builtin_trap();
}

}  // namespace

EmuCtx *emu_ctx() { return &g_cur->ctx; }

bool g_direct = false;   // threads run to completion on the scheduler's stack

void emu_syncthreads()
{
    if (g_direct) {
        std::fprintf(stderr, "emu: barrier in a block whose thread 0 finished without one\n");
        std::abort();
    }
    Block &b = *g_blk;
    g_cur->wait = 1;
    g_cur->wait_gen = b.gen;
    if (++b.arrived == b.live) {
        b.arrived = 0;
        b.gen++;
    }
    while (b.gen == g_cur->wait_gen) to_sched();
    g_cur->wait = 0;
}

void emu_wave_barrier()
{
    if (g_direct) {
        std::fprintf(stderr, "emu: wave barrier in a block whose thread 0 finished without one\n");
        std::abort();
    }
    Block &b = *g_blk;
    const int w = int(g_cur->ctx.tid.x / 64);
    g_cur->wait = 2;
    g_cur->wait_gen = b.wgen[w];
    if (++b.warrived[w] == b.wlive[w]) {
        b.warrived[w] = 0;
        b.wgen[w]++;
    }
    while (b.wgen[w] == g_cur->wait_gen) to_sched();
    g_cur->wait = 0;
}

void *emu_wave_xchg() { return g_blk->xchg[g_cur->ctx.tid.x / 64]; }
void *emu_dyn_shared() { return g_dyn.data(); }

void emu_run_grid(void (*entry)(void *), void *arg, dim3 g, dim3 bd, size_t shmem, const char *name)
{
    g_launches[name]++;
    const int nt = int(bd.x * bd.y * bd.z);
    if (nt > 1024 || bd.y != 1 || bd.z != 1) {
        std::fprintf(stderr, "emu: unsupported block shape\n");
        std::abort();
    }
    while (int(g_stacks.size()) < nt) g_stacks.push_back(static_cast<char *>(std::malloc(kStack)));
    g_entry = entry;
    g_arg = arg;
    Block blk;
    blk.f.resize(size_t(nt));
    g_blk = &blk;
    for (unsigned bz = 0; bz < g.z; ++bz)
        for (unsigned by = 0; by < g.y; ++by)
            for (unsigned bx = 0; bx < g.x; ++bx) {
                g_dyn.assign(shmem, 0);
                blk.live = nt;
                blk.arrived = 0;
                blk.gen = 0;
                for (int w = 0; w < 64; ++w) {
                    blk.wlive[w] = std::max(0, std::min(64, nt - 64 * w));
                    blk.warrived[w] = 0;
                    blk.wgen[w] = 0;
                }
                for (int t = 0; t < nt; ++t) {
                    Fiber &f = blk.f[size_t(t)];
                    f.done = false;
                    f.wait = 0;
                    f.ctx.tid = emu_u3{unsigned(t), 0, 0};
                    f.ctx.bid = emu_u3{bx, by, bz};
                    f.ctx.bdim = bd;
                    f.ctx.gdim = g;
                    f.stack = g_stacks[size_t(t)];
                    // initial frame: six callee-saved registers, then the
                    // trampoline as the return address of the first switch
                    uintptr_t top = (reinterpret_cast<uintptr_t>(f.stack) + kStack) & ~uintptr_t(15);
                    void **sp = reinterpret_cast<void **>(top - 8);
                    *--sp = reinterpret_cast<void *>(&trampoline);
                    for (int r = 0; r < 6; ++r) *--sp = nullptr;
                    f.sp = sp;
                }
                int remaining = nt;
                // thread 0 first: if it ends without reaching a barrier, no
                // thread of the block does (barriers are block-uniform), and
                // the others run as plain calls
                {
                    Fiber &f = blk.f[0];
                    g_cur = &f;
                    void *fs = nullptr;
                    __sanitizer_start_switch_fiber(&fs, f.stack, kStack);
                    emu_swap(&g_sched_sp, f.sp);
                    __sanitizer_finish_switch_fiber(fs, nullptr, nullptr);
                    if (f.done) {
                        --remaining;
                        g_direct = true;
                        for (int t = 1; t < nt; ++t) {
                            g_cur = &blk.f[size_t(t)];
                            g_entry(g_arg);
                            blk.f[size_t(t)].done = true;
                            --remaining;
                        }
                        g_direct = false;
                    }
                }
                while (remaining > 0) {
                    bool progress = false;
                    for (int t = 0; t < nt; ++t) {
                        Fiber &f = blk.f[size_t(t)];
                        if (f.done) continue;
                        if (f.wait == 1 && blk.gen == f.wait_gen) continue;
                        if (f.wait == 2 && blk.wgen[t / 64] == f.wait_gen) continue;
                        g_cur = &f;
                        void *fs = nullptr;
                        __sanitizer_start_switch_fiber(&fs, f.stack, kStack);
                        emu_swap(&g_sched_sp, f.sp);
                        __sanitizer_finish_switch_fiber(fs, nullptr, nullptr);
                        progress = true;
                        if (f.done) --remaining;
                    }
                    if (!progress) {
                        std::fprintf(stderr, "emu: barrier deadlock in %s block (%u,%u,%u)\n", name, bx, by, bz);
                        std::abort();
                    }
                }
            }
    g_blk = nullptr;
    g_cur = nullptr;
}

void emu_print_launches()
{
    for (auto &kv : g_launches) std::printf("  %8ld  %s\n", kv.second, kv.first.c_str());
}

// ---- raw buffer access ------------------------------------------------------
typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

static char *emu_buf_addr(i32x4 r, int voff, int soff, size_t bytes)
{
    const uint64_t base = (uint64_t(uint32_t(r.y) & 0xffffu) << 32) | uint64_t(uint32_t(r.x));
    const uint64_t off = uint64_t(uint32_t(voff)) + uint64_t(uint32_t(soff));
    if (off + bytes > uint64_t(uint32_t(r.z))) {
        std::fprintf(stderr, "emu: raw buffer access past num_records (voff %d soff %d)\n", voff, soff);
        std::abort();
    }
    return reinterpret_cast<char *>(base + off);
}

// a raw-buffer access whose lane offset lies at or past the descriptor's
// range touches no memory: a load returns zeros, a store is dropped (the
// hardware's range check)
static bool emu_buf_oob(i32x4 r, int voff, size_t bytes)
{
    return uint64_t(uint32_t(voff)) + bytes > uint64_t(uint32_t(r.z));
}

float emu_raw_ld_f32(i32x4 r, int voff, int soff, int aux) __asm("emu_raw_ld_f32");
f32x2 emu_raw_ld_v2f32(i32x4 r, int voff, int soff, int aux) __asm("emu_raw_ld_v2f32");
f32x4 emu_raw_ld_v4f32(i32x4 r, int voff, int soff, int aux) __asm("emu_raw_ld_v4f32");
void emu_raw_st_f32(float v, i32x4 r, int voff, int soff, int aux) __asm("emu_raw_st_f32");
void emu_raw_st_v2f32(f32x2 v, i32x4 r, int voff, int soff, int aux) __asm("emu_raw_st_v2f32");

float emu_raw_ld_f32(i32x4 r, int voff, int soff, int aux)
{
    float v = 0.f;
    if (emu_buf_oob(r, voff, 4)) return v;
    std::memcpy(&v, emu_buf_addr(r, voff, soff, 4), 4);
    return v;
}
f32x2 emu_raw_ld_v2f32(i32x4 r, int voff, int soff, int aux)
{
    f32x2 v = f32x2{0.f, 0.f};
    if (emu_buf_oob(r, voff, 8)) return v;
    std::memcpy(&v, emu_buf_addr(r, voff, soff, 8), 8);
    return v;
}
f32x4 emu_raw_ld_v4f32(i32x4 r, int voff, int soff, int aux)
{
    f32x4 v = f32x4{0.f, 0.f, 0.f, 0.f};
    if (emu_buf_oob(r, voff, 16)) return v;
    std::memcpy(&v, emu_buf_addr(r, voff, soff, 16), 16);
    return v;
}
void emu_raw_st_f32(float v, i32x4 r, int voff, int soff, int aux)
{
    if (emu_buf_oob(r, voff, 4)) return;   // dropped, as the hardware drops it
    std::memcpy(emu_buf_addr(r, voff, soff, 4), &v, 4);
}
void emu_raw_st_v2f32(f32x2 v, i32x4 r, int voff, int soff, int aux)
{
    if (emu_buf_oob(r, voff, 8)) return;
    std::memcpy(emu_buf_addr(r, voff, soff, 8), &v, 8);
}

// ---- host API -----------------------------------------------------------------
struct EmuStream {
    int dummy;
};
struct EmuEvent {
    int dummy;
};
struct EmuGraph {
    int dummy;
};
struct EmuGraphExec {
    int dummy;
};

const char *hipGetErrorString(hipError_t e) { return e ? "emulated error" : "no error"; }
hipError_t hipGetLastError() { return hipSuccess; }
hipError_t hipGetDeviceCount(int *n)
{
    *n = 1;
    return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipMemGetInfo(size_t *fr, size_t *tot)
{
    *tot = size_t(288) << 30;
    *fr = size_t(280) << 30;
    return hipSuccess;
}
hipError_t hipMalloc(void **p, size_t n)
{
    *p = std::malloc(n);
    if (!*p) return hipErrorOutOfMemory;
    std::memset(*p, 0xff, n);   // NaN pattern: nothing may rely on fresh memory
    return hipSuccess;
}
hipError_t hipFree(void *p)
{
    std::free(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
hipError_t hipHostFree(void *p) { return hipFree(p); }
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t n, hipMemcpyKind, hipStream_t)
{
    std::memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void *dst, int v, size_t n, hipStream_t)
{
    std::memset(dst, v, n);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned)
{
    *s = new EmuStream{};
    return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s)
{
    delete s;
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = new EmuEvent{};
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t)
{
    *ms = 1.0f;
    return hipSuccess;
}
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipErrorNotSupported; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *) { return hipErrorNotSupported; }
hipError_t hipGraphGetNodes(hipGraph_t, hipGraphNode_t *, size_t *) { return hipErrorNotSupported; }
hipError_t hipGraphInstantiate(hipGraphExec_t *, hipGraph_t, hipGraphNode_t *, char *, size_t)
{
    return hipErrorNotSupported;
}
hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
