// hostemu.cpp -- the CPU stand-in of the HIP runtime declared in
// hip/hip_runtime.h: blocks run one after another, the threads of a block
// are ucontext fibers on the calling OS thread, switched at barriers only.
#include "hip/hip_runtime.h"

#include <ucontext.h>

#include <cstdlib>
#include <vector>

namespace hipemu {

enum State { RUN, AT_BLOCK, AT_WAVE, DONE };

struct Fiber {
    ucontext_t ctx;
    State state = RUN;
    uint3 tid{0, 0, 0};
    int lane = 0, wave = 0;
};

static ucontext_t g_sched;
static std::vector<Fiber> g_fib;
static std::vector<char *> g_stacks;
static Fiber *g_cur = nullptr;
static uint3 g_bid{0, 0, 0};
static dim3 g_bdim, g_gdim;
static void (*g_fn)(void *) = nullptr;
static void *g_arg = nullptr;
static uint64_t g_slot[1024];
static constexpr size_t STACK = 512 * 1024;

Fiber *current() { return g_cur; }
const uint3 &thread_idx() { return g_cur->tid; }
const uint3 &block_idx() { return g_bid; }
const dim3 &block_dim() { return g_bdim; }
const dim3 &grid_dim() { return g_gdim; }
int lane_id() { return g_cur->lane; }

static void yield_as(State s)
{
    g_cur->state = s;
    swapcontext(&g_cur->ctx, &g_sched);
}

void block_barrier() { yield_as(AT_BLOCK); }

static void wave_barrier() { yield_as(AT_WAVE); }

uint64_t wave_exchange(uint64_t mine, int src)
{
    const int base = g_cur->wave * 64;
    g_slot[base + g_cur->lane] = mine;
    wave_barrier();
    const int n = (int)g_bdim.x;
    const uint64_t v = (src >= 0 && src < 64 && base + src < n) ? g_slot[base + src] : mine;
    wave_barrier();
    return v;
}

uint64_t wave_ballot(bool pred)
{
    const int base = g_cur->wave * 64;
    g_slot[base + g_cur->lane] = pred ? 1u : 0u;
    wave_barrier();
    uint64_t m = 0;
    const int n = (int)g_bdim.x;
    for (int l = 0; l < 64 && base + l < n; ++l)
        if (g_fib[base + l].state != DONE && g_slot[base + l]) m |= 1ull << l;
    wave_barrier();
    return m;
}

// all 64 lanes' values (lanes that exited read as 0)
static void wave_gather(uint64_t mine, uint64_t out[64])
{
    const int base = g_cur->wave * 64;
    g_slot[base + g_cur->lane] = mine;
    wave_barrier();
    const int n = (int)g_bdim.x;
    for (int l = 0; l < 64; ++l)
        out[l] = (base + l < n && g_fib[base + l].state != DONE) ? g_slot[base + l] : 0;
    wave_barrier();
}

static void fiber_main(int k)
{
    g_fn(g_arg);
    g_fib[k].state = DONE;
    swapcontext(&g_fib[k].ctx, &g_sched);
}

static void trampoline(unsigned lo, unsigned hi)
{
    (void)hi;
    fiber_main((int)lo);
}

void run_launch(dim3 grid, dim3 block, void (*fn)(void *), void *arg)
{
    if (block.y != 1 || block.z != 1 || grid.y != 1 || grid.z != 1 || block.x == 0 || block.x > 1024) {
        fprintf(stderr, "hostemu: only 1-D launches of up to 1024 threads\n");
        abort();
    }
    const int nt = (int)block.x;
    g_fn = fn;
    g_arg = arg;
    g_bdim = block;
    g_gdim = grid;
    if ((int)g_stacks.size() < nt) {
        for (int k = (int)g_stacks.size(); k < nt; ++k) g_stacks.push_back((char *)malloc(STACK));
    }
    g_fib.assign(nt, Fiber());
    for (unsigned b = 0; b < grid.x; ++b) {
        g_bid = uint3{b, 0, 0};
        for (int k = 0; k < nt; ++k) {
            Fiber &f = g_fib[k];
            f.state = RUN;
            f.tid = uint3{(unsigned)k, 0, 0};
            f.lane = k % 64;
            f.wave = k / 64;
            getcontext(&f.ctx);
            f.ctx.uc_stack.ss_sp = g_stacks[k];
            f.ctx.uc_stack.ss_size = STACK;
            f.ctx.uc_link = nullptr;
            makecontext(&f.ctx, (void (*)())trampoline, 2, (unsigned)k, 0u);
        }
        for (;;) {
            // run every runnable fiber until it waits or ends
            for (int k = 0; k < nt; ++k) {
                if (g_fib[k].state != RUN) continue;
                g_cur = &g_fib[k];
                swapcontext(&g_sched, &g_fib[k].ctx);
            }
            g_cur = nullptr;
            // release wavefront barriers whose live lanes all arrived
            bool progress = false, any_live = false;
            const int nw = (nt + 63) / 64;
            for (int w = 0; w < nw; ++w) {
                int live = 0, at_wave = 0, at_block = 0;
                for (int k = w * 64; k < nt && k < w * 64 + 64; ++k) {
                    const State s = g_fib[k].state;
                    if (s == DONE) continue;
                    ++live;
                    at_wave += s == AT_WAVE;
                    at_block += s == AT_BLOCK;
                }
                any_live |= live > 0;
                if (at_wave && at_wave != live) {
                    fprintf(stderr, "hostemu: block %u wavefront %d: %d lanes at a wavefront operation, %d "
                                    "at a block barrier (divergent wavefront operation)\n",
                            b, w, at_wave, at_block);
                    abort();
                }
                if (at_wave) {
                    for (int k = w * 64; k < nt && k < w * 64 + 64; ++k)
                        if (g_fib[k].state == AT_WAVE) g_fib[k].state = RUN;
                    progress = true;
                }
            }
            if (progress) continue;
            if (!any_live) break;
            // every live fiber waits at the block barrier: release them
            for (int k = 0; k < nt; ++k)
                if (g_fib[k].state == AT_BLOCK) g_fib[k].state = RUN;
        }
    }
}

}  // namespace hipemu

// BF16 matrix-core product of one 16x16x16 tile: lane l = r + 16 q holds
// A[r][4q..4q+3], B[4q..4q+3][r] and C[4q..4q+3][r]
hipemu_v4f hipemu_mfma_16x16x16_bf16(hipemu_v4s a, hipemu_v4s b, hipemu_v4f c)
{
    uint64_t A[64], B[64];
    uint64_t ma, mb;
    memcpy(&ma, &a, 8);
    memcpy(&mb, &b, 8);
    hipemu::wave_gather(ma, A);
    hipemu::wave_gather(mb, B);
    auto bf = [](uint64_t w, int j) {
        const uint32_t u = (uint32_t)((w >> (16 * j)) & 0xffffu) << 16;
        float f;
        memcpy(&f, &u, 4);
        return f;
    };
    const int l = hipemu::lane_id(), r = l & 15, q = l >> 4;
    hipemu_v4f out = c;
    for (int j = 0; j < 4; ++j) {
        const int m = 4 * q + j;
        float s = 0.f;
        for (int k = 0; k < 16; ++k) s += bf(A[m + 16 * (k / 4)], k % 4) * bf(B[r + 16 * (k / 4)], k % 4);
        out[j] += s;
    }
    return out;
}

// ---------------------------------------------------------------- runtime
static hipError_t g_last = hipSuccess;

hipError_t hipMalloc(void **p, size_t n)
{
    *p = aligned_alloc(256, (n + 255) & ~(size_t)255);
    if (*p) memset(*p, getenv("HIPEMU_ZERO") ? 0 : 0xff, n);
    return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p)
{
    free(p);
    return hipSuccess;
}
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind)
{
    memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t)
{
    memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t)
{
    memset(d, v, n);
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipGetLastError()
{
    hipError_t e = g_last;
    g_last = hipSuccess;
    return e;
}
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "hostemu error"; }
struct hipemu_event {
    int dummy;
};
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = new hipemu_event{0};
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t)
{
    *ms = 0.f;
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **p, const void *sym)
{
    *p = (void *)sym;
    return hipSuccess;
}

extern "C" void *hipemu_alloc(size_t n)
{
    void *p = nullptr;
    hipMalloc(&p, n);
    // fresh device memory holds arbitrary bytes: fill with a pattern that
    // reads as NaN (doubles, floats) and -1 (integers)
    if (p) memset(p, getenv("HIPEMU_ZERO") ? 0 : 0xff, n);
    return p;
}
extern "C" void hipemu_free(void *p) { free(p); }
