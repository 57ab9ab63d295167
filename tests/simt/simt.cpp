// Fiber scheduler and host-runtime stand-ins of the CPU emulation declared
// in hip/hip_runtime.h (test infrastructure only).  SIMT_CUS sets the
// compute-unit count the library sees (default 256, as on the MI355X).
// Ordinary launches run their workgroups one after another; a cooperative
// launch keeps every workgroup live and switches between them whenever all
// of a workgroup's threads wait (at a wave operation, a barrier, or a
// __builtin_amdgcn_s_sleep, which yields), each workgroup with its own copy
// of the __shared__ variables (poison-filled when it starts).
#include <sys/mman.h>
#include <unistd.h>

#include <algorithm>
#include <map>
#include <random>
#include <vector>

#include "hip/hip_runtime.h"

#if defined(__SANITIZE_ADDRESS__)
#define SIMT_ASAN 1
extern "C" void __sanitizer_start_switch_fiber(void** fake_stack_save, const void* bottom, size_t size);
extern "C" void __sanitizer_finish_switch_fiber(void* fake_stack_save, const void** bottom_old, size_t* size_old);
#else
#define SIMT_ASAN 0
#endif

extern "C" char __start_simt_lds[] __attribute__((weak));
extern "C" char __stop_simt_lds[] __attribute__((weak));

extern "C" void simt_switch(void** save_sp, void* load_sp);
asm(R"(
.text
.globl simt_switch
.type simt_switch,@function
simt_switch:
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
.size simt_switch, .-simt_switch
)");

namespace simt {

enum State { RUN = 0, AT_WAVE = 1, AT_BAR = 2, DONE = 3, YIELD = 4 };

struct Fiber {
    void* sp;
    char* stack;
    size_t stack_size;
    uint3s tid;
    uint3s block;
    int lane, wave, lin;
    int state;
    int op, arg;
    long long val, res;
    void* site;
    void* fake;
};

Fiber* cur = nullptr;
uint3s g_block{0, 0, 0}, g_bdim{1, 1, 1}, g_gdim{1, 1, 1};
static void* g_sched_sp = nullptr;
static void (*g_tramp)(void*) = nullptr;
static void* g_ctx = nullptr;
static std::vector<Fiber> g_f;
static const size_t STACK = 256 * 1024;
static const void* g_sched_bottom = nullptr;
static size_t g_sched_size = 0;
static unsigned long long g_launches = 0;

uint3s& tidx() { return cur->tid; }
int lane_id() { return cur->lane; }

static void die(const char* what) {
    fprintf(stderr, "SIMT ERROR: %s (launch %llu block %u thread %u)\n", what, g_launches, g_block.x,
            cur ? cur->lin : 0u);
    fflush(stderr);
    abort();
}

static void to_sched(bool finished) {
    Fiber* f = cur;
#if SIMT_ASAN
    __sanitizer_start_switch_fiber(finished ? nullptr : &f->fake, g_sched_bottom, g_sched_size);
#endif
    simt_switch(&f->sp, g_sched_sp);
#if SIMT_ASAN
    __sanitizer_finish_switch_fiber(f->fake, &g_sched_bottom, &g_sched_size);
#endif
}

extern "C" void simt_fiber_entry() {
#if SIMT_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &g_sched_bottom, &g_sched_size);
#endif
    g_tramp(g_ctx);
    cur->state = DONE;
    to_sched(true);
    die("finished fiber resumed");
}

long long wave_op(int op, long long v, int arg) {
    Fiber* f = cur;
    f->op = op;
    f->val = v;
    f->arg = arg;
    f->site = __builtin_return_address(0);
    f->state = AT_WAVE;
    to_sched(false);
    return f->res;
}

void sync_block() {
    Fiber* f = cur;
    f->state = AT_BAR;
    f->site = __builtin_return_address(0);
    to_sched(false);
}

void yield() {
    cur->state = YIELD;
    to_sched(false);
}

static void* init_stack(Fiber& f) {
    char* top = f.stack + f.stack_size;
    uintptr_t t = ((uintptr_t)top) & ~(uintptr_t)15;
    void** sp = (void**)(t - 64);
    for (int i = 0; i < 6; ++i) sp[i] = nullptr;
    sp[6] = (void*)&simt_fiber_entry;
    return (void*)sp;
}

static void resume(Fiber& f) {
    cur = &f;
    g_block = f.block;
#if SIMT_ASAN
    void* fake = nullptr;
    __sanitizer_start_switch_fiber(&fake, f.stack, f.stack_size);
#endif
    simt_switch(&g_sched_sp, f.sp);
#if SIMT_ASAN
    __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
#endif
    cur = nullptr;
}

static std::mt19937_64 g_rng(12345);

static void dump_block(Fiber* F, int nf) {
    for (int w = 0; w * 64 < nf; ++w) {
        fprintf(stderr, " wave %d:", w);
        for (int l = 0; l < 64 && w * 64 + l < nf; ++l) {
            Fiber& f = F[w * 64 + l];
            fprintf(stderr, " %d/%d/%p", f.state, f.op, f.site);
        }
        fprintf(stderr, "\n");
    }
}

static void ensure_fibers(size_t count) {
    if (g_f.size() >= count) return;
    size_t old = g_f.size();
    g_f.resize(count);
    for (size_t i = old; i < g_f.size(); ++i) {
        void* p = mmap(nullptr, STACK, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
        if (p == MAP_FAILED) die("mmap stack");
        g_f[i].stack = (char*)p;
        g_f[i].stack_size = STACK;
    }
}

static void init_block(Fiber* F, int nf, uint3s block) {
    for (int i = 0; i < nf; ++i) {
        Fiber& f = F[i];
        f.sp = init_stack(f);
        f.state = RUN;
        f.lin = i;
        f.tid = uint3s{(unsigned)(i % g_bdim.x), (unsigned)((i / g_bdim.x) % g_bdim.y),
                       (unsigned)(i / (g_bdim.x * g_bdim.y))};
        f.block = block;
        f.lane = i & 63;
        f.wave = i >> 6;
    }
}

// Resolve the wave operations and barriers the workgroup's threads wait at.
// Returns true if some thread was released.
static bool release(Fiber* F, int nf) {
    const int nw = (nf + 63) / 64;
    bool prog = false;
    for (int w = 0; w < nw; ++w) {
        const int b = w * 64, e = std::min(nf, b + 64);
        int live = 0, atw = 0;
        Fiber* first = nullptr;
        for (int i = b; i < e; ++i) {
            if (F[i].state == DONE) continue;
            ++live;
            if (F[i].state == AT_WAVE) {
                ++atw;
                if (!first) first = &F[i];
            }
        }
        if (!live || atw != live) continue;
        for (int i = b; i < e; ++i) {
            Fiber& f = F[i];
            if (f.state == DONE) continue;
            if (f.op != first->op || f.site != first->site) {
                cur = &f;
                fprintf(stderr, "divergent wave ops: op %d site %p vs op %d site %p\n", f.op, f.site, first->op,
                        first->site);
                dump_block(F, nf);
                die("divergent wave op");
            }
        }
        const int op = first->op;
        unsigned long long mask = 0;
        long long vals[64];
        for (int i = b; i < e; ++i) {
            vals[i - b] = F[i].val;
            if (F[i].state != DONE && op == OP_BALLOT && F[i].val) mask |= 1ull << (i - b);
        }
        for (int i = b; i < e; ++i) {
            Fiber& f = F[i];
            if (f.state == DONE) continue;
            const int l = i - b;
            int src = l;
            switch (op) {
                case OP_SHFL: src = ((f.arg % 64) + 64) % 64; break;
                case OP_SHFL_UP: src = l >= f.arg ? l - f.arg : l; break;
                case OP_SHFL_DOWN: src = l + f.arg < 64 ? l + f.arg : l; break;
                case OP_SHFL_XOR: src = (l ^ f.arg) & 63; break;
                default: break;
            }
            if (op != OP_BALLOT && op != OP_WBAR && (b + src >= e || F[b + src].state == DONE)) {
                cur = &f;
                fprintf(stderr, "shuffle reads lane %d (inactive) from lane %d op %d\n", src, l, op);
                die("shuffle from an inactive lane");
            }
            if (op == OP_BALLOT) f.res = (long long)mask;
            else if (op == OP_WBAR) f.res = 0;
            else f.res = vals[src];
            f.state = RUN;
        }
        prog = true;
    }
    if (prog) return true;
    int atb = 0, live = 0;
    void* site = nullptr;
    bool same = true;
    for (int i = 0; i < nf; ++i) {
        if (F[i].state == DONE) continue;
        ++live;
        if (F[i].state == AT_BAR) {
            ++atb;
            if (!site) site = F[i].site;
            else if (site != F[i].site) same = false;
        }
    }
    if (live && atb == live && same) {
        for (int i = 0; i < nf; ++i)
            if (F[i].state == AT_BAR) F[i].state = RUN;
        return true;
    }
    return false;
}

// Run a workgroup's threads until every one has finished or waits.  Returns
// true when all have finished.  A thread that yields waits for the next turn
// (coop) or runs again at once (otherwise).
static bool run_block(Fiber* F, int nf, bool coop) {
    for (;;) {
        for (int i = 0; i < nf; ++i) {
            while (F[i].state == RUN) resume(F[i]);
            if (!coop && F[i].state == YIELD) F[i].state = RUN, --i;
        }
        int ndone = 0, nyield = 0;
        for (int i = 0; i < nf; ++i) {
            ndone += F[i].state == DONE;
            nyield += F[i].state == YIELD;
        }
        if (ndone == nf) return true;
        if (release(F, nf)) continue;
        if (coop && nyield) return false;
        fprintf(stderr, "deadlock in a workgroup\n");
        dump_block(F, nf);
        die("deadlock");
    }
}

static size_t lds_bytes() { return (__start_simt_lds && __stop_simt_lds) ? (size_t)(__stop_simt_lds - __start_simt_lds) : 0; }

__attribute__((no_sanitize_address)) static void lds_copy(char* dst, const char* src, size_t n) {
    for (size_t i = 0; i < n; ++i) dst[i] = src[i];
}

void run_launch(dim3 g, dim3 b, void (*tramp)(void*), void* ctx, bool coop) {
    const int nf = (int)(b.x * b.y * b.z);
    if (nf <= 0 || nf > 1024) die("bad block size");
    ++g_launches;
    g_tramp = tramp;
    g_ctx = ctx;
    g_bdim = uint3s{b.x, b.y, b.z};
    g_gdim = uint3s{g.x, g.y, g.z};
    const unsigned nb = g.x * g.y * g.z;
    auto bidx = [&](unsigned i) { return uint3s{i % g.x, (i / g.x) % g.y, i / (g.x * g.y)}; };
    if (!coop) {
        ensure_fibers((size_t)nf);
        std::vector<unsigned> order(nb);
        for (unsigned i = 0; i < nb; ++i) order[i] = i;
        if (getenv("SIMT_SHUFFLE")) std::shuffle(order.begin(), order.end(), g_rng);
        for (unsigned kk = 0; kk < nb; ++kk) {
            init_block(g_f.data(), nf, bidx(order[kk]));
            run_block(g_f.data(), nf, false);
        }
        return;
    }
    // cooperative: every workgroup live, each with its own __shared__ copy
    ensure_fibers((size_t)nf * nb);
    const size_t L = lds_bytes();
    std::vector<char> lds((size_t)nb * L, (char)0xA5);
    std::vector<char> done(nb, 0);
    for (unsigned i = 0; i < nb; ++i) init_block(g_f.data() + (size_t)i * nf, nf, bidx(i));
    for (unsigned left = nb; left > 0;) {
        for (unsigned i = 0; i < nb; ++i) {
            if (done[i]) continue;
            Fiber* F = g_f.data() + (size_t)i * nf;
            for (int t = 0; t < nf; ++t)
                if (F[t].state == YIELD) F[t].state = RUN;
            lds_copy(__start_simt_lds, lds.data() + (size_t)i * L, L);
            const bool fin = run_block(F, nf, true);
            lds_copy(lds.data() + (size_t)i * L, __start_simt_lds, L);
            if (fin) {
                done[i] = 1;
                --left;
            }
        }
    }
}

}  // namespace simt

// "device" memory: poison-filled, ends at a guard page
struct Alloc {
    void* base;
    size_t len;
};
static std::map<void*, Alloc> g_allocs;

hipError_t simt_malloc(void** p, size_t bytes) {
    static long pg = sysconf(_SC_PAGESIZE);
    if (bytes == 0) bytes = 1;
    size_t body = (bytes + 255) & ~(size_t)255;   // keep 256-byte alignment of the start
    size_t len = ((body + pg - 1) / pg) * pg + pg;
    char* base = (char*)mmap(nullptr, len, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (base == MAP_FAILED) return hipErrorOutOfMemory;
    mprotect(base + len - pg, pg, PROT_NONE);
    char* user = base + len - pg - body;
    memset(user, getenv("SIMT_ZERO") ? 0 : 0xA5, body);
    g_allocs[user] = Alloc{base, len};
    *p = user;
    return hipSuccess;
}

hipError_t hipFree(void* p) {
    auto it = g_allocs.find(p);
    if (it == g_allocs.end()) return p ? hipErrorInvalidValue : hipSuccess;
    munmap(it->second.base, it->second.len);
    g_allocs.erase(it);
    return hipSuccess;
}

hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
    memset(p, 0, sizeof(*p));
    const char* c = getenv("SIMT_CUS");
    p->multiProcessorCount = c ? atoi(c) : 256;
    p->maxThreadsPerBlock = 1024;
    p->sharedMemPerBlock = 160 * 1024;
    strcpy(p->gcnArchName, "gfx950:sramecc+:xnack-");
    strcpy(p->name, "simt");
    return hipSuccess;
}

extern "C" void* simt_alloc(size_t bytes) {
    void* p = nullptr;
    simt_malloc(&p, bytes);
    return p;
}
extern "C" void simt_free(void* p) { hipFree(p); }
