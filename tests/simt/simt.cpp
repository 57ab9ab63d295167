// Fiber scheduler and host-runtime stand-ins of the CPU emulation declared
// in hip/hip_runtime.h (test infrastructure only).  SIMT_CUS sets the
// compute-unit count the library sees (default 256, as on the MI355X).
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

enum State { RUN = 0, AT_WAVE = 1, AT_BAR = 2, DONE = 3 };

struct Fiber {
    void* sp;
    char* stack;
    size_t stack_size;
    uint3s tid;
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
static const size_t STACK = 512 * 1024;
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

static void dump_block(int nf) {
    for (int w = 0; w * 64 < nf; ++w) {
        fprintf(stderr, " wave %d:", w);
        for (int l = 0; l < 64 && w * 64 + l < nf; ++l) {
            Fiber& f = g_f[w * 64 + l];
            fprintf(stderr, " %d/%d/%p", f.state, f.op, f.site);
        }
        fprintf(stderr, "\n");
    }
}

static void run_block(int nf) {
    for (int i = 0; i < nf; ++i) {
        Fiber& f = g_f[i];
        f.sp = init_stack(f);
        f.state = RUN;
        f.lin = i;
        f.tid = uint3s{(unsigned)(i % g_bdim.x), (unsigned)((i / g_bdim.x) % g_bdim.y),
                       (unsigned)(i / (g_bdim.x * g_bdim.y))};
        f.lane = i & 63;
        f.wave = i >> 6;
    }
    const int nw = (nf + 63) / 64;
    for (;;) {
        for (int i = 0; i < nf; ++i)
            while (g_f[i].state == RUN) resume(g_f[i]);
        int ndone = 0;
        for (int i = 0; i < nf; ++i) ndone += g_f[i].state == DONE;
        if (ndone == nf) return;
        bool prog = false;
        for (int w = 0; w < nw; ++w) {
            const int b = w * 64, e = std::min(nf, b + 64);
            int live = 0, atw = 0;
            Fiber* first = nullptr;
            for (int i = b; i < e; ++i) {
                if (g_f[i].state == DONE) continue;
                ++live;
                if (g_f[i].state == AT_WAVE) {
                    ++atw;
                    if (!first) first = &g_f[i];
                }
            }
            if (!live || atw != live) continue;
            // every live lane waits at a wave op: they must be at the same one
            for (int i = b; i < e; ++i) {
                Fiber& f = g_f[i];
                if (f.state == DONE) continue;
                if (f.op != first->op || f.site != first->site) {
                    cur = &f;
                    fprintf(stderr, "divergent wave ops: op %d site %p vs op %d site %p\n", f.op, f.site, first->op,
                            first->site);
                    dump_block(nf);
                    die("divergent wave op");
                }
            }
            const int op = first->op;
            unsigned long long mask = 0;
            for (int i = b; i < e; ++i)
                if (g_f[i].state != DONE && op == OP_BALLOT && g_f[i].val) mask |= 1ull << (i - b);
            for (int i = b; i < e; ++i) {
                Fiber& f = g_f[i];
                if (f.state == DONE) continue;
                const int l = i - b;
                int src = l;
                switch (op) {
                    case OP_BALLOT: f.res = (long long)mask; break;
                    case OP_WBAR: f.res = 0; break;
                    case OP_SHFL: src = ((f.arg % 64) + 64) % 64; break;
                    case OP_SHFL_UP: src = l >= f.arg ? l - f.arg : l; break;
                    case OP_SHFL_DOWN: src = l + f.arg < 64 ? l + f.arg : l; break;
                    case OP_SHFL_XOR: src = (l ^ f.arg) & 63; break;
                }
                if (op != OP_BALLOT && op != OP_WBAR) {
                    if (b + src >= e || g_f[b + src].state == DONE) {
                        cur = &f;
                        fprintf(stderr, "shuffle reads lane %d (inactive) from lane %d op %d\n", src, l, op);
                        die("shuffle from an inactive lane");
                    }
                }
            }
            // second pass: values (all reads before writes)
            std::vector<long long> vals(64);
            for (int i = b; i < e; ++i) vals[i - b] = g_f[i].val;
            for (int i = b; i < e; ++i) {
                Fiber& f = g_f[i];
                if (f.state == DONE) continue;
                const int l = i - b;
                int src = l;
                switch (op) {
                    case OP_SHFL: src = ((f.arg % 64) + 64) % 64; break;
                    case OP_SHFL_UP: src = l >= f.arg ? l - f.arg : l; break;
                    case OP_SHFL_DOWN: src = l + f.arg < 64 ? l + f.arg : l; break;
                    case OP_SHFL_XOR: src = (l ^ f.arg) & 63; break;
                }
                if (op != OP_BALLOT && op != OP_WBAR) f.res = vals[src];
                f.state = RUN;
            }
            prog = true;
        }
        if (prog) continue;
        // block barrier: every live thread must be at one
        int atb = 0, live = 0;
        void* site = nullptr;
        bool same = true;
        for (int i = 0; i < nf; ++i) {
            if (g_f[i].state == DONE) continue;
            ++live;
            if (g_f[i].state == AT_BAR) {
                ++atb;
                if (!site) site = g_f[i].site;
                else if (site != g_f[i].site) same = false;
            }
        }
        if (atb == live && same) {
            for (int i = 0; i < nf; ++i)
                if (g_f[i].state == AT_BAR) g_f[i].state = RUN;
            continue;
        }
        fprintf(stderr, "deadlock: %d live, %d at barrier, same site %d\n", live, atb, (int)same);
        dump_block(nf);
        die("deadlock");
    }
}

void run_launch(dim3 g, dim3 b, void (*tramp)(void*), void* ctx) {
    const int nf = (int)(b.x * b.y * b.z);
    if (nf <= 0 || nf > 1024) die("bad block size");
    if ((int)g_f.size() < nf) {
        size_t old = g_f.size();
        g_f.resize(nf);
        for (size_t i = old; i < g_f.size(); ++i) {
            void* p = mmap(nullptr, STACK, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
            if (p == MAP_FAILED) die("mmap stack");
            g_f[i].stack = (char*)p;
            g_f[i].stack_size = STACK;
        }
    }
    ++g_launches;
    g_tramp = tramp;
    g_ctx = ctx;
    g_bdim = uint3s{b.x, b.y, b.z};
    g_gdim = uint3s{g.x, g.y, g.z};
    const unsigned nb = g.x * g.y * g.z;
    std::vector<unsigned> order(nb);
    for (unsigned i = 0; i < nb; ++i) order[i] = i;
    if (getenv("SIMT_SHUFFLE")) std::shuffle(order.begin(), order.end(), g_rng);
    for (unsigned k = 0; k < nb; ++k) {
        const unsigned i = order[k];
        g_block = uint3s{i % g.x, (i / g.x) % g.y, i / (g.x * g.y)};
        run_block(nf);
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
