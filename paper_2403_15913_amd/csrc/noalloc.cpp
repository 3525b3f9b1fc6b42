// Allocation-free refined solve (kkt_solve_noalloc): for callers that cannot
// allocate device memory -- code under HIP graph capture, tight serving
// loops, harnesses that forbid hipMalloc.
//
// The per-solve workspace of kkt_solve (the permuted work vector, the
// forward sweep's update vectors, the residual, the previous iterate, the
// residual block maxima, the refinement record and the stop counter), and
// redirected copies of the factor's instance and front descriptors that
// point into it, live in one file-scope device array, `scratch`, of
// kScratchBytes. Each GPU holds its own copy of the array (at its own
// address) until the process ends. Host code never passes the array's name
// to a kernel or a copy: its device address is looked up once per device
// with hipGetSymbolAddress and kept.
//
// Every call on a GPU shares that GPU's array and leaves its contents
// behind; every part a solve reads is written by that solve first (the
// descriptors by the redirect kernel, the stop counter and the refinement
// record by the solve's own reset kernels), so nothing carries over. Calls
// that overlap on one GPU (two streams, two host threads) race on the array.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "api_internal.hpp"

namespace kkt {

constexpr size_t kScratchBytes = size_t(32) << 20;

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

// device address of the current device's scratch array
kkt_status scratch_address(char** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "current device");
    if (dev < 0 || dev >= kMaxDevices) return fail(KKT_ERR_DEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "scratch symbol address");
        g_scratch_ptr[dev] = (char*)p;
    }
    *out = g_scratch_ptr[dev];
    return KKT_OK;
}

// bump layout over the scratch array (256-byte aligned pieces)
struct Layout {
    char* base;
    size_t off = 0;
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += (count ? count : 1) * sizeof(T);
        return p;
    }
};

// Points the engine's descriptor, stop-counter and refinement-record
// pointers at the workspace for the duration of one call.
struct Redirect {
    Engine& E;
    InstDev* d;
    FrontDesc* f;
    int* nd;
    RefineState* rs;
    bool timing;
    Redirect(Engine& e, const SolveWs& w, int* ndone)
        : E(e), d(e.dinsts), f(e.fdesc), nd(e.ndone), rs(e.rs), timing(e.timer.on) {
        E.dinsts = w.inst;
        E.fdesc = w.fd;
        E.ndone = ndone;
        E.rs = w.rs;
        E.timer.on = false;  // the per-launch timers create events
    }
    ~Redirect() {
        E.dinsts = d;
        E.fdesc = f;
        E.ndone = nd;
        E.rs = rs;
        E.timer.on = timing;
    }
};
}  // namespace

}  // namespace kkt

using namespace kkt;

extern "C" kkt_status kkt_solve_noalloc(kkt_factor* f, const double* b, double* x, const kkt_refine_opts* ro,
                                        kkt_solve_info* info, void* stream) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    const Symbolic& S = f->sym->S;
    const int n = S.n;
    if (n > 0 && (!b || !x)) return fail(KKT_ERR_INVALID_ARG, "NULL vector");
    if (b == x && n > 0) return fail(KKT_ERR_INVALID_ARG, "x aliases b");
    Engine& E = f->eng;
    if (!E.factored) return fail(KKT_ERR_STATE, "solve before refactor");
    const int maxit = ro ? ro->max_iter : 10;
    const double tol = ro ? ro->tol : 1e-14;
    if (maxit < 0 || !(tol >= 0.0)) return fail(KKT_ERR_INVALID_ARG, "bad refinement options");
    const int nf = E.lvl_ptr.empty() ? 0 : E.lvl_ptr.back();
    const size_t nres = 5 * (size_t)((n + kBlock - 1) / kBlock) * kResidualSplit;
    // the workspace must fit the array
    Layout probe{nullptr};
    probe.take<InstDev>(1);
    probe.take<FrontDesc>(nf);
    probe.take<double>(n);
    probe.take<double>(S.vsize);
    probe.take<double>(n);
    probe.take<double>(n);
    probe.take<double>(nres);
    probe.take<RefineState>(1);
    probe.take<int>(4);
    if (probe.off > kScratchBytes)
        return fail(KKT_ERR_BUDGET, "the solve workspace (" + std::to_string(probe.off) + " bytes) exceeds the " +
                                        std::to_string(kScratchBytes) + "-byte scratch of kkt_solve_noalloc");
    char* base = nullptr;
    kkt_status ks = scratch_address(&base);
    if (ks != KKT_OK) return ks;
    Layout L{base};
    SolveWs w;
    w.inst = L.take<InstDev>(1);
    w.fd = L.take<FrontDesc>(nf);
    w.y = L.take<double>(n);
    w.V = L.take<double>(S.vsize);
    w.r = L.take<double>(n);
    w.xprev = L.take<double>(n);
    w.rpart = L.take<double>(nres);
    w.rs = L.take<RefineState>(1);
    int* nd = L.take<int>(4);
    const hipStream_t st = (hipStream_t)stream;
    launch_ws_redirect(E.dinsts, E.fdesc, nf, w, st);
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.b = b;
    C.x = x;
    Redirect R(E, w, nd);
    if (info) return E.solve(C, maxit, tol, info, st);
    E.last_stream = st;
    E.solve_start(C, maxit, tol, st);
    E.solve_rounds(C, maxit, st);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KKT_OK : hip_fail(e, "solve launch");
}
