// Internal host-side objects behind the opaque C ABI handles.
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/kkt.h"
#include "device.hpp"
#include "kernels.hpp"
#include "symbolic.hpp"

namespace kkt {

extern thread_local std::string g_last_error;
kkt_status fail(kkt_status st, const std::string& msg);
kkt_status hip_fail(hipError_t e, const char* what);
kkt_status ensure_runtime();

// Owning device allocation.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf();
    void release();
    hipError_t alloc(size_t nb);
};

// Symbolic arrays of one pattern uploaded to the device, plus the single
// instance work lists.
struct DevPattern {
    PatDev desc{};
    DevBuf b_col0, b_ncol, b_nrow, b_rowofs, b_lofs, b_uofs, b_vofs, b_rows, b_rel, b_chptr, b_chlist,
        b_ksnptr, b_kloc, b_kw, b_kdiag, b_kpptr, b_pa, b_pb, b_jrow, b_perm, b_iperm, b_spptr, b_spe, b_spcol,
        b_jptr, b_jcol, b_jtptr, b_jte, b_jtrow;
    DevBuf b_snitems, b_nitems, b_mitems, b_kitems;
    int n_nitems = 0, n_mitems = 0, n_kitems = 0;
    std::vector<int> lvl_ptr;
    size_t lds_factor = 0, lds_solve = 0;
    hipError_t build(const Symbolic& S);
};

// Per-launch HIP event timers, grouped by phase.
struct LaunchTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<int> phase;     // phase of event pair q (events 2q, 2q+1)
    size_t used = 0;            // pairs recorded since the last read
    hipEvent_t cur = nullptr;
    int cur_phase = 0;
    ~LaunchTimer();
    void begin(int ph, hipStream_t st);
    void end(hipStream_t st);
    hipError_t read(double* ms, int* launches, int nph);
};

}  // namespace kkt

struct kkt_symbolic {
    kkt::Symbolic S;
};

struct kkt_factor {
    const kkt_symbolic* sym = nullptr;
    kkt::DevPattern pat;
    kkt::DevBuf L, U, V, kval, y, r, xprev, tn, fg, cvec, rvec, pvec, qvec, red, status, rs, cg, ndone, jcopy, dinst;
    kkt::InstDev hinst{};
    void* hpin = nullptr;          // pinned host staging (4 KB)
    hipStream_t last_stream = nullptr;
    int mode = 0;                  // 0 none, 1 Lifted-KKT, 2 HyKKT (K_gamma)
    double gamma = 0.0;
    bool factored = false;
    kkt::LaunchTimer timer;
    ~kkt_factor() {
        if (hpin) (void)hipHostFree(hpin);
    }
};
