// Internal host-side objects behind the opaque C ABI handles.
//
// An Engine owns the device storage and work lists of a set of instances
// (one instance for a kkt_factor, many for a kkt_batch). Every instance is a
// symbolic pattern uploaded once (DevPattern, shared by instances with the
// same analysis), a slice of the numeric storage, and the offsets of its
// values inside the caller's concatenated arrays. Refactor, solve and CG run
// the same kernels for one or many instances.
#pragma once
#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "../../include/kkt.h"
#include "device.hpp"
#include "kernels.hpp"
#include "lds_layout.hpp"
#include "symbolic.hpp"

// Launch `expr` on stream `st`, bracketed by timer events when timing is on.
#define TL(ph, expr)                              \
    do {                                          \
        if (timer.on) timer.begin(ph, st);        \
        expr;                                     \
        if (timer.on) timer.end(st);              \
    } while (0)

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

// Symbolic arrays of one pattern on the device.
struct DevPattern {
    PatDev desc{};
    DevBuf b_col0, b_ncol, b_nrow, b_rowofs, b_lofs, b_uofs, b_vofs, b_rows, b_rel, b_relnp, b_chptr, b_chlist, b_pinvofs, b_pinv,
        b_ksnptr, b_kloc, b_kw, b_kdiag, b_kpptr, b_pa, b_pb, b_jrow, b_perm, b_iperm, b_spptr, b_kcsr, b_spcol,
        b_jptr, b_jcol, b_jtptr, b_jte, b_jtrow, b_jtpptr, b_jtprow, b_jtpe, b_jcolp;
    hipError_t build(const Symbolic& S);
};

// Per-launch HIP event timers, grouped by phase.
struct LaunchTimer {
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<int> phase;     // phase of event pair q (events 2q, 2q+1)
    size_t used = 0;            // pairs recorded since the last read
    hipEvent_t cur = nullptr;
    ~LaunchTimer();
    void begin(int ph, hipStream_t st);
    void end(hipStream_t st);
    hipError_t read(double* ms, int* launches, int nph);
};

// Value staging of a served wave: the requests' inputs gathered into
// concatenated arrays so the batched kernels can address them by offset.
struct Staging {
    double *w = nullptr, *j = nullptr, *sx = nullptr, *ss = nullptr, *b = nullptr, *x = nullptr;
};

struct Engine {
    int ninst = 0;
    std::vector<const Symbolic*> syms;
    std::vector<const DevPattern*> pat_of;
    std::vector<std::unique_ptr<DevPattern>> pats;  // patterns uploaded by this engine itself
    DevBuf own;                                     // arena owned by a factor / batch
    // views into the arena
    double *L = nullptr, *U = nullptr, *V = nullptr, *kval = nullptr, *kcsr = nullptr, *rpart = nullptr, *dinv = nullptr, *y = nullptr, *r = nullptr,
           *xprev = nullptr, *fg = nullptr, *cvec = nullptr, *rvec = nullptr, *pvec = nullptr,
           *pvec2 = nullptr, *qvec = nullptr, *red = nullptr, *jcopy = nullptr, *jtv = nullptr, *k0csr = nullptr,
           *jraw = nullptr, *ssv = nullptr, *aug_b = nullptr, *aug_t = nullptr, *aug_e = nullptr, *aug_prev = nullptr;
    AugState* aug = nullptr;
    int *status = nullptr, *ndone = nullptr;
    RefineState* rs = nullptr;
    CgState* cg = nullptr;
    InstDev* dinsts = nullptr;
    WorkItem *snitems = nullptr, *nitems = nullptr, *mitems = nullptr, *kitems = nullptr, *jitems = nullptr,
             *hitems = nullptr;
    FrontDesc* fdesc = nullptr;                     // one per front work item (same order as snitems)
    int *dep_parent = nullptr, *dep_nchild = nullptr, *dep_ctr = nullptr;  // queue scheduling
    StripItem* upitems = nullptr;                   // update-matrix tiles by level (level schedule)
    std::vector<int> up_ptr;
    std::vector<int> upl_ptr;                       // per level: first tile of its large fronts
    std::vector<int> lvl_large;                     // per level: first large front (they come last)
    std::vector<int> lvl_lmaxc, lvl_lmaxr;          // per level: widest and tallest large front
    int n_large = 0;                                // large fronts (panels factored in HBM)
    std::vector<int> lvl_maxu;                      // widest update part of each level
    std::vector<size_t> lvl_flds;                   // factor LDS of each level's largest front
    std::vector<int> lvl_maxc;                      // widest front (columns) of each level
    int small_front_cols = 0;                       // levels whose fronts have at most this many columns: four-wave factor
    bool split_update = true;                       // level schedule: update matrices in their own launch
    int split_max_fronts = kSplitMaxFronts;         // ... on levels with fewer fronts than this
    int split_min_rows = kSplitMinRows;             // ... whose widest update part has at least this many rows
    bool queue_sched = false;                       // dependency-driven launches (else one launch per level)
    bool assembly_only = false;                     // no supernodal factor storage (stage-structured solver)
    bool single_storage = false;                    // single factors: K0, J and Sigma_s kept for the HyKKT CG
                                                    // and the augmented-system solve
    double delta_last = 0.0;                        // inertia correction: last delta that made K definite
    bool keep_aug = false;                          // Lifted-KKT refactors keep K0, J and Sigma_s (augmented solve)
    bool aug_ready = false;                         // the current factorization kept them
    DevBuf eqmask;                                  // general HyKKT: 1 on the equality rows of J (m ints)
    DevBuf ipm_ws;                                  // interior-point loop vectors (allocated on first use)
    int n_eq = 0;                                   // equality rows set (0: none)
    // captured refactor + solve (batched form)
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;
    hipEvent_t ctl_event = nullptr, ctl_event2 = nullptr;  // refinement / CG control readback
    Calls g_calls{};
    int g_rounds = 0, g_maxit = 0;
    double g_tol = 0.0;
    Staging stage;                                  // used by served waves only
    std::vector<InstDev> hinst;
    std::vector<int> lvl_ptr;
    // sweep launches: each level split into LDS size classes (small fronts
    // first), parts sw_lvl[l] .. sw_lvl[l + 1] of sw_part
    struct SweepPart { int begin, count; size_t lds; };
    std::vector<SweepPart> sw_part;
    std::vector<int> sw_lvl;
    int n_nitems = 0, n_mitems = 0, n_kitems = 0, n_jitems = 0, n_hitems = 0;
    size_t lds_factor = 0, lds_solve = 0;
    std::vector<int64_t> n_ofs, m_ofs, w_ofs, j_ofs;  // ninst + 1 prefix offsets
    void* hpin = nullptr;                              // pinned host staging (uploads, readback)
    size_t hpin_bytes = 0;
    LaunchTimer timer;
    hipStream_t last_stream = nullptr;
    int mode = 0;                                      // 0 none, 1 Lifted-KKT, 2 HyKKT (K_gamma),
                                                       // 3 general HyKKT (equality and inequality rows)
    double gamma = 0.0;
    bool factored = false;

    Engine() = default;
    Engine(const Engine&) = delete;
    Engine& operator=(const Engine&) = delete;
    ~Engine();

    // Lays the instances out in `mem` (cap bytes; mem == NULL only measures)
    // and uploads descriptors and work lists on `st`. Returns the bytes used
    // through *used. With staging, also carves the served-wave value arrays.
    kkt_status place(const std::vector<const Symbolic*>& s, const std::vector<const DevPattern*>& p, char* mem,
                     size_t cap, bool staging, hipStream_t st, size_t* used);
    // factor / batch: uploads the distinct patterns, allocates an own arena, places, waits
    kkt_status init_owned(const std::vector<const Symbolic*>& s);
    const InstDev* di() const { return dinsts; }
    kkt_status refactor(const Calls& C, hipStream_t st);
    kkt_status assemble(const Calls& C, hipStream_t st);
    void sweeps(hipStream_t st, int skip_done);
    // Lifted-KKT solve with refinement; infos (ninst entries) filled when non-NULL.
    kkt_status solve(const Calls& C, int maxit, double tol, kkt_solve_info* infos, hipStream_t st);
    void solve_start(const Calls& C, int maxit, double tol, hipStream_t st);
    void refine_check(const Calls& C, hipStream_t st);
    void refine_correct(const Calls& C, hipStream_t st);
    kkt_status solve_finish(const Calls& C, int iter0, int maxit, double tol, kkt_solve_info* infos,
                            hipStream_t st);
    // hipGraph of refactor + first solve + `rounds` refinement rounds, and its replay
    kkt_status capture(const Calls& C, int maxit, double tol, int rounds);
    kkt_status replay(kkt_solve_info* infos, hipStream_t st);
    void drop_graph();
    kkt_status cg_schur(const Calls& C, double tol, int maxit, double eta_tol, kkt_cg_info* info, hipStream_t st);
    void cg_iteration(int k, int maxit, bool eta_test, hipStream_t st);
    Calls cg_calls{};
    // asynchronous solve: the first solve and max_iter refinement rounds,
    // every kernel gated by the instance's stop flag, no read-back
    void solve_rounds(const Calls& C, int maxit, hipStream_t st);
    // augmented system (Lifted-KKT): condensed solve, slack and multiplier
    // recovery, refinement on the full system
    kkt_status solve_augmented(const AugCall& A, int maxit, double tol, kkt_aug_info* info, hipStream_t st);
    // waits for st and returns each instance's latched status and failing column (original index)
    kkt_status read_status(int* st_out, int* bad_out);
    kkt_status parse_status(int derr, const int* hs, int* st_out, int* bad_out);
    hipError_t ensure_pinned(size_t bytes);
    DepLists deps() const;
};

// bytes of one instance of a pattern in an engine arena (with staging)
size_t instance_bytes(const Symbolic& S);

}  // namespace kkt

struct kkt_symbolic {
    kkt::Symbolic S;
};

struct kkt_factor {
    const kkt_symbolic* sym = nullptr;
    kkt::Engine eng;
};

struct kkt_batch {
    std::vector<const kkt_symbolic*> syms;
    kkt::Engine eng;
};
