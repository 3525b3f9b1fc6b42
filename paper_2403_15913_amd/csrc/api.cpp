// C ABI of libkkt (declared in include/kkt.h): symbolic objects, device
// factors and batches, the Lifted-KKT solve with Richardson refinement and
// the HyKKT Schur-complement CG (Pacaud & Shin, arXiv 2403.15913, sections
// "Condensed KKT system" and "Hybrid linear solver").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/kkt.h"
#include "api_internal.hpp"

using namespace kkt;


namespace kkt {

thread_local std::string g_last_error;

kkt_status fail(kkt_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

kkt_status hip_fail(hipError_t e, const char* what) {
    return fail(e == hipErrorOutOfMemory ? KKT_ERR_OOM : KKT_ERR_DEVICE,
                std::string(what) + ": " + hipGetErrorString(e));
}

static bool g_attr_done = false;

kkt_status ensure_runtime() {
    if (g_attr_done) return KKT_OK;
    hipError_t e = set_kernel_attributes();
    if (e != hipSuccess) return hip_fail(e, "hipFuncSetAttribute");
    g_attr_done = true;
    return KKT_OK;
}

DevBuf::~DevBuf() { release(); }
void DevBuf::release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
}
hipError_t DevBuf::alloc(size_t nb) {
    release();
    if (nb == 0) nb = 8;
    hipError_t e = hipMalloc(&p, nb);
    if (e == hipSuccess) bytes = nb;
    else p = nullptr;
    return e;
}

template <class T>
static hipError_t upload(DevBuf& b, const std::vector<T>& v) {
    hipError_t e = b.alloc(v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    if (!v.empty()) e = hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return e;
}

LaunchTimer::~LaunchTimer() {
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
}

void LaunchTimer::begin(int ph, hipStream_t st) {
    if (used >= 100000) return;  // bounded: read the timers regularly
    while (pool.size() < 2 * (used + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        pool.push_back(e);
    }
    if (phase.size() < used + 1) phase.resize(used + 1);
    phase[used] = ph;
    cur = pool[2 * used];
    (void)hipEventRecord(cur, st);
}

void LaunchTimer::end(hipStream_t st) {
    if (!cur) return;
    (void)hipEventRecord(pool[2 * used + 1], st);
    cur = nullptr;
    used++;
}

hipError_t LaunchTimer::read(double* ms, int* launches, int nph) {
    for (int q = 0; q < nph; q++) { ms[q] = 0.0; launches[q] = 0; }
    if (used == 0) return hipSuccess;
    hipError_t e = hipEventSynchronize(pool[2 * used - 1]);
    if (e != hipSuccess) return e;
    for (size_t q = 0; q < used; q++) {
        float t = 0.f;
        e = hipEventElapsedTime(&t, pool[2 * q], pool[2 * q + 1]);
        if (e != hipSuccess) return e;
        if (phase[q] >= 0 && phase[q] < nph) { ms[phase[q]] += t; launches[phase[q]]++; }
    }
    used = 0;
    return hipSuccess;
}

hipError_t DevPattern::build(const Symbolic& S) {
    hipError_t e;
#define UP(buf, vec, field, type)                         \
    if ((e = upload(buf, S.vec)) != hipSuccess) return e; \
    desc.field = (const type*)buf.p;
    desc.n = S.n;
    desc.m = S.m;
    desc.ns = S.ns;
    desc.nlevels = S.nlevels;
    UP(b_col0, sn_col0, sn_col0, int)
    UP(b_ncol, sn_ncol, sn_ncol, int)
    UP(b_nrow, sn_nrow, sn_nrow, int)
    UP(b_rowofs, sn_rowofs, sn_rowofs, int64_t)
    UP(b_lofs, sn_lofs, sn_lofs, int64_t)
    UP(b_uofs, sn_uofs, sn_uofs, int64_t)
    UP(b_vofs, sn_vofs, sn_vofs, int64_t)
    UP(b_rows, rows, rows, int)
    UP(b_rel, rel, rel, int)
    UP(b_relnp, rel_np, rel_np, int)
    UP(b_chptr, ch_ptr, ch_ptr, int)
    UP(b_chlist, ch_list, ch_list, int)
    UP(b_pinvofs, pinv_ofs, pinv_ofs, int64_t)
    UP(b_pinv, pinv, pinv, int)
    UP(b_ksnptr, k_snptr, k_snptr, int64_t)
    UP(b_kloc, k_loc, k_loc, int)
    UP(b_kw, k_w, k_w, int)
    UP(b_kdiag, k_diag, k_diag, int)
    UP(b_kpptr, k_pptr, k_pptr, int64_t)
    UP(b_pa, pair_a, pair_a, int)
    UP(b_pb, pair_b, pair_b, int)
    UP(b_jrow, jrow, jrow, int)
    UP(b_perm, perm, perm, int)
    UP(b_iperm, iperm, iperm, int)
    UP(b_spptr, sp_ptr, sp_ptr, int64_t)
    UP(b_kcsr, k_csr, k_csr, int)
    UP(b_spcol, sp_col, sp_col, int)
    UP(b_jptr, j_ptr, j_ptr, int)
    UP(b_jcol, j_col, j_col, int)
    UP(b_jtptr, jt_ptr, jt_ptr, int)
    UP(b_jte, jt_e, jt_e, int)
    UP(b_jtrow, jt_row, jt_row, int)
#undef UP
    // J by columns in pivot order, and the pivot position of every J entry's
    // column (the CG reads and writes the sweep vector directly)
    std::vector<int> tp(S.n + 1, 0), trow(S.jt_row.size()), te(S.jt_e.size()), colp(S.j_col.size());
    for (int k = 0; k < S.n; k++) {
        const int j = S.perm[k];
        tp[k + 1] = tp[k] + (S.jt_ptr[j + 1] - S.jt_ptr[j]);
        for (int q = S.jt_ptr[j], o = tp[k]; q < S.jt_ptr[j + 1]; q++, o++) {
            trow[o] = S.jt_row[q];
            te[o] = S.jt_e[q];
        }
    }
    for (size_t p = 0; p < S.j_col.size(); p++) colp[p] = S.iperm[S.j_col[p]];
    if ((e = upload(b_jtpptr, tp)) != hipSuccess || (e = upload(b_jtprow, trow)) != hipSuccess ||
        (e = upload(b_jtpe, te)) != hipSuccess || (e = upload(b_jcolp, colp)) != hipSuccess)
        return e;
    desc.jtp_ptr = (const int*)b_jtpptr.p;
    desc.jtp_row = (const int*)b_jtprow.p;
    desc.jtp_e = (const int*)b_jtpe.p;
    desc.j_colp = (const int*)b_jcolp.p;
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Engine
// ---------------------------------------------------------------------------
Engine::~Engine() {
    drop_graph();
    if (ctl_event) (void)hipEventDestroy(ctl_event);
    if (ctl_event2) (void)hipEventDestroy(ctl_event2);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (hpin) (void)hipHostFree(hpin);
}

hipError_t Engine::ensure_pinned(size_t bytes) {
    if (bytes <= hpin_bytes) return hipSuccess;
    if (hpin) (void)hipHostFree(hpin);
    hpin = nullptr;
    hpin_bytes = 0;
    bytes = std::max<size_t>(bytes, 4096);
    hipError_t e = hipHostMalloc(&hpin, bytes, hipHostMallocDefault);
    if (e == hipSuccess) hpin_bytes = bytes;
    return e;
}

namespace {
// a front whose panel does not fit the symbolic analysis' LDS budget: factored
// and solved in place in HBM
bool is_large(const Symbolic& S, int k) { return front_lds_bytes(S.sn_nrow[k], S.sn_ncol[k]) > S.lds_budget; }

// bump allocator over an arena (256-byte aligned pieces); measures when base is NULL
struct Carver {
    char* base;
    size_t off = 0, cap;
    Carver(char* b, size_t c) : base(b), cap(c) {}
    template <class T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += std::max<size_t>(count, 1) * sizeof(T);
        return p;
    }
};
}  // namespace

kkt_status Engine::place(const std::vector<const Symbolic*>& s, const std::vector<const DevPattern*>& p, char* mem,
                         size_t cap, bool staging, hipStream_t st, size_t* used) {
    syms = s;
    pat_of = p;
    ninst = (int)s.size();
    n_large = 0;
    n_ofs.assign(ninst + 1, 0);
    m_ofs.assign(ninst + 1, 0);
    w_ofs.assign(ninst + 1, 0);
    j_ofs.assign(ninst + 1, 0);
    std::vector<int64_t> lo(ninst + 1, 0), uo(ninst + 1, 0), vo(ninst + 1, 0), ko(ninst + 1, 0), ro(ninst + 1, 0),
        co(ninst + 1, 0), po(ninst + 1, 0);
    lds_factor = lds_solve = 0;
    int nlev = 0;
    size_t nsn = 0, nnb = 0, nmb = 0, nkb = 0, nup = 0, njb = 0;
    // entries of K with long product lists, assembled 16 lanes per entry
    std::vector<WorkItem> hv;
    for (int q = 0; q < ninst; q++) {
        const Symbolic& S = *s[q];
        for (const int e : S.k_heavy) hv.push_back(WorkItem{q, e});
        n_ofs[q + 1] = n_ofs[q] + S.n;
        m_ofs[q + 1] = m_ofs[q] + S.m;
        w_ofs[q + 1] = w_ofs[q] + S.nnz_w;
        j_ofs[q + 1] = j_ofs[q] + S.nnz_j;
        lo[q + 1] = lo[q] + S.lsize;
        uo[q + 1] = uo[q] + S.usize;
        vo[q + 1] = vo[q] + S.vsize;
        ko[q + 1] = ko[q] + S.nnzk;
        co[q + 1] = co[q] + S.sp_ptr[S.n];
        po[q + 1] = po[q] + 5 * (int64_t)((S.n + kBlock - 1) / kBlock) * kResidualSplit;
        // reduction slots of the CG and the augmented solve: up to 8 per
        // 256-row block of n and of m
        ro[q + 1] = ro[q] + 8 * (int64_t)((S.n + kBlock - 1) / kBlock + (S.m + kBlock - 1) / kBlock) + 4;
        for (int k = 0; k < S.ns; k++) {
            // large fronts are factored and solved in HBM (no panel in LDS)
            if (is_large(S, k)) {
                if (S.sn_ncol[k] > kLargeFrontCols) return fail(KKT_ERR_PATTERN, "large front wider than 64 columns");
                n_large++;
            } else {
                lds_factor = std::max(lds_factor, (size_t)factor_lds_bytes(S.sn_nrow[k], S.sn_ncol[k]));
                lds_solve = std::max(lds_solve, (size_t)solve_lds_bytes(S.sn_nrow[k], S.sn_ncol[k]));
            }
            const size_t nbu = (size_t)(S.sn_nrow[k] - S.sn_ncol[k] + 15) / 16;
            nup += nbu * (nbu + 1) / 2;
        }
        nlev = std::max(nlev, S.nlevels);
        nsn += S.ns;
        nnb += (S.n + kBlock - 1) / kBlock;
        nmb += (S.m + kBlock - 1) / kBlock;
        nkb += (S.nnzk + kBlock - 1) / kBlock;
        njb += (S.nnz_j + kBlock - 1) / kBlock;
    }
    if (lds_factor > (size_t)kMaxDynLds || lds_solve > (size_t)kMaxDynLds)
        return fail(KKT_ERR_PATTERN, "a front exceeds the per-workgroup LDS budget");
    const size_t N = (size_t)n_ofs[ninst], M = (size_t)m_ofs[ninst];
    Carver cv(mem, cap);
    // the stage-structured solver uses the engine for assembly and refinement
    // only: no supernode panels, update matrices or vectors
    L = cv.take<double>(assembly_only ? 0 : lo[ninst]);
    U = cv.take<double>(assembly_only ? 0 : uo[ninst]);
    V = cv.take<double>(assembly_only ? 0 : vo[ninst]);
    kval = cv.take<double>(ko[ninst]);
    kcsr = cv.take<double>(co[ninst]);
    rpart = cv.take<double>(po[ninst]);
    dinv = cv.take<double>(N);
    y = cv.take<double>(N);
    r = cv.take<double>(N);
    xprev = cv.take<double>(N);
    fg = cv.take<double>(N);
    cvec = cv.take<double>(M);
    rvec = cv.take<double>(M);
    pvec = cv.take<double>(M);
    pvec2 = cv.take<double>(M);
    qvec = cv.take<double>(M);
    red = cv.take<double>(ro[ninst]);
    jcopy = cv.take<double>(j_ofs[ninst]);
    jtv = single_storage ? cv.take<double>(j_ofs[ninst]) : nullptr;
    k0csr = single_storage ? cv.take<double>(co[ninst]) : nullptr;
    jraw = single_storage ? cv.take<double>(j_ofs[ninst]) : nullptr;
    ssv = single_storage ? cv.take<double>(M) : nullptr;
    aug_b = single_storage ? cv.take<double>(N) : nullptr;
    aug_t = single_storage ? cv.take<double>(N) : nullptr;
    aug_e = single_storage ? cv.take<double>(N + 2 * M) : nullptr;
    aug_prev = single_storage ? cv.take<double>(N + 2 * M) : nullptr;
    aug = single_storage ? cv.take<AugState>(ninst) : nullptr;
    status = cv.take<int>(2 * (size_t)ninst);
    ndone = cv.take<int>(4);
    rs = cv.take<RefineState>(ninst);
    cg = cv.take<CgState>(ninst);
    dinsts = cv.take<InstDev>(ninst);
    snitems = cv.take<WorkItem>(nsn);
    fdesc = cv.take<FrontDesc>(nsn);
    nitems = cv.take<WorkItem>(nnb);
    mitems = cv.take<WorkItem>(nmb);
    kitems = cv.take<WorkItem>(nkb);
    jitems = cv.take<WorkItem>(njb);
    hitems = cv.take<WorkItem>(hv.size());
    dep_parent = cv.take<int>(nsn);
    dep_nchild = cv.take<int>(nsn);
    dep_ctr = cv.take<int>(3 * nsn + 2);
    upitems = cv.take<StripItem>(nup);
    stage = Staging{};
    if (staging) {
        stage.w = cv.take<double>(w_ofs[ninst]);
        stage.j = cv.take<double>(j_ofs[ninst]);
        stage.sx = cv.take<double>(N);
        stage.ss = cv.take<double>(M);
        stage.b = cv.take<double>(N);
        stage.x = cv.take<double>(N);
    }
    const size_t total = (cv.off + 255) & ~(size_t)255;
    if (used) *used = total;
    if (!mem) return KKT_OK;
    if (total > cap) return fail(KKT_ERR_BUDGET, "instances do not fit the arena");

    hinst.assign(ninst, InstDev{});
    for (int q = 0; q < ninst; q++) {
        InstDev& I = hinst[q];
        std::memset(&I, 0, sizeof(I));
        I.P = p[q]->desc;
        I.w_off = w_ofs[q];
        I.j_off = j_ofs[q];
        I.n_off = n_ofs[q];
        I.m_off = m_ofs[q];
        I.L = L + lo[q];
        I.U = U + uo[q];
        I.V = V + vo[q];
        I.kval = kval + ko[q];
        I.kcsr = kcsr + co[q];
        I.rpart = rpart + po[q];
        I.js = jcopy + j_ofs[q];
        I.dinv = dinv + n_ofs[q];
        I.y = y + n_ofs[q];
        I.r = r + n_ofs[q];
        I.xprev = xprev + n_ofs[q];
        I.fg = fg + n_ofs[q];
        I.cvec = cvec + m_ofs[q];
        I.rvec = rvec + m_ofs[q];
        I.pvec = pvec + m_ofs[q];
        I.pvec2 = pvec2 + m_ofs[q];
        I.qvec = qvec + m_ofs[q];
        I.jtv = jtv ? jtv + j_ofs[q] : nullptr;
        I.k0csr = k0csr ? k0csr + co[q] : nullptr;
        I.jraw = jraw ? jraw + j_ofs[q] : nullptr;
        I.ssv = ssv ? ssv + m_ofs[q] : nullptr;
        // the augmented solve is offered for single factors (one instance)
        I.aug_b = aug_b;
        I.aug_t = aug_t;
        I.aug_e = aug_e;
        I.aug_prev = aug_prev;
        I.aug = aug ? aug + q : nullptr;
        I.red = red + ro[q];
        I.status = status + 2 * q;
        I.rs = rs + q;
        I.cg = cg + q;
    }
    // work lists: supernodes by tree level (leaves first) across instances,
    // and row / entry blocks of each instance
    std::vector<WorkItem> sn, nb, mb, kb, jb;
    sn.reserve(nsn);
    lvl_ptr.assign(1, 0);
    lvl_large.clear();
    sw_part.clear();
    sw_lvl.assign(1, 0);
    for (int l = 0; l < nlev; l++) {
        for (int q = 0; q < ninst; q++) {
            const Symbolic& S = *s[q];
            if (l >= S.nlevels) continue;
            for (int t = S.lvl_ptr[l]; t < S.lvl_ptr[l + 1]; t++) sn.push_back(WorkItem{q, S.lvl_list[t]});
        }
        // Each sweep launch takes the LDS of its own largest front, so a level
        // of small fronts runs two workgroups per compute unit. Fronts of one
        // level are independent and their order in the launch is free: where
        // the small fronts alone fill two workgroups on every compute unit,
        // they get a launch of their own after the larger fronts' (launches
        // on one stream run one after the other, so a split pays only for
        // wide levels).
        const int b0 = lvl_ptr.back();
        // large fronts last in the level (their own launches)
        const int bl = (int)(std::stable_partition(sn.begin() + b0, sn.end(),
                                                   [&](const WorkItem& w) { return !is_large(*s[w.inst], w.id); }) -
                             sn.begin());
        lvl_large.push_back(bl);
        auto slds = [&](const WorkItem& w) {
            const Symbolic& S = *s[w.inst];
            return (size_t)solve_lds_bytes(S.sn_nrow[w.id], S.sn_ncol[w.id]);
        };
        int nsmall = 0;
        for (int t = b0; t < bl; t++) nsmall += slds(sn[t]) <= kSweepHalfLds;
        int b1 = b0;
        if (nsmall >= kSweepSplitMin && nsmall < bl - b0)
            b1 = (int)(std::stable_partition(sn.begin() + b0, sn.begin() + bl,
                                             [&](const WorkItem& w) { return slds(w) > kSweepHalfLds; }) -
                       sn.begin());
        const int b2 = bl;
        // largest fronts first in each launch (and in the level's factor
        // launch), so the small ones fill the last round
        auto by_size = [&](const WorkItem& a, const WorkItem& b) { return slds(a) > slds(b); };
        std::stable_sort(sn.begin() + b0, sn.begin() + b1, by_size);
        std::stable_sort(sn.begin() + b1, sn.begin() + b2, by_size);
        for (int c = 0; c < 2; c++) {
            const int lo_i = c ? b1 : b0, hi_i = c ? b2 : b1;
            if (hi_i == lo_i) continue;
            size_t mx = 0;
            for (int t = lo_i; t < hi_i; t++) mx = std::max(mx, slds(sn[t]));
            sw_part.push_back(SweepPart{lo_i, hi_i - lo_i, mx});
        }
        sw_lvl.push_back((int)sw_part.size());
        lvl_ptr.push_back((int)sn.size());
    }
    // update-matrix tiles (lower part) of the same fronts, level by level
    std::vector<StripItem> up;
    up.reserve(nup);
    up_ptr.assign(1, 0);
    upl_ptr.clear();
    lvl_maxu.assign(lvl_ptr.size() - 1, 0);
    lvl_flds.assign(lvl_ptr.size() - 1, 0);
    lvl_maxc.assign(lvl_ptr.size() - 1, 0);
    lvl_lmaxc.assign(lvl_ptr.size() - 1, 0);
    lvl_lmaxr.assign(lvl_ptr.size() - 1, 0);
    // per level: the LDS fronts' tiles, then the large fronts' tiles
    for (size_t l = 0; l + 1 < lvl_ptr.size(); l++) {
        for (int t = lvl_ptr[l]; t < lvl_ptr[l + 1]; t++) {
            if (t == lvl_large[l]) upl_ptr.push_back((int)up.size());
            const Symbolic& S = *s[sn[t].inst];
            const int u = S.sn_nrow[sn[t].id] - S.sn_ncol[sn[t].id];
            if (t >= lvl_large[l]) {
                lvl_lmaxc[l] = std::max(lvl_lmaxc[l], S.sn_ncol[sn[t].id]);
                lvl_lmaxr[l] = std::max(lvl_lmaxr[l], S.sn_nrow[sn[t].id]);
            } else {
                lvl_maxu[l] = std::max(lvl_maxu[l], u);
                lvl_flds[l] = std::max(lvl_flds[l], (size_t)factor_lds_bytes(S.sn_nrow[sn[t].id], S.sn_ncol[sn[t].id]));
                lvl_maxc[l] = std::max(lvl_maxc[l], S.sn_ncol[sn[t].id]);
            }
            const int nbu = (u + 15) / 16;
            for (int tj = 0; tj < nbu; tj++)
                for (int ti = tj; ti < nbu; ti++) up.push_back(StripItem{sn[t].inst, sn[t].id, (ti << 16) | tj, t});
        }
        if (lvl_large[l] == lvl_ptr[l + 1]) upl_ptr.push_back((int)up.size());
        up_ptr.push_back((int)up.size());
    }
    // dependency lists in the same (topological) item order
    std::vector<int> dpar(sn.size(), -1), dnch(sn.size(), 0);
    {
        std::vector<std::vector<int>> item_of(ninst);
        for (int q = 0; q < ninst; q++) item_of[q].assign(s[q]->ns, -1);
        for (size_t t = 0; t < sn.size(); t++) item_of[sn[t].inst][sn[t].id] = (int)t;
        for (size_t t = 0; t < sn.size(); t++) {
            const Symbolic& S = *s[sn[t].inst];
            const int par = S.sn_parent[sn[t].id];
            if (par >= 0) {
                dpar[t] = item_of[sn[t].inst][par];
                dnch[dpar[t]]++;
            }
        }
    }
    // front descriptors in item order (absolute device addresses)
    std::vector<FrontDesc> fd(sn.size());
    for (size_t t = 0; t < sn.size(); t++) {
        const int q = sn[t].inst, k = sn[t].id;
        const Symbolic& S = *s[q];
        const PatDev& PD = p[q]->desc;
        const InstDev& I = hinst[q];
        FrontDesc& F = fd[t];
        std::memset(&F, 0, sizeof(F));
        F.r = S.sn_nrow[k];
        F.c = S.sn_ncol[k];
        F.col0 = S.sn_col0[k];
        F.nk = (int)(S.k_snptr[k + 1] - S.k_snptr[k]);
        F.kv = I.kval + S.k_snptr[k];
        F.kl = PD.k_loc + S.k_snptr[k];
        F.L = I.L + S.sn_lofs[k];
        F.U = I.U + S.sn_uofs[k];
        F.V = I.V + S.sn_vofs[k];
        F.y = I.y + F.col0;
        F.dinv = I.dinv + F.col0;
        F.rw = PD.rows + S.sn_rowofs[k] + F.c;
        F.done = (const int*)((const char*)I.rs + offsetof(RefineState, done));
        F.cgdone = (const int*)((const char*)I.cg + offsetof(CgState, done));
        F.ch0 = S.ch_ptr[k];
        F.nch = S.ch_ptr[k + 1] - S.ch_ptr[k];
        for (int j = 0; j < 2 && j < F.nch; j++) {
            const int ch = S.ch_list[F.ch0 + j], cc = S.sn_ncol[ch];
            F.cuc[j] = S.sn_nrow[ch] - cc;
            F.cnb[j] = S.rel_np[ch];
            F.cU[j] = I.U + S.sn_uofs[ch];
            F.cV[j] = I.V + S.sn_vofs[ch];
            F.crl[j] = PD.rel + S.sn_rowofs[ch] + cc;
            F.cinv[j] = PD.pinv + S.pinv_ofs[F.ch0 + j];
        }
        F.inst = q;
        F.id = k;
    }
    for (int q = 0; q < ninst; q++) {
        const Symbolic& S = *s[q];
        for (int i = 0; i < S.n; i += kBlock) nb.push_back(WorkItem{q, i});
        for (int i = 0; i < S.m; i += kBlock) mb.push_back(WorkItem{q, i});
        for (int64_t i = 0; i < S.nnzk; i += kBlock) kb.push_back(WorkItem{q, (int)i});
        for (int64_t i = 0; i < S.nnz_j; i += kBlock) jb.push_back(WorkItem{q, (int)i});
    }
    n_nitems = (int)nb.size();
    n_mitems = (int)mb.size();
    n_kitems = (int)kb.size();
    n_jitems = (int)jb.size();
    n_hitems = (int)hv.size();
    // one packed upload from pinned memory
    struct Piece { void* dst; const void* src; size_t bytes; } pieces[] = {
        {dinsts, hinst.data(), (size_t)ninst * sizeof(InstDev)},
        {snitems, sn.data(), sn.size() * sizeof(WorkItem)},
        {fdesc, fd.data(), fd.size() * sizeof(FrontDesc)},
        {nitems, nb.data(), nb.size() * sizeof(WorkItem)},
        {mitems, mb.data(), mb.size() * sizeof(WorkItem)},
        {kitems, kb.data(), kb.size() * sizeof(WorkItem)},
        {jitems, jb.data(), jb.size() * sizeof(WorkItem)},
        {hitems, hv.data(), hv.size() * sizeof(WorkItem)},
        {dep_parent, dpar.data(), dpar.size() * sizeof(int)},
        {dep_nchild, dnch.data(), dnch.size() * sizeof(int)},
        {upitems, up.data(), up.size() * sizeof(StripItem)},
    };
    size_t up_bytes = 0;
    for (auto& pc : pieces) up_bytes += pc.bytes;
    // read-back area: error latch, status words, refinement or CG records
    const size_t readback = 128 + (size_t)ninst * (8 + std::max(sizeof(RefineState), sizeof(CgState))) + 64;
    hipError_t e = ensure_pinned(std::max(up_bytes, readback));
    if (e != hipSuccess) return hip_fail(e, "pinned host buffer");
    // one packed staging buffer, one copy per piece
    char* h = (char*)hpin;
    size_t off = 0;
    for (auto& pc : pieces) {
        if (pc.bytes) {
            std::memcpy(h + off, pc.src, pc.bytes);
            if ((e = hipMemcpyAsync(pc.dst, h + off, pc.bytes, hipMemcpyHostToDevice, st)) != hipSuccess)
                return hip_fail(e, "descriptor upload");
        }
        off += pc.bytes;
    }
    if ((e = hipMemsetAsync(status, 0, 2 * (size_t)ninst * sizeof(int), st)) != hipSuccess ||
        (e = hipMemsetAsync(rs, 0, (size_t)ninst * sizeof(RefineState), st)) != hipSuccess ||
        (e = hipMemsetAsync(cg, 0, (size_t)ninst * sizeof(CgState), st)) != hipSuccess ||
        (e = hipMemsetAsync(dep_ctr, 0, (3 * sn.size() + 2) * sizeof(int), st)) != hipSuccess)
        return hip_fail(e, "state init");
    last_stream = st;
    factored = false;
    return KKT_OK;
}

size_t instance_bytes(const Symbolic& S) {
    Engine probe;
    std::vector<const Symbolic*> one{&S};
    std::vector<const DevPattern*> none{nullptr};
    size_t used = 0;
    probe.place(one, none, nullptr, 0, true, nullptr, &used);
    return used;
}

kkt_status Engine::init_owned(const std::vector<const Symbolic*>& s) {
    kkt_status st = ensure_runtime();
    if (st) return st;
    hipError_t e;
    std::map<const Symbolic*, const DevPattern*> up;
    std::vector<const DevPattern*> p(s.size());
    for (size_t q = 0; q < s.size(); q++) {
        auto it = up.find(s[q]);
        if (it == up.end()) {
            pats.emplace_back(new DevPattern);
            if ((e = pats.back()->build(*s[q])) != hipSuccess) return hip_fail(e, "pattern upload");
            it = up.emplace(s[q], pats.back().get()).first;
        }
        p[q] = it->second;
    }
    size_t need = 0;
    if ((st = place(s, p, nullptr, 0, false, nullptr, &need)) != KKT_OK) return st;
    if ((e = own.alloc(need)) != hipSuccess) return hip_fail(e, "device allocation");
    // control events of the refinement and CG loops (created here, so that
    // no solve call allocates)
    if ((e = hipEventCreateWithFlags(&ctl_event, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&ctl_event2, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "control events");
    if ((st = place(s, p, (char*)own.p, need, false, nullptr, nullptr)) != KKT_OK) return st;
    if ((e = hipStreamSynchronize(nullptr)) != hipSuccess) return hip_fail(e, "init");
    return KKT_OK;
}

DepLists Engine::deps() const {
    DepLists D;
    const int N = lvl_ptr.empty() ? 0 : lvl_ptr.back();
    D.parent = dep_parent;
    D.nchild = dep_nchild;
    D.cnt = dep_ctr;
    D.fdone = dep_ctr + N;
    D.bdone = dep_ctr + 2 * N;
    D.ticket = dep_ctr + 3 * N;
    D.err = dep_ctr + 3 * N + 1;
    D.nitems = N;
    return D;
}

// the assembly of K alone (the stage-structured solver factors it itself)
kkt_status Engine::assemble(const Calls& C, hipStream_t st) {
    last_stream = st;
    mode = 1;
    gamma = 0.0;
    TL(KKT_PHASE_CONTROL, launch_status_init(status, ninst, st));
    if (C.ss) TL(KKT_PHASE_ASSEMBLE, launch_jscale(di(), C, jitems, n_jitems, st));
    TL(KKT_PHASE_ASSEMBLE, launch_assemble(di(), C, kitems, n_kitems, st));
    TL(KKT_PHASE_ASSEMBLE, launch_assemble_heavy(di(), C, hitems, n_hitems, st));
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KKT_OK : hip_fail(e, "assembly launch");
}

kkt_status Engine::refactor(const Calls& Cin, hipStream_t st) {
    if (queue_sched && n_large > 0) return fail(KKT_ERR_INVALID_ARG, "the queue schedule needs every front in LDS");
    last_stream = st;
    mode = Cin.eqm ? 3 : (Cin.gamma == 0.0 ? 1 : 2);
    gamma = Cin.gamma;
    // K0 (K_k) and the J / Sigma_s copies: always for the CG modes, on request
    // for Lifted-KKT (the augmented solve)
    aug_ready = single_storage && (mode != 1 || keep_aug);
    Calls C = Cin;
    C.keep_k0 = aug_ready ? 1 : 0;
    // per instance: status[0] = 0, status[1] = INT_MAX (first failing pivot)
    TL(KKT_PHASE_CONTROL, launch_status_init(status, ninst, st));
    if (C.ss) TL(KKT_PHASE_ASSEMBLE, launch_jscale(di(), C, jitems, n_jitems, st));
    TL(KKT_PHASE_ASSEMBLE, launch_assemble(di(), C, kitems, n_kitems, st));
    TL(KKT_PHASE_ASSEMBLE, launch_assemble_heavy(di(), C, hitems, n_hitems, st));
    if (queue_sched) {
        const DepLists D = deps();
        // counters, ticket and the error latch (the latch is cleared only here)
        TL(KKT_PHASE_CONTROL, launch_fill_i32(dep_ctr, 0, 3 * (int64_t)D.nitems + 2, st));
        TL(KKT_PHASE_FACTOR, launch_factor_queue(di(), fdesc, D, std::min(D.nitems, 512), lds_factor, st));
    } else {
        // A level with few fronts leaves most compute units idle: its update
        // matrices then go to a launch of their own with one wave per 16 x 16
        // tile, where they are large enough to repay the launch. Wide levels
        // keep them in the factor kernel. Both paths give every entry the
        // same operations in the same order.
        for (size_t l = 0; l + 1 < lvl_ptr.size(); l++) {
            const int nf = lvl_large[l] - lvl_ptr[l], nlarge = lvl_ptr[l + 1] - lvl_large[l];
            if (nf > 0) {
                const bool split = split_update && nf < split_max_fronts && lvl_maxu[l] >= split_min_rows;
                // levels of narrow fronts: four-wave workgroups sized to the
                // level's own largest front, so several share a compute unit
                if (lvl_maxc[l] <= small_front_cols)
                    TL(KKT_PHASE_FACTOR,
                       launch_factor_small(di(), fdesc + lvl_ptr[l], nf, lvl_flds[l], split ? 0 : 1, st));
                else
                    TL(KKT_PHASE_FACTOR, launch_factor(di(), fdesc + lvl_ptr[l], nf, lds_factor, split ? 0 : 1, st));
                if (split)
                    TL(KKT_PHASE_FACTOR,
                       launch_update(di(), fdesc, upitems + up_ptr[l], upl_ptr[l] - up_ptr[l], st));
            }
            // large fronts: panels factored in HBM, then their update matrices by tiles
            if (nlarge > 0) {
                TL(KKT_PHASE_FACTOR,
                   launch_big_factor(di(), fdesc + lvl_large[l], nlarge, lvl_lmaxc[l], lvl_lmaxr[l], st));
                TL(KKT_PHASE_FACTOR, launch_update(di(), fdesc, upitems + upl_ptr[l], up_ptr[l + 1] - upl_ptr[l], st));
            }
        }
    }
    if (mode == 2) TL(KKT_PHASE_ASSEMBLE, launch_jcopy(di(), C, jitems, n_jitems, st));
    if (mode != 2 && aug_ready)
        TL(KKT_PHASE_ASSEMBLE, launch_keep_lifted(di(), C, jitems, n_jitems, mitems, n_mitems, st));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "refactor launch");
    factored = true;
    return KKT_OK;
}

void Engine::sweeps(hipStream_t st, int skip_done) {
    if (queue_sched) {
        const DepLists D = deps();
        TL(KKT_PHASE_CONTROL, launch_fill_i32(dep_ctr, 0, 3 * (int64_t)D.nitems + 1, st));
        TL(KKT_PHASE_FWD, launch_sweeps_queue(di(), fdesc, D, std::min(2 * D.nitems, 1024), lds_solve, skip_done, st));
        return;
    }
    const int nl = (int)lvl_ptr.size() - 1;
    for (int l = 0; l < nl; l++) {
        for (int k = sw_lvl[l]; k < sw_lvl[l + 1]; k++) {
            const SweepPart& P = sw_part[k];
            TL(KKT_PHASE_FWD, launch_fwd(di(), fdesc + P.begin, P.count, P.lds, skip_done, st));
        }
        if (lvl_large[l] < lvl_ptr[l + 1])
            TL(KKT_PHASE_FWD, launch_big_fwd(di(), fdesc + lvl_large[l], lvl_ptr[l + 1] - lvl_large[l], skip_done, st));
    }
    for (int l = nl - 1; l >= 0; l--) {
        if (lvl_large[l] < lvl_ptr[l + 1])
            TL(KKT_PHASE_BWD, launch_big_bwd(fdesc + lvl_large[l], lvl_ptr[l + 1] - lvl_large[l], skip_done, st));
        for (int k = sw_lvl[l]; k < sw_lvl[l + 1]; k++) {
            const SweepPart& P = sw_part[k];
            TL(KKT_PHASE_BWD, launch_bwd(fdesc + P.begin, P.count, P.lds, skip_done, st));
        }
    }
}

kkt_status Engine::read_status(int* st_out, int* bad_out) {
    hipError_t e = hipStreamSynchronize(last_stream);
    int derr = 0;
    if (e == hipSuccess) e = hipMemcpy(&derr, deps().err, sizeof(int), hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(hpin, status, (size_t)ninst * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "status read");
    return parse_status(derr, (const int*)hpin, st_out, bad_out);
}

// status words (2 per instance) and the queue schedule's error latch
kkt_status Engine::parse_status(int derr, const int* hs, int* st_out, int* bad_out) {
    if (derr) return fail(KKT_ERR_DEVICE, "a dependency wait of the queue schedule timed out");
    kkt_status worst = KKT_OK;
    for (int q = 0; q < ninst; q++) {
        const int code = hs[2 * q];
        int bad = -1;
        if (code == KKT_ERR_NOT_SPD && hs[2 * q + 1] >= 0 && hs[2 * q + 1] < syms[q]->n) bad = syms[q]->perm[hs[2 * q + 1]];
        if (st_out) st_out[q] = code;
        if (bad_out) bad_out[q] = bad;
        if (code != KKT_OK && worst == KKT_OK) worst = code;
    }
    return worst;
}

// first solve from the right-hand side (refinement state reset)
void Engine::solve_start(const Calls& C, int maxit, double tol, hipStream_t st) {
    TL(KKT_PHASE_CONTROL, launch_refine_reset(di(), ninst, tol, maxit, st));
    TL(KKT_PHASE_CONTROL, launch_fill_i32(ndone, 0, 1, st));
    TL(KKT_PHASE_PERMUTE, launch_perm_in(di(), C, nitems, n_nitems, PIN_B, st));
    sweeps(st, SKIP_NONE);
    TL(KKT_PHASE_PERMUTE, launch_perm_out(di(), C, nitems, n_nitems, POUT_X, st));
}

// residual + stop decision of every instance still refining
void Engine::refine_check(const Calls& C, hipStream_t st) {
    TL(KKT_PHASE_RESIDUAL, launch_residual(di(), C, nitems, n_nitems, st));
    TL(KKT_PHASE_CONTROL, launch_refine_decide(di(), ninst, ndone, st));
}

// one correction x += K^{-1} r of every instance still refining
void Engine::refine_correct(const Calls& C, hipStream_t st) {
    TL(KKT_PHASE_PERMUTE, launch_perm_in(di(), C, nitems, n_nitems, PIN_R, st));
    sweeps(st, SKIP_REFINE);
    TL(KKT_PHASE_PERMUTE, launch_perm_out(di(), C, nitems, n_nitems, POUT_X_UPDATE, st));
}

kkt_status Engine::solve(const Calls& C, int maxit, double tol, kkt_solve_info* infos, hipStream_t st) {
    last_stream = st;
    solve_start(C, maxit, tol, st);
    return solve_finish(C, 0, maxit, tol, infos, st);
}

// The same operations as the host-driven loop of solve_finish in its longest
// case (maxit + 1 checks, maxit corrections); the refinement kernels and the
// sweeps of an instance that has stopped return at once, so the result is
// the same bit for bit and nothing is read back.
void Engine::solve_rounds(const Calls& C, int maxit, hipStream_t st) {
    refine_check(C, st);
    for (int q = 0; q < maxit; q++) {
        refine_correct(C, st);
        refine_check(C, st);
    }
    TL(KKT_PHASE_PERMUTE, launch_refine_revert(di(), C, nitems, n_nitems, st));
}

// Host-driven refinement from round `iter0` on: check, stop when every
// instance is done, else correct. Then the better-of-last-two rule, the
// factor status and the per-instance reports.
kkt_status Engine::solve_finish(const Calls& C, int iter0, int maxit, double tol, kkt_solve_info* infos,
                                hipStream_t st) {
    // With several instances, one round of lookahead: the next correction
    // and check are queued before the host reads the current count of
    // stopped instances, so the GPU does not idle on the round trip. Every
    // refinement kernel skips stopped instances, so the extra queued round
    // changes no result. A single instance reads its decision first (after
    // its last correction a queued round would only delay the return).
    volatile int* hp = (volatile int*)hpin;
    hipError_t e = hipSuccess;
    if (!ctl_event && (e = hipEventCreateWithFlags(&ctl_event, hipEventDisableTiming)) != hipSuccess)
        return hip_fail(e, "refinement control event");
    refine_check(C, st);
    for (int iter = iter0; iter <= maxit + 1 && ninst == 1; iter++) {
        if ((e = hipMemcpyAsync((void*)hp, ndone, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(e, "refinement control");
        if (hp[0] >= ninst) break;
        refine_correct(C, st);
        refine_check(C, st);
    }
    for (int iter = iter0; iter <= maxit + 1 && ninst > 1; iter++) {
        // ndone after the check of round iter
        if ((e = hipMemcpyAsync((void*)hp, ndone, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipEventRecord(ctl_event, st)) != hipSuccess)
            return hip_fail(e, "refinement control");
        refine_correct(C, st);
        refine_check(C, st);
        if ((e = hipEventSynchronize(ctl_event)) != hipSuccess) return hip_fail(e, "refinement control");
        if (hp[0] >= ninst) break;
    }
    TL(KKT_PHASE_PERMUTE, launch_refine_revert(di(), C, nitems, n_nitems, st));
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "solve launch");
    // One synchronisation: the error latch, the status words and the
    // refinement records are copied behind the queued work, then read.
    char* hb = (char*)hpin;
    int* hderr = (int*)hb;
    const int* hs = (const int*)(hb + 64);
    const RefineState* hr = (const RefineState*)(hb + 64 + (((size_t)ninst * 8 + 63) & ~(size_t)63));
    if ((e = hipMemcpyAsync(hderr, deps().err, sizeof(int), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipMemcpyAsync((void*)hs, status, (size_t)ninst * 8, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (infos && (e = hipMemcpyAsync((void*)hr, rs, (size_t)ninst * sizeof(RefineState), hipMemcpyDeviceToHost,
                                      st)) != hipSuccess) ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(e, "solve read-back");
    // a failed factor makes the solve meaningless: report it
    kkt_status fst = parse_status(*hderr, hs, nullptr, nullptr);
    if (fst == KKT_ERR_DEVICE || fst == KKT_ERR_OOM) return fst;
    if (fst != KKT_OK) return fail(fst, "factor failed; solve result invalid");
    if (!infos) return KKT_OK;
    kkt_status worst = KKT_OK;
    for (int q = 0; q < ninst; q++) {
        const RefineState& S = hr[q];
        const bool rev = S.revert != 0;
        kkt_solve_info& inf = infos[q];
        inf.iters = rev ? S.it - 1 : S.it;
        inf.eta = rev ? S.eta_prev : S.eta;
        inf.omega = rev ? S.omega_prev : S.omega;
        inf.relres = rev ? S.relres_prev : S.relres;
        inf.status = inf.omega <= tol ? KKT_OK : KKT_ERR_NOT_CONVERGED;
        if (inf.status != KKT_OK) worst = inf.status;
    }
    return worst;
}

void Engine::drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
}

// Records refactor + first solve + `rounds` refinement rounds on a private
// stream. Kernels only (no memset or copy nodes); the per-launch timers are
// off while recording.
kkt_status Engine::capture(const Calls& C, int maxit, double tol, int rounds) {
    drop_graph();
    hipError_t e = hipSuccess;
    if (!cap_stream && (e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking)) != hipSuccess)
        return hip_fail(e, "capture stream");
    const bool timing = timer.on;
    timer.on = false;
    hipStream_t st = cap_stream;
    if ((e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal)) != hipSuccess) {
        timer.on = timing;
        return hip_fail(e, "begin capture");
    }
    kkt_status ks = refactor(C, st);
    if (ks == KKT_OK) {
        solve_start(C, maxit, tol, st);
        for (int q = 0; q < rounds; q++) {
            refine_check(C, st);
            refine_correct(C, st);
        }
    }
    hipGraph_t g = nullptr;
    const hipError_t ee = hipStreamEndCapture(st, &g);
    timer.on = timing;
    factored = false;  // nothing ran yet
    if (ks != KKT_OK) {
        if (g) (void)hipGraphDestroy(g);
        return ks;
    }
    if (ee != hipSuccess) return hip_fail(ee, "end capture");
    graph = g;
    if ((e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0)) != hipSuccess) {
        drop_graph();
        return hip_fail(e, "graph instantiation");
    }
    g_calls = C;
    g_rounds = rounds;
    g_maxit = maxit;
    g_tol = tol;
    return KKT_OK;
}

kkt_status Engine::replay(kkt_solve_info* infos, hipStream_t st) {
    if (!gexec) return fail(KKT_ERR_STATE, "no captured graph");
    last_stream = st;
    hipError_t e = hipGraphLaunch(gexec, st);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    mode = 1;
    gamma = 0.0;
    factored = true;
    return solve_finish(g_calls, g_rounds, g_maxit, g_tol, infos, st);
}

// CG iteration k: the stop tests of dy_k and the direction (k_cg_dir), the
// eta test when asked for, then S_gamma p_k and the update; iteration maxit
// is the last test only.
void Engine::cg_iteration(int k, int maxit, bool eta_test, hipStream_t st) {
    TL(KKT_PHASE_CG, launch_cg_dir(di(), nitems, n_nitems, k, ndone, st));
    if (k >= maxit) return;
    if (eta_test) TL(KKT_PHASE_CONTROL, launch_cg_eta_test(di(), cg_calls, ninst, k, ndone, st));
    sweeps(st, SKIP_CG);
    TL(KKT_PHASE_CG, launch_cg_q(di(), cg_calls, mitems, n_mitems, k, st));
    TL(KKT_PHASE_CG, launch_cg_upd(di(), cg_calls, mitems, n_mitems, k, ndone, st));
}

kkt_status Engine::cg_schur(const Calls& C, double tol, int maxit, double eta_tol, kkt_cg_info* info,
                            hipStream_t st) {
    last_stream = st;
    cg_calls = C;
    int* nd = ndone;
    const bool eta_test = eta_tol > 0.0;
    TL(KKT_PHASE_CONTROL, launch_fill_i32(nd, 0, 1, st));
    // f_gamma = f + gamma J^T g (pivot order), c = J K_gamma^{-1} f_gamma - g
    TL(KKT_PHASE_CG, launch_cg_fg(di(), C, nitems, n_nitems, tol, maxit, eta_tol, st));
    sweeps(st, SKIP_NONE);
    TL(KKT_PHASE_CG, launch_cg_c(di(), C, mitems, n_mitems, ninst, st));
    hipError_t e = hipSuccess;
    if (!info) {
        // asynchronous: every iteration is queued; once an instance's CG has
        // stopped, its kernels of the later iterations return at once
        for (int k = 0; k <= maxit; k++) cg_iteration(k, maxit, eta_test, st);
    } else {
        // With one iteration of lookahead: iteration k+1 is queued before
        // the host reads the count of stopped instances after iteration k.
        // The kernels of a stopped instance return at once, so the queued
        // iteration changes nothing.
        volatile int* slot[2] = {(volatile int*)hpin, (volatile int*)hpin + 16};
        hipEvent_t ev[2] = {ctl_event, ctl_event2};
        auto issue = [&](int k) -> hipError_t {
            cg_iteration(k, maxit, eta_test, st);
            hipError_t r = hipMemcpyAsync((void*)slot[k & 1], nd, 4, hipMemcpyDeviceToHost, st);
            if (r == hipSuccess) r = hipEventRecord(ev[k & 1], st);
            return r;
        };
        kkt_status fst = read_status(nullptr, nullptr);
        if (fst != KKT_OK) return fail(fst, "factor failed; solve refused");
        int issued = 0;
        while (issued <= maxit && issued < 2)
            if ((e = issue(issued++)) != hipSuccess) return hip_fail(e, "cg control");
        for (int k = 0; k < issued; k++) {
            if ((e = hipEventSynchronize(ev[k & 1])) != hipSuccess) return hip_fail(e, "cg control");
            if (*slot[k & 1] >= ninst) break;
            if (issued <= maxit && (e = issue(issued++)) != hipSuccess) return hip_fail(e, "cg control");
        }
    }
    // dx = K_gamma^{-1}(f_gamma - J^T dy), then the saddle-system residual and eta
    TL(KKT_PHASE_CG, launch_cg_dxrhs(di(), C, nitems, n_nitems, st));
    sweeps(st, SKIP_NONE);
    TL(KKT_PHASE_PERMUTE, launch_perm_out(di(), C, nitems, n_nitems, POUT_DX, st));
    TL(KKT_PHASE_RESIDUAL, launch_cg_residual(di(), C, nitems, n_nitems, mitems, n_mitems, ninst, st));
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "cg launch");
    if (!info) return KKT_OK;
    e = hipMemcpyAsync(hpin, cg, sizeof(CgState), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "cg info");
    CgState G;
    std::memcpy(&G, hpin, sizeof(G));
    info->iters = G.it;
    info->rel_res = G.cnorm > 0 ? std::sqrt(G.rr_new) / G.cnorm : 0.0;
    info->eta = G.eta;
    info->eta_stop = G.eta_stop;
    info->status = G.status == 0 ? (G.done ? KKT_OK : KKT_ERR_NOT_CONVERGED) : G.status;
    if (info->status != KKT_OK)
        return fail(info->status, info->status == KKT_ERR_BREAKDOWN ? "CG breakdown (p^T S p <= 0)"
                                                                    : "CG reached its iteration limit");
    return KKT_OK;
}

// Augmented system (Lifted-KKT): condensed solve with refinement, recovery of
// ds and dz, then refinement on the full system with the host reading each
// stop decision.
kkt_status Engine::solve_augmented(const AugCall& A, int maxit, double tol, kkt_aug_info* info, hipStream_t st) {
    last_stream = st;
    const int ni = 10;  // refinement of the first condensed solve: kkt_solve's defaults
    const double itol = 1e-14;
    TL(KKT_PHASE_RESIDUAL, launch_aug_rhs(di(), A, nitems, n_nitems, 0, st));
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.b = aug_b;
    C.x = A.dx;
    kkt_solve_info inner{};
    kkt_status ks = solve(C, ni, itol, &inner, st);
    if (ks != KKT_OK && ks != KKT_ERR_NOT_CONVERGED) return ks;
    TL(KKT_PHASE_RESIDUAL, launch_aug_recover(di(), A, nitems, n_nitems, mitems, n_mitems, 0, st));
    TL(KKT_PHASE_CONTROL, launch_aug_reset(di(), ninst, tol, maxit, st));
    Calls Ct;
    std::memset(&Ct, 0, sizeof(Ct));
    Ct.b = aug_b;
    Ct.x = aug_t;
    AugState S{};
    hipError_t e = hipSuccess;
    for (int round = 0; round <= maxit + 1; round++) {
        TL(KKT_PHASE_RESIDUAL, launch_aug_check(di(), A, nitems, n_nitems, mitems, n_mitems, ninst, st));
        if ((e = hipMemcpyAsync(hpin, aug, sizeof(AugState), hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(e, "augmented refinement control");
        std::memcpy(&S, hpin, sizeof(S));
        if (S.done) break;
        // correction: condensed right-hand side of e, one solve with the
        // factor, recovery of the slack and multiplier parts, update
        TL(KKT_PHASE_RESIDUAL, launch_aug_rhs(di(), A, nitems, n_nitems, 1, st));
        solve_start(Ct, 0, 0.0, st);
        TL(KKT_PHASE_RESIDUAL, launch_aug_recover(di(), A, nitems, n_nitems, mitems, n_mitems, 1, st));
    }
    TL(KKT_PHASE_PERMUTE, launch_aug_revert(di(), A, nitems, n_nitems, mitems, n_mitems, st));
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(st)) != hipSuccess)
        return hip_fail(e, "augmented solve");
    const bool rev = S.revert != 0;
    const double om = rev ? S.omega_prev : S.omega;
    if (info) {
        info->iters = rev ? S.it - 1 : S.it;
        info->eta = rev ? S.eta_prev : S.eta;
        info->omega = om;
        info->inner_iters = inner.iters;
        info->status = om <= tol ? KKT_OK : KKT_ERR_NOT_CONVERGED;
    }
    return om <= tol ? KKT_OK : fail(KKT_ERR_NOT_CONVERGED, "augmented refinement stopped above tol");
}

}  // namespace kkt

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

void kkt_options_default(kkt_options* opt) {
    if (!opt) return;
    opt->ordering = KKT_ORDER_AUTO;
    opt->nd_leaf = 0;
    opt->max_super = 96;
    opt->relax_small = 16;
    opt->relax_frac = 0.5;
    opt->front_lds_max = 0;
}

const char* kkt_status_string(kkt_status s) {
    switch (s) {
        case KKT_OK: return "OK";
        case KKT_ERR_INVALID_ARG: return "INVALID_ARG";
        case KKT_ERR_PATTERN: return "PATTERN";
        case KKT_ERR_STATE: return "STATE";
        case KKT_ERR_NOT_SPD: return "NOT_SPD";
        case KKT_ERR_NONFINITE: return "NONFINITE";
        case KKT_ERR_NOT_CONVERGED: return "NOT_CONVERGED";
        case KKT_ERR_BREAKDOWN: return "BREAKDOWN";
        case KKT_ERR_OOM: return "OOM";
        case KKT_ERR_BUDGET: return "BUDGET";
        case KKT_ERR_DEVICE: return "DEVICE";
        default: return "UNKNOWN";
    }
}

const char* kkt_last_error(void) { return g_last_error.c_str(); }

kkt_status kkt_symbolic_analyze(int32_t n, int32_t m, const int32_t* w_rowptr, const int32_t* w_colind,
                                const int32_t* j_rowptr, const int32_t* j_colind, const kkt_options* opt,
                                kkt_symbolic** out) {
    if (!out) return fail(KKT_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    kkt_options o;
    kkt_options_default(&o);
    if (opt) o = *opt;
    if (o.ordering < 0 || o.ordering > 2) return fail(KKT_ERR_INVALID_ARG, "unknown ordering");
    SymOptions so;
    so.ordering = o.ordering;
    so.nd_leaf = o.nd_leaf;
    so.max_super = o.max_super > 0 ? o.max_super : 96;
    if (so.max_super > 128) return fail(KKT_ERR_INVALID_ARG, "max_super must be <= 128");
    so.relax_small = o.relax_small == 0 ? 16 : (o.relax_small < 0 ? 0 : o.relax_small);
    so.relax_frac = o.relax_frac < 0 ? 0.5 : o.relax_frac;
    if (o.front_lds_max < 0) return fail(KKT_ERR_INVALID_ARG, "negative front_lds_max");
    // at least one 16 x 16 block of a front must fit
    so.lds_bytes = o.front_lds_max == 0 ? kMaxDynLds : std::min(std::max(o.front_lds_max, 4096), kMaxDynLds);
    kkt_symbolic* sym = new (std::nothrow) kkt_symbolic;
    if (!sym) return fail(KKT_ERR_OOM, "host allocation");
    std::string err;
    int st;
    try {
        st = analyze(n, m, w_rowptr, w_colind, j_rowptr, j_colind, so, sym->S, err);
    } catch (const std::bad_alloc&) {
        st = KKT_ERR_OOM;
        err = "host allocation during analysis";
    }
    if (st != KKT_OK) {
        delete sym;
        return fail(st, err);
    }
    *out = sym;
    return KKT_OK;
}

kkt_status kkt_symbolic_get_stats(const kkt_symbolic* sym, kkt_symbolic_stats* out) {
    if (!sym || !out) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    const Symbolic& S = sym->S;
    out->n = S.n;
    out->m = S.m;
    out->nsuper = S.ns;
    out->levels = S.nlevels;
    out->max_rows = S.max_nrow;
    out->max_cols = S.max_ncol;
    out->nnz_k = S.nnzk;
    int64_t nl = 0;
    for (int s = 0; s < S.ns; s++) {
        int64_t r = S.sn_nrow[s], c = S.sn_ncol[s];
        nl += r * c - c * (c - 1) / 2;
    }
    out->nnz_l = nl;
    out->nnz_l_exact = S.nnzl_exact;
    out->n_pairs = (int64_t)S.pair_a.size();
    out->flops = S.flops;
    out->flops_exact = S.flops_exact;
    out->analyze_seconds = S.analyze_seconds;
    out->large_fronts = S.n_large;
    return KKT_OK;
}

kkt_status kkt_symbolic_get_perm(const kkt_symbolic* sym, int32_t* perm) {
    if (!sym || !perm) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    std::copy(sym->S.perm.begin(), sym->S.perm.end(), perm);
    return KKT_OK;
}

kkt_status kkt_symbolic_get_supernodes(const kkt_symbolic* sym, int32_t* col_ptr, int32_t* parent, int32_t* nrows) {
    if (!sym) return fail(KKT_ERR_INVALID_ARG, "NULL symbolic");
    const Symbolic& S = sym->S;
    if (col_ptr) std::copy(S.sn_col0.begin(), S.sn_col0.end(), col_ptr);
    if (parent) std::copy(S.sn_parent.begin(), S.sn_parent.end(), parent);
    if (nrows) std::copy(S.sn_nrow.begin(), S.sn_nrow.end(), nrows);
    return KKT_OK;
}

void kkt_symbolic_destroy(kkt_symbolic* sym) { delete sym; }

kkt_status kkt_factor_create(const kkt_symbolic* sym, kkt_factor** out) {
    if (!sym || !out) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    *out = nullptr;
    kkt_factor* f = new (std::nothrow) kkt_factor;
    if (!f) return fail(KKT_ERR_OOM, "host allocation");
    f->sym = sym;
    f->eng.single_storage = true;
    kkt_status st = f->eng.init_owned({&sym->S});
    if (st != KKT_OK) {
        delete f;
        return st;
    }
    *out = f;
    return KKT_OK;
}

void kkt_factor_destroy(kkt_factor* f) { delete f; }

static kkt_status check_values(const Engine& E, const double* w_vals, const double* j_vals, const double* sigma_x,
                               const double* sigma_s, double gamma) {
    const int64_t nw = E.w_ofs[E.ninst], nj = E.j_ofs[E.ninst], n = E.n_ofs[E.ninst], m = E.m_ofs[E.ninst];
    if ((nw > 0 && !w_vals) || (nj > 0 && !j_vals) || (n > 0 && !sigma_x))
        return fail(KKT_ERR_INVALID_ARG, "NULL value array");
    if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(KKT_ERR_INVALID_ARG, "gamma must be finite and >= 0");
    if (E.n_eq > 0) {
        if (!(gamma > 0.0) || (m > 0 && !sigma_s))
            return fail(KKT_ERR_INVALID_ARG, "with equality rows set, refactor needs gamma > 0 and sigma_s");
        return KKT_OK;
    }
    if (gamma == 0.0 && m > 0 && !sigma_s) return fail(KKT_ERR_INVALID_ARG, "Lifted-KKT (gamma == 0) needs sigma_s");
    if (gamma > 0.0 && sigma_s) return fail(KKT_ERR_INVALID_ARG, "HyKKT (gamma > 0) takes sigma_s = NULL");
    return KKT_OK;
}

// values of one refactor call (general HyKKT when equality rows are set)
static Calls refactor_calls(const Engine& E, const double* w_vals, const double* j_vals, const double* sigma_x,
                            const double* sigma_s, double gamma) {
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.w = w_vals; C.jv = j_vals; C.sx = sigma_x; C.gamma = gamma;
    C.ss = (gamma == 0.0 || E.n_eq > 0) ? sigma_s : nullptr;
    C.eqm = E.n_eq > 0 ? (const int*)E.eqmask.p : nullptr;
    return C;
}

kkt_status kkt_refactor(kkt_factor* f, const double* w_vals, const double* j_vals, const double* sigma_x,
                        const double* sigma_s, double gamma, void* stream) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    kkt_status st = check_values(f->eng, w_vals, j_vals, sigma_x, sigma_s, gamma);
    if (st) return st;
    return f->eng.refactor(refactor_calls(f->eng, w_vals, j_vals, sigma_x, sigma_s, gamma), (hipStream_t)stream);
}

void kkt_inertia_opts_default(kkt_inertia_opts* o) {
    if (!o) return;
    o->delta_first = 1e-4;
    o->delta_min = 1e-20;
    o->delta_max = 1e40;
    o->kappa_minus = 1.0 / 3.0;
    o->kappa_plus = 8.0;
    o->kappa_plus_first = 100.0;
}

kkt_status kkt_refactor_inertia(kkt_factor* f, const double* w_vals, const double* j_vals, const double* sigma_x,
                                const double* sigma_s, double gamma, const kkt_inertia_opts* opts,
                                kkt_inertia_info* info, void* stream) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    kkt_status st = check_values(f->eng, w_vals, j_vals, sigma_x, sigma_s, gamma);
    if (st) return st;
    kkt_inertia_opts o;
    kkt_inertia_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.delta_first > 0.0) || !(o.delta_min >= 0.0) || !(o.delta_max >= o.delta_first) ||
        !(o.kappa_minus > 0.0) || !(o.kappa_plus > 1.0) || !(o.kappa_plus_first > 1.0))
        return fail(KKT_ERR_INVALID_ARG, "bad inertia-correction options");
    Engine& E = f->eng;
    Calls C = refactor_calls(E, w_vals, j_vals, sigma_x, sigma_s, gamma);
    const hipStream_t s = (hipStream_t)stream;
    int trials = 0;
    auto attempt = [&](double delta, int* code) -> kkt_status {
        C.delta = delta;
        kkt_status r = E.refactor(C, s);
        if (r != KKT_OK) return r;
        trials++;
        int bad = -1;
        r = E.read_status(code, &bad);
        return (r == KKT_ERR_DEVICE || r == KKT_ERR_OOM) ? r : KKT_OK;
    };
    int code = 0;
    double delta = 0.0;
    if ((st = attempt(0.0, &code)) != KKT_OK) return st;
    if (code == KKT_ERR_NOT_SPD) {
        const bool first = E.delta_last == 0.0;
        delta = first ? o.delta_first : std::max(o.delta_min, o.kappa_minus * E.delta_last);
        for (;;) {
            if ((st = attempt(delta, &code)) != KKT_OK) return st;
            if (code != KKT_ERR_NOT_SPD) break;
            delta *= first ? o.kappa_plus_first : o.kappa_plus;
            if (delta > o.delta_max) break;
        }
        if (code == KKT_OK) E.delta_last = delta;
    }
    if (info) {
        info->status = code;
        info->trials = trials;
        info->delta = code == KKT_OK ? delta : -1.0;
    }
    if (code != KKT_OK)
        return fail(code, code == KKT_ERR_NOT_SPD ? "no delta up to delta_max makes K positive definite"
                                                  : "factor status " + std::string(kkt_status_string(code)));
    return KKT_OK;
}

kkt_status kkt_solve_augmented(kkt_factor* f, const double* r1, const double* r2, const double* r4, double* dx,
                               double* ds, double* dz, const kkt_refine_opts* ro, kkt_aug_info* info,
                               void* stream) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    const Symbolic& S = f->sym->S;
    if ((S.n > 0 && (!r1 || !dx)) || (S.m > 0 && (!r2 || !r4 || !ds || !dz)))
        return fail(KKT_ERR_INVALID_ARG, "NULL vector");
    if (!f->eng.factored || f->eng.mode != 1) return fail(KKT_ERR_STATE, "the augmented solve needs a Lifted-KKT factor");
    if (!f->eng.aug_ready)
        return fail(KKT_ERR_STATE, "the factor was refactored without kkt_factor_keep_augmented(f, 1)");
    const int maxit = ro ? ro->max_iter : 10;
    const double tol = ro ? ro->tol : 1e-14;
    if (maxit < 0 || !(tol >= 0.0)) return fail(KKT_ERR_INVALID_ARG, "bad refinement options");
    kkt_status fst = f->eng.read_status(nullptr, nullptr);
    if (fst != KKT_OK) return fail(fst, "factor failed; solve refused");
    AugCall A{r1, r2, r4, dx, ds, dz};
    return f->eng.solve_augmented(A, maxit, tol, info, (hipStream_t)stream);
}

kkt_status kkt_status_sync(kkt_factor* f, kkt_factor_info* info) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    int code = 0, bad = -1;
    kkt_status st = f->eng.read_status(&code, &bad);
    if (st == KKT_ERR_DEVICE || st == KKT_ERR_OOM) return st;
    if (info) { info->status = code; info->bad_col = bad; }
    if (code != KKT_OK) g_last_error = std::string("factor status ") + kkt_status_string(code);
    return code;
}

kkt_status kkt_solve(kkt_factor* f, const double* b, double* x, const kkt_refine_opts* ro, kkt_solve_info* info,
                     void* stream) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    const int n = f->sym->S.n;
    if (n > 0 && (!b || !x)) return fail(KKT_ERR_INVALID_ARG, "NULL vector");
    if (b == x && n > 0) return fail(KKT_ERR_INVALID_ARG, "x aliases b");
    if (!f->eng.factored) return fail(KKT_ERR_STATE, "solve before refactor");
    const int maxit = ro ? ro->max_iter : 10;
    const double tol = ro ? ro->tol : 1e-14;
    if (maxit < 0 || !(tol >= 0.0)) return fail(KKT_ERR_INVALID_ARG, "bad refinement options");
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.b = b;
    C.x = x;
    Engine& E = f->eng;
    const hipStream_t st = (hipStream_t)stream;
    if (info) return E.solve(C, maxit, tol, info, st);
    E.last_stream = st;
    E.solve_start(C, maxit, tol, st);
    E.solve_rounds(C, maxit, st);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? KKT_OK : hip_fail(e, "solve launch");
}

void kkt_cg_opts_default(kkt_cg_opts* o) {
    if (!o) return;
    o->tol = 1e-10;
    o->maxit = 200;
    o->eta_tol = 0.0;
}

kkt_status kkt_cg_schur(kkt_factor* f, const double* fv, const double* g, const kkt_cg_opts* opts, double* dx,
                        double* dy, kkt_cg_info* info, void* stream) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    const Symbolic& S = f->sym->S;
    if ((S.n > 0 && (!fv || !dx)) || (S.m > 0 && (!g || !dy))) return fail(KKT_ERR_INVALID_ARG, "NULL vector");
    if (S.m > S.n) return fail(KKT_ERR_INVALID_ARG, "the Schur system needs m <= n (J of full row rank)");
    if (!f->eng.factored || f->eng.mode < 2) return fail(KKT_ERR_STATE, "cg_schur needs a K_gamma factor");
    kkt_cg_opts o;
    kkt_cg_opts_default(&o);
    if (opts) o = *opts;
    if (o.maxit < 0 || !(o.tol >= 0.0) || !(o.eta_tol >= 0.0)) return fail(KKT_ERR_INVALID_ARG, "bad CG options");
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.gamma = f->eng.gamma;
    C.eqm = f->eng.mode == 3 ? (const int*)f->eng.eqmask.p : nullptr;
    C.f = fv; C.g = g; C.dx = dx; C.dy = dy;
    return f->eng.cg_schur(C, o.tol, o.maxit, o.eta_tol, info, (hipStream_t)stream);
}

kkt_status kkt_factor_keep_augmented(kkt_factor* f, int32_t enable) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    f->eng.keep_aug = enable != 0;
    return KKT_OK;
}

kkt_status kkt_factor_set_equality_rows(kkt_factor* f, const int32_t* rows, int32_t count) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    const int m = f->sym->S.m;
    if (count < 0 || count > m || (count > 0 && !rows)) return fail(KKT_ERR_INVALID_ARG, "bad equality-row list");
    std::vector<int> mask(std::max(m, 1), 0);
    for (int k = 0; k < count; k++) {
        const int r = rows[k];
        if (r < 0 || r >= m || mask[r]) return fail(KKT_ERR_INVALID_ARG, "equality row out of range or repeated");
        mask[r] = 1;
    }
    Engine& E = f->eng;
    hipError_t e = hipSuccess;
    if (!E.eqmask.p && (e = E.eqmask.alloc(mask.size() * sizeof(int))) != hipSuccess)
        return hip_fail(e, "equality-row mask");
    if ((e = hipMemcpy(E.eqmask.p, mask.data(), mask.size() * sizeof(int), hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail(e, "equality-row mask upload");
    E.n_eq = count;
    E.factored = false;  // the next refactor defines the mode
    return KKT_OK;
}

kkt_status kkt_matvec(kkt_factor* f, const double* x, double* y, void* stream) {
    if (!f || (!x && f->sym->S.n > 0) || (!y && f->sym->S.n > 0)) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    if (!f->eng.factored) return fail(KKT_ERR_STATE, "matvec before refactor");
    Engine& E = f->eng;
    LaunchTimer& timer = E.timer;
    hipStream_t st = (hipStream_t)stream;
    TL(KKT_PHASE_RESIDUAL, launch_matvec(E.di(), x, y, E.nitems, E.n_nitems, st));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? KKT_OK : hip_fail(e, "matvec launch");
}

static kkt_status timing_read(Engine& E, kkt_timing* out) {
    int launches[KKT_NPHASES];
    hipError_t e = E.timer.read(out->ms, launches, KKT_NPHASES);
    if (e != hipSuccess) return hip_fail(e, "timer read");
    for (int q = 0; q < KKT_NPHASES; q++) out->launches[q] = launches[q];
    return KKT_OK;
}

kkt_status kkt_factor_set_timing(kkt_factor* f, int32_t enable) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    f->eng.timer.on = enable != 0;
    return KKT_OK;
}

kkt_status kkt_factor_set_schedule(kkt_factor* f, int32_t schedule) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    if (schedule != KKT_SCHEDULE_LEVELS && schedule != KKT_SCHEDULE_QUEUE)
        return fail(KKT_ERR_INVALID_ARG, "unknown schedule");
    if (schedule == KKT_SCHEDULE_QUEUE && f->eng.n_large > 0)
        return fail(KKT_ERR_INVALID_ARG, "the queue schedule needs every front in LDS (this pattern has large fronts)");
    f->eng.queue_sched = schedule == KKT_SCHEDULE_QUEUE;
    return KKT_OK;
}

kkt_status kkt_factor_set_update_split(kkt_factor* f, int32_t max_fronts, int32_t min_rows) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    if (max_fronts < 0 || min_rows < 0) return fail(KKT_ERR_INVALID_ARG, "negative split threshold");
    f->eng.split_max_fronts = max_fronts;
    f->eng.split_min_rows = min_rows;
    return KKT_OK;
}

kkt_status kkt_factor_set_small_fronts(kkt_factor* f, int32_t max_cols) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    if (max_cols < 0) return fail(KKT_ERR_INVALID_ARG, "negative column threshold");
    f->eng.small_front_cols = max_cols;
    return KKT_OK;
}

kkt_status kkt_factor_read_timing(kkt_factor* f, kkt_timing* out) {
    if (!f || !out) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    return timing_read(f->eng, out);
}

// ---------------------------------------------------------------------------
// batches
// ---------------------------------------------------------------------------
kkt_status kkt_batch_create(int32_t count, const kkt_symbolic* const* syms, kkt_batch** out) {
    if (!out || count < 1 || !syms) return fail(KKT_ERR_INVALID_ARG, "bad batch arguments");
    *out = nullptr;
    std::vector<const Symbolic*> v(count);
    for (int q = 0; q < count; q++) {
        if (!syms[q]) return fail(KKT_ERR_INVALID_ARG, "NULL symbolic in batch");
        v[q] = &syms[q]->S;
    }
    kkt_batch* b = new (std::nothrow) kkt_batch;
    if (!b) return fail(KKT_ERR_OOM, "host allocation");
    b->syms.assign(syms, syms + count);
    kkt_status st = b->eng.init_owned(v);
    if (st != KKT_OK) {
        delete b;
        return st;
    }
    *out = b;
    return KKT_OK;
}

void kkt_batch_destroy(kkt_batch* b) { delete b; }

kkt_status kkt_batch_offsets(const kkt_batch* b, int64_t* n_ofs, int64_t* m_ofs, int64_t* w_ofs, int64_t* j_ofs) {
    if (!b) return fail(KKT_ERR_INVALID_ARG, "NULL batch");
    const Engine& E = b->eng;
    if (n_ofs) std::copy(E.n_ofs.begin(), E.n_ofs.end(), n_ofs);
    if (m_ofs) std::copy(E.m_ofs.begin(), E.m_ofs.end(), m_ofs);
    if (w_ofs) std::copy(E.w_ofs.begin(), E.w_ofs.end(), w_ofs);
    if (j_ofs) std::copy(E.j_ofs.begin(), E.j_ofs.end(), j_ofs);
    return KKT_OK;
}

kkt_status kkt_batch_refactor(kkt_batch* b, const double* w_vals, const double* j_vals, const double* sigma_x,
                              const double* sigma_s, void* stream) {
    if (!b) return fail(KKT_ERR_INVALID_ARG, "NULL batch");
    kkt_status st = check_values(b->eng, w_vals, j_vals, sigma_x, sigma_s, 0.0);
    if (st) return st;
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.w = w_vals; C.jv = j_vals; C.sx = sigma_x; C.ss = sigma_s;
    return b->eng.refactor(C, (hipStream_t)stream);
}

kkt_status kkt_batch_solve(kkt_batch* b, const double* rhs, double* x, const kkt_refine_opts* ro,
                           kkt_solve_info* infos, void* stream) {
    if (!b) return fail(KKT_ERR_INVALID_ARG, "NULL batch");
    const int64_t n = b->eng.n_ofs[b->eng.ninst];
    if (n > 0 && (!rhs || !x)) return fail(KKT_ERR_INVALID_ARG, "NULL vector");
    if (rhs == x && n > 0) return fail(KKT_ERR_INVALID_ARG, "x aliases b");
    if (!b->eng.factored) return fail(KKT_ERR_STATE, "solve before refactor");
    const int maxit = ro ? ro->max_iter : 10;
    const double tol = ro ? ro->tol : 1e-14;
    if (maxit < 0 || !(tol >= 0.0)) return fail(KKT_ERR_INVALID_ARG, "bad refinement options");
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.b = rhs;
    C.x = x;
    return b->eng.solve(C, maxit, tol, infos, (hipStream_t)stream);
}

kkt_status kkt_batch_capture(kkt_batch* b, const double* w_vals, const double* j_vals, const double* sigma_x,
                             const double* sigma_s, const double* rhs, double* x, const kkt_refine_opts* ro,
                             int32_t rounds) {
    if (!b) return fail(KKT_ERR_INVALID_ARG, "NULL batch");
    Engine& E = b->eng;
    kkt_status st = check_values(E, w_vals, j_vals, sigma_x, sigma_s, 0.0);
    if (st) return st;
    const int64_t n = E.n_ofs[E.ninst];
    if (n > 0 && (!rhs || !x)) return fail(KKT_ERR_INVALID_ARG, "NULL vector");
    if (rhs == x && n > 0) return fail(KKT_ERR_INVALID_ARG, "x aliases b");
    const int maxit = ro ? ro->max_iter : 10;
    const double tol = ro ? ro->tol : 1e-14;
    if (maxit < 0 || !(tol >= 0.0)) return fail(KKT_ERR_INVALID_ARG, "bad refinement options");
    if (rounds < 0 || rounds > maxit + 1) return fail(KKT_ERR_INVALID_ARG, "rounds outside 0..max_iter+1");
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.w = w_vals; C.jv = j_vals; C.sx = sigma_x; C.ss = sigma_s;
    C.b = rhs;
    C.x = x;
    return E.capture(C, maxit, tol, rounds);
}

kkt_status kkt_batch_replay(kkt_batch* b, kkt_solve_info* infos, void* stream) {
    if (!b) return fail(KKT_ERR_INVALID_ARG, "NULL batch");
    return b->eng.replay(infos, (hipStream_t)stream);
}

kkt_status kkt_batch_set_schedule(kkt_batch* b, int32_t schedule) {
    if (!b) return fail(KKT_ERR_INVALID_ARG, "NULL batch");
    if (schedule != KKT_SCHEDULE_LEVELS && schedule != KKT_SCHEDULE_QUEUE)
        return fail(KKT_ERR_INVALID_ARG, "unknown schedule");
    if (schedule == KKT_SCHEDULE_QUEUE && b->eng.n_large > 0)
        return fail(KKT_ERR_INVALID_ARG, "the queue schedule needs every front in LDS (this pattern has large fronts)");
    b->eng.queue_sched = schedule == KKT_SCHEDULE_QUEUE;
    return KKT_OK;
}

kkt_status kkt_batch_set_update_split(kkt_batch* b, int32_t max_fronts, int32_t min_rows) {
    if (!b) return fail(KKT_ERR_INVALID_ARG, "NULL batch");
    if (max_fronts < 0 || min_rows < 0) return fail(KKT_ERR_INVALID_ARG, "negative split threshold");
    b->eng.split_max_fronts = max_fronts;
    b->eng.split_min_rows = min_rows;
    return KKT_OK;
}

kkt_status kkt_batch_set_small_fronts(kkt_batch* b, int32_t max_cols) {
    if (!b) return fail(KKT_ERR_INVALID_ARG, "NULL batch");
    if (max_cols < 0) return fail(KKT_ERR_INVALID_ARG, "negative column threshold");
    b->eng.small_front_cols = max_cols;
    return KKT_OK;
}

kkt_status kkt_batch_status(kkt_batch* b, int32_t* status, int32_t* bad_col) {
    if (!b) return fail(KKT_ERR_INVALID_ARG, "NULL batch");
    return b->eng.read_status(status, bad_col);
}

kkt_status kkt_batch_set_timing(kkt_batch* b, int32_t enable) {
    if (!b) return fail(KKT_ERR_INVALID_ARG, "NULL batch");
    b->eng.timer.on = enable != 0;
    return KKT_OK;
}

kkt_status kkt_batch_read_timing(kkt_batch* b, kkt_timing* out) {
    if (!b || !out) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    return timing_read(b->eng, out);
}

}  // extern "C"
