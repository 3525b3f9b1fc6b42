// C ABI of libkkt (declared in include/kkt.h): symbolic objects, device
// factors, the Lifted-KKT solve with Richardson refinement and the HyKKT
// Schur-complement CG (Pacaud & Shin, arXiv 2403.15913, sections "Condensed
// KKT system" and "Hybrid linear solver").
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/kkt.h"
#include "api_internal.hpp"

using namespace kkt;

// Launch `expr` on stream `st`, bracketed by timer events when timing is on.
#define TL(ph, expr)                               \
    do {                                           \
        if (f->timer.on) f->timer.begin(ph, st);   \
        expr;                                      \
        if (f->timer.on) f->timer.end(st);         \
    } while (0)

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
#define UP(buf, vec, field, type)                  \
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
    UP(b_chptr, ch_ptr, ch_ptr, int)
    UP(b_chlist, ch_list, ch_list, int)
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
    UP(b_spe, sp_e, sp_e, int)
    UP(b_spcol, sp_col, sp_col, int)
    UP(b_jptr, j_ptr, j_ptr, int)
    UP(b_jcol, j_col, j_col, int)
    UP(b_jtptr, jt_ptr, jt_ptr, int)
    UP(b_jte, jt_e, jt_e, int)
    UP(b_jtrow, jt_row, jt_row, int)
#undef UP
    // level lists and row-block work items (single instance 0)
    std::vector<WorkItem> sn(S.ns), nb, mb, kb;
    for (int q = 0; q < S.ns; q++) sn[q] = WorkItem{0, S.lvl_list[q]};
    for (int i = 0; i < S.n; i += kBlock) nb.push_back(WorkItem{0, i});
    for (int i = 0; i < S.m; i += kBlock) mb.push_back(WorkItem{0, i});
    for (int64_t i = 0; i < S.nnzk; i += kBlock) kb.push_back(WorkItem{0, (int)i});
    if ((e = upload(b_snitems, sn)) != hipSuccess) return e;
    if ((e = upload(b_nitems, nb)) != hipSuccess) return e;
    if ((e = upload(b_mitems, mb)) != hipSuccess) return e;
    if ((e = upload(b_kitems, kb)) != hipSuccess) return e;
    n_nitems = (int)nb.size();
    n_mitems = (int)mb.size();
    n_kitems = (int)kb.size();
    lvl_ptr = S.lvl_ptr;
    size_t lf = 0, ls = 0;
    for (int s = 0; s < S.ns; s++) {
        size_t r = S.sn_nrow[s], c = S.sn_ncol[s];
        lf = std::max(lf, r * c * 8);
        ls = std::max(ls, (r * c + r) * 8);
    }
    lds_factor = lf;
    lds_solve = ls;
    return hipSuccess;
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
    SymOptions so;
    so.ordering = o.ordering;
    so.nd_leaf = o.nd_leaf;
    so.max_super = o.max_super > 0 ? o.max_super : 96;
    so.relax_small = o.relax_small == 0 ? 16 : (o.relax_small < 0 ? 0 : o.relax_small);
    so.relax_frac = o.relax_frac < 0 ? 0.5 : o.relax_frac;
    if (o.ordering < 0 || o.ordering > 2) return fail(KKT_ERR_INVALID_ARG, "unknown ordering");
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
    kkt_status st = ensure_runtime();
    if (st) return st;
    kkt_factor* f = new (std::nothrow) kkt_factor;
    if (!f) return fail(KKT_ERR_OOM, "host allocation");
    f->sym = sym;
    const Symbolic& S = sym->S;
    hipError_t e = f->pat.build(S);
    if (e != hipSuccess) { delete f; return hip_fail(e, "pattern upload"); }
    const size_t n = std::max(S.n, 1), m = std::max(S.m, 1);
    const size_t nred = (std::max(S.n, S.m) + kBlock - 1) / kBlock + 1;
    struct { DevBuf* b; size_t bytes; } al[] = {
        {&f->L, (size_t)S.lsize * 8}, {&f->U, (size_t)S.usize * 8}, {&f->V, (size_t)S.vsize * 8},
        {&f->kval, (size_t)S.nnzk * 8},
        {&f->y, n * 8}, {&f->r, n * 8}, {&f->xprev, n * 8}, {&f->tn, n * 8}, {&f->fg, n * 8},
        {&f->cvec, m * 8}, {&f->rvec, m * 8}, {&f->pvec, m * 8}, {&f->qvec, m * 8}, {&f->red, nred * 8},
        {&f->status, 16}, {&f->rs, sizeof(RefineState)}, {&f->cg, sizeof(CgState)}, {&f->ndone, 16},
        {&f->jcopy, std::max<size_t>((size_t)S.nnz_j, 1) * 8}, {&f->dinst, sizeof(InstDev)},
    };
    for (auto& a : al) {
        e = a.b->alloc(a.bytes);
        if (e != hipSuccess) { delete f; return hip_fail(e, "factor allocation"); }
    }
    InstDev I;
    std::memset(&I, 0, sizeof(I));
    I.P = f->pat.desc;
    I.L = (double*)f->L.p; I.U = (double*)f->U.p; I.V = (double*)f->V.p; I.kval = (double*)f->kval.p;
    I.y = (double*)f->y.p; I.r = (double*)f->r.p; I.xprev = (double*)f->xprev.p; I.tn = (double*)f->tn.p;
    I.fg = (double*)f->fg.p; I.cvec = (double*)f->cvec.p; I.rvec = (double*)f->rvec.p;
    I.pvec = (double*)f->pvec.p; I.qvec = (double*)f->qvec.p; I.red = (double*)f->red.p;
    I.status = (int*)f->status.p; I.rs = (RefineState*)f->rs.p; I.cg = (CgState*)f->cg.p;
    f->hinst = I;
    e = hipMemcpy(f->dinst.p, &I, sizeof(I), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipHostMalloc((void**)&f->hpin, 4096, hipHostMallocDefault);
    if (e == hipSuccess) e = hipMemset(f->status.p, 0, 16);
    if (e == hipSuccess) e = hipMemset(f->rs.p, 0, sizeof(RefineState));
    if (e == hipSuccess) e = hipMemset(f->cg.p, 0, sizeof(CgState));
    if (e != hipSuccess) { delete f; return hip_fail(e, "factor setup"); }
    *out = f;
    return KKT_OK;
}

void kkt_factor_destroy(kkt_factor* f) { delete f; }

kkt_status kkt_refactor(kkt_factor* f, const double* w_vals, const double* j_vals, const double* sigma_x,
                        const double* sigma_s, double gamma, void* stream) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    const Symbolic& S = f->sym->S;
    if ((S.nnz_w > 0 && !w_vals) || (S.nnz_j > 0 && !j_vals) || (S.n > 0 && !sigma_x))
        return fail(KKT_ERR_INVALID_ARG, "NULL value array");
    if (!(gamma >= 0.0) || !std::isfinite(gamma)) return fail(KKT_ERR_INVALID_ARG, "gamma must be finite and >= 0");
    const bool lifted = gamma == 0.0;
    if (lifted && S.m > 0 && !sigma_s) return fail(KKT_ERR_INVALID_ARG, "Lifted-KKT (gamma == 0) needs sigma_s");
    if (!lifted && sigma_s) return fail(KKT_ERR_INVALID_ARG, "HyKKT (gamma > 0) takes sigma_s = NULL");
    hipStream_t st = (hipStream_t)stream;
    f->last_stream = st;
    f->mode = lifted ? 1 : 2;
    f->gamma = gamma;
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.one.w = w_vals; C.one.jv = j_vals; C.one.sx = sigma_x; C.one.ss = sigma_s; C.one.gamma = gamma;
    const InstDev* di = (const InstDev*)f->dinst.p;
    int* status = (int*)f->status.p;
    TL(KKT_PHASE_CONTROL, launch_fill_i32(status, 0, 1, st));
    TL(KKT_PHASE_CONTROL, launch_fill_i32(status + 1, INT_MAX, 1, st));
    TL(KKT_PHASE_ASSEMBLE, launch_assemble(di, C, (const WorkItem*)f->pat.b_kitems.p, f->pat.n_kitems, st));
    const WorkItem* items = (const WorkItem*)f->pat.b_snitems.p;
    for (size_t l = 0; l + 1 < f->pat.lvl_ptr.size(); l++) {
        int a = f->pat.lvl_ptr[l], b = f->pat.lvl_ptr[l + 1];
        TL(KKT_PHASE_FACTOR, launch_factor(di, items + a, b - a, f->pat.lds_factor, st));
    }
    if (!lifted && S.nnz_j > 0) {
        hipError_t e = hipMemcpyAsync(f->jcopy.p, j_vals, S.nnz_j * 8, hipMemcpyDeviceToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "copy J values");
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "refactor launch");
    f->factored = true;
    return KKT_OK;
}

kkt_status kkt_status_sync(kkt_factor* f, kkt_factor_info* info) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    hipError_t e = hipStreamSynchronize(f->last_stream);
    if (e != hipSuccess) return hip_fail(e, "stream sync");
    int hs[2];
    e = hipMemcpy(hs, f->status.p, 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "status read");
    kkt_status st = hs[0] == 0 ? KKT_OK : hs[0];
    int bad = -1;
    if (hs[0] == KKT_ERR_NOT_SPD && hs[1] >= 0 && hs[1] < f->sym->S.n) bad = f->sym->S.perm[hs[1]];
    if (info) { info->status = st; info->bad_col = bad; }
    if (st != KKT_OK) g_last_error = std::string("factor status ") + kkt_status_string(st);
    return st;
}

}  // extern "C"

namespace kkt {

// forward + backward sweeps over the level schedule; y holds the permuted vector
void sweeps(kkt_factor* f, hipStream_t st) {
    const InstDev* di = (const InstDev*)f->dinst.p;
    const WorkItem* items = (const WorkItem*)f->pat.b_snitems.p;
    const auto& lp = f->pat.lvl_ptr;
    const int nl = (int)lp.size() - 1;
    for (int l = 0; l < nl; l++) TL(KKT_PHASE_FWD, launch_fwd(di, items + lp[l], lp[l + 1] - lp[l], f->pat.lds_solve, st));
    for (int l = nl - 1; l >= 0; l--) TL(KKT_PHASE_BWD, launch_bwd(di, items + lp[l], lp[l + 1] - lp[l], f->pat.lds_solve, st));
}

}  // namespace kkt

extern "C" {

kkt_status kkt_solve(kkt_factor* f, const double* b, double* x, const kkt_refine_opts* ro, kkt_solve_info* info,
                     void* stream) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    const Symbolic& S = f->sym->S;
    if (S.n > 0 && (!b || !x)) return fail(KKT_ERR_INVALID_ARG, "NULL vector");
    if (b == x && S.n > 0) return fail(KKT_ERR_INVALID_ARG, "x aliases b");
    if (!f->factored) return fail(KKT_ERR_STATE, "solve before refactor");
    int maxit = ro ? ro->max_iter : 10;
    double tol = ro ? ro->tol : 1e-14;
    if (maxit < 0) return fail(KKT_ERR_INVALID_ARG, "negative max_iter");
    hipStream_t st = (hipStream_t)stream;
    f->last_stream = st;
    const InstDev* di = (const InstDev*)f->dinst.p;
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.one.b = b;
    C.one.x = x;
    const WorkItem* nit = (const WorkItem*)f->pat.b_nitems.p;
    const int nn = f->pat.n_nitems;
    int* ndone = (int*)f->ndone.p;
    TL(KKT_PHASE_CONTROL, launch_refine_reset(di, 1, tol, maxit, st));
    TL(KKT_PHASE_CONTROL, launch_fill_i32(ndone, 0, 1, st));
    TL(KKT_PHASE_PERMUTE, launch_perm_in(di, C, nit, nn, PIN_B, st));
    sweeps(f, st);
    TL(KKT_PHASE_PERMUTE, launch_perm_out(di, C, nit, nn, POUT_X, st));
    int* hp = (int*)f->hpin;
    for (int iter = 0; iter <= maxit + 1; iter++) {
        TL(KKT_PHASE_RESIDUAL, launch_residual(di, C, nit, nn, st));
        TL(KKT_PHASE_CONTROL, launch_refine_decide(di, 1, ndone, st));
        hipError_t e = hipMemcpyAsync(hp, ndone, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(hp + 1, f->status.p, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "refinement control");
        if (hp[1] != 0) return fail(hp[1], "factor failed; solve refused");
        if (hp[0] >= 1) break;
        TL(KKT_PHASE_PERMUTE, launch_perm_in(di, C, nit, nn, PIN_R, st));
        sweeps(f, st);
        TL(KKT_PHASE_PERMUTE, launch_perm_out(di, C, nit, nn, POUT_X_UPDATE, st));
    }
    TL(KKT_PHASE_PERMUTE, launch_refine_revert(di, C, nit, nn, st));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "solve launch");
    if (!info) return KKT_OK;
    RefineState rs;
    e = hipMemcpyAsync(f->hpin, f->rs.p, sizeof(RefineState), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "solve info");
    std::memcpy(&rs, f->hpin, sizeof(rs));
    const bool rev = rs.revert != 0;
    info->iters = rev ? rs.it - 1 : rs.it;
    info->eta = rev ? rs.eta_prev : rs.eta;
    info->omega = rev ? rs.omega_prev : rs.omega;
    info->relres = rev ? rs.relres_prev : rs.relres;
    info->status = info->omega <= tol ? KKT_OK : KKT_ERR_NOT_CONVERGED;
    return info->status;
}

kkt_status kkt_cg_schur(kkt_factor* f, const double* fv, const double* g, double tol, int32_t maxit, double* dx,
                        double* dy, kkt_cg_info* info, void* stream) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    const Symbolic& S = f->sym->S;
    if ((S.n > 0 && (!fv || !dx)) || (S.m > 0 && (!g || !dy))) return fail(KKT_ERR_INVALID_ARG, "NULL vector");
    if (!f->factored || f->mode != 2) return fail(KKT_ERR_STATE, "cg_schur needs a K_gamma factor");
    if (maxit < 0 || !(tol >= 0.0)) return fail(KKT_ERR_INVALID_ARG, "bad tol/maxit");
    hipStream_t st = (hipStream_t)stream;
    f->last_stream = st;
    const InstDev* di = (const InstDev*)f->dinst.p;
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.one.jv = (const double*)f->jcopy.p;
    C.one.gamma = f->gamma;
    C.one.f = fv; C.one.g = g; C.one.dx = dx; C.one.dy = dy;
    const WorkItem* nit = (const WorkItem*)f->pat.b_nitems.p;
    const WorkItem* mit = (const WorkItem*)f->pat.b_mitems.p;
    const int nn = f->pat.n_nitems, nm = f->pat.n_mitems;
    int* ndone = (int*)f->ndone.p;
    int* hp = (int*)f->hpin;
    TL(KKT_PHASE_CONTROL, launch_fill_i32(ndone, 0, 1, st));
    TL(KKT_PHASE_CG, launch_cg_fgamma(di, C, nit, nn, st));
    TL(KKT_PHASE_PERMUTE, launch_perm_in(di, C, nit, nn, PIN_FG, st));
    sweeps(f, st);
    TL(KKT_PHASE_PERMUTE, launch_perm_out(di, C, nit, nn, POUT_TN, st));
    TL(KKT_PHASE_CG, launch_cg_init(di, C, mit, nm, st));
    TL(KKT_PHASE_CONTROL, launch_cg_start(di, 1, tol, maxit, ndone, st));
    hipError_t e = hipMemcpyAsync(hp, ndone, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(hp + 1, f->status.p, 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "cg control");
    if (hp[1] != 0) return fail(hp[1], "factor failed; solve refused");
    for (int it = 0; hp[0] == 0 && it < maxit; it++) {
        TL(KKT_PHASE_CG, launch_cg_jt(di, C, nit, nn, 0, st));
        TL(KKT_PHASE_PERMUTE, launch_perm_in(di, C, nit, nn, PIN_TN, st));
        sweeps(f, st);
        TL(KKT_PHASE_PERMUTE, launch_perm_out(di, C, nit, nn, POUT_TN, st));
        TL(KKT_PHASE_CG, launch_cg_jq(di, C, mit, nm, st));
        TL(KKT_PHASE_CONTROL, launch_cg_alpha(di, 1, ndone, st));
        TL(KKT_PHASE_CG, launch_cg_update(di, C, mit, nm, st));
        TL(KKT_PHASE_CONTROL, launch_cg_beta(di, 1, ndone, st));
        TL(KKT_PHASE_CG, launch_cg_p(di, mit, nm, st));
        e = hipMemcpyAsync(hp, ndone, 4, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) return hip_fail(e, "cg control");
    }
    TL(KKT_PHASE_CG, launch_cg_jt(di, C, nit, nn, 1, st));
    TL(KKT_PHASE_PERMUTE, launch_perm_in(di, C, nit, nn, PIN_TN, st));
    sweeps(f, st);
    TL(KKT_PHASE_PERMUTE, launch_perm_out(di, C, nit, nn, POUT_DX, st));
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "cg launch");
    if (!info) return KKT_OK;
    e = hipMemcpyAsync(f->hpin, f->cg.p, sizeof(CgState), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "cg info");
    CgState G;
    std::memcpy(&G, f->hpin, sizeof(G));
    info->iters = G.it;
    info->rel_res = G.cnorm > 0 ? std::sqrt(G.done && G.status == 0 && G.it > 0 ? G.rr_new : G.rr) / G.cnorm : 0.0;
    info->status = G.status == 0 ? (G.done ? KKT_OK : KKT_ERR_NOT_CONVERGED) : G.status;
    return info->status;
}

kkt_status kkt_matvec(kkt_factor* f, const double* x, double* y, void* stream) {
    if (!f || (!x && f->sym->S.n > 0) || (!y && f->sym->S.n > 0)) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    if (!f->factored) return fail(KKT_ERR_STATE, "matvec before refactor");
    hipStream_t st = (hipStream_t)stream;
    TL(KKT_PHASE_RESIDUAL,
       launch_matvec((const InstDev*)f->dinst.p, x, y, (const WorkItem*)f->pat.b_nitems.p, f->pat.n_nitems, st));
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? KKT_OK : hip_fail(e, "matvec launch");
}

kkt_status kkt_factor_set_timing(kkt_factor* f, int32_t enable) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    f->timer.on = enable != 0;
    return KKT_OK;
}

kkt_status kkt_factor_read_timing(kkt_factor* f, kkt_timing* out) {
    if (!f || !out) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    int launches[KKT_NPHASES];
    hipError_t e = f->timer.read(out->ms, launches, KKT_NPHASES);
    if (e != hipSuccess) return hip_fail(e, "timer read");
    for (int q = 0; q < KKT_NPHASES; q++) out->launches[q] = launches[q];
    return KKT_OK;
}

}  // extern "C"
