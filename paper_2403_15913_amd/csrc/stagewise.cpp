// Stage-structured solver for dynamic programs.
//
// The condensed matrix K = W + Sigma_x + J^T Sigma_s J of a dynamic program is
// block-banded (section "Future Works" of the paper: it can be factorized by
// a block-structured solver instead of a general sparse one). When every
// stage owns a contiguous range of variables, W couples variables of one
// stage or of consecutive stages, and every row of J spans at most two
// consecutive stages, K is block tridiagonal:
//   K = tridiag(E_{k-1}, D_k, E_k^T),  D_k = K(k, k),  E_k = K(k+1, k).
// It is factored by block cyclic reduction: at each level the stages at odd
// positions of the active chain are eliminated together (they are not
// coupled to each other), the stages at even positions form the next chain.
// The result is the Cholesky factor of K in that elimination order, kept as
// dense blocks: L_k for each stage and L(l,k), L(r,k) for its two active
// neighbours at its level. Levels are ceil(log2 N) + 1, so the work of a
// horizon of N stages runs in that many launches (one workgroup per stage
// still in the chain: the eliminated ones factor their front, the others
// take the updates their eliminated neighbours left on the level before).
// K is assembled by the general kernels (same bits as the supernodal path),
// then scattered into the blocks; the refined solve reuses the residual and
// stop-rule kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "api_internal.hpp"

using namespace kkt;

// the tasks of one level and width class (stage widths <= 16 nb), the
// eliminating ones first
struct CrClass {
    int start = 0, nelim = 0, nkept = 0, nb = 1;
    size_t lds = 0;     // factor LDS bytes
};
struct CrLevel {
    int start = 0, end = 0;  // all tasks of the level
    std::vector<CrClass> classes;
};

struct kkt_stagewise {
    Engine eng;                      // assembly, residuals, refinement records
    DevBuf store;                    // D, L, C, P, U, t, tasks, pulls, scatter list
    CrArrays A{};
    const CrScatter* dscat = nullptr;
    int64_t nscat = 0, nd = 0, ne = 0;
    std::vector<CrLevel> levels;
    int ninst = 0;
};

namespace {

struct StageTask {
    CrTask t;
    std::vector<CrPull> pulls;
};

kkt_status check_stages(const Symbolic& S, const int32_t* sp, int N, std::string& err) {
    if (N < 1 || !sp) { err = "each instance needs at least one stage"; return KKT_ERR_INVALID_ARG; }
    if (sp[0] != 0 || sp[N] != S.n) { err = "stage_ptr must start at 0 and end at n"; return KKT_ERR_INVALID_ARG; }
    for (int k = 0; k < N; k++) {
        const int s = sp[k + 1] - sp[k];
        if (s < 1) { err = "empty stage"; return KKT_ERR_INVALID_ARG; }
        if (s > kCrMaxStage) { err = "a stage is wider than the block buffers hold (80)"; return KKT_ERR_PATTERN; }
    }
    return KKT_OK;
}

// Builds the elimination schedule of one instance: per level, the tasks of
// the stages eliminated there and of the stages that stay, with their block
// offsets (running counters nc / np / nu, shared by all instances) and the
// (at most two) contributions each takes from the previous level.
void schedule_instance(int q, int n_off, const std::vector<int>& sp, const std::vector<int64_t>& dofs,
                       const std::vector<int64_t>& eofs, int64_t& nc, int64_t& np, int64_t& nu,
                       std::vector<std::vector<StageTask>>& elim_lv, std::vector<std::vector<StageTask>>& kept_lv) {
    const int N = (int)sp.size() - 1;
    auto width = [&](int k) { return sp[k + 1] - sp[k]; };
    std::vector<std::vector<CrPull>> pulls(N);  // contributions from the previous level
    std::vector<int64_t> f_of(N, -1), ul_of(N, -1), ur_of(N, -1), pl_of(N, -1), pr_of(N, -1);
    std::vector<int> left_prev(N, -1), right_prev(N, -1);  // eliminated neighbours at the previous level
    std::vector<int> active(N);
    for (int k = 0; k < N; k++) active[k] = k;
    auto base_task = [&](int k) {
        StageTask st;
        CrTask& T = st.t;
        std::memset(&T, 0, sizeof(T));
        T.inst = q;
        T.sk = width(k);
        T.var0 = sp[k];
        T.v0 = n_off + sp[k];
        T.d = dofs[k];
        T.kl = T.kr = T.pl = T.pr = T.f = T.ul = T.ur = -1;
        st.pulls = pulls[k];
        T.npull = (int)st.pulls.size();
        return st;
    };
    for (int lev = 0; !active.empty(); lev++) {
        const int na = (int)active.size();
        if ((int)elim_lv.size() <= lev) {
            elim_lv.emplace_back();
            kept_lv.emplace_back();
        }
        const int p0 = na == 1 ? 0 : 1;
        for (int p = p0; p < na; p += 2) {
            const int k = active[p];
            const int l = p > 0 ? active[p - 1] : -1;
            const int r = p + 1 < na ? active[p + 1] : -1;
            StageTask st = base_task(k);
            CrTask& T = st.t;
            T.sl = l >= 0 ? width(l) : 0;
            T.sr = r >= 0 ? width(r) : 0;
            T.vl = l >= 0 ? n_off + sp[l] : 0;
            T.vr = r >= 0 ? n_off + sp[r] : 0;
            if (l >= 0) T.kl = lev == 0 ? eofs[k - 1] : f_of[left_prev[k]];
            if (r >= 0) T.kr = lev == 0 ? eofs[k] : f_of[right_prev[k]];
            if (l >= 0) {
                T.pl = pl_of[k] = np;
                np += (int64_t)T.sl * T.sk;
                T.ul = ul_of[k] = nu;
                nu += (int64_t)T.sl * T.sl;
            }
            if (r >= 0) {
                T.pr = pr_of[k] = np;
                np += (int64_t)T.sr * T.sk;
                T.ur = ur_of[k] = nu;
                nu += (int64_t)T.sr * T.sr;
            }
            if (l >= 0 && r >= 0) {
                T.f = f_of[k] = nc;
                nc += (int64_t)T.sr * T.sl;
            }
            elim_lv[lev].push_back(std::move(st));
        }
        if (na == 1) break;
        // stages that stay: a task of their own (previous level's updates; on
        // the first level the copy of the right-hand side), then the
        // contributions of their eliminated neighbours for the next level
        std::vector<int> next;
        for (int p = 0; p < na; p += 2) kept_lv[lev].push_back(base_task(active[p]));
        for (int p = 0; p < na; p += 2) {
            const int k = active[p];
            pulls[k].clear();
            left_prev[k] = right_prev[k] = -1;
            if (p > 0) {
                const int il = active[p - 1];  // k is its right neighbour
                pulls[k].push_back(CrPull{ur_of[il], pr_of[il], n_off + sp[il], width(il)});
                left_prev[k] = il;
            }
            if (p + 1 < na) {
                const int ir = active[p + 1];  // k is its left neighbour
                pulls[k].push_back(CrPull{ul_of[ir], pl_of[ir], n_off + sp[ir], width(ir)});
                right_prev[k] = ir;
            }
            next.push_back(k);
        }
        active.swap(next);
    }
}

}  // namespace

extern "C" kkt_status kkt_stagewise_create(int32_t count, const kkt_symbolic* const* syms,
                                           const int32_t* const* stage_ptrs, const int32_t* nstages,
                                           kkt_stagewise** out) {
    if (!out || count < 1 || !syms || !stage_ptrs || !nstages) return fail(KKT_ERR_INVALID_ARG, "bad arguments");
    *out = nullptr;
    // host checks first: stage ranges, then the block-tridiagonal structure
    std::vector<const Symbolic*> ss(count);
    std::vector<std::vector<int>> stage_ptr(count);
    std::vector<CrScatter> hsc;
    std::vector<std::vector<int64_t>> dofs(count), eofs(count);
    int64_t nd = 0, ne = 0;
    for (int q = 0; q < count; q++) {
        if (!syms[q]) return fail(KKT_ERR_INVALID_ARG, "NULL symbolic");
        const Symbolic& S = syms[q]->S;
        ss[q] = &S;
        std::string err;
        const kkt_status st = check_stages(S, stage_ptrs[q], nstages[q], err);
        if (st) return fail(st, err);
        const std::vector<int> sp(stage_ptrs[q], stage_ptrs[q] + nstages[q] + 1);
        const int N = nstages[q];
        std::vector<int> stage(S.n);
        for (int k = 0; k < N; k++)
            for (int v = sp[k]; v < sp[k + 1]; v++) stage[v] = k;
        dofs[q].resize(N);
        eofs[q].assign(std::max(N - 1, 1), -1);
        for (int k = 0; k < N; k++) {
            const int64_t s = sp[k + 1] - sp[k];
            dofs[q][k] = nd;
            nd += s * s;
            if (k + 1 < N) {
                eofs[q][k] = ne;
                ne += (int64_t)(sp[k + 2] - sp[k + 1]) * s;
            }
        }
        for (int i = 0; i < S.n; i++)
            for (int64_t p = S.sp_ptr[i]; p < S.sp_ptr[i + 1]; p++) {
                const int j = S.sp_col[p];
                if (j > i) continue;
                const int ki = stage[i], kj = stage[j];
                CrScatter c;
                c.inst = q;
                c.pos = (int)p;
                if (ki == kj) {
                    const int s0 = sp[ki], s = sp[ki + 1] - s0;
                    c.dst = dofs[q][ki] + (int64_t)(j - s0) * s + (i - s0);
                } else if (ki == kj + 1) {
                    const int s1 = sp[ki + 1] - sp[ki];
                    c.dst = -(eofs[q][kj] + (int64_t)(j - sp[kj]) * s1 + (i - sp[ki])) - 1;
                } else {
                    return fail(KKT_ERR_PATTERN, "K couples stages more than one apart");
                }
                hsc.push_back(c);
            }
        stage_ptr[q] = sp;
    }
    std::unique_ptr<kkt_stagewise> W(new (std::nothrow) kkt_stagewise);
    if (!W) return fail(KKT_ERR_OOM, "host allocation");
    W->eng.assembly_only = true;
    kkt_status st = W->eng.init_owned(ss);
    if (st) return st;
    W->ninst = count;
    // the elimination schedule of every instance, tasks grouped by level
    int64_t nc = ne, np = 0, nu = 0;
    std::vector<std::vector<StageTask>> elim_lv, kept_lv;
    for (int q = 0; q < count; q++)
        schedule_instance(q, (int)W->eng.n_ofs[q], stage_ptr[q], dofs[q], eofs[q], nc, np, nu, elim_lv, kept_lv);
    std::vector<CrTask> htasks;
    std::vector<CrPull> hpulls;
    auto nb_of = [](const CrTask& T) { return (std::max({T.sk, T.sl, T.sr}) + 15) / 16; };
    for (size_t lv = 0; lv < elim_lv.size(); lv++) {
        CrLevel L;
        L.start = (int)htasks.size();
        for (int nb = 1; nb <= kCrMaxStage / 16; nb++) {
            CrClass K;
            K.start = (int)htasks.size();
            K.nb = nb;
            int front = 0;
            for (int pass = 0; pass < 2; pass++)
                for (auto& stt : pass == 0 ? elim_lv[lv] : kept_lv[lv]) {
                    CrTask T = stt.t;
                    if (nb_of(T) != nb) continue;
                    T.elim = pass == 0;
                    // from the third level on, the block has been updated by
                    // the stage's own task on an earlier level
                    T.from_work = lv >= 2;
                    T.pull0 = (int)hpulls.size();
                    hpulls.insert(hpulls.end(), stt.pulls.begin(), stt.pulls.end());
                    front = std::max(front, (T.sl + T.sr) * T.sk);
                    htasks.push_back(T);
                    (pass == 0 ? K.nelim : K.nkept)++;
                }
            if (K.nelim + K.nkept == 0) continue;
            // two column buffers of 48 nb rows, 16 nb pivots, then the rows
            // below the stage (s_k columns of s_l + s_r) with 32 nb entries
            // of padding
            K.lds = (size_t)(2 * 48 * nb + 16 * nb + front + 32 * nb) * sizeof(double);
            L.classes.push_back(K);
        }
        L.end = (int)htasks.size();
        W->levels.push_back(L);
    }
    const int64_t ntot = W->eng.n_ofs[count];
    // every block a task or pull touches lies inside its array
    auto in = [](int64_t o, int64_t len, int64_t size) { return len == 0 || (o >= 0 && o + len <= size); };
    for (const CrTask& T : htasks) {
        const int64_t sk = T.sk, sl = T.sl, sr = T.sr;
        bool ok = in(T.d, sk * sk, nd) && in(T.v0, sk, ntot) && in(T.vl, sl, ntot) && in(T.vr, sr, ntot) &&
                  in(T.kl, sk * sl, nc) && in(T.kr, sr * sk, nc) && in(T.pl, sl * sk, np) && in(T.pr, sr * sk, np) &&
                  in(T.f, sl && sr ? sr * sl : 0, nc) && in(T.ul, sl * sl, nu) && in(T.ur, sr * sr, nu);
        for (int u = 0; ok && u < T.npull; u++) {
            const CrPull& P = hpulls[T.pull0 + u];
            ok = in(P.u, sk * sk, nu) && in(P.p, sk * P.si, np) && in(P.vi, P.si, ntot);
        }
        if (!ok) return fail(KKT_ERR_PATTERN, "internal: stage-structured schedule out of bounds");
    }
    for (const CrScatter& c : hsc)
        if (c.dst >= 0 ? c.dst >= nd : (-c.dst - 1) >= ne) return fail(KKT_ERR_PATTERN, "internal: scatter out of bounds");
    // one device allocation
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        const size_t at = off;
        off += std::max<size_t>(bytes, 8);
        return at;
    };
    const size_t oD = take(nd * 8), oL = take(nd * 8), oC = take(nc * 8), oP = take(np * 8), oU = take(nu * 8),
                 oT = take(ntot * 8);
    const size_t oTk = take(htasks.size() * sizeof(CrTask)), oPl = take(hpulls.size() * sizeof(CrPull));
    const size_t oSc = take(hsc.size() * sizeof(CrScatter));
    hipError_t e = W->store.alloc(off);
    if (e != hipSuccess) return hip_fail(e, "stage-structured storage");
    char* base = (char*)W->store.p;
    W->A.D = (double*)(base + oD);
    W->A.L = (double*)(base + oL);
    W->A.C = (double*)(base + oC);
    W->A.P = (double*)(base + oP);
    W->A.U = (double*)(base + oU);
    W->A.t = (double*)(base + oT);
    W->A.tasks = (const CrTask*)(base + oTk);
    W->A.pulls = (const CrPull*)(base + oPl);
    W->dscat = (const CrScatter*)(base + oSc);
    W->nscat = (int64_t)hsc.size();
    W->nd = nd;
    W->ne = ne;
    struct Piece {
        size_t at;
        const void* src;
        size_t bytes;
    } pieces[] = {{oTk, htasks.data(), htasks.size() * sizeof(CrTask)},
                  {oPl, hpulls.data(), hpulls.size() * sizeof(CrPull)},
                  {oSc, hsc.data(), hsc.size() * sizeof(CrScatter)}};
    for (auto& pc : pieces)
        if (pc.bytes && (e = hipMemcpy(base + pc.at, pc.src, pc.bytes, hipMemcpyHostToDevice)) != hipSuccess)
            return hip_fail(e, "stage-structured upload");
    // the positions of D and E outside K's pattern stay zero: only the
    // scatter writes these arrays afterwards
    launch_fill_f64(W->A.D, 0.0, nd, nullptr);
    launch_fill_f64(W->A.C, 0.0, ne, nullptr);
    if ((e = hipGetLastError()) != hipSuccess || (e = hipStreamSynchronize(nullptr)) != hipSuccess)
        return hip_fail(e, "stage-structured initialisation");
    *out = W.release();
    return KKT_OK;
}

extern "C" void kkt_stagewise_destroy(kkt_stagewise* w) { delete w; }

extern "C" kkt_status kkt_stagewise_refactor(kkt_stagewise* w, const double* w_vals, const double* j_vals,
                                             const double* sigma_x, const double* sigma_s, void* stream) {
    if (!w) return fail(KKT_ERR_INVALID_ARG, "NULL stagewise solver");
    Engine& E = w->eng;
    const int64_t nw = E.w_ofs[E.ninst], nj = E.j_ofs[E.ninst], n = E.n_ofs[E.ninst], m = E.m_ofs[E.ninst];
    if ((nw > 0 && !w_vals) || (nj > 0 && !j_vals) || (n > 0 && !sigma_x) || (m > 0 && !sigma_s))
        return fail(KKT_ERR_INVALID_ARG, "NULL value array");
    const hipStream_t st = (hipStream_t)stream;
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.w = w_vals;
    C.jv = j_vals;
    C.sx = sigma_x;
    C.ss = sigma_s;
    const kkt_status ks = E.assemble(C, st);
    if (ks) return ks;
    LaunchTimer& timer = E.timer;
    TL(KKT_PHASE_ASSEMBLE, launch_cr_scatter(E.di(), w->A, w->dscat, w->nscat, st));
    // the first level's stages that stay have nothing to update yet
    for (size_t l = 0; l < w->levels.size(); l++)
        for (const CrClass& K : w->levels[l].classes)
            TL(KKT_PHASE_FACTOR,
               launch_cr_factor(E.di(), w->A, K.start, K.nelim + (l ? K.nkept : 0), K.nb, K.lds, st));
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "stage-structured factor launch");
    E.factored = true;
    return KKT_OK;
}

extern "C" kkt_status kkt_stagewise_status(kkt_stagewise* w, int32_t* status, int32_t* bad_col) {
    if (!w) return fail(KKT_ERR_INVALID_ARG, "NULL stagewise solver");
    Engine& E = w->eng;
    hipError_t e = hipStreamSynchronize(E.last_stream);
    if (e == hipSuccess) e = hipMemcpy(E.hpin, E.status, (size_t)E.ninst * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "status read");
    const int* hs = (const int*)E.hpin;
    kkt_status worst = KKT_OK;
    for (int q = 0; q < E.ninst; q++) {
        const int code = hs[2 * q];
        if (status) status[q] = code;
        // the failed variable is recorded in the original numbering
        if (bad_col) bad_col[q] = code == KKT_ERR_NOT_SPD ? hs[2 * q + 1] : -1;
        if (code != KKT_OK && worst == KKT_OK) worst = code;
    }
    return worst;
}

namespace {
// one pass of both sweeps over all levels: mode 0 x = K^{-1} b, mode 1 x += K^{-1} r
void cr_sweeps(kkt_stagewise* w, const Calls& C, int mode, hipStream_t st) {
    Engine& E = w->eng;
    LaunchTimer& timer = E.timer;
    const int nl = (int)w->levels.size();
    for (int l = 0; l < nl; l++) {
        const CrLevel& L = w->levels[l];
        TL(KKT_PHASE_FWD, launch_cr_fwd(E.di(), w->A, L.start, L.end - L.start, C, mode, l == 0, st));
    }
    // the tasks of stages that stay return at once
    for (int l = nl - 1; l >= 0; l--) {
        const CrLevel& L = w->levels[l];
        TL(KKT_PHASE_BWD, launch_cr_bwd(E.di(), w->A, L.start, L.end - L.start, C, mode, st));
    }
}
}  // namespace

// Refined solve: the first solve with the block factor, then rounds of the
// residual, the stop rule (as kkt_solve) and a correction, the host reading
// the count of stopped instances after each round.
extern "C" kkt_status kkt_stagewise_solve(kkt_stagewise* w, const double* rhs, double* x, const kkt_refine_opts* ro,
                                          kkt_solve_info* infos, void* stream) {
    if (!w) return fail(KKT_ERR_INVALID_ARG, "NULL stagewise solver");
    Engine& E = w->eng;
    const int64_t n = E.n_ofs[E.ninst];
    if (n > 0 && (!rhs || !x)) return fail(KKT_ERR_INVALID_ARG, "NULL vector");
    if (rhs == x && n > 0) return fail(KKT_ERR_INVALID_ARG, "x aliases rhs");
    if (!E.factored) return fail(KKT_ERR_STATE, "solve before refactor");
    const int maxit = ro ? ro->max_iter : 10;
    const double tol = ro ? ro->tol : 1e-14;
    if (maxit < 0 || !(tol >= 0.0)) return fail(KKT_ERR_INVALID_ARG, "bad refinement options");
    const hipStream_t st = (hipStream_t)stream;
    E.last_stream = st;
    LaunchTimer& timer = E.timer;
    Calls C;
    std::memset(&C, 0, sizeof(C));
    C.b = rhs;
    C.x = x;
    TL(KKT_PHASE_CONTROL, launch_refine_reset(E.di(), E.ninst, tol, maxit, st));
    TL(KKT_PHASE_CONTROL, launch_fill_i32(E.ndone, 0, 1, st));
    cr_sweeps(w, C, 0, st);
    volatile int* hp = (volatile int*)E.hpin;
    hipError_t e = hipSuccess;
    for (int iter = 0; iter <= maxit + 1; iter++) {
        TL(KKT_PHASE_RESIDUAL, launch_residual(E.di(), C, E.nitems, E.n_nitems, st));
        TL(KKT_PHASE_CONTROL, launch_refine_decide(E.di(), E.ninst, E.ndone, st));
        if ((e = hipMemcpyAsync((void*)hp, E.ndone, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(e, "refinement control");
        if (hp[0] >= E.ninst) break;
        cr_sweeps(w, C, 1, st);
    }
    TL(KKT_PHASE_PERMUTE, launch_refine_revert(E.di(), C, E.nitems, E.n_nitems, st));
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "solve launch");
    kkt_status worst = kkt_stagewise_status(w, nullptr, nullptr);
    if (worst == KKT_ERR_DEVICE) return worst;
    if (worst != KKT_OK) return fail(worst, "factor failed; solve result invalid");
    if (!infos) return KKT_OK;
    if ((e = hipMemcpy(E.hpin, E.rs, (size_t)E.ninst * sizeof(RefineState), hipMemcpyDeviceToHost)) != hipSuccess)
        return hip_fail(e, "refinement records");
    const RefineState* hr = (const RefineState*)E.hpin;
    for (int q = 0; q < E.ninst; q++) {
        const RefineState& R = hr[q];
        const bool rev = R.revert != 0;
        kkt_solve_info& inf = infos[q];
        inf.iters = rev ? R.it - 1 : R.it;
        inf.eta = rev ? R.eta_prev : R.eta;
        inf.omega = rev ? R.omega_prev : R.omega;
        inf.relres = rev ? R.relres_prev : R.relres;
        inf.status = inf.omega <= tol ? KKT_OK : KKT_ERR_NOT_CONVERGED;
        if (inf.status != KKT_OK) worst = inf.status;
    }
    return worst;
}

extern "C" kkt_status kkt_stagewise_set_timing(kkt_stagewise* w, int32_t enable) {
    if (!w) return fail(KKT_ERR_INVALID_ARG, "NULL stagewise solver");
    w->eng.timer.on = enable != 0;
    return KKT_OK;
}

extern "C" kkt_status kkt_stagewise_read_timing(kkt_stagewise* w, kkt_timing* out) {
    if (!w || !out) return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    int launches[KKT_NPHASES];
    const hipError_t e = w->eng.timer.read(out->ms, launches, KKT_NPHASES);
    if (e != hipSuccess) return hip_fail(e, "timer read");
    for (int q = 0; q < KKT_NPHASES; q++) out->launches[q] = launches[q];
    return KKT_OK;
}
