// Host-side symbolic analysis (see symbolic.hpp).
//
// Steps: validate the CSR inputs; pattern of K = pattern(W) + diagonal +
// pattern(J^T J); fill-reducing ordering (natural, or nested dissection by
// BFS level structures); elimination tree and postorder; column counts by
// row subtrees; fundamental supernodes; relaxed amalgamation capped by the
// LDS that one front panel may use; front row structures; relative indices
// of every child's update rows inside its parent's front; the map that
// scatters every assembled entry of K into its front panel; J^T J
// contribution pairs for the assembly; the symmetric row lists used by the
// residual K x; level schedules.
#include "symbolic.hpp"

#include "device.hpp"
#include "lds_layout.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>

namespace kkt {
namespace {

enum { ST_OK = 0, ST_INVALID = 1, ST_PATTERN = 2 };

struct Graph {  // symmetric adjacency of K without self loops, original numbering
    int n = 0;
    std::vector<int64_t> p;
    std::vector<int> a;
};

int64_t panel_lds_bytes(int r, int c) { return front_lds_bytes(r, c); }

int validate(int n, int m, const int32_t* wp, const int32_t* wi, const int32_t* jp, const int32_t* ji,
             std::string& err) {
    if (n < 0 || m < 0) { err = "negative dimension"; return ST_INVALID; }
    if (!wp || !jp) { err = "NULL row pointer"; return ST_INVALID; }
    if (wp[0] != 0 || jp[0] != 0) { err = "row pointers must start at 0"; return ST_PATTERN; }
    for (int i = 0; i < n; i++) {
        if (wp[i + 1] < wp[i]) { err = "W row pointer decreases"; return ST_PATTERN; }
        for (int p = wp[i]; p < wp[i + 1]; p++) {
            int j = wi[p];
            if (j < 0 || j > i) { err = "W entry outside the lower triangle (row " + std::to_string(i) + ")"; return ST_PATTERN; }
            if (p > wp[i] && wi[p - 1] >= j) { err = "W columns not strictly ascending (row " + std::to_string(i) + ")"; return ST_PATTERN; }
        }
    }
    if (wp[n] > 0 && !wi) { err = "NULL W column indices"; return ST_INVALID; }
    for (int r = 0; r < m; r++) {
        if (jp[r + 1] < jp[r]) { err = "J row pointer decreases"; return ST_PATTERN; }
        for (int p = jp[r]; p < jp[r + 1]; p++) {
            int c = ji[p];
            if (c < 0 || c >= n) { err = "J column out of range (row " + std::to_string(r) + ")"; return ST_PATTERN; }
            if (p > jp[r] && ji[p - 1] >= c) { err = "J columns not strictly ascending (row " + std::to_string(r) + ")"; return ST_PATTERN; }
        }
    }
    if (jp[m] > 0 && !ji) { err = "NULL J column indices"; return ST_INVALID; }
    return ST_OK;
}

// ---------------------------------------------------------------------------
// nested dissection by BFS level structures
// ---------------------------------------------------------------------------
struct Dissector {
    const Graph& G;
    int leaf;
    std::vector<int>& out;
    std::vector<int> mark, vis, lev, queue, side;
    int mstamp = 0, vstamp = 0;

    Dissector(const Graph& g, int lf, std::vector<int>& o)
        : G(g), leaf(lf), out(o), mark(g.n, 0), vis(g.n, 0), lev(g.n, 0), queue(g.n), side(g.n, 0) {}

    int bfs(int s) {
        ++vstamp;
        int head = 0, tail = 0;
        queue[tail++] = s;
        vis[s] = vstamp;
        lev[s] = 0;
        while (head < tail) {
            int v = queue[head++];
            for (int64_t p = G.p[v]; p < G.p[v + 1]; p++) {
                int w = G.a[p];
                if (mark[w] == mstamp && vis[w] != vstamp) {
                    vis[w] = vstamp;
                    lev[w] = lev[v] + 1;
                    queue[tail++] = w;
                }
            }
        }
        return tail;
    }

    void emit(std::vector<int>& V) {
        std::sort(V.begin(), V.end());
        out.insert(out.end(), V.begin(), V.end());
    }

    void run(std::vector<int> V) {
        const int nv = (int)V.size();
        if (nv <= leaf) { emit(V); return; }
        ++mstamp;
        int my = mstamp;
        for (int v : V) mark[v] = my;
        int s = *std::min_element(V.begin(), V.end());
        int cnt = bfs(s);
        if (cnt < nv) {  // disconnected: order the components one after another
            std::vector<int> C(queue.begin(), queue.begin() + cnt), R;
            int vs = vstamp;
            for (int v : V) if (vis[v] != vs) R.push_back(v);
            run(std::move(C));
            run(std::move(R));
            return;
        }
        // pseudo-peripheral start vertex
        int ecc = lev[queue[cnt - 1]];
        for (int iter = 0; iter < 8; iter++) {
            int best = -1;
            int64_t bdeg = INT64_MAX;
            for (int q = cnt - 1; q >= 0 && lev[queue[q]] == ecc; q--) {
                int v = queue[q];
                int64_t d = G.p[v + 1] - G.p[v];
                if (d < bdeg || (d == bdeg && v < best)) { bdeg = d; best = v; }
            }
            bfs(best);
            int e2 = lev[queue[cnt - 1]];
            if (e2 <= ecc) { bfs(s); break; }
            ecc = e2;
            s = best;
        }
        // level sizes
        int h = ecc;
        std::vector<int> lsz(h + 1, 0);
        for (int q = 0; q < cnt; q++) lsz[lev[queue[q]]]++;
        int best_l = -1;
        int64_t best_sz = INT64_MAX, best_imb = INT64_MAX;
        int acc = 0;
        for (int l = 0; l <= h; l++) {
            int a = acc, b = nv - acc - lsz[l];
            acc += lsz[l];
            if (l == 0 || l == h) continue;
            if (std::min(a, b) < nv / 5) continue;
            int64_t imb = std::abs(a - b);
            if (lsz[l] < best_sz || (lsz[l] == best_sz && imb < best_imb)) { best_sz = lsz[l]; best_imb = imb; best_l = l; }
        }
        if (best_l < 0) { emit(V); return; }
        for (int v : V) side[v] = lev[v] < best_l ? 0 : (lev[v] == best_l ? 1 : 2);
        // thin the separator: drop vertices with no neighbour on the far side
        for (int v : V) {
            if (side[v] != 1) continue;
            bool nb_b = false;
            for (int64_t p = G.p[v]; p < G.p[v + 1] && !nb_b; p++) {
                int w = G.a[p];
                if (mark[w] == my && side[w] == 2) nb_b = true;
            }
            if (!nb_b) side[v] = 0;
        }
        for (int v : V) {
            if (side[v] != 1) continue;
            bool nb_a = false;
            for (int64_t p = G.p[v]; p < G.p[v + 1] && !nb_a; p++) {
                int w = G.a[p];
                if (mark[w] == my && side[w] == 0) nb_a = true;
            }
            if (!nb_a) side[v] = 2;
        }
        std::vector<int> A, B, S;
        for (int v : V) (side[v] == 0 ? A : side[v] == 1 ? S : B).push_back(v);
        if (A.empty() || B.empty()) { emit(V); return; }
        run(std::move(A));
        run(std::move(B));
        emit(S);
    }
};

}  // namespace

int analyze(int n, int m, const int32_t* wp, const int32_t* wi, const int32_t* jp, const int32_t* ji,
            const SymOptions& opt, Symbolic& S, std::string& err) {
    auto t0 = std::chrono::steady_clock::now();
    int st = validate(n, m, wp, wi, jp, ji, err);
    if (st) return st;
    if (opt.max_super < 1 || opt.lds_bytes < 16 * 16 * 8) { err = "invalid supernode options"; return ST_INVALID; }
    S = Symbolic();
    S.n = n;
    S.m = m;
    S.nnz_w = wp[n];
    S.nnz_j = jp[m];
    const int64_t nnzj = S.nnz_j;

    // ---- J by rows and by columns -----------------------------------------
    S.j_ptr.assign(jp, jp + m + 1);
    S.j_col.assign(ji, ji + nnzj);
    S.jrow.resize(nnzj);
    for (int r = 0; r < m; r++)
        for (int p = jp[r]; p < jp[r + 1]; p++) S.jrow[p] = r;
    S.jt_ptr.assign(n + 1, 0);
    for (int64_t p = 0; p < nnzj; p++) S.jt_ptr[ji[p] + 1]++;
    for (int i = 0; i < n; i++) S.jt_ptr[i + 1] += S.jt_ptr[i];
    S.jt_e.resize(nnzj);
    S.jt_row.resize(nnzj);
    {
        std::vector<int> fill(S.jt_ptr.begin(), S.jt_ptr.end() - 1);
        for (int r = 0; r < m; r++)
            for (int p = jp[r]; p < jp[r + 1]; p++) {
                int q = fill[ji[p]]++;
                S.jt_e[q] = p;
                S.jt_row[q] = r;
            }
    }

    // ---- pattern of the lower triangle of K (original numbering) -----------
    std::vector<int64_t> Kp(n + 1, 0);
    std::vector<int> Kj;
    {
        std::vector<int> marker(n, -1), rowbuf;
        Kj.reserve((size_t)wp[n] + n + 2 * (size_t)nnzj);
        for (int i = 0; i < n; i++) {
            rowbuf.clear();
            auto add = [&](int j) { if (marker[j] != i) { marker[j] = i; rowbuf.push_back(j); } };
            add(i);
            for (int p = wp[i]; p < wp[i + 1]; p++) add(wi[p]);
            for (int q = S.jt_ptr[i]; q < S.jt_ptr[i + 1]; q++) {
                int r = S.jt_row[q];
                for (int p = jp[r]; p < jp[r + 1] && ji[p] <= i; p++) add(ji[p]);
            }
            std::sort(rowbuf.begin(), rowbuf.end());
            Kj.insert(Kj.end(), rowbuf.begin(), rowbuf.end());
            Kp[i + 1] = (int64_t)Kj.size();
        }
    }
    const int64_t nnzk = Kp[n];
    S.nnzk = nnzk;

    // ---- symmetric graph (no self loops) -------------------------------------
    Graph G;
    G.n = n;
    G.p.assign(n + 1, 0);
    for (int i = 0; i < n; i++)
        for (int64_t p = Kp[i]; p < Kp[i + 1]; p++)
            if (Kj[p] != i) { G.p[i + 1]++; G.p[Kj[p] + 1]++; }
    for (int i = 0; i < n; i++) G.p[i + 1] += G.p[i];
    G.a.resize(G.p[n]);
    {
        std::vector<int64_t> fill(G.p.begin(), G.p.end() - 1);
        for (int i = 0; i < n; i++)
            for (int64_t p = Kp[i]; p < Kp[i + 1]; p++) {
                int j = Kj[p];
                if (j == i) continue;
                G.a[fill[i]++] = j;
                G.a[fill[j]++] = i;
            }
    }

    // ---- ordering -------------------------------------------------------------
    int ordering = opt.ordering;
    int leaf = opt.nd_leaf > 0 ? opt.nd_leaf : std::max(128, n / 256);
    if (ordering == 0) ordering = (n > 2 * leaf) ? 2 : 1;
    std::vector<int> perm;
    perm.reserve(n);
    if (ordering == 1) {
        perm.resize(n);
        std::iota(perm.begin(), perm.end(), 0);
    } else if (ordering == 2) {
        std::vector<int> all(n);
        std::iota(all.begin(), all.end(), 0);
        Dissector D(G, leaf, perm);
        if (n > 0) D.run(std::move(all));
    } else {
        err = "unknown ordering";
        return ST_INVALID;
    }
    std::vector<int> iperm(n);
    for (int k = 0; k < n; k++) iperm[perm[k]] = k;

    // ---- elimination tree ------------------------------------------------------
    auto etree = [&](const std::vector<int>& pm, const std::vector<int>& ipm, std::vector<int>& parent) {
        std::vector<int> anc(n, -1);
        parent.assign(n, -1);
        for (int k = 0; k < n; k++) {
            int v = pm[k];
            for (int64_t p = G.p[v]; p < G.p[v + 1]; p++) {
                int i = ipm[G.a[p]];
                while (i != -1 && i < k) {
                    int nx = anc[i];
                    anc[i] = k;
                    if (nx == -1) parent[i] = k;
                    i = nx;
                }
            }
        }
    };
    std::vector<int> parent;
    etree(perm, iperm, parent);

    // ---- postorder --------------------------------------------------------------
    {
        std::vector<int> head(n, -1), next(n, -1), post;
        post.reserve(n);
        for (int j = n - 1; j >= 0; j--)
            if (parent[j] != -1) { next[j] = head[parent[j]]; head[parent[j]] = j; }
        std::vector<int> stack;
        for (int r = 0; r < n; r++) {
            if (parent[r] != -1) continue;
            stack.push_back(r);
            while (!stack.empty()) {
                int v = stack.back();
                if (head[v] != -1) {
                    int c = head[v];
                    head[v] = next[c];
                    stack.push_back(c);
                } else {
                    stack.pop_back();
                    post.push_back(v);
                }
            }
        }
        std::vector<int> perm2(n);
        for (int k = 0; k < n; k++) perm2[k] = perm[post[k]];
        perm.swap(perm2);
        for (int k = 0; k < n; k++) iperm[perm[k]] = k;
        etree(perm, iperm, parent);
    }
    S.perm = perm;
    S.iperm = iperm;

    // ---- column counts (row subtrees) -----------------------------------------
    std::vector<int> cc(n, 1), markc(n, -1);
    for (int i = 0; i < n; i++) {
        markc[i] = i;
        int v = perm[i];
        for (int64_t p = G.p[v]; p < G.p[v + 1]; p++) {
            int k = iperm[G.a[p]];
            if (k >= i) continue;
            while (markc[k] != i) {
                cc[k]++;
                markc[k] = i;
                k = parent[k];
            }
        }
    }
    S.nnzl_exact = 0;
    S.flops_exact = 0;
    for (int j = 0; j < n; j++) { S.nnzl_exact += cc[j]; S.flops_exact += (double)cc[j] * cc[j]; }

    // ---- fundamental supernodes ---------------------------------------------------
    std::vector<int> nchild(n, 0);
    for (int j = 0; j < n; j++) if (parent[j] != -1) nchild[parent[j]]++;
    std::vector<int> fs_start;  // first column of each fundamental supernode
    for (int j = 0; j < n; j++) {
        bool cont = j > 0 && parent[j - 1] == j && cc[j - 1] == cc[j] + 1 && nchild[j] == 1 &&
                    (j - fs_start.back()) < opt.max_super;
        if (!cont) fs_start.push_back(j);
    }
    int nf = (int)fs_start.size();
    fs_start.push_back(n);
    std::vector<int> col2f(n);
    for (int f = 0; f < nf; f++)
        for (int j = fs_start[f]; j < fs_start[f + 1]; j++) col2f[j] = f;

    // ---- relaxed amalgamation (merge a child into its parent when contiguous) ---
    // Represented on fundamental supernodes: first[], ncol, nupd, true nnz, parent.
    std::vector<int> f_first(nf), f_ncol(nf), f_nupd(nf), f_par(nf), alive(nf, 1);
    std::vector<int64_t> f_true(nf, 0);
    for (int f = 0; f < nf; f++) {
        f_first[f] = fs_start[f];
        f_ncol[f] = fs_start[f + 1] - fs_start[f];
        f_nupd[f] = cc[fs_start[f]] - f_ncol[f];
        int last = fs_start[f + 1] - 1;
        f_par[f] = parent[last] == -1 ? -1 : col2f[parent[last]];
        for (int j = fs_start[f]; j < fs_start[f + 1]; j++) f_true[f] += cc[j];
    }
    // f_owner[col] resolved after merging; merging p absorbs the child ending at first(p)-1.
    for (int p = 0; p < nf; p++) {
        for (;;) {
            int fc = f_first[p];
            if (fc == 0) break;
            int c = col2f[fc - 1];
            // follow merges: the supernode currently owning column fc-1
            while (!alive[c]) c = f_par[c];  // absorbed nodes point at their absorber
            if (c == p) break;
            int pc = f_par[c];
            while (pc != -1 && !alive[pc]) pc = f_par[pc];
            if (pc != p) break;
            int nc = f_ncol[c] + f_ncol[p];
            int r = nc + f_nupd[p];
            int64_t stored = (int64_t)nc * r - (int64_t)nc * (nc - 1) / 2;
            int64_t zeros = stored - (f_true[c] + f_true[p]);
            // a merged front must fit the LDS budget, or be a large front (too
            // tall for LDS at any width) of at most kLargeFrontCols columns
            const bool fits = panel_lds_bytes(r, nc) <= opt.lds_bytes ||
                              (panel_lds_bytes(r, 1) > opt.lds_bytes && nc <= kLargeFrontCols);
            bool ok = nc <= opt.max_super && fits &&
                      (nc <= opt.relax_small || (double)zeros <= opt.relax_frac * (double)stored);
            if (!ok) break;
            f_first[p] = f_first[c];
            f_ncol[p] = nc;
            f_true[p] += f_true[c];
            alive[c] = 0;
            f_par[c] = p;  // absorbed: redirect to p
        }
    }
    // surviving supernodes in column order
    std::vector<int> sn_first, sn_last;
    for (int f = 0; f < nf; f++)
        if (alive[f]) { sn_first.push_back(f_first[f]); sn_last.push_back(f_first[f] + f_ncol[f] - 1); }
    std::vector<int> ord(sn_first.size());
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return sn_first[a] < sn_first[b]; });
    std::vector<int> c0, c1;
    for (int i : ord) { c0.push_back(sn_first[i]); c1.push_back(sn_last[i]); }

    // ---- row structures (union of column structures and children updates) ------
    // built bottom-up; a supernode whose panel does not fit the LDS budget is
    // split into column chunks afterwards.
    auto build_structs = [&](const std::vector<int>& a0, const std::vector<int>& a1,
                             std::vector<int>& spar, std::vector<int64_t>& rofs, std::vector<int>& rws) -> bool {
        int ns = (int)a0.size();
        std::vector<int> c2s(n);
        for (int s = 0; s < ns; s++)
            for (int j = a0[s]; j <= a1[s]; j++) c2s[j] = s;
        spar.assign(ns, -1);
        for (int s = 0; s < ns; s++) spar[s] = parent[a1[s]] == -1 ? -1 : c2s[parent[a1[s]]];
        std::vector<int> chp(ns + 1, 0), chl;
        for (int s = 0; s < ns; s++) if (spar[s] != -1) chp[spar[s] + 1]++;
        for (int s = 0; s < ns; s++) chp[s + 1] += chp[s];
        chl.resize(chp[ns]);
        {
            std::vector<int> fill(chp.begin(), chp.end() - 1);
            for (int s = 0; s < ns; s++) if (spar[s] != -1) chl[fill[spar[s]]++] = s;
        }
        rofs.assign(ns + 1, 0);
        rws.clear();
        std::vector<int> mk(n, -1), buf;
        for (int s = 0; s < ns; s++) {
            if (spar[s] != -1 && spar[s] <= s) return false;  // postorder violated
            buf.clear();
            for (int j = a0[s]; j <= a1[s]; j++) { mk[j] = s; buf.push_back(j); }
            for (int j = a0[s]; j <= a1[s]; j++) {
                int v = perm[j];
                for (int64_t p = G.p[v]; p < G.p[v + 1]; p++) {
                    int i = iperm[G.a[p]];
                    if (i > a1[s] && mk[i] != s) { mk[i] = s; buf.push_back(i); }
                }
            }
            for (int q = chp[s]; q < chp[s + 1]; q++) {
                int c = chl[q];
                for (int64_t p = rofs[c] + (a1[c] - a0[c] + 1); p < rofs[c + 1]; p++) {
                    int i = rws[p];
                    if (i > a1[s] && mk[i] != s) { mk[i] = s; buf.push_back(i); }
                }
            }
            std::sort(buf.begin() + (a1[s] - a0[s] + 1), buf.end());
            rws.insert(rws.end(), buf.begin(), buf.end());
            rofs[s + 1] = (int64_t)rws.size();
        }
        return true;
    };
    std::vector<int> spar, rws;
    std::vector<int64_t> rofs;
    if (!build_structs(c0, c1, spar, rofs, rws)) { err = "internal: supernodes not in postorder"; return ST_INVALID; }
    // Split panels that exceed the LDS budget into column chunks. A chunk
    // starting at column a keeps the front rows >= a of its supernode, so every
    // chunk's update rows are exactly the next chunk's front; the last chunk
    // keeps the original update rows. Parents are then re-derived below.
    {
        std::vector<int> d0, d1, d2s;
        std::vector<int64_t> drofs(1, 0);
        std::vector<int> drws;
        for (size_t s = 0; s < c0.size(); s++) {
            int r = (int)(rofs[s + 1] - rofs[s]);
            int a = c0[s];
            while (a <= c1[s]) {
                int rr = r - (a - c0[s]);
                if (rr >= 65536) { err = "front exceeds 65535 rows"; return ST_PATTERN; }
                int w = 1;
                if (panel_lds_bytes(rr, 1) > opt.lds_bytes) {
                    // too tall for the LDS budget at any width: a large front
                    // (factored and solved in HBM), in chunks of up to
                    // kLargeFrontCols columns
                    w = std::min(c1[s] - a + 1, kLargeFrontCols);
                } else {
                    while (a + w <= c1[s] && panel_lds_bytes(rr, w + 1) <= opt.lds_bytes) w++;
                }
                d0.push_back(a);
                d1.push_back(a + w - 1);
                drws.insert(drws.end(), rws.begin() + rofs[s] + (a - c0[s]), rws.begin() + rofs[s + 1]);
                drofs.push_back((int64_t)drws.size());
                a += w;
            }
        }
        c0.swap(d0);
        c1.swap(d1);
        rofs.swap(drofs);
        rws.swap(drws);
        std::vector<int> c2s(n);
        for (size_t s = 0; s < c0.size(); s++)
            for (int j = c0[s]; j <= c1[s]; j++) c2s[j] = (int)s;
        spar.assign(c0.size(), -1);
        for (size_t s = 0; s < c0.size(); s++) {
            int nr = (int)(rofs[s + 1] - rofs[s]), nc = c1[s] - c0[s] + 1;
            // the parent front contains the smallest update row
            spar[s] = nr > nc ? c2s[rws[rofs[s] + nc]] : -1;
            if (spar[s] != -1 && spar[s] <= (int)s) { err = "internal: supernodes not in postorder"; return ST_INVALID; }
        }
    }

    // ---- supernode arrays ---------------------------------------------------------
    const int ns = (int)c0.size();
    S.ns = ns;
    S.sn_col0.resize(ns + 1);
    S.sn_ncol.resize(ns);
    S.sn_nrow.resize(ns);
    S.sn_parent = spar;
    S.sn_rowofs = rofs;
    S.rows = rws;
    for (int s = 0; s < ns; s++) {
        S.sn_col0[s] = c0[s];
        S.sn_ncol[s] = c1[s] - c0[s] + 1;
        S.sn_nrow[s] = (int)(rofs[s + 1] - rofs[s]);
    }
    S.sn_col0[ns] = n;
    std::vector<int> col2s(n);
    for (int s = 0; s < ns; s++)
        for (int j = c0[s]; j <= c1[s]; j++) col2s[j] = s;

    S.ch_ptr.assign(ns + 1, 0);
    for (int s = 0; s < ns; s++) if (spar[s] != -1) S.ch_ptr[spar[s] + 1]++;
    for (int s = 0; s < ns; s++) S.ch_ptr[s + 1] += S.ch_ptr[s];
    S.ch_list.resize(S.ch_ptr[ns]);
    {
        std::vector<int> fill(S.ch_ptr.begin(), S.ch_ptr.end() - 1);
        for (int s = 0; s < ns; s++) if (spar[s] != -1) S.ch_list[fill[spar[s]]++] = s;
    }
    S.sn_level.assign(ns, 0);
    S.nlevels = ns > 0 ? 1 : 0;
    for (int s = 0; s < ns; s++) {
        if (spar[s] != -1) S.sn_level[spar[s]] = std::max(S.sn_level[spar[s]], S.sn_level[s] + 1);
        S.nlevels = std::max(S.nlevels, S.sn_level[s] + 1);
    }
    S.lvl_ptr.assign(S.nlevels + 1, 0);
    for (int s = 0; s < ns; s++) S.lvl_ptr[S.sn_level[s] + 1]++;
    for (int l = 0; l < S.nlevels; l++) S.lvl_ptr[l + 1] += S.lvl_ptr[l];
    S.lvl_list.resize(ns);
    {
        std::vector<int> fill(S.lvl_ptr.begin(), S.lvl_ptr.end() - 1);
        for (int s = 0; s < ns; s++) S.lvl_list[fill[S.sn_level[s]]++] = s;
    }

    // relative indices of update rows in the parent's front; rel_np[s] counts
    // the update rows of s that land in the parent's own columns
    S.rel.assign(S.rows.size(), -1);
    S.rel_np.assign(ns, 0);
    for (int s = 0; s < ns; s++) {
        int p = spar[s];
        int c = S.sn_ncol[s];
        if (p == -1) {
            if (S.sn_nrow[s] != c) { err = "internal: root with update rows"; return ST_INVALID; }
            continue;
        }
        const int* pr = S.rows.data() + S.sn_rowofs[p];
        int pn = S.sn_nrow[p];
        for (int64_t q = S.sn_rowofs[s] + c; q < S.sn_rowofs[s + 1]; q++) {
            const int* it = std::lower_bound(pr, pr + pn, S.rows[q]);
            if (it == pr + pn || *it != S.rows[q]) { err = "internal: update row missing from parent front"; return ST_INVALID; }
            S.rel[q] = (int)(it - pr);
            if (S.rel[q] < S.sn_ncol[p]) S.rel_np[s]++;
        }
    }

    // inverse maps: for the child at ch_list position q of front p, the
    // update row of the child that lands on each update row of p (or -1), so
    // the entries a child passes through to p's update matrix can be
    // gathered where p's update matrix is formed
    S.pinv_ofs.assign(S.ch_list.size() + 1, 0);
    for (int p = 0; p < ns; p++)
        for (int q = S.ch_ptr[p]; q < S.ch_ptr[p + 1]; q++)
            S.pinv_ofs[q + 1] = S.pinv_ofs[q] + (S.sn_nrow[p] - S.sn_ncol[p]);
    S.pinv.assign(S.pinv_ofs.back(), -1);
    for (int p = 0; p < ns; p++)
        for (int q = S.ch_ptr[p]; q < S.ch_ptr[p + 1]; q++) {
            const int s = S.ch_list[q], cs = S.sn_ncol[s], us = S.sn_nrow[s] - cs, cp = S.sn_ncol[p];
            for (int k = S.rel_np[s]; k < us; k++) {
                const int a = S.rel[S.sn_rowofs[s] + cs + k] - cp;
                if (a < 0 || a >= S.sn_nrow[p] - cp) { err = "internal: pass-through row outside the parent's update"; return ST_INVALID; }
                S.pinv[S.pinv_ofs[q] + a] = k;
            }
        }

    // storage offsets and statistics
    S.sn_lofs.assign(ns + 1, 0);
    S.sn_uofs.assign(ns + 1, 0);
    S.sn_vofs.assign(ns + 1, 0);
    S.flops = 0;
    for (int s = 0; s < ns; s++) {
        int r = S.sn_nrow[s], c = S.sn_ncol[s], u = r - c;
        // panel stored column-major with leading dimension r|1 (odd, as in
        // LDS), padded to an even count so every panel starts 16-byte aligned
        S.sn_lofs[s + 1] = S.sn_lofs[s] + (((int64_t)(r | 1) * c + 1) & ~(int64_t)1);
        // update matrices and vectors start on 256-byte boundaries: no cache
        // line holds entries of two fronts, which matters where fronts of
        // one launch hand their results to each other on other compute units
        S.sn_uofs[s + 1] = S.sn_uofs[s] + (((int64_t)u * u + 31) & ~(int64_t)31);
        S.sn_vofs[s + 1] = S.sn_vofs[s] + ((u + 31) & ~31);
        for (int k = 0; k < c; k++) S.flops += (double)(r - k - 1) * (r - k) + (r - k - 1);
        S.max_nrow = std::max(S.max_nrow, r);
        S.max_ncol = std::max(S.max_ncol, c);
        S.max_nupd = std::max(S.max_nupd, u);
        S.n_large += panel_lds_bytes(r, c) > opt.lds_bytes ? 1 : 0;
    }
    S.lds_budget = opt.lds_bytes;
    S.lsize = S.sn_lofs[ns];
    S.usize = S.sn_uofs[ns];
    S.vsize = S.sn_vofs[ns];

    // ---- assembly map: contributions of every entry of K's lower triangle -------
    // K is walked row by row with a dense position map (pos[j] = id of entry
    // (i, j)), so every lookup is O(1). The J^T d J pairs (a, b) of entry
    // (i, j) come in ascending J-row order: the rows r holding column i, and
    // in row r the position a of column j (rows are sorted, so a <= b).
    std::vector<int> kw(nnzk, -1), kd(nnzk, -1);
    std::vector<int64_t> kpp(nnzk + 1, 0);
    std::vector<int> pa, pb;
    {
        std::vector<int64_t> pos(n, -1), fill;
        for (int pass = 0; pass < 2; pass++) {  // 0: count pairs per entry, 1: place them
            if (pass == 1) {
                for (int64_t e = 0; e < nnzk; e++) kpp[e + 1] += kpp[e];
                pa.resize(kpp[nnzk]);
                pb.resize(kpp[nnzk]);
                fill.assign(kpp.begin(), kpp.end() - 1);
            }
            for (int i = 0; i < n; i++) {
                for (int64_t e = Kp[i]; e < Kp[i + 1]; e++) pos[Kj[e]] = e;
                if (pass == 0) {
                    for (int p = wp[i]; p < wp[i + 1]; p++) kw[pos[wi[p]]] = p;
                    kd[pos[i]] = i;
                }
                for (int q = S.jt_ptr[i]; q < S.jt_ptr[i + 1]; q++) {
                    const int r = S.jt_row[q], b = S.jt_e[q];
                    for (int a = jp[r]; a <= b; a++) {
                        const int64_t e = pos[ji[a]];
                        if (pass == 0) {
                            kpp[e + 1]++;
                        } else {
                            const int64_t t = fill[e]++;
                            pa[t] = a;
                            pb[t] = b;
                        }
                    }
                }
            }
        }
    }
    // destination of each entry, then regroup entries by supernode
    std::vector<int> krow_o(nnzk), kcol_o(nnzk), ksn(nnzk), kloc(nnzk), kpr(nnzk), kpc(nnzk);
    for (int i = 0; i < n; i++)
        for (int64_t e = Kp[i]; e < Kp[i + 1]; e++) {
            int j = Kj[e];
            krow_o[e] = i;
            kcol_o[e] = j;
            int pi = iperm[i], pj = iperm[j];
            int pr = std::max(pi, pj), pc = std::min(pi, pj);
            int s = col2s[pc];
            const int* rb = S.rows.data() + S.sn_rowofs[s];
            const int* it = std::lower_bound(rb, rb + S.sn_nrow[s], pr);
            if (it == rb + S.sn_nrow[s] || *it != pr) { err = "internal: K entry outside the front"; return ST_INVALID; }
            ksn[e] = s;
            kloc[e] = ((pc - S.sn_col0[s]) << 16) | (int)(it - rb);
            kpr[e] = pr;
            kpc[e] = pc;
        }
    // Supernodes are contiguous column ranges in order and front rows are
    // sorted, so (supernode, kloc) order is (permuted column, permuted row)
    // order: two stable counting passes, by row and then by column.
    std::vector<int64_t> eord(nnzk);
    {
        std::vector<int64_t> cnt(n + 1), tmp(nnzk);
        auto pass = [&](const std::vector<int>& key, const int64_t* src, int64_t* dst) {
            std::fill(cnt.begin(), cnt.end(), 0);
            for (int64_t q = 0; q < nnzk; q++) cnt[key[src ? src[q] : q] + 1]++;
            for (int t = 0; t < n; t++) cnt[t + 1] += cnt[t];
            for (int64_t q = 0; q < nnzk; q++) {
                const int64_t e = src ? src[q] : q;
                dst[cnt[key[e]]++] = e;
            }
        };
        pass(kpr, nullptr, tmp.data());
        pass(kpc, tmp.data(), eord.data());
    }
    std::vector<int64_t> newid(nnzk);
    for (int64_t q = 0; q < nnzk; q++) newid[eord[q]] = q;
    S.k_snptr.assign(ns + 1, 0);
    S.k_loc.resize(nnzk);
    S.k_w.resize(nnzk);
    S.k_diag.resize(nnzk);
    S.k_pptr.assign(nnzk + 1, 0);
    for (int64_t q = 0; q < nnzk; q++) {
        int64_t e = eord[q];
        S.k_snptr[ksn[e] + 1]++;
        S.k_loc[q] = kloc[e];
        S.k_w[q] = kw[e];
        S.k_diag[q] = kd[e];
        S.k_pptr[q + 1] = S.k_pptr[q] + (kpp[e + 1] - kpp[e]);
    }
    for (int s = 0; s < ns; s++) S.k_snptr[s + 1] += S.k_snptr[s];
    S.pair_a.resize(kpp[nnzk]);
    S.pair_b.resize(kpp[nnzk]);
    for (int64_t q = 0; q < nnzk; q++) {
        int64_t e = eord[q];
        std::copy(pa.begin() + kpp[e], pa.begin() + kpp[e + 1], S.pair_a.begin() + S.k_pptr[q]);
        std::copy(pb.begin() + kpp[e], pb.begin() + kpp[e + 1], S.pair_b.begin() + S.k_pptr[q]);
    }
    S.k_heavy.clear();
    for (int64_t q = 0; q < nnzk; q++)
        if (S.k_pptr[q + 1] - S.k_pptr[q] > kHeavyPairs) S.k_heavy.push_back((int)q);

    // ---- symmetric row lists for K x (original numbering) -----------------------
    S.sp_ptr.assign(n + 1, 0);
    for (int64_t e = 0; e < nnzk; e++) {
        S.sp_ptr[krow_o[e] + 1]++;
        if (krow_o[e] != kcol_o[e]) S.sp_ptr[kcol_o[e] + 1]++;
    }
    for (int i = 0; i < n; i++) S.sp_ptr[i + 1] += S.sp_ptr[i];
    S.sp_e.resize(S.sp_ptr[n]);
    S.sp_col.resize(S.sp_ptr[n]);
    {
        std::vector<int64_t> fill(S.sp_ptr.begin(), S.sp_ptr.end() - 1);
        for (int i = 0; i < n; i++)  // row i: its own lower entries, then the entries (i', i), i' > i
            for (int64_t e = Kp[i]; e < Kp[i + 1]; e++) {
                int j = kcol_o[e];
                int64_t q = fill[i]++;
                S.sp_e[q] = (int)newid[e];
                S.sp_col[q] = j;
                if (j != i) {
                    int64_t q2 = fill[j]++;
                    S.sp_e[q2] = (int)newid[e];
                    S.sp_col[q2] = i;
                }
            }
    }
    // positions of every K entry in the symmetric row lists: assembly writes
    // the row-ordered copy of K that the residual reads sequentially
    S.k_csr.assign(2 * (size_t)nnzk, -1);
    for (int64_t q = 0; q < S.sp_ptr[n]; q++) {
        const int e = S.sp_e[q];
        if (S.k_csr[2 * (size_t)e] < 0) S.k_csr[2 * (size_t)e] = (int)q;
        else S.k_csr[2 * (size_t)e + 1] = (int)q;
    }
    if (nnzk >= INT32_MAX || S.sp_ptr[n] >= INT32_MAX || (int64_t)S.pair_a.size() >= INT32_MAX * 2LL) {
        err = "pattern too large for 32-bit entry ids";
        return ST_PATTERN;
    }
    S.analyze_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return ST_OK;
}

}  // namespace kkt
