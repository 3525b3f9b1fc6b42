// HIP kernels for gfx950 (MI355X): the numeric phase of the Newton-step KKT
// solve (Pacaud & Shin, arXiv 2403.15913, sections "Condensed KKT system" and
// "Hybrid linear solver").
//
//   k_assemble   K = W + Sigma_x + J^T diag(d) J for every lower entry of K
//                (eq. (kkt:condensed); d = Sigma_s for Lifted-KKT, eq.
//                (liftedkkt); d = gamma for K_gamma, eq. (hykkt)).
//   k_factor     multifrontal supernodal Cholesky, one workgroup per front:
//                the front panel lives in LDS, children's update matrices are
//                extend-added in a fixed order (deterministic), then a dense
//                partial Cholesky (POTRF + TRSM) and the update-matrix SYRK.
//   k_fwd/k_bwd  supernodal triangular sweeps L y = P b and L^T z = y.
//   k_residual   r = b - K x with the normwise / componentwise backward-error
//                reductions that drive Richardson refinement.
//   CG kernels   J^T p, J t, dots and axpys of the Schur-complement CG.
//
// All arithmetic is FP64.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <utility>

#include "device.hpp"
#include "kernels.hpp"

namespace kkt {

#ifndef KKT_BWD_SMALL_PU
#define KKT_BWD_SMALL_PU 16
#endif
#ifndef KKT_SMALL_WAVES_PER_EU
#define KKT_SMALL_WAVES_PER_EU 2
#endif
#ifndef KKT_SMALL_EU
#define KKT_SMALL_EU 12
#endif
#define KKT_ST_NOT_SPD 4
#define KKT_ST_NONFINITE 5


// ---------------------------------------------------------------------------
// fills (used instead of hipMemsetAsync so the sequences stay graph-safe)
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int* __restrict__ p, int v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// per-instance factor status pairs: (0 = ok, INT_MAX = no failing column yet)
__global__ void k_status_init(int* __restrict__ status, int ninst) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q < ninst) {
        status[2 * q] = 0;
        status[2 * q + 1] = INT_MAX;
    }
}

// segment copies: blocks (segment, part) stride over one segment each
constexpr int kCopyParts = 8;
__global__ __launch_bounds__(256) void k_copy_segments(const CopySeg* __restrict__ segs) {
    const CopySeg sg = segs[blockIdx.x / kCopyParts];
    const int part = blockIdx.x % kCopyParts;
    for (int64_t i = (int64_t)part * blockDim.x + threadIdx.x; i < sg.len; i += (int64_t)kCopyParts * blockDim.x)
        sg.dst[i] = sg.src[i];
}

// Workgroups go to the 8 XCDs in turn (workgroup b runs on XCD b mod 8) and
// every XCD has an L2 of its own. This renumbering hands each XCD one
// contiguous share of the launch's items, so neighbouring items, which read
// the same data (rows of J, a front's stored panel), meet in one L2 instead
// of being fetched into all eight.
constexpr int kNumXcd = 8;
__device__ __forceinline__ int xcd_block() {
    const int b = blockIdx.x, nb = gridDim.x;
    const int x = b % kNumXcd, q = nb / kNumXcd, rem = nb % kNumXcd;
    return x * q + min(x, rem) + b / kNumXcd;
}

// ---------------------------------------------------------------------------
// assembly: one thread per lower entry of K
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_assemble(const InstDev* __restrict__ insts, Calls C,
                                                  const WorkItem* __restrict__ items) {
    const WorkItem it = items[xcd_block()];
    const InstDev& I = insts[it.inst];
    const int64_t nnzk = I.P.k_snptr[I.P.ns];
    const int64_t e = (int64_t)it.id + threadIdx.x;
    if (e >= nnzk) return;
    const int64_t p0 = I.P.k_pptr[e], p1 = I.P.k_pptr[e + 1];
    if (p1 - p0 > kHeavyPairs) return;  // k_assemble_heavy's entry
    double v = 0.0;
    const int wi = I.P.k_w[e];
    if (wi >= 0) v += C.w[I.w_off + wi];
    const int di = I.P.k_diag[e];
    if (di >= 0) v += C.sx[I.n_off + di] + C.delta;
    const double* __restrict__ jv = C.jv + I.j_off;
    // single factors that need it keep W + Sigma_x + delta I (general HyKKT:
    // plus the inequality rows' J^T Sigma_s J, the condensed matrix K_k), for
    // the saddle-system and augmented-system residuals
    if (C.keep_k0) {
        double v0 = v;
        if (C.eqm) {
            // (J_a w) J_b with w = Sigma_s on inequality rows, 0 on equality rows
            const double* __restrict__ ss = C.ss + I.m_off;
            for (int64_t p = p0; p < p1; p++) {
                const int a = I.P.pair_a[p], r = I.P.jrow[a];
                const double w = C.eqm[r] ? 0.0 : ss[r];
                v0 += (jv[a] * w) * jv[I.P.pair_b[p]];
            }
        }
        const int c0 = I.P.k_csr[2 * e], c1 = I.P.k_csr[2 * e + 1];
        I.k0csr[c0] = v0;
        if (c1 >= 0) I.k0csr[c1] = v0;
    }
    if (C.ss) {
        // js[a] = J_a * Sigma_s[row of a] (k_jscale), so each product is
        // (J_a Sigma_s) J_b with two gathers
        const double* __restrict__ js = I.js;
        // four pairs per round: indices, then values, all loads issued before
        // the products are added in pair order
        for (int64_t p = p0; p < p1; p += 4) {
            int a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const int64_t pc = min(p + q, p1 - 1);
                a[q] = I.P.pair_a[pc];
                b[q] = I.P.pair_b[pc];
            }
            double x[4], y[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                x[q] = js[a[q]];
                y[q] = jv[b[q]];
            }
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (p + q < p1) v += x[q] * y[q];
        }
    } else {
        double acc = 0.0;
        for (int64_t p = p0; p < p1; p++) acc += jv[I.P.pair_a[p]] * jv[I.P.pair_b[p]];
        v += C.gamma * acc;
    }
    I.kval[e] = v;
    // row-ordered copy (both triangles) for the residual and K x
    const int c0 = I.P.k_csr[2 * e], c1 = I.P.k_csr[2 * e + 1];
    I.kcsr[c0] = v;
    if (c1 >= 0) I.kcsr[c1] = v;
    if (!isfinite(v)) atomicMax(&I.status[0], KKT_ST_NONFINITE);
}

// Entries of K with more than kHeavyPairs products: columns of J that many
// rows share (a stage's coupling variables) give a few entries long product
// lists, which would keep a whole wave of the one-thread-per-entry kernel
// looping for one lane. Here 16 lanes take one entry: lane l sums products
// l, l + 16, ... in order, then a fixed butterfly over the 16 lanes, so every
// run gives the same value.
__global__ __launch_bounds__(256) void k_assemble_heavy(const InstDev* __restrict__ insts, Calls C,
                                                        const WorkItem* __restrict__ items, int nitems) {
    const int h = blockIdx.x * 16 + (threadIdx.x >> 4), l = threadIdx.x & 15;
    if (h >= nitems) return;  // whole 16-lane groups leave together
    const WorkItem it = items[h];
    const InstDev& I = insts[it.inst];
    const int64_t e = it.id;
    const int64_t p0 = I.P.k_pptr[e], p1 = I.P.k_pptr[e + 1];
    const double* __restrict__ jv = C.jv + I.j_off;
    // Lifted-KKT: (J_a Sigma_s) J_b from k_jscale's scaled copy; K_gamma: J_a J_b
    const double* __restrict__ ja = C.ss ? I.js : jv;
    // HU products per lane and round: indices, then values, all loads issued
    // before the products are added in the lane's order
    constexpr int HU = 5;
    double acc = 0.0;
    for (int64_t p = p0 + l; p < p1; p += 16 * HU) {
        int a[HU], b[HU];
#pragma unroll
        for (int q = 0; q < HU; q++) {
            const int64_t pc = min(p + 16 * q, p1 - 1);
            a[q] = I.P.pair_a[pc];
            b[q] = I.P.pair_b[pc];
        }
        double x[HU], y[HU];
#pragma unroll
        for (int q = 0; q < HU; q++) {
            x[q] = ja[a[q]];
            y[q] = jv[b[q]];
        }
#pragma unroll
        for (int q = 0; q < HU; q++)
            if (p + 16 * q < p1) acc += x[q] * y[q];
    }
    // general HyKKT, single factors: the inequality rows' part alone, for K_k
    double accH = 0.0;
    if (C.eqm && C.keep_k0) {
        const double* __restrict__ ss = C.ss + I.m_off;
        for (int64_t p = p0 + l; p < p1; p += 16) {
            const int a = I.P.pair_a[p], r = I.P.jrow[a];
            const double w = C.eqm[r] ? 0.0 : ss[r];
            accH += (jv[a] * w) * jv[I.P.pair_b[p]];
        }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) {
        acc += __shfl_xor(acc, o, 16);
        accH += __shfl_xor(accH, o, 16);
    }
    if (l != 0) return;
    double v = 0.0;
    const int wi = I.P.k_w[e];
    if (wi >= 0) v += C.w[I.w_off + wi];
    const int di = I.P.k_diag[e];
    if (di >= 0) v += C.sx[I.n_off + di] + C.delta;
    const int c0 = I.P.k_csr[2 * e], c1 = I.P.k_csr[2 * e + 1];
    if (C.keep_k0) {
        I.k0csr[c0] = v + accH;
        if (c1 >= 0) I.k0csr[c1] = v + accH;
    }
    v += C.ss ? acc : C.gamma * acc;
    I.kval[e] = v;
    I.kcsr[c0] = v;
    if (c1 >= 0) I.kcsr[c1] = v;
    if (!isfinite(v)) atomicMax(&I.status[0], KKT_ST_NONFINITE);
}

// Lifted-KKT: J values scaled by their row's Sigma_s (general HyKKT: by gamma
// on the equality rows), one thread per entry
__global__ __launch_bounds__(256) void k_jscale(const InstDev* __restrict__ insts, Calls C,
                                                const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int p = it.id + threadIdx.x;
    if (p >= I.P.j_ptr[I.P.m]) return;
    const int row = I.P.jrow[p];
    const double d = (C.eqm && C.eqm[row]) ? C.gamma : C.ss[I.m_off + row];
    I.js[p] = C.jv[I.j_off + p] * d;
}

// Lifted-KKT, single factors: J's values by rows (jraw) and by columns in
// pivot order (jtv) over the entry blocks of J, or Sigma_s (rows = 1) over the
// row blocks, kept for the augmented-system solve
__global__ __launch_bounds__(256) void k_keep_lifted(const InstDev* __restrict__ insts, Calls C,
                                                     const WorkItem* __restrict__ items, int rows) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int p = it.id + threadIdx.x;
    if (rows) {
        if (p < I.P.m) I.ssv[p] = C.ss[I.m_off + p];
        return;
    }
    if (p >= I.P.j_ptr[I.P.m]) return;
    const double* __restrict__ jv = C.jv + I.j_off;
    I.jraw[p] = jv[p];
    I.jtv[p] = jv[I.P.jtp_e[p]];
}

// K_gamma: the factor keeps J's values, by rows (jraw) and by columns in pivot
// order (jtv), for the Schur-complement CG; one thread per entry
__global__ __launch_bounds__(256) void k_jcopy(const InstDev* __restrict__ insts, Calls C,
                                               const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int p = it.id + threadIdx.x;
    if (p >= I.P.j_ptr[I.P.m]) return;
    const double* __restrict__ jv = C.jv + I.j_off;
    I.jraw[p] = jv[p];
    I.jtv[p] = jv[I.P.jtp_e[p]];
}

// ---------------------------------------------------------------------------
// dense building blocks
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4f64 on gfx950: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; element e of the result in lane l is D[4e + l/16][l%16].
__device__ inline d4 mfma_f64_16x16x4(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline int rup16(int x) { return (x + 15) & ~15; }

// value of a wave-uniform lane (scalar broadcast)
__device__ inline double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// value of lane K of this lane's 16-lane row (DPP row broadcast: a
// cross-lane move inside the vector unit, no LDS round trip)
template <int K>
__device__ __forceinline__ double row_bcast(double v) {
    return __longlong_as_double(__builtin_amdgcn_mov_dpp(__double_as_longlong(v), 0x150 + K, 0xF, 0xF, false));
}

// value of the wave's first active lane, as a wave-uniform (scalar) value
__device__ inline double readfirstlane_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)b);
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Square root and its reciprocal of a Cholesky pivot d > 0 (finite): the
// hardware estimate of 1/sqrt(d) (relative error about 3e-8, subnormal d
// included) and one Newton step, which leaves a relative error of about
// 1.5e-15 over the whole positive range; no scaling or range test needed.
__device__ __forceinline__ void pivot_roots(const double d, double& inv, double& ljj) {
    const double t = __builtin_amdgcn_rsq(d);
    inv = fma(0.5 * t, fma(-d * t, t, 1.0), t);
    ljj = d * inv;
}

// f(integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time
template <int... I, class F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, I...>, F&& f) {
    (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

// 16x16 tile of A B^T from a column-major LDS panel P (leading dimension ld):
// A = rows i0..i0+15, B = rows j0..j0+15, both over columns k0..k0+K-1
// (K a multiple of 4). Rows >= rlim read as zero.
__device__ inline d4 tile_abt(const double* P, int ld, int i0, int j0, int k0, int K, int rlim, int lane) {
    const int lr = lane & 15, lk = lane >> 4;
    const int ia = i0 + lr, jb = j0 + lr;
    const bool va = ia < rlim, vb = jb < rlim;
    // rows clamped into the panel so every load is valid and unpredicated
    const int iac = min(ia, rlim - 1), jbc = min(jb, rlim - 1);
    d4 acc = {0.0, 0.0, 0.0, 0.0};
    int kk = 0;
    for (; kk + 16 <= K; kk += 16) {
        double a[4], b[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const int col = (k0 + kk + 4 * q + lk) * ld;
            a[q] = P[col + iac];
            b[q] = P[col + jbc];
        }
#pragma unroll
        for (int q = 0; q < 4; q++) acc = mfma_f64_16x16x4(va ? a[q] : 0.0, vb ? b[q] : 0.0, acc);
    }
    for (; kk < K; kk += 4) {
        const int col = (k0 + kk + lk) * ld;
        const double a = P[col + iac], b = P[col + jbc];
        acc = mfma_f64_16x16x4(va ? a : 0.0, vb ? b : 0.0, acc);
    }
    return acc;
}

// Empty asm that takes a value in a vector register: emits nothing, but
// keeps the optimizer from sinking a batch of loads into the predicated
// blocks that consume them (which would serialise the loads).
__device__ inline void pin(double& x) { asm volatile("" : "+v"(x)); }
__device__ inline void pin(double2& x) { asm volatile("" : "+v"(x.x), "+v"(x.y)); }
__device__ inline void pin(int& x) { asm volatile("" : "+v"(x)); }

// Copy n doubles (n even, both 16-byte aligned) with UNR independent 16-byte
// loads in flight per thread.
template <int UNR = 16>
__device__ inline void copy_vec(double* __restrict__ dst, const double* __restrict__ src, int n, int tid, int nt) {
    const double2* s2 = (const double2*)src;
    double2* d2 = (double2*)dst;
    const int n2 = n >> 1;
    // loads use a clamped (always valid) index so all UNR are issued
    // unconditionally and stay in registers; only the stores are predicated
    for (int base = tid; base < n2; base += nt * UNR) {
        double2 v[UNR];
#pragma unroll
        for (int k = 0; k < UNR; k++) v[k] = s2[min(base + k * nt, n2 - 1)];
#pragma unroll
        for (int k = 0; k < UNR; k++) pin(v[k]);
#pragma unroll
        for (int k = 0; k < UNR; k++) {
            const int q = base + k * nt;
            if (q < n2) d2[q] = v[k];
        }
    }
}

__device__ inline int even_up(int x) { return (x + 1) & ~1; }

// Loop over q in [0, tot) in batches: every thread first issues up to UNR
// independent loads (load(q)), then consumes them (use(q, value)), so up to
// UNR global loads per thread are in flight at once.
template <int UNR, class LoadF, class UseF>
__device__ inline void batched(int tot, int tid, int nt, LoadF load, UseF use) {
    for (int base = tid; base < tot; base += nt * UNR) {
        double v[UNR];
        // clamped indices: every load is valid, so none is predicated
#pragma unroll
        for (int k = 0; k < UNR; k++) v[k] = load(min(base + k * nt, tot - 1));
#pragma unroll
        for (int k = 0; k < UNR; k++) pin(v[k]);
#pragma unroll
        for (int k = 0; k < UNR; k++) {
            const int q = base + k * nt;
            if (q < tot) use(q, v[k]);
        }
    }
}

// lower-triangular tile enumeration: t -> (ti, tj) with tj0 <= tj <= ti < nb
__device__ inline void tri_tile(int t, int tj0, int nb, int& ti, int& tj) {
    tj = tj0;
    int span = nb - tj;
    while (t >= span) { t -= span; tj++; span = nb - tj; }
    ti = tj + t;
}

// ---------------------------------------------------------------------------
// multifrontal factorisation of one front per workgroup
// ---------------------------------------------------------------------------
// The front panel (r rows x c columns) lives in LDS, column-major with an odd
// leading dimension. It is assembled from the original entries of K and the
// children's update matrices, factored in 16-column blocks (diagonal block by
// one wave in registers, TRSM by all threads, trailing update on the matrix
// cores), then the update matrix U = -L21 L21^T is formed on the matrix cores
// and the children's pass-through entries are added to it.
constexpr int kFactorThreads = 512;
// small fronts: four waves per workgroup, so several fronts share a
// compute unit (registers for two workgroups per compute unit at least)
constexpr int kFactorThreadsSmall = 256;
static_assert(kFactorThreads == 512 && kFactorThreadsSmall == 256,
              "the panel schedule is written for eight or four waves");

// EU: extend-add entries per thread and batch (register budget of the caller)
template <int EU>
__device__ __forceinline__ void factor_front(const InstDev& I, const FrontDesc& F, double* __restrict__ P,
                                             double* invd, const bool fused_update, const bool fused_panel) {
    const PatDev& T = I.P;
    const int c = F.c, r = F.r;
    const int u = r - c, col0 = F.col0;
    // descriptor fields used inside the loops below, read once
    int* const status = I.status;
    double* const dinv = F.dinv;
    const double* const Ubase = I.U;
    const int* const chl = T.ch_list;
    const int* const sn_ncol = T.sn_ncol;
    const int* const sn_nrow = T.sn_nrow;
    const int* const rel_np = T.rel_np;
    const int64_t* const sn_uofs = T.sn_uofs;
    const int* const rel = T.rel;
    const int64_t* const sn_rowofs = T.sn_rowofs;
    const int ch0 = F.ch0, ch1 = F.ch0 + F.nch;
    const int rp = rup16(r), cp = rup16(c);
    const int ld = r | 1;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;

    // Assembly of the front: the original entries of K, then the children's
    // update matrices (entries (a, b), a >= b, whose column b maps into the
    // panel), child by child in a fixed order (two children can add into the
    // same entry). The loads of the K entries and of the first batch of the
    // first two children are all issued before the first wait, so their
    // memory round trips overlap; later batches are loaded and added in turn.
    // Loads use clamped indices, nothing is predicated.
    struct Child {
        const double* Uc;
        const int* rl;
        int uc, nb, tot;
    };
    struct ExtBatch {
        double v[EU];
        int ra[EU], rb[EU];  // relative row / column
        unsigned keep;       // bit k: entry k is in range and in the lower part
    };
    // child k (0-based): the first two from the front descriptor
    auto child_at = [&](const int k) {
        Child C;
        if (k < 2) {
            C.uc = k ? F.cuc[1] : F.cuc[0];
            C.nb = k ? F.cnb[1] : F.cnb[0];
            C.Uc = k ? F.cU[1] : F.cU[0];
            C.rl = k ? F.crl[1] : F.crl[0];
        } else {
            const int ch = __builtin_amdgcn_readfirstlane(chl[ch0 + k]);
            const int cc = __builtin_amdgcn_readfirstlane(sn_ncol[ch]);
            C.uc = __builtin_amdgcn_readfirstlane(sn_nrow[ch]) - cc;
            C.nb = __builtin_amdgcn_readfirstlane(rel_np[ch]);
            C.Uc = Ubase + sn_uofs[ch];
            C.rl = rel + sn_rowofs[ch] + cc;
        }
        C.tot = C.nb * C.uc;
        return C;
    };
    // (column, row) of the flat index q0 + k*nt by stepping, not dividing
    auto ext_load = [&](ExtBatch& B, const Child& C, const int q0) {
        const int uc = C.uc, tot = C.tot;
        const int db = nt / uc, da = nt - db * uc;
        int bq = q0 / uc, aq = q0 - bq * uc;
        // the keep flags come from the indices alone, so no load waits for
        // another before all of them are issued
        B.keep = 0;
#pragma unroll
        for (int k = 0; k < EU; k++) {
            const int qa = q0 + k * nt;
            B.keep |= (qa < tot && aq >= bq) ? 1u << k : 0u;
            B.v[k] = C.Uc[min(qa, tot - 1)];
            B.ra[k] = C.rl[qa < tot ? aq : uc - 1];
            B.rb[k] = C.rl[min(bq, C.nb - 1)];
            aq += da;
            bq += db;
            if (aq >= uc) {
                aq -= uc;
                bq++;
            }
        }
    };
    auto ext_pin = [&](ExtBatch& B) {
#pragma unroll
        for (int k = 0; k < EU; k++) {
            pin(B.v[k]);
            pin(B.ra[k]);
            pin(B.rb[k]);
        }
    };
    // the destinations of one child are distinct: read all, then write
    auto ext_add = [&](const ExtBatch& B) {
        double cur[EU];
        int dst[EU];
#pragma unroll
        for (int k = 0; k < EU; k++) {
            dst[k] = B.rb[k] * ld + B.ra[k];
            cur[k] = P[dst[k]];
        }
#pragma unroll
        for (int k = 0; k < EU; k++)
            if ((B.keep >> k) & 1u) P[dst[k]] = cur[k] + B.v[k];
    };
    // all batches of child C; the first one is already loaded when pre
    auto ext_child = [&](const Child& C, ExtBatch& B, const bool pre) {
        for (int q0 = tid; q0 < C.tot; q0 += nt * EU) {
            if (!(pre && q0 == tid)) {
                ext_load(B, C, q0);
                ext_pin(B);
            }
            ext_add(B);
        }
        __syncthreads();
    };
    const int nch = ch1 - ch0;
    Child C0 = {}, C1 = {};
    ExtBatch B0, B1;
    if (nch > 0) C0 = child_at(0);
    if (nch > 1) C1 = child_at(1);
    const bool pre0 = nch > 0 && C0.tot > 0, pre1 = nch > 1 && C1.tot > 0;
    const int nk = F.nk;
    const int* __restrict__ kl = F.kl;
    const double* __restrict__ kv = F.kv;
    constexpr int KU = 8;
    double kvv[KU];
    int klv[KU];
#pragma unroll
    for (int k = 0; k < KU; k++) {
        const int q = min(tid + k * nt, nk - 1);
        kvv[k] = kv[max(q, 0)];
        klv[k] = kl[max(q, 0)];
    }
    if (pre0) ext_load(B0, C0, tid);
    if (pre1) ext_load(B1, C1, tid);
#pragma unroll
    for (int k = 0; k < KU; k++) {
        pin(kvv[k]);
        pin(klv[k]);
    }
    if (pre0) ext_pin(B0);
    if (pre1) ext_pin(B1);
    for (int q = tid; q < ld * cp; q += nt) P[q] = 0.0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KU; k++)
        if (tid + k * nt < nk) P[(klv[k] >> 16) * ld + (klv[k] & 0xffff)] = kvv[k];
    for (int q = tid + KU * nt; q < nk; q += nt) {
        const int loc = kl[q];
        P[(loc >> 16) * ld + (loc & 0xffff)] = kv[q];
    }
    __syncthreads();
    if (nch > 0) ext_child(C0, B0, pre0);
    if (nch > 1) ext_child(C1, B1, pre1);
    for (int q = 2; q < nch; q++) {
        const Child C = child_at(q);
        ext_child(C, B0, false);
    }

    const int nbc = cp >> 4, nbr = rp >> 4;
    // diagonal block kb by one wave (the pivot chain)
    auto diag_block = [&](const int kb) {
        const int j0 = kb << 4, w = min(16, c - j0);
        // Diagonal block: each 16-lane row of the wave holds the block, lane
        // i of a row holding row j0+i (entries right of the diagonal are
        // never read back; rows past r are zero). Step j: the pivot comes
        // from lane j, column j is scaled, and every lane takes column j's
        // entries of the later rows by row broadcasts for its rank-one
        // update.
        const int i = lane & 15;
        const bool live = j0 + i < r;
        const int row = min(j0 + i, r - 1);
        double a[16];
#pragma unroll
        for (int k = 0; k < 16; k++) a[k] = P[(j0 + k) * ld + row];
        if (!live) {
#pragma unroll
            for (int k = 0; k < 16; k++) a[k] = 0.0;
        }
        static_for<16>([&](auto J) {
            constexpr int j = J;
            if (j < w) {
                double d = readfirstlane_d(row_bcast<j>(a[j]));
                if (!(d > 0.0) || !isfinite(d)) {
                    if (lane == 0) {
                        atomicMin(&status[1], col0 + j0 + j);
                        atomicMax(&status[0], KKT_ST_NOT_SPD);
                    }
                    d = 1.0;
                }
                double inv, ljj;
                pivot_roots(d, inv, ljj);
                a[j] = i == j ? ljj : a[j] * inv;
                if (lane == 0) invd[j] = inv;
                // the next pivot's column first
                static_for<16>([&](auto K) {
                    constexpr int k = K;
                    if constexpr (k > j) a[k] = fma(-a[j], row_bcast<k>(a[j]), a[k]);
                });
            }
        });
        if (lane < 16 && live) {
#pragma unroll
            for (int k = 0; k < 16; k++)
                if (k < w && k <= i) P[(j0 + k) * ld + j0 + i] = a[k];
        }
    };
    // rows below diagonal block kb, by all threads (after diag_block(kb))
    auto trsm_block = [&](const int kb) {
        const int j0 = kb << 4, w = min(16, c - j0);
        if (tid < w) dinv[j0 + tid] = invd[tid];
        // rows below the diagonal block: x = p L_kk^{-T}; column j of L_kk
        // is fetched (contiguous, broadcast to all lanes) while step j-1
        // computes
        for (int i = j0 + 16 + tid; i < r; i += nt) {
            double x[16], lc[16], ln[16];
#pragma unroll
            for (int k = 0; k < 16; k++) x[k] = P[(j0 + k) * ld + i];
#pragma unroll
            for (int k = 0; k < 16; k++) lc[k] = P[j0 * ld + j0 + k];
#pragma unroll
            for (int j = 0; j < 16; j++) {
                if (j + 1 < 16) {
#pragma unroll
                    for (int k = 0; k < 16; k++) ln[k] = P[(j0 + j + 1) * ld + j0 + k];
                }
                if (j < w) {
                    x[j] *= invd[j];
#pragma unroll
                    for (int k = j + 1; k < 16; k++) x[k] = fma(-x[j], lc[k], x[k]);
                }
#pragma unroll
                for (int k = 0; k < 16; k++) lc[k] = ln[k];
            }
#pragma unroll
            for (int k = 0; k < 16; k++)
                if (k < w) P[(j0 + k) * ld + i] = x[k];
        }
    };
    // update by block kb of the column blocks [tj0, tj1) (matrix cores);
    // tiles t0, t0 + ts, ... of that range
    auto update_tiles = [&](const int kb, const int tj0, const int tj1, const int t0, const int ts) {
        const int j0 = kb << 4;
        int ntile = 0;
        for (int jt = tj0; jt < tj1; jt++) ntile += nbr - jt;
        for (int t = t0; t < ntile; t += ts) {
            int ti, tj;
            tri_tile(t, tj0, nbr, ti, tj);
            const d4 acc = tile_abt(P, ld, ti << 4, tj << 4, j0, 16, r, lane);
            const int col = (tj << 4) + (lane & 15);
#pragma unroll
            for (int e = 0; e < 4; e++) {
                const int row = (ti << 4) + 4 * e + (lane >> 4);
                if (col < c && row >= col && row < r) P[col * ld + row] -= acc[e];
            }
        }
    };
    // Column block kb of the panel in one pass by each panel wave (0-3): every
    // 16-lane row of a wave holds the diagonal block (lane i: row j0+i) and
    // runs the pivot chain on it, and each lane also carries one row below
    // the block (wave w, lane l: row j0+16+64w+l). Step j scales column j
    // and broadcasts its entries of the diagonal rows across the 16-lane
    // rows; the same broadcast values serve the rank-one update of the
    // diagonal rows and the substitution step of the rows below. Each entry
    // sees the same operations in the same order as a pivot chain followed
    // by a row-by-row triangular solve.
    double dsave[16];  // wave 0: the last factored diagonal block (see flush_diag)
    auto panel_block = [&](const int kb) {
        const int j0 = kb << 4, w = min(16, c - j0);
        const int i = lane & 15;
        const bool live = j0 + i < r;
        const int row = min(j0 + i, r - 1);
        const int prow = j0 + 16 + (wave << 6) + lane;
        const bool plive = prow < r;
        const int prc = min(prow, r - 1);
        double a[16], x[16];
#pragma unroll
        for (int k = 0; k < 16; k++) {
            a[k] = P[(j0 + k) * ld + row];
            x[k] = P[(j0 + k) * ld + prc];
        }
        if (!live) {
#pragma unroll
            for (int k = 0; k < 16; k++) a[k] = 0.0;
        }
        // Without branches inside the steps (a failing pivot is recorded and
        // replaced by one, every step of a full block is unconditional), so
        // the updates of step j can be scheduled alongside the pivot of step
        // j+1.
        double myinv = 0.0;
        unsigned badv = 0;  // the same in every lane
        auto steps = [&](auto full) {
            static_for<16>([&](auto J) {
                constexpr int j = J;
                if (decltype(full)::value || j < w) {
                    const double dp = row_bcast<j>(a[j]);
                    const bool ok = dp > 0.0 && isfinite(dp);
                    badv |= ok ? 0u : 1u << j;
                    double inv, ljj;
                    pivot_roots(ok ? dp : 1.0, inv, ljj);
                    a[j] = i == j ? ljj : a[j] * inv;
                    myinv = i == j ? inv : myinv;
                    x[j] *= inv;
                    double lk[16];
                    static_for<16>([&](auto K) {
                        constexpr int k = K;
                        if constexpr (k > j) lk[k] = row_bcast<k>(a[j]);
                    });
                    static_for<16>([&](auto K) {
                        constexpr int k = K;
                        if constexpr (k > j) {
                            a[k] = fma(-a[j], lk[k], a[k]);
                            x[k] = fma(-x[j], lk[k], x[k]);
                        }
                    });
                }
            });
        };
        if (w == 16)
            steps(std::true_type{});
        else
            steps(std::false_type{});
        const unsigned bad = __builtin_amdgcn_readfirstlane(badv);
        if (bad && tid == 0) {
            atomicMin(&status[1], col0 + j0 + __builtin_ctz(bad));
            atomicMax(&status[0], KKT_ST_NOT_SPD);
        }
        // The other panel waves load this diagonal block at their start, in
        // the same phase: wave 0 keeps the factored block in registers and
        // writes it back after the phase's barrier (flush_diag).
        if (wave == 0) {
#pragma unroll
            for (int k = 0; k < 16; k++) dsave[k] = a[k];
            if (lane < w) dinv[j0 + lane] = myinv;
        }
        if (plive) {
#pragma unroll
            for (int k = 0; k < 16; k++)
                if (k < w) P[(j0 + k) * ld + prow] = x[k];
        }
    };
    // Right-looking blocked Cholesky with one block of look-ahead: column
    // block kb+1 takes block kb's update first; then the first waves (up to
    // four) factor column block kb+1 while the others apply block kb's
    // update to the columns beyond it. Every entry still receives the block updates in
    // block order. Fronts taller than waves 0-3 can cover, and the
    // persistent queue kernel, take the pivot chain by wave 0 and a
    // separate triangular solve of the rows below (same arithmetic).
    // panel waves: at most four, and at least one wave is left for the
    // look-ahead update
    const int maxp = min(4, nwave - 1);
    if (fused_panel && r <= 16 + maxp * 64) {
        // panel waves: one per 64 rows below the diagonal block (at least
        // one), the rest take the look-ahead update
        auto npanel = [&](const int kb) { return min(maxp, max(1, (r - (kb << 4) - 16 + 63) >> 6)); };
        // wave 0, after the barrier that ends panel_block(kb): the factored
        // diagonal block kb into the panel. Nothing reads or writes that block
        // until the panel is copied out (the updates touch the rows below it
        // and later column blocks).
        auto flush_diag = [&](const int kb) {
            const int j0 = kb << 4, w = min(16, c - j0);
            const int i = lane & 15;
            if (lane < 16 && j0 + i < r) {
#pragma unroll
                for (int k = 0; k < 16; k++)
                    if (k < w && k <= i) P[(j0 + k) * ld + j0 + i] = dsave[k];
            }
        };
        if (wave < npanel(0)) panel_block(0);
        __syncthreads();
        for (int kb = 0; kb + 1 < nbc; kb++) {
            if (wave == 0) flush_diag(kb);
            update_tiles(kb, kb + 1, kb + 2, wave, nwave);
            __syncthreads();
            const int np = npanel(kb + 1);
            if (wave < np) panel_block(kb + 1);
            else update_tiles(kb, kb + 2, nbc, wave - np, nwave - np);
            __syncthreads();
        }
        if (wave == 0) flush_diag(nbc - 1);
        __syncthreads();
    } else {
        // with eight waves, the wave that shares wave 0's SIMD (wave 4) stays
        // out of the look-ahead update, so the pivot chain has its SIMD to
        // itself; with four waves, waves 1-3 take it
        const bool eight = nwave == 8;
        const int upd_w = wave - 1 - (eight && wave > 4 ? 1 : 0), upd_n = eight ? nwave - 2 : nwave - 1;
        if (wave == 0) diag_block(0);
        __syncthreads();
        trsm_block(0);
        __syncthreads();
        for (int kb = 0; kb + 1 < nbc; kb++) {
            update_tiles(kb, kb + 1, kb + 2, wave, nwave);
            __syncthreads();
            if (wave == 0) diag_block(kb + 1);
            else if (!eight || wave != 4) update_tiles(kb, kb + 2, nbc, upd_w, upd_n);
            __syncthreads();
            trsm_block(kb + 1);
            __syncthreads();
        }
    }

    // panel -> HBM: same layout, contiguous 16-byte stores
    copy_vec(F.L, P, even_up(ld * c), tid, nt);
    if (u == 0 || !fused_update) return;
    // Update matrix U = -L21 L21^T (lower part) on the matrix cores, with
    // the children's entries that pass through to it: each lane's places
    // (a, b) of a tile find a child's entry through the child's inverse row
    // map (this front's update row -> the child's, or -1), and the entries are
    // added child by child in child order, the same additions in the same
    // order as the strip kernel's read-modify-write, with one store per
    // place. The first two children's values are read before the tile's
    // matrix-core steps (indices clamped into range, so no load is
    // predicated); further children are gathered after them.
    double* __restrict__ Us = F.U;
    const int nbu = (u + 15) >> 4;
    const int ntu = nbu * (nbu + 1) / 2;
    const int K4 = (c + 3) & ~3;
    struct PassChild {
        const double* Uc;
        const int* inv;
        int uc;
    };
    auto pass_child = [&](const int k) {
        PassChild C;
        if (k < 2) {
            C.Uc = k ? F.cU[1] : F.cU[0];
            C.inv = k ? F.cinv[1] : F.cinv[0];
            C.uc = k ? F.cuc[1] : F.cuc[0];
        } else {
            const int ch = __builtin_amdgcn_readfirstlane(chl[ch0 + k]);
            C.Uc = Ubase + sn_uofs[ch];
            C.inv = T.pinv + T.pinv_ofs[ch0 + k];
            C.uc = __builtin_amdgcn_readfirstlane(sn_nrow[ch]) - __builtin_amdgcn_readfirstlane(sn_ncol[ch]);
        }
        return C;
    };
    // this lane's four values of child C at rows a0 + 4e, column b (lower
    // places of this front's update matrix only)
    auto pass_gather = [&](const PassChild& C, const int a0, const int b, double* v, bool* in) {
        const int ib = C.inv[min(b, u - 1)];
        int ia[4];
#pragma unroll
        for (int e = 0; e < 4; e++) ia[e] = C.inv[min(a0 + 4 * e, u - 1)];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int a = a0 + 4 * e;
            in[e] = a < u && b <= a && ia[e] >= 0 && ib >= 0;
            v[e] = C.Uc[(int64_t)max(ib, 0) * C.uc + max(ia[e], 0)];
        }
    };
    PassChild P0 = {}, P1 = {};
    if (nch > 0) P0 = pass_child(0);
    if (nch > 1) P1 = pass_child(1);
    for (int t = wave; t < ntu; t += nwave) {
        int ti, tj;
        tri_tile(t, 0, nbu, ti, tj);
        const int b = (tj << 4) + (lane & 15);
        const int a0 = (ti << 4) + (lane >> 4);
        double v0[4] = {0.0, 0.0, 0.0, 0.0}, v1[4] = {0.0, 0.0, 0.0, 0.0};
        bool in0[4] = {false, false, false, false}, in1[4] = {false, false, false, false};
        if (nch > 0) pass_gather(P0, a0, b, v0, in0);
        if (nch > 1) pass_gather(P1, a0, b, v1, in1);
        const d4 acc = tile_abt(P, ld, c + (ti << 4), c + (tj << 4), 0, K4, r, lane);
        double w[4];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            w[e] = -acc[e];
            if (in0[e]) w[e] += v0[e];
            if (in1[e]) w[e] += v1[e];
        }
        for (int k = 2; k < nch; k++) {
            double vk[4];
            bool ink[4];
            pass_gather(pass_child(k), a0, b, vk, ink);
#pragma unroll
            for (int e = 0; e < 4; e++)
                if (ink[e]) w[e] += vk[e];
        }
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int a = a0 + 4 * e;
            if (a < u && b <= a) Us[(int64_t)b * u + a] = w[e];
        }
    }
    // every wave is done with the panel in LDS and with its stores before
    // the caller reuses the LDS or publishes the front
    __syncthreads();
}

__global__ __launch_bounds__(kFactorThreads) void k_factor(const InstDev* __restrict__ insts,
                                                          const FrontDesc* __restrict__ fds, int fused_update) {
    extern __shared__ __align__(16) double P[];
    __shared__ double invd[16];
    const FrontDesc& F = fds[blockIdx.x];
    factor_front<18>(insts[F.inst], F, P, invd, fused_update != 0, true);
}

// the same front factorization by four waves (every entry takes the same
// operations in the same order as in k_factor)
__global__ __launch_bounds__(kFactorThreadsSmall) __attribute__((amdgpu_waves_per_eu(KKT_SMALL_WAVES_PER_EU)))
void k_factor_small(const InstDev* __restrict__ insts, const FrontDesc* __restrict__ fds, int fused_update) {
    extern __shared__ __align__(16) double P[];
    __shared__ double invd[16];
    const FrontDesc& F = fds[blockIdx.x];
    factor_front<KKT_SMALL_EU>(insts[F.inst], F, P, invd, fused_update != 0, true);
}

// ---------------------------------------------------------------------------
// update matrix of a front by 16-column strips (level schedule)
// ---------------------------------------------------------------------------
// 16x16 tile of L21 L21^T read from a stored panel (column-major, leading
// dimension ld, kmax columns): the same k steps as tile_abt over the
// zero-padded LDS panel, with columns >= kmax contributing zeros.
__device__ inline d4 tile_abt_g(const double* __restrict__ Lp, int ld, int i0, int j0, int kmax, int rlim,
                                int lane) {
    const int lr = lane & 15, lk = lane >> 4;
    const int ia = i0 + lr, jb = j0 + lr;
    const bool va = ia < rlim, vb = jb < rlim;
    const int iac = min(ia, rlim - 1), jbc = min(jb, rlim - 1);
    // every column's loads are issued before the first step (kmax <= 128:
    // at most 32 steps of 4); indices past the last step repeat it, so no
    // load is predicated, and only the steps below nq run
    const int nq = (kmax + 3) >> 2;
    double a[32], b[32];
#pragma unroll
    for (int q = 0; q < 32; q++) {
        const int col = min(4 * min(q, nq - 1) + lk, kmax - 1) * ld;
        a[q] = Lp[col + iac];
        b[q] = Lp[col + jbc];
    }
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 32; q++) {
        if (q < nq) {
            const bool vk = 4 * q + lk < kmax;
            acc = mfma_f64_16x16x4(va && vk ? a[q] : 0.0, vb && vk ? b[q] : 0.0, acc);
        }
    }
    return acc;
}

// One wave per 16 x 16 tile of U = -L21 L21^T (lower part), on the matrix
// cores from the stored panel, with the children's update entries that pass
// through to it added in the tile epilogue. Each entry of U receives the same
// operations, in the same order, as in the factor kernel's fused path, so the
// two paths agree bitwise. (A tile per wave keeps each wave to one round trip
// for its loads and one matrix-core chain.)
constexpr int kUpdThreads = 64;
__global__ __launch_bounds__(kUpdThreads) void k_update(const InstDev* __restrict__ insts,
                                                       const FrontDesc* __restrict__ fds,
                                                       const StripItem* __restrict__ items) {
    const StripItem it = items[xcd_block()];
    const FrontDesc& F = fds[it.item];
    const InstDev& I = insts[F.inst];
    const PatDev& T = I.P;
    const int c = F.c, r = F.r;
    const int u = r - c, ld = r | 1;
    const int lane = threadIdx.x;
    const double* __restrict__ Lp = F.L;
    double* __restrict__ Us = F.U;
    const int ti = it.tile >> 16, tj = it.tile & 0xffff;
    const int nch = F.nch;
    // the children's pass-through entries of this lane's places, through
    // their inverse row maps, added in child order before the one store
    auto child_vals = [&](const int k, const int a0, const int b, double* v, bool* in) {
        const double* Uc;
        const int* inv;
        int uc;
        if (k < 2) {
            Uc = k ? F.cU[1] : F.cU[0];
            inv = k ? F.cinv[1] : F.cinv[0];
            uc = k ? F.cuc[1] : F.cuc[0];
        } else {
            const int ch = __builtin_amdgcn_readfirstlane(T.ch_list[F.ch0 + k]);
            Uc = I.U + T.sn_uofs[ch];
            inv = T.pinv + T.pinv_ofs[F.ch0 + k];
            uc = __builtin_amdgcn_readfirstlane(T.sn_nrow[ch]) - __builtin_amdgcn_readfirstlane(T.sn_ncol[ch]);
        }
        const int ib = inv[min(b, u - 1)];
        int ia[4];
#pragma unroll
        for (int e = 0; e < 4; e++) ia[e] = inv[min(a0 + 4 * e, u - 1)];
#pragma unroll
        for (int e = 0; e < 4; e++) {
            const int a = a0 + 4 * e;
            in[e] = a < u && b <= a && ia[e] >= 0 && ib >= 0;
            v[e] = Uc[(int64_t)max(ib, 0) * uc + max(ia[e], 0)];
        }
    };
    const int b = (tj << 4) + (lane & 15);
    const int a0 = (ti << 4) + (lane >> 4);
    double v0[4] = {0.0, 0.0, 0.0, 0.0}, v1[4] = {0.0, 0.0, 0.0, 0.0};
    bool in0[4] = {false, false, false, false}, in1[4] = {false, false, false, false};
    if (nch > 0) child_vals(0, a0, b, v0, in0);
    if (nch > 1) child_vals(1, a0, b, v1, in1);
    const d4 acc = tile_abt_g(Lp, ld, c + (ti << 4), c + (tj << 4), c, r, lane);
    double w[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
        w[e] = -acc[e];
        if (in0[e]) w[e] += v0[e];
        if (in1[e]) w[e] += v1[e];
    }
    for (int k = 2; k < nch; k++) {
        double vk[4];
        bool ink[4];
        child_vals(k, a0, b, vk, ink);
#pragma unroll
        for (int e = 0; e < 4; e++)
            if (ink[e]) w[e] += vk[e];
    }
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const int a = a0 + 4 * e;
        if (a < u && b <= a) Us[(int64_t)b * u + a] = w[e];
    }
}

// ---------------------------------------------------------------------------
// large fronts: panels too tall for a workgroup's LDS (level schedule)
// ---------------------------------------------------------------------------
// The panel is assembled and factored in place in its HBM slot by one
// workgroup per front; the update matrix is then formed by k_update's tiles,
// which read the stored panel. Each entry of the panel takes the operations
// of the LDS front kernel's non-fused path in the same order (assembly, the
// pivot chain of each diagonal block, the row-by-row solve below it, the
// blocks' updates in block order), so the factor does not depend on where
// the panel lives. Columns past the panel read as zero, as the zero-padded
// LDS panel does. Large fronts have at most 64 columns.
constexpr int kBigThreads = 256;
constexpr int kBigMaxCols = kLargeFrontCols;

// Pivot chain of diagonal block j0 (width w) of a panel in HBM, by one wave:
// lane i of each 16-lane row ends with row j0 + i of L_kk in a[0 .. i] (and
// the scaled entries of rows past the block's columns), lanes 0 .. w-1 of
// invd the pivot reciprocals; the returned mask has bit j set for a failed
// pivot j (replaced by one).
__device__ inline unsigned big_diag_chain(const double* P, int ld, int r, int j0, int w, int lane, double* a,
                                          double* invd) {
    const int i = lane & 15;
    const bool live = j0 + i < r;
    const int row = min(j0 + i, r - 1);
#pragma unroll
    for (int k = 0; k < 16; k++) a[k] = (live && k < w) ? P[(int64_t)(j0 + k) * ld + row] : 0.0;
    unsigned bad = 0;
    static_for<16>([&](auto J) {
        constexpr int j = J;
        if (j < w) {
            double d = readfirstlane_d(row_bcast<j>(a[j]));
            if (!(d > 0.0) || !isfinite(d)) {
                bad |= 1u << j;
                d = 1.0;
            }
            double inv, ljj;
            pivot_roots(d, inv, ljj);
            a[j] = i == j ? ljj : a[j] * inv;
            if (lane == 0) invd[j] = inv;
            static_for<16>([&](auto K) {
                constexpr int k = K;
                if constexpr (k > j) a[k] = fma(-a[j], row_bcast<k>(a[j]), a[k]);
            });
        }
    });
    return bad;
}

// Assembly of large fronts: workgroup (f, b, z) takes column block b and
// rows 256 z .. 256 z + 255 of large front f: zeroes that part of its
// columns, writes K's entries there, then adds the children's update entries
// that land there, child by child (the entries of one child are distinct; a
// child's update columns mapping into the block, and its update rows mapping
// into the row range, are contiguous ranges, its relative rows being
// ascending). Every entry belongs to one workgroup and takes the same
// operations in the same order as with whole columns per workgroup.
constexpr int kBigInitRows = 256;
__global__ __launch_bounds__(kBigThreads) void k_big_init(const InstDev* __restrict__ insts,
                                                        const FrontDesc* __restrict__ fds) {
    const FrontDesc& F = fds[blockIdx.x];
    const int c = F.c, r = F.r, ld = r | 1;
    const int b0 = blockIdx.y << 4, r0 = (int)blockIdx.z * kBigInitRows;
    if (b0 >= c || r0 >= r) return;
    const int b1 = min(c, b0 + 16), r1 = min(r, r0 + kBigInitRows), nr = r1 - r0;
    const InstDev& I = insts[F.inst];
    const PatDev& T = I.P;
    double* const P = F.L;
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int q = tid; q < (b1 - b0) * nr; q += nt) {
        const int col = b0 + q / nr, row = r0 + (q - (q / nr) * nr);
        P[(int64_t)col * ld + row] = 0.0;
    }
    __syncthreads();
    for (int q = tid; q < F.nk; q += nt) {
        const int loc = F.kl[q];
        const int col = loc >> 16, row = loc & 0xffff;
        if (col >= b0 && col < b1 && row >= r0 && row < r1) P[(int64_t)col * ld + row] = F.kv[q];
    }
    __syncthreads();
    // first index of the ascending rl[0 .. n) at or above v
    auto lower = [](const int* rl, int n, int v) {
        int lo = 0, hi = n;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (rl[mid] < v) lo = mid + 1;
            else hi = mid;
        }
        return lo;
    };
    for (int k = 0; k < F.nch; k++) {
        const int ch = T.ch_list[F.ch0 + k];
        const int cc = T.sn_ncol[ch];
        const int uc = T.sn_nrow[ch] - cc, nb = T.rel_np[ch];
        const double* const Uc = I.U + T.sn_uofs[ch];
        const int* const rl = T.rel + T.sn_rowofs[ch] + cc;
        // child update columns e0 .. e1-1 map into columns b0 .. b1-1, its
        // update rows a0 .. a1-1 into rows r0 .. r1-1
        const int e0 = lower(rl, nb, b0), e1 = lower(rl, nb, b1);
        const int a0 = lower(rl, uc, r0), a1 = lower(rl, uc, r1), na = a1 - a0;
        const int64_t ctot = (int64_t)(e1 - e0) * na;
        for (int64_t q = tid; q < ctot; q += nt) {
            const int b = e0 + (int)(q / na), a = a0 + (int)(q - (int64_t)(b - e0) * na);
            if (a >= b) P[(int64_t)rl[b] * ld + rl[a]] += Uc[(int64_t)b * uc + a];
        }
        __syncthreads();
    }
}

// Rows below diagonal block kb of large fronts: workgroup (f, g) recomputes
// the block's pivot chain from the panel (every workgroup the same values),
// then solves rows j0 + 16 + 256 g + tid (x = p L_kk^{-T}, the row-by-row
// arithmetic of the LDS kernel). The factored block itself is written by
// k_big_tiles, after every workgroup here has read it.
__global__ __launch_bounds__(kBigThreads) void k_big_trsm(const FrontDesc* __restrict__ fds, int kb) {
    __shared__ double Ld[16 * 17];
    __shared__ double invd[16];
    const FrontDesc& F = fds[blockIdx.x];
    const int c = F.c, r = F.r, ld = r | 1;
    const int j0 = kb << 4;
    const int rows0 = j0 + 16 + (int)blockIdx.y * kBigThreads;
    if (j0 >= c || rows0 >= r) return;
    const int w = min(16, c - j0);
    double* const P = F.L;
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid < 64) {
        double a[16];
        big_diag_chain(P, ld, r, j0, w, lane, a, invd);
        const int i = lane & 15;
        if (lane < 16) {
#pragma unroll
            for (int k = 0; k < 16; k++) Ld[k * 17 + i] = a[k];  // column k, row j0 + i
        }
    }
    __syncthreads();
    const int i = rows0 + tid;
    if (i >= r) return;
    double x[16], lc[16];
#pragma unroll
    for (int k = 0; k < 16; k++) x[k] = k < w ? P[(int64_t)(j0 + k) * ld + i] : 0.0;
#pragma unroll
    for (int j = 0; j < 16; j++) {
        if (j < w) {
#pragma unroll
            for (int k = 0; k < 16; k++) lc[k] = Ld[j * 17 + k];
            x[j] *= invd[j];
#pragma unroll
            for (int k = j + 1; k < 16; k++) x[k] = fma(-x[j], lc[k], x[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 16; k++)
        if (k < w) P[(int64_t)(j0 + k) * ld + i] = x[k];
}

// After k_big_trsm(kb): the later column blocks of large fronts take block
// kb's update on the matrix cores, one 16 x 16 tile per wave (workgroup
// (f, h) takes tiles 4h .. 4h+3 of front f), and workgroup (f, 0) writes the
// factored diagonal block kb, its pivot reciprocals and any failed pivot.
__global__ __launch_bounds__(kBigThreads) void k_big_tiles(const InstDev* __restrict__ insts,
                                                         const FrontDesc* __restrict__ fds, int kb) {
    __shared__ double invd[16];
    const FrontDesc& F = fds[blockIdx.x];
    const int c = F.c, r = F.r, ld = r | 1;
    const int j0 = kb << 4;
    if (j0 >= c) return;
    const int w = min(16, c - j0);
    double* const P = F.L;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    if (blockIdx.y == 0 && wave == 0) {
        double a[16];
        const unsigned bad = big_diag_chain(P, ld, r, j0, w, lane, a, invd);
        if (bad && lane == 0) {
            int* const status = insts[F.inst].status;
            atomicMin(&status[1], F.col0 + j0 + __builtin_ctz(bad));
            atomicMax(&status[0], KKT_ST_NOT_SPD);
        }
        const int i = lane & 15;
        if (lane < 16 && j0 + i < r) {
#pragma unroll
            for (int k = 0; k < 16; k++)
                if (k < w && k <= i) P[(int64_t)(j0 + k) * ld + j0 + i] = a[k];
        }
        if (lane < w) F.dinv[j0 + lane] = invd[lane];
    }
    const int nbc = (c + 15) >> 4, nbr = (r + 15) >> 4;
    if (kb + 1 >= nbc) return;
    int ntile = 0;
    for (int jt = kb + 1; jt < nbc; jt++) ntile += nbr - jt;
    const int t = (int)blockIdx.y * (kBigThreads >> 6) + wave;
    if (t >= ntile) return;
    int ti, tj;
    tri_tile(t, kb + 1, nbr, ti, tj);
    const d4 acc = tile_abt(P, ld, ti << 4, tj << 4, j0, 16, r, lane);
    const int col = (tj << 4) + (lane & 15);
#pragma unroll
    for (int e = 0; e < 4; e++) {
        const int row = (ti << 4) + 4 * e + (lane >> 4);
        if (col < c && row >= col && row < r) P[(int64_t)col * ld + row] -= acc[e];
    }
}

// ---------------------------------------------------------------------------
// dependency-driven (persistent) scheduling
// ---------------------------------------------------------------------------
// Workgroups take tickets in a topological order of the fronts (children
// before parents), wait until the children have published, process the
// front, release their writes at agent scope and count themselves done in
// the parent. A workgroup holding ticket t only waits for fronts with smaller
// tickets, which are held by running workgroups, so the queue always drains.
// Every wait is bounded: past the limit it latches an error and proceeds.
//
// All control flow of the persistent loops is wave-uniform. The scheduling
// steps run on wave 0 with every lane active (the test is on an SGPR), and
// only lane 0 adds to a counter, through the value it adds rather than a
// branch. A lane-divergent test such as threadIdx.x == 0 at both ends of the
// loop lets the optimizer thread the back-edge past the barriers; the loop
// then exits lane by lane and the other lanes of wave 0 re-run the body with
// the previous ticket.
constexpr long kSpinLimit = 1L << 22;

__device__ inline bool sched_wave() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0; }
__device__ inline int lane0() { return (threadIdx.x & 63) == 0 ? 1 : 0; }

// called by a whole wave; the counter is read into a scalar register
__device__ inline void wait_at_least(const int* p, int v, int* err) {
    for (long spins = 0;; ++spins) {
        const int cur = __builtin_amdgcn_readfirstlane(__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
        if (cur >= v) break;
        if (spins > kSpinLimit) {
            atomicMax(err, 1);
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

// called by a whole wave; adds exactly one
__device__ inline void publish_add(int* p) {
    __hip_atomic_fetch_add(p, lane0(), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// The ticket is broadcast through LDS and then moved to a scalar register,
// so everything derived from it (front index, sizes, loop bounds) is
// wave-uniform and every barrier below sits in uniform control flow.
__device__ inline int take_ticket(int* ticket, int* slot) {
    if (sched_wave()) {
        // lane 0 adds one; its return value is the ticket whatever the lane order
        const int old = atomicAdd(ticket, lane0());
        *slot = __builtin_amdgcn_readfirstlane(old);
    }
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(*slot);
    __syncthreads();
    return t;
}

// the persistent loop keeps its scheduling state live across the front, so
// its extend-add batches are smaller (no register spills)
constexpr int kQueueExtBatch = 12;

__global__ __launch_bounds__(kFactorThreads) void k_factor_queue(const InstDev* __restrict__ insts,
                                                                const FrontDesc* __restrict__ fds, DepLists D) {
    extern __shared__ __align__(16) double P[];
    __shared__ double invd[16];
    __shared__ int slot;
    for (;;) {
        const int t = take_ticket(D.ticket, &slot);
        if (t >= D.nitems) break;
        const int need = __builtin_amdgcn_readfirstlane(D.nchild[t]);
        const int par = __builtin_amdgcn_readfirstlane(D.parent[t]);
        if (sched_wave()) wait_at_least(D.cnt + t, need, D.err);
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const FrontDesc& F = fds[t];
        factor_front<kQueueExtBatch>(insts[F.inst], F, P, invd, true, true);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (sched_wave() && par >= 0) publish_add(D.cnt + par);
    }
}

// ---------------------------------------------------------------------------
// triangular solve with the c x c diagonal triangle of a staged panel, by
// one wave (c <= 128): lane l carries rows l and l + 64 in x0 and x1, dv
// holds the pivot reciprocals. Blocks of 16 columns: the block's own
// triangle is read into registers first, so its 16 dependent steps are
// register FMAs with row broadcasts; the rows outside the block then take
// the block's contribution with all their LDS loads issued together.
// Each row's terms are subtracted in the same order as plain substitution.
// ---------------------------------------------------------------------------
// L11^T x = t (backward), blocks from the last one down
__device__ inline void tri_bwd_wave(const double* __restrict__ P, int ld, int c, const double* __restrict__ dv,
                                    double& x0, double& x1, int lane) {
    for (int j0 = (c - 1) & ~15; j0 >= 0; j0 -= 16) {
        const int nb = min(16, c - j0);
        const bool hi = j0 >= 64;
        const int rb = lane - (j0 & 63);
        const bool inblk = rb >= 0 && rb < nb;
        const int rbc = min(max(rb, 0), nb - 1);
        // Lc[k] = L[j0 + k][j0 + rb] for k > rb (row k of the block, this lane's column)
        double Lc[16];
        const double* colr = P + (j0 + rbc) * ld + j0;
#pragma unroll
        for (int k = 0; k < 16; k++) Lc[k] = colr[min(k, nb - 1)];
#pragma unroll
        for (int k = 0; k < 16; k++) Lc[k] = (inblk && k > rb && k < nb) ? Lc[k] : 0.0;
        const double d = dv[j0 + rbc];
        double tb = hi ? x1 : x0;
        // the chain runs inside the block's 16-lane row: step k takes lane
        // k's value by a row broadcast (lanes of the row past the block
        // hold zeros and have zero coefficients; other rows' results are
        // discarded)
        static_for<16>([&](auto K) {
            constexpr int k = 15 - decltype(K)::value;
            tb = fma(-Lc[k], row_bcast<k>(tb * d), tb);
        });
        const double xv = tb * d;
        if (inblk) {
            if (hi) x1 = xv;
            else x0 = xv;
        }
        // the block's values for the rows above it, from every lane
        double x[16];
#pragma unroll
        for (int k = 0; k < 16; k++) x[k] = j0 > 0 ? readlane_d(xv, (j0 & 63) + k) : 0.0;
        if (j0 > 0) {  // rows 0 .. j0-1 lie above the block
            const int i0 = min(lane, j0 - 1), i1 = min(lane + 64, j0 - 1);
            double a0[16], a1[16];
#pragma unroll
            for (int k = 0; k < 16; k++) {
                const int kr = j0 + min(k, nb - 1);
                a0[k] = P[i0 * ld + kr];
                a1[k] = P[i1 * ld + kr];
            }
            double s0 = x0, s1 = x1;
#pragma unroll
            for (int k = 15; k >= 0; k--) {
                s0 = fma(-a0[k], x[k], s0);
                s1 = fma(-a1[k], x[k], s1);
            }
            if (lane < j0) x0 = s0;
            if (lane + 64 < j0) x1 = s1;
        }
    }
}

// ---------------------------------------------------------------------------
// triangular sweeps (y holds the permuted right-hand side, then the solution)
// ---------------------------------------------------------------------------
// The panel is staged in LDS (odd leading dimension); the c x c triangle is
// solved by one wave in 16-column blocks (each block's 16-step chain by
// DPP row broadcasts), the rectangular part by all threads. Reciprocals of
// the pivots come from the factorisation.
constexpr int kSolveThreads = 256;
static_assert(kSolveThreads == 256, "the sweep work splits assume 256 threads");

__device__ __forceinline__ void fwd_front(const InstDev& I, const FrontDesc& F, double* __restrict__ sh) {
    const PatDev& T = I.P;
    const int c = F.c, r = F.r;
    const int u = r - c;
    const int ld = r | 1;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
    double* P = sh;
    double* w = sh + even_up(ld * c);
    double* va = w + c;
    double* dv = va + u;
    // The panel is staged one 16-column block at a time: block b is one
    // contiguous range of 8 ld double2 in HBM and in LDS. Block 0 comes
    // with the prologue; block kb+1 is loaded into registers while phase
    // kb computes and stored before the phase's barrier. Every load of the
    // prologue is issued before the first wait: panel block 0, the
    // right-hand side and pivot reciprocals of the front's columns
    // (c <= 128 < threads), and the first entries of the first two
    // children's update vectors with their relative indices.
    constexpr int BU = 8;  // double2 per thread and block in registers (ld < 256)
    const double2* __restrict__ s2 = (const double2*)F.L;
    double2* d2 = (double2*)P;
    const int n2 = even_up(ld * c) >> 1;
    const int bw2 = 8 * ld;
    double2 pb[BU];
    auto blk_load = [&](const int bk) {
        const int q0 = bk * bw2, q1 = min(q0 + bw2, n2);
#pragma unroll
        for (int k = 0; k < BU; k++) pb[k] = s2[min(q0 + tid + k * nt, q1 - 1)];
    };
    auto blk_store = [&](const int bk) {
        const int q0 = bk * bw2, q1 = min(q0 + bw2, n2);
#pragma unroll
        for (int k = 0; k < BU; k++) pin(pb[k]);
#pragma unroll
        for (int k = 0; k < BU; k++)
            if (q0 + tid + k * nt < q1) d2[q0 + tid + k * nt] = pb[k];
        for (int q = q0 + tid + BU * nt; q < q1; q += nt) d2[q] = s2[q];
    };
    const int nblk = (c + 15) >> 4;
    blk_load(0);
    const int tc = min(tid, c - 1);
    double wy = F.y[tc], wd = F.dinv[tc];
    const int ch0 = F.ch0, nch = F.nch, ch1 = ch0 + nch;
    struct VChild {
        const double* Vc;
        const int* rl;
        int uc;
    };
    // child at ch_list position q; the first two from the front descriptor
    auto vchild = [&](const int q) {
        VChild C;
        const int k = q - ch0;
        if (k < 2) {
            C.uc = k ? F.cuc[1] : F.cuc[0];
            C.Vc = k ? F.cV[1] : F.cV[0];
            C.rl = k ? F.crl[1] : F.crl[0];
        } else {
            const int ch = __builtin_amdgcn_readfirstlane(T.ch_list[q]);
            const int cc = __builtin_amdgcn_readfirstlane(T.sn_ncol[ch]);
            C.uc = __builtin_amdgcn_readfirstlane(T.sn_nrow[ch]) - cc;
            C.Vc = I.V + T.sn_vofs[ch];
            C.rl = T.rel + T.sn_rowofs[ch] + cc;
        }
        return C;
    };
    VChild V0 = {}, V1 = {};
    double v0 = 0.0, v1 = 0.0;
    int r0 = 0, r1 = 0;
    if (nch > 0) {
        V0 = vchild(ch0);
        const int a = min(tid, V0.uc - 1);
        v0 = V0.Vc[a];
        r0 = V0.rl[a];
    }
    if (nch > 1) {
        V1 = vchild(ch0 + 1);
        const int a = min(tid, V1.uc - 1);
        v1 = V1.Vc[a];
        r1 = V1.rl[a];
    }
    pin(wy);
    pin(wd);
    pin(v0);
    pin(v1);
    pin(r0);
    pin(r1);
    blk_store(0);
    if (tid < c) {
        w[tid] = wy;
        dv[tid] = wd;
    }
    for (int t = tid; t < u; t += nt) va[t] = 0.0;
    __syncthreads();
    if (nblk > 1) blk_load(1);
    // children's update vectors, child by child (entries of one child are
    // distinct; two children can add into the same entry)
    auto add_child = [&](const VChild& C, const bool pre, const double vp, const int rp) {
        for (int a = tid; a < C.uc; a += nt) {
            const bool first = pre && a == tid;
            const int ra = first ? rp : C.rl[a];
            const double v = first ? vp : C.Vc[a];
            if (ra < c) w[ra] += v;
            else va[ra - c] += v;
        }
        __syncthreads();
    };
    if (nch > 0) add_child(V0, true, v0, r0);
    if (nch > 1) add_child(V1, true, v1, r1);
    for (int q = ch0 + 2; q < ch1; q++) add_child(vchild(q), false, 0.0, 0);
    // L11 y = w and the update rows' GEMV, pipelined by 16-column blocks.
    // Phase kb: wave 0 takes block kb-1's contribution into block kb's
    // rows, then solves block kb (its triangle in registers, row
    // broadcasts); meanwhile the other waves take block kb-1's contribution
    // into every later row (triangle rows past block kb and the update
    // rows). Every row subtracts its terms in ascending column order.
    const int wave = tid >> 6;
    for (int kb = 0; kb <= nblk; kb++) {
        const int p0 = (kb - 1) << 4, nprev = min(16, c - p0);
        if (wave == 0 && kb < nblk) {
            const int j0 = kb << 4, nbk = min(16, c - j0);
            const bool inb = lane < nbk;
            const int row = j0 + min(lane, nbk - 1);
            double wb = w[row];
            if (kb > 0) {
                double a[16], yv[16];
#pragma unroll
                for (int j = 0; j < 16; j++) {
                    a[j] = P[(p0 + j) * ld + row];
                    yv[j] = w[p0 + j];
                }
#pragma unroll
                for (int j = 0; j < 16; j++) wb = fma(-a[j], yv[j], wb);
            }
            double Lr[16];
#pragma unroll
            for (int k = 0; k < 16; k++) Lr[k] = P[min(j0 + k, c - 1) * ld + row];
#pragma unroll
            for (int k = 0; k < 16; k++) Lr[k] = (inb && k < lane) ? Lr[k] : 0.0;
            const double d = dv[row];
            // lanes 0-15 hold the block's rows; step k takes lane k's value
            // by a row broadcast (coefficients past the block are zero)
            static_for<16>([&](auto K) {
                constexpr int k = K;
                wb = fma(-Lr[k], row_bcast<k>(wb * d), wb);
            });
            if (inb) w[j0 + lane] = wb * d;
        } else if (kb > 0) {
            // rows after block kb: triangle rows, then the update rows
            const int r1 = min(c, (kb + 1) << 4), ntr = c - r1;
            const int t0 = kb < nblk ? tid - 64 : tid, ts = kb < nblk ? nt - 64 : nt;
            double yv[16];
#pragma unroll
            for (int j = 0; j < 16; j++) yv[j] = j < nprev ? w[p0 + j] : 0.0;
            for (int q = t0; q < ntr + u; q += ts) {
                const int prow = q < ntr ? r1 + q : c + (q - ntr);
                double a[16];
#pragma unroll
                for (int j = 0; j < 16; j++) a[j] = P[(p0 + min(j, nprev - 1)) * ld + prow];
                double acc = q < ntr ? w[prow] : va[q - ntr];
#pragma unroll
                for (int j = 0; j < 16; j++) acc = fma(-a[j], yv[j], acc);
                if (q < ntr) w[prow] = acc;
                else va[q - ntr] = acc;
            }
        }
        if (kb + 1 < nblk) blk_store(kb + 1);
        __syncthreads();
        if (kb + 2 < nblk) blk_load(kb + 2);
    }
    double* __restrict__ Vs = F.V;
    for (int i = tid; i < u; i += nt) Vs[i] = va[i];
    for (int t = tid; t < c; t += nt) F.y[t] = w[t];
}

// PU: 16-byte panel loads per thread in flight while staging (fewer for
// small panels keeps the registers low enough for more fronts per compute
// unit; the arithmetic does not depend on it)
template <int PU = 32>
__device__ __forceinline__ void bwd_front(const FrontDesc& F, double* __restrict__ sh) {
    const int c = F.c, r = F.r;
    const int u = r - c;
    double* const yb = F.y - F.col0;  // the instance's work vector
    const int ld = r | 1;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
    double* P = sh;
    double* t = sh + even_up(ld * c);
    double* zu = t + c;
    double* dv = zu + u;
    const int* __restrict__ rw = F.rw;
    // The update rows' indices are loaded first, so the gather of their
    // values waits only for them while the panel loads stay in flight.
    int ri = u > 0 ? rw[min(tid, u - 1)] : 0;
    const double2* __restrict__ s2 = (const double2*)F.L;
    double2* d2 = (double2*)P;
    const int n2 = even_up(ld * c) >> 1;
    double2 pv[PU];
#pragma unroll
    for (int k = 0; k < PU; k++) pv[k] = s2[min(tid + k * nt, n2 - 1)];
    double wd = F.dinv[min(tid, c - 1)];
    pin(ri);
    double zy = u > 0 ? yb[ri] : 0.0;
#pragma unroll
    for (int k = 0; k < PU; k++) pin(pv[k]);
    pin(wd);
    pin(zy);
#pragma unroll
    for (int k = 0; k < PU; k++)
        if (tid + k * nt < n2) d2[tid + k * nt] = pv[k];
    for (int q = tid + PU * nt; q < n2; q += nt) d2[q] = s2[q];
    if (tid < u) zu[tid] = zy;
    for (int i = tid + nt; i < u; i += nt) zu[i] = yb[rw[i]];
    if (tid < c) dv[tid] = wd;
    __syncthreads();
    // t = y1 - L21^T z: G consecutive lanes per column (G c <= 256 for
    // c <= 128), each with four running sums over rows g, g + G, ...; a
    // group's sums are combined in a fixed order
    {
        const int lg = c <= 16 ? 4 : c <= 32 ? 3 : c <= 64 ? 2 : 1, G = 1 << lg;
        const int k = tid >> lg, g = tid & (G - 1);
        double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
        if (k < c) {
            const double* col = P + k * ld + c;
            int i = g;
            for (; i + 3 * G < u; i += 4 * G) {
                a0 = fma(col[i], zu[i], a0);
                a1 = fma(col[i + G], zu[i + G], a1);
                a2 = fma(col[i + 2 * G], zu[i + 2 * G], a2);
                a3 = fma(col[i + 3 * G], zu[i + 3 * G], a3);
            }
            for (; i < u; i += G) a0 = fma(col[i], zu[i], a0);
        }
        double part = (a0 + a1) + (a2 + a3);
        for (int off = G >> 1; off > 0; off >>= 1) part += __shfl_xor(part, off);
        if (k < c && g == 0) t[k] = F.y[k] - part;
    }
    __syncthreads();
    if (tid < 64) {
        double x0 = lane < c ? t[lane] : 0.0;
        double x1 = lane + 64 < c ? t[lane + 64] : 0.0;
        tri_bwd_wave(P, ld, c, dv, x0, x1, lane);
        if (lane < c) F.y[lane] = x0;
        if (lane + 64 < c) F.y[lane + 64] = x1;
    }
}

// skip modes of the sweeps: SKIP_NONE runs every front; SKIP_REFINE skips
// the fronts of instances whose refinement has stopped, SKIP_CG those whose
// CG has stopped (the queued rounds after a stop decision do nothing)
__device__ __forceinline__ bool front_idle(const FrontDesc& F, int skip) {
    return skip == SKIP_REFINE ? *F.done != 0 : (skip == SKIP_CG ? *F.cgdone != 0 : false);
}

// Forward sweep of large fronts, one workgroup per front: the c x c triangle
// is staged in LDS, the children's update vectors are added child by child
// (the update part in the front's own HBM slot), the triangle is solved by
// one wave (y_j = w_j / l_jj, then w_i -= l_ij y_j for i > j, in column
// order) and the update rows take -L21 y by one thread per row (column order).
__global__ __launch_bounds__(kBigThreads) void k_big_fwd(const InstDev* __restrict__ insts,
                                                       const FrontDesc* __restrict__ fds, int skip_done) {
    __shared__ double Ls[kBigMaxCols * (kBigMaxCols + 1)];
    __shared__ double w[kBigMaxCols], dv[kBigMaxCols];
    const FrontDesc& F = fds[blockIdx.x];
    if (front_idle(F, skip_done)) return;
    const InstDev& I = insts[F.inst];
    const PatDev& T = I.P;
    const int c = F.c, r = F.r, u = r - c, ld = r | 1, ldl = c | 1;
    const double* const P = F.L;
    double* const V = F.V;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63;
    for (int q = tid; q < c * c; q += nt) {
        const int j = q / c, i = q - j * c;
        Ls[j * ldl + i] = P[(int64_t)j * ld + i];
    }
    if (tid < c) {
        w[tid] = F.y[tid];
        dv[tid] = F.dinv[tid];
    }
    for (int a = tid; a < u; a += nt) V[a] = 0.0;
    __syncthreads();
    for (int k = 0; k < F.nch; k++) {
        const int ch = T.ch_list[F.ch0 + k];
        const int cc = T.sn_ncol[ch];
        const int uc = T.sn_nrow[ch] - cc;
        const double* const Vc = I.V + T.sn_vofs[ch];
        const int* const rl = T.rel + T.sn_rowofs[ch] + cc;
        for (int a = tid; a < uc; a += nt) {
            const int ra = rl[a];
            const double v = Vc[a];
            if (ra < c) w[ra] += v;
            else V[ra - c] += v;
        }
        __syncthreads();
    }
    if (tid < 64) {
        double wi = lane < c ? w[lane] : 0.0;
        for (int j = 0; j < c; j++) {
            const double yj = readlane_d(wi, j) * dv[j];
            if (lane > j && lane < c) wi = fma(-Ls[j * ldl + lane], yj, wi);
        }
        if (lane < c) w[lane] = wi * dv[lane];
    }
    __syncthreads();
    for (int a = tid; a < u; a += nt) {
        double acc = V[a];
        for (int j = 0; j < c; j++) acc = fma(-P[(int64_t)j * ld + c + a], w[j], acc);
        V[a] = acc;
    }
    if (tid < c) F.y[tid] = w[tid];
}

// Backward sweep of large fronts: t = y1 - L21^T z by one wave per column
// (lanes over rows, a fixed butterfly), then the triangle by one wave.
__global__ __launch_bounds__(kBigThreads) void k_big_bwd(const FrontDesc* __restrict__ fds, int skip_done) {
    __shared__ double Ls[kBigMaxCols * (kBigMaxCols + 1)];
    __shared__ double t[kBigMaxCols], dv[kBigMaxCols];
    const FrontDesc& F = fds[blockIdx.x];
    if (front_idle(F, skip_done)) return;
    const int c = F.c, r = F.r, u = r - c, ld = r | 1, ldl = c | 1;
    const double* const P = F.L;
    const double* const yb = F.y - F.col0;  // the instance's work vector
    const int* const rw = F.rw;
    const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
    for (int q = tid; q < c * c; q += nt) {
        const int j = q / c, i = q - j * c;
        Ls[j * ldl + i] = P[(int64_t)j * ld + i];
    }
    if (tid < c) dv[tid] = F.dinv[tid];
    for (int j = wave; j < c; j += nwave) {
        const double* const col = P + (int64_t)j * ld + c;
        double s = 0.0;
        for (int a = lane; a < u; a += 64) s = fma(col[a], yb[rw[a]], s);
        for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
        if (lane == 0) t[j] = F.y[j] - s;
    }
    __syncthreads();
    if (tid < 64) {
        double x0 = lane < c ? t[lane] : 0.0, x1 = 0.0;
        tri_bwd_wave(Ls, ldl, c, dv, x0, x1, lane);
        if (lane < c) F.y[lane] = x0;
    }
}

__global__ __launch_bounds__(kSolveThreads) void k_fwd(const InstDev* __restrict__ insts,
                                                      const FrontDesc* __restrict__ fds, int skip_done) {
    extern __shared__ __align__(16) double sh[];
    const FrontDesc& F = fds[blockIdx.x];
    if (front_idle(F, skip_done)) return;
    fwd_front(insts[F.inst], F, sh);
}

__global__ __launch_bounds__(kSolveThreads) void k_bwd(const FrontDesc* __restrict__ fds, int skip_done) {
    extern __shared__ __align__(16) double sh[];
    const FrontDesc& F = fds[blockIdx.x];
    if (front_idle(F, skip_done)) return;
    bwd_front(F, sh);
}

// the same for launches of small panels (at most kSweepHalfLds of LDS):
// sixteen staged loads per thread (110 registers instead of 184), so the
// registers allow four workgroups per compute unit where the LDS does
// (measured on the 256-instance batch: backward sweeps 1.13 -> 1.05 ms; eight
// loads per thread: 1.14 ms)
__global__ __launch_bounds__(kSolveThreads) void k_bwd_small(const FrontDesc* __restrict__ fds, int skip_done) {
    extern __shared__ __align__(16) double sh[];
    const FrontDesc& F = fds[blockIdx.x];
    if (front_idle(F, skip_done)) return;
    bwd_front<KKT_BWD_SMALL_PU>(F, sh);
}

// Both sweeps in one launch: tickets 0..N-1 are the forward sweep in
// topological order, tickets N..2N-1 the backward sweep in reverse order. A
// front's backward step waits for its parent's (a root waits for its own
// forward step, the last of its tree).
__global__ __launch_bounds__(kSolveThreads) void k_sweeps_queue(const InstDev* __restrict__ insts,
                                                               const FrontDesc* __restrict__ fds, DepLists D,
                                                               int skip_done) {
    extern __shared__ __align__(16) double sh[];
    __shared__ int slot;
    const int N = D.nitems;
    for (;;) {
        const int t = take_ticket(D.ticket, &slot);
        if (t >= 2 * N) break;
        const bool fwd = t < N;
        const int k = fwd ? t : 2 * N - 1 - t;
        const int par = __builtin_amdgcn_readfirstlane(D.parent[k]);
        if (sched_wave()) {
            if (fwd) wait_at_least(D.cnt + k, __builtin_amdgcn_readfirstlane(D.nchild[k]), D.err);
            else if (par >= 0) wait_at_least(D.bdone + par, 1, D.err);
            else wait_at_least(D.fdone + k, 1, D.err);
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const FrontDesc& F = fds[k];
        const int idle = __builtin_amdgcn_readfirstlane((int)front_idle(F, skip_done));
        if (!idle) {
            if (fwd) fwd_front(insts[F.inst], F, sh);
            else bwd_front(F, sh);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (sched_wave()) {
            if (!fwd) publish_add(D.bdone + k);
            else if (par >= 0) publish_add(D.cnt + par);
            else publish_add(D.fdone + k);
        }
    }
}

// ---------------------------------------------------------------------------
// permutations between original and pivot order (row blocks of 256)
// ---------------------------------------------------------------------------
// y[k] = src[perm[k]] with src = b (PIN_B) or r (PIN_R)
__global__ __launch_bounds__(256) void k_perm_in(const InstDev* __restrict__ insts, Calls C,
                                                 const WorkItem* __restrict__ items, int mode) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (mode == PIN_R && I.rs->done) return;
    const int k = it.id + threadIdx.x;
    if (k >= I.P.n) return;
    const double* src = mode == PIN_B ? C.b + I.n_off : I.r;
    I.y[k] = src[I.P.perm[k]];
}

// POUT_X: x[perm[k]] = y[k]; POUT_X_UPDATE: xprev = x, x += y[iperm];
// POUT_DX: dx[perm[k]] = y[k]
__global__ __launch_bounds__(256) void k_perm_out(const InstDev* __restrict__ insts, Calls C,
                                                  const WorkItem* __restrict__ items, int mode) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (mode == POUT_X_UPDATE && I.rs->done) return;
    const int k = it.id + threadIdx.x;
    if (k >= I.P.n) return;
    const int i = I.P.perm[k];
    const double v = I.y[k];
    if (mode == POUT_X) {
        C.x[I.n_off + i] = v;
    } else if (mode == POUT_X_UPDATE) {
        double* x = C.x + I.n_off;
        const double xo = x[i];
        I.xprev[i] = xo;
        x[i] = xo + v;
    } else {
        C.dx[I.n_off + i] = v;
    }
}

// ---------------------------------------------------------------------------
// residual r = b - K x and backward-error reductions (original numbering)
// ---------------------------------------------------------------------------
__global__ void k_refine_reset(const InstDev* __restrict__ insts, int ninst, double tol, int maxit) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ninst) return;
    RefineState* S = insts[q].rs;
    S->omega = S->omega_prev = INFINITY;
    S->eta = S->eta_prev = INFINITY;
    S->relres = S->relres_prev = INFINITY;
    S->tol = tol;
    S->maxit = maxit;
    S->it = 0;
    S->done = 0;
    S->revert = 0;
}

// block maxima of five values, written to this block's slot (no atomics:
// the decision kernel takes the maximum over the slots)
__device__ inline void block_max5(double v0, double v1, double v2, double v3, double v4, double* out) {
    __shared__ double red[5][256];
    const int tid = threadIdx.x;
    red[0][tid] = v0; red[1][tid] = v1; red[2][tid] = v2; red[3][tid] = v3; red[4][tid] = v4;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int q = 0; q < 5; q++) red[q][tid] = fmax(red[q][tid], red[q][tid + h]);
        __syncthreads();
    }
    if (tid < 5) out[tid] = red[tid][0];
}

// 16 lanes per row (coalesced reads of the row's entries); each 16-lane
// group takes NR rows, 16 apart, and issues the loads of all of them before
// the first wait: many short independent rows in flight hide the dependent
// loads (row bounds, then columns, then x), and each block's reduction is
// shared by 16 NR rows.
__global__ __launch_bounds__(256) void k_residual(const InstDev* __restrict__ insts, Calls C,
                                                  const WorkItem* __restrict__ items) {
    constexpr int NR = 16 / kResidualSplit;  // rows per 16-lane group
    const WorkItem it = items[blockIdx.x / kResidualSplit];
    const InstDev& I = insts[it.inst];
    if (I.rs->done) return;  // uniform per block
    const double* __restrict__ x = C.x + I.n_off;
    const double* __restrict__ b = C.b + I.n_off;
    const int n = I.P.n;
    const int g = threadIdx.x >> 4, l = threadIdx.x & 15;
    double ra = 0.0, om = 0.0, rs = 0.0, xa = 0.0, ba = 0.0;
    const int row0 = it.id + (blockIdx.x % kResidualSplit) * 16 * NR + g;
    // rows past the end load the last row (valid addresses) and are discarded
    int64_t pb[NR], pe[NR];
#pragma unroll
    for (int j = 0; j < NR; j++) {
        const int i = min(row0 + 16 * j, n - 1);
        pb[j] = I.P.sp_ptr[i];
        pe[j] = I.P.sp_ptr[i + 1];
    }
    // the first three entries of each lane and row in one round (values,
    // columns, then the gathered x), clamped so no load is predicated; the
    // terms are then summed in the lane's order, as in the loop for the rest
    constexpr int RU = 3;
    double kv[NR][RU], xv[NR][RU];
    int cl[NR][RU];
#pragma unroll
    for (int j = 0; j < NR; j++)
#pragma unroll
        for (int q = 0; q < RU; q++) {
            const int64_t p = min(pb[j] + l + 16 * q, pe[j] - 1);
            kv[j][q] = I.kcsr[p];
            cl[j][q] = I.P.sp_col[p];
        }
#pragma unroll
    for (int j = 0; j < NR; j++)
#pragma unroll
        for (int q = 0; q < RU; q++) xv[j][q] = x[cl[j][q]];
#pragma unroll
    for (int j = 0; j < NR; j++) {
        double sum = 0.0, den = 0.0, ks = 0.0;
#pragma unroll
        for (int q = 0; q < RU; q++) {
            if (pb[j] + l + 16 * q < pe[j]) {
                const double t = kv[j][q] * xv[j][q];
                sum += t;
                den += fabs(t);
                ks += fabs(kv[j][q]);
            }
        }
        for (int64_t p = pb[j] + l + 16 * RU; p < pe[j]; p += 16) {
            const double kp = I.kcsr[p];
            const double t = kp * x[I.P.sp_col[p]];
            sum += t;
            den += fabs(t);
            ks += fabs(kp);
        }
#pragma unroll
        for (int o = 8; o > 0; o >>= 1) {
            sum += __shfl_xor(sum, o, 16);
            den += __shfl_xor(den, o, 16);
            ks += __shfl_xor(ks, o, 16);
        }
        const int i = row0 + 16 * j;
        if (l == 0 && i < n) {
            const double bi = b[i];
            const double ri = bi - sum;
            I.r[i] = ri;
            const double ai = fabs(ri);
            den += fabs(bi);
            ra = fmax(ra, ai);
            om = fmax(om, den > 0.0 ? ai / den : (ai > 0.0 ? INFINITY : 0.0));
            rs = fmax(rs, ks);
            xa = fmax(xa, fabs(x[i]));
            ba = fmax(ba, fabs(bi));
        }
    }
    const int slot = (it.id >> 8) * kResidualSplit + (int)(blockIdx.x % kResidualSplit);
    block_max5(ra, om, rs, xa, ba, I.rpart + 5 * slot);
}

// One workgroup per instance: the maxima over the residual blocks' slots
// (order-independent), then eta / omega and the refinement stop rule
// (omega <= tol, maxit corrections, or omega not halving; in the last case
// the previous iterate wins if omega grew).
__global__ __launch_bounds__(256) void k_refine_decide(const InstDev* __restrict__ insts, int* ndone) {
    const InstDev& I = insts[blockIdx.x];
    RefineState* S = I.rs;
    if (S->done) return;  // uniform per block
    const int nslots = ((I.P.n + 255) >> 8) * kResidualSplit;
    double m[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    // eight slots per thread in flight at once; a maximum is unchanged by
    // repeats, so indices past the end repeat the last slot
    constexpr int UNR = 8;
    const double* __restrict__ rp = I.rpart;
    for (int t0 = threadIdx.x; t0 < nslots; t0 += blockDim.x * UNR) {
        double v[UNR][5];
#pragma unroll
        for (int k = 0; k < UNR; k++) {
            const int t = min(t0 + k * (int)blockDim.x, nslots - 1);
#pragma unroll
            for (int q = 0; q < 5; q++) v[k][q] = rp[5 * t + q];
        }
#pragma unroll
        for (int k = 0; k < UNR; k++)
#pragma unroll
            for (int q = 0; q < 5; q++) m[q] = fmax(m[q], v[k][q]);
    }
    __shared__ double red[5][256];
    for (int q = 0; q < 5; q++) red[q][threadIdx.x] = m[q];
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int q = 0; q < 5; q++) red[q][threadIdx.x] = fmax(red[q][threadIdx.x], red[q][threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double rmax = red[0][0], om = red[1][0], kn = red[2][0], xm = red[3][0], bm = red[4][0];
    const double den = kn * xm + bm;
    S->eta_prev = S->eta;
    S->relres_prev = S->relres;
    S->omega_prev = S->omega;
    S->eta = den > 0.0 ? rmax / den : 0.0;
    S->relres = bm > 0.0 ? rmax / bm : rmax;
    S->omega = om;
    bool stop = om <= S->tol || S->it >= S->maxit;
    if (S->it > 0 && om > 0.5 * S->omega_prev) {
        stop = true;
        if (om > S->omega_prev) S->revert = 1;
    }
    if (stop) {
        S->done = 1;
        atomicAdd(ndone, 1);
    } else {
        S->it += 1;
    }
}

__global__ __launch_bounds__(256) void k_refine_revert(const InstDev* __restrict__ insts, Calls C,
                                                       const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (!I.rs->revert) return;
    const int i = it.id + threadIdx.x;
    if (i >= I.P.n) return;
    C.x[I.n_off + i] = I.xprev[i];
}

__global__ __launch_bounds__(256) void k_matvec(const InstDev* __restrict__ insts, const double* __restrict__ x,
                                                double* __restrict__ y, const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int i = it.id + threadIdx.x;
    if (i >= I.P.n) return;
    double sum = 0.0;
    for (int64_t p = I.P.sp_ptr[i]; p < I.P.sp_ptr[i + 1]; p++) sum += I.kcsr[p] * x[I.P.sp_col[p]];
    y[i] = sum;
}

// ---------------------------------------------------------------------------
// Schur-complement CG (eq. (schurcomp)). The m-vectors (c, r, p, q, dy) are in
// the numbering of J's rows; the n-vectors handed to the sweeps are in pivot
// order, so J^T v is written straight into the sweep vector (pivot position k
// holds column perm[k]) and J t reads the sweep output through j_colp.
//
// Iteration k is three launches around the sweep pair:
//   k_cg_dir  the stop tests of the iterate dy_k, then p_k = r_k + beta_k p_{k-1}
//             (row owners) and y = J^T p_k for the sweeps, each entry of p_k
//             formed on the fly by the same fma as its stored value;
//   k_cg_q    q = J K_gamma^{-1} J^T p_k and the partial sums of p.q;
//   k_cg_upd  alpha = r.r / p.q, dy += alpha p, r -= alpha q, and the partial
//             sums of r.r and maxima of |dy|.
// Each scalar (r.r, p.q, the norms) is reduced from the previous launch's
// per-workgroup partial sums by every workgroup that needs it, in one fixed
// order, so every workgroup takes the same decision without any
// synchronisation inside a launch; workgroup 0 of the instance records it.
// Every kernel returns at once when the instance's CG has stopped, so the
// iterations can be queued without reading decisions back.
//
// Reduction slots of one instance (4 per 256-row block):
//   N-region red[4 b + k], n-side blocks:  0 max row sum of |A|, 1 max |f|
//                                          (k_cg_fg); 2 max |r|, 3 max
//                                          |J^T r| (k_cg_dir, eta test);
//                                          0, 1 again for the final residual
//   M-region red[mslot0 + 4 b + k]:        0 r.r, 1 max |dy| (k_cg_c with
//                                          dy = 0, then k_cg_upd); 2 max |g|,
//                                          3 max row sum of |J| (k_cg_c)
//   Q-region red[qslot0 + 2 b + k]:        p.q (k_cg_q, stride 1); the final
//                                          residual's max |g - J dx|, |dy|
// ---------------------------------------------------------------------------
// deterministic block sum of v (every thread gets the sum)
__device__ inline double block_sum(double v) {
    __shared__ double sred[256];
    const int tid = threadIdx.x;
    sred[tid] = v;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (tid < h) sred[tid] += sred[tid + h];
        __syncthreads();
    }
    const double t = sred[0];
    __syncthreads();
    return t;
}

__device__ inline double block_max(double v) {
    __shared__ double smax[256];
    const int tid = threadIdx.x;
    smax[tid] = v;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (tid < h) smax[tid] = fmax(smax[tid], smax[tid + h]);
        __syncthreads();
    }
    const double t = smax[0];
    __syncthreads();
    return t;
}

__device__ __forceinline__ int cg_nb(int len) { return (len + 255) >> 8; }
__device__ __forceinline__ int cg_mslot0(const InstDev& I) { return 4 * cg_nb(I.P.n); }
__device__ __forceinline__ int cg_qslot0(const InstDev& I) { return 4 * (cg_nb(I.P.n) + cg_nb(I.P.m)); }

// fixed-order sum / maximum over slot k of nb blocks (stride `stride`)
__device__ inline double slots_sum(const double* red, int nb, int stride, int k) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v += red[stride * b + k];
    return block_sum(v);
}
__device__ inline double slots_max(const double* red, int nb, int stride, int k) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v = fmax(v, red[stride * b + k]);
    return block_max(v);
}
// maximum of the negated slots (a minimum, for slots that may all be positive)
__device__ inline double slots_max_neg(const double* red, int nb, int stride, int k) {
    double v = -INFINITY;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) v = fmax(v, -red[stride * b + k]);
    return block_max(v);
}

// sum_q a[q] * v[idx[q]] over q in [q0, q1), four loads in flight per round,
// terms added in q order
template <class F>
__device__ __forceinline__ double gather_dot(int q0, int q1, const double* __restrict__ a,
                                             const int* __restrict__ idx, F&& v) {
    double s = 0.0;
    for (int q = q0; q < q1; q += 4) {
        int id[4];
        double av[4], xv[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int qc = min(q + u, q1 - 1);
            id[u] = idx[qc];
            av[u] = a[qc];
        }
#pragma unroll
        for (int u = 0; u < 4; u++) xv[u] = v(id[u]);
#pragma unroll
        for (int u = 0; u < 4; u++)
            if (q + u < q1) s += av[u] * xv[u];
    }
    return s;
}

// f_gamma = f + gamma J^T g in pivot order (sweep vector and a copy for dx),
// the n-side norms (per row i of the saddle matrix, sum_j |K0_ij| +
// sum_r |J_ri|; |f_i|), and the CG record's set-up (workgroup 0).
__global__ __launch_bounds__(256) void k_cg_fg(const InstDev* __restrict__ insts, Calls C,
                                               const WorkItem* __restrict__ items, double tol, int maxit,
                                               double eta_tol) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (it.id == 0 && threadIdx.x == 0) {
        CgState* G = I.cg;
        G->tol = tol;
        G->maxit = maxit;
        G->eta_tol = eta_tol;
        G->it = 0;
        G->status = 0;
        G->done = 0;
        G->eta_stop = 0;
        G->eta = 0.0;
    }
    const int k = it.id + threadIdx.x;
    double arow = 0.0, fa = 0.0;
    if (k < I.P.n) {
        const int j = I.P.perm[k];
        const double* __restrict__ g = C.g + I.m_off;
        double s = 0.0, csum = 0.0;
        for (int q = I.P.jtp_ptr[k]; q < I.P.jtp_ptr[k + 1]; q++) {
            const int row = I.P.jtp_row[q];
            if (C.eqm && !C.eqm[row]) continue;  // general HyKKT: equality rows only
            const double a = I.jtv[q];
            s += a * g[row];
            csum += fabs(a);
        }
        const double fj = C.f[I.n_off + j];
        const double v = fj + C.gamma * s;
        I.fg[k] = v;
        I.y[k] = v;
        double ka = 0.0;
        for (int64_t p = I.P.sp_ptr[j]; p < I.P.sp_ptr[j + 1]; p++) ka += fabs(I.k0csr[p]);
        arow = ka + csum;
        fa = fabs(fj);
    }
    arow = block_max(arow);
    fa = block_max(fa);
    if (threadIdx.x == 0) {
        double* s = I.red + 4 * (it.id >> 8);
        s[0] = arow;
        s[1] = fa;
    }
}

// After the sweeps: c = J K_gamma^{-1} f_gamma - g; r = c; p_old = 0; dy = 0;
// partial sums of c.c and the m-side norms.
__global__ __launch_bounds__(256) void k_cg_c(const InstDev* __restrict__ insts, Calls C,
                                              const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int i = it.id + threadIdx.x;
    double cc = 0.0, ga = 0.0, jrow = 0.0;
    if (i < I.P.m) {
        const int p0 = I.P.j_ptr[i], p1 = I.P.j_ptr[i + 1];
        const double* __restrict__ y = I.y;
        // general HyKKT: the inequality rows are not in the Schur system; their
        // entries of c, r, p and dy stay 0
        const bool eq = !C.eqm || C.eqm[i];
        const double s = gather_dot(p0, p1, I.jraw, I.P.j_colp, [&](int c) { return y[c]; });
        if (eq)
            for (int p = p0; p < p1; p++) jrow += fabs(I.jraw[p]);
        const double gi = eq ? C.g[I.m_off + i] : 0.0;
        const double ci = eq ? s - gi : 0.0;
        I.cvec[i] = ci;
        I.rvec[i] = ci;
        I.pvec2[i] = 0.0;
        C.dy[I.m_off + i] = 0.0;
        cc = ci * ci;
        ga = fabs(gi);
    }
    cc = block_sum(cc);
    ga = block_max(ga);
    jrow = block_max(jrow);
    if (threadIdx.x == 0) {
        double* s = I.red + cg_mslot0(I) + 4 * (it.id >> 8);
        s[0] = cc;
        s[1] = 0.0;  // ||dy_0||_inf
        s[2] = ga;
        s[3] = jrow;
    }
}

// Iteration k: stop tests of dy_k (r_k . r_k from the M-region partials),
// p_k = r_k + beta_k p_{k-1} for the instance's rows (row i by thread i of the
// n-side blocks; the Schur system needs m <= n) and y[k'] = (J^T p_k)_{perm[k']}.
// Stops: ||r_k||_2 <= tol ||c||_2 (converged) or k == maxit (NOT_CONVERGED).
// With eta_tol > 0 the maxima of |r_k| and |J^T r_k| go to the N-region for
// k_cg_eta_test.
__global__ __launch_bounds__(256) void k_cg_dir(const InstDev* __restrict__ insts,
                                                const WorkItem* __restrict__ items, int k, int* ndone) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    CgState* G = I.cg;
    if (G->done) return;  // uniform per block
    const int nbm = cg_nb(I.P.m);
    const double rr = slots_sum(I.red + cg_mslot0(I), nbm, 4, 0);
    const double cnorm = k == 0 ? sqrt(rr) : G->cnorm;
    const bool conv = k == 0 ? rr == 0.0 : sqrt(rr) <= G->tol * cnorm;
    const bool lead = it.id == 0 && threadIdx.x == 0;
    if (conv || k >= G->maxit) {
        if (lead) {
            G->rr_new = rr;
            if (k == 0) G->cnorm = cnorm;
            G->it = k;
            G->status = conv ? 0 : 6;  // not converged after maxit iterations
            G->done = 1;
            atomicAdd(ndone, 1);
        }
        return;
    }
    const double beta = k == 0 ? 0.0 : rr / G->rrs[(k - 1) & 1];
    if (lead) {
        G->rrs[k & 1] = rr;
        G->rr_new = rr;
        G->it = k;
        if (k == 0) G->cnorm = cnorm;
    }
    const int parity = k & 1;
    double* __restrict__ pn = parity ? I.pvec2 : I.pvec;
    const double* __restrict__ po = parity ? I.pvec : I.pvec2;
    const double* __restrict__ r = I.rvec;
    const int kk = it.id + threadIdx.x;
    double ra = 0.0, ja = 0.0;
    if (kk < I.P.m) {
        pn[kk] = fma(beta, po[kk], r[kk]);
        ra = fabs(r[kk]);
    }
    const bool eta_test = G->eta_tol > 0.0;
    if (kk < I.P.n) {
        const int q0 = I.P.jtp_ptr[kk], q1 = I.P.jtp_ptr[kk + 1];
        double s = 0.0, t = 0.0;
        for (int q = q0; q < q1; q += 4) {
            int row[4];
            double a[4], rv[4], pv[4];
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const int qc = min(q + u, q1 - 1);
                row[u] = I.P.jtp_row[qc];
                a[u] = I.jtv[qc];
            }
#pragma unroll
            for (int u = 0; u < 4; u++) {
                rv[u] = r[row[u]];
                pv[u] = po[row[u]];
            }
#pragma unroll
            for (int u = 0; u < 4; u++)
                if (q + u < q1) {
                    s += a[u] * fma(beta, pv[u], rv[u]);
                    t += a[u] * rv[u];
                }
        }
        I.y[kk] = s;
        ja = fabs(t);
    }
    if (!eta_test) return;  // uniform per launch
    ra = block_max(ra);
    ja = block_max(ja);
    if (threadIdx.x == 0) {
        double* sl = I.red + 4 * (it.id >> 8);
        sl[2] = ra;
        sl[3] = ja;
    }
}

// eta_tol > 0, one workgroup per instance, between k_cg_dir and the sweeps:
// for dx = K_gamma^{-1}(f_gamma - J^T dy) the saddle system's residual is
// (gamma J^T r, r), so
//   max(gamma ||J^T r||_inf, ||r||_inf) / (||A||_inf ||dy||_inf + ||(f, g)||_inf)
// bounds its normwise backward error from above (the denominator leaves out
// ||dx||); the CG stops at dy_k when the bound is <= eta_tol.
__global__ __launch_bounds__(256) void k_cg_eta_test(const InstDev* __restrict__ insts, Calls C, int k,
                                                     int* ndone) {
    const InstDev& I = insts[blockIdx.x];
    CgState* G = I.cg;
    if (G->done || !(G->eta_tol > 0.0)) return;  // uniform
    const int nbn = cg_nb(I.P.n), nbm = cg_nb(I.P.m);
    const double* Nr = I.red;
    const double* Mr = I.red + cg_mslot0(I);
    const double norm_a = fmax(slots_max(Nr, nbn, 4, 0), slots_max(Mr, nbm, 4, 3));
    const double norm_rhs = fmax(slots_max(Nr, nbn, 4, 1), slots_max(Mr, nbm, 4, 2));
    const double rmax = slots_max(Nr, nbn, 4, 2);
    const double jrmax = slots_max(Nr, nbn, 4, 3);
    const double dymax = slots_max(Mr, nbm, 4, 1);
    if (threadIdx.x == 0) {
        G->norm_a = norm_a;
        G->norm_rhs = norm_rhs;
        G->rmax = rmax;
        G->dymax = dymax;
        if (fmax(C.gamma * jrmax, rmax) <= G->eta_tol * (norm_a * dymax + norm_rhs)) {
            G->it = k;
            G->done = 1;
            G->eta_stop = 1;
            atomicAdd(ndone, 1);
        }
    }
}

// q = J t with t = K_gamma^{-1} J^T p_k (the sweep output, pivot order) and the
// partial sums of p_k . q
__global__ __launch_bounds__(256) void k_cg_q(const InstDev* __restrict__ insts, Calls C,
                                              const WorkItem* __restrict__ items, int k) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (I.cg->done) return;  // uniform per block
    const double* __restrict__ pn = (k & 1) ? I.pvec2 : I.pvec;
    const int i = it.id + threadIdx.x;
    double v = 0.0;
    if (i < I.P.m) {
        const double* __restrict__ y = I.y;
        double s = gather_dot(I.P.j_ptr[i], I.P.j_ptr[i + 1], I.jraw, I.P.j_colp, [&](int c) { return y[c]; });
        if (C.eqm && !C.eqm[i]) s = 0.0;  // general HyKKT: equality rows only
        I.qvec[i] = s;
        v = pn[i] * s;
    }
    v = block_sum(v);
    if (threadIdx.x == 0) I.red[cg_qslot0(I) + (it.id >> 8)] = v;
}

// alpha = r_k . r_k / p_k . q (p_k^T S p_k <= 0: BREAKDOWN), dy += alpha p_k,
// r -= alpha q, and the partial sums of r.r and maxima of |dy|.
__global__ __launch_bounds__(256) void k_cg_upd(const InstDev* __restrict__ insts, Calls C,
                                                const WorkItem* __restrict__ items, int k, int* ndone) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    CgState* G = I.cg;
    if (G->done) return;  // uniform per block
    const int nbm = cg_nb(I.P.m);
    const double pq = slots_sum(I.red + cg_qslot0(I), nbm, 1, 0);
    if (!(pq > 0.0)) {
        if (it.id == 0 && threadIdx.x == 0) {
            G->pq = pq;
            G->it = k;
            G->status = 7;  // breakdown
            G->done = 1;
            atomicAdd(ndone, 1);
        }
        return;
    }
    const double a = G->rrs[k & 1] / pq;
    const double* __restrict__ pn = (k & 1) ? I.pvec2 : I.pvec;
    const int i = it.id + threadIdx.x;
    double rr = 0.0, da = 0.0;
    if (i < I.P.m) {
        double* dy = C.dy + I.m_off;
        const double d = fma(a, pn[i], dy[i]);
        dy[i] = d;
        const double ri = fma(-a, I.qvec[i], I.rvec[i]);
        I.rvec[i] = ri;
        rr = ri * ri;
        da = fabs(d);
    }
    rr = block_sum(rr);
    da = block_max(da);
    if (threadIdx.x == 0) {
        double* s = I.red + cg_mslot0(I) + 4 * (it.id >> 8);
        s[0] = rr;
        s[1] = da;
    }
}

// right-hand side of the last solve: y[k] = f_gamma[k] - (J^T dy)_{perm[k]}
__global__ __launch_bounds__(256) void k_cg_dxrhs(const InstDev* __restrict__ insts, Calls C,
                                                  const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int k = it.id + threadIdx.x;
    if (k >= I.P.n) return;
    const double* __restrict__ dy = C.dy + I.m_off;
    const double s = gather_dot(I.P.jtp_ptr[k], I.P.jtp_ptr[k + 1], I.jtv, I.P.jtp_row, [&](int r) { return dy[r]; });
    I.y[k] = I.fg[k] - s;
}

// Saddle-system residual of (dx, dy): rows of the primal block,
// f - K0 dx - J^T dy (original numbering), with the maxima of |res| and |dx|.
__global__ __launch_bounds__(256) void k_cg_res_n(const InstDev* __restrict__ insts, Calls C,
                                                  const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int j = it.id + threadIdx.x;
    double ra = 0.0, xa = 0.0;
    if (j < I.P.n) {
        const double* __restrict__ dx = C.dx + I.n_off;
        const double* __restrict__ dy = C.dy + I.m_off;
        double s = 0.0;
        for (int64_t p = I.P.sp_ptr[j]; p < I.P.sp_ptr[j + 1]; p++) s += I.k0csr[p] * dx[I.P.sp_col[p]];
        for (int q = I.P.jt_ptr[j]; q < I.P.jt_ptr[j + 1]; q++) s += I.jraw[I.P.jt_e[q]] * dy[I.P.jt_row[q]];
        ra = fabs(C.f[I.n_off + j] - s);
        xa = fabs(dx[j]);
    }
    ra = block_max(ra);
    xa = block_max(xa);
    if (threadIdx.x == 0) {
        double* s = I.red + 4 * (it.id >> 8);
        s[0] = ra;
        s[1] = xa;
    }
}

// constraint rows, g - J dx, with |dy|
__global__ __launch_bounds__(256) void k_cg_res_m(const InstDev* __restrict__ insts, Calls C,
                                                  const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int i = it.id + threadIdx.x;
    double ra = 0.0, ya = 0.0;
    if (i < I.P.m && (!C.eqm || C.eqm[i])) {  // general HyKKT: equality rows only
        const double* __restrict__ dx = C.dx + I.n_off;
        double s = 0.0;
        for (int p = I.P.j_ptr[i]; p < I.P.j_ptr[i + 1]; p++) s += I.jraw[p] * dx[I.P.j_col[p]];
        ra = fabs(C.g[I.m_off + i] - s);
        ya = fabs(C.dy[I.m_off + i]);
    }
    ra = block_max(ra);
    ya = block_max(ya);
    if (threadIdx.x == 0) {
        double* s = I.red + cg_qslot0(I) + 2 * (it.id >> 8);
        s[0] = ra;
        s[1] = ya;
    }
}

// one workgroup per instance: eta = ||res||_inf / (||A||_inf ||(dx, dy)||_inf
// + ||(f, g)||_inf) from the residual kernels' maxima and the norms kept in
// the record by k_cg_norms
__global__ __launch_bounds__(256) void k_cg_eta(const InstDev* __restrict__ insts) {
    const InstDev& I = insts[blockIdx.x];
    CgState* G = I.cg;
    const int nbn = cg_nb(I.P.n), nbm = cg_nb(I.P.m);
    const double* Nr = I.red;
    const double* Qr = I.red + cg_qslot0(I);
    const double r1 = slots_max(Nr, nbn, 4, 0), x1 = slots_max(Nr, nbn, 4, 1);
    const double r2 = slots_max(Qr, nbm, 2, 0), y2 = slots_max(Qr, nbm, 2, 1);
    if (threadIdx.x == 0) {
        const double den = G->norm_a * fmax(x1, y2) + G->norm_rhs;
        const double res = fmax(r1, r2);
        G->eta = den > 0.0 ? res / den : (res > 0.0 ? INFINITY : 0.0);
    }
}

// one workgroup per instance, before the iterations: ||A||_inf (the n-side
// part) and ||f||_inf from k_cg_fg's partials, kept in the record (the eta
// test and the final residual overwrite the N-region)
__global__ __launch_bounds__(256) void k_cg_norms(const InstDev* __restrict__ insts) {
    const InstDev& I = insts[blockIdx.x];
    CgState* G = I.cg;
    const int nbn = cg_nb(I.P.n), nbm = cg_nb(I.P.m);
    const double* Mr = I.red + cg_mslot0(I);
    const double an = fmax(slots_max(I.red, nbn, 4, 0), slots_max(Mr, nbm, 4, 3));
    const double fm = fmax(slots_max(I.red, nbn, 4, 1), slots_max(Mr, nbm, 4, 2));
    if (threadIdx.x == 0) {
        G->norm_a = an;
        G->norm_rhs = fm;
    }
}

// ---------------------------------------------------------------------------
// Augmented system of eq. (kkt:augmented) with no equality rows (the Lifted-KKT
// form, H = J, D_s = Sigma_s), regularised on the Hessian block as the
// condensed matrix K = W + Sigma_x + delta I + J^T Sigma_s J is:
//   [[K0, 0, J^T], [0, Sigma_s, I], [J, I, 0]] [dx; ds; dz] = -[r1; r2; r4],
// K0 = W + Sigma_x + delta I. Condensation (eq. (kkt:condensed)) gives
// K dx = -(r1 + J^T (Sigma_s r4 - r2)), and the slack and multiplier steps
// follow as ds = -r4 - J dx, dz = -r2 - Sigma_s ds. The refinement on the
// full system (section "Hybrid linear solver") takes the residual e of the
// augmented system and solves for the correction the same way.
// Slots: N-region 8 per block (k_aug_res_n), M-region 8 per block after it.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int aug_mslot0(const InstDev& I) { return 8 * cg_nb(I.P.n); }

// b_j = p1_j - sum_q J_qj (p2_q - Sigma_s,q p4_q) with p = -r (mode 0) or
// p = e (mode 1); pivot-ordered threads, b in original numbering
__global__ __launch_bounds__(256) void k_aug_rhs(const InstDev* __restrict__ insts, AugCall A,
                                                 const WorkItem* __restrict__ items, int mode) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (mode == 1 && I.aug->done) return;  // uniform per block
    const int k = it.id + threadIdx.x;
    if (k >= I.P.n) return;
    const int n = I.P.n, m = I.P.m;
    const int j = I.P.perm[k];
    const double* __restrict__ p2 = mode ? I.aug_e + n : A.r2;
    const double* __restrict__ p4 = mode ? I.aug_e + n + m : A.r4;
    const double sgn = mode ? 1.0 : -1.0;
    double s = 0.0;
    for (int q = I.P.jtp_ptr[k]; q < I.P.jtp_ptr[k + 1]; q++) {
        const int row = I.P.jtp_row[q];
        s += I.jtv[q] * (sgn * p2[row] - I.ssv[row] * (sgn * p4[row]));
    }
    const double p1 = mode ? I.aug_e[j] : -A.r1[j];
    I.aug_b[j] = p1 - s;
}

// mode 0: ds = p4 - J dx, dz = p2 - Sigma_s ds with p = -r.
// mode 1: t = K^{-1} b is in aug_t; the iterate moves to aug_prev and
// dx += t, ds += e4 - J t, dz += e2 - Sigma_s (e4 - J t).
__global__ __launch_bounds__(256) void k_aug_recover_m(const InstDev* __restrict__ insts, AugCall A,
                                                       const WorkItem* __restrict__ items, int mode) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (mode == 1 && I.aug->done) return;
    const int i = it.id + threadIdx.x;
    if (i >= I.P.m) return;
    const int n = I.P.n, m = I.P.m;
    const double* __restrict__ v = mode ? I.aug_t : A.dx;
    double s = 0.0;
    for (int p = I.P.j_ptr[i]; p < I.P.j_ptr[i + 1]; p++) s += I.jraw[p] * v[I.P.j_col[p]];
    const double p2 = mode ? I.aug_e[n + i] : -A.r2[i];
    const double p4 = mode ? I.aug_e[n + m + i] : -A.r4[i];
    const double ds = p4 - s;
    const double dz = p2 - I.ssv[i] * ds;
    if (mode == 0) {
        A.ds[i] = ds;
        A.dz[i] = dz;
    } else {
        const double so = A.ds[i], zo = A.dz[i];
        I.aug_prev[n + i] = so;
        I.aug_prev[n + m + i] = zo;
        A.ds[i] = so + ds;
        A.dz[i] = zo + dz;
    }
}

__global__ __launch_bounds__(256) void k_aug_update_x(const InstDev* __restrict__ insts, AugCall A,
                                                      const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (I.aug->done) return;
    const int j = it.id + threadIdx.x;
    if (j >= I.P.n) return;
    const double xo = A.dx[j];
    I.aug_prev[j] = xo;
    A.dx[j] = xo + I.aug_t[j];
}

__global__ void k_aug_reset(const InstDev* __restrict__ insts, int ninst, double tol, int maxit) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ninst) return;
    AugState* S = insts[q].aug;
    S->eta = S->eta_prev = S->omega = S->omega_prev = INFINITY;
    S->tol = tol;
    S->maxit = maxit;
    S->it = 0;
    S->done = 0;
    S->revert = 0;
}

// ratio for the componentwise backward error (0/0 taken as 0)
__device__ __forceinline__ double aug_ratio(double r, double den) {
    return den > 0.0 ? r / den : (r > 0.0 ? INFINITY : 0.0);
}

// primal rows: e1 = -r1 - K0 dx - J^T dz, with |K0||dx| + |J|^T|dz| + |r1|,
// the row sums of |A| and the maxima of |dx| and |r1|
__global__ __launch_bounds__(256) void k_aug_res_n(const InstDev* __restrict__ insts, AugCall A,
                                                   const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (I.aug->done) return;
    const int j = it.id + threadIdx.x;
    double ea = 0.0, om = 0.0, ar = 0.0, xa = 0.0, ba = 0.0;
    if (j < I.P.n) {
        double s = 0.0, den = 0.0, rs = 0.0;
        for (int64_t p = I.P.sp_ptr[j]; p < I.P.sp_ptr[j + 1]; p++) {
            const double a = I.k0csr[p], t = a * A.dx[I.P.sp_col[p]];
            s += t;
            den += fabs(t);
            rs += fabs(a);
        }
        for (int q = I.P.jt_ptr[j]; q < I.P.jt_ptr[j + 1]; q++) {
            const double a = I.jraw[I.P.jt_e[q]], t = a * A.dz[I.P.jt_row[q]];
            s += t;
            den += fabs(t);
            rs += fabs(a);
        }
        const double p1 = -A.r1[j];
        const double e1 = p1 - s;
        I.aug_e[j] = e1;
        ea = fabs(e1);
        om = aug_ratio(ea, den + fabs(p1));
        ar = rs;
        xa = fabs(A.dx[j]);
        ba = fabs(p1);
    }
    ea = block_max(ea);
    om = block_max(om);
    ar = block_max(ar);
    xa = block_max(xa);
    ba = block_max(ba);
    if (threadIdx.x == 0) {
        double* sl = I.red + 8 * (it.id >> 8);
        sl[0] = ea;
        sl[1] = om;
        sl[2] = ar;
        sl[3] = xa;
        sl[4] = ba;
    }
}

// slack rows e2 = -r2 - Sigma_s ds - dz and constraint rows e4 = -r4 - J dx - ds
__global__ __launch_bounds__(256) void k_aug_res_m(const InstDev* __restrict__ insts, AugCall A,
                                                   const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (I.aug->done) return;
    const int i = it.id + threadIdx.x;
    const int n = I.P.n, m = I.P.m;
    double ea = 0.0, om = 0.0, ar = 0.0, xa = 0.0, ba = 0.0;
    if (i < m) {
        const double sg = I.ssv[i], ds = A.ds[i], dz = A.dz[i];
        const double p2 = -A.r2[i], p4 = -A.r4[i];
        const double t2 = sg * ds;
        const double e2 = p2 - t2 - dz;
        double s = 0.0, den4 = 0.0, rs4 = 0.0;
        for (int p = I.P.j_ptr[i]; p < I.P.j_ptr[i + 1]; p++) {
            const double a = I.jraw[p], t = a * A.dx[I.P.j_col[p]];
            s += t;
            den4 += fabs(t);
            rs4 += fabs(a);
        }
        const double e4 = p4 - s - ds;
        I.aug_e[n + i] = e2;
        I.aug_e[n + m + i] = e4;
        ea = fmax(fabs(e2), fabs(e4));
        om = fmax(aug_ratio(fabs(e2), fabs(t2) + fabs(dz) + fabs(p2)),
                  aug_ratio(fabs(e4), den4 + fabs(ds) + fabs(p4)));
        ar = fmax(sg + 1.0, rs4 + 1.0);
        xa = fmax(fabs(ds), fabs(dz));
        ba = fmax(fabs(p2), fabs(p4));
    }
    ea = block_max(ea);
    om = block_max(om);
    ar = block_max(ar);
    xa = block_max(xa);
    ba = block_max(ba);
    if (threadIdx.x == 0) {
        double* sl = I.red + aug_mslot0(I) + 8 * (it.id >> 8);
        sl[0] = ea;
        sl[1] = om;
        sl[2] = ar;
        sl[3] = xa;
        sl[4] = ba;
    }
}

// one workgroup per instance: eta and omega of the augmented system, and the
// stop rule of the refinement (omega <= tol, maxit corrections, or omega not
// halving; the previous iterate wins if omega grew)
__global__ __launch_bounds__(256) void k_aug_decide(const InstDev* __restrict__ insts) {
    const InstDev& I = insts[blockIdx.x];
    AugState* S = I.aug;
    if (S->done) return;
    const int nbn = cg_nb(I.P.n), nbm = cg_nb(I.P.m);
    const double* Nr = I.red;
    const double* Mr = I.red + aug_mslot0(I);
    double v[5];
    for (int k = 0; k < 5; k++) v[k] = fmax(slots_max(Nr, nbn, 8, k), slots_max(Mr, nbm, 8, k));
    if (threadIdx.x != 0) return;
    const double den = v[2] * v[3] + v[4];
    S->eta_prev = S->eta;
    S->omega_prev = S->omega;
    S->eta = den > 0.0 ? v[0] / den : (v[0] > 0.0 ? INFINITY : 0.0);
    S->omega = v[1];
    bool stop = S->omega <= S->tol || S->it >= S->maxit;
    if (S->it > 0 && S->omega > 0.5 * S->omega_prev) {
        stop = true;
        if (S->omega > S->omega_prev) S->revert = 1;
    }
    if (stop) S->done = 1;
    else S->it += 1;
}

__global__ __launch_bounds__(256) void k_aug_revert_n(const InstDev* __restrict__ insts, AugCall A,
                                                      const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (!I.aug->revert) return;
    const int j = it.id + threadIdx.x;
    if (j < I.P.n) A.dx[j] = I.aug_prev[j];
}

__global__ __launch_bounds__(256) void k_aug_revert_m(const InstDev* __restrict__ insts, AugCall A,
                                                      const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (!I.aug->revert) return;
    const int i = it.id + threadIdx.x;
    if (i >= I.P.m) return;
    A.ds[i] = I.aug_prev[I.P.n + i];
    A.dz[i] = I.aug_prev[I.P.n + I.P.m + i];
}

// ---------------------------------------------------------------------------
// Interior-point loop (section "INTERIOR-POINT METHOD": the smoothed KKT
// system eq. (smoothkkt), Newton steps eq. (newtonstep) through the
// augmented system, fraction-to-boundary steps) on the convex QP
//   min 1/2 x^T W x + c^T x  s.t.  J x + s = u, s >= 0,
// multipliers z, D_s = S^{-1} Z. Per iteration (vectors in original numbering):
//   r1 = W x + c + J^T z, r4 = J x + s - u, gap = s^T z / m,
//   err = max(||r1|| / (1 + ||c||), ||r4|| / (1 + ||u||), gap) (inf-norms),
//   mu = sigma gap, r2 = z - mu / s, tau = max(tau_min, 1 - mu),
//   the Newton step (dx, ds, dz) from the augmented system, the largest
//   alpha_p, alpha_d <= 1 keeping s and z above (1 - tau) of their values.
// W x comes from the factor's kept K0 = W + delta I (Sigma_x = 0).
// Slots: red[4 b + k] for the n-side blocks, red[4 nbn + 4 b + k] for m-side.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int ipm_m0(const InstDev& I) { return 4 * cg_nb(I.P.n); }

// n-side: max |c|; m-side: max |u|; then the record (one workgroup per
// instance reduces in the second kernel)
__global__ __launch_bounds__(256) void k_ipm_norm_n(const InstDev* __restrict__ insts, IpmCall P,
                                                    const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int j = it.id + threadIdx.x;
    const double v = block_max(j < I.P.n ? fabs(P.c[j]) : 0.0);
    if (threadIdx.x == 0) P.red[4 * (it.id >> 8)] = v;
}
__global__ __launch_bounds__(256) void k_ipm_norm_m(const InstDev* __restrict__ insts, IpmCall P,
                                                    const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int i = it.id + threadIdx.x;
    const double v = block_max(i < I.P.m ? fabs(P.u[i]) : 0.0);
    if (threadIdx.x == 0) P.red[ipm_m0(I) + 4 * (it.id >> 8)] = v;
}
__global__ __launch_bounds__(256) void k_ipm_init(const InstDev* __restrict__ insts, IpmCall P, double tol, int maxit,
                                                  double sigma, double tau_min) {
    const InstDev& I = insts[0];
    const double cm = slots_max(P.red, cg_nb(I.P.n), 4, 0);
    const double um = slots_max(P.red + ipm_m0(I), cg_nb(I.P.m), 4, 0);
    if (threadIdx.x != 0) return;
    IpmState* S = P.st;
    S->cn = 1.0 + cm;
    S->un = 1.0 + um;
    S->tol = tol;
    S->maxit = maxit;
    S->sigma = sigma;
    S->tau_min = tau_min;
    S->it = 0;
    S->done = 0;
    S->status = 0;
    S->mu = S->gap = S->err = S->r1max = S->r4max = S->ap = S->ad = S->delta = 0.0;
}

// D_s = z / s, the slack weights of the refactor
__global__ __launch_bounds__(256) void k_ipm_dsw(const InstDev* __restrict__ insts, IpmCall P,
                                                 const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int i = it.id + threadIdx.x;
    if (i < I.P.m) P.dsw[i] = P.z[i] / P.s[i];
}

// r1 = (K0 - delta I) x + c + J^T z
__global__ __launch_bounds__(256) void k_ipm_res_n(const InstDev* __restrict__ insts, IpmCall P,
                                                   const WorkItem* __restrict__ items, double delta) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int j = it.id + threadIdx.x;
    double ra = 0.0;
    if (j < I.P.n) {
        double s = 0.0;
        for (int64_t p = I.P.sp_ptr[j]; p < I.P.sp_ptr[j + 1]; p++) s += I.k0csr[p] * P.x[I.P.sp_col[p]];
        s -= delta * P.x[j];
        double t = 0.0;
        for (int q = I.P.jt_ptr[j]; q < I.P.jt_ptr[j + 1]; q++) t += P.jv[I.P.jt_e[q]] * P.z[I.P.jt_row[q]];
        const double r = s + P.c[j] + t;
        P.r1[j] = r;
        ra = fabs(r);
    }
    ra = block_max(ra);
    if (threadIdx.x == 0) P.red[4 * (it.id >> 8)] = ra;
}

// r4 = J x + s - u, partial s^T z
__global__ __launch_bounds__(256) void k_ipm_res_m(const InstDev* __restrict__ insts, IpmCall P,
                                                   const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int i = it.id + threadIdx.x;
    double ra = 0.0, sz = 0.0;
    if (i < I.P.m) {
        double t = 0.0;
        for (int p = I.P.j_ptr[i]; p < I.P.j_ptr[i + 1]; p++) t += P.jv[p] * P.x[I.P.j_col[p]];
        const double r = t + P.s[i] - P.u[i];
        P.r4[i] = r;
        ra = fabs(r);
        sz = P.s[i] * P.z[i];
    }
    ra = block_max(ra);
    sz = block_sum(sz);
    if (threadIdx.x == 0) {
        double* sl = P.red + ipm_m0(I) + 4 * (it.id >> 8);
        sl[0] = ra;
        sl[1] = sz;
    }
}

// the stop test and mu, tau of this iteration
__global__ __launch_bounds__(256) void k_ipm_decide(const InstDev* __restrict__ insts, IpmCall P, double delta) {
    const InstDev& I = insts[0];
    const int nbn = cg_nb(I.P.n), nbm = cg_nb(I.P.m);
    const double r1 = slots_max(P.red, nbn, 4, 0);
    const double r4 = slots_max(P.red + ipm_m0(I), nbm, 4, 0);
    const double sz = slots_sum(P.red + ipm_m0(I), nbm, 4, 1);
    if (threadIdx.x != 0) return;
    IpmState* S = P.st;
    S->r1max = r1;
    S->r4max = r4;
    S->delta = fmax(S->delta, delta);
    S->gap = I.P.m > 0 ? sz / I.P.m : 0.0;
    S->err = fmax(fmax(r1 / S->cn, r4 / S->un), S->gap);
    if (S->err <= S->tol) {
        S->done = 1;
    } else if (S->it >= S->maxit) {
        S->done = 1;
        S->status = 6;  // not converged
    } else {
        S->mu = S->sigma * S->gap;
        S->tau = fmax(S->tau_min, 1.0 - S->mu);
    }
}

// r2 = z - mu / s
__global__ __launch_bounds__(256) void k_ipm_r2(const InstDev* __restrict__ insts, IpmCall P,
                                                const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int i = it.id + threadIdx.x;
    if (i < I.P.m) P.r2[i] = P.z[i] - P.st->mu / P.s[i];
}

// fraction to the boundary: per block the smallest -tau v / dv over dv < 0
// (2 when no entry decreases), for s and for z
__global__ __launch_bounds__(256) void k_ipm_alpha(const InstDev* __restrict__ insts, IpmCall P,
                                                   const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int i = it.id + threadIdx.x;
    const double tau = P.st->tau;
    double as = 2.0, az = 2.0;
    if (i < I.P.m) {
        if (P.ds[i] < 0.0) as = -tau * P.s[i] / P.ds[i];
        if (P.dz[i] < 0.0) az = -tau * P.z[i] / P.dz[i];
    }
    as = -block_max(-as);
    az = -block_max(-az);
    if (threadIdx.x == 0) {
        double* sl = P.red + ipm_m0(I) + 4 * (it.id >> 8);
        sl[2] = as;
        sl[3] = az;
    }
}

__global__ __launch_bounds__(256) void k_ipm_alpha_fin(const InstDev* __restrict__ insts, IpmCall P) {
    const InstDev& I = insts[0];
    const int nbm = cg_nb(I.P.m);
    const double as = -slots_max_neg(P.red + ipm_m0(I), nbm, 4, 2);
    const double az = -slots_max_neg(P.red + ipm_m0(I), nbm, 4, 3);
    if (threadIdx.x != 0) return;
    P.st->ap = fmin(1.0, as);
    P.st->ad = fmin(1.0, az);
    P.st->it += 1;
}

// x += alpha_p dx (n-side blocks); s += alpha_p ds, z += alpha_d dz (m-side)
__global__ __launch_bounds__(256) void k_ipm_update_n(const InstDev* __restrict__ insts, IpmCall P,
                                                      const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int j = it.id + threadIdx.x;
    if (j < I.P.n) P.x[j] = fma(P.st->ap, P.dx[j], P.x[j]);
}
__global__ __launch_bounds__(256) void k_ipm_update_m(const InstDev* __restrict__ insts, IpmCall P,
                                                      const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int i = it.id + threadIdx.x;
    if (i < I.P.m) {
        P.s[i] = fma(P.st->ap, P.ds[i], P.s[i]);
        P.z[i] = fma(P.st->ad, P.dz[i], P.z[i]);
    }
}

// ---------------------------------------------------------------------------
// Stage-structured solver: the condensed matrix of a dynamic program is
// block-banded (section "Future Works"); with stage-contiguous variables and
// couplings between consecutive stages only, K is block tridiagonal and is
// factored here by block cyclic reduction: the stages at odd positions of the
// active chain are eliminated together (one workgroup each), the rest form
// the next, half as long, chain. This is a Cholesky factorization of K in
// the cyclic-reduction order, with dense blocks: per eliminated stage k with
// active neighbours l and r, the front [D_k; K(l,k); K(r,k)] is factored,
//   L_k = chol(D_k),  L(l,k) = K(l,k) L_k^{-T},  L(r,k) = K(r,k) L_k^{-T},
// and it leaves to the next level the updates L(l,k) L(l,k)^T (to D_l),
// L(r,k) L(r,k)^T (to D_r) and the fill K(r,l) = -L(r,k) L(l,k)^T. Every
// launch also runs one workgroup per stage that stays in the chain, which
// applies the updates of the previous level to its D (so each stage takes at
// most two updates, from the level just before). K itself comes from the
// general assembly (kcsr), so its entries are the same bits as the
// supernodal path's.
// ---------------------------------------------------------------------------
// 1/d: the hardware reciprocal estimate refined by two steps of Newton's
// iteration r <- r + r (1 - d r), each of which doubles the correct bits
__device__ __forceinline__ double recip_f64(double d) {
    double r = __builtin_amdgcn_rcp(d);
    r = fma(r, fma(-d, r, 1.0), r);
    r = fma(r, fma(-d, r, 1.0), r);
    return r;
}

// the value of v in lane `lane` (uniform), through the scalar unit
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__global__ void k_fill_f64(double* __restrict__ p, double v, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_cr_scatter(const InstDev* __restrict__ insts, CrArrays A,
                                                    const CrScatter* __restrict__ items, int64_t nitems) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nitems) return;
    const CrScatter it = items[t];
    const double v = insts[it.inst].kcsr[it.pos];
    if (it.dst >= 0) A.D[it.dst] = v;
    else A.C[-it.dst - 1] = v;
}

// One workgroup per task of one level (NB: stage widths <= 16 NB). A task
// eliminates its stage or applies the previous level's updates to a stage
// that stays. Thread (ti, tc) = (tid % 16, tid / 16)
// holds the front entries of rows ti + 16 a and columns tc + 16 b in
// registers. The front's rows: [0, s_k) stage k, then l, then r; columns
// [0, s_k). Right-looking Cholesky, one barrier per column: the owners of
// column j publish it (unscaled) to LDS, every thread reads the pivot and
// updates its entries right of j, the owners scale their part of column j.
// Then the update block Q = P P^T of the rows below (P = [L(l,k); L(r,k)])
// from LDS, register-tiled the same way (lower half only).
template <int NB>
__global__ __launch_bounds__(256) void k_cr_factor(const InstDev* __restrict__ insts, CrArrays AR, int task0) {
    constexpr int RA = 3 * NB;  // row slots of the front (<= 48 NB rows)
    constexpr int QA = 2 * NB;  // row / column slots of the update block (<= 32 NB)
    constexpr int CB = 48 * NB;
    extern __shared__ __align__(16) double sh[];
    const CrTask T = AR.tasks[task0 + blockIdx.x];
    const int tid = threadIdx.x, ti = tid & 15, tc = tid >> 4;
    const int sk = T.sk;
    const int64_t u0 = T.npull > 0 ? AR.pulls[T.pull0].u : -1;
    const int64_t u1 = T.npull > 1 ? AR.pulls[T.pull0 + 1].u : -1;
    const double* Dk = (T.from_work ? AR.L : AR.D) + T.d;
    double* Lk = AR.L + T.d;
    if (!T.elim) {
        // a stage that stays: D_k -= the previous level's updates (lower part)
        double v[NB][NB], w0[NB][NB], w1[NB][NB];
#pragma unroll
        for (int a = 0; a < NB; a++)
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const int i = ti + 16 * a, c = tc + 16 * b;
                const bool ok = i < sk && c < sk && i >= c;
                const int64_t idx = (int64_t)c * sk + i;
                v[a][b] = ok ? Dk[idx] : 0.0;
                w0[a][b] = ok && u0 >= 0 ? AR.U[u0 + idx] : 0.0;
                w1[a][b] = ok && u1 >= 0 ? AR.U[u1 + idx] : 0.0;
            }
#pragma unroll
        for (int a = 0; a < NB; a++)
#pragma unroll
            for (int b = 0; b < NB; b++) {
                const int i = ti + 16 * a, c = tc + 16 * b;
                if (i < sk && c < sk && i >= c) Lk[(int64_t)c * sk + i] = (v[a][b] - w0[a][b]) - w1[a][b];
            }
        return;
    }
    const InstDev& I = insts[T.inst];
    const int sl = T.sl, sr = T.sr, np = sl + sr, mr = sk + np;
    // all loads issued before any is used: the rows below the stage (one load
    // each, K(l,k) = K(k,l)^T and K(r,k)), then D_k and its updates
    double m[RA][NB];
#pragma unroll
    for (int a = 0; a < RA; a++)
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int i = ti + 16 * a, c = tc + 16 * b;
            const bool below = c < sk && i >= sk && i < mr;
            const int64_t at = i < sk + sl ? T.kl + (int64_t)(i - sk) * sk + c : T.kr + (int64_t)c * sr + (i - sk - sl);
            m[a][b] = below ? AR.C[at] : 0.0;
        }
    double dv[NB][NB], w0[NB][NB], w1[NB][NB];
#pragma unroll
    for (int a = 0; a < NB; a++)
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int i = ti + 16 * a, c = tc + 16 * b;
            const bool ok = i < sk && c < sk && i >= c;
            const int64_t idx = (int64_t)c * sk + i;
            dv[a][b] = ok ? Dk[idx] : 0.0;
            w0[a][b] = ok && u0 >= 0 ? AR.U[u0 + idx] : 0.0;
            w1[a][b] = ok && u1 >= 0 ? AR.U[u1 + idx] : 0.0;
        }
#pragma unroll
    for (int a = 0; a < NB; a++)
#pragma unroll
        for (int b = 0; b < NB; b++)
            if (ti + 16 * a < sk) m[a][b] = (dv[a][b] - w0[a][b]) - w1[a][b];
    // Right-looking Cholesky in unscaled form: step j subtracts M(i,j)
    // M(c,j) / M(j,j) from M(i,c), and the columns are scaled by the square
    // roots of their pivots (kept in LDS) in one pass at the end, which keeps
    // the square roots off the per-column chain. The update of step j
    // touches entry (i, c) with i >= c > j. With i = ti + 16 a and c = tc +
    // 16 b that is: slot pairs a > b always (given c > j), a == b when ti >=
    // tc, a < b never; so the pairs are fixed at compile time and the rest is
    // masked by selects (no branches in the loop).
    double* colbuf = sh;            // two column buffers of CB rows
    double* piv = sh + 2 * CB;      // the pivots (after substitution of failed ones)
    bool rowok[RA];
#pragma unroll
    for (int a = 0; a < RA; a++) rowok[a] = ti + 16 * a < mr;
    const bool diag_ok = ti >= tc;
    int par = 0;
#pragma unroll
    for (int jb = 0; jb < NB; jb++) {
        for (int jj = 0; jj < 16; jj++) {
            const int j = 16 * jb + jj;
            if (j >= sk) break;
            double* cb = colbuf + par * CB;
            if (tc == jj) {
#pragma unroll
                for (int a = jb; a < RA; a++) cb[ti + 16 * a] = m[a][jb];
            }
            __syncthreads();
            // every read of the column first, then the pivot
            double d = cb[j];
            double cv[RA], cc[NB];
#pragma unroll
            for (int a = jb; a < RA; a++) cv[a] = cb[ti + 16 * a];
#pragma unroll
            for (int b = jb; b < NB; b++) cc[b] = cb[tc + 16 * b];
            if (!(d > 0.0) || !isfinite(d)) {
                if (tid == 0) {
                    atomicMin(&I.status[1], T.var0 + j);
                    atomicMax(&I.status[0], KKT_ST_NOT_SPD);
                }
                d = 1.0;
            }
            if (tid == 0) piv[j] = d;
            const double inv_d = recip_f64(d);
#pragma unroll
            for (int a = jb; a < RA; a++) cv[a] = rowok[a] ? cv[a] : 0.0;
#pragma unroll
            for (int b = jb; b < NB; b++) {
                const int c = tc + 16 * b;
                const double lc = (c > j && c < sk) ? cc[b] * inv_d : 0.0;
                m[b][b] = fma(-(diag_ok ? cv[b] : 0.0), lc, m[b][b]);
#pragma unroll
                for (int a = b + 1; a < RA; a++) m[a][b] = fma(-cv[a], lc, m[a][b]);
            }
            par ^= 1;
        }
    }
    __syncthreads();
    // scale: L(i,c) = M(i,c) / sqrt(d_c) below the diagonal, sqrt(d_c) on it
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int c = tc + 16 * b;
        const double dc = c < sk ? piv[c] : 1.0;
        const double ls = sqrt(dc), inv_ls = recip_f64(ls);
#pragma unroll
        for (int a = 0; a < RA; a++) {
            const int i = ti + 16 * a;
            m[a][b] = i == c ? ls : m[a][b] * inv_ls;
        }
    }
    // L_k to L (lower), L(l,k) and L(r,k) to P, and P = the rows below into LDS
    double* Pb = sh + 2 * CB + 16 * NB;  // s_k columns of np rows
#pragma unroll
    for (int a = 0; a < RA; a++)
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int i = ti + 16 * a, c = tc + 16 * b;
            if (c >= sk || i >= mr) continue;
            if (i < sk) {
                if (i >= c) Lk[(int64_t)c * sk + i] = m[a][b];
            } else {
                Pb[c * np + (i - sk)] = m[a][b];
                if (i < sk + sl) AR.P[T.pl + (int64_t)c * sl + (i - sk)] = m[a][b];
                else AR.P[T.pr + (int64_t)c * sr + (i - sk - sl)] = m[a][b];
            }
        }
    if (np == 0) return;  // uniform: the last stage of its instance
    __syncthreads();
    // Q = P P^T, lower half: UL = Q(l, l), UR = Q(r, r), fill F = -Q(r, l)
    double q[QA][QA];
#pragma unroll
    for (int a = 0; a < QA; a++)
#pragma unroll
        for (int b = 0; b <= a; b++) q[a][b] = 0.0;
    // Pb holds s_k np entries plus 32 NB of padding, so these reads stay in
    // bounds for every slot; slots past np are masked to zero. The reads of
    // column c + 1 are issued before the products of column c.
    bool pok[QA], qok[QA];
#pragma unroll
    for (int a = 0; a < QA; a++) {
        pok[a] = ti + 16 * a < np;
        qok[a] = tc + 16 * a < np;
    }
    double pr[QA], pc[QA];
#pragma unroll
    for (int a = 0; a < QA; a++) {
        pr[a] = Pb[ti + 16 * a];
        pc[a] = Pb[tc + 16 * a];
    }
    for (int c = 0; c < sk; c++) {
        const int cn = c + 1 < sk ? c + 1 : c;
        double prn[QA], pcn[QA];
#pragma unroll
        for (int a = 0; a < QA; a++) {
            prn[a] = Pb[cn * np + ti + 16 * a];
            pcn[a] = Pb[cn * np + tc + 16 * a];
        }
#pragma unroll
        for (int a = 0; a < QA; a++) {
            pr[a] = pok[a] ? pr[a] : 0.0;
            pc[a] = qok[a] ? pc[a] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < QA; a++)
#pragma unroll
            for (int b = 0; b <= a; b++) q[a][b] = fma(pr[a], pc[b], q[a][b]);
#pragma unroll
        for (int a = 0; a < QA; a++) {
            pr[a] = prn[a];
            pc[a] = pcn[a];
        }
    }
#pragma unroll
    for (int a = 0; a < QA; a++)
#pragma unroll
        for (int b = 0; b <= a; b++) {
            const int p = ti + 16 * a, p2 = tc + 16 * b;
            if (p >= np || p2 >= np || p < p2) continue;
            if (p < sl) AR.U[T.ul + (int64_t)p2 * sl + p] = q[a][b];
            else if (p2 >= sl) AR.U[T.ur + (int64_t)(p2 - sl) * sr + (p - sl)] = q[a][b];
            else AR.C[T.f + (int64_t)p2 * sr + (p - sl)] = -q[a][b];
        }
}

// Stages L_k (s_k x s_k, column-major) into LDS: every thread issues its
// loads before the first store.
__device__ inline void cr_stage_block(double* __restrict__ dst, const double* __restrict__ src, int n) {
    constexpr int PER = (kCrMaxStage * kCrMaxStage + 255) / 256;
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int q = threadIdx.x + 256 * u;
        v[u] = q < n ? src[q] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < PER; u++) {
        const int q = threadIdx.x + 256 * u;
        if (q < n) dst[q] = v[u];
    }
}

// y (s_k rows) -= sum over columns c = g, g + 4, ... of P(:, c) x_c, P
// column-major with s_k rows: this thread's part for rows r and r + 64
__device__ inline void cr_matvec_part(const double* __restrict__ P, int rows, int cols,
                                      const double* __restrict__ x, int r, int g, double& s0, double& s1) {
    constexpr int U = kCrMaxStage / 4;
    double xv[U], p0[U], p1[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int c = g + 4 * u;
        xv[u] = c < cols ? x[c] : 0.0;
        p0[u] = c < cols && r < rows ? P[(int64_t)c * rows + r] : 0.0;
        p1[u] = c < cols && r + 64 < rows ? P[(int64_t)c * rows + r + 64] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
        s0 = fma(p0[u], xv[u], s0);
        s1 = fma(p1[u], xv[u], s1);
    }
}

// this thread's part of (P^T x)(r), (P^T x)(r + 64) over rows a = g, g + 4,
// ... of P (column-major, prow rows)
__device__ inline void cr_matvec_t_part(const double* __restrict__ P, int prow, int cols,
                                        const double* __restrict__ x, int r, int g, double& s0, double& s1) {
    constexpr int U = kCrMaxStage / 4;
    double xv[U], p0[U], p1[U];
#pragma unroll
    for (int u = 0; u < U; u++) {
        const int a = g + 4 * u;
        xv[u] = a < prow ? x[a] : 0.0;
        p0[u] = a < prow && r < cols ? P[(int64_t)r * prow + a] : 0.0;
        p1[u] = a < prow && r + 64 < cols ? P[(int64_t)(r + 64) * prow + a] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
        s0 = fma(p0[u], xv[u], s0);
        s1 = fma(p1[u], xv[u], s1);
    }
}

// Forward solve L y = b, per level: a task eliminating its stage takes t_k -
// the previous level's contributions, then y_k = L_k^{-1} t_k by
// substitution in wave 0 (lane i holds rows i and i + 64, the pivot value is
// broadcast by a lane shuffle, the pivots' reciprocals come from LDS); a
// task of a stage that stays only subtracts the contributions. On
// level 0 t_k starts from b (mode 0) or the refinement residual (mode 1,
// stopped instances skipped); later levels from t.
__global__ __launch_bounds__(256) void k_cr_fwd(const InstDev* __restrict__ insts, CrArrays AR, int task0,
                                                Calls C, int mode, int level0) {
    __shared__ double Ls[kCrMaxStage * kCrMaxStage];
    __shared__ double red[4][128];
    __shared__ double inv[kCrMaxStage];
    const CrTask T = AR.tasks[task0 + blockIdx.x];
    const InstDev& I = insts[T.inst];
    if (mode == 1 && I.rs->done) return;  // uniform per block
    const bool elim = T.elim != 0;
    const int tid = threadIdx.x, r = tid & 63, g = tid >> 6, sk = T.sk;
    double s0 = 0.0, s1 = 0.0;
    for (int u = 0; u < T.npull; u++) {
        const CrPull Pu = AR.pulls[T.pull0 + u];
        cr_matvec_part(AR.P + Pu.p, sk, Pu.si, AR.t + Pu.vi, r, g, s0, s1);
    }
    red[g][r] = s0;
    red[g][r + 64] = s1;
    if (elim) {
        cr_stage_block(Ls, AR.L + T.d, sk * sk);
        if (tid < sk) inv[tid] = 1.0 / AR.L[T.d + (int64_t)tid * sk + tid];
    }
    __syncthreads();
    if (tid >= 64) return;
    const double* src = level0 ? (mode == 0 ? C.b + T.v0 : I.r + T.var0) : AR.t + T.v0;
    const int i0 = r, i1 = r + 64;
    double t0 = i0 < sk ? src[i0] - ((red[0][i0] + red[1][i0]) + (red[2][i0] + red[3][i0])) : 0.0;
    double t1 = i1 < sk ? src[i1] - ((red[0][i1] + red[1][i1]) + (red[2][i1] + red[3][i1])) : 0.0;
    if (elim) {
        // column j + 1 of L is read while step j runs (rows clamped into the
        // block; their values are not used past s_k)
        const int c0 = min(i0, sk - 1), c1 = min(i1, sk - 1);
        double l0 = Ls[c0], l1 = Ls[c1], iv = inv[0];
        for (int j = 0; j < sk; j++) {
            const int jn = j + 1 < sk ? j + 1 : j;
            const double l0n = Ls[jn * sk + c0], l1n = Ls[jn * sk + c1], ivn = inv[jn];
            const double tj = j < 64 ? readlane_f64(t0, j) : readlane_f64(t1, j - 64);
            const double yj = tj * iv;
            t0 = i0 == j ? yj : (i0 > j ? fma(-l0, yj, t0) : t0);
            t1 = i1 == j ? yj : (i1 > j ? fma(-l1, yj, t1) : t1);
            l0 = l0n;
            l1 = l1n;
            iv = ivn;
        }
    }
    if (i0 < sk) AR.t[T.v0 + i0] = t0;
    if (i1 < sk) AR.t[T.v0 + i1] = t1;
}

// Backward solve L^T x = y, levels in reverse, eliminated stages only: x_k =
// L_k^{-T} (y_k - L(l,k)^T x_l - L(r,k)^T x_r), the neighbours being
// eliminated later (their x already in t). x_k goes to t and to the output:
// mode 0 x = x_k; mode 1 xprev = x, x += x_k.
__global__ __launch_bounds__(256) void k_cr_bwd(const InstDev* __restrict__ insts, CrArrays AR, int task0, Calls C,
                                                int mode) {
    __shared__ double Ls[kCrMaxStage * kCrMaxStage];
    __shared__ double red[4][128];
    __shared__ double inv[kCrMaxStage];
    const CrTask T = AR.tasks[task0 + blockIdx.x];
    const InstDev& I = insts[T.inst];
    if (!T.elim || (mode == 1 && I.rs->done)) return;  // uniform per block
    const int tid = threadIdx.x, r = tid & 63, g = tid >> 6, sk = T.sk;
    double s0 = 0.0, s1 = 0.0;
    if (T.sl > 0) cr_matvec_t_part(AR.P + T.pl, T.sl, sk, AR.t + T.vl, r, g, s0, s1);
    if (T.sr > 0) cr_matvec_t_part(AR.P + T.pr, T.sr, sk, AR.t + T.vr, r, g, s0, s1);
    red[g][r] = s0;
    red[g][r + 64] = s1;
    cr_stage_block(Ls, AR.L + T.d, sk * sk);
    if (tid < sk) inv[tid] = 1.0 / AR.L[T.d + (int64_t)tid * sk + tid];
    __syncthreads();
    if (tid >= 64) return;
    const int i0 = r, i1 = r + 64;
    double t0 = i0 < sk ? AR.t[T.v0 + i0] - ((red[0][i0] + red[1][i0]) + (red[2][i0] + red[3][i0])) : 0.0;
    double t1 = i1 < sk ? AR.t[T.v0 + i1] - ((red[0][i1] + red[1][i1]) + (red[2][i1] + red[3][i1])) : 0.0;
    // row j of L (entries L(j, i), i < j) is read one step ahead
    const int c0 = min(i0, sk - 1), c1 = min(i1, sk - 1);
    double l0 = Ls[c0 * sk + sk - 1], l1 = Ls[c1 * sk + sk - 1], iv = inv[sk - 1];
    for (int j = sk - 1; j >= 0; j--) {
        const int jn = j > 0 ? j - 1 : 0;
        const double l0n = Ls[c0 * sk + jn], l1n = Ls[c1 * sk + jn], ivn = inv[jn];
        const double tj = j < 64 ? readlane_f64(t0, j) : readlane_f64(t1, j - 64);
        const double xj = tj * iv;
        t0 = i0 == j ? xj : (i0 < j ? fma(-l0, xj, t0) : t0);
        t1 = i1 == j ? xj : (i1 < j ? fma(-l1, xj, t1) : t1);
        l0 = l0n;
        l1 = l1n;
        iv = ivn;
    }
    double* x = C.x + T.v0;
    if (i0 < sk) {
        AR.t[T.v0 + i0] = t0;
        if (mode == 0) {
            x[i0] = t0;
        } else {
            const double xo = x[i0];
            I.xprev[T.var0 + i0] = xo;
            x[i0] = xo + t0;
        }
    }
    if (i1 < sk) {
        AR.t[T.v0 + i1] = t1;
        if (mode == 0) {
            x[i1] = t1;
        } else {
            const double xo = x[i1];
            I.xprev[T.var0 + i1] = xo;
            x[i1] = xo + t1;
        }
    }
}

// ---------------------------------------------------------------------------
// workspace redirection (allocation-free solve): copies of a factor's instance
// descriptor and front descriptors whose per-solve vectors point into a
// caller-provided workspace
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_ws_redirect(const InstDev* __restrict__ src_inst,
                                                     const FrontDesc* __restrict__ src_fd, int nf, SolveWs w) {
    const InstDev& S = src_inst[0];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        InstDev D = S;
        D.y = w.y;
        D.V = w.V;
        D.r = w.r;
        D.xprev = w.xprev;
        D.rpart = w.rpart;
        D.rs = w.rs;
        w.inst[0] = D;
    }
    if (t >= nf) return;
    FrontDesc F = src_fd[t];
    F.y = w.y + F.col0;
    F.V = w.V + (F.V - S.V);
    for (int j = 0; j < 2; j++)
        if (j < F.nch) F.cV[j] = w.V + (F.cV[j] - S.V);
    F.done = &w.rs->done;
    w.fd[t] = F;
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
hipError_t set_kernel_attributes() {
    const int lds = kMaxDynLds;
    hipError_t e = hipFuncSetAttribute((const void*)k_factor, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_factor_small, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_factor_queue, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_sweeps_queue, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_cr_factor<1>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_cr_factor<2>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_cr_factor<3>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_cr_factor<4>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_cr_factor<5>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_bwd_small, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_aug_rhs(const InstDev* insts, const AugCall& A, const WorkItem* ncols, int nitems, int mode,
                    hipStream_t st) {
    if (nitems > 0) k_aug_rhs<<<nitems, kBlock, 0, st>>>(insts, A, ncols, mode);
}
void launch_aug_recover(const InstDev* insts, const AugCall& A, const WorkItem* ncols, int nn, const WorkItem* mrows,
                        int nm, int mode, hipStream_t st) {
    if (mode == 1 && nn > 0) k_aug_update_x<<<nn, kBlock, 0, st>>>(insts, A, ncols);
    if (nm > 0) k_aug_recover_m<<<nm, kBlock, 0, st>>>(insts, A, mrows, mode);
}
void launch_aug_reset(const InstDev* insts, int ninst, double tol, int maxit, hipStream_t st) {
    if (ninst > 0) k_aug_reset<<<blocks_for(ninst, 64), 64, 0, st>>>(insts, ninst, tol, maxit);
}
void launch_aug_check(const InstDev* insts, const AugCall& A, const WorkItem* ncols, int nn, const WorkItem* mrows,
                      int nm, int ninst, hipStream_t st) {
    if (nn > 0) k_aug_res_n<<<nn, kBlock, 0, st>>>(insts, A, ncols);
    if (nm > 0) k_aug_res_m<<<nm, kBlock, 0, st>>>(insts, A, mrows);
    if (ninst > 0) k_aug_decide<<<ninst, kBlock, 0, st>>>(insts);
}
void launch_aug_revert(const InstDev* insts, const AugCall& A, const WorkItem* ncols, int nn, const WorkItem* mrows,
                       int nm, hipStream_t st) {
    if (nn > 0) k_aug_revert_n<<<nn, kBlock, 0, st>>>(insts, A, ncols);
    if (nm > 0) k_aug_revert_m<<<nm, kBlock, 0, st>>>(insts, A, mrows);
}
void launch_ipm_start(const InstDev* insts, const IpmCall& P, const WorkItem* ncols, int nn, const WorkItem* mrows,
                      int nm, double tol, int maxit, double sigma, double tau_min, hipStream_t st) {
    if (nn > 0) k_ipm_norm_n<<<nn, kBlock, 0, st>>>(insts, P, ncols);
    if (nm > 0) k_ipm_norm_m<<<nm, kBlock, 0, st>>>(insts, P, mrows);
    k_ipm_init<<<1, kBlock, 0, st>>>(insts, P, tol, maxit, sigma, tau_min);
}
void launch_ipm_dsw(const InstDev* insts, const IpmCall& P, const WorkItem* mrows, int nm, hipStream_t st) {
    if (nm > 0) k_ipm_dsw<<<nm, kBlock, 0, st>>>(insts, P, mrows);
}
void launch_ipm_residuals(const InstDev* insts, const IpmCall& P, const WorkItem* ncols, int nn, const WorkItem* mrows,
                          int nm, double delta, hipStream_t st) {
    if (nn > 0) k_ipm_res_n<<<nn, kBlock, 0, st>>>(insts, P, ncols, delta);
    if (nm > 0) k_ipm_res_m<<<nm, kBlock, 0, st>>>(insts, P, mrows);
    k_ipm_decide<<<1, kBlock, 0, st>>>(insts, P, delta);
}
void launch_ipm_r2(const InstDev* insts, const IpmCall& P, const WorkItem* mrows, int nm, hipStream_t st) {
    if (nm > 0) k_ipm_r2<<<nm, kBlock, 0, st>>>(insts, P, mrows);
}
void launch_ipm_step(const InstDev* insts, const IpmCall& P, const WorkItem* ncols, int nn, const WorkItem* mrows,
                     int nm, hipStream_t st) {
    if (nm > 0) k_ipm_alpha<<<nm, kBlock, 0, st>>>(insts, P, mrows);
    k_ipm_alpha_fin<<<1, kBlock, 0, st>>>(insts, P);
    if (nn > 0) k_ipm_update_n<<<nn, kBlock, 0, st>>>(insts, P, ncols);
    if (nm > 0) k_ipm_update_m<<<nm, kBlock, 0, st>>>(insts, P, mrows);
}
void launch_fill_f64(double* p, double v, int64_t n, hipStream_t st) {
    if (n > 0) k_fill_f64<<<blocks_for(n, kBlock), kBlock, 0, st>>>(p, v, n);
}
void launch_cr_scatter(const InstDev* insts, const CrArrays& A, const CrScatter* items, int64_t nitems,
                       hipStream_t st) {
    if (nitems > 0) k_cr_scatter<<<blocks_for(nitems, kBlock), kBlock, 0, st>>>(insts, A, items, nitems);
}
void launch_cr_factor(const InstDev* insts, const CrArrays& A, int task0, int ntask, int nb, size_t lds,
                      hipStream_t st) {
    if (ntask <= 0) return;
    switch (nb) {
        case 1: k_cr_factor<1><<<ntask, kBlock, lds, st>>>(insts, A, task0); break;
        case 2: k_cr_factor<2><<<ntask, kBlock, lds, st>>>(insts, A, task0); break;
        case 3: k_cr_factor<3><<<ntask, kBlock, lds, st>>>(insts, A, task0); break;
        case 4: k_cr_factor<4><<<ntask, kBlock, lds, st>>>(insts, A, task0); break;
        default: k_cr_factor<5><<<ntask, kBlock, lds, st>>>(insts, A, task0); break;
    }
}
void launch_cr_fwd(const InstDev* insts, const CrArrays& A, int task0, int ntask, const Calls& C, int mode,
                   int level0, hipStream_t st) {
    if (ntask > 0) k_cr_fwd<<<ntask, 256, 0, st>>>(insts, A, task0, C, mode, level0);
}
void launch_cr_bwd(const InstDev* insts, const CrArrays& A, int task0, int ntask, const Calls& C, int mode,
                   hipStream_t st) {
    if (ntask > 0) k_cr_bwd<<<ntask, 256, 0, st>>>(insts, A, task0, C, mode);
}
void launch_ws_redirect(const InstDev* src_inst, const FrontDesc* src_fd, int nf, const SolveWs& w, hipStream_t st) {
    k_ws_redirect<<<blocks_for(nf > 0 ? nf : 1, 256), 256, 0, st>>>(src_inst, src_fd, nf, w);
}
void launch_copy_segments(const CopySeg* segs, int nseg, hipStream_t st) {
    if (nseg > 0) k_copy_segments<<<nseg * kCopyParts, 256, 0, st>>>(segs);
}
void launch_fill_i32(int* p, int v, int64_t n, hipStream_t st) {
    if (n > 0) k_fill_i32<<<blocks_for(n, kBlock), kBlock, 0, st>>>(p, v, n);
}
void launch_status_init(int* status, int ninst, hipStream_t st) {
    if (ninst > 0) k_status_init<<<blocks_for(ninst, kBlock), kBlock, 0, st>>>(status, ninst);
}
void launch_jscale(const InstDev* insts, const Calls& C, const WorkItem* items, int nitems, hipStream_t st) {
    if (nitems > 0) k_jscale<<<nitems, kBlock, 0, st>>>(insts, C, items);
}
void launch_keep_lifted(const InstDev* insts, const Calls& C, const WorkItem* jentries, int nj, const WorkItem* mrows,
                        int nm, hipStream_t st) {
    if (nj > 0) k_keep_lifted<<<nj, kBlock, 0, st>>>(insts, C, jentries, 0);
    if (nm > 0) k_keep_lifted<<<nm, kBlock, 0, st>>>(insts, C, mrows, 1);
}
void launch_jcopy(const InstDev* insts, const Calls& C, const WorkItem* items, int nitems, hipStream_t st) {
    if (nitems > 0) k_jcopy<<<nitems, kBlock, 0, st>>>(insts, C, items);
}
void launch_assemble_heavy(const InstDev* insts, const Calls& C, const WorkItem* items, int nitems, hipStream_t st) {
    if (nitems > 0) k_assemble_heavy<<<(nitems + 15) / 16, kBlock, 0, st>>>(insts, C, items, nitems);
}
void launch_assemble(const InstDev* insts, const Calls& C, const WorkItem* items, int nitems, hipStream_t st) {
    if (nitems > 0) k_assemble<<<nitems, kBlock, 0, st>>>(insts, C, items);
}
void launch_factor(const InstDev* insts, const FrontDesc* fds, int nitems, size_t lds, int fused_update,
                   hipStream_t st) {
    if (nitems > 0) k_factor<<<nitems, kFactorThreads, lds, st>>>(insts, fds, fused_update);
}
void launch_factor_small(const InstDev* insts, const FrontDesc* fds, int nitems, size_t lds, int fused_update,
                         hipStream_t st) {
    if (nitems > 0) k_factor_small<<<nitems, kFactorThreadsSmall, lds, st>>>(insts, fds, fused_update);
}
void launch_big_factor(const InstDev* insts, const FrontDesc* fds, int nitems, int max_cols, int max_rows,
                       hipStream_t st) {
    if (nitems <= 0) return;
    const int nbc = (max_cols + 15) / 16, nbr = (max_rows + 15) / 16;
    k_big_init<<<dim3(nitems, nbc, (max_rows + kBigInitRows - 1) / kBigInitRows), kBigThreads, 0, st>>>(insts, fds);
    for (int kb = 0; kb < nbc; kb++) {
        const int below = max_rows - 16 * kb - 16;
        if (below > 0) k_big_trsm<<<dim3(nitems, (below + kBigThreads - 1) / kBigThreads), kBigThreads, 0, st>>>(fds, kb);
        int ntile = 0;
        for (int jt = kb + 1; jt < nbc; jt++) ntile += nbr - jt;
        const int wpg = kBigThreads / 64;
        k_big_tiles<<<dim3(nitems, std::max(1, (ntile + wpg - 1) / wpg)), kBigThreads, 0, st>>>(insts, fds, kb);
    }
}
void launch_big_fwd(const InstDev* insts, const FrontDesc* fds, int nitems, int skip_done, hipStream_t st) {
    if (nitems > 0) k_big_fwd<<<nitems, kBigThreads, 0, st>>>(insts, fds, skip_done);
}
void launch_big_bwd(const FrontDesc* fds, int nitems, int skip_done, hipStream_t st) {
    if (nitems > 0) k_big_bwd<<<nitems, kBigThreads, 0, st>>>(fds, skip_done);
}
void launch_update(const InstDev* insts, const FrontDesc* fds, const StripItem* items, int nitems, hipStream_t st) {
    if (nitems > 0) k_update<<<nitems, kUpdThreads, 0, st>>>(insts, fds, items);
}
void launch_factor_queue(const InstDev* insts, const FrontDesc* fds, const DepLists& D, int grid, size_t lds,
                         hipStream_t st) {
    if (D.nitems > 0) k_factor_queue<<<grid, kFactorThreads, lds, st>>>(insts, fds, D);
}
void launch_sweeps_queue(const InstDev* insts, const FrontDesc* fds, const DepLists& D, int grid, size_t lds,
                         int skip_done, hipStream_t st) {
    if (D.nitems > 0) k_sweeps_queue<<<grid, kSolveThreads, lds, st>>>(insts, fds, D, skip_done);
}
void launch_fwd(const InstDev* insts, const FrontDesc* fds, int nitems, size_t lds, int skip_done, hipStream_t st) {
    if (nitems > 0) k_fwd<<<nitems, kSolveThreads, lds, st>>>(insts, fds, skip_done);
}
void launch_bwd(const FrontDesc* fds, int nitems, size_t lds, int skip_done, hipStream_t st) {
    if (nitems <= 0) return;
    if (lds <= kSweepHalfLds) k_bwd_small<<<nitems, kSolveThreads, lds, st>>>(fds, skip_done);
    else k_bwd<<<nitems, kSolveThreads, lds, st>>>(fds, skip_done);
}
void launch_perm_in(const InstDev* insts, const Calls& C, const WorkItem* rows, int nitems, int mode, hipStream_t st) {
    if (nitems > 0) k_perm_in<<<nitems, kBlock, 0, st>>>(insts, C, rows, mode);
}
void launch_perm_out(const InstDev* insts, const Calls& C, const WorkItem* rows, int nitems, int mode, hipStream_t st) {
    if (nitems > 0) k_perm_out<<<nitems, kBlock, 0, st>>>(insts, C, rows, mode);
}
void launch_refine_reset(const InstDev* insts, int ninst, double tol, int maxit, hipStream_t st) {
    k_refine_reset<<<blocks_for(ninst, 64), 64, 0, st>>>(insts, ninst, tol, maxit);
}
void launch_residual(const InstDev* insts, const Calls& C, const WorkItem* rows, int nitems, hipStream_t st) {
    if (nitems > 0) k_residual<<<nitems * kResidualSplit, kBlock, 0, st>>>(insts, C, rows);
}
void launch_refine_decide(const InstDev* insts, int ninst, int* ndone, hipStream_t st) {
    if (ninst > 0) k_refine_decide<<<ninst, 256, 0, st>>>(insts, ndone);
}
void launch_refine_revert(const InstDev* insts, const Calls& C, const WorkItem* rows, int nitems, hipStream_t st) {
    if (nitems > 0) k_refine_revert<<<nitems, kBlock, 0, st>>>(insts, C, rows);
}
void launch_matvec(const InstDev* insts, const double* x, double* y, const WorkItem* rows, int nitems, hipStream_t st) {
    if (nitems > 0) k_matvec<<<nitems, kBlock, 0, st>>>(insts, x, y, rows);
}
void launch_cg_fg(const InstDev* insts, const Calls& C, const WorkItem* ncols, int nitems, double tol, int maxit,
                  double eta_tol, hipStream_t st) {
    if (nitems > 0) k_cg_fg<<<nitems, kBlock, 0, st>>>(insts, C, ncols, tol, maxit, eta_tol);
}
void launch_cg_c(const InstDev* insts, const Calls& C, const WorkItem* mrows, int nitems, int ninst, hipStream_t st) {
    if (nitems > 0) k_cg_c<<<nitems, kBlock, 0, st>>>(insts, C, mrows);
    if (ninst > 0) k_cg_norms<<<ninst, kBlock, 0, st>>>(insts);
}
void launch_cg_dir(const InstDev* insts, const WorkItem* ncols, int nitems, int k, int* ndone, hipStream_t st) {
    if (nitems > 0) k_cg_dir<<<nitems, kBlock, 0, st>>>(insts, ncols, k, ndone);
}
void launch_cg_eta_test(const InstDev* insts, const Calls& C, int ninst, int k, int* ndone, hipStream_t st) {
    if (ninst > 0) k_cg_eta_test<<<ninst, kBlock, 0, st>>>(insts, C, k, ndone);
}
void launch_cg_q(const InstDev* insts, const Calls& C, const WorkItem* mrows, int nitems, int k, hipStream_t st) {
    if (nitems > 0) k_cg_q<<<nitems, kBlock, 0, st>>>(insts, C, mrows, k);
}
void launch_cg_upd(const InstDev* insts, const Calls& C, const WorkItem* mrows, int nitems, int k, int* ndone,
                   hipStream_t st) {
    if (nitems > 0) k_cg_upd<<<nitems, kBlock, 0, st>>>(insts, C, mrows, k, ndone);
}
void launch_cg_dxrhs(const InstDev* insts, const Calls& C, const WorkItem* ncols, int nitems, hipStream_t st) {
    if (nitems > 0) k_cg_dxrhs<<<nitems, kBlock, 0, st>>>(insts, C, ncols);
}
void launch_cg_residual(const InstDev* insts, const Calls& C, const WorkItem* ncols, int nn, const WorkItem* mrows,
                        int nm, int ninst, hipStream_t st) {
    if (nn > 0) k_cg_res_n<<<nn, kBlock, 0, st>>>(insts, C, ncols);
    if (nm > 0) k_cg_res_m<<<nm, kBlock, 0, st>>>(insts, C, mrows);
    if (ninst > 0) k_cg_eta<<<ninst, kBlock, 0, st>>>(insts);
}

}  // namespace kkt
