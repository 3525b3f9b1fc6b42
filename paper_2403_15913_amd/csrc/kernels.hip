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

#include <cstdint>

#include "device.hpp"
#include "kernels.hpp"

namespace kkt {

#define KKT_ST_NOT_SPD 4
#define KKT_ST_NONFINITE 5

__device__ inline const CallPtrs& callp(const Calls& C, int inst) { return C.arr ? C.arr[inst] : C.one; }

__device__ inline unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }
__device__ inline double bitsd(unsigned long long v) { return __longlong_as_double((long long)v); }

// ---------------------------------------------------------------------------
// fills (used instead of hipMemsetAsync so the sequences stay graph-safe)
// ---------------------------------------------------------------------------
__global__ void k_fill_i32(int* __restrict__ p, int v, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// assembly: one thread per lower entry of K
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_assemble(const InstDev* __restrict__ insts, Calls C,
                                                  const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const CallPtrs& cp = callp(C, it.inst);
    const int64_t nnzk = I.P.k_snptr[I.P.ns];
    const int64_t e = (int64_t)it.id + threadIdx.x;
    if (e >= nnzk) return;
    double v = 0.0;
    const int wi = I.P.k_w[e];
    if (wi >= 0) v += cp.w[wi];
    const int di = I.P.k_diag[e];
    if (di >= 0) v += cp.sx[di];
    const int64_t p0 = I.P.k_pptr[e], p1 = I.P.k_pptr[e + 1];
    const double* __restrict__ jv = cp.jv;
    if (cp.ss) {
        for (int64_t p = p0; p < p1; p++) {
            const int a = I.P.pair_a[p], b = I.P.pair_b[p];
            v += jv[a] * cp.ss[I.P.jrow[a]] * jv[b];
        }
    } else {
        double acc = 0.0;
        for (int64_t p = p0; p < p1; p++) acc += jv[I.P.pair_a[p]] * jv[I.P.pair_b[p]];
        v += cp.gamma * acc;
    }
    I.kval[e] = v;
    if (!isfinite(v)) atomicMax(&I.status[0], KKT_ST_NONFINITE);
}

// ---------------------------------------------------------------------------
// multifrontal factorisation of one front per workgroup
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_factor(const InstDev* __restrict__ insts, const WorkItem* __restrict__ items) {
    extern __shared__ double P[];  // front panel r x c, column-major, ld = r
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const PatDev& T = I.P;
    const int s = it.id;
    const int c = T.sn_ncol[s], r = T.sn_nrow[s], u = r - c, col0 = T.sn_col0[s];
    const int ld = r;
    const int tid = threadIdx.x, nt = blockDim.x;

    for (int q = tid; q < ld * c; q += nt) P[q] = 0.0;
    __syncthreads();
    for (int64_t e = T.k_snptr[s] + tid; e < T.k_snptr[s + 1]; e += nt) {
        const int loc = T.k_loc[e];
        P[(loc >> 16) * ld + (loc & 0xffff)] = I.kval[e];
    }
    __syncthreads();
    // extend-add the children's update matrices into the panel columns
    for (int q = T.ch_ptr[s]; q < T.ch_ptr[s + 1]; q++) {
        const int ch = T.ch_list[q];
        const int cc = T.sn_ncol[ch], uc = T.sn_nrow[ch] - cc;
        const double* __restrict__ Uc = I.U + T.sn_uofs[ch];
        const int* __restrict__ rl = T.rel + T.sn_rowofs[ch] + cc;
        for (int b = 0; b < uc; b++) {
            const int rb = rl[b];
            if (rb >= c) break;  // relative indices increase
            for (int a = b + tid; a < uc; a += nt) P[rb * ld + rl[a]] += Uc[(int64_t)b * uc + a];
        }
        __syncthreads();
    }
    // dense partial Cholesky of the panel (right-looking, column by column)
    for (int j = 0; j < c; j++) {
        double d = P[j * ld + j];
        if (!(d > 0.0) || !isfinite(d)) {
            if (tid == 0) {
                atomicMin(&I.status[1], col0 + j);
                atomicMax(&I.status[0], KKT_ST_NOT_SPD);
            }
            d = 1.0;
        }
        const double ljj = sqrt(d);
        const double inv = 1.0 / ljj;
        __syncthreads();
        if (tid == 0) P[j * ld + j] = ljj;
        for (int i = j + 1 + tid; i < r; i += nt) P[j * ld + i] *= inv;
        __syncthreads();
        for (int i = j + 1 + tid; i < r; i += nt) {
            const double lij = P[j * ld + i];
            const int kmax = min(i, c - 1);
            for (int k = j + 1; k <= kmax; k++) P[k * ld + i] -= lij * P[j * ld + k];
        }
        __syncthreads();
    }
    double* __restrict__ Ls = I.L + T.sn_lofs[s];
    for (int q = tid; q < r * c; q += nt) Ls[q] = P[q];
    if (u == 0) return;
    // update matrix U = -L21 L21^T (lower part), 4x4 register blocks
    double* __restrict__ Us = I.U + T.sn_uofs[s];
    const int nb = (u + 3) >> 2;
    const int nblk = nb * (nb + 1) / 2;
    for (int q = tid; q < nblk; q += nt) {
        int bi = (int)((sqrt(8.0 * q + 1.0) - 1.0) * 0.5);
        while (bi * (bi + 1) / 2 > q) bi--;
        while ((bi + 1) * (bi + 2) / 2 <= q) bi++;
        const int bj = q - bi * (bi + 1) / 2;
        double acc[4][4];
#pragma unroll
        for (int t = 0; t < 4; t++)
#pragma unroll
            for (int t2 = 0; t2 < 4; t2++) acc[t][t2] = 0.0;
        for (int k = 0; k < c; k++) {
            double av[4], bv[4];
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const int a = 4 * bi + t, b = 4 * bj + t;
                av[t] = a < u ? P[k * ld + c + a] : 0.0;
                bv[t] = b < u ? P[k * ld + c + b] : 0.0;
            }
#pragma unroll
            for (int t = 0; t < 4; t++)
#pragma unroll
                for (int t2 = 0; t2 < 4; t2++) acc[t][t2] += av[t] * bv[t2];
        }
#pragma unroll
        for (int t = 0; t < 4; t++)
#pragma unroll
            for (int t2 = 0; t2 < 4; t2++) {
                const int a = 4 * bi + t, b = 4 * bj + t2;
                if (a < u && b <= a) Us[(int64_t)b * u + a] = -acc[t][t2];
            }
    }
    __syncthreads();
    // extend-add the children's entries that pass through to the update matrix
    for (int q = T.ch_ptr[s]; q < T.ch_ptr[s + 1]; q++) {
        const int ch = T.ch_list[q];
        const int cc = T.sn_ncol[ch], uc = T.sn_nrow[ch] - cc;
        const double* __restrict__ Uc = I.U + T.sn_uofs[ch];
        const int* __restrict__ rl = T.rel + T.sn_rowofs[ch] + cc;
        for (int b = 0; b < uc; b++) {
            const int rb = rl[b];
            if (rb < c) continue;
            for (int a = b + tid; a < uc; a += nt)
                Us[(int64_t)(rb - c) * u + (rl[a] - c)] += Uc[(int64_t)b * uc + a];
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// triangular sweeps (y holds the permuted right-hand side, then the solution)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_fwd(const InstDev* __restrict__ insts, const WorkItem* __restrict__ items) {
    extern __shared__ double sh[];
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const PatDev& T = I.P;
    const int s = it.id;
    const int c = T.sn_ncol[s], r = T.sn_nrow[s], u = r - c, col0 = T.sn_col0[s];
    const int tid = threadIdx.x, nt = blockDim.x;
    double* P = sh;
    double* w = sh + (int64_t)r * c;
    double* va = w + c;
    const double* __restrict__ Ls = I.L + T.sn_lofs[s];
    for (int q = tid; q < r * c; q += nt) P[q] = Ls[q];
    for (int t = tid; t < c; t += nt) w[t] = I.y[col0 + t];
    for (int t = tid; t < u; t += nt) va[t] = 0.0;
    __syncthreads();
    for (int q = T.ch_ptr[s]; q < T.ch_ptr[s + 1]; q++) {
        const int ch = T.ch_list[q];
        const int cc = T.sn_ncol[ch], uc = T.sn_nrow[ch] - cc;
        const double* __restrict__ Vc = I.V + T.sn_vofs[ch];
        const int* __restrict__ rl = T.rel + T.sn_rowofs[ch] + cc;
        for (int a = tid; a < uc; a += nt) {
            const int ra = rl[a];
            if (ra < c) w[ra] += Vc[a];
            else va[ra - c] += Vc[a];
        }
        __syncthreads();
    }
    for (int j = 0; j < c; j++) {
        if (tid == 0) w[j] /= P[j * r + j];
        __syncthreads();
        const double wj = w[j];
        for (int i = j + 1 + tid; i < c; i += nt) w[i] -= P[j * r + i] * wj;
        __syncthreads();
    }
    double* __restrict__ Vs = I.V + T.sn_vofs[s];
    for (int i = tid; i < u; i += nt) {
        double sum = va[i];
        for (int k = 0; k < c; k++) sum -= P[k * r + c + i] * w[k];
        Vs[i] = sum;
    }
    for (int t = tid; t < c; t += nt) I.y[col0 + t] = w[t];
}

__global__ __launch_bounds__(256) void k_bwd(const InstDev* __restrict__ insts, const WorkItem* __restrict__ items) {
    extern __shared__ double sh[];
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const PatDev& T = I.P;
    const int s = it.id;
    const int c = T.sn_ncol[s], r = T.sn_nrow[s], u = r - c, col0 = T.sn_col0[s];
    const int tid = threadIdx.x, nt = blockDim.x;
    double* P = sh;
    double* t = sh + (int64_t)r * c;
    double* zu = t + c;
    const double* __restrict__ Ls = I.L + T.sn_lofs[s];
    const int* __restrict__ rw = T.rows + T.sn_rowofs[s] + c;
    for (int q = tid; q < r * c; q += nt) P[q] = Ls[q];
    for (int i = tid; i < u; i += nt) zu[i] = I.y[rw[i]];
    __syncthreads();
    for (int k = tid; k < c; k += nt) {
        double sum = I.y[col0 + k];
        for (int i = 0; i < u; i++) sum -= P[k * r + c + i] * zu[i];
        t[k] = sum;
    }
    __syncthreads();
    for (int j = c - 1; j >= 0; j--) {
        if (tid == 0) t[j] /= P[j * r + j];
        __syncthreads();
        const double xj = t[j];
        for (int i = tid; i < j; i += nt) t[i] -= P[i * r + j] * xj;
        __syncthreads();
    }
    for (int k = tid; k < c; k += nt) I.y[col0 + k] = t[k];
}

// ---------------------------------------------------------------------------
// permutations between original and pivot order (row blocks of 256)
// ---------------------------------------------------------------------------
__device__ inline bool inst_idle(const InstDev& I, int use_cg) { return use_cg ? I.cg->done : I.rs->done; }

// y[k] = src[perm[k]] with src = b (PIN_B), r (PIN_R), tn (PIN_TN) or f_gamma (PIN_FG)
__global__ __launch_bounds__(256) void k_perm_in(const InstDev* __restrict__ insts, Calls C,
                                                 const WorkItem* __restrict__ items, int mode) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (mode == PIN_R && I.rs->done) return;
    const int k = it.id + threadIdx.x;
    if (k >= I.P.n) return;
    const double* src = mode == PIN_B ? callp(C, it.inst).b : (mode == PIN_R ? I.r : (mode == PIN_TN ? I.tn : I.fg));
    I.y[k] = src[I.P.perm[k]];
}

// POUT_X: x[perm[k]] = y[k]; POUT_X_UPDATE: xprev = x, x += y[iperm]; POUT_TN: tn[perm[k]] = y[k];
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
        callp(C, it.inst).x[i] = v;
    } else if (mode == POUT_X_UPDATE) {
        double* x = callp(C, it.inst).x;
        const double xo = x[i];
        I.xprev[i] = xo;
        x[i] = xo + v;
    } else if (mode == POUT_TN) {
        I.tn[i] = v;
    } else {
        callp(C, it.inst).dx[i] = v;
    }
}

// ---------------------------------------------------------------------------
// residual r = b - K x and backward-error reductions (original numbering)
// ---------------------------------------------------------------------------
__global__ void k_refine_reset(const InstDev* __restrict__ insts, int ninst, double tol, int maxit) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ninst) return;
    RefineState* S = insts[q].rs;
    for (int k = 0; k < ACC_N; k++) S->acc[k] = 0ull;
    S->omega = S->omega_prev = INFINITY;
    S->eta = S->eta_prev = INFINITY;
    S->relres = S->relres_prev = INFINITY;
    S->tol = tol;
    S->maxit = maxit;
    S->it = 0;
    S->done = 0;
    S->revert = 0;
}

__device__ inline void block_max5(double v0, double v1, double v2, double v3, double v4, unsigned long long* acc) {
    __shared__ double red[5][256];
    const int tid = threadIdx.x;
    red[0][tid] = v0; red[1][tid] = v1; red[2][tid] = v2; red[3][tid] = v3; red[4][tid] = v4;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (tid < h)
            for (int q = 0; q < 5; q++) red[q][tid] = fmax(red[q][tid], red[q][tid + h]);
        __syncthreads();
    }
    if (tid == 0)
        for (int q = 0; q < 5; q++) atomicMax(&acc[q], dbits(red[q][0]));
}

__global__ __launch_bounds__(256) void k_residual(const InstDev* __restrict__ insts, Calls C,
                                                  const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (I.rs->done) return;  // uniform per block
    const CallPtrs& cp = callp(C, it.inst);
    const int i = it.id + threadIdx.x;
    double ra = 0.0, om = 0.0, rs = 0.0, xa = 0.0, ba = 0.0;
    if (i < I.P.n) {
        double sum = 0.0, den = 0.0;
        for (int64_t p = I.P.sp_ptr[i]; p < I.P.sp_ptr[i + 1]; p++) {
            const double kv = I.kval[I.P.sp_e[p]];
            const double t = kv * cp.x[I.P.sp_col[p]];
            sum += t;
            den += fabs(t);
            rs += fabs(kv);
        }
        const double bi = cp.b[i];
        const double ri = bi - sum;
        I.r[i] = ri;
        ra = fabs(ri);
        den += fabs(bi);
        om = den > 0.0 ? ra / den : (ra > 0.0 ? INFINITY : 0.0);
        xa = fabs(cp.x[i]);
        ba = fabs(bi);
    }
    block_max5(ra, om, rs, xa, ba, I.rs->acc);
}

// One thread per instance: turn the accumulated maxima into eta / omega and
// apply the refinement stop rule (omega <= tol, maxit corrections, or omega
// not halving; in the last case the previous iterate wins if omega grew).
__global__ void k_refine_decide(const InstDev* __restrict__ insts, int ninst, int* ndone) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= ninst) return;
    RefineState* S = insts[q].rs;
    if (S->done) return;
    const double rmax = bitsd(S->acc[ACC_RMAX]), om = bitsd(S->acc[ACC_OMEGA]);
    const double kn = bitsd(S->acc[ACC_KNORM]), xm = bitsd(S->acc[ACC_XMAX]), bm = bitsd(S->acc[ACC_BMAX]);
    const double den = kn * xm + bm;
    for (int k = 0; k < ACC_N; k++) S->acc[k] = 0ull;
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
    callp(C, it.inst).x[i] = I.xprev[i];
}

__global__ __launch_bounds__(256) void k_matvec(const InstDev* __restrict__ insts, const double* __restrict__ x,
                                                double* __restrict__ y, const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const int i = it.id + threadIdx.x;
    if (i >= I.P.n) return;
    double sum = 0.0;
    for (int64_t p = I.P.sp_ptr[i]; p < I.P.sp_ptr[i + 1]; p++) sum += I.kval[I.P.sp_e[p]] * x[I.P.sp_col[p]];
    y[i] = sum;
}

// ---------------------------------------------------------------------------
// Schur-complement CG (eq. (schurcomp)); vectors in original numbering
// ---------------------------------------------------------------------------
// deterministic block sum of v into red[blockslot]
__device__ inline void block_sum_to(double v, double* out) {
    __shared__ double sred[256];
    const int tid = threadIdx.x;
    sred[tid] = v;
    __syncthreads();
    for (int h = blockDim.x / 2; h > 0; h >>= 1) {
        if (tid < h) sred[tid] += sred[tid + h];
        __syncthreads();
    }
    if (tid == 0) *out = sred[0];
}

// one block per instance: fixed-order sum of nb partials
__device__ inline double block_sum_partials(const double* red, int nb) {
    __shared__ double sred[256];
    const int tid = threadIdx.x;
    double v = 0.0;
    for (int q = tid; q < nb; q += blockDim.x) v += red[q];
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

// f_gamma = f + gamma J^T g (one thread per column of J)
__global__ __launch_bounds__(256) void k_cg_fgamma(const InstDev* __restrict__ insts, Calls C,
                                                   const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const CallPtrs& cp = callp(C, it.inst);
    const int j = it.id + threadIdx.x;
    if (j >= I.P.n) return;
    double sum = 0.0;
    for (int p = I.P.jt_ptr[j]; p < I.P.jt_ptr[j + 1]; p++) sum += cp.jv[I.P.jt_e[p]] * cp.g[I.P.jt_row[p]];
    I.fg[j] = cp.f[j] + cp.gamma * sum;
}

// c = J w - g with w = K_gamma^{-1} f_gamma in tn; r = p = c; dy = 0; partial c.c
__global__ __launch_bounds__(256) void k_cg_init(const InstDev* __restrict__ insts, Calls C,
                                                 const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    const CallPtrs& cp = callp(C, it.inst);
    const int i = it.id + threadIdx.x;
    double v = 0.0;
    if (i < I.P.m) {
        double sum = 0.0;
        for (int p = I.P.j_ptr[i]; p < I.P.j_ptr[i + 1]; p++) sum += cp.jv[p] * I.tn[I.P.j_col[p]];
        const double ci = sum - cp.g[i];
        I.cvec[i] = ci;
        I.rvec[i] = ci;
        I.pvec[i] = ci;
        cp.dy[i] = 0.0;
        v = ci * ci;
    }
    block_sum_to(v, &I.red[it.id / 256]);
}

__global__ __launch_bounds__(256) void k_cg_start(const InstDev* __restrict__ insts, double tol, int maxit, int* ndone) {
    const InstDev& I = insts[blockIdx.x];
    const int nb = (I.P.m + 255) / 256;
    const double rr = block_sum_partials(I.red, nb);
    if (threadIdx.x == 0) {
        CgState* G = I.cg;
        G->rr = rr;
        G->cnorm = sqrt(rr);
        G->tol = tol;
        G->maxit = maxit;
        G->it = 0;
        G->status = 0;
        G->done = (sqrt(rr) <= tol * G->cnorm) ? 1 : 0;  // c == 0
        G->alpha = G->beta = 0.0;
        if (G->done) atomicAdd(ndone, 1);
    }
}

// tn = J^T p (dx_rhs = 0), or tn = f_gamma - J^T dy (dx_rhs = 1)
__global__ __launch_bounds__(256) void k_cg_jt(const InstDev* __restrict__ insts, Calls C,
                                               const WorkItem* __restrict__ items, int dx_rhs) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (!dx_rhs && I.cg->done) return;
    const CallPtrs& cp = callp(C, it.inst);
    const int j = it.id + threadIdx.x;
    if (j >= I.P.n) return;
    const double* v = dx_rhs ? cp.dy : I.pvec;
    double sum = 0.0;
    for (int p = I.P.jt_ptr[j]; p < I.P.jt_ptr[j + 1]; p++) sum += cp.jv[I.P.jt_e[p]] * v[I.P.jt_row[p]];
    I.tn[j] = dx_rhs ? I.fg[j] - sum : sum;
}

// q = J t (t in tn), partial p.q
__global__ __launch_bounds__(256) void k_cg_jq(const InstDev* __restrict__ insts, Calls C,
                                               const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (I.cg->done) return;
    const CallPtrs& cp = callp(C, it.inst);
    const int i = it.id + threadIdx.x;
    double v = 0.0;
    if (i < I.P.m) {
        double sum = 0.0;
        for (int p = I.P.j_ptr[i]; p < I.P.j_ptr[i + 1]; p++) sum += cp.jv[p] * I.tn[I.P.j_col[p]];
        I.qvec[i] = sum;
        v = I.pvec[i] * sum;
    }
    block_sum_to(v, &I.red[it.id / 256]);
}

__global__ __launch_bounds__(256) void k_cg_alpha(const InstDev* __restrict__ insts, int* ndone) {
    const InstDev& I = insts[blockIdx.x];
    if (I.cg->done) return;
    const int nb = (I.P.m + 255) / 256;
    const double pq = block_sum_partials(I.red, nb);
    if (threadIdx.x == 0) {
        CgState* G = I.cg;
        G->pq = pq;
        if (!(pq > 0.0)) {
            G->status = 7;  // breakdown
            G->done = 1;
            atomicAdd(ndone, 1);
        } else {
            G->alpha = G->rr / pq;
        }
    }
}

// dy += alpha p; r -= alpha q; partial r.r
__global__ __launch_bounds__(256) void k_cg_update(const InstDev* __restrict__ insts, Calls C,
                                                   const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (I.cg->done) return;
    const CallPtrs& cp = callp(C, it.inst);
    const int i = it.id + threadIdx.x;
    const double a = I.cg->alpha;
    double v = 0.0;
    if (i < I.P.m) {
        cp.dy[i] += a * I.pvec[i];
        const double ri = I.rvec[i] - a * I.qvec[i];
        I.rvec[i] = ri;
        v = ri * ri;
    }
    block_sum_to(v, &I.red[it.id / 256]);
}

__global__ __launch_bounds__(256) void k_cg_beta(const InstDev* __restrict__ insts, int* ndone) {
    const InstDev& I = insts[blockIdx.x];
    if (I.cg->done) return;
    const int nb = (I.P.m + 255) / 256;
    const double rr2 = block_sum_partials(I.red, nb);
    if (threadIdx.x == 0) {
        CgState* G = I.cg;
        G->it += 1;
        G->rr_new = rr2;
        if (sqrt(rr2) <= G->tol * G->cnorm) {
            G->done = 1;
        } else if (G->it >= G->maxit) {
            G->status = 6;  // not converged
            G->done = 1;
        } else {
            G->beta = rr2 / G->rr;
            G->rr = rr2;
        }
        if (G->done) atomicAdd(ndone, 1);
    }
}

__global__ __launch_bounds__(256) void k_cg_p(const InstDev* __restrict__ insts, const WorkItem* __restrict__ items) {
    const WorkItem it = items[blockIdx.x];
    const InstDev& I = insts[it.inst];
    if (I.cg->done) return;
    const int i = it.id + threadIdx.x;
    if (i >= I.P.m) return;
    I.pvec[i] = I.rvec[i] + I.cg->beta * I.pvec[i];
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
hipError_t set_kernel_attributes() {
    const int lds = 160 * 1024;
    hipError_t e = hipFuncSetAttribute((const void*)k_factor, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void*)k_fwd, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void*)k_bwd, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

static inline unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_fill_i32(int* p, int v, int64_t n, hipStream_t st) {
    if (n > 0) k_fill_i32<<<blocks_for(n, kBlock), kBlock, 0, st>>>(p, v, n);
}
void launch_assemble(const InstDev* insts, const Calls& C, const WorkItem* items, int nitems, hipStream_t st) {
    if (nitems > 0) k_assemble<<<nitems, kBlock, 0, st>>>(insts, C, items);
}
void launch_factor(const InstDev* insts, const WorkItem* items, int nitems, size_t lds, hipStream_t st) {
    if (nitems > 0) k_factor<<<nitems, kBlock, lds, st>>>(insts, items);
}
void launch_fwd(const InstDev* insts, const WorkItem* items, int nitems, size_t lds, hipStream_t st) {
    if (nitems > 0) k_fwd<<<nitems, kBlock, lds, st>>>(insts, items);
}
void launch_bwd(const InstDev* insts, const WorkItem* items, int nitems, size_t lds, hipStream_t st) {
    if (nitems > 0) k_bwd<<<nitems, kBlock, lds, st>>>(insts, items);
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
    if (nitems > 0) k_residual<<<nitems, kBlock, 0, st>>>(insts, C, rows);
}
void launch_refine_decide(const InstDev* insts, int ninst, int* ndone, hipStream_t st) {
    k_refine_decide<<<blocks_for(ninst, 64), 64, 0, st>>>(insts, ninst, ndone);
}
void launch_refine_revert(const InstDev* insts, const Calls& C, const WorkItem* rows, int nitems, hipStream_t st) {
    if (nitems > 0) k_refine_revert<<<nitems, kBlock, 0, st>>>(insts, C, rows);
}
void launch_matvec(const InstDev* insts, const double* x, double* y, const WorkItem* rows, int nitems, hipStream_t st) {
    if (nitems > 0) k_matvec<<<nitems, kBlock, 0, st>>>(insts, x, y, rows);
}
void launch_cg_fgamma(const InstDev* insts, const Calls& C, const WorkItem* ncols, int nitems, hipStream_t st) {
    if (nitems > 0) k_cg_fgamma<<<nitems, kBlock, 0, st>>>(insts, C, ncols);
}
void launch_cg_init(const InstDev* insts, const Calls& C, const WorkItem* mrows, int nitems, hipStream_t st) {
    if (nitems > 0) k_cg_init<<<nitems, kBlock, 0, st>>>(insts, C, mrows);
}
void launch_cg_start(const InstDev* insts, int ninst, double tol, int maxit, int* ndone, hipStream_t st) {
    k_cg_start<<<ninst, kBlock, 0, st>>>(insts, tol, maxit, ndone);
}
void launch_cg_jt(const InstDev* insts, const Calls& C, const WorkItem* ncols, int nitems, int dx_rhs, hipStream_t st) {
    if (nitems > 0) k_cg_jt<<<nitems, kBlock, 0, st>>>(insts, C, ncols, dx_rhs);
}
void launch_cg_jq(const InstDev* insts, const Calls& C, const WorkItem* mrows, int nitems, hipStream_t st) {
    if (nitems > 0) k_cg_jq<<<nitems, kBlock, 0, st>>>(insts, C, mrows);
}
void launch_cg_alpha(const InstDev* insts, int ninst, int* ndone, hipStream_t st) {
    k_cg_alpha<<<ninst, kBlock, 0, st>>>(insts, ndone);
}
void launch_cg_update(const InstDev* insts, const Calls& C, const WorkItem* mrows, int nitems, hipStream_t st) {
    if (nitems > 0) k_cg_update<<<nitems, kBlock, 0, st>>>(insts, C, mrows);
}
void launch_cg_beta(const InstDev* insts, int ninst, int* ndone, hipStream_t st) {
    k_cg_beta<<<ninst, kBlock, 0, st>>>(insts, ndone);
}
void launch_cg_p(const InstDev* insts, const WorkItem* mrows, int nitems, hipStream_t st) {
    if (nitems > 0) k_cg_p<<<nitems, kBlock, 0, st>>>(insts, mrows);
}

}  // namespace kkt
