// Host-callable launch wrappers for the HIP kernels in kernels.hip.
#pragma once
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "lds_layout.hpp"

namespace kkt {

// Base pointers of one call (values of a refactorisation, vectors of a
// solve), passed by value. Instance q uses base + its offsets (InstDev
// w_off / j_off / n_off / m_off), so a batch reads concatenated arrays.
struct Calls {
    const double* w;
    const double* jv;
    const double* sx;
    const double* ss;   // NULL -> K_gamma with row weight gamma
    double gamma;
    double delta;       // primal regularisation added to the diagonal of K (inertia correction)
    const int* eqm;     // general HyKKT: 1 for the equality rows of J (weight gamma), 0 for the
                        // inequality rows (weight sigma_s); NULL otherwise
    int keep_k0;        // assembly also writes K0 (or K_k) into k0csr (single factors that need it)
    const double* b;    // Lifted-KKT solve
    double* x;
    const double* f;    // HyKKT solve
    const double* g;
    double* dx;
    double* dy;
};

constexpr int kBlock = 256;
constexpr int kSplitMaxFronts = 140;  // levels with fewer fronts launch their update matrices by tiles
constexpr int kSplitMinRows = 64;     // ... when the level's widest update part has at least this many rows
constexpr int kResidualSplit = 8;    // residual blocks per 256-row item (two rows per 16-lane group)
static_assert(16 % kResidualSplit == 0, "a 256-row item splits into whole rows per 16-lane group");

// Dependency lists of a persistent (queue-scheduled) launch over the fronts
// in topological order: parent item (-1 for roots), number of children, and
// per-item counters reset before every launch.
struct DepLists {
    const int* parent;
    const int* nchild;
    int* cnt;     // children done (factor / forward sweep)
    int* fdone;   // root forward step done
    int* bdone;   // backward step done
    int* ticket;
    int* err;     // set when a bounded wait expired
    int nitems;
};

// Dynamic LDS a front may use (the kernels also hold a little static LDS;
// gfx950 gives a workgroup 160 KiB in total).
constexpr int kMaxDynLds = 158 * 1024;
// sweep fronts at or below this LDS size run two workgroups per compute unit
// (160 KiB of LDS per CU; the sweep kernels' registers allow two)
constexpr size_t kSweepHalfLds = 79 * 1024;
// a level's small fronts get a sweep launch of their own from this many on
// (two workgroups on each of the 256 compute units)
constexpr int kSweepSplitMin = 512;

hipError_t set_kernel_attributes();

// Per-solve workspace of one instance held outside the factor (the
// allocation-free solve): redirected copies of the instance and front
// descriptors and the vectors a refined solve writes.
struct SolveWs {
    InstDev* inst;       // 1
    FrontDesc* fd;       // one per front, in the factor's launch order
    double* y;           // n: permuted work vector
    double* V;           // forward-sweep update vectors (the factor's V layout)
    double* r;           // n: residual
    double* xprev;       // n: previous iterate
    double* rpart;       // residual block maxima
    RefineState* rs;     // 1
};
// Writes ws.inst and ws.fd from the factor's descriptors (src_inst[0],
// src_fd[0 .. nf)) with every per-solve pointer moved into ws.
void launch_ws_redirect(const InstDev* src_inst, const FrontDesc* src_fd, int nf, const SolveWs& ws, hipStream_t st);

// A device-to-device copy of `len` doubles (gathering a served wave's inputs).
struct CopySeg {
    const double* src;
    double* dst;
    int64_t len;
};
void launch_copy_segments(const CopySeg* segs, int nseg, hipStream_t st);

void launch_fill_i32(int* p, int v, int64_t n, hipStream_t st);
void launch_status_init(int* status, int ninst, hipStream_t st);
void launch_jscale(const InstDev* insts, const Calls& C, const WorkItem* items, int nitems, hipStream_t st);
// Lifted-KKT, single factors: J's values by rows and by columns in pivot
// order and Sigma_s, kept for the augmented-system solve
void launch_keep_lifted(const InstDev* insts, const Calls& C, const WorkItem* jentries, int nj, const WorkItem* mrows,
                        int nm, hipStream_t st);
// K_gamma: J's values by rows and by columns in pivot order, kept for the CG
void launch_jcopy(const InstDev* insts, const Calls& C, const WorkItem* items, int nitems, hipStream_t st);
void launch_assemble(const InstDev* insts, const Calls& C, const WorkItem* items, int nitems, hipStream_t st);
// entries of K with more than kHeavyPairs products of J entries are left to
// launch_assemble_heavy (one item per entry, 16 lanes each)
void launch_assemble_heavy(const InstDev* insts, const Calls& C, const WorkItem* items, int nitems, hipStream_t st);
void launch_factor(const InstDev* insts, const FrontDesc* fds, int nitems, size_t lds, int fused_update,
                   hipStream_t st);
// the same with four-wave workgroups (lds: the level's own largest front)
void launch_factor_small(const InstDev* insts, const FrontDesc* fds, int nitems, size_t lds, int fused_update,
                         hipStream_t st);
// large fronts (panels too tall for LDS, at most kLargeFrontCols columns):
// assembly and factorization in place in HBM (the update matrices then by
// launch_update), and their sweeps
// (several workgroups per front: assembly by column block, then per column
// block the rows below the diagonal block and the later blocks' update;
// max_cols / max_rows bound the fronts of the launch)
void launch_big_factor(const InstDev* insts, const FrontDesc* fds, int nitems, int max_cols, int max_rows,
                       hipStream_t st);
void launch_big_fwd(const InstDev* insts, const FrontDesc* fds, int nitems, int skip_done, hipStream_t st);
void launch_big_bwd(const FrontDesc* fds, int nitems, int skip_done, hipStream_t st);
// update matrices by 16-column strips (after the factor launch of the same level)
void launch_update(const InstDev* insts, const FrontDesc* fds, const StripItem* items, int nitems, hipStream_t st);
void launch_factor_queue(const InstDev* insts, const FrontDesc* fds, const DepLists& D, int grid, size_t lds,
                         hipStream_t st);
void launch_sweeps_queue(const InstDev* insts, const FrontDesc* fds, const DepLists& D, int grid, size_t lds,
                         int skip_done, hipStream_t st);
void launch_fwd(const InstDev* insts, const FrontDesc* fds, int nitems, size_t lds, int skip_done, hipStream_t st);
void launch_bwd(const FrontDesc* fds, int nitems, size_t lds, int skip_done, hipStream_t st);

// permutation modes
enum { PIN_B = 0, PIN_R = 1 };
enum { POUT_X = 0, POUT_X_UPDATE = 1, POUT_DX = 3 };
// sweep skip modes (see front_idle)
enum { SKIP_NONE = 0, SKIP_REFINE = 1, SKIP_CG = 2 };
void launch_perm_in(const InstDev* insts, const Calls& C, const WorkItem* rows, int nitems, int mode, hipStream_t st);
void launch_perm_out(const InstDev* insts, const Calls& C, const WorkItem* rows, int nitems, int mode, hipStream_t st);

void launch_refine_reset(const InstDev* insts, int ninst, double tol, int maxit, hipStream_t st);
void launch_residual(const InstDev* insts, const Calls& C, const WorkItem* rows, int nitems, hipStream_t st);
void launch_refine_decide(const InstDev* insts, int ninst, int* ndone, hipStream_t st);
void launch_refine_revert(const InstDev* insts, const Calls& C, const WorkItem* rows, int nitems, hipStream_t st);
void launch_matvec(const InstDev* insts, const double* x, double* y, const WorkItem* rows, int nitems, hipStream_t st);

// Schur-complement CG (one CgState per instance); k is the iteration index
void launch_cg_fg(const InstDev* insts, const Calls& C, const WorkItem* ncols, int nitems, double tol, int maxit,
                  double eta_tol, hipStream_t st);
void launch_cg_c(const InstDev* insts, const Calls& C, const WorkItem* mrows, int nitems, int ninst, hipStream_t st);
void launch_cg_dir(const InstDev* insts, const WorkItem* ncols, int nitems, int k, int* ndone, hipStream_t st);
void launch_cg_eta_test(const InstDev* insts, const Calls& C, int ninst, int k, int* ndone, hipStream_t st);
void launch_cg_q(const InstDev* insts, const Calls& C, const WorkItem* mrows, int nitems, int k, hipStream_t st);
void launch_cg_upd(const InstDev* insts, const Calls& C, const WorkItem* mrows, int nitems, int k, int* ndone,
                   hipStream_t st);
void launch_cg_dxrhs(const InstDev* insts, const Calls& C, const WorkItem* ncols, int nitems, hipStream_t st);
// saddle-system residual of (dx, dy) and its normwise backward error (CgState::eta)
void launch_cg_residual(const InstDev* insts, const Calls& C, const WorkItem* ncols, int nn, const WorkItem* mrows,
                        int nm, int ninst, hipStream_t st);

// Augmented system of eq. (kkt:augmented) without equality rows (see the
// kernels): the caller's right-hand sides r1, r2, r4 and unknowns dx, ds, dz
struct AugCall {
    const double* r1;   // n
    const double* r2;   // m
    const double* r4;   // m
    double* dx;         // n
    double* ds;         // m
    double* dz;         // m
};
// mode 0: b = -(r1 + J^T (Sigma_s r4 - r2)); mode 1: the same with -r = e,
// the current residual (correction right-hand side)
void launch_aug_rhs(const InstDev* insts, const AugCall& A, const WorkItem* ncols, int nitems, int mode,
                    hipStream_t st);
// mode 0: ds = -r4 - J dx, dz = -r2 - Sigma_s ds; mode 1: the correction from
// t = K^{-1} b (in aug_t): the previous iterate is kept, then dx += t,
// ds += e4 - J t, dz += e2 - Sigma_s (e4 - J t)
void launch_aug_recover(const InstDev* insts, const AugCall& A, const WorkItem* ncols, int nn, const WorkItem* mrows,
                        int nm, int mode, hipStream_t st);
void launch_aug_reset(const InstDev* insts, int ninst, double tol, int maxit, hipStream_t st);
// residual of the augmented system, its backward errors and the stop rule
void launch_aug_check(const InstDev* insts, const AugCall& A, const WorkItem* ncols, int nn, const WorkItem* mrows,
                      int nm, int ninst, hipStream_t st);
void launch_aug_revert(const InstDev* insts, const AugCall& A, const WorkItem* ncols, int nn, const WorkItem* mrows,
                       int nm, hipStream_t st);

// Interior-point loop on a convex QP (min 1/2 x^T W x + c^T x, J x <= u) over
// one factor's pattern; vectors in original numbering (see the kernels)
struct IpmCall {
    const double* w;    // W values (lower CSR entry order)
    const double* jv;   // J values
    const double* c;    // n
    const double* u;    // m
    double* x;          // n
    double* s;          // m
    double* z;          // m
    double* dsw;        // m: D_s = z / s (the refactor's sigma_s)
    double* r1;         // n
    double* r2;         // m
    double* r4;         // m
    double* dx;         // n
    double* ds;         // m
    double* dz;         // m
    double* red;        // reduction slots (4 per 256-row block of n, then of m)
    IpmState* st;
};
void launch_ipm_start(const InstDev* insts, const IpmCall& P, const WorkItem* ncols, int nn, const WorkItem* mrows,
                      int nm, double tol, int maxit, double sigma, double tau_min, hipStream_t st);
void launch_ipm_dsw(const InstDev* insts, const IpmCall& P, const WorkItem* mrows, int nm, hipStream_t st);
void launch_ipm_residuals(const InstDev* insts, const IpmCall& P, const WorkItem* ncols, int nn, const WorkItem* mrows,
                          int nm, double delta, hipStream_t st);
void launch_ipm_r2(const InstDev* insts, const IpmCall& P, const WorkItem* mrows, int nm, hipStream_t st);
void launch_ipm_step(const InstDev* insts, const IpmCall& P, const WorkItem* ncols, int nn, const WorkItem* mrows,
                     int nm, hipStream_t st);

// Stage-structured (block-tridiagonal) K factored by block cyclic reduction:
// one task per stage, run at the level where the stage is eliminated.
constexpr int kCrMaxStage = 80;  // widest stage the LDS buffers hold
struct CrTask {
    int inst;            // InstDev index (status, refinement records)
    int elim;            // 1: the stage is eliminated at this level; 0: it stays
    int from_work;       // 1: the stage's block is read from the work copy in L (updated on an earlier level)
    int sk, sl, sr;      // widths of the stage and of its active left / right neighbours (0: none)
    int var0;            // first variable of the stage, instance numbering
    int v0, vl, vr;      // first variables of the stage and the neighbours, concatenated numbering
    int pull0, npull;    // its entries in the pull list (at most two, from the previous level)
    int64_t d;           // D_k (s_k x s_k), and its place in L: the updated copy, then L_k  [D, L]
    int64_t kl;          // K(k,l) (s_k x s_l): E_{k-1} or a fill block     [C]
    int64_t kr;          // K(r,k) (s_r x s_k): E_k or a fill block         [C]
    int64_t pl, pr;      // L(l,k) (s_l x s_k), L(r,k) (s_r x s_k)          [P]
    int64_t f;           // fill K(r,l) = -L(r,k) L(l,k)^T (s_r x s_l)      [C]
    int64_t ul, ur;      // L(l,k) L(l,k)^T, L(r,k) L(r,k)^T (lower parts)  [U]
};
// one contribution to a stage from a neighbour eliminated at the previous level
struct CrPull {
    int64_t u;           // update block subtracted from D_k (s_k x s_k)    [U]
    int64_t p;           // the factor block L(k,i) (s_k x s_i)            [P]
    int vi, si;          // y_i: first variable (concatenated), width
};
struct CrArrays {
    double* D;           // assembled diagonal blocks (column-major); only the scatter writes them
    double* L;           // same layout: the updated blocks of stages that stay, then L_k
    double* C;           // couplings: the assembled E_k first, then the fill blocks
    double* P;           // off-diagonal factor blocks
    double* U;           // symmetric updates
    double* t;           // solve work vector (concatenated numbering)
    const CrTask* tasks;
    const CrPull* pulls;
};
// an entry of the assembled K (kcsr, lower positions) and its place in D or C
struct CrScatter {
    int inst;            // InstDev index
    int pos;             // position in the instance's kcsr
    int64_t dst;         // >= 0: index into D; < 0: -dst - 1 into C
};
void launch_fill_f64(double* p, double v, int64_t n, hipStream_t st);
void launch_cr_scatter(const InstDev* insts, const CrArrays& A, const CrScatter* items, int64_t nitems,
                       hipStream_t st);
// one launch per level and width class (nb: widths <= 16 nb): each task
// eliminates its stage or applies the previous level's updates to a stage
// that stays (CrTask::elim)
void launch_cr_factor(const InstDev* insts, const CrArrays& A, int task0, int ntask, int nb, size_t lds,
                      hipStream_t st);
// mode 0: from b; mode 1 (refinement, skips stopped instances): from the
// residual, x += correction; level0: the first level (reads b or r)
void launch_cr_fwd(const InstDev* insts, const CrArrays& A, int task0, int ntask, const Calls& C, int mode,
                   int level0, hipStream_t st);
void launch_cr_bwd(const InstDev* insts, const CrArrays& A, int task0, int ntask, const Calls& C, int mode,
                   hipStream_t st);

}  // namespace kkt
