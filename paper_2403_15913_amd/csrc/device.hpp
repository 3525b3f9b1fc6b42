// Device-side descriptors shared by the host orchestration (api.cpp) and the
// HIP kernels (kernels.hip). Plain structs of device pointers: one PatDev per
// uploaded symbolic analysis, one InstDev per numeric instance (a factor, or
// one member of a batch). Kernels receive an array of InstDev and a work list
// of (instance, supernode) or (instance, row block) pairs, so the single
// instance, the batched and the served forms run the same kernels.
#pragma once
#include <cstdint>

namespace kkt {

// Entries of K with more than this many products of J entries are assembled
// by a 16-lane group each instead of one thread (the symbolic analysis lists
// them once per pattern).
constexpr int kHeavyPairs = 8;

struct PatDev {
    int n, m, ns;
    int nlevels;
    const int* sn_col0;     // ns+1
    const int* sn_ncol;
    const int* sn_nrow;
    const int64_t* sn_rowofs;
    const int64_t* sn_lofs;
    const int64_t* sn_uofs;
    const int64_t* sn_vofs;
    const int* rows;
    const int* rel;
    const int* rel_np;
    const int* ch_ptr;
    const int* ch_list;
    const int64_t* pinv_ofs;  // per ch_list entry
    const int* pinv;          // parent update row -> child update row, or -1
    const int64_t* k_snptr;
    const int* k_loc;
    const int* k_w;
    const int* k_diag;
    const int64_t* k_pptr;
    const int* pair_a;
    const int* pair_b;
    const int* jrow;
    const int* perm;
    const int* iperm;
    const int64_t* sp_ptr;
    const int* k_csr;
    const int* sp_col;
    const int* j_ptr;
    const int* j_col;
    const int* jt_ptr;
    const int* jt_e;
    const int* jt_row;
    // J by columns in pivot order: the entries of column perm[k] are
    // jtp_ptr[k] .. jtp_ptr[k+1], with their rows and CSR entry indices
    const int* jtp_ptr;
    const int* jtp_row;
    const int* jtp_e;
    const int* j_colp;      // pivot position of the column of every CSR entry of J
};

struct RefineState {
    double omega, omega_prev, eta, eta_prev, relres, relres_prev;
    double tol;
    int maxit;
    int it;        // corrections applied so far
    int done;      // 1: stop refining this instance
    int revert;    // 1: the previous iterate is the better one
};

// Conjugate-gradient record of one instance (eq. (schurcomp)), written by the
// instance's workgroup 0 of the kernel that takes each decision.
struct CgState {
    double rrs[2];           // r_k . r_k of iteration k in rrs[k & 1]
    double rr_new, pq, cnorm, tol;
    double eta_tol;          // > 0: also stop once the saddle system's eta bound is below it
    double norm_a;           // ||[[K0, J^T], [J, 0]]||_inf
    double norm_rhs;         // max(||f||_inf, ||g||_inf)
    double rmax, dymax;      // ||r||_inf and ||dy||_inf of the last eta test
    double eta;              // normwise backward error of (dx, dy) on the saddle system
    int it, maxit, done, status;
    int eta_stop;            // 1: stopped by the eta bound
};

// Full-system (augmented) refinement record of one instance: the backward
// errors of the current and previous iterates and the stop rule's state.
struct AugState {
    double eta, eta_prev, omega, omega_prev, tol;
    int it, maxit, done, revert;
};

// Interior-point loop record (one problem per factor)
struct IpmState {
    double mu, tau, gap, err, r1max, r4max, cn, un, ap, ad, delta, tol, sigma, tau_min;
    int it, done, status, maxit;
};

struct InstDev {
    PatDev P;
    // offsets of this instance inside the caller's concatenated arrays
    int64_t w_off, j_off, n_off, m_off;
    // numeric storage owned by the factor
    double* L;          // supernode panels, column-major, leading dimension = front rows
    double* U;          // update matrices, column-major u x u
    double* V;          // solve update vectors
    double* kval;       // assembled lower-triangle entries of K (grouped by supernode)
    double* kcsr;       // the same values in the symmetric row lists (both triangles, original rows)
    double* rpart;      // residual block maxima: 5 per residual block
    double* js;         // Lifted-KKT: J values scaled by their row's Sigma_s (HyKKT: copy of J)
    double* dinv;       // reciprocals of the pivots of L (pivot order)
    double* y;          // permuted work vector (n)
    double* r;          // residual (n)
    double* xprev;      // previous refinement iterate (n)
    double* tn;         // scratch (n)
    double* fg;         // HyKKT f_gamma in pivot order (n)
    double* cvec;       // HyKKT Schur right-hand side c (m)
    double* rvec;       // CG residual (m)
    double* pvec;       // CG direction (m)
    double* qvec;       // S_gamma p (m)
    double* pvec2;      // CG direction, second buffer (m): iterations alternate
    double* jtv;        // HyKKT: J values by columns in pivot order (jtp_ptr layout)
    double* k0csr;      // single factors: W + Sigma_x + delta I in the symmetric row lists (kcsr layout)
    double* jraw;       // Lifted-KKT, single factors: J values by rows (js holds them scaled)
    double* ssv;        // Lifted-KKT, single factors: Sigma_s (m)
    double* aug_b;      // augmented solve: condensed right-hand side (n, original numbering)
    double* aug_t;      // augmented solve: correction K^{-1} b (n)
    double* aug_e;      // augmented solve: residual (e1 n, e2 m, e4 m)
    double* aug_prev;   // augmented solve: previous iterate (dx n, ds m, dz m)
    AugState* aug;
    double* red;        // per-block partial sums (deterministic reductions)
    int* status;        // [0] latched status, [1] first failing pivot (permuted index)
    RefineState* rs;
    CgState* cg;
};

// One per front work item, in launch order: what a front's kernels read
// first, as absolute addresses, so its first data loads wait for this record
// alone instead of a chain of descriptor lookups. The first two children are
// inline; later children are read from the pattern arrays.
struct FrontDesc {
    const double* kv;       // original entries of K in the front
    const int* kl;          // their panel places (column << 16 | row)
    double* L;              // stored panel
    double* U;              // update matrix (u x u)
    double* V;              // update vector (u)
    double* y;              // work vector at the front's first column
    double* dinv;           // pivot reciprocals at the front's first column
    const int* rw;          // rows of the update part (instance numbering)
    const int* done;        // the instance's refinement stop flag
    const int* cgdone;      // the instance's CG stop flag
    const double* cU[2];    // first two children: update matrices,
    const double* cV[2];    //   update vectors,
    const int* crl[2];      //   relative rows of their update parts,
    const int* cinv[2];     //   inverse maps (this front's update row -> theirs, or -1),
    int cuc[2], cnb[2];     //   update sizes, and rows mapping into this front's columns
    int r, c, col0, nk;     // rows, columns, first column, entries of K
    int nch, ch0, inst, id; // children, first child in ch_list, instance, supernode
};

struct WorkItem {
    int inst;
    int id;   // supernode, or first row of a block
};

// one 16 x 16 tile (lower part) of a front's update matrix
struct StripItem {
    int inst;
    int id;     // supernode
    int tile;   // (row block << 16) | column block
    int item;   // the front's work item (index into the front descriptors)
};

}  // namespace kkt
