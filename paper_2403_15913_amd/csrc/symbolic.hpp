// Host-side symbolic analysis of the condensed KKT matrix
//   K = W + Sigma_x + J^T diag(d) J
// (Pacaud & Shin, arXiv 2403.15913: condensed matrix of eq. (kkt:condensed),
// Lifted-KKT eq. (liftedkkt), K_gamma of eq. (hykkt)). The pattern of K is
// fixed across interior-point iterations, so this analysis runs once per
// pattern and is reused by every refactorisation (section "Hybrid linear
// solver": symbolic factorisation computed once, refactorised many times).
//
// Everything here is integer work on the host; nothing touches the GPU.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace kkt {

struct SymOptions {
    int ordering = 0;        // 0 auto, 1 natural, 2 nested dissection
    int nd_leaf = 0;         // ND: parts with at most this many vertices are not split (0: auto)
    int max_super = 96;      // widest supernode (columns)
    double relax_frac = 0.5; // amalgamation: allowed fraction of explicit zeros in a merged supernode
    int relax_small = 16;    // amalgamation: supernodes up to this width merge regardless of zeros
    int lds_bytes = 160 * 1024; // per-workgroup LDS available to one front panel
};

// Row index r of supernode s lives at rows[rowofs[s] + r]; the first ncol
// rows are the supernode's own columns (permuted numbering), the remaining
// nrow - ncol are its update rows, sorted ascending.
struct Symbolic {
    int n = 0, m = 0;
    int64_t nnz_w = 0, nnz_j = 0;
    std::vector<int> perm, iperm;          // perm[k] = original index of pivot k

    int ns = 0;
    std::vector<int> sn_col0, sn_ncol, sn_nrow, sn_parent, sn_level;
    std::vector<int64_t> sn_rowofs, sn_lofs, sn_uofs, sn_vofs;  // panels: ld = nrow|1, even length
    std::vector<int> rows;                 // row structure of every front
    std::vector<int> rel;                  // rel[rowofs[s]+ncol+a]: local row of update row a in the parent front
    std::vector<int> rel_np;               // update rows of s that fall in the parent's own columns
    std::vector<int> ch_ptr, ch_list;      // children, ascending
    std::vector<int64_t> pinv_ofs;         // per ch_list entry: its inverse map in pinv
    std::vector<int> pinv;                 // child's inverse map: parent update row -> child update row, or -1
    std::vector<int> lvl_ptr, lvl_list;    // supernodes grouped by tree level (leaves first)
    int nlevels = 0;
    int64_t lsize = 0, usize = 0, vsize = 0;

    // Entries of the lower triangle of K, grouped by destination supernode
    // (then by local column, then by local row).
    int64_t nnzk = 0;
    std::vector<int64_t> k_snptr;          // ns + 1
    std::vector<int> k_loc;                // (local col << 16) | local row in the front panel
    std::vector<int> k_w;                  // index into W values, or -1
    std::vector<int> k_diag;               // original index i for Sigma_x[i], or -1
    std::vector<int64_t> k_pptr;           // nnzk + 1: range of J-entry pairs
    std::vector<int> pair_a, pair_b;       // J entry indices (same row of J)
    std::vector<int> k_heavy;              // entries with more than kHeavyPairs pairs
    std::vector<int> jrow;                 // row of every J entry
    std::vector<int64_t> sp_ptr;           // n + 1: symmetric K x by original rows
    std::vector<int> sp_e, sp_col;         // entry id and column for each stored product
    std::vector<int> k_csr;                // 2 per K entry: its positions in the row lists (-1: diagonal)
    std::vector<int> j_ptr, j_col;         // J as CSR (copy)
    std::vector<int> jt_ptr, jt_e, jt_row; // J^T as CSR (i.e. J by columns)

    // statistics
    double flops = 0;          // dense front work (what the kernels execute)
    double flops_exact = 0;    // sum over columns of (column count)^2
    int64_t nnzl_exact = 0;    // nnz(L) of the exact (unpadded) structure, diagonal included
    int max_nrow = 0, max_ncol = 0, max_nupd = 0;
    int lds_budget = 0;        // LDS a front panel may use; taller fronts are large fronts
    int n_large = 0;           // large fronts (factored and solved in HBM)
    double analyze_seconds = 0;
};

// Returns a kkt_status value (0 ok); err receives a message on failure.
int analyze(int n, int m, const int32_t* wp, const int32_t* wi, const int32_t* jp, const int32_t* ji,
            const SymOptions& opt, Symbolic& S, std::string& err);

}  // namespace kkt
