// Interior-point outer loop on a convex QP over one factor's pattern
// (kkt_ipm_qp). Each iteration refactors the condensed matrix with the new
// slack weights D_s = Z S^{-1} (same analysis, inertia correction), takes the
// Newton step through the augmented system, and moves by fraction-to-boundary
// steps; the vector work runs in the k_ipm_* kernels, the host reads one
// record per iteration to decide whether to stop.
#include <hip/hip_runtime.h>

#include <cstring>

#include "api_internal.hpp"

using namespace kkt;

namespace {
// the loop's device vectors, carved from one allocation made on first use
struct IpmBuffers {
    double *sx0, *dsw, *r1, *r2, *r4, *dx, *ds, *dz, *red;
    IpmState* st;
};

size_t carve(char* base, int n, int m, IpmBuffers* B) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        off = (off + 255) & ~(size_t)255;
        char* p = base ? base + off : nullptr;
        off += bytes > 0 ? bytes : 8;
        return p;
    };
    const size_t nn = (size_t)std::max(n, 1) * 8, mm = (size_t)std::max(m, 1) * 8;
    B->sx0 = (double*)take(nn);
    B->dsw = (double*)take(mm);
    B->r1 = (double*)take(nn);
    B->r2 = (double*)take(mm);
    B->r4 = (double*)take(mm);
    B->dx = (double*)take(nn);
    B->ds = (double*)take(mm);
    B->dz = (double*)take(mm);
    B->red = (double*)take(8 * (size_t)(4 * ((n + 255) / 256) + 4 * ((m + 255) / 256) + 8));
    B->st = (IpmState*)take(sizeof(IpmState));
    return off;
}
}  // namespace

extern "C" void kkt_ipm_opts_default(kkt_ipm_opts* o) {
    if (!o) return;
    o->tol = 1e-8;
    o->maxit = 100;
    o->sigma = 0.1;
    o->tau_min = 0.99;
}

extern "C" kkt_status kkt_ipm_qp(kkt_factor* f, const double* w_vals, const double* j_vals, const double* c,
                                 const double* u, double* x, double* s, double* z, const kkt_ipm_opts* opts,
                                 kkt_ipm_info* info, void* stream) {
    if (!f) return fail(KKT_ERR_INVALID_ARG, "NULL factor");
    const Symbolic& S = f->sym->S;
    const int n = S.n, m = S.m;
    if ((n > 0 && (!c || !x)) || (m > 0 && (!u || !s || !z)) || (S.nnz_w > 0 && !w_vals) || (S.nnz_j > 0 && !j_vals))
        return fail(KKT_ERR_INVALID_ARG, "NULL argument");
    Engine& E = f->eng;
    if (E.n_eq > 0) return fail(KKT_ERR_STATE, "the interior-point loop takes inequality rows only");
    kkt_ipm_opts o;
    kkt_ipm_opts_default(&o);
    if (opts) o = *opts;
    if (!(o.tol > 0.0) || o.maxit < 0 || !(o.sigma > 0.0 && o.sigma < 1.0) || !(o.tau_min > 0.0 && o.tau_min < 1.0))
        return fail(KKT_ERR_INVALID_ARG, "bad interior-point options");
    const hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    IpmBuffers B{};
    const size_t need = carve(nullptr, n, m, &B);
    if (E.ipm_ws.bytes < need) {
        E.ipm_ws.release();
        if ((e = E.ipm_ws.alloc(need)) != hipSuccess) return hip_fail(e, "interior-point workspace");
    }
    carve((char*)E.ipm_ws.p, n, m, &B);
    if ((e = hipMemsetAsync(B.sx0, 0, (size_t)std::max(n, 1) * 8, st)) != hipSuccess)
        return hip_fail(e, "interior-point workspace");
    E.keep_aug = true;  // the residuals use the kept W, the steps the augmented solve
    IpmCall P;
    std::memset(&P, 0, sizeof(P));
    P.w = w_vals; P.jv = j_vals; P.c = c; P.u = u; P.x = x; P.s = s; P.z = z;
    P.dsw = B.dsw; P.r1 = B.r1; P.r2 = B.r2; P.r4 = B.r4; P.dx = B.dx; P.ds = B.ds; P.dz = B.dz;
    P.red = B.red; P.st = B.st;
    launch_ipm_start(E.di(), P, E.nitems, E.n_nitems, E.mitems, E.n_mitems, o.tol, o.maxit, o.sigma, o.tau_min, st);
    IpmState H{};
    double max_delta = 0.0;
    int aug_iters = 0;
    for (;;) {
        launch_ipm_dsw(E.di(), P, E.mitems, E.n_mitems, st);
        kkt_inertia_info ii{};
        kkt_status ks = kkt_refactor_inertia(f, w_vals, j_vals, B.sx0, B.dsw, 0.0, nullptr, &ii, stream);
        if (ks != KKT_OK) return ks;
        max_delta = std::max(max_delta, ii.delta);
        launch_ipm_residuals(E.di(), P, E.nitems, E.n_nitems, E.mitems, E.n_mitems, ii.delta, st);
        if ((e = hipMemcpyAsync(E.hpin, B.st, sizeof(IpmState), hipMemcpyDeviceToHost, st)) != hipSuccess ||
            (e = hipStreamSynchronize(st)) != hipSuccess)
            return hip_fail(e, "interior-point control");
        std::memcpy(&H, E.hpin, sizeof(H));
        if (H.done) break;
        launch_ipm_r2(E.di(), P, E.mitems, E.n_mitems, st);
        AugCall A{B.r1, B.r2, B.r4, B.dx, B.ds, B.dz};
        kkt_aug_info ai{};
        ks = E.solve_augmented(A, 10, 1e-14, &ai, st);
        if (ks != KKT_OK && ks != KKT_ERR_NOT_CONVERGED) return ks;
        aug_iters += ai.iters;
        launch_ipm_step(E.di(), P, E.nitems, E.n_nitems, E.mitems, E.n_mitems, st);
    }
    if ((e = hipGetLastError()) != hipSuccess) return hip_fail(e, "interior-point launch");
    if (info) {
        info->status = H.status == 0 ? KKT_OK : H.status;
        info->iterations = H.it;
        info->err = H.err;
        info->gap = H.gap;
        info->r1 = H.r1max;
        info->r4 = H.r4max;
        info->max_delta = max_delta;
        info->aug_corrections = aug_iters;
    }
    if (H.status != 0) return fail(H.status, "interior-point iteration limit reached");
    return KKT_OK;
}
