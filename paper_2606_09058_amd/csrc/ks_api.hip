// ks_api.hip -- the C-ABI (include/ks.h): plan, argument validation,
// workspace, and the host-side enqueueing of the device pipeline
//   Cholesky -> reduction -> tridiagonalisation -> divide and conquer ->
//   back-transform -> (I (x) L)^-H, then Fermi level and density, and the adjoint.
// Argument errors are detected here before any HIP call.
#include <stdlib.h>
#include <string.h>

#include <new>

#include "ks_internal.hpp"

using namespace ks;

struct ks_plan {
    ks_plan_desc d;
    int order = 0, nsp = 1;
    bool is_c = false;
    size_t es = 8;
    hipStream_t s = nullptr;
    char* base = nullptr;      // the one workspace allocation
    size_t bytes = 0;
    void* L = nullptr;         // batch x n x n cached Cholesky factors
    void* Li = nullptr;        // batch x n x n their inverses
    void* A = nullptr;         // order x order
    void* W = nullptr;         // order x order (reduction scratch, then reflectors)
    void* tau = nullptr;       // order
    double* dv = nullptr;      // order (diagonal of T)
    double* ev = nullptr;      // order (off-diagonal of T)
    double* Z = nullptr;       // order x order (x4 with Z2, U, Qp)
    double* Z2 = nullptr;
    double* U = nullptr;
    double* Qp = nullptr;
    double* occ = nullptr;     // batch x order
    int* info = nullptr;       // [2]
    int* kwin = nullptr;       // occupied-window width found by the Fermi kernel
    Prof prof;
    HetrdWork<double> hr;
    HetrdWork<cplx> hc;
    BacktrWork<double> br;
    BacktrWork<cplx> bc;
    DcWork dc;
    DcTree tree;
    bool have_L = false;
    // adjoint scratch, allocated at the first backward call
    char* adj = nullptr;
    void* aW1 = nullptr;
    void* aW2 = nullptr;
    void* aW3 = nullptr;
    double* ascal = nullptr;
};

namespace {

struct Layout {
    size_t off = 0;
    size_t take(size_t bytes) {
        size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

bool desc_valid(const ks_plan_desc* d) {
    if (!d) return false;
    if (d->n < 1 || d->batch < 1) return false;
    if (d->dtype != KS_REAL64 && d->dtype != KS_COMPLEX128) return false;
    if (d->spin != KS_COLLINEAR && d->spin != KS_NONCOLLINEAR) return false;
    if (d->precision != KS_FP64 && d->precision != KS_MIXED) return false;
    long order = (long)d->n * (d->spin == KS_NONCOLLINEAR ? 2 : 1);
    if (order > 60000) return false;
    if (d->ld_h < order || d->ld_s < d->n) return false;
    if (d->flags & ~(uint32_t)KS_PLAN_GRAPH) return false;
    return true;
}

ks_status desc_supported(const ks_plan_desc* d) {
    if (d->spin == KS_NONCOLLINEAR && d->dtype != KS_COMPLEX128) return KS_ERR_NOT_SUPPORTED;
    if (d->precision != KS_FP64) return KS_ERR_NOT_SUPPORTED;
    if (d->batch > MAX_KW) return KS_ERR_NOT_SUPPORTED;
    return KS_OK;
}

// Lays out (or, with plan == nullptr, only measures) the workspace.
size_t layout(const ks_plan_desc* d, ks_plan* p) {
    int nsp = d->spin == KS_NONCOLLINEAR ? 2 : 1;
    size_t n = d->n, order = n * nsp, B = d->batch;
    size_t es = d->dtype == KS_COMPLEX128 ? 16 : 8;
    size_t nb = HETRD_NB, bt = BACKTR_BT;
    std::vector<int> mlo, mmid, mhi, llo, lhi, mk;
    int depth = 0;
    dc_tree_host((int)order, mlo, mmid, mhi, llo, lhi, depth, mk);
    size_t nm = mlo.size(), nl = llo.size();
    size_t maxm = depth > 0 ? ((size_t)1 << (depth - 1)) : 1;
    Layout L;
    size_t oL = L.take(B * n * n * es);
    size_t oLi = L.take(B * n * n * es);
    size_t oA = L.take(order * order * es);
    size_t oW = L.take(order * order * es);
    size_t oTau = L.take(order * es);
    size_t oD = L.take(order * 8), oE = L.take(order * 8);
    size_t oZ = L.take(order * order * 8), oZ2 = L.take(order * order * 8);
    size_t oU = L.take(order * order * 8), oQp = L.take(order * order * 8);
    size_t oOcc = L.take(B * order * 8);
    size_t oInfo = L.take(2 * sizeof(int));
    size_t oKwin = L.take(sizeof(int));
    // tridiagonalisation
    size_t oVW = L.take(order * 2 * nb * es), oWV = L.take(order * 2 * nb * es);
    size_t oX = L.take(order * es), oV = L.take(order * es), oY = L.take(order * es), oWw = L.take(order * es);
    size_t np1 = (order + 255) / 256, np3 = (order + 15) / 16;
    size_t oP1 = L.take(np1 * 8), oPQ = L.take((np1 * (1 + 2 * nb) + np3 * 2 * nb) * es);
    size_t oPS = L.take(2 * (np1 + np3) * 8);
    size_t ntl = (order + HETRD_TILE - 1) / HETRD_TILE, nchl = (ntl + HETRD_SCH - 1) / HETRD_SCH;
    size_t oPR = L.take(ntl * nchl * HETRD_TILE * es), oPC = L.take(ntl * ntl * HETRD_TILE * es);
    size_t oPQv = L.take((2 + 2 * nb) * es);
    // back-transform
    size_t oG = L.take(bt * bt * es), oT = L.take(bt * bt * es);
    size_t oW1 = L.take(bt * order * es), oW2 = L.take(bt * order * es);
    size_t pel = 16 * bt * order;  // up to 16 K-chunks of a BT x order product
    size_t oSK = L.take(pel * es);
    // divide and conquer
    size_t oDd[10];
    for (int i = 0; i < 10; ++i) oDd[i] = L.take(order * 8);
    size_t oRcs = L.take(2 * order * 8);
    size_t oDi[5];
    for (int i = 0; i < 5; ++i) oDi[i] = L.take(order * sizeof(int));
    size_t oRidx = L.take(2 * order * sizeof(int));
    size_t oKK = L.take(maxm * sizeof(int)), oNR = L.take(maxm * sizeof(int)), oRho = L.take(maxm * 8);
    size_t oT1 = L.take((nm + 1) * sizeof(int)), oT2 = L.take((nm + 1) * sizeof(int));
    size_t oT3 = L.take((nm + 1) * sizeof(int));
    size_t oL1 = L.take(nl * sizeof(int)), oL2 = L.take(nl * sizeof(int));
    size_t total = L.off;
    if (!p) return total;
    char* b = p->base;
    p->L = b + oL;
    p->Li = b + oLi;
    p->A = b + oA;
    p->W = b + oW;
    p->tau = b + oTau;
    p->dv = (double*)(b + oD);
    p->ev = (double*)(b + oE);
    p->Z = (double*)(b + oZ);
    p->Z2 = (double*)(b + oZ2);
    p->U = (double*)(b + oU);
    p->Qp = (double*)(b + oQp);
    p->occ = (double*)(b + oOcc);
    p->info = (int*)(b + oInfo);
    p->kwin = (int*)(b + oKwin);
    auto setH = [&](auto& h, auto* tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        h.VW = (T*)(b + oVW);
        h.WV = (T*)(b + oWV);
        h.x = (T*)(b + oX);
        h.v = (T*)(b + oV);
        h.y = (T*)(b + oY);
        h.w = (T*)(b + oWw);
        h.part1 = (double*)(b + oP1);
        h.partPQ = (T*)(b + oPQ);
        h.partS = (double*)(b + oPS);
        h.prow = (T*)(b + oPR);
        h.pcol = (T*)(b + oPC);
        h.pq = (T*)(b + oPQv);
        h.prof = &p->prof;
    };
    setH(p->hr, (double*)nullptr);
    setH(p->hc, (cplx*)nullptr);
    auto setB = [&](auto& w, auto* tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        w.G = (T*)(b + oG);
        w.Tf = (T*)(b + oT);
        w.W1 = (T*)(b + oW1);
        w.W2 = (T*)(b + oW2);
        w.P = (T*)(b + oSK);
        w.pelems = (long)pel;
    };
    setB(p->br, (double*)nullptr);
    setB(p->bc, (cplx*)nullptr);
    DcWork& w = p->dc;
    w.dw = (double*)(b + oDd[0]);
    w.ds = (double*)(b + oDd[1]);
    w.zs = (double*)(b + oDd[2]);
    w.dfval = (double*)(b + oDd[3]);
    w.dnd = (double*)(b + oDd[4]);
    w.znd = (double*)(b + oDd[5]);
    w.tau = (double*)(b + oDd[6]);
    w.zhat = (double*)(b + oDd[7]);
    w.cinv = (double*)(b + oDd[8]);
    w.fval = (double*)(b + oDd[9]);
    w.rot_cs = (double*)(b + oRcs);
    w.perm = (int*)(b + oDi[0]);
    w.ndl = (int*)(b + oDi[1]);
    w.dfl = (int*)(b + oDi[2]);
    w.orig = (int*)(b + oDi[3]);
    w.fsrc = (int*)(b + oDi[4]);
    w.rot_idx = (int*)(b + oRidx);
    w.kk = (int*)(b + oKK);
    w.nrot = (int*)(b + oNR);
    w.rho = (double*)(b + oRho);
    DcTree& t = p->tree;
    t.n = (int)order;
    t.depth = depth;
    t.nleaf = (int)nl;
    t.nmerge_total = (int)nm;
    t.max_k0 = mk;
    t.d_mlo = (int*)(b + oT1);
    t.d_mmid = (int*)(b + oT2);
    t.d_mhi = (int*)(b + oT3);
    t.d_mid_all = t.d_mmid;
    t.d_leaf_lo = (int*)(b + oL1);
    t.d_leaf_hi = (int*)(b + oL2);
    // upload the tree (small, synchronous, at plan creation only)
    if (nm) {
        (void)hipMemcpy(t.d_mlo, mlo.data(), nm * sizeof(int), hipMemcpyHostToDevice);
        (void)hipMemcpy(t.d_mmid, mmid.data(), nm * sizeof(int), hipMemcpyHostToDevice);
        (void)hipMemcpy(t.d_mhi, mhi.data(), nm * sizeof(int), hipMemcpyHostToDevice);
    }
    (void)hipMemcpy(t.d_leaf_lo, llo.data(), nl * sizeof(int), hipMemcpyHostToDevice);
    (void)hipMemcpy(t.d_leaf_hi, lhi.data(), nl * sizeof(int), hipMemcpyHostToDevice);
    return total;
}

bool range_ok(const ks_plan* p, int il, int iu) { return il >= 1 && il <= iu && iu <= p->order; }

KWeights make_weights(const ks_plan* p, const double* kw) {
    KWeights w;
    for (int i = 0; i < MAX_KW; ++i) w.w[i] = 0.0;
    for (int b = 0; b < p->d.batch; ++b) w.w[b] = kw ? kw[b] : 1.0 / p->d.batch;
    return w;
}

template <typename T>
ks_status gevd_impl(ks_plan* p, const T* H, const T* S, double* eps, T* C, int il, int iu,
                    uint32_t flags) {
    hipStream_t s = p->s;
    int n = p->d.n, nsp = p->nsp, order = p->order, B = p->d.batch;
    int ldh = p->d.ld_h, lds = p->d.ld_s;
    T* L = (T*)p->L;
    T* A = (T*)p->A;
    T* W = (T*)p->W;
    T* tau = (T*)p->tau;
    HetrdWork<T>& hw = *reinterpret_cast<HetrdWork<T>*>(is_cplx<T>::value ? (void*)&p->hc : (void*)&p->hr);
    BacktrWork<T>& bw = *reinterpret_cast<BacktrWork<T>*>(is_cplx<T>::value ? (void*)&p->bc : (void*)&p->br);
    Prof& pf = p->prof;
    T* Li = (T*)p->Li;
    if (!(flags & KS_REUSE_S)) {
        hipEvent_t e = pf.begin();
        herm_complete<T>(s, n, S, lds, (long)n * lds, L, n, (long)n * n, B, p->info);
        potrf<T>(s, n, L, n, (long)n * n, B, p->info);
        tri_inverse<T>(s, n, L, n, (long)n * n, Li, (long)n * n, B);
        pf.end(KS_PHASE_CHOLESKY, e);
        p->have_L = true;
    }
    int ncols = iu - il + 1;
    for (int b = 0; b < B; ++b) {
        const T* Hb = H + (long)b * order * ldh;
        T* Cb = C + (long)b * order * ldh;
        const T* Lib = Li + (long)b * n * n;
        hipEvent_t e = pf.begin();
        reduce_to_standard<T>(s, n, nsp, Hb, ldh, Lib, n, A, W, p->info);
        pf.end(KS_PHASE_REDUCE, e);
        e = pf.begin();
        hetrd<T>(s, order, A, order, p->dv, p->ev, tau, W, hw);
        pf.end(KS_PHASE_TRIDIAG, e);
        e = pf.begin();
        stedc(s, p->tree, p->dv, p->ev, eps + (long)b * order, p->Z, p->Z2, p->U, p->Qp, p->dc, p->info);
        pf.end(KS_PHASE_DC, e);
        e = pf.begin();
        // X = Q Z[:, il-1 : iu] in A (order x ncols), then C_sigma = Linv^H X_sigma per spin block
        load_z<T>(s, order, ncols, p->Z, il - 1, A, ncols);
        backtransform_q<T>(s, order, W, tau, ncols, A, ncols, bw);
        gemm<T>(s, OP_C, OP_N, n, ncols, n, 1.0, Lib, n, 0, A, ncols, (long)n * ncols, 0.0, Cb, ldh,
                (long)n * ldh, nsp, nullptr, 0, UPLO_FULL, nullptr, TRI_A_UPPER);
        pf.end(KS_PHASE_BACKTR, e);
    }
    if (hipPeekAtLastError() != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}

}  // namespace

extern "C" {

const char* ks_status_string(ks_status st) {
    switch (st) {
        case KS_OK: return "success";
        case KS_ERR_INVALID_ARG: return "invalid argument";
        case KS_ERR_NOT_POSDEF: return "overlap matrix S is not positive definite";
        case KS_ERR_NO_CONVERGENCE: return "iteration did not converge";
        case KS_ERR_ELECTRON_COUNT: return "electron count out of range";
        case KS_ERR_WINDOW: return "occupied states outside the computed eigenvector window";
        case KS_ERR_NONFINITE: return "non-finite value in H or S";
        case KS_ERR_ALLOC: return "device workspace does not fit";
        case KS_ERR_HIP: return "HIP runtime error";
        case KS_ERR_NOT_SUPPORTED: return "unsupported combination";
    }
    return "unknown status";
}

uint64_t ks_plan_workspace_bytes(const ks_plan_desc* d) {
    if (!desc_valid(d)) return 0;
    return (uint64_t)layout(d, nullptr);
}

ks_status ks_plan_create(const ks_plan_desc* d, ks_plan** out) {
    if (!out) return KS_ERR_INVALID_ARG;
    *out = nullptr;
    if (!desc_valid(d)) return KS_ERR_INVALID_ARG;
    ks_status sup = desc_supported(d);
    if (sup != KS_OK) return sup;
    size_t bytes = layout(d, nullptr);
    size_t freeb = 0, totb = 0;
    if (hipMemGetInfo(&freeb, &totb) != hipSuccess) return KS_ERR_HIP;
    if (bytes > freeb) return KS_ERR_ALLOC;
    ks_plan* p = new (std::nothrow) ks_plan();
    if (!p) return KS_ERR_ALLOC;
    p->d = *d;
    p->nsp = d->spin == KS_NONCOLLINEAR ? 2 : 1;
    p->order = d->n * p->nsp;
    p->is_c = d->dtype == KS_COMPLEX128;
    p->es = p->is_c ? 16 : 8;
    p->s = (hipStream_t)d->stream;
    p->prof.s = p->s;
    if (hipMalloc((void**)&p->base, bytes) != hipSuccess) {
        delete p;
        return KS_ERR_ALLOC;
    }
    p->bytes = bytes;
    layout(d, p);
    if (hipMemset(p->info, 0, 2 * sizeof(int)) != hipSuccess) {
        (void)hipFree(p->base);
        delete p;
        return KS_ERR_HIP;
    }
    *out = p;
    return KS_OK;
}

void ks_plan_destroy(ks_plan* p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->s);
    if (p->base) (void)hipFree(p->base);
    if (p->adj) (void)hipFree(p->adj);
    delete p;
}

ks_status ks_gevd(ks_plan* p, const void* H, const void* S, double* eps, void* C, int32_t il,
                  int32_t iu, uint32_t flags) {
    if (!p || !H || !eps || !C) return KS_ERR_INVALID_ARG;
    if (flags & ~(uint32_t)KS_REUSE_S) return KS_ERR_INVALID_ARG;
    if (!(flags & KS_REUSE_S) && !S) return KS_ERR_INVALID_ARG;
    if ((flags & KS_REUSE_S) && !p->have_L) return KS_ERR_INVALID_ARG;
    if (!range_ok(p, il, iu)) return KS_ERR_INVALID_ARG;
    if (p->is_c)
        return gevd_impl<cplx>(p, (const cplx*)H, (const cplx*)S, eps, (cplx*)C, il, iu, flags);
    return gevd_impl<double>(p, (const double*)H, (const double*)S, eps, (double*)C, il, iu, flags);
}

ks_status ks_density(ks_plan* p, const double* eps, const void* C, int32_t il, int32_t iu,
                     double ne, double kT, const double* kweights, void* rho, double* mu,
                     double* eband, double* occ) {
    if (!p || !eps || !C || !rho || !mu || !eband) return KS_ERR_INVALID_ARG;
    if (!range_ok(p, il, iu)) return KS_ERR_INVALID_ARG;
    if (!(kT > 0.0) || !isfinite(kT)) return KS_ERR_INVALID_ARG;
    double g = p->nsp == 2 ? 1.0 : 2.0;
    if (!(ne > 0.0) || !(ne <= g * p->order) || !isfinite(ne)) return KS_ERR_ELECTRON_COUNT;
    if (kweights) {
        for (int b = 0; b < p->d.batch; ++b)
            if (!(kweights[b] >= 0.0) || !isfinite(kweights[b])) return KS_ERR_INVALID_ARG;
    }
    KWeights kw = make_weights(p, kweights);
    double* f = occ ? occ : p->occ;
    hipStream_t s = p->s;
    int order = p->order, ldh = p->d.ld_h, ncols = iu - il + 1;
    hipEvent_t e = p->prof.begin();
    fermi(s, p->d.batch, order, eps, kw, g, ne, kT, il, iu, f, mu, eband, p->kwin, p->info);
    long mat = (long)order * ldh;
    // rho = C diag(f) C^H over the window columns that carry occupation (count on the device)
    if (p->is_c)
        gemm<cplx>(s, OP_N, OP_C, order, order, ncols, 1.0, (const cplx*)C, ldh, mat, (const cplx*)C, ldh,
                   mat, 0.0, (cplx*)rho, ldh, mat, p->d.batch, f + il - 1, order, UPLO_FULL, p->kwin);
    else
        gemm<double>(s, OP_N, OP_T, order, order, ncols, 1.0, (const double*)C, ldh, mat,
                     (const double*)C, ldh, mat, 0.0, (double*)rho, ldh, mat, p->d.batch, f + il - 1,
                     order, UPLO_FULL, p->kwin);
    p->prof.end(KS_PHASE_DENSITY, e);
    if (hipPeekAtLastError() != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}

ks_status ks_density_backward(ks_plan* p, const double* eps, const void* C, const double* mu,
                              const double* occ, double kT, const void* grad_rho,
                              const double* grad_eband, void* grad_H, void* grad_S) {
    if (!p || !eps || !C || !mu || !occ || !grad_H || !grad_S) return KS_ERR_INVALID_ARG;
    if (!(kT > 0.0) || !isfinite(kT)) return KS_ERR_INVALID_ARG;
    int order = p->order, B = p->d.batch;
    if (!p->adj) {
        size_t m = (size_t)order * order * p->es;
        size_t bytes = 3 * ((m + 255) & ~(size_t)255) + ((2 + (size_t)B * order) * 8 + 255);
        if (hipMalloc((void**)&p->adj, bytes) != hipSuccess) {
            p->adj = nullptr;
            return KS_ERR_ALLOC;
        }
        size_t mm = (m + 255) & ~(size_t)255;
        p->aW1 = p->adj;
        p->aW2 = p->adj + mm;
        p->aW3 = p->adj + 2 * mm;
        p->ascal = (double*)(p->adj + 3 * mm);
    }
    double g = p->nsp == 2 ? 1.0 : 2.0;
    KWeights kw = make_weights(p, nullptr);
    hipEvent_t e = p->prof.begin();
    if (p->is_c)
        density_backward<cplx>(p->s, p->d.n, p->nsp, B, eps, (const cplx*)C, p->d.ld_h, mu, kT, g, kw,
                               (const cplx*)grad_rho, grad_eband, (cplx*)grad_H, (cplx*)grad_S, p->d.ld_s,
                               (cplx*)p->aW1, (cplx*)p->aW2, (cplx*)p->aW3, p->ascal);
    else
        density_backward<double>(p->s, p->d.n, p->nsp, B, eps, (const double*)C, p->d.ld_h, mu, kT, g,
                                 kw, (const double*)grad_rho, grad_eband, (double*)grad_H,
                                 (double*)grad_S, p->d.ld_s, (double*)p->aW1, (double*)p->aW2,
                                 (double*)p->aW3, p->ascal);
    p->prof.end(KS_PHASE_ADJOINT, e);
    if (hipPeekAtLastError() != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}

ks_status ks_plan_set_profiling(ks_plan* p, int32_t enable, int32_t stride) {
    if (!p || (enable && stride < 1)) return KS_ERR_INVALID_ARG;
    p->prof.on = enable != 0;
    p->prof.stride = enable ? stride : 1;
    p->prof.counter = 0;
    return KS_OK;
}

ks_status ks_plan_get_profile(ks_plan* p, ks_profile* out) {
    if (!p || !out) return KS_ERR_INVALID_ARG;
    memset(out, 0, sizeof(*out));
    if (hipStreamSynchronize(p->s) != hipSuccess) return KS_ERR_HIP;
    for (auto& r : p->prof.recs) {
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return KS_ERR_HIP;
        if (r.tag == PROF_HEMV) {
            out->hemv_ms += ms;
            out->hemv_launches += 1;
            out->hemv_bytes += r.bytes;
        } else if (r.tag >= 0 && r.tag < KS_NPHASE) {
            out->phase_ms[r.tag] += ms;
            out->phase_calls[r.tag] += 1;
        }
        p->prof.pool.push_back(r.a);
        p->prof.pool.push_back(r.b);
    }
    p->prof.recs.clear();
    return KS_OK;
}

ks_status ks_plan_get_info(ks_plan* p, int32_t* info) {
    if (!p || !info) return KS_ERR_INVALID_ARG;
    if (hipStreamSynchronize(p->s) != hipSuccess) return KS_ERR_HIP;
    int h[2] = {0, 0};
    if (hipMemcpy(h, p->info, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return KS_ERR_HIP;
    int z[2] = {0, 0};
    if (hipMemcpy(p->info, z, sizeof(z), hipMemcpyHostToDevice) != hipSuccess) return KS_ERR_HIP;
    if (h[0] == 0) {
        *info = 0;
        return KS_OK;
    }
    *info = (h[0] == KS_ERR_NOT_POSDEF) ? h[1] : -h[0];
    return (ks_status)h[0];
}

}  // extern "C"

// Internal stage drivers used by the test hooks (ks_testhooks.hip).
void ks_internal_stedc(ks_plan* p, const double* d, const double* e, double* lam, double* Z) {
    stedc(p->s, p->tree, d, e, lam, Z, p->Z2, p->U, p->Qp, p->dc, p->info);
}

void ks_internal_hetrd(ks_plan* p, void* A, double* d, double* e, const double* X, int ncols, void* Y) {
    int n = p->order;
    if (p->is_c) {
        hetrd<cplx>(p->s, n, (cplx*)A, n, d, e, (cplx*)p->tau, (cplx*)p->W, p->hc);
        load_z<cplx>(p->s, n, ncols, X, 0, (cplx*)Y, ncols);
        backtransform_q<cplx>(p->s, n, (cplx*)p->W, (cplx*)p->tau, ncols, (cplx*)Y, ncols, p->bc);
    } else {
        hetrd<double>(p->s, n, (double*)A, n, d, e, (double*)p->tau, (double*)p->W, p->hr);
        load_z<double>(p->s, n, ncols, X, 0, (double*)Y, ncols);
        backtransform_q<double>(p->s, n, (double*)p->W, (double*)p->tau, ncols, (double*)Y, ncols, p->br);
    }
}
