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
    // batches of two or more: a second stream for half of the tridiagonalisation
    hipStream_t side = nullptr;
    hipEvent_t side_fork = nullptr, side_join = nullptr;
    char* base = nullptr;      // the one workspace allocation
    size_t bytes = 0;
    void* L = nullptr;         // batch x n x n cached Cholesky factors
    void* Li = nullptr;        // batch x n x n their inverses
    // per matrix of the batch, consecutive:
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
    double* fe = nullptr;      // batch x order: f eps, the energy-density weights
    int* info = nullptr;       // [2]
    int* kwin = nullptr;       // occupied-window width found by the Fermi kernel
    Prof prof;
    HetrdWork<double> hr;
    HetrdWork<cplx> hc;
    BacktrWork<double> br;
    BacktrWork<cplx> bc;
    BandWork<double> bandr;    // KS_PLAN_TWOSTAGE buffers
    BandWork<cplx> bandc;
    DcWork dc;
    DcTree tree;
    bool have_L = false;
    // KS_PLAN_GRAPH: the launch sequence of the last ks_gevd argument set,
    // captured from the plan stream once and replayed while the arguments repeat
    struct GraphKey {
        const void* H;
        const void* S;
        double* eps;
        void* C;
        int il, iu;
        uint32_t flags;
        bool operator==(const GraphKey& o) const {
            return H == o.H && S == o.S && eps == o.eps && C == o.C && il == o.il && iu == o.iu &&
                   flags == o.flags;
        }
    };
    GraphKey gkey{};
    ks_tuning tuning{};
    // KS_MIXED: FP32 copies for the tridiagonalisation and back-transforms, FP64
    // refinement buffers (all per matrix of the batch) and the Rayleigh-Ritz plan
    void* A32 = nullptr;       // order x order   reduced matrix in FP32
    void* W32 = nullptr;       // order x order   reflectors in FP32
    void* Tall32 = nullptr;    // compact-WY factors of the back-transform in FP32
    float* Z32 = nullptr;      // order x order   tridiagonal eigenvectors in FP32
    void* mY = nullptr;        // order x order   A X, then X y
    void* mR = nullptr;        // order x order   residual, then the Ritz vectors y
    void* mG = nullptr;        // order x order   X^H A X
    void* mB = nullptr;        // order x order   X^H X
    void* mP = nullptr;        // order x order   FP32 work
    void* mP2 = nullptr;       // order x order   FP32 work
    double* theta = nullptr;   // order           refined window values
    void* mS = nullptr;        // order x order   M x M scratch of the subspace refinement
    void* mS2 = nullptr;       // order x order   M x M scratch of the subspace refinement
    int* mI = nullptr;         // 3 x order       cluster starts, sizes and ranks of the window
    ks_plan* rr = nullptr;     // unused (kept null)
    // KS_PLAN_LOWDIN: V = U s^-1/2 lives in L (batch x n x n); sev holds the
    // eigenvalues s of S; spinor plans solve the order-n eigenproblem of S on
    // the collinear plan ov (collinear plans use their own buffers)
    double* sev = nullptr;     // batch x n
    int* nkeep = nullptr;      // batch: eigenvectors of S kept
    double* fpart = nullptr;   // batch x row blocks: |H'|_F^2 partials
    double ov_tau = 0.0;       // cutoff tau of ks_plan_set_overlap_cutoff
    double v_tau = 0.0;        // the cutoff the V in use was formed with
    ks_plan* ov = nullptr;
    int mixed_sweeps = 1;
    // k weights of the last ks_density call (uniform until then); the adjoint's
    // chemical-potential and band-energy terms use the same weights
    KWeights kw_last{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    long graph_captures = 0, graph_replays = 0;
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
    if (d->flags & ~(uint32_t)(KS_PLAN_GRAPH | KS_PLAN_AUTOTUNE | KS_PLAN_LOWDIN | KS_PLAN_TWOSTAGE |
                               KS_PLAN_REAL_OVERLAP))
        return false;
    return true;
}

ks_status desc_supported(const ks_plan_desc* d) {
    if ((d->flags & KS_PLAN_GRAPH) && d->stream == nullptr) return KS_ERR_NOT_SUPPORTED;  // no capture there
    if (d->spin == KS_NONCOLLINEAR && d->dtype != KS_COMPLEX128) return KS_ERR_NOT_SUPPORTED;
    if (d->batch > MAX_KW) return KS_ERR_NOT_SUPPORTED;
    if ((d->flags & KS_PLAN_LOWDIN) && d->precision == KS_MIXED) return KS_ERR_NOT_SUPPORTED;
    if ((d->flags & KS_PLAN_TWOSTAGE) && d->precision == KS_MIXED) return KS_ERR_NOT_SUPPORTED;
    return KS_OK;
}

// The order-n collinear plan on which a spinor KS_PLAN_LOWDIN plan solves the
// eigenproblem of S (same batch, type, stream and tuning request).
ks_plan_desc lowdin_overlap_desc(const ks_plan_desc* d) {
    ks_plan_desc c{};
    c.n = d->n;
    c.batch = d->batch;
    c.dtype = d->dtype;
    c.spin = KS_COLLINEAR;
    c.precision = KS_FP64;
    c.ld_h = d->n;
    c.ld_s = d->n;
    c.stream = d->stream;
    c.flags = d->flags & KS_PLAN_AUTOTUNE;
    return c;
}

// Compact-WY blocks of bt reflectors (128 or 256; the buffers hold 256).
template <typename T>
void set_backtr_block(BacktrWork<T>& w, int order, int bt) {
    const long nblk = order > 1 ? (order - 1 + bt - 1) / bt : 1;
    w.bt = bt;
    w.sTall = nblk * bt * bt;
}

// Tear tree with leaves of at most `leaf` rows (DC_LEAF_MIN .. DC_LEAF; the
// arrays hold the tree of the smallest), uploaded synchronously: at plan
// creation and from ks_plan_set_tuning only.
ks_status set_dc_leaf(ks_plan* p, int leaf) {
    std::vector<int> mlo, mmid, mhi, llo, lhi, mk;
    int depth = 0;
    dc_tree_host(p->order, leaf, mlo, mmid, mhi, llo, lhi, depth, mk);
    DcTree& t = p->tree;
    t.depth = depth;
    t.nleaf = (int)llo.size();
    t.nmerge_total = (int)mlo.size();
    t.max_k0 = mk;
    const size_t nm = mlo.size(), nl = llo.size();
    if (nm && (hipMemcpy(t.d_mlo, mlo.data(), nm * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
               hipMemcpy(t.d_mmid, mmid.data(), nm * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
               hipMemcpy(t.d_mhi, mhi.data(), nm * sizeof(int), hipMemcpyHostToDevice) != hipSuccess))
        return KS_ERR_HIP;
    if (hipMemcpy(t.d_leaf_lo, llo.data(), nl * sizeof(int), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(t.d_leaf_hi, lhi.data(), nl * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
        return KS_ERR_HIP;
    p->tuning.dc_leaf = leaf;
    return KS_OK;
}

// Lays out (or, with plan == nullptr, only measures) the workspace.
size_t layout(const ks_plan_desc* d, ks_plan* p) {
    int nsp = d->spin == KS_NONCOLLINEAR ? 2 : 1;
    size_t n = d->n, order = n * nsp, B = d->batch;
    size_t es = d->dtype == KS_COMPLEX128 ? 16 : 8;
    // back-transform buffers for the largest block the autotuner may choose,
    // and divide-and-conquer tree arrays for the smallest leaf
    size_t nb = HETRD_NB, bt = BACKTR_BT;
    std::vector<int> mlo, mmid, mhi, llo, lhi, mk;
    int depth = 0;
    dc_tree_host((int)order, DC_LEAF_MIN, mlo, mmid, mhi, llo, lhi, depth, mk);
    size_t nm = mlo.size(), nl = llo.size();
    size_t maxm = depth > 0 ? ((size_t)1 << (depth - 1)) : 1;
    Layout L;
    size_t oL = L.take(B * n * n * es);
    size_t oLi = L.take(B * n * n * es);
    size_t oA = L.take(B * order * order * es);
    size_t oW = L.take(B * order * order * es);
    size_t oTau = L.take(B * order * es);
    size_t oD = L.take(B * order * 8), oE = L.take(B * order * 8);
    size_t oZ = L.take(B * order * order * 8), oZ2 = L.take(B * order * order * 8);
    size_t oU = L.take(B * order * order * 8), oQp = L.take(B * order * order * 8);
    size_t oOcc = L.take(B * order * 8);
    size_t oFe = L.take(B * order * 8);  // occupation x eigenvalue weights of the energy-density matrix
    size_t oInfo = L.take(2 * sizeof(int));
    size_t oKwin = L.take(sizeof(int));
    // tridiagonalisation (per matrix of the batch)
    size_t ntl = (order + HETRD_TILE - 1) / HETRD_TILE, nchl = (ntl + HETRD_SCH_MIN - 1) / HETRD_SCH_MIN;
    size_t hVW = order * 2 * nb, hX = order, hPQ = ntl * (1 + 2 * nb), hPR = ntl * nchl * HETRD_TILE;
    size_t hPC = ntl * ntl * HETRD_TILE, hPV = ntl * nchl, hPQv = 5 + 2 * nb;
    size_t oVW = L.take(B * hVW * es), oWV = L.take(B * hVW * es);
    size_t oX = L.take(B * hX * es);
    size_t oPQ = L.take(2 * B * hPQ * es);  // one partial buffer per column parity
    size_t oPR = L.take(B * hPR * es), oPC = L.take(B * hPC * es);
    size_t oPV = L.take(B * hPV * 8);
    size_t oPQv = L.take(B * hPQv * es);
    // back-transform
    const size_t nblk_bt = order > 1 ? (order - 1 + bt - 1) / bt : 1;
    size_t oG = L.take(B * bt * bt * es), oT = L.take(B * nblk_bt * bt * bt * es);
    size_t oW1 = L.take(B * bt * order * es), oW2 = L.take(B * bt * order * es);
    // split-K partial products of a BT x order product: as many K-chunks as the
    // GEMM cuts K = order into (at most max(16, order / 256)), for every matrix
    size_t pel = std::max<size_t>(16, (order + 255) / 256) * bt * order * B;
    size_t oSK = L.take(pel * es);
    // divide and conquer (per matrix of the batch)
    size_t oDd[10];
    for (int i = 0; i < 10; ++i) oDd[i] = L.take(B * order * 8);
    size_t oRcs = L.take(B * 2 * order * 8);
    size_t oDi[6];
    for (int i = 0; i < 6; ++i) oDi[i] = L.take(B * order * sizeof(int));
    size_t oRidx = L.take(B * 2 * order * sizeof(int));
    size_t oKK = L.take(B * maxm * sizeof(int)), oNR = L.take(B * maxm * sizeof(int));
    size_t oKK1 = L.take(B * maxm * sizeof(int));
    size_t oRho = L.take(B * maxm * 8);
    size_t oT1 = L.take((nm + 1) * sizeof(int)), oT2 = L.take((nm + 1) * sizeof(int));
    size_t oT3 = L.take((nm + 1) * sizeof(int));
    size_t oL1 = L.take(nl * sizeof(int)), oL2 = L.take(nl * sizeof(int));
    // mixed precision (only when asked for)
    const bool mixed = d->precision == KS_MIXED;
    const size_t es32 = es / 2, mat = order * order;
    size_t oA32 = 0, oW32 = 0, oT32 = 0, oZ32 = 0, oMY = 0, oMR = 0, oMG = 0, oMB = 0, oMP = 0, oMP2 = 0;
    size_t oTh = 0, oVWl = 0, oWVl = 0, oMS = 0, oMS2 = 0, oMI = 0;
    if (mixed) {
        oA32 = L.take(B * mat * es32);
        oW32 = L.take(B * mat * es32);
        oT32 = L.take(B * nblk_bt * bt * bt * es32);
        oZ32 = L.take(B * mat * 4);
        oMY = L.take(B * mat * es);
        oMR = L.take(B * mat * es);
        oMG = L.take(B * mat * es);
        oMB = L.take(B * mat * es);
        oMP = L.take(B * mat * es32);
        oMP2 = L.take(B * mat * es32);
        oTh = L.take(B * order * 8);
        oMS = L.take(B * mat * es);
        oMS2 = L.take(B * mat * es);
        oMI = L.take(3 * B * order * sizeof(int));
        oVWl = L.take(B * hVW * es32);
        oWVl = L.take(B * hVW * es32);
    }
    // two-stage reduction (only when asked for)
    const bool two = (d->flags & KS_PLAN_TWOSTAGE) != 0;
    const size_t tm = order > 1 ? (size_t)s2_steps((int)order, 0) : 1;       // steps of the longest sweep
    const size_t q2nb = (size_t)q2_nb(es == 16);                           // sweeps per group
    const size_t jg = order > 1 ? (order - 1 + q2nb - 1) / q2nb : 1;           // groups of sweeps
    const size_t prow = (size_t)panel_rows(es == 16);
    const size_t pmax = (order + prow - 1) / prow;
    const size_t npan = (order + KB - 1) / KB;
    constexpr size_t GMAX = 64;  // bulge-chasing workgroups per matrix
    size_t oBX = 0, oB3 = 0, oBT = 0, oBM = 0, oBN = 0, oRec = 0, oCnt = 0, oGp = 0, oAb = 0, oVpk = 0, oTaupk = 0;
    size_t oQ2p = 0;
    if (two) {
        oBX = L.take(B * order * KB * es);
        oB3 = L.take(B * order * 3 * KB * es);
        oBT = L.take(B * KB * KB * es);
        oBM = L.take(B * KB * KB * es);
        oBN = L.take(B * KB * KB * es);
        oRec = L.take(B * 2 * pmax * 2 * KB * es);
        oCnt = L.take(B * npan * sizeof(int));
        oGp = L.take(B * GMAX * sizeof(int));
        oAb = L.take(sizeof(int));
        oVpk = L.take(B * jg * tm * q2nb * KB * es);
        oTaupk = L.take(B * jg * tm * q2nb * es);
        const size_t q2w = (size_t)q2_passes(es == 16);
        oQ2p = L.take(B * ((jg + q2w - 1) / q2w) * ((order + 63) / 64) * sizeof(int));
    }
    const bool lw = (d->flags & KS_PLAN_LOWDIN) != 0;
    const size_t oSev = lw ? L.take(B * n * 8) : 0;
    const size_t oNkeep = lw ? L.take(B * sizeof(int)) : 0;
    const size_t oFpart = lw ? L.take(B * ((order + 63) / 64) * 8) : 0;
    size_t total = L.off;
    if (!p) return total;
    char* b = p->base;
    p->L = b + oL;
    if (lw) {
        p->sev = (double*)(b + oSev);
        p->nkeep = (int*)(b + oNkeep);
        p->fpart = (double*)(b + oFpart);
    }
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
    p->fe = (double*)(b + oFe);
    p->info = (int*)(b + oInfo);
    p->kwin = (int*)(b + oKwin);
    auto setH = [&](auto& h, auto* tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        h.VW = (T*)(b + oVW);
        h.WV = (T*)(b + oWV);
        h.x = (T*)(b + oX);
        h.partPQ = (T*)(b + oPQ);
        h.prow = (T*)(b + oPR);
        h.pcol = (T*)(b + oPC);
        h.pvav = (double*)(b + oPV);
        h.pq = (T*)(b + oPQv);
        h.sbuf = (long)(B * hPQ);
        h.sVW = (long)hVW;
        h.sx = (long)hX;
        h.spart = (long)hPQ;
        h.sprow = (long)hPR;
        h.spcol = (long)hPC;
        h.spvav = (long)hPV;
        h.spq = (long)hPQv;
        h.VWlo = mixed ? (void*)(b + oVWl) : nullptr;
        h.WVlo = mixed ? (void*)(b + oWVl) : nullptr;
        h.prof = &p->prof;
    };
    if (mixed) {
        p->A32 = b + oA32;
        p->W32 = b + oW32;
        p->Tall32 = b + oT32;
        p->Z32 = (float*)(b + oZ32);
        p->mY = b + oMY;
        p->mR = b + oMR;
        p->mG = b + oMG;
        p->mB = b + oMB;
        p->mP = b + oMP;
        p->mP2 = b + oMP2;
        p->theta = (double*)(b + oTh);
        p->mS = b + oMS;
        p->mS2 = b + oMS2;
        p->mI = (int*)(b + oMI);
    }
    setH(p->hr, (double*)nullptr);
    setH(p->hc, (cplx*)nullptr);
    auto setB = [&](auto& w, auto* tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        w.G = (T*)(b + oG);
        w.Tall = (T*)(b + oT);
        set_backtr_block(w, (int)order, backtr_block((int)order));
        w.W1 = (T*)(b + oW1);
        w.W2 = (T*)(b + oW2);
        w.P = (T*)(b + oSK);
        w.pelems = (long)pel;
    };
    setB(p->br, (double*)nullptr);
    setB(p->bc, (cplx*)nullptr);
    auto setBand = [&](auto& w, auto* tag) {
        using T = std::remove_pointer_t<decltype(tag)>;
        if (!two) return;
        w.X = (T*)(b + oBX);
        w.sX = (long)(order * KB);
        w.buf3 = (T*)(b + oB3);
        w.sbuf = (long)(order * 3 * KB);
        w.Tf = (T*)(b + oBT);
        w.sTf = (long)(KB * KB);
        w.M = (T*)(b + oBM);
        w.N = (T*)(b + oBN);
        w.rec = (T*)(b + oRec);
        w.srec = (long)(2 * pmax * 2 * KB);
        w.cnt = (int*)(b + oCnt);
        w.scnt = (long)npan;
        w.gprog = (int*)(b + oGp);
        w.sgp = (long)GMAX;
        w.abort_ = (int*)(b + oAb);
        w.Vpk = (T*)(b + oVpk);
        w.sVpk = (long)(jg * tm * q2nb * KB);
        w.taupk = (T*)(b + oTaupk);
        w.staupk = (long)(jg * tm * q2nb);
        w.q2prog = (int*)(b + oQ2p);
        w.P = (T*)(b + oSK);
        w.pelems = (long)pel;
    };
    setBand(p->bandr, (double*)nullptr);
    setBand(p->bandc, (cplx*)nullptr);
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
    w.gpos = (int*)(b + oDi[5]);
    w.rot_idx = (int*)(b + oRidx);
    w.kk = (int*)(b + oKK);
    w.kk1 = (int*)(b + oKK1);
    w.nrot = (int*)(b + oNR);
    w.rho = (double*)(b + oRho);
    DcTree& t = p->tree;
    t.n = (int)order;
    t.d_mlo = (int*)(b + oT1);
    t.d_mmid = (int*)(b + oT2);
    t.d_mhi = (int*)(b + oT3);
    t.d_mid_all = t.d_mmid;
    t.d_leaf_lo = (int*)(b + oL1);
    t.d_leaf_hi = (int*)(b + oL2);
    set_dc_leaf(p, DC_LEAF);
    return total;
}

bool range_ok(const ks_plan* p, int il, int iu) { return il >= 1 && il <= iu && iu <= p->order; }

void graph_release(ks_plan* p) {
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->gexec = nullptr;
    p->graph = nullptr;
}

KWeights make_weights(const ks_plan* p, const double* kw) {
    KWeights w;
    for (int i = 0; i < MAX_KW; ++i) w.w[i] = 0.0;
    for (int b = 0; b < p->d.batch; ++b) w.w[b] = kw ? kw[b] : 1.0 / p->d.batch;
    return w;
}

template <typename T>
BacktrWork<typename Lo<T>::type> lo_view(const BacktrWork<T>& w) {
    using L = typename Lo<T>::type;
    BacktrWork<L> v;
    v.G = (L*)w.G;
    v.Tall = nullptr;  // the FP32 factors have a buffer of their own
    v.sTall = w.sTall;
    v.bt = w.bt;
    v.W1 = (L*)w.W1;
    v.W2 = (L*)w.W2;
    v.P = (L*)w.P;
    v.pelems = w.pelems;
    return v;
}

// C_sigma = Linv^H X_sigma per spin block for every matrix of the batch
// (X: order x ncols, stride sX).
template <typename T>
void apply_linv_h(ks_plan* p, const T* Li, const T* X, long sX, int ncols, T* C) {
    const int n = p->d.n, nsp = p->nsp, B = p->d.batch, ldh = p->d.ld_h, order = p->order;
    const long sL = (long)n * n, sH = (long)order * ldh;
    if constexpr (is_cplx<T>::value) {
        if (p->d.flags & KS_PLAN_REAL_OVERLAP) {
            // real Linv: X and C as real matrices of interleaved (re, im) columns
            const double* Lr = (const double*)Li;
            for (int b = 0; b < B; ++b)
                gemm<double>(p->s, OP_T, OP_N, n, 2 * ncols, n, 1.0, Lr + b * sL, n, 0,
                             (const double*)(X + b * sX), 2 * ncols, 2L * n * ncols, 0.0, (double*)(C + b * sH),
                             2 * ldh, 2L * n * ldh, nsp, nullptr, 0, UPLO_FULL, nullptr, TRI_A_UPPER);
            return;
        }
    }
    if (nsp == 1) {
        gemm<T>(p->s, OP_C, OP_N, n, ncols, n, 1.0, Li, n, sL, X, ncols, sX, 0.0, C, ldh, sH, B, nullptr, 0,
                UPLO_FULL, nullptr, TRI_A_UPPER);
    } else {
        for (int b = 0; b < B; ++b)
            gemm<T>(p->s, OP_C, OP_N, n, ncols, n, 1.0, Li + b * sL, n, 0, X + b * sX, ncols, (long)n * ncols, 0.0,
                    C + b * sH, ldh, (long)n * ldh, nsp, nullptr, 0, UPLO_FULL, nullptr, TRI_A_UPPER);
    }
}

// The Cholesky factor of S and its inverse into the plan (L, Li); with
// KS_PLAN_REAL_OVERLAP on a complex plan both are real matrices (n x n
// doubles per matrix) in the same buffers.
template <typename T>
void factor_overlap(ks_plan* p, const T* S) {
    const int n = p->d.n, B = p->d.batch, lds = p->d.ld_s;
    const long sL = (long)n * n, sw = (long)p->order * p->order;
    if constexpr (is_cplx<T>::value) {
        if (p->d.flags & KS_PLAN_REAL_OVERLAP) {
            real_sym_complete(p->s, n, S, lds, (long)n * lds, (double*)p->L, n, sL, B, p->info);
            // W (order^2 complex per matrix, free until the reduction) holds the inverse's intermediate
            potrf_inv<double>(p->s, n, (double*)p->L, n, sL, (double*)p->Li, n, sL, (double*)p->W, 2 * sw, B,
                              p->info);
            return;
        }
    }
    herm_complete<T>(p->s, n, S, lds, (long)n * lds, (T*)p->L, n, sL, B, p->info);
    potrf_inv<T>(p->s, n, (T*)p->L, n, sL, (T*)p->Li, n, sL, (T*)p->W, sw, B, p->info);
}

// A = (I (x) Linv) H (I (x) Linv)^H with the plan's factor (lower triangle
// only with lower_only).
template <typename T>
void reduce_h(ks_plan* p, const T* H, T* A, T* W, bool lower_only) {
    const int n = p->d.n, nsp = p->nsp, B = p->d.batch, ldh = p->d.ld_h;
    const long sL = (long)n * n, sH = (long)p->order * ldh;
    if constexpr (is_cplx<T>::value) {
        if (p->d.flags & KS_PLAN_REAL_OVERLAP) {
            reduce_to_standard_real(p->s, n, nsp, B, H, ldh, sH, (const double*)p->Li, n, sL, A, W, p->info,
                                    lower_only);
            return;
        }
    }
    reduce_to_standard<T>(p->s, n, nsp, B, H, ldh, sH, (const T*)p->Li, n, sL, A, W, p->info, lower_only);
}

template <typename T>
HetrdWork<T>& hetrd_work(ks_plan* p) {
    return *reinterpret_cast<HetrdWork<T>*>(is_cplx<T>::value ? (void*)&p->hc : (void*)&p->hr);
}
template <typename T>
BacktrWork<T>& backtr_work(ks_plan* p) {
    return *reinterpret_cast<BacktrWork<T>*>(is_cplx<T>::value ? (void*)&p->bc : (void*)&p->br);
}
template <typename T>
BandWork<T>& band_work(ks_plan* p) {
    return *reinterpret_cast<BandWork<T>*>(is_cplx<T>::value ? (void*)&p->bandc : (void*)&p->bandr);
}

// A (order x order per matrix, lower triangle read) = Q T Q^H into (dv, ev),
// the reflectors of Q in W and tau: one-stage Householder, or with
// KS_PLAN_TWOSTAGE dense -> band -> tridiagonal (the stage-1 reflectors in W
// and tau, the stage-2 ones in the band buffers).
template <typename T>
void tridiagonalize(ks_plan* p, T* A, T* W, T* tau) {
    const int order = p->order, B = p->d.batch;
    const long sA = (long)order * order;
    if (p->d.flags & KS_PLAN_TWOSTAGE) {
        he2hb<T>(p->s, order, A, order, sA, B, W, tau, band_work<T>(p), p->info);
        hb2st<T>(p->s, order, A, order, sA, B, p->dv, p->ev, band_work<T>(p), p->info);
    } else {
        hetrd<T, T>(p->s, order, A, order, sA, B, p->dv, p->ev, tau, W, hetrd_work<T>(p));
    }
}

// X = Q Z[:, c0 : c0 + ncols] (order x ncols per matrix, matrix stride
// order^2) for the Q that tridiagonalize() left in W and tau.
template <typename T>
void back_q(ks_plan* p, const T* W, const T* tau, int c0, int ncols, T* X) {
    const int order = p->order, B = p->d.batch;
    const long sA = (long)order * order;
    load_z<T>(p->s, order, B, ncols, p->Z, c0, X, ncols, sA);
    if (p->d.flags & KS_PLAN_TWOSTAGE) q2_apply<T>(p->s, order, B, ncols, X, ncols, sA, band_work<T>(p), p->info);
    backtransform_prepare<T>(p->s, order, B, W, tau, backtr_work<T>(p));
    backtransform_q<T>(p->s, order, B, W, ncols, X, ncols, sA, backtr_work<T>(p));
}

// Mixed-precision eigensolve after the Cholesky factor is in place:
//   A (FP64, full) = Linv H Linv^H; its FP32 copy is tridiagonalised (trailing
//   matrix in FP32, rank-2NB updates on the FP32 matrix cores, panels in FP64);
//   divide and conquer in FP64 gives lam_hat and Z; the window vectors
//   X = Q Z[:, window] come from the FP32 back-transform.  Refinement in FP64:
//   mixed_sweeps correction sweeps X -= Q Z S(Z^T Q^H (A X - X lam_hat)) (the
//   products with Q and Z in FP32) remove the components outside the window;
//   the window's own eigenproblem in span(X), G = X^H A X, is then solved by
//   M x M refinement passes (subspace_refine).  Eigenvalues outside the window
//   are lam_hat.
template <typename T>
ks_status gevd_mixed(ks_plan* p, const T* H, double* eps, T* C, int il, int iu) {
    using L = typename Lo<T>::type;
    hipStream_t s = p->s;
    const int n = p->d.n, nsp = p->nsp, order = p->order, B = p->d.batch, ldh = p->d.ld_h;
    const int M = iu - il + 1, c0 = il - 1;
    const long sA = (long)order * order, sL = (long)n * n, sH = (long)order * ldh, sM = (long)order * M;
    const long sMM = (long)M * M;
    T* A = (T*)p->A;
    T* W = (T*)p->W;
    T* tau = (T*)p->tau;
    T* Li = (T*)p->Li;
    L* A32 = (L*)p->A32;
    L* W32 = (L*)p->W32;
    float* Z32 = p->Z32;
    HetrdWork<T>& hw = *reinterpret_cast<HetrdWork<T>*>(is_cplx<T>::value ? (void*)&p->hc : (void*)&p->hr);
    BacktrWork<T>& bw = *reinterpret_cast<BacktrWork<T>*>(is_cplx<T>::value ? (void*)&p->bc : (void*)&p->br);
    BacktrWork<L> bl = lo_view(bw);
    bl.Tall = (L*)p->Tall32;
    Prof& pf = p->prof;
    hipEvent_t e = pf.begin();
    // the lower triangle, then the upper one as its mirror (the residuals take
    // products with the whole matrix)
    reduce_h<T>(p, H, A, W, true);
    mirror_lower<T>(s, order, A, order, sA, B);
    convert<T, L>(s, B, order, order, A, order, sA, A32, order, sA);
    pf.end(KS_PHASE_REDUCE, e);
    e = pf.begin();
    hetrd<T, L>(s, order, A32, order, sA, B, p->dv, p->ev, tau, W, hw);
    pf.end(KS_PHASE_TRIDIAG, e);
    e = pf.begin();
    stedc(s, p->tree, B, p->dv, p->ev, eps, p->Z, p->Z2, p->U, p->Qp, p->dc, p->info);
    pf.end(KS_PHASE_DC, e);
    e = pf.begin();
    // FP32 copies of the reflectors, their compact-WY factors and of Z, then
    // X = Q Z[:, window] in FP32, widened into W
    backtransform_prepare<T>(s, order, B, W, tau, bw);
    convert<T, L>(s, B, 1, (int)bw.sTall, bw.Tall, (int)bw.sTall, bw.sTall, bl.Tall, (int)bw.sTall, bw.sTall);
    convert<T, L>(s, B, order, order, W, order, sA, W32, order, sA);
    convert<double, float>(s, B, order, order, p->Z, order, sA, Z32, order, sA);
    L* P = (L*)p->mP;
    load_z<L>(s, order, B, M, p->Z, c0, P, M, sM);
    backtransform_q<L>(s, order, B, W32, M, P, M, sM, bl);
    T* X = W;  // the FP64 reflectors are no longer needed
    convert<L, T>(s, B, order, M, P, M, sM, X, M, sM);
    pf.end(KS_PHASE_BACKTR, e);
    e = pf.begin();
    T* Y = (T*)p->mY;
    T* R = (T*)p->mR;
    const int wv = is_cplx<T>::value ? 2 : 1;  // a complex FP32 row of m entries is 2m floats
    float* Pf = (float*)p->mP;
    float* P2f = (float*)p->mP2;
    for (int sw = 0; sw < p->mixed_sweeps; ++sw) {
        gemm<T>(s, OP_N, OP_N, order, M, order, 1.0, A, order, sA, X, M, sM, 0.0, Y, M, sM, B);
        residual<T>(s, B, order, M, Y, X, sM, eps, order, c0, R);
        convert<T, L>(s, B, order, M, R, M, sM, P, M, sM);
        backtransform_q<L>(s, order, B, W32, M, P, M, sM, bl, true);  // Q^H R
        gemm<float>(s, OP_T, OP_N, order, wv * M, order, 1.0, Z32, order, sA, Pf, wv * M, wv * sM, 0.0, P2f,
                    wv * M, wv * sM, B);  // Z^T Q^H R
        correction_scale(s, B, order, M, wv, P2f, wv * sM, eps, order, c0);
        gemm<float>(s, OP_N, OP_N, order, wv * M, order, 1.0, Z32, order, sA, P2f, wv * M, wv * sM, 0.0, Pf,
                    wv * M, wv * sM, B);
        backtransform_q<L>(s, order, B, W32, M, P, M, sM, bl);  // Q Z S(...)
        sub_widened<T, L>(s, B, sM, X, P, sM);
    }
    // the window inside the refined subspace: G = X^H A X, then M x M
    // refinement (subspace_refine) instead of a nested eigensolve; X comes back
    // refined, with its columns in ascending order of the window values
    T* G = (T*)p->mG;
    T* Bm = (T*)p->mB;
    gemm<T>(s, OP_N, OP_N, order, M, order, 1.0, A, order, sA, X, M, sM, 0.0, Y, M, sM, B);
    gemm<T>(s, OP_C, OP_N, M, M, order, 1.0, X, M, sM, Y, M, sM, 0.0, G, M, sMM, B);
    subspace_refine<T>(s, B, order, M, X, sM, Y, G, Bm, R, (T*)p->mS, (T*)p->mS2, p->theta, order, p->mI,
                       p->mI + (long)B * order, p->mI + 2L * B * order, order, eps, order, c0, 2);
    pf.end(KS_PHASE_REFINE, e);
    e = pf.begin();
    apply_linv_h<T>(p, Li, X, sM, M, C);
    pf.end(KS_PHASE_BACKTR, e);
    if (hipPeekAtLastError() != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}

// V = U s^-1/2 (Part 2-2 / 3-2) with the columns in descending order of s:
// column j of V is eigenvector n-1-j of S scaled by 1/sqrt(s), or zero when
// s <= tau * max(s) (canonical orthogonalisation drops it), so that the kept
// columns come first; nkeep gets their number.  With tau = 0 a non-positive
// s is a failure, KS_ERR_NOT_POSDEF with detail = the number of s_j <= 0
// (s ascends, so that is the index of the last one); with tau > 0 only a
// non-positive max(s) is.
template <typename T>
__global__ void lowdin_v_kernel(int n, const T* U, const double* sv, double tau, T* V, int* nkeep, int* info) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x, i = blockIdx.y;
    if (j >= n) return;
    const long b = blockIdx.z;
    const double* sb = sv + b * n;
    const double smax = sb[n - 1], thr = tau * smax;
    const int src = n - 1 - j;
    const double sj = sb[src];
    const bool keep = sj > thr && smax > 0.0;
    if (i == 0) {
        // src is the smallest kept eigenvalue: the kept count is n - src
        if (keep && (src == 0 || !(sb[src - 1] > thr))) nkeep[b] = n - src;
        if (!(smax > 0.0) && j == 0) {
            nkeep[b] = 0;
            set_info(info, KS_ERR_NOT_POSDEF, n);
        } else if (tau == 0.0 && !(sj > 0.0) && (src == n - 1 || sb[src + 1] > 0.0)) {
            set_info(info, KS_ERR_NOT_POSDEF, src + 1);
        }
    }
    const long o = b * n * n + (long)i * n;
    V[o + j] = keep ? U[o + src] * (1.0 / sqrt(sj)) : zero_<T>();
}

// |H'|_F^2 of the lower triangle (off-diagonal entries twice), one partial per
// 64-row block and matrix, summed in a fixed order.
template <typename T>
__global__ __launch_bounds__(256) void frob_lower_kernel(int order, const T* A, long sA, double* part) {
    __shared__ double red[4];
    const int r0 = blockIdx.x * 64, z = blockIdx.y;
    A += z * sA;
    double acc = 0.0;
    for (int r = r0; r < min(r0 + 64, order); ++r)
        for (int c = threadIdx.x; c <= r; c += blockDim.x) acc += (c < r ? 2.0 : 1.0) * abs2_(A[(long)r * order + c]);
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[(long)z * gridDim.x + blockIdx.x] = acc;
}

// The dropped directions of H' (zero rows and columns) get a diagonal
// placeholder sigma = 2 |H'|_F + 1, above every kept eigenvalue, so that they
// sort last with zero eigenvectors C = V_NC e_j and zero occupation.
template <typename T>
__global__ __launch_bounds__(256) void lowdin_sigma_kernel(int n, int nsp, int order, T* A, long sA,
                                                           const double* part, int nblk, const int* nkeep) {
    __shared__ double sig;
    const int z = blockIdx.x;
    if (threadIdx.x == 0) {
        double f = 0.0;
        for (int q = 0; q < nblk; ++q) f += part[(long)z * nblk + q];
        sig = 2.0 * sqrt(f) + 1.0;
    }
    __syncthreads();
    const int nk = nkeep[z], nd = n - nk;
    A += z * sA;
    for (int e = threadIdx.x; e < nsp * nd; e += blockDim.x) {
        const int r = (e / nd) * n + nk + e % nd;
        A[(long)r * order + r] = from_re<T>(sig);
    }
}

// Loewdin route (Sec. 3.1 Parts 2-1..2-5; Sec. 3.2 Parts 3-1..3-6): eigenvectors
// U and eigenvalues s of S (Hermitian eigensolve of order n: the same
// tridiagonalisation, divide and conquer and back-transform as the main solve,
// on plan q); V = U s^-1/2; H' = V_NC^H H V_NC with V_NC = diag(V, V);
// H' C' = C' eps; C = V_NC C'.  Under KS_REUSE_S the V of the previous call is
// kept (the paper's SCF cycles 2 onwards skip Parts 2-1 and 2-2).
template <typename T>
ks_status gevd_lowdin(ks_plan* p, const T* H, const T* S, double* eps, T* C, int il, int iu, uint32_t flags) {
    hipStream_t s = p->s;
    const int n = p->d.n, nsp = p->nsp, order = p->order, B = p->d.batch, ldh = p->d.ld_h, lds = p->d.ld_s;
    const long sA = (long)order * order, sV = (long)n * n, sH = (long)order * ldh;
    T* A = (T*)p->A;
    T* W = (T*)p->W;
    T* V = (T*)p->L;
    Prof& pf = p->prof;
    if (!(flags & KS_REUSE_S)) {
        hipEvent_t e = pf.begin();
        ks_plan* q = p->ov ? p->ov : p;  // an order-n plan
        T* Aq = (T*)q->A;
        T* Wq = (T*)q->W;
        HetrdWork<T>& qh = *reinterpret_cast<HetrdWork<T>*>(is_cplx<T>::value ? (void*)&q->hc : (void*)&q->hr);
        BacktrWork<T>& qb = *reinterpret_cast<BacktrWork<T>*>(is_cplx<T>::value ? (void*)&q->bc : (void*)&q->br);
        herm_complete<T>(s, n, S, lds, (long)n * lds, Aq, n, sV, B, p->info);
        hetrd<T, T>(s, n, Aq, n, sV, B, q->dv, q->ev, (T*)q->tau, Wq, qh);
        stedc(s, q->tree, B, q->dv, q->ev, p->sev, q->Z, q->Z2, q->U, q->Qp, q->dc, p->info);
        load_z<T>(s, n, B, n, q->Z, 0, Aq, n, sV);
        backtransform_prepare<T>(s, n, B, Wq, (T*)q->tau, qb);
        backtransform_q<T>(s, n, B, Wq, n, Aq, n, sV, qb);
        hipLaunchKernelGGL(lowdin_v_kernel<T>, dim3(cdiv(n, 256), n, B), dim3(256), 0, s, n, (const T*)Aq,
                           (const double*)p->sev, p->ov_tau, V, p->nkeep, p->info);
        p->v_tau = p->ov_tau;
        pf.end(KS_PHASE_CHOLESKY, e);
        p->have_L = true;
    }
    const int ncols = iu - il + 1;
    hipEvent_t e = pf.begin();
    // H' = V_NC^H (H V_NC): the full H in A, W = A V_NC, then the lower triangle
    // of H' (the part the tridiagonalisation reads) into A
    herm_complete<T>(s, order, H, ldh, sH, A, order, sA, B, p->info);
    for (int b = 0; b < nsp; ++b)
        gemm<T>(s, OP_N, OP_N, order, n, n, 1.0, A + b * n, order, sA, V, n, sV, 0.0, W + b * n, order, sA, B);
    for (int b = 0; b < nsp; ++b)
        gemm<T>(s, OP_C, OP_N, n, order, n, 1.0, V, n, sV, W + (long)b * n * order, order, sA, 0.0,
                A + (long)b * n * order, order, sA, B, nullptr, 0, b == 0 ? UPLO_LOWER : UPLO_FULL);
    if (p->v_tau > 0.0) {  // V has dropped (zero) columns: give them their placeholder
        const int nblk = cdiv(order, 64);
        hipLaunchKernelGGL(frob_lower_kernel<T>, dim3(nblk, B), dim3(256), 0, s, order, (const T*)A, sA, p->fpart);
        hipLaunchKernelGGL(lowdin_sigma_kernel<T>, dim3(B), dim3(256), 0, s, n, nsp, order, A, sA,
                           (const double*)p->fpart, nblk, (const int*)p->nkeep);
    }
    pf.end(KS_PHASE_REDUCE, e);
    e = pf.begin();
    tridiagonalize<T>(p, A, W, (T*)p->tau);
    pf.end(KS_PHASE_TRIDIAG, e);
    e = pf.begin();
    stedc(s, p->tree, B, p->dv, p->ev, eps, p->Z, p->Z2, p->U, p->Qp, p->dc, p->info);
    pf.end(KS_PHASE_DC, e);
    e = pf.begin();
    back_q<T>(p, W, (const T*)p->tau, il - 1, ncols, A);
    // C_sigma = V C'_sigma per spin block
    for (int b = 0; b < nsp; ++b)
        gemm<T>(s, OP_N, OP_N, n, ncols, n, 1.0, V, n, sV, A + (long)b * n * ncols, ncols, sA, 0.0,
                C + (long)b * n * ldh, ldh, sH, B);
    pf.end(KS_PHASE_BACKTR, e);
    if (hipPeekAtLastError() != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}

template <typename T>
ks_status gevd_impl(ks_plan* p, const T* H, const T* S, double* eps, T* C, int il, int iu,
                    uint32_t flags) {
    hipStream_t s = p->s;
    const int order = p->order, B = p->d.batch;
    T* A = (T*)p->A;
    T* W = (T*)p->W;
    T* tau = (T*)p->tau;
    Prof& pf = p->prof;
    T* Li = (T*)p->Li;
    if (p->d.flags & KS_PLAN_LOWDIN) return gevd_lowdin<T>(p, H, S, eps, C, il, iu, flags);
    if (!(flags & KS_REUSE_S)) {
        hipEvent_t e = pf.begin();
        factor_overlap<T>(p, S);
        pf.end(KS_PHASE_CHOLESKY, e);
        p->have_L = true;
    }
    if (p->d.precision == KS_MIXED) return gevd_mixed<T>(p, H, eps, C, il, iu);
    // every step below takes the whole batch of k-points in each launch
    const int ncols = iu - il + 1;
    const long sA = (long)order * order;
    hipEvent_t e = pf.begin();
    // only the lower triangle: the tridiagonalisation reads nothing else
    reduce_h<T>(p, H, A, W, true);
    pf.end(KS_PHASE_REDUCE, e);
    e = pf.begin();
    tridiagonalize<T>(p, A, W, tau);
    pf.end(KS_PHASE_TRIDIAG, e);
    e = pf.begin();
    stedc(s, p->tree, B, p->dv, p->ev, eps, p->Z, p->Z2, p->U, p->Qp, p->dc, p->info);
    pf.end(KS_PHASE_DC, e);
    e = pf.begin();
    // X = Q Z[:, il-1 : iu] in A (order x ncols per matrix), then C_sigma = Linv^H X_sigma per spin block
    back_q<T>(p, W, tau, il - 1, ncols, A);
    apply_linv_h<T>(p, Li, A, sA, ncols, C);
    pf.end(KS_PHASE_BACKTR, e);
    if (hipPeekAtLastError() != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}

}  // namespace

namespace {

// The plan's knobs into its work descriptors.
void apply_tuning(ks_plan* p) {
    const ks_tuning& tu = p->tuning;
    p->hr.sch = p->hc.sch = tu.tiles_per_workgroup;
    p->hr.nseg = p->hc.nseg = tu.nseg;
    for (int i = 0; i < tu.nseg; ++i) {
        p->hr.seg_first[i] = p->hc.seg_first[i] = tu.seg_first[i];
        p->hr.seg_sch[i] = p->hc.seg_sch[i] = tu.seg_tiles[i];
    }
    set_backtr_block(p->br, p->order, tu.backtr_block);
    set_backtr_block(p->bc, p->order, tu.backtr_block);
}

// Milliseconds of `rounds` runs of f after one untimed run, the least.
template <typename F>
float time_min(hipStream_t s, int rounds, F f) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -1.f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1.f;
    }
    f();
    float best = 3.0e38f;
    for (int r = 0; r < rounds; ++r) {
        (void)hipEventRecord(e0, s);
        f();
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
            best = -1.f;
            break;
        }
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e0, e1);
        best = std::min(best, t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
}

// Back-transform block and large-GEMM threshold: one back-transform of all
// eigenvectors (the plan's own shapes and buffers, zero reflectors: the
// products' time does not depend on the values) per candidate pair.
template <typename T>
ks_status tune_backtr(ks_plan* p) {
    ks_tuning& tu = p->tuning;
    const int order = p->order, B = p->d.batch;
    const long sA = (long)order * order;
    BacktrWork<T>& w = backtr_work<T>(p);
    T* V = (T*)p->W;
    T* tau = (T*)p->tau;
    T* X = (T*)p->A;
    fill_zero<T>(p->s, V, sA * B);
    fill_zero<T>(p->s, tau, (long)order * B);
    fill_zero<T>(p->s, X, sA * B);
    float best = 3.0e38f;
    for (int bi = 0; bi < 2; ++bi)
        for (int gi = 0; gi < 2; ++gi) {
            const int bt = 128 << bi, gk = gi ? KS_TUNE_NEVER : 256;
            set_backtr_block(w, order, bt);
            GemmPolicy gp(gk);
            const float t = time_min(p->s, 2, [&]() {
                backtransform_prepare<T>(p->s, order, B, V, tau, w);
                backtransform_q<T>(p->s, order, B, V, order, X, order, sA, w);
            });
            if (t < 0.f) return KS_ERR_HIP;
            tu.backtr_ms[bi][gi] = t;
            if (t < best) {
                best = t;
                tu.backtr_block = bt;
                tu.gemm_big_min_k = gk;
            }
        }
    return KS_OK;
}

__global__ void synth_tridiag_kernel(int n, long total, double* d, double* e) {
    const long i = blockIdx.x * (long)blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int k = (int)(i % n);
    d[i] = 2.0 * cos(0.731 * k) + (double)k / n;
    e[i] = 0.5 + 0.25 * sin(1.37 * k);
}

// Divide-and-conquer leaf: one solve of a fixed tridiagonal of the plan's
// order (smooth, non-degenerate entries) per candidate.
ks_status tune_dc(ks_plan* p) {
    const int order = p->order, B = p->d.batch;
    const long tot = (long)order * B;
    hipLaunchKernelGGL(synth_tridiag_kernel, dim3((unsigned)cdiv(tot, 256)), dim3(256), 0, p->s, order, tot, p->dv,
                       p->ev);
    float best = 3.0e38f;
    int leaf_best = DC_LEAF;
    for (int li = 0; li < 2; ++li) {
        const int leaf = DC_LEAF_MIN << li;
        if (hipStreamSynchronize(p->s) != hipSuccess) return KS_ERR_HIP;
        ks_status st = set_dc_leaf(p, leaf);
        if (st != KS_OK) return st;
        const float t = time_min(p->s, 2, [&]() {
            stedc(p->s, p->tree, B, p->dv, p->ev, p->occ, p->Z, p->Z2, p->U, p->Qp, p->dc, p->info);
        });
        if (t < 0.f) return KS_ERR_HIP;
        p->tuning.dc_ms[li] = t;
        if (t < best) {
            best = t;
            leaf_best = leaf;
        }
    }
    ks_status st = set_dc_leaf(p, leaf_best);
    if (st != KS_OK) return st;
    if (hipMemset(p->info, 0, 2 * sizeof(int)) != hipSuccess) return KS_ERR_HIP;
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
    uint64_t bytes = layout(d, nullptr);
    if ((d->flags & KS_PLAN_LOWDIN) && d->spin == KS_NONCOLLINEAR) {
        ks_plan_desc c = lowdin_overlap_desc(d);
        bytes += layout(&c, nullptr);
    }
    return bytes;
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
    if (d->flags & KS_PLAN_TWOSTAGE) {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) {
            (void)hipFree(p->base);
            delete p;
            return KS_ERR_HIP;
        }
        p->bandr.ncu = p->bandc.ncu = ncu;
        // the panel factorisation's workgroups of one matrix must all be resident together
        if (cdiv(p->order, panel_rows(p->is_c)) > ncu) {
            (void)hipFree(p->base);
            delete p;
            return KS_ERR_NOT_SUPPORTED;
        }
    }
    if (d->batch >= 2) {
        if (hipStreamCreateWithFlags(&p->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&p->side_fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&p->side_join, hipEventDisableTiming) != hipSuccess) {
            ks_plan_destroy(p);
            return KS_ERR_HIP;
        }
        p->hr.side = p->hc.side = p->side;
        p->hr.fork = p->hc.fork = p->side_fork;
        p->hr.join = p->hc.join = p->side_join;
    }
    p->kw_last = make_weights(p, nullptr);
    if (hipMemset(p->info, 0, 2 * sizeof(int)) != hipSuccess) {
        (void)hipFree(p->base);
        delete p;
        return KS_ERR_HIP;
    }
    if ((d->flags & KS_PLAN_LOWDIN) && p->nsp == 2) {
        ks_plan_desc c = lowdin_overlap_desc(d);
        ks_status st = ks_plan_create(&c, &p->ov);
        if (st != KS_OK) {
            ks_plan_destroy(p);
            return st;
        }
    }
    p->tuning.tiles_per_workgroup = HETRD_SCH;
    p->tuning.nseg = 1;
    p->tuning.seg_first[0] = 0;
    p->tuning.seg_tiles[0] = HETRD_SCH;
    p->tuning.backtr_block = backtr_block(p->order);
    p->tuning.gemm_big_min_k = 256;
    if (d->flags & KS_PLAN_AUTOTUNE) {
        ks_tuning& tu = p->tuning;
        const long sA = (long)p->order * p->order;
        // the symmetric product in the storage precision of the trailing matrix
        // (FP32 in the mixed form)
        const bool lo = d->precision == KS_MIXED;
        if (p->is_c && lo)
            tu.ncand = hetrd_tune<cplx, cplx32>(p->s, p->order, (cplx32*)p->A32, p->order, sA, d->batch, p->dv,
                                                p->ev, (cplx*)p->tau, p->hc, tu.cand, tu.ms, 8, tu.seg_first,
                                                tu.seg_tiles);
        else if (p->is_c)
            tu.ncand = hetrd_tune<cplx, cplx>(p->s, p->order, (cplx*)p->A, p->order, sA, d->batch, p->dv, p->ev,
                                              (cplx*)p->tau, p->hc, tu.cand, tu.ms, 8, tu.seg_first, tu.seg_tiles);
        else if (lo)
            tu.ncand = hetrd_tune<double, float>(p->s, p->order, (float*)p->A32, p->order, sA, d->batch, p->dv,
                                                 p->ev, (double*)p->tau, p->hr, tu.cand, tu.ms, 8, tu.seg_first,
                                                 tu.seg_tiles);
        else
            tu.ncand = hetrd_tune<double, double>(p->s, p->order, (double*)p->A, p->order, sA, d->batch, p->dv,
                                                  p->ev, (double*)p->tau, p->hr, tu.cand, tu.ms, 8, tu.seg_first,
                                                  tu.seg_tiles);
        int best = 0;
        for (int c = 1; c < tu.ncand; ++c)
            if (tu.ms[c] < tu.ms[best]) best = c;
        if (tu.ncand > 0) tu.tiles_per_workgroup = tu.cand[best];
        tu.nseg = KS_TUNE_SEGMENTS;
        if (hipStreamSynchronize(p->s) != hipSuccess || tu.ncand == 0) {
            ks_plan_destroy(p);
            return KS_ERR_HIP;
        }
        ks_status st = p->is_c ? tune_backtr<cplx>(p) : tune_backtr<double>(p);
        if (st == KS_OK) st = tune_dc(p);
        if (st != KS_OK) {
            ks_plan_destroy(p);
            return st;
        }
    }
    apply_tuning(p);
    *out = p;
    return KS_OK;
}

void ks_plan_destroy(ks_plan* p) {
    if (!p) return;
    (void)hipStreamSynchronize(p->s);
    if (p->side) (void)hipStreamSynchronize(p->side);
    graph_release(p);
    if (p->side_join) (void)hipEventDestroy(p->side_join);
    if (p->side_fork) (void)hipEventDestroy(p->side_fork);
    if (p->side) (void)hipStreamDestroy(p->side);
    if (p->rr) ks_plan_destroy(p->rr);
    if (p->ov) ks_plan_destroy(p->ov);
    if (p->base) (void)hipFree(p->base);
    if (p->adj) (void)hipFree(p->adj);
    delete p;
}

ks_status ks_plan_set_overlap_cutoff(ks_plan* p, double tau) {
    if (!p || !(tau >= 0.0 && tau < 1.0)) return KS_ERR_INVALID_ARG;
    if (!(p->d.flags & KS_PLAN_LOWDIN)) return KS_ERR_NOT_SUPPORTED;
    if (p->ov_tau != tau) graph_release(p);  // a captured sequence would keep the old cutoff
    p->ov_tau = tau;
    return KS_OK;
}

ks_status ks_plan_get_overlap_rank(ks_plan* p, int32_t* nkeep) {
    if (!p || !nkeep) return KS_ERR_INVALID_ARG;
    if (!(p->d.flags & KS_PLAN_LOWDIN)) return KS_ERR_NOT_SUPPORTED;
    if (!p->have_L) return KS_ERR_INVALID_ARG;
    if (hipStreamSynchronize(p->s) != hipSuccess) return KS_ERR_HIP;
    if (hipMemcpy(nkeep, p->nkeep, sizeof(int) * p->d.batch, hipMemcpyDeviceToHost) != hipSuccess)
        return KS_ERR_HIP;
    return KS_OK;
}

ks_status ks_plan_set_refinement(ks_plan* p, int32_t sweeps) {
    if (!p || sweeps < 0 || sweeps > 4) return KS_ERR_INVALID_ARG;
    if (p->d.precision != KS_MIXED) return KS_ERR_NOT_SUPPORTED;
    if (p->mixed_sweeps != sweeps) graph_release(p);  // a captured sequence would keep the old count
    p->mixed_sweeps = sweeps;
    return KS_OK;
}

ks_status ks_plan_get_tuning(ks_plan* p, ks_tuning* out) {
    if (!p || !out) return KS_ERR_INVALID_ARG;
    *out = p->tuning;
    return KS_OK;
}

ks_status ks_plan_set_tuning(ks_plan* p, const ks_tuning* t) {
    if (!p || !t) return KS_ERR_INVALID_ARG;
    auto tiles_ok = [](int v) { return v == 2 || v == 4 || v == 8; };
    if (!tiles_ok(t->tiles_per_workgroup)) return KS_ERR_INVALID_ARG;
    if (t->nseg < 1 || t->nseg > KS_TUNE_SEGMENTS || t->seg_first[0] != 0) return KS_ERR_INVALID_ARG;
    for (int i = 0; i < t->nseg; ++i) {
        if (!tiles_ok(t->seg_tiles[i])) return KS_ERR_INVALID_ARG;
        if (i > 0 && t->seg_first[i] <= t->seg_first[i - 1]) return KS_ERR_INVALID_ARG;
    }
    if (t->backtr_block != 128 && t->backtr_block != 256) return KS_ERR_INVALID_ARG;
    if (t->gemm_big_min_k < 16) return KS_ERR_INVALID_ARG;
    if (t->dc_leaf != DC_LEAF_MIN && t->dc_leaf != DC_LEAF) return KS_ERR_INVALID_ARG;
    // work in flight may use the tree and the block layout
    if (hipStreamSynchronize(p->s) != hipSuccess) return KS_ERR_HIP;
    ks_status st = set_dc_leaf(p, t->dc_leaf);
    if (st != KS_OK) return st;
    p->tuning = *t;
    p->tuning.from_cache = 1;
    apply_tuning(p);
    graph_release(p);
    return KS_OK;
}

ks_status ks_plan_get_graph_stats(ks_plan* p, int64_t* captures, int64_t* replays) {
    if (!p || !captures || !replays) return KS_ERR_INVALID_ARG;
    *captures = p->graph_captures;
    *replays = p->graph_replays;
    return KS_OK;
}

ks_status ks_gevd(ks_plan* p, const void* H, const void* S, double* eps, void* C, int32_t il,
                  int32_t iu, uint32_t flags) {
    if (!p || !H || !eps || !C) return KS_ERR_INVALID_ARG;
    GemmPolicy gpol(p->tuning.gemm_big_min_k);  // the plan's large-tile threshold for its launches
    if (flags & ~(uint32_t)KS_REUSE_S) return KS_ERR_INVALID_ARG;
    if (!(flags & KS_REUSE_S) && !S) return KS_ERR_INVALID_ARG;
    if ((flags & KS_REUSE_S) && !p->have_L) return KS_ERR_INVALID_ARG;
    if (!range_ok(p, il, iu)) return KS_ERR_INVALID_ARG;
    auto enqueue = [&]() -> ks_status {
        if (p->is_c)
            return gevd_impl<cplx>(p, (const cplx*)H, (const cplx*)S, eps, (cplx*)C, il, iu, flags);
        return gevd_impl<double>(p, (const double*)H, (const double*)S, eps, (double*)C, il, iu, flags);
    };
    if (!(p->d.flags & KS_PLAN_GRAPH)) return enqueue();
    ks_plan::GraphKey key{H, S, eps, C, il, iu, flags};
    if (!(p->gexec && key == p->gkey)) {
        graph_release(p);
        const bool prof = p->prof.on;
        p->prof.on = false;  // no timing events inside a graph
        if (hipStreamBeginCapture(p->s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            p->prof.on = prof;
            return KS_ERR_HIP;
        }
        ks_status st = enqueue();
        hipGraph_t g = nullptr;
        hipError_t ec = hipStreamEndCapture(p->s, &g);
        p->prof.on = prof;
        if (st != KS_OK || ec != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return st != KS_OK ? st : KS_ERR_HIP;
        }
        hipGraphExec_t ex = nullptr;
        if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return KS_ERR_HIP;
        }
        p->graph = g;
        p->gexec = ex;
        p->gkey = key;
        ++p->graph_captures;
    } else {
        ++p->graph_replays;
    }
    if (hipGraphLaunch(p->gexec, p->s) != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}

ks_status ks_density(ks_plan* p, const double* eps, const void* C, int32_t il, int32_t iu,
                     double ne, double kT, const double* kweights, void* rho, double* mu,
                     double* eband, double* occ) {
    if (!p || !eps || !C || !rho || !mu || !eband) return KS_ERR_INVALID_ARG;
    GemmPolicy gpol(p->tuning.gemm_big_min_k);  // the plan's large-tile threshold for its launches
    if (!range_ok(p, il, iu)) return KS_ERR_INVALID_ARG;
    if (!(kT > 0.0) || !isfinite(kT)) return KS_ERR_INVALID_ARG;
    double g = p->nsp == 2 ? 1.0 : 2.0;
    if (!(ne > 0.0) || !(ne <= g * p->order) || !isfinite(ne)) return KS_ERR_ELECTRON_COUNT;
    if (kweights) {
        for (int b = 0; b < p->d.batch; ++b)
            if (!(kweights[b] >= 0.0) || !isfinite(kweights[b])) return KS_ERR_INVALID_ARG;
    }
    KWeights kw = make_weights(p, kweights);
    p->kw_last = kw;
    double* f = occ ? occ : p->occ;
    hipStream_t s = p->s;
    int order = p->order, ldh = p->d.ld_h, ncols = iu - il + 1;
    hipEvent_t e = p->prof.begin();
    fermi(s, p->d.batch, order, eps, kw, g, ne, kT, il, iu, f, mu, eband, p->kwin, p->info);
    long mat = (long)order * ldh;
    // rho = C diag(f) C^H over the window columns that carry occupation (count
    // on the device): the lower triangle, then the upper one as its mirror
    if (p->is_c) {
        gemm<cplx>(s, OP_N, OP_C, order, order, ncols, 1.0, (const cplx*)C, ldh, mat, (const cplx*)C, ldh,
                   mat, 0.0, (cplx*)rho, ldh, mat, p->d.batch, f + il - 1, order, UPLO_LOWER, p->kwin);
        mirror_lower<cplx>(s, order, (cplx*)rho, ldh, mat, p->d.batch);
    } else {
        gemm<double>(s, OP_N, OP_T, order, order, ncols, 1.0, (const double*)C, ldh, mat,
                     (const double*)C, ldh, mat, 0.0, (double*)rho, ldh, mat, p->d.batch, f + il - 1,
                     order, UPLO_LOWER, p->kwin);
        mirror_lower<double>(s, order, (double*)rho, ldh, mat, p->d.batch);
    }
    p->prof.end(KS_PHASE_DENSITY, e);
    if (hipPeekAtLastError() != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}

// Bloch sums over 32x32 tiles of the lower triangle: the workgroup of tile
// (I, J), I >= J, accumulates X_R[i][j] exp(i k.R) over R for up to BS_KC
// k-points at once (blockIdx.z selects the chunk; the phases of the chunk are
// formed once per workgroup in LDS), writes its tile, and writes the mirrored
// tile X[j][i] = conj(X[i][j]) through an LDS transpose, so that both
// triangles leave in coalesced rows and every X_R entry is read once per chunk.
constexpr int BS_KC = 16;
constexpr int BS_MAXR = 64;
constexpr int BS_T = 32;
__global__ __launch_bounds__(BS_T * BS_T) void bloch_sum_kernel(int n, int nk, int nR, const double* R,
                                                                const double* kvec, const double* XR, int ld_r,
                                                                cplx* Xk, int ld_k) {
    __shared__ double pc[BS_KC][BS_MAXR], ps[BS_KC][BS_MAXR];
    __shared__ cplx tr[2][BS_T][BS_T + 1];
    const int t = blockIdx.x;
    int I = (int)((sqrt(8.0 * t + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    const int J = t - I * (I + 1) / 2;
    const int k0 = blockIdx.z * BS_KC, kc = min(BS_KC, nk - k0);
    for (int e = threadIdx.x; e < kc * nR; e += blockDim.x) {
        const int q = e / nR, r = e % nR;
        const double* kv = kvec + 3L * (k0 + q);
        const double* rv = R + 3L * r;
        double sn, cs;
        sincos(kv[0] * rv[0] + kv[1] * rv[1] + kv[2] * rv[2], &sn, &cs);
        pc[q][r] = cs;
        ps[q][r] = sn;
    }
    __syncthreads();
    const int tx = threadIdx.x % BS_T, ty = threadIdx.x / BS_T;
    const int i = I * BS_T + ty, j = J * BS_T + tx;
    const bool in = i < n && j < n && (I > J || tx <= ty);
    double re[BS_KC], im[BS_KC];
#pragma unroll
    for (int q = 0; q < BS_KC; ++q) re[q] = im[q] = 0.0;
    if (in) {
        const double* x = XR + (long)i * ld_r + j;
        const long sr = (long)n * ld_r;
        int r = 0;
        for (; r + 4 <= nR; r += 4) {
            double xv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) xv[u] = x[(r + u) * sr];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int q = 0; q < BS_KC; ++q) {
                    re[q] += xv[u] * pc[q][r + u];
                    im[q] += xv[u] * ps[q][r + u];
                }
        }
        for (; r < nR; ++r) {
            const double xv = x[r * sr];
#pragma unroll
            for (int q = 0; q < BS_KC; ++q) {
                re[q] += xv * pc[q][r];
                im[q] += xv * ps[q][r];
            }
        }
    }
    // the mirrored entry this thread writes: row J*32+ty, column I*32+tx
    const int mi = J * BS_T + ty, mj = I * BS_T + tx;
    const bool min_ = mi < n && mj < n && (I > J || tx > ty);
#pragma unroll
    for (int q = 0; q < BS_KC; ++q) {
        if (q < kc) {
            cplx* o = Xk + (long)(k0 + q) * n * ld_k;
            const cplx v = mk(re[q], i == j ? 0.0 : im[q]);
            if (in) o[(long)i * ld_k + j] = v;
            tr[q & 1][ty][tx] = v;
            __syncthreads();
            if (min_) o[(long)mi * ld_k + mj] = conj_(tr[q & 1][tx][ty]);
        }
    }
}

ks_status ks_bloch_sum(ks_plan* p, int32_t nR, const double* R, const double* kvec, const double* XR,
                       int32_t ld_r, void* Xk, int32_t ld_k) {
    if (!p || !R || !kvec || !XR || !Xk || nR < 1) return KS_ERR_INVALID_ARG;
    const int n = p->d.n, nk = p->d.batch;
    if (ld_r < n || ld_k < n) return KS_ERR_INVALID_ARG;
    if (!p->is_c || p->nsp != 1) return KS_ERR_NOT_SUPPORTED;
    if (nR > BS_MAXR) return KS_ERR_INVALID_ARG;
    hipStream_t s = p->s;
    const int nt = cdiv(n, BS_T);
    hipLaunchKernelGGL(bloch_sum_kernel, dim3(nt * (nt + 1) / 2, 1, cdiv(nk, BS_KC)), dim3(BS_T * BS_T), 0, s, n, nk,
                       nR, R, kvec, XR, ld_r, (cplx*)Xk, ld_k);
    if (hipPeekAtLastError() != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}

// f_ik eps_ik for the window columns of every matrix of the batch.
__global__ void edm_weights_kernel(int order, int c0, int ncols, const double* occ, const double* eps, double* fe) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ncols) return;
    const long o = (long)blockIdx.y * order + c0 + i;
    fe[o] = occ[o] * eps[o];
}

ks_status ks_energy_density(ks_plan* p, const double* eps, const void* C, int32_t il, int32_t iu,
                            const double* occ, void* edm) {
    if (!p || !eps || !C || !occ || !edm) return KS_ERR_INVALID_ARG;
    GemmPolicy gpol(p->tuning.gemm_big_min_k);  // the plan's large-tile threshold for its launches
    if (!range_ok(p, il, iu)) return KS_ERR_INVALID_ARG;
    hipStream_t s = p->s;
    const int order = p->order, ldh = p->d.ld_h, ncols = iu - il + 1, c0 = il - 1;
    const long mat = (long)order * ldh;
    hipLaunchKernelGGL(edm_weights_kernel, dim3(cdiv(ncols, 256), p->d.batch), dim3(256), 0, s, order, c0, ncols,
                       occ, eps, p->fe);
    // E = C diag(f eps) C^H: the lower triangle, then the upper one as its mirror
    if (p->is_c) {
        gemm<cplx>(s, OP_N, OP_C, order, order, ncols, 1.0, (const cplx*)C, ldh, mat, (const cplx*)C, ldh, mat,
                   0.0, (cplx*)edm, ldh, mat, p->d.batch, p->fe + c0, order, UPLO_LOWER);
        mirror_lower<cplx>(s, order, (cplx*)edm, ldh, mat, p->d.batch);
    } else {
        gemm<double>(s, OP_N, OP_T, order, order, ncols, 1.0, (const double*)C, ldh, mat, (const double*)C, ldh,
                     mat, 0.0, (double*)edm, ldh, mat, p->d.batch, p->fe + c0, order, UPLO_LOWER);
        mirror_lower<double>(s, order, (double*)edm, ldh, mat, p->d.batch);
    }
    if (hipPeekAtLastError() != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}

ks_status ks_density_backward(ks_plan* p, const double* eps, const void* C, const double* mu,
                              const double* occ, double kT, const void* grad_rho,
                              const double* grad_eband, void* grad_H, void* grad_S) {
    if (!p || !eps || !C || !mu || !occ || !grad_H || !grad_S) return KS_ERR_INVALID_ARG;
    GemmPolicy gpol(p->tuning.gemm_big_min_k);  // the plan's large-tile threshold for its launches
    if (!(kT > 0.0) || !isfinite(kT)) return KS_ERR_INVALID_ARG;
    // the gradient formulas use the completeness of the eigenvectors in the
    // S metric, which a basis reduced by the overlap cutoff does not have
    if (p->v_tau > 0.0) return KS_ERR_NOT_SUPPORTED;
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
    const KWeights kw = p->kw_last;
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
    *info = (h[0] == KS_ERR_NOT_POSDEF || h[0] == KS_ERR_INVALID_ARG) ? h[1] : -h[0];
    return (ks_status)h[0];
}

}  // extern "C"

// Internal stage drivers used by the test hooks (ks_testhooks.hip).
void ks_internal_he2hb(ks_plan* p, void* A, const double* X, int ncols, void* Y) {
    int n = p->order;
    long sA = (long)n * n;
    if (p->is_c) {
        he2hb<cplx>(p->s, n, (cplx*)A, n, sA, 1, (cplx*)p->W, (cplx*)p->tau, p->bandc, p->info);
        load_z<cplx>(p->s, n, 1, ncols, X, 0, (cplx*)Y, ncols, 0);
        backtransform_prepare<cplx>(p->s, n, 1, (cplx*)p->W, (cplx*)p->tau, p->bc);
        backtransform_q<cplx>(p->s, n, 1, (cplx*)p->W, ncols, (cplx*)Y, ncols, 0, p->bc);
    } else {
        he2hb<double>(p->s, n, (double*)A, n, sA, 1, (double*)p->W, (double*)p->tau, p->bandr, p->info);
        load_z<double>(p->s, n, 1, ncols, X, 0, (double*)Y, ncols, 0);
        backtransform_prepare<double>(p->s, n, 1, (double*)p->W, (double*)p->tau, p->br);
        backtransform_q<double>(p->s, n, 1, (double*)p->W, ncols, (double*)Y, ncols, 0, p->br);
    }
}

void ks_internal_stedc(ks_plan* p, const double* d, const double* e, double* lam, double* Z) {
    stedc(p->s, p->tree, 1, d, e, lam, Z, p->Z2, p->U, p->Qp, p->dc, p->info);
}

void ks_internal_hetrd(ks_plan* p, void* A, double* d, double* e, const double* X, int ncols, void* Y) {
    int n = p->order;
    long sA = (long)n * n;
    if (p->d.flags & KS_PLAN_TWOSTAGE) {
        if (p->is_c) {
            BandWork<cplx>& w = p->bandc;
            he2hb<cplx>(p->s, n, (cplx*)A, n, sA, 1, (cplx*)p->W, (cplx*)p->tau, w, p->info);
            hb2st<cplx>(p->s, n, (cplx*)A, n, sA, 1, d, e, w, p->info);
            load_z<cplx>(p->s, n, 1, ncols, X, 0, (cplx*)Y, ncols, 0);
            q2_apply<cplx>(p->s, n, 1, ncols, (cplx*)Y, ncols, 0, w, p->info);
            backtransform_prepare<cplx>(p->s, n, 1, (cplx*)p->W, (cplx*)p->tau, p->bc);
            backtransform_q<cplx>(p->s, n, 1, (cplx*)p->W, ncols, (cplx*)Y, ncols, 0, p->bc);
        } else {
            BandWork<double>& w = p->bandr;
            he2hb<double>(p->s, n, (double*)A, n, sA, 1, (double*)p->W, (double*)p->tau, w, p->info);
            hb2st<double>(p->s, n, (double*)A, n, sA, 1, d, e, w, p->info);
            load_z<double>(p->s, n, 1, ncols, X, 0, (double*)Y, ncols, 0);
            q2_apply<double>(p->s, n, 1, ncols, (double*)Y, ncols, 0, w, p->info);
            backtransform_prepare<double>(p->s, n, 1, (double*)p->W, (double*)p->tau, p->br);
            backtransform_q<double>(p->s, n, 1, (double*)p->W, ncols, (double*)Y, ncols, 0, p->br);
        }
        return;
    }
    if (p->is_c) {
        hetrd<cplx, cplx>(p->s, n, (cplx*)A, n, sA, 1, d, e, (cplx*)p->tau, (cplx*)p->W, p->hc);
        load_z<cplx>(p->s, n, 1, ncols, X, 0, (cplx*)Y, ncols, 0);
        backtransform_prepare<cplx>(p->s, n, 1, (cplx*)p->W, (cplx*)p->tau, p->bc);
        backtransform_q<cplx>(p->s, n, 1, (cplx*)p->W, ncols, (cplx*)Y, ncols, 0, p->bc);
    } else {
        hetrd<double, double>(p->s, n, (double*)A, n, sA, 1, d, e, (double*)p->tau, (double*)p->W, p->hr);
        load_z<double>(p->s, n, 1, ncols, X, 0, (double*)Y, ncols, 0);
        backtransform_prepare<double>(p->s, n, 1, (double*)p->W, (double*)p->tau, p->br);
        backtransform_q<double>(p->s, n, 1, (double*)p->W, ncols, (double*)Y, ncols, 0, p->br);
    }
}
