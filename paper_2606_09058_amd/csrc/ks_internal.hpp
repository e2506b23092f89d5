// ks_internal.hpp -- internal interfaces between the host orchestration
// (ks_api.hip) and the kernel files.
#pragma once

#include <vector>
#include <algorithm>
#include <type_traits>

#include "ks_common.hpp"

namespace ks {

template <> __host__ __device__ inline int zero_<int>() { return 0; }

constexpr int HETRD_NB = 32;   // panel width of the tridiagonalisation
constexpr int HETRD_TILE = 64; // tile edge of the trailing symmetric product
constexpr int HETRD_SCH = 4;      // default tiles per workgroup of the trailing symmetric product
constexpr int HETRD_SCH_MIN = 2;  // smallest candidate (sizes the partial buffers)
constexpr int BACKTR_BT = 256;  // largest number of reflectors per compact-WY block of the back-transform
constexpr int BACKTR_SUB = 64;  // reflectors per triangular factor solved directly (a power of two)
// reflectors per compact-WY block for a given order: 256 from order 4096 up
// (rank-256 updates run on the large-tile GEMM), 128 below (smaller orders
// pay more for the larger factors than they gain)
inline int backtr_block(int order) { return order >= 4096 ? 256 : 128; }
constexpr int DC_LEAF_MIN = 16;  // smallest leaf the autotuner tries (the workspace fits its tree)

// Large GEMM tiles from this inner dimension on (KS_TUNE_NEVER: never), for
// the launches the calling thread enqueues; GemmPolicy sets it for a scope.
void gemm_set_big_min_k(int k);
int gemm_big_min_k();
struct GemmPolicy {
    int prev;
    explicit GemmPolicy(int k) : prev(gemm_big_min_k()) { gemm_set_big_min_k(k); }
    ~GemmPolicy() { gemm_set_big_min_k(prev); }
};
constexpr int DC_LEAF = 32;    // largest divide-and-conquer leaf
constexpr int MAX_KW = 64;     // k-point weights passed by value

struct KWeights {
    double w[MAX_KW];
};

// Event-based profiler of a plan: phases of the solve and sampled launches of
// the trailing matrix-vector kernel of the tridiagonalisation.  Host code only;
// events are recorded on the plan's stream and read back on request.
struct Prof {
    bool on = false;
    int stride = 1;
    long counter = 0;
    hipStream_t s = nullptr;
    struct Rec {
        int tag;
        hipEvent_t a, b;
        double bytes;
    };
    std::vector<hipEvent_t> pool;
    std::vector<Rec> recs;
    hipEvent_t rec_event() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            return nullptr;
        }
        (void)hipEventRecord(e, s);
        return e;
    }
    hipEvent_t begin() { return on ? rec_event() : nullptr; }
    // an unrecorded event, for a launch that records it itself
    hipEvent_t take() {
        hipEvent_t e = nullptr;
        if (!pool.empty()) {
            e = pool.back();
            pool.pop_back();
        } else if (hipEventCreate(&e) != hipSuccess) {
            return nullptr;
        }
        return e;
    }
    void push(int tag, hipEvent_t a, hipEvent_t b, double bytes) {
        if (a && b) recs.push_back({tag, a, b, bytes});
    }
    void end(int tag, hipEvent_t a, double bytes = 0.0) {
        if (!on || !a) return;
        hipEvent_t b = rec_event();
        if (b) recs.push_back({tag, a, b, bytes});
    }
    bool sample() { return on && (counter++ % stride == 0); }
    ~Prof() {
        for (auto& r : recs) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};
constexpr int PROF_HEMV = 100;  // tag of the sampled kernel

template <typename T>
struct HetrdWork {
    Prof* prof = nullptr;
    T* VW;          // 2NB x n   V then W of the current panel, transposed
    T* WV;          // 2NB x n   conj(W) then conj(V), transposed
    T* x;           // n         updated column
    T* partPQ;      // 2 x cdiv(n, 64) x (1 + 2NB) partial |x|^2, W^H x, V^H x; one buffer
                    // per column parity, sbuf apart
    T* prow;        // nt x cdiv(nt, HETRD_SCH_MIN) x HETRD_TILE, nt = cdiv(n, HETRD_TILE): row partials
    T* pcol;        // nt x nt x HETRD_TILE                                           column partials
    double* pvav;   // partial x^H A x of the product's workgroups (at most nt x cdiv(nt, HETRD_SCH_MIN))
    T* pq;          // 5 + 2 NB: x_{k+1}, unused, raw W^H x, V^H x of the current column,
                    // then the reflector's s, tau and beta
    void* VWlo = nullptr;  // mixed form: VW and WV in FP32 for the trailing update
    void* WVlo = nullptr;
    // strides (elements) between the buffers of consecutive matrices of a batch
    long sVW = 0, sx = 0, spart = 0, sprow = 0, spcol = 0, spvav = 0, spq = 0;
    long sbuf = 0;  // offset of the odd-column partial buffer
    // batches of two or more: the stream of the second half and the events that
    // fork it from and join it back to the caller's stream (none: one stream)
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    int sch = HETRD_SCH;  // tiles per workgroup of the symmetric product (tuned per plan)
    // tuned per column segment: columns from seg_first[i] use seg_sch[i]
    int nseg = 0;
    int seg_first[KS_TUNE_SEGMENTS] = {};
    int seg_sch[KS_TUNE_SEGMENTS] = {};
    int sch_for(int k) const {
        int v = sch;
        for (int i = 0; i < nseg; ++i)
            if (k >= seg_first[i]) v = seg_sch[i];
        return v;
    }
};

template <typename T>
struct BacktrWork {
    T* G;         // BT x BT per matrix: V_b^H V_b
    T* W1;        // BT x n per matrix
    T* W2;        // BT x n per matrix
    T* P;         // split-K partial products
    long pelems;  // capacity of P in elements
    T* Tall;      // cdiv(n-1, BT) x BT x BT per matrix: the compact-WY factors
    long sTall;   // matrix stride of Tall
    int bt = BACKTR_BT;  // reflectors per block for this plan's order (a multiple of BACKTR_SUB)
};

// Buffers of the two-stage reduction (ks_band.hip) for one element type; every
// pointer holds `batch` consecutive per-matrix buffers of the given stride.
template <typename T>
struct BandWork {
    T* X = nullptr;      long sX = 0;     // order x KB: A22 V of a panel
    T* buf3 = nullptr;   long sbuf = 0;   // order x 3KB: [V | X T, then W | V] of a panel
    T* Tf = nullptr;     long sTf = 0;    // KB x KB: compact-WY factor of a panel
    T* M = nullptr;      T* N = nullptr;  // KB x KB each (stride KB^2): V^H X T, T^H V^H X T
    T* rec = nullptr;    long srec = 0;   // 2 x pmax x 2KB: per-workgroup partial sums of a panel column
    int* cnt = nullptr;  long scnt = 0;   // one arrival counter per panel
    int* gprog = nullptr; long sgp = 0;   // bulge chasing: progress of each workgroup's last sweep
    int* abort_ = nullptr;                // set by a wait that gave up: every wait then leaves
    T* Vpk = nullptr;    long sVpk = 0;   // J x Tmax x Q2_NB x KB: bulge-chasing reflectors per group
    T* taupk = nullptr;  long staupk = 0; // J x Tmax x Q2_NB
    int* q2prog = nullptr;                // stage-2 back-transform: progress per (pass block, matrix, 64-column slice)
    T* P = nullptr;      long pelems = 0; // split-K partial products (shared with the back-transform)
    int ncu = 1;                          // compute units: every workgroup of a waiting kernel must be resident
};

// Divide-and-conquer scratch; all position-indexed arrays have n entries and
// each merge uses the slice [lo, hi) of its rows.
struct DcWork {
    double* dw;
    double* ds;
    double* zs;
    int* perm;
    int* ndl;
    int* dfl;
    double* dfval;
    double* dnd;
    double* znd;
    int* rot_idx;   // 2 n
    double* rot_cs; // 2 n
    int* orig;
    double* tau;
    double* zhat;
    double* cinv;
    double* fval;
    int* fsrc;
    int* kk;        // per merge of the current level
    int* kk1;       // per merge: kept columns of the first child (< 0: columns not grouped)
    int* gpos;      // kept entry (secular order) -> its column in the child-grouped order
    int* nrot;
    double* rho;
};

struct DcTree {
    int n = 0, depth = 0, nleaf = 0, nmerge_total = 0;
    std::vector<int> max_k0;  // per level (index = level)
    int* d_mlo = nullptr;     // merges, level l at offset 2^l - 1
    int* d_mmid = nullptr;
    int* d_mhi = nullptr;
    int* d_mid_all = nullptr; // same as d_mmid (all tears)
    int* d_leaf_lo = nullptr;
    int* d_leaf_hi = nullptr;
};

template <typename T>
void fill_zero(hipStream_t s, T* p, long n);

// Cholesky S = L L^H in place in L (lower) and L^-1 into Li (lower, zeros
// above) for a batch (strides sl, si); work holds n^2/4 elements per matrix
// (stride sw).  A failing pivot records its 1-based column in info.
template <typename T>
void potrf_inv(hipStream_t s, int n, T* L, int ldl, long sl, T* Li, int ldi, long si, T* work, long sw,
               int batch, int* info);



template <typename T>
void herm_complete(hipStream_t s, int n, const T* src, int lds, long ss, T* dst, int ldd, long sd,
                   int batch, int* info);

// X[i][j] = conj(X[j][i]) for j > i (the upper triangle from the lower one),
// in place, for a batch of n x n matrices.
template <typename T>
void mirror_lower(hipStream_t s, int n, T* X, int ldx, long sx, int batch);

// A = (I (x) Linv) H (I (x) Linv)^H for a batch (H: row stride ldh, matrix
// stride sH; Linv: n x n, stride sL; A, W: order x order, consecutive).  With
// lower_only only the lower triangle of A is formed (all the tridiagonalisation
// reads), which halves the second product.
template <typename T>
void reduce_to_standard(hipStream_t s, int n, int nsp, int batch, const T* H, int ldh, long sH, const T* Linv,
                        int ldi, long sL, T* A, T* W, int* info, bool lower_only = false);

// A real overlap given in complex storage: dst (n x n real, ld ldd, stride sd)
// = Re of the symmetric completion of src's lower triangle.  An imaginary part
// other than zero on or below the diagonal records KS_ERR_INVALID_ARG (info =
// its 1-based row), a non-finite entry KS_ERR_NONFINITE.
void real_sym_complete(hipStream_t s, int n, const cplx* src, int lds, long ss, double* dst, int ldd, long sd,
                       int batch, int* info);

// The reduction of a complex H with a real factor Linv (real overlap):
// A = M H M^T with M = I (x) Linv.  Both products take the complex matrices
// as real ones of interleaved (re, im) columns, so a product with M costs two
// real products per complex one instead of three; the right-hand product is
// A = M (M H)^H (H Hermitian, M real), a conjugate transpose and a second
// left product.  Same arguments and lower_only meaning as reduce_to_standard.
void reduce_to_standard_real(hipStream_t s, int n, int nsp, int batch, const cplx* H, int ldh, long sH,
                             const double* Linv, int ldi, long sL, cplx* A, cplx* W, int* info,
                             bool lower_only = false);



template <typename T, typename S>
void hetrd(hipStream_t s, int n, S* A, int lda, long sA, int batch, double* d, double* e, T* tau, T* Vall,
           HetrdWork<T>& w);

// Tiles-per-workgroup candidates of the symmetric product for element type T,
// and the time of `reps` launches of each at a few trailing sizes of an order-n
// batch (the matrix contents do not matter for the timing).  Writes the
// candidates to cand[] and times (ms) to ms[]; returns their number.
template <typename T, typename S>
int hetrd_tune(hipStream_t s, int n, S* A, int lda, long sA, int batch, double* d, double* e, T* tau,
               HetrdWork<T>& w, int* cand, double* ms, int reps, int* seg_first, int* seg_tiles);

// Two-stage reduction of a batch of Hermitian matrices (A: order n, row
// stride lda, matrix stride sA; the lower triangle is read) to real symmetric
// tridiagonal form: he2hb reduces A to a band of half-bandwidth KB (panel QR
// + two-sided rank-2KB updates on the matrix cores) and leaves the panel
// reflectors in Vall (n x n per matrix, reflector c in column c from row c+KB
// on, zeros elsewhere) with tau; hb2st chases the band to tridiagonal form
// (d, e: stride n) and keeps its reflectors grouped for q2_apply, which forms
// X <- Q2 X for the n x ncols blocks of X.  A wait that gives up (a resident
// workgroup never arrived) records KS_ERR_NO_CONVERGENCE with detail -1
// (stage 1), -2 (stage 2) or -3 (stage-2 back-transform) and every kernel
// still ends.
template <typename T>
void he2hb(hipStream_t s, int n, T* A, int lda, long sA, int batch, T* Vall, T* tau, BandWork<T>& w, int* info);
template <typename T>
void hb2st(hipStream_t s, int n, T* A, int lda, long sA, int batch, double* d, double* e, BandWork<T>& w,
           int* info);
template <typename T>
void q2_apply(hipStream_t s, int n, int batch, int ncols, T* X, int ldx, long sX, BandWork<T>& w, int* info);

// Divide and conquer for a batch of tridiagonals of order tr.n (d, e, lam:
// stride n; Z, Z2, U, Qp: stride n^2; the work arrays of w: stride n, with
// kk, nrot, rho holding batch x (merges of the widest level)).
void stedc(hipStream_t s, const DcTree& tr, int batch, const double* d, const double* e, double* lam,
           double* Z, double* Z2, double* U, double* Qp, DcWork& w, int* info);

// Test hook: iteration caps of the leaf Jacobi and the secular solver (<= 0
// restores the defaults, 40 sweeps and 120 iterations).
void stedc_set_caps(int leaf_sweeps, int secular_iters);

void dc_tree_host(int n, int leaf, std::vector<int>& mlo, std::vector<int>& mmid, std::vector<int>& mhi,
                  std::vector<int>& leaf_lo, std::vector<int>& leaf_hi, int& depth,
                  std::vector<int>& max_k0);

// Z columns [c0, c0 + ncols) of each matrix of a batch (Z: n x n, consecutive)
// into X (n x ncols, row stride ldx, matrix stride sX).
template <typename T>
void load_z(hipStream_t s, int n, int batch, int ncols, const double* Z, int c0, T* X, int ldx, long sX);

// The compact-WY factors of every block of reflectors of a batch (Vall: n x n
// per matrix, the tridiagonalisation's layout; tau: n per matrix) into w.Tall.
template <typename T>
void backtransform_prepare(hipStream_t s, int n, int batch, const T* Vall, const T* tau, BacktrWork<T>& w);

// X <- Q X (or Q^H X with adjoint) for a batch, with the factors prepared above.
template <typename T>
void backtransform_q(hipStream_t s, int n, int batch, const T* Vall, int ncols, T* X, int ldx, long sX,
                     BacktrWork<T>& w, bool adjoint = false);

void fermi(hipStream_t s, int batch, int order, const double* eps, const KWeights& kw, double g,
           double ne, double kT, int il, int iu, double* occ, double* mu, double* eband, int* kwin,
           int* info);

template <typename T>
void density_backward(hipStream_t s, int n, int nsp, int batch, const double* eps, const T* C, int ldc,
                      const double* mu, double kT, double g, const KWeights& kw, const T* grad_rho,
                      const double* grad_eband, T* grad_H, T* grad_S, int lds, T* W1, T* W2, T* W3,
                      double* scal);

// ---------------------------------------------------------------- mixed precision
// Element kernels of the mixed-precision solve (ks_mixed.hip); every one takes
// a batch of matrices (blockIdx.y) with the given element strides.
template <typename Src, typename Dst>
void convert(hipStream_t s, int batch, int rows, int cols, const Src* src, int lds, long ss, Dst* dst, int ldd,
             long sd);
template <typename T>
void residual(hipStream_t s, int batch, int order, int m, const T* Y, const T* X, long sm, const double* lam,
              long sl, int c0, T* R);
void correction_scale(hipStream_t s, int batch, int order, int m, int w, float* P, long sp, const double* lam,
                      long sl, int c0);
// The window's eigenproblem inside the refined subspace span(X) (X: order x M,
// ld M, matrix stride sX): with G = X^H A X given (M x M, ld M) and B = X^H X
// formed here, `passes` refinement passes in M-space (first-order correction
// between clusters, an exact small solve inside each cluster of nearly equal
// values) give W with W^H B W = I, W^H G W diagonal; X <- X W with its columns
// in ascending order of the values, which go to eps[c0 ..] (matrix stride se).
// Tm, W, Tmp: M x M scratch; theta: M per matrix (stride st); cstart, csize,
// rank: M ints per matrix (stride sc); Y: order x M scratch.
template <typename T>
void subspace_refine(hipStream_t s, int batch, int order, int M, T* X, long sX, T* Y, T* G, T* Bm, T* Tm, T* W,
                     T* Tmp, double* theta, long st, int* cstart, int* csize, int* rank, long sc, double* eps,
                     long se, int c0, int passes);
template <typename T, typename S>
void sub_widened(hipStream_t s, int batch, long cnt, T* X, const S* D, long sm);
void put_window(hipStream_t s, int batch, int m, const double* theta, long st, double* eps, long se, int c0);
void merge_info(hipStream_t s, int* inner, int* outer);

}  // namespace ks

// Stage drivers behind the test hooks (defined in ks_api.hip).
void ks_internal_stedc(ks_plan* p, const double* d, const double* e, double* lam, double* Z);
void ks_internal_hetrd(ks_plan* p, void* A, double* d, double* e, const double* X, int ncols, void* Y);
void ks_internal_he2hb(ks_plan* p, void* A, const double* X, int ncols, void* Y);
