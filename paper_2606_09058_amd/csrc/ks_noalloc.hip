// ks_noalloc.hip -- ks_density_noalloc: the density build of ks_density
// (Fermi level by bisection, occupations, band energy, rho = C f C^H) for
// callers that cannot allocate device memory (code under stream capture, tight
// serving loops).  It takes a plan descriptor instead of a plan, so nothing is
// allocated before or during the call: the kernels' scratch (the occupied
// window count, and the occupations and the info word when the caller passes
// none) lives in one static device array of SCRATCH_BYTES per GPU, held until
// the process ends.  The kernels are ks_density's own, so the results equal
// ks_density's bit for bit.
#include <mutex>

#include "ks_internal.hpp"

using namespace ks;

// Scratch of the kernels of ks_density_noalloc: one copy per GPU, at its own
// address there; host code takes that address from hipGetSymbolAddress and
// never passes the symbol itself.
static __device__ __align__(256) unsigned char scratch[size_t(1) << 20];

namespace {

constexpr size_t SCRATCH_BYTES = sizeof(scratch);
constexpr size_t OFF_INFO = 0;    // int[2]
constexpr size_t OFF_KWIN = 256;  // int
constexpr size_t OFF_OCC = 512;   // double[batch * order]
constexpr size_t MAX_OCC = (SCRATCH_BYTES - OFF_OCC) / sizeof(double);
constexpr int MAX_DEVICES = 64;

std::mutex g_lock;
void* g_scratch[MAX_DEVICES] = {};  // device address of `scratch` on each device

// The device address of this device's copy of the array (looked up once per
// device, with that device current; host code never uses the symbol itself).
ks_status scratch_address(void** out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return KS_ERR_HIP;
    if (dev < 0 || dev >= MAX_DEVICES) return KS_ERR_NOT_SUPPORTED;
    std::lock_guard<std::mutex> g(g_lock);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return KS_ERR_HIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return KS_OK;
}

__global__ void clear_info_kernel(int* info) {
    if (threadIdx.x < 2) info[threadIdx.x] = 0;
}

}  // namespace

extern "C" ks_status ks_density_noalloc(const ks_plan_desc* d, const double* eps, const void* C, int32_t il,
                                        int32_t iu, double ne, double kT, const double* kweights, void* rho,
                                        double* mu, double* eband, double* occ, int32_t* info) {
    if (!d || !eps || !C || !rho || !mu || !eband) return KS_ERR_INVALID_ARG;
    if (d->n < 1 || d->batch < 1 || d->batch > MAX_KW) return KS_ERR_INVALID_ARG;
    if (d->dtype != KS_REAL64 && d->dtype != KS_COMPLEX128) return KS_ERR_INVALID_ARG;
    if (d->spin != KS_COLLINEAR && d->spin != KS_NONCOLLINEAR) return KS_ERR_INVALID_ARG;
    if (d->spin == KS_NONCOLLINEAR && d->dtype != KS_COMPLEX128) return KS_ERR_NOT_SUPPORTED;
    const int nsp = d->spin == KS_NONCOLLINEAR ? 2 : 1;
    const long order = (long)d->n * nsp;
    if (order > 60000 || d->ld_h < order) return KS_ERR_INVALID_ARG;
    if (il < 1 || il > iu || iu > order) return KS_ERR_INVALID_ARG;
    if (!(kT > 0.0) || !isfinite(kT)) return KS_ERR_INVALID_ARG;
    const double g = nsp == 2 ? 1.0 : 2.0;
    if (!(ne > 0.0) || !(ne <= g * order) || !isfinite(ne)) return KS_ERR_ELECTRON_COUNT;
    KWeights kw;
    for (int b = 0; b < MAX_KW; ++b) kw.w[b] = 0.0;
    for (int b = 0; b < d->batch; ++b) {
        if (kweights && (!(kweights[b] >= 0.0) || !isfinite(kweights[b]))) return KS_ERR_INVALID_ARG;
        kw.w[b] = kweights ? kweights[b] : 1.0 / d->batch;
    }
    // the occupations go to the static array only when the caller keeps none
    if (!occ && (size_t)d->batch * (size_t)order > MAX_OCC) return KS_ERR_ALLOC;
    void* base = nullptr;
    ks_status st = scratch_address(&base);
    if (st != KS_OK) return st;
    char* sp = (char*)base;
    int* inf = info ? (int*)info : (int*)(sp + OFF_INFO);
    int* kwin = (int*)(sp + OFF_KWIN);
    double* f = occ ? occ : (double*)(sp + OFF_OCC);
    hipStream_t s = (hipStream_t)d->stream;
    const int B = d->batch, ldh = d->ld_h, ncols = iu - il + 1;
    const long mat = order * ldh;
    // a failure is recorded only if none is recorded yet: clear the word (a
    // kernel, so that the call can be captured into a graph)
    hipLaunchKernelGGL(clear_info_kernel, dim3(1), dim3(64), 0, s, inf);
    fermi(s, B, (int)order, eps, kw, g, ne, kT, il, iu, f, mu, eband, kwin, inf);
    if (d->dtype == KS_COMPLEX128) {
        gemm<cplx>(s, OP_N, OP_C, (int)order, (int)order, ncols, 1.0, (const cplx*)C, ldh, mat, (const cplx*)C, ldh,
                   mat, 0.0, (cplx*)rho, ldh, mat, B, f + il - 1, order, UPLO_LOWER, kwin);
        mirror_lower<cplx>(s, (int)order, (cplx*)rho, ldh, mat, B);
    } else {
        gemm<double>(s, OP_N, OP_T, (int)order, (int)order, ncols, 1.0, (const double*)C, ldh, mat,
                     (const double*)C, ldh, mat, 0.0, (double*)rho, ldh, mat, B, f + il - 1, order, UPLO_LOWER,
                     kwin);
        mirror_lower<double>(s, (int)order, (double*)rho, ldh, mat, B);
    }
    if (hipPeekAtLastError() != hipSuccess) return KS_ERR_HIP;
    return KS_OK;
}
