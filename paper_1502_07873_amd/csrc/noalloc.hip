// Greedy receiver selection for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc).  Same kernels and reduction order as design_greedy; the
// scratch it needs (the prior, per-(sample, candidate) D^_KL values, the
// candidates' weighted sums, the running per-sample Hessian and the chosen
// flags) lives in one file-scope device array instead of the context's
// workspace, and the caller's inputs are device arrays.
#include <mutex>

#include "host.h"

namespace eig {

constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

// One copy per device, held until the process ends.  Host code must never
// pass `scratch` itself to a kernel or a copy: on the host it names a stand-in,
// not device memory.  Its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

__global__ void store_prior_kernel(eig_prior p, eig_prior* dst) { *dst = p; }

// Bytes the greedy search keeps in scratch, each piece 256-byte aligned.
struct ScratchPlan {
    size_t o_prior, o_work, o_ival, o_H, o_ch, end;
};

ScratchPlan plan(int nsample, int ncand) {
    Carve cv;
    ScratchPlan p;
    p.o_prior = cv.take(sizeof(eig_prior));
    p.o_work = cv.take((size_t)nsample * ncand * sizeof(double));
    p.o_ival = cv.take((size_t)ncand * sizeof(double));
    p.o_H = cv.take((size_t)nsample * kNT * kNT * sizeof(double));
    p.o_ch = cv.take((size_t)ncand);
    p.end = cv.off;
    return p;
}

}  // namespace

// Device address of this device's scratch array (the current device must be
// `device`), looked up once per device.
int noalloc_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices)
        return set_error(EIG_EUNSUPPORTED, "device index beyond the no-alloc scratch table");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return EIG_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return set_error(EIG_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                       hipGetErrorString(e));
    g_scratch_ptr[device] = (char*)p;
    return EIG_OK;
}

}  // namespace eig

extern "C" {

int design_greedy_noalloc(eig_ctx* c, int32_t nsample, int32_t ncand, const double* H1r,
                          const eig_prior* prior, const double* theta, const double* w,
                          int32_t kmax, int32_t* order, double* curve, void* stream) {
    if (!c) return set_error(EIG_EINVAL, "ctx is NULL");
    if (nsample <= 0 || ncand <= 0 || kmax <= 0 || !H1r || !w || !order || !curve || !prior)
        return set_error(EIG_EINVAL, "design_greedy_noalloc arguments");
    if (prior->active < 0 || prior->active >= (1 << kNT))
        return set_error(EIG_EINVAL, "prior active mask");
    if (prior->kind == EIG_PRIOR_UNIFORM) {
        for (int j = 0; j < kNT; ++j)
            if (!(prior->hi[j] > prior->lo[j])) return set_error(EIG_EINVAL, "prior box lo < hi");
    } else if (prior->kind == EIG_PRIOR_GAUSSIAN) {
        if (!theta) return set_error(EIG_EINVAL, "gaussian prior needs theta");
    } else {
        return set_error(EIG_EINVAL, "prior kind");
    }
    const ScratchPlan sp = plan(nsample, ncand);
    if (sp.end > kScratchBytes)
        return set_error(EIG_EBUDGET,
                         "design_greedy_noalloc: nsample * (ncand + 49) * 8 bytes (plus "
                         "small tables) exceed its " + std::to_string(kScratchBytes >> 20) +
                             " MiB scratch; use design_greedy");
    HIP_TRY(hipSetDevice(c->device));
    // looked up when the context was created; retried here if that failed
    const int rc = noalloc_scratch_init(c->device);
    if (rc) return rc;
    char* base = g_scratch_ptr[c->device];
    hipStream_t s = (hipStream_t)stream;
    eig_prior* dprior = (eig_prior*)(base + sp.o_prior);
    store_prior_kernel<<<1, 1, 0, s>>>(*prior, dprior);
    // the running Hessians and the chosen flags start at zero (kernels, not
    // memset: the call may be captured into a graph)
    launch_fill_zero(base + sp.o_H, (size_t)nsample * kNT * kNT * sizeof(double), s);
    launch_fill_zero(base + sp.o_ch, (size_t)ncand, s);
    // theta is only read for a Gaussian prior; a uniform prior's kernels get
    // a valid address they never dereference
    const double* th = theta ? theta : (const double*)(base + sp.o_work);
    for (int k = 0; k < kmax; ++k)
        launch_greedy_step(H1r, nsample, ncand, dprior, th, w, (double*)(base + sp.o_H),
                           (uint8_t*)(base + sp.o_ch), (double*)(base + sp.o_work),
                           (double*)(base + sp.o_ival), k, order, curve, s);
    HIP_TRY(hipGetLastError());
    return EIG_OK;
}

}  // extern "C"
