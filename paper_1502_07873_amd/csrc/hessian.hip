// Receiver Jacobian and Gauss-Newton Hessian, FP64 on the device.
//
// From the 14 deviation solves of a sample (traces of g(theta +- d_j e_j) -
// g(theta), FP32) the central differences J_j = (w+_j - w-_j) / (2 d_j) are
// formed in FP64 (or, from the 7 sensitivity solves of Algorithm 1, the
// traces are the columns J_j themselves), and H_1 = sigma^-2 sum_{m,r,c}
// J^T J accumulated (paper
// Theorem 2, H_1 with C_eps = sigma^2 I; Section 3.3.2, H_I, whose
// receiver-selection Hessian is diagonal).  Every thread owns a fixed subset
// of the (level, receiver) pairs and the 28 distinct products are reduced
// with wavefront shuffles and LDS in a fixed order, so the result does not
// depend on how solves were batched.
#include "internal.h"

namespace eig {

namespace {

constexpr int kTri = kNT * (kNT + 1) / 2;  // 28

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// A sample of n elements is cut into sample_ranges(n) ranges: at least
// kRangeMin elements each (so the block partials stay cheap next to the
// sums), at most kSampleSplit.  The count depends on n alone.
__device__ __forceinline__ int sample_ranges(int n) {
    return min(kSampleSplit, max(1, n / kRangeMin));
}

__device__ __forceinline__ void sample_range(int n, int b, int& lo, int& hi) {
    const int nr = sample_ranges(n);
    const int chunk = (n + nr - 1) / nr;
    lo = min(n, b * chunk);
    hi = min(n, lo + chunk);
}

// Stability of the leapfrog step at free node (i, k): the larger of the two
// absolute row sums (x and depth components) of B = -dt^2 rho^-1 A_h, the
// operator the stencil kernels apply (a = lambda + 2 mu; n, m: the rows
// below and above; R, L: the columns right and left; rigid neighbours are
// counted too, which only raises the bound).  The step u^{m+1} = (2 - B) u^m
// - u^{m-1} keeps a positive conserved energy when every eigenvalue of B is
// at most 4; by Gershgorin's theorem that holds when every row sum is, so a
// return value <= 1 guarantees stability.
__device__ double stability_bound(const SampleDesc& sd, int i, int k) {
    const int nx = sd.nx;
    const bool nodal = sd.med_kind == EIG_MEDIUM_NODAL;
    auto at = [&](const double* a, int ii, int kk) {
        return a[nodal ? (size_t)kk * nx + ii : (size_t)kk];
    };
    const double* L = sd.lam;
    const double* M = sd.mu;
    const double l = at(L, i, k), m = at(M, i, k), ac = l + 2.0 * m;
    const double lR = at(L, i + 1, k), mR = at(M, i + 1, k), aR = lR + 2.0 * mR;
    const double lL = at(L, i - 1, k), mL = at(M, i - 1, k), aL = lL + 2.0 * mL;
    const double ln = at(L, i, k + 1), mn = at(M, i, k + 1), an = ln + 2.0 * mn;
    double ru, rv;
    if (k == 0) {  // traction-free row
        ru = (ac + aR) + (aL + ac) + 2.0 * (m + mn) +
             0.5 * (fabs(lR + mn) + fabs(m - lR) + fabs(lL + mn) + fabs(lL - m));
        rv = (m + mR) + (mL + m) + 2.0 * (ac + an) +
             0.5 * (fabs(ln + mR) + fabs(l - mR) + fabs(ln + mL) + fabs(l - mL));
    } else {
        const double lm = at(L, i, k - 1), mm = at(M, i, k - 1), am = lm + 2.0 * mm;
        ru = (ac + aR) + (aL + ac) + (m + mn) + (mm + m) +
             0.25 * (fabs(lR + mn) + fabs(lL + mn) + fabs(lR + mm) + fabs(lL + mm));
        rv = (m + mR) + (mL + m) + (ac + an) + (am + ac) +
             0.25 * (fabs(ln + mR) + fabs(ln + mL) + fabs(lm + mR) + fabs(lm + mL));
    }
    return sd.dt2_h2 / at(sd.rho, i, k) * fmax(ru, rv) * 0.25;
}

// Per-sample status and noise level.  mode EIG_SIGMA_GIVEN: sigma = given;
// EIG_SIGMA_NOMINAL_PEAK: sigma = given * max |nominal trace value|.
// Block (s, b) covers range b of sample s's trace elements and of its free
// nodes and leaves the trace maximum, the non-finite flag and the largest
// stability bound in work (the maximum of a set and the flag do not depend on
// how the set is cut); sample_check_finish_kernel combines the ranges.
__global__ void __launch_bounds__(256)
sample_check_kernel(const SampleDesc* __restrict__ samples, double* __restrict__ work) {
    const SampleDesc& sd = samples[blockIdx.x];
    const int nr = sample_ranges(sd.nt * sd.nrec);
    if ((int)blockIdx.y >= nr) return;
    int lo, hi;
    sample_range(sd.nt * sd.nrec, blockIdx.y, lo, hi);
    // free nodes whose bound is checked: the rows of a depth-only medium (its
    // bound does not vary along x), every free node of a nodal one
    double gmax = 0.0;
    if (sd.rho) {
        const bool nodal = sd.med_kind == EIG_MEDIUM_NODAL;
        const int ncol = nodal ? sd.nx - 2 : 1;
        const long long nnode = (long long)ncol * (sd.nz - 1);
        const long long chunk = (nnode + nr - 1) / nr;
        const long long n0 = min(nnode, (long long)blockIdx.y * chunk);
        const long long n1 = min(nnode, n0 + chunk);
        for (long long q = n0 + threadIdx.x; q < n1; q += blockDim.x) {
            const int k = (int)(q / ncol), i = 1 + (int)(q % ncol);
            gmax = fmax(gmax, stability_bound(sd, i, k));
        }
    }
    float mx = 0.f;
    int bad = 0;
    for (int e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        const float2 v = sd.nominal[e];
        if (!isfinite(v.x) || !isfinite(v.y)) bad = 1;
        mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
    }
    for (int j = 0; j < 2 * kNT && !bad; ++j)
        for (int e = lo + threadIdx.x; e < hi && sd.dev[j]; e += blockDim.x) {
            const float2 v = sd.dev[j][e];
            if (!isfinite(v.x) || !isfinite(v.y)) { bad = 1; break; }
        }
    __shared__ float smx[256];
    __shared__ int sbad[256];
    __shared__ double sg[256];
    smx[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    sg[threadIdx.x] = gmax;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            smx[threadIdx.x] = fmaxf(smx[threadIdx.x], smx[threadIdx.x + o]);
            sbad[threadIdx.x] |= sbad[threadIdx.x + o];
            sg[threadIdx.x] = fmax(sg[threadIdx.x], sg[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double* w = work + 3 * ((size_t)blockIdx.x * kSampleSplit + blockIdx.y);
        w[0] = (double)smx[0];
        w[1] = (double)sbad[0];
        w[2] = sg[0];
    }
}

__global__ void sample_check_finish_kernel(const SampleDesc* __restrict__ samples,
                                           const double* __restrict__ work, int nsample,
                                           const double* __restrict__ given, int mode,
                                           double* __restrict__ sigma,
                                           int32_t* __restrict__ status) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsample) return;
    float mx = 0.f;
    int bad = 0;
    double gmax = 0.0;
    const int nr = sample_ranges(samples[s].nt * samples[s].nrec);
    for (int b = 0; b < nr; ++b) {
        const double* w = work + 3 * ((size_t)s * kSampleSplit + b);
        mx = fmaxf(mx, (float)w[0]);
        bad |= w[1] != 0.0;
        gmax = fmax(gmax, w[2]);
    }
    const double g = given[s];
    // a step the bound does not vouch for poisons the sample's H_1 (through
    // a NaN noise level) as a non-finite solve does through its traces
    const bool unstable = !(gmax <= 1.0);
    sigma[s] = unstable ? __longlong_as_double(0x7ff8000000000000ULL)
                        : (mode == EIG_SIGMA_NOMINAL_PEAK ? g * (double)mx : g);
    if (status) status[s] = bad ? EIG_ENONFINITE : (unstable ? EIG_EUNSTABLE : EIG_OK);
}

// Block (s, b) sums J^T J (and J^T r for the gradient) over range b of
// sample s's (level, receiver) elements and leaves the kTri + kNT sums in
// work; hessian_finish_kernel adds the ranges in order and scales.
__global__ void __launch_bounds__(256)
hessian_kernel(const SampleDesc* __restrict__ samples, const double* __restrict__ sigma,
               double* __restrict__ work) {
    const int s = blockIdx.x;
    const SampleDesc& sd = samples[s];
    const int nt = sd.nt, nrec = sd.nrec;
    if ((int)blockIdx.y >= sample_ranges(nt * nrec)) return;
    double acc[kTri + kNT];
    for (int t = 0; t < kTri + kNT; ++t) acc[t] = 0.0;
    const bool want_grad = sd.grad != nullptr;
    const double sgm = sigma[s];
    double inv2d[kNT];
    for (int j = 0; j < kNT; ++j) inv2d[j] = sd.inv2d[j];
    int lo, hi;
    sample_range(nt * nrec, blockIdx.y, lo, hi);
    for (int e = lo + threadIdx.x; e < hi; e += blockDim.x) {
        double Jx[kNT], Jz[kNT];
        for (int j = 0; j < kNT; ++j) {
            const float2 p = sd.dev[2 * j][e];
            if (sd.dev[2 * j + 1]) {
                const float2 n = sd.dev[2 * j + 1][e];
                Jx[j] = ((double)p.x - (double)n.x) * inv2d[j];
                Jz[j] = ((double)p.y - (double)n.y) * inv2d[j];
            } else {  // sensitivity solve: the traces are the column itself
                Jx[j] = (double)p.x;
                Jz[j] = (double)p.y;
            }
        }
        if (sd.J) {
            double* o = sd.J + (size_t)e * 2 * kNT;
            for (int j = 0; j < kNT; ++j) {
                o[j] = Jx[j];
                o[kNT + j] = Jz[j];
            }
        }
        int t = 0;
        for (int a = 0; a < kNT; ++a)
            for (int b = a; b < kNT; ++b, ++t) acc[t] += Jx[a] * Jx[b] + Jz[a] * Jz[b];
        if (want_grad) {
            const float2 ys = sd.ystar[e], nm = sd.nominal[e], ns = sd.noise[e];
            const double rx = ((double)ys.x - (double)nm.x) + sgm * (double)ns.x;
            const double rz = ((double)ys.y - (double)nm.y) + sgm * (double)ns.y;
            for (int j = 0; j < kNT; ++j) acc[kTri + j] += Jx[j] * rx + Jz[j] * rz;
        }
    }
    __shared__ double part[kWavesPerBlock][kTri + kNT];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int t = 0; t < kTri + (want_grad ? kNT : 0); ++t) {
        const double v = wave_sum(acc[t]);
        if (lane == 0) part[wave][t] = v;
    }
    __syncthreads();
    if (threadIdx.x < kTri + (want_grad ? kNT : 0)) {
        const int t = threadIdx.x;
        double v = 0.0;
        for (int w = 0; w < kWavesPerBlock; ++w) v += part[w][t];
        work[((size_t)s * kSampleSplit + blockIdx.y) * (kTri + kNT) + t] = v;
    }
}

__global__ void hessian_finish_kernel(const SampleDesc* __restrict__ samples,
                                      const double* __restrict__ sigma,
                                      const double* __restrict__ work,
                                      double* __restrict__ H1) {
    const int s = blockIdx.x, t = threadIdx.x;
    const SampleDesc& sd = samples[s];
    const bool want_grad = sd.grad != nullptr;
    if (t >= kTri + (want_grad ? kNT : 0)) return;
    double v = 0.0;
    const int nr = sample_ranges(sd.nt * sd.nrec);
    for (int b = 0; b < nr; ++b)
        v += work[((size_t)s * kSampleSplit + b) * (kTri + kNT) + t];
    const double sg = sigma[s];
    if (t >= kTri) {
        sd.grad[t - kTri] = -v / (sg * sg);
        return;
    }
    v /= sg * sg;
    // map t back to (a, b)
    int a = 0, base = 0;
    while (t >= base + (kNT - a)) { base += kNT - a; ++a; }
    const int b = a + (t - base);
    double* H = H1 + (size_t)s * kNT * kNT;
    H[a * kNT + b] = v;
    H[b * kNT + a] = v;
}

// Per-receiver H_1 (design evaluation needs one H_1 per candidate): a
// sample's levels are cut into receiver_splits(nt) contiguous ranges of at
// least kRecvLevelsMin levels, at most kRecvSplit of them, one block each;
// in a block a thread owns receivers r = threadIdx.x, + blockDim.x, ... and
// sums that receiver's levels of the range in order, so consecutive threads
// read consecutive receivers of a level (the traces are
// [level][receiver][2]).  The partial sums go to work as [range][entry]
// [receiver] (coalesced) and the finishing kernel adds the ranges in order.
// The cut depends on nt alone, so a sample's result does not depend on the
// batch.  Same Jacobian columns, products and scaling as hessian_kernel.
__device__ __forceinline__ int receiver_splits(int nt) {
    return min(kRecvSplit, max(1, nt / kRecvLevelsMin));
}

__global__ void __launch_bounds__(256)
hessian_receiver_kernel(const SampleDesc* __restrict__ samples, size_t stride,
                        double* __restrict__ work) {
    const int s = blockIdx.x;
    const SampleDesc& sd = samples[s];
    const int nt = sd.nt, nrec = sd.nrec;
    const int nb = receiver_splits(nt);
    if ((int)blockIdx.y >= nb) return;
    const int lo = (int)((long long)nt * blockIdx.y / nb);
    const int hi = (int)((long long)nt * (blockIdx.y + 1) / nb);
    double inv2d[kNT];
    for (int j = 0; j < kNT; ++j) inv2d[j] = sd.inv2d[j];
    double* w = work + (size_t)s * stride + (size_t)blockIdx.y * kTri * nrec;
    for (int r = threadIdx.x; r < nrec; r += blockDim.x) {
        double acc[kTri];
        for (int t = 0; t < kTri; ++t) acc[t] = 0.0;
        for (int q = lo; q < hi; ++q) {
            const int e = q * nrec + r;
            double Jx[kNT], Jz[kNT];
            for (int j = 0; j < kNT; ++j) {
                const float2 p = sd.dev[2 * j][e];
                if (sd.dev[2 * j + 1]) {
                    const float2 n = sd.dev[2 * j + 1][e];
                    Jx[j] = ((double)p.x - (double)n.x) * inv2d[j];
                    Jz[j] = ((double)p.y - (double)n.y) * inv2d[j];
                } else {  // sensitivity solve: the traces are the column itself
                    Jx[j] = (double)p.x;
                    Jz[j] = (double)p.y;
                }
            }
            if (sd.J) {
                double* o = sd.J + (size_t)e * 2 * kNT;
                for (int j = 0; j < kNT; ++j) {
                    o[j] = Jx[j];
                    o[kNT + j] = Jz[j];
                }
            }
            int t = 0;
            for (int a = 0; a < kNT; ++a)
                for (int b = a; b < kNT; ++b, ++t) acc[t] += Jx[a] * Jx[b] + Jz[a] * Jz[b];
        }
        for (int t = 0; t < kTri; ++t) w[(size_t)t * nrec + r] = acc[t];
    }
}

__global__ void __launch_bounds__(256)
hessian_receiver_finish_kernel(const SampleDesc* __restrict__ samples, int ngroup,
                               const double* __restrict__ sigma, size_t stride,
                               const double* __restrict__ work, double* __restrict__ H1) {
    const int s = blockIdx.x;
    const SampleDesc& sd = samples[s];
    const int nrec = sd.nrec;
    const int nb = receiver_splits(sd.nt);
    const double sg = sigma[s];
    const double* w = work + (size_t)s * stride;
    for (int r = threadIdx.x; r < nrec; r += blockDim.x) {
        double* H = H1 + ((size_t)s * ngroup + r) * kNT * kNT;
        int t = 0;
        for (int a = 0; a < kNT; ++a)
            for (int b = a; b < kNT; ++b, ++t) {
                double v = 0.0;
                for (int k = 0; k < nb; ++k) v += w[((size_t)k * kTri + t) * nrec + r];
                v = v / (sg * sg);
                H[a * kNT + b] = v;
                H[b * kNT + a] = v;
            }
    }
}

__global__ void surface_peak_kernel(const float2* __restrict__ tr, int count,
                                    double rel, double* __restrict__ out) {
    float mx = 0.f;
    for (int e = threadIdx.x; e < count; e += blockDim.x) {
        const float2 v = tr[e];
        mx = fmaxf(mx, fmaxf(fabsf(v.x), fabsf(v.y)));
        if (!isfinite(v.x) || !isfinite(v.y)) mx = __int_as_float(0x7fc00000);
    }
    __shared__ float smx[256];
    smx[threadIdx.x] = mx;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const float a = smx[threadIdx.x], b = smx[threadIdx.x + o];
            smx[threadIdx.x] = (isnan(a) || isnan(b)) ? __int_as_float(0x7fc00000) : fmaxf(a, b);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = rel * (double)smx[0];
}

}  // namespace

void launch_sample_check(const SampleDesc* samples, int nsample, const double* given,
                         int mode, double* sigma, int32_t* status, double* work,
                         hipStream_t s) {
    if (nsample <= 0) return;
    sample_check_kernel<<<dim3(nsample, kSampleSplit), 256, 0, s>>>(samples, work);
    sample_check_finish_kernel<<<(nsample + 63) / 64, 64, 0, s>>>(samples, work, nsample,
                                                                   given, mode,
                                                                   sigma, status);
}

void launch_hessian(const SampleDesc* samples, int nsample, int per_receiver,
                    int ngroup, const double* sigma, double* H1, double* work, hipStream_t s,
                    size_t receiver_stride) {
    if (nsample <= 0) return;
    if (per_receiver) {
        hessian_receiver_kernel<<<dim3(nsample, kRecvSplit), 256, 0, s>>>(
            samples, receiver_stride, work);
        hessian_receiver_finish_kernel<<<nsample, 256, 0, s>>>(samples, ngroup, sigma,
                                                               receiver_stride, work, H1);
        return;
    }
    hessian_kernel<<<dim3(nsample, kSampleSplit), 64 * kWavesPerBlock, 0, s>>>(samples, sigma,
                                                                             work);
    hessian_finish_kernel<<<nsample, 64, 0, s>>>(samples, sigma, work, H1);
}

void launch_surface_peak(const float2* traces, int count, double rel, double* out,
                         hipStream_t s) {
    surface_peak_kernel<<<1, 256, 0, s>>>(traces, count, rel, out);
}

}  // namespace eig
