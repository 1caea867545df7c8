// Laplace KL estimate, quadrature averages and design search, FP64.
//
// D^_KL(theta) = -1/2 log((2 pi)^N |H_1^-1|) - N/2 - h(theta)   (Theorem 4;
// N = 7, or the number of inferred parameters when the prior marks a subset)
// with log det H_1 taken through the scaled Hessian of Section 3.3.3,
// S = sqrt(diag H_1), H~ = S^-1 H_1 S^-1 = L L^T, so that the ~30 decades
// spanned by the raw entries never reach the factorisation;
// I = sum_s w_s D^_KL(theta_s) (Section 3.3.4, Monte Carlo or sparse
// quadrature).  Designs are receiver subsets (Section 4.5); H_1 is additive
// over receivers, so a design's H_1 is the sum of per-receiver Hessians.
#include "internal.h"

namespace eig {

namespace {

// log det of a symmetric n x n matrix (full storage, row stride n, n <= 7)
// via the scaled Cholesky factorisation; false if it is not positive
// definite or not finite.
__device__ bool scaled_logdet(const double* H, int n, double* out) {
    double s[kNT];
    double ld = 0.0;
    for (int j = 0; j < n; ++j) {
        const double d = H[j * n + j];
        if (!(d > 0.0) || !isfinite(d)) return false;
        s[j] = sqrt(d);
        ld += 2.0 * log(s[j]);
    }
    double L[kNT][kNT];
    for (int j = 0; j < n; ++j) {
        double v = H[j * n + j] / (s[j] * s[j]);
        for (int k = 0; k < j; ++k) v -= L[j][k] * L[j][k];
        if (!(v > 0.0) || !isfinite(v)) return false;
        L[j][j] = sqrt(v);
        ld += 2.0 * log(L[j][j]);
        for (int i = j + 1; i < n; ++i) {
            double w = H[i * n + j] / (s[i] * s[j]);
            for (int k = 0; k < j; ++k) w -= L[i][k] * L[j][k];
            L[i][j] = w / L[j][j];
        }
    }
    *out = ld;
    return true;
}

// Indices of the inferred parameters (all seven when the mask is 0).
__device__ int active_set(const eig_prior& pr, int* idx) {
    const int act = pr.active ? pr.active : (1 << kNT) - 1;
    int n = 0;
    for (int j = 0; j < kNT; ++j)
        if ((act >> j) & 1) idx[n++] = j;
    return n;
}

// h(theta) = log p(theta), the prior's marginal over the active parameters.
__device__ double log_prior(const eig_prior& pr, const double* th, const int* idx, int n) {
    if (pr.kind == EIG_PRIOR_UNIFORM) {
        double v = 0.0;
        for (int a = 0; a < n; ++a) v -= log(pr.hi[idx[a]] - pr.lo[idx[a]]);
        return v;
    }
    // Gaussian: -1/2 r^T C^-1 r - 1/2 (n log 2 pi + log det C), via C = L L^T
    double L[kNT][kNT];
    double ld = 0.0;
    for (int j = 0; j < n; ++j) {
        double v = pr.cov[idx[j] * kNT + idx[j]];
        for (int k = 0; k < j; ++k) v -= L[j][k] * L[j][k];
        L[j][j] = sqrt(v);
        ld += 2.0 * log(L[j][j]);
        for (int i = j + 1; i < n; ++i) {
            double w = pr.cov[idx[i] * kNT + idx[j]];
            for (int k = 0; k < j; ++k) w -= L[i][k] * L[j][k];
            L[i][j] = w / L[j][j];
        }
    }
    double y[kNT];
    double q = 0.0;
    for (int i = 0; i < n; ++i) {
        double v = th[idx[i]] - pr.mean[idx[i]];
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v / L[i][i];
        q += y[i] * y[i];
    }
    return -0.5 * q - 0.5 * (n * log(2.0 * M_PI) + ld);
}

// Theorem 4 on the active sub-block of a full 7x7 H_1.
__device__ bool dkl_of(const double* H, const eig_prior& pr, const double* th,
                       double* dkl, double* logdet) {
    int idx[kNT];
    const int n = active_set(pr, idx);
    double Hs[kNT * kNT];
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) Hs[a * n + b] = H[idx[a] * kNT + idx[b]];
    double ld;
    if (!scaled_logdet(Hs, n, &ld)) {
        *dkl = __longlong_as_double(0x7ff8000000000000ULL);
        *logdet = *dkl;
        return false;
    }
    *logdet = ld;
    *dkl = -0.5 * (n * log(2.0 * M_PI) - ld) - 0.5 * n - log_prior(pr, th, idx, n);
    return true;
}

// Cholesky of an n x n SPD matrix (row stride n); false if not SPD.
__device__ bool chol_n(const double* A, int n, double L[kNT][kNT]) {
    for (int j = 0; j < n; ++j) {
        double v = A[j * n + j];
        for (int k = 0; k < j; ++k) v -= L[j][k] * L[j][k];
        if (!(v > 0.0) || !isfinite(v)) return false;
        L[j][j] = sqrt(v);
        for (int i = j + 1; i < n; ++i) {
            double w = A[i * n + j];
            for (int k = 0; k < j; ++k) w -= L[i][k] * L[j][k];
            L[i][j] = w / L[j][j];
        }
    }
    return true;
}

// x = A^-1 b from the Cholesky factor of A.
__device__ void chol_solve(const double L[kNT][kNT], int n, const double* b, double* x) {
    double y[kNT];
    for (int i = 0; i < n; ++i) {
        double v = b[i];
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v / L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < n; ++k) v -= L[k][i] * x[k];
        x[i] = v / L[i][i];
    }
}

// Theorem 3 at theta^: H = H_1 + H_2 - grad grad h on the active parameters,
//   -1/2 log((2 pi)^N |H^-1|) - N/2 - h(theta^) - 1/2 tr(H^-1 grad grad h),
// grad grad h = 0 for the uniform prior and -Gamma^-1 for the Gaussian one.
__global__ void theorem3_kernel(const double* __restrict__ H1, const double* __restrict__ H2,
                                int nsample, const eig_prior* __restrict__ prior,
                                const double* __restrict__ theta, double* __restrict__ val,
                                int32_t* __restrict__ status) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsample) return;
    const eig_prior& pr = *prior;
    int idx[kNT];
    const int n = active_set(pr, idx);
    double H[kNT * kNT];
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            const size_t o = (size_t)s * kNT * kNT + idx[a] * kNT + idx[b];
            H[a * n + b] = H1[o] + H2[o];
        }
    double Gi[kNT * kNT];   // Gamma^-1 on the active parameters (Gaussian prior)
    bool ok = true;
    const bool gauss = pr.kind == EIG_PRIOR_GAUSSIAN;
    if (gauss) {
        double C[kNT * kNT], L[kNT][kNT];
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) C[a * n + b] = pr.cov[idx[a] * kNT + idx[b]];
        ok = chol_n(C, n, L);
        for (int c = 0; c < n && ok; ++c) {
            double e[kNT] = {0, 0, 0, 0, 0, 0, 0}, x[kNT];
            e[c] = 1.0;
            chol_solve(L, n, e, x);
            for (int a = 0; a < n; ++a) Gi[a * n + c] = x[a];
        }
        for (int a = 0; a < n * n && ok; ++a) H[a] += Gi[a];
    }
    double ld = 0.0;
    ok = ok && scaled_logdet(H, n, &ld);
    double tr = 0.0;   // tr(H^-1 Gamma^-1) = -tr(H^-1 grad grad h)
    if (ok && gauss) {
        double L[kNT][kNT];
        ok = chol_n(H, n, L);
        for (int c = 0; c < n && ok; ++c) {
            double col[kNT], x[kNT];
            for (int a = 0; a < n; ++a) col[a] = Gi[a * n + c];
            chol_solve(L, n, col, x);
            tr += x[c];
        }
    }
    const double th_nan = __longlong_as_double(0x7ff8000000000000ULL);
    val[s] = ok ? -0.5 * (n * log(2.0 * M_PI) - ld) - 0.5 * n -
                      log_prior(pr, theta + (size_t)s * kNT, idx, n) + 0.5 * tr
                : th_nan;
    if (status) status[s] = ok ? EIG_OK : EIG_ENOTPD;
}

__global__ void laplace_kernel(const double* __restrict__ H1, int nsample,
                               const eig_prior* __restrict__ prior,
                               const double* __restrict__ theta,
                               double* __restrict__ dkl, double* __restrict__ logdet,
                               int32_t* __restrict__ status) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsample) return;
    double H[kNT * kNT];
    for (int j = 0; j < kNT * kNT; ++j) H[j] = H1[(size_t)s * kNT * kNT + j];
    double v, ld;
    const bool ok = dkl_of(H, *prior, theta + (size_t)s * kNT, &v, &ld);
    dkl[s] = v;
    if (logdet) logdet[s] = ld;
    if (status) status[s] = ok ? EIG_OK : EIG_ENOTPD;
}

// out[r] = sum_s w[s] * x[r * n + s] for every row r (one block per row),
// summed in a fixed order: strided per-thread partials, then a tree.
__global__ void weighted_rows_kernel(const double* __restrict__ x, int n,
                                     const double* __restrict__ w,
                                     double* __restrict__ out,
                                     const uint8_t* __restrict__ skip) {
    const int r = blockIdx.x;
    __shared__ double part[256];
    double v = 0.0;
    for (int s = threadIdx.x; s < n; s += blockDim.x) v += w[s] * x[(size_t)r * n + s];
    part[threadIdx.x] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        out[r] = (skip && skip[r]) ? __longlong_as_double(0x7ff8000000000000ULL) : part[0];
}

__global__ void design_dkl_kernel(const double* __restrict__ H1r, int nsample,
                                  int ncand, const uint8_t* __restrict__ mask,
                                  const eig_prior* __restrict__ prior,
                                  const double* __restrict__ theta,
                                  double* __restrict__ work) {
    const int d = blockIdx.y;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsample) return;
    double H[kNT * kNT];
    for (int j = 0; j < kNT * kNT; ++j) H[j] = 0.0;
    const uint8_t* md = mask + (size_t)d * ncand;
    for (int c = 0; c < ncand; ++c) {
        if (!md[c]) continue;
        const double* src = H1r + ((size_t)s * ncand + c) * kNT * kNT;
        for (int j = 0; j < kNT * kNT; ++j) H[j] += src[j];
    }
    double v, ld;
    dkl_of(H, *prior, theta + (size_t)s * kNT, &v, &ld);
    work[(size_t)d * nsample + s] = v;
}

__global__ void greedy_dkl_kernel(const double* __restrict__ H1r, int nsample,
                                  int ncand, const eig_prior* __restrict__ prior,
                                  const double* __restrict__ theta,
                                  const double* __restrict__ Hcur,
                                  const uint8_t* __restrict__ chosen,
                                  double* __restrict__ work) {
    const int c = blockIdx.y;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nsample) return;
    if (chosen[c]) {
        work[(size_t)c * nsample + s] = 0.0;
        return;
    }
    double H[kNT * kNT];
    const double* src = H1r + ((size_t)s * ncand + c) * kNT * kNT;
    const double* cur = Hcur + (size_t)s * kNT * kNT;
    for (int j = 0; j < kNT * kNT; ++j) H[j] = cur[j] + src[j];
    double v, ld;
    dkl_of(H, *prior, theta + (size_t)s * kNT, &v, &ld);
    work[(size_t)c * nsample + s] = v;
}

// Pick argmax over candidates not yet chosen with a finite value (ties to
// the lowest index), record it, and add its Hessians to the running sum.
__global__ void greedy_pick_kernel(const double* __restrict__ H1r, int nsample,
                                   int ncand, const double* __restrict__ ival,
                                   double* __restrict__ Hcur, uint8_t* __restrict__ chosen,
                                   int k, int32_t* __restrict__ order,
                                   double* __restrict__ curve) {
    __shared__ double bv[256];
    __shared__ int bc[256];
    double best = -INFINITY;
    int bi = -1;
    for (int c = threadIdx.x; c < ncand; c += blockDim.x) {
        const double v = ival[c];
        if (chosen[c] || isnan(v)) continue;
        if (bi < 0 || v > best) { best = v; bi = c; }
    }
    bv[threadIdx.x] = best;
    bc[threadIdx.x] = bi;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            const int c2 = bc[threadIdx.x + o];
            const double v2 = bv[threadIdx.x + o];
            const int c1 = bc[threadIdx.x];
            const double v1 = bv[threadIdx.x];
            if (c2 >= 0 && (c1 < 0 || v2 > v1 || (v2 == v1 && c2 < c1))) {
                bv[threadIdx.x] = v2;
                bc[threadIdx.x] = c2;
            }
        }
        __syncthreads();
    }
    const int pick = bc[0];
    if (threadIdx.x == 0) {
        order[k] = pick;
        curve[k] = pick >= 0 ? bv[0] : __longlong_as_double(0x7ff8000000000000ULL);
        if (pick >= 0) chosen[pick] = 1;
    }
    if (pick < 0) return;
    for (size_t e = threadIdx.x; e < (size_t)nsample * kNT * kNT; e += blockDim.x) {
        const size_t s = e / (kNT * kNT), j = e % (kNT * kNT);
        Hcur[e] += H1r[(s * ncand + pick) * kNT * kNT + j];
    }
}

}  // namespace

void launch_laplace(const double* H1, int nsample, const eig_prior* prior_dev,
                    const double* theta, const double* w, double* dkl,
                    double* logdet, int32_t* status, double* eig, hipStream_t s) {
    if (nsample <= 0) return;
    laplace_kernel<<<(nsample + 127) / 128, 128, 0, s>>>(H1, nsample, prior_dev, theta,
                                                         dkl, logdet, status);
    weighted_rows_kernel<<<1, 256, 0, s>>>(dkl, nsample, w, eig, nullptr);
}

void launch_theorem3(const double* H1, const double* H2, int nsample,
                     const eig_prior* prior_dev, const double* theta_hat, const double* w,
                     double* val, int32_t* status, double* eig, hipStream_t s) {
    if (nsample <= 0) return;
    theorem3_kernel<<<(nsample + 127) / 128, 128, 0, s>>>(H1, H2, nsample, prior_dev,
                                                          theta_hat, val, status);
    if (eig) weighted_rows_kernel<<<1, 256, 0, s>>>(val, nsample, w, eig, nullptr);
}

void launch_design_eval(const double* H1r, int nsample, int ncand,
                        const uint8_t* mask, int ndesign, const eig_prior* prior_dev,
                        const double* theta, const double* w, double* work,
                        double* eig, hipStream_t s) {
    if (nsample <= 0 || ndesign <= 0) return;
    dim3 grid((nsample + 127) / 128, ndesign);
    design_dkl_kernel<<<grid, 128, 0, s>>>(H1r, nsample, ncand, mask, prior_dev, theta,
                                           work);
    weighted_rows_kernel<<<ndesign, 256, 0, s>>>(work, nsample, w, eig, nullptr);
}

void launch_greedy_step(const double* H1r, int nsample, int ncand,
                        const eig_prior* prior_dev, const double* theta,
                        const double* w, double* Hcur, uint8_t* chosen, double* work,
                        double* ival, int k, int32_t* order, double* curve,
                        hipStream_t s) {
    dim3 grid((nsample + 127) / 128, ncand);
    greedy_dkl_kernel<<<grid, 128, 0, s>>>(H1r, nsample, ncand, prior_dev, theta, Hcur,
                                           chosen, work);
    weighted_rows_kernel<<<ncand, 256, 0, s>>>(work, nsample, w, ival, chosen);
    greedy_pick_kernel<<<1, 256, 0, s>>>(H1r, nsample, ncand, ival, Hcur, chosen, k,
                                         order, curve);
}

}  // namespace eig
