// Nested (double-loop) Monte Carlo estimate of the expected information gain
// (the direct sample-average estimator of the introduction, compared with the
// Laplace method in Section 4.4).  FP32 inputs, FP64 arithmetic.
//
// For outer samples n (model output g_n at theta*_n, data y_n = g_n +
// sigma e_n with e_n standard normal draws given by the caller) and inner
// prior samples m (outputs g_m), with C_eps = sigma^2 I:
//   logratio_n = -|e_n|^2 / 2 - ( LSE_m( -|y_n - g_m|^2 / (2 sigma^2) ) - log M ).
// y_n is formed in FP64, where its rounding is ~1e-14 of sigma e_n even when
// |g_n| is hundreds of sigma (in FP32 it would lose sigma e_n to g_n).
//
// Work decomposition: a 256-thread block owns 64 outer rows and a range of
// inner samples (the range is split over several blocks when the outer rows
// alone cannot fill the chip), swept in tiles of 64; observations are
// staged through LDS in chunks of 16 as FP64 (y = g + sigma e of the rows,
// g of the columns); each thread accumulates a 4 x 4 block of squared
// distances and keeps an online log-sum-exp per row; the 16 threads sharing
// a row, then the inner-range splits, are merged in a fixed order.  The log
// ratios grow with the data's information (hundreds to thousands of nats
// for few inner samples), so distances are kept in FP64 (full-rate vector
// FP64 on this chip, the same issue rate as unpacked FP32).  It is bound by
// vector ALU throughput: 2 FP64 operations (sub, FMA) per (n, m, k).
#include "internal.h"

namespace eig {

namespace {

constexpr int kTN = 64, kTM = 64, kKC = 16;

// Partial log-sum-exp of rows [n0, n0+64) over inner samples [mb, me):
// part_max / part_sum [split][nouter].
__global__ void __launch_bounds__(256)
nested_lse_kernel(const float* __restrict__ gout, const float* __restrict__ noise,
                  const float* __restrict__ gin, int nouter, int ninner, int nobs,
                  double sigma, double inv2s2, int mchunk, double* __restrict__ part_max,
                  double* __restrict__ part_sum) {
    __shared__ double sY[kKC][kTN];   // y = g + sigma e of the rows
    __shared__ double sB[kKC][kTM];   // g of the columns
    __shared__ double pmx[16][kTN], psum[16][kTN];
    const int t = threadIdx.x;
    const int tr = t >> 4, tc = t & 15;
    const int n0 = blockIdx.x * kTN;
    const int mb = blockIdx.y * mchunk, me = min(ninner, mb + mchunk);
    double mx[4], sm[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        mx[i] = -INFINITY;
        sm[i] = 0.0;
    }
    for (int m0 = mb; m0 < me; m0 += kTM) {
        double acc[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
        for (int k0 = 0; k0 < nobs; k0 += kKC) {
            // stage 1024 elements of each tile, 4 per thread, k fastest; in
            // FP64 the sum g + sigma e keeps sigma e to ~1e-14 relative
            for (int e = t; e < kKC * kTN; e += 256) {
                const int r = e / kKC, kk = e % kKC;
                const int n = n0 + r, m = m0 + r, k = k0 + kk;
                double y = 0.0, b = 0.0;
                if (k < nobs) {
                    if (n < nouter)
                        y = (double)gout[(size_t)n * nobs + k] +
                            sigma * (double)noise[(size_t)n * nobs + k];
                    if (m < me) b = gin[(size_t)m * nobs + k];
                }
                sY[kk][r] = y;
                sB[kk][r] = b;
            }
            __syncthreads();
#pragma unroll
            for (int kk = 0; kk < kKC; ++kk) {
                double y[4], b[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    y[i] = sY[kk][tr + 16 * i];
                    b[i] = sB[kk][tc + 16 * i];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const double d = y[i] - b[j];
                        acc[i][j] = fma(d, d, acc[i][j]);
                    }
            }
            __syncthreads();
        }
        // online log-sum-exp over this tile's columns
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double tmax = -INFINITY;
            double ll[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = m0 + tc + 16 * j;
                ll[j] = m < me ? -acc[i][j] * inv2s2 : -INFINITY;
                tmax = fmax(tmax, ll[j]);
            }
            if (tmax == -INFINITY) continue;
            const double nm = fmax(mx[i], tmax);
            double s = sm[i] * exp(mx[i] - nm);
#pragma unroll
            for (int j = 0; j < 4; ++j) s += exp(ll[j] - nm);
            mx[i] = nm;
            sm[i] = s;
        }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        pmx[tc][tr + 16 * i] = mx[i];
        psum[tc][tr + 16 * i] = sm[i];
    }
    __syncthreads();
    if (t < kTN && n0 + t < nouter) {
        double M = -INFINITY;
        for (int c = 0; c < 16; ++c) M = fmax(M, pmx[c][t]);
        double S = 0.0;
        for (int c = 0; c < 16; ++c)
            if (pmx[c][t] > -INFINITY) S += psum[c][t] * exp(pmx[c][t] - M);
        part_max[(size_t)blockIdx.y * nouter + n0 + t] = M;
        part_sum[(size_t)blockIdx.y * nouter + n0 + t] = S;
    }
}

// Merge the inner-range partials (fixed order) into the log ratios.
__global__ void nested_merge_kernel(const float* __restrict__ noise, int nouter, int ninner,
                                    int nobs, int nsplit, const double* __restrict__ part_max,
                                    const double* __restrict__ part_sum,
                                    double* __restrict__ logratio) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= nouter) return;
    double M = -INFINITY;
    for (int c = 0; c < nsplit; ++c) M = fmax(M, part_max[(size_t)c * nouter + n]);
    double S = 0.0;
    for (int c = 0; c < nsplit; ++c) {
        const double pm = part_max[(size_t)c * nouter + n];
        if (pm > -INFINITY) S += part_sum[(size_t)c * nouter + n] * exp(pm - M);
    }
    double e2 = 0.0;
    for (int k = 0; k < nobs; ++k) {
        const double e = noise[(size_t)n * nobs + k];
        e2 += e * e;
    }
    logratio[n] = -0.5 * e2 - (M + log(S) - log((double)ninner));
}

// out[0] = (1/n) sum x, fixed order (strided partials, then a tree).
__global__ void mean_kernel(const double* __restrict__ x, int n, double* __restrict__ out) {
    __shared__ double part[256];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) v += x[i];
    part[threadIdx.x] = v;
    __syncthreads();
    for (int o = blockDim.x / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) part[threadIdx.x] += part[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0] / n;
}

}  // namespace

size_t nested_workspace(int nouter, int ninner) {
    return 2 * (size_t)nested_splits(nouter, ninner) * nouter * sizeof(double);
}

// Inner-range splits: enough blocks to fill the chip when the outer rows
// are few, each split at least four column tiles long.
int nested_splits(int nouter, int ninner) {
    const int rows = (nouter + kTN - 1) / kTN;
    int split = 1;
    while (rows * split < 2048 && (ninner + split * 2 - 1) / (split * 2) >= 4 * kTM) split *= 2;
    return split;
}

void launch_nested(const float* gout, const float* noise, const float* gin, int nouter,
                   int ninner, int nobs, double sigma, double* logratio, double* eig,
                   double* work, hipStream_t s) {
    const int split = nested_splits(nouter, ninner);
    int mchunk = (ninner + split - 1) / split;
    mchunk = (mchunk + kTM - 1) / kTM * kTM;
    double* pmax = work;
    double* psum = work + (size_t)split * nouter;
    const dim3 grid((nouter + kTN - 1) / kTN, split);
    nested_lse_kernel<<<grid, 256, 0, s>>>(gout, noise, gin, nouter, ninner, nobs, sigma,
                                           1.0 / (2.0 * sigma * sigma), mchunk, pmax, psum);
    nested_merge_kernel<<<(nouter + 255) / 256, 256, 0, s>>>(noise, nouter, ninner, nobs,
                                                             split, pmax, psum, logratio);
    if (eig) mean_kernel<<<1, 256, 0, s>>>(logratio, nouter, eig);
}

}  // namespace eig
