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
// Distances in Gram form, |y_n - g_m|^2 = |y_n|^2 + |g_m|^2 - 2 <y_n, g_m>:
// the (n, m, k) work becomes one FP64 multiply-add of the dense product
// Y G^T, which runs on the FP64 matrix cores (16x16x4 MFMA); the squared
// norms come from a small pass of their own.  The expansion's rounding is
// about K u (|y_n|^2 + |g_m|^2) in a squared distance (u = 2^-53), i.e.
// K u (|y_n|^2 + |g_m|^2) / (2 sigma^2) nats in a log ratio: ~1e-9 nats for
// traces of ~100 sigma over K ~ 200 values, ~1e-5 at ~3000 sigma.
//
// Work decomposition: a 512-thread block (8 waves, 4 x 2) owns 128 outer rows
// and a range of inner samples (the range is split over several blocks when
// the rows alone cannot fill the chip), swept in tiles of 128 columns; each
// wave accumulates 2 x 4 MFMA tiles (32 rows x 64 columns).  A first pass
// writes y and g as FP64, k-major and zero-padded to whole tiles and chunks
// (Yt[k][n], Gt[k][m]); k is then staged through LDS in chunks of 16 with
// 16-byte copies and nothing else (no conversion, no bounds), double
// buffered, with the global loads of the chunk after next in flight while
// the current one is multiplied: one barrier per chunk.  After a
// tile's last chunk every lane folds its 32 distances into an online
// log-sum-exp per row: the running maximum and the rescaling of the running
// sum in FP64, the terms within 40 nats of the maximum as FP32 exponentials
// (relative error ~3e-6 each, so at most ~3e-6 nats in a log ratio).  Terms
// further down are dropped: each is below exp(-40) = 4.2e-18 of the maximum
// term, M of them below M * 4.2e-18 of the sum.  Per-lane partials are
// merged over the block, then over the inner-range splits, in a fixed order.
#include "internal.h"

namespace eig {

namespace {

typedef double dv4 __attribute__((ext_vector_type(4)));

// Tile geometry: 8 waves as kGR x kGC, each kWR x kWC 16x16 MFMA tiles.
constexpr int kWR = 2, kWC = 4, kGR = 4, kGC = 2, kKC = 16;
constexpr int kThreads = 64 * kGR * kGC;          // 512
constexpr int kTN = 16 * kGR * kWR;               // 128 outer rows per block
constexpr int kTM = 16 * kGC * kWC;               // 128 inner columns per tile
constexpr int kLY = kTN + 2, kLB = kTM + 2;       // padded LDS rows (16-byte aligned pairs)
constexpr int kQY = kKC * kTN / (2 * kThreads);   // y pairs staged per thread and chunk
constexpr int kQB = kKC * kTM / (2 * kThreads);   // g pairs staged per thread and chunk
constexpr int kNP = 16 * kGC;                     // per-row partials in a block
constexpr int kBuf = kKC * (kLY + kLB);
constexpr int kLds = 2 * kBuf > 2 * kNP * kTN ? 2 * kBuf : 2 * kNP * kTN;
static_assert(2 * kQY * kThreads == kKC * kTN && 2 * kQB * kThreads == kKC * kTM,
              "staging split");
typedef double dv2 __attribute__((ext_vector_type(2)));
constexpr double kDrop = -40.0;                   // terms below max - 40 nats are dropped

// Squared norms of y_n = g_n + sigma e_n (noise != NULL) or of g_m, one
// wave per row, FP64.  The same fma forms y as the staging below.
__global__ void __launch_bounds__(256)
nested_sqnorm_kernel(const float* __restrict__ g, const float* __restrict__ noise, int rows,
                     int nobs, double sigma, double* __restrict__ out) {
    const int row = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
    if (row >= rows) return;
    double s = 0.0;
    for (int k = l; k < nobs; k += 64) {
        double y = (double)g[(size_t)row * nobs + k];
        if (noise) y = fma(sigma, (double)noise[(size_t)row * nobs + k], y);
        s = fma(y, y, s);
    }
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (l == 0) out[row] = s;
}

// out[k][r] (rows rpad apart, k < kpad) = y_r[k] = g_r[k] + sigma e_r[k]
// (noise != NULL) or g_r[k], in FP64 (the same fma as the norms), zero for
// r >= rows or k >= nobs.  32 x 32 tiles transposed through LDS.
__global__ void __launch_bounds__(256)
nested_pack_kernel(const float* __restrict__ g, const float* __restrict__ noise, int rows,
                   int nobs, double sigma, int rpad, int kpad, double* __restrict__ out) {
    __shared__ double tile[32][33];
    const int r0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int j = ty; j < 32; j += 8) {
        const int r = r0 + j, k = k0 + tx;
        double v = 0.0;
        if (r < rows && k < nobs) {
            v = (double)g[(size_t)r * nobs + k];
            if (noise) v = fma(sigma, (double)noise[(size_t)r * nobs + k], v);
        }
        tile[j][tx] = v;
    }
    __syncthreads();
    for (int j = ty; j < 32; j += 8) {
        const int k = k0 + j, r = r0 + tx;
        if (k < kpad) out[(size_t)k * rpad + r] = tile[tx][j];
    }
}

// Partial log-sum-exp of rows [n0, n0+128) over inner samples [mb, me):
// part_max / part_sum [split][nouter].  Yt, Gt: the packed y and g (rows
// npad and mpad apart).
__global__ void __launch_bounds__(kThreads)
nested_lse_kernel(const double* __restrict__ Yt, const double* __restrict__ Gt, int npad,
                  int mpad, const double* __restrict__ ynorm,
                  const double* __restrict__ gnorm, int nouter, int ninner, int nobs,
                  double inv2s2, int mchunk, double* __restrict__ part_max,
                  double* __restrict__ part_sum) {
    __shared__ __attribute__((aligned(16))) double smem[kLds];
    const int t = threadIdx.x, w = t >> 6, l = t & 63;
    const int wr = w / kGC, wc = w % kGC;
    // MFMA lane layout: operand lane (li, lk) holds row/column li of k-slice
    // lk; accumulator register v of lane l holds row lk + 4 v, column li
    const int li = l & 15, lk = l >> 4;
    const int n0 = blockIdx.x * kTN;
    const int mb = blockIdx.y * mchunk, me = min(ninner, mb + mchunk);
    const int ntile = me > mb ? (me - mb + kTM - 1) / kTM : 0;
    const int nk = (nobs + kKC - 1) / kKC;
    const int nchunks = ntile * nk;

    double mx[kWR][4], sm[kWR][4], yn[kWR][4];
#pragma unroll
    for (int x = 0; x < kWR; ++x)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int n = n0 + wr * 16 * kWR + 16 * x + lk + 4 * v;
            yn[x][v] = n < nouter ? ynorm[n] : 0.0;
            mx[x][v] = -INFINITY;
            sm[x][v] = 0.0;
        }

    // chunk c = (column tile c / nk, k chunk c % nk); thread t copies the
    // pairs q * kThreads + t: k row (pair / 64), columns 2 (pair % 64), +1
    dv2 ry[2][kQY], rb[2][kQB];
    auto fetch = [&](int c, dv2* y, dv2* b) {
        if (c >= nchunks) return;
        const int m0 = mb + (c / nk) * kTM, k0 = (c % nk) * kKC;
#pragma unroll
        for (int q = 0; q < kQY; ++q) {
            const int i = t + kThreads * q;
            y[q] = *(const dv2*)(Yt + (size_t)(k0 + i / (kTN / 2)) * npad + n0 +
                                 2 * (i % (kTN / 2)));
        }
#pragma unroll
        for (int q = 0; q < kQB; ++q) {
            const int i = t + kThreads * q;
            b[q] = *(const dv2*)(Gt + (size_t)(k0 + i / (kTM / 2)) * mpad + m0 +
                                 2 * (i % (kTM / 2)));
        }
    };
    auto store = [&](int c, const dv2* y, const dv2* b) {
        double* sY = smem + (c & 1) * kBuf;
        double* sB = sY + kKC * kLY;
#pragma unroll
        for (int q = 0; q < kQY; ++q) {
            const int i = t + kThreads * q;
            *(dv2*)(sY + (i / (kTN / 2)) * kLY + 2 * (i % (kTN / 2))) = y[q];
        }
#pragma unroll
        for (int q = 0; q < kQB; ++q) {
            const int i = t + kThreads * q;
            *(dv2*)(sB + (i / (kTM / 2)) * kLB + 2 * (i % (kTM / 2))) = b[q];
        }
    };
    dv4 acc[kWR][kWC];
    auto compute = [&](int c) {
        const double* sY = smem + (c & 1) * kBuf;
        const double* sB = sY + kKC * kLY;
        const int kc = c % nk;
        if (kc == 0) {
#pragma unroll
            for (int x = 0; x < kWR; ++x)
#pragma unroll
                for (int y = 0; y < kWC; ++y) acc[x][y] = dv4{0.0, 0.0, 0.0, 0.0};
        }
#pragma unroll
        for (int ks = 0; ks < kKC / 4; ++ks) {
            double a[kWR], b[kWC];
#pragma unroll
            for (int x = 0; x < kWR; ++x) a[x] = sY[(4 * ks + lk) * kLY + wr * 16 * kWR + 16 * x + li];
#pragma unroll
            for (int y = 0; y < kWC; ++y) b[y] = sB[(4 * ks + lk) * kLB + wc * 16 * kWC + 16 * y + li];
#pragma unroll
            for (int x = 0; x < kWR; ++x)
#pragma unroll
                for (int y = 0; y < kWC; ++y)
                    acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
        if (kc != nk - 1) return;
        // online log-sum-exp over this tile's columns
        const int m0 = mb + (c / nk) * kTM;
        double gn[kWC];
        bool ok[kWC];
#pragma unroll
        for (int y = 0; y < kWC; ++y) {
            const int m = m0 + wc * 16 * kWC + 16 * y + li;
            ok[y] = m < me;
            gn[y] = ok[y] ? gnorm[m] : 0.0;
        }
#pragma unroll
        for (int x = 0; x < kWR; ++x)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double ll[kWC], tmax = -INFINITY;
#pragma unroll
                for (int y = 0; y < kWC; ++y) {
                    const double d2 = fma(-2.0, acc[x][y][v], yn[x][v] + gn[y]);
                    ll[y] = ok[y] ? -d2 * inv2s2 : -INFINITY;
                    tmax = fmax(tmax, ll[y]);
                }
                if (tmax == -INFINITY) continue;
                const double nm = fmax(mx[x][v], tmax);
                double s = sm[x][v];
                if (mx[x][v] != nm) s = mx[x][v] - nm > kDrop ? s * exp(mx[x][v] - nm) : 0.0;
                float f = 0.f;
#pragma unroll
                for (int y = 0; y < kWC; ++y) {
                    const double z = ll[y] - nm;
                    if (z > kDrop) f += __expf((float)z);
                }
                mx[x][v] = nm;
                sm[x][v] = s + (double)f;
            }
    };

    fetch(0, ry[0], rb[0]);
    fetch(1, ry[1], rb[1]);
    for (int c = 0; c < nchunks; c += 2) {
        store(c, ry[0], rb[0]);
        __syncthreads();
        fetch(c + 2, ry[0], rb[0]);
        compute(c);
        if (c + 1 < nchunks) {
            store(c + 1, ry[1], rb[1]);
            __syncthreads();
            fetch(c + 3, ry[1], rb[1]);
            compute(c + 1);
        }
    }
    __syncthreads();
    double* pmx = smem;
    double* psum = smem + kNP * kTN;
#pragma unroll
    for (int x = 0; x < kWR; ++x)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int r = wr * 16 * kWR + 16 * x + lk + 4 * v;
            pmx[(wc * 16 + li) * kTN + r] = mx[x][v];
            psum[(wc * 16 + li) * kTN + r] = sm[x][v];
        }
    __syncthreads();
    if (t < kTN && n0 + t < nouter) {
        double M = -INFINITY;
        for (int c = 0; c < kNP; ++c) M = fmax(M, pmx[c * kTN + t]);
        double S = 0.0;
        for (int c = 0; c < kNP; ++c)
            if (pmx[c * kTN + t] > -INFINITY) S += psum[c * kTN + t] * exp(pmx[c * kTN + t] - M);
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

// Rows and k of the packed copies: whole tiles and whole k chunks.
static int nested_rpad(int rows, int tile) { return (rows + tile - 1) / tile * tile; }
static int nested_kpad(int nobs) { return (nobs + kKC - 1) / kKC * kKC; }

// Partials (max, sum) per split and outer sample, the squared norms of the
// y_n and of the g_m, then the packed Yt and Gt (256-byte aligned).
size_t nested_workspace(int nouter, int ninner, int nobs) {
    const size_t head = (2 * (size_t)nested_splits(nouter, ninner) * nouter + nouter + ninner) *
                        sizeof(double);
    const size_t kp = (size_t)nested_kpad(nobs);
    return (head + 255) / 256 * 256 +
           kp * ((size_t)nested_rpad(nouter, kTN) + nested_rpad(ninner, kTM)) * sizeof(double);
}

// Inner-range splits, each at least two column tiles long: enough blocks to
// fill the chip when the outer rows are few, and a block count whose last
// round of the chip's block slots is nearly full.  Every block of a launch
// does the same work, so with b blocks on kSlots slots the launch takes
// ceil(b / kSlots) rounds: 3125 blocks at N = 4e5 take 13 rounds for 12.2
// rounds of work (6 % idle), 12500 take 49 for 48.8.
constexpr int kSlots = 256;   // one block per CU: 8 waves of ~214 VGPRs fill its 4 SIMDs
int nested_splits(int nouter, int ninner) {
    const long rows = (nouter + kTN - 1) / kTN;
    auto fill = [&](long split) {
        const long b = rows * split, rounds = (b + kSlots - 1) / kSlots;
        return (double)b / (double)(rounds * kSlots);
    };
    int split = 1;
    while ((rows * split < 2048 || fill(split) < 0.98) &&
           (ninner + split * 2 - 1) / (split * 2) >= 2 * kTM)
        split *= 2;
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
    double* ynorm = psum + (size_t)split * nouter;
    double* gnorm = ynorm + nouter;
    const size_t head = (2 * (size_t)split * nouter + nouter + ninner) * sizeof(double);
    const int npad = nested_rpad(nouter, kTN), mpad = nested_rpad(ninner, kTM);
    const int kpad = nested_kpad(nobs);
    double* Yt = (double*)((char*)work + (head + 255) / 256 * 256);
    double* Gt = Yt + (size_t)kpad * npad;
    nested_sqnorm_kernel<<<(nouter + 3) / 4, 256, 0, s>>>(gout, noise, nouter, nobs, sigma, ynorm);
    nested_sqnorm_kernel<<<(ninner + 3) / 4, 256, 0, s>>>(gin, nullptr, ninner, nobs, 0.0, gnorm);
    nested_pack_kernel<<<dim3(npad / 32, (kpad + 31) / 32), 256, 0, s>>>(
        gout, noise, nouter, nobs, sigma, npad, kpad, Yt);
    nested_pack_kernel<<<dim3(mpad / 32, (kpad + 31) / 32), 256, 0, s>>>(
        gin, nullptr, ninner, nobs, 0.0, mpad, kpad, Gt);
    const dim3 grid((nouter + kTN - 1) / kTN, split);
    nested_lse_kernel<<<grid, kThreads, 0, s>>>(Yt, Gt, npad, mpad, ynorm, gnorm, nouter, ninner,
                                                nobs, 1.0 / (2.0 * sigma * sigma), mchunk, pmax,
                                                psum);
    nested_merge_kernel<<<(nouter + 255) / 256, 256, 0, s>>>(noise, nouter, ninner, nobs,
                                                             split, pmax, psum, logratio);
    if (eig) mean_kernel<<<1, 256, 0, s>>>(logratio, nouter, eig);
}

}  // namespace eig
