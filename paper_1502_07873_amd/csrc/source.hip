// Device-side tables: medium coefficients (FP64 in, FP32 out) and the point
// moment-tensor forcing f = S(t) M grad(delta(x - x_s)) of every solve.
//
// The singular source is discretised with the fourth-order, twice
// continuously differentiable regularised delta and delta' of the paper
// (Section 3.3.2, item 2) on the six nodes k-2..k+3 around the source cell,
// and the 2-D gradient is their Cartesian product.  Tables are built in FP64;
// for the perturbed solves of the central-difference Jacobian the difference
// F(theta + step e_j) - F(theta) is formed in FP64 and only then rounded to
// FP32, so the small perturbation is not lost to FP32 cancellation.
#include "internal.h"

namespace eig {

namespace {

// Regularised delta weights (times h) for node offset o in -2..3 and
// alpha = (x_s - x_k)/h.
__device__ double delta_w(double a, int o) {
    const double a2 = a * a, a3 = a2 * a, a4 = a3 * a;
    const double P = a4 * a * (5.0 / 3.0 + a * (-7.0 / 24.0 + a * (-17.0 / 12.0 + a * (9.0 / 8.0 - a / 4.0))));
    switch (o) {
        case -2: return a / 12.0 - a2 / 24.0 - a3 / 12.0 - 19.0 * a4 / 24.0 + P;
        case -1: return -2.0 * a / 3.0 + 2.0 * a2 / 3.0 + a3 / 6.0 + 4.0 * a4 - 5.0 * P;
        case 0: return 1.0 - 5.0 * a2 / 4.0 - 97.0 * a4 / 12.0 + 10.0 * P;
        case 1: return 2.0 * a / 3.0 + 2.0 * a2 / 3.0 - a3 / 6.0 + 49.0 * a4 / 6.0 - 10.0 * P;
        case 2: return -a / 12.0 - a2 / 24.0 + a3 / 12.0 - 33.0 * a4 / 8.0 + 5.0 * P;
        case 3: return 5.0 * a4 / 6.0 - P;
        default: return 0.0;
    }
}

// Regularised delta' weights (times h^2).
__device__ double ddelta_w(double a, int o) {
    const double a2 = a * a, a3 = a2 * a, a4 = a3 * a;
    const double R = a4 * (-25.0 / 12.0 + a * (-3.0 / 4.0 + a * (59.0 / 12.0 + a * (-4.0 + a))));
    switch (o) {
        case -2: return -1.0 / 12.0 + a / 12.0 + a2 / 4.0 + 2.0 * a3 / 3.0 + R;
        case -1: return 2.0 / 3.0 - 4.0 * a / 3.0 - a2 / 2.0 - 7.0 * a3 / 2.0 - 5.0 * R;
        case 0: return 5.0 * a / 2.0 + 22.0 * a3 / 3.0 + 10.0 * R;
        case 1: return -2.0 / 3.0 - 4.0 * a / 3.0 + a2 / 2.0 - 23.0 * a3 / 3.0 - 10.0 * R;
        case 2: return 1.0 / 12.0 + a / 12.0 - a2 / 4.0 + 4.0 * a3 + 5.0 * R;
        case 3: return -5.0 * a3 / 6.0 - R;
        default: return 0.0;
    }
}

// d/dalpha of the delta weights (times h).
__device__ double delta_w_da(double a, int o) {
    const double a2 = a * a, a3 = a2 * a;
    const double Pd = a3 * a * (25.0 / 3.0 + a * (-7.0 / 4.0 + a * (-119.0 / 12.0 + a * (9.0 - 9.0 * a / 4.0))));
    switch (o) {
        case -2: return 1.0 / 12.0 - a / 12.0 - a2 / 4.0 - 19.0 * a3 / 6.0 + Pd;
        case -1: return -2.0 / 3.0 + 4.0 * a / 3.0 + a2 / 2.0 + 16.0 * a3 - 5.0 * Pd;
        case 0: return -5.0 * a / 2.0 - 97.0 * a3 / 3.0 + 10.0 * Pd;
        case 1: return 2.0 / 3.0 + 4.0 * a / 3.0 - a2 / 2.0 + 98.0 * a3 / 3.0 - 10.0 * Pd;
        case 2: return -1.0 / 12.0 - a / 12.0 + a2 / 4.0 - 33.0 * a3 / 2.0 + 5.0 * Pd;
        case 3: return 10.0 * a3 / 3.0 - Pd;
        default: return 0.0;
    }
}

// d/dalpha of the delta' weights (times h^2).
__device__ double ddelta_w_da(double a, int o) {
    const double a2 = a * a, a3 = a2 * a;
    const double Rd = a3 * (-25.0 / 3.0 + a * (-15.0 / 4.0 + a * (59.0 / 2.0 + a * (-28.0 + 8.0 * a))));
    switch (o) {
        case -2: return 1.0 / 12.0 + a / 2.0 + 2.0 * a2 + Rd;
        case -1: return -4.0 / 3.0 - a - 21.0 * a2 / 2.0 - 5.0 * Rd;
        case 0: return 5.0 / 2.0 + 22.0 * a2 + 10.0 * Rd;
        case 1: return -4.0 / 3.0 + a - 23.0 * a2 - 10.0 * Rd;
        case 2: return 1.0 / 12.0 - a / 2.0 + 12.0 * a2 + 5.0 * Rd;
        case 3: return -5.0 * a2 / 2.0 - Rd;
        default: return 0.0;
    }
}

// d/dx_s (axis 0) or d/dz_s (axis 1) of source_weight: on that axis the
// weights are differentiated in alpha and divided by h.
__device__ double dsource_weight(const double* th, int kx, int kz, double h, int ic, int kr,
                                 int c, int axis) {
    const int ox = ic - kx, oz = kr - kz;
    if (ox < -2 || ox > 3 || oz < -2 || oz > 3) return 0.0;
    const double ax = th[0] / h - kx, az = th[1] / h - kz;
    double dx = delta_w(ax, ox) / h, dpx = ddelta_w(ax, ox) / (h * h);
    double dz = delta_w(az, oz) / h, dpz = ddelta_w(az, oz) / (h * h);
    if (axis == 0) {
        dx = delta_w_da(ax, ox) / (h * h);
        dpx = ddelta_w_da(ax, ox) / (h * h * h);
    } else {
        dz = delta_w_da(az, oz) / (h * h);
        dpz = ddelta_w_da(az, oz) / (h * h * h);
    }
    const double gx = dpx * dz, gz = dx * dpz;
    return c == 0 ? th[4] * gx + th[5] * gz : th[5] * gx + th[6] * gz;
}

// d^2/dalpha^2 of the delta weights (times h).
__device__ double delta_w_da2(double a, int o) {
    const double a2 = a * a, a3 = a2 * a;
    const double Pdd = a3 * (100.0 / 3.0 + a * (-35.0 / 4.0 + a * (-119.0 / 2.0 + a * (63.0 - 18.0 * a))));
    switch (o) {
        case -2: return -1.0 / 12.0 - a / 2.0 - 19.0 * a2 / 2.0 + Pdd;
        case -1: return 4.0 / 3.0 + a + 48.0 * a2 - 5.0 * Pdd;
        case 0: return -5.0 / 2.0 - 97.0 * a2 + 10.0 * Pdd;
        case 1: return 4.0 / 3.0 - a + 98.0 * a2 - 10.0 * Pdd;
        case 2: return -1.0 / 12.0 + a / 2.0 - 99.0 * a2 / 2.0 + 5.0 * Pdd;
        case 3: return 10.0 * a2 - Pdd;
        default: return 0.0;
    }
}

// d^2/dalpha^2 of the delta' weights (times h^2).
__device__ double ddelta_w_da2(double a, int o) {
    const double a2 = a * a;
    const double Rdd = a2 * (-25.0 + a * (-15.0 + a * (295.0 / 2.0 + a * (-168.0 + 56.0 * a))));
    switch (o) {
        case -2: return 1.0 / 2.0 + 4.0 * a + Rdd;
        case -1: return -1.0 - 21.0 * a - 5.0 * Rdd;
        case 0: return 44.0 * a + 10.0 * Rdd;
        case 1: return 1.0 - 46.0 * a - 10.0 * Rdd;
        case 2: return -1.0 / 2.0 + 24.0 * a + 5.0 * Rdd;
        case 3: return -5.0 * a - Rdd;
        default: return 0.0;
    }
}

// delta (dp = false) or delta' (dp = true) weight of node offset o along one
// axis, differentiated der times (0..2) in the source coordinate.
__device__ double axis_weight(double a, int o, bool dp, int der, double h) {
    double v;
    if (!dp) v = der == 0 ? delta_w(a, o) : der == 1 ? delta_w_da(a, o) : delta_w_da2(a, o);
    else v = der == 0 ? ddelta_w(a, o) : der == 1 ? ddelta_w_da(a, o) : ddelta_w_da2(a, o);
    double sc = dp ? h * h : h;
    for (int q = 0; q < der; ++q) sc *= h;
    return v / sc;
}

// Window weight (component c) of M grad(delta), differentiated ox times in
// x_s and oz times in z_s, for the moments m = (mxx, mxz, mzz).
__device__ double window_weight(const double* th, const double* m, int kx, int kz, double h,
                                int ic, int kr, int c, int ox, int oz) {
    const int o1 = ic - kx, o2 = kr - kz;
    if (o1 < -2 || o1 > 3 || o2 < -2 || o2 > 3) return 0.0;
    const double ax = th[0] / h - kx, az = th[1] / h - kz;
    const double gx = axis_weight(ax, o1, true, ox, h) * axis_weight(az, o2, false, oz, h);
    const double gz = axis_weight(ax, o1, false, ox, h) * axis_weight(az, o2, true, oz, h);
    return c == 0 ? m[0] * gx + m[1] * gz : m[1] * gx + m[2] * gz;
}

// Force density on node (ic, kr), component c, of the source theta whose
// cell is (kx, kz): M grad(delta) with grad(delta) = (delta'(x) delta(z),
// delta(x) delta'(z)).
__device__ double source_weight(const double* th, int kx, int kz, double h, int ic,
                                int kr, int c) {
    const int ox = ic - kx, oz = kr - kz;
    if (ox < -2 || ox > 3 || oz < -2 || oz > 3) return 0.0;
    const double ax = th[0] / h - kx, az = th[1] / h - kz;
    const double dx = delta_w(ax, ox) / h, dpx = ddelta_w(ax, ox) / (h * h);
    const double dz = delta_w(az, oz) / h, dpz = ddelta_w(az, oz) / (h * h);
    const double gx = dpx * dz, gz = dx * dpz;
    return c == 0 ? th[4] * gx + th[5] * gz : th[5] * gx + th[6] * gz;
}

__device__ double wavelet(int kind, double t, double t0, double p) {
    if (kind == EIG_STF_GAUSS) {
        const double w = p;
        return w / sqrt(2.0 * M_PI) * exp(-0.5 * w * w * (t - t0) * (t - t0));
    }
    const double w = 2.0 * M_PI * p;
    const double g = w / sqrt(2.0 * M_PI) * exp(-0.5 * w * w * (t - t0) * (t - t0));
    return -w * w * (t - t0) * g;
}

// d/dt0 (wrt 0) or d/d(frequency parameter) (wrt 1) of the wavelet.
__device__ double dwavelet(int kind, double t, double t0, double p, int wrt) {
    const double tau = t - t0;
    const double c = 1.0 / sqrt(2.0 * M_PI);
    if (kind == EIG_STF_GAUSS) {
        const double w = p;
        const double e = exp(-0.5 * w * w * tau * tau);
        return wrt == 0 ? c * w * w * w * tau * e : c * e * (1.0 - w * w * tau * tau);
    }
    const double w = 2.0 * M_PI * p;
    const double e = exp(-0.5 * w * w * tau * tau);
    if (wrt == 0) return c * w * e * (w * w - w * w * w * w * tau * tau);
    return 2.0 * M_PI * c * e * (-3.0 * w * w * tau + w * w * w * w * tau * tau * tau);
}

// Second derivatives of the wavelet: wrt 0 = t0 t0, 1 = t0 p, 2 = p p.
__device__ double d2wavelet(int kind, double t, double t0, double p, int wrt) {
    const double tau = t - t0;
    const double c = 1.0 / sqrt(2.0 * M_PI);
    if (kind == EIG_STF_GAUSS) {
        const double w = p, wt2 = w * w * tau * tau;
        const double e = exp(-0.5 * wt2);
        if (wrt == 0) return c * w * w * w * e * (wt2 - 1.0);
        if (wrt == 1) return c * w * w * tau * e * (3.0 - wt2);
        return c * w * tau * tau * e * (wt2 - 3.0);
    }
    const double w = 2.0 * M_PI * p, wt2 = w * w * tau * tau;
    const double e = exp(-0.5 * wt2);
    if (wrt == 0) return c * w * w * w * w * w * tau * e * (3.0 - wt2);
    if (wrt == 1) return 2.0 * M_PI * c * w * w * e * (wt2 * wt2 - 6.0 * wt2 + 3.0);
    return 4.0 * M_PI * M_PI * c * w * tau * e * (-wt2 * wt2 + 7.0 * wt2 - 6.0);
}

__global__ void source_kernel(const SourceJob* __restrict__ jobs) {
    const SourceJob& J = jobs[blockIdx.x];
    double th[kNT], tp[kNT];
    for (int j = 0; j < kNT; ++j) th[j] = tp[j] = J.theta[j];
    if (J.param >= 0) tp[J.param] = J.theta[J.param] + J.step;
    const bool spatial = (J.param == 0 || J.param == 1 || J.param >= 4);
    const bool temporal = (J.param == 2 || J.param == 3);
    if (J.deriv) {
        // sensitivity forcing dF/dtheta_param (Algorithm 1)
        double tu[kNT];
        for (int j = 0; j < kNT; ++j) tu[j] = th[j];
        if (J.param >= 4) {
            tu[4] = tu[5] = tu[6] = 0.0;
            tu[J.param] = 1.0;
        }
        for (int e = threadIdx.x; e < 2 * kSrcW * kSrcW; e += blockDim.x) {
            const int c = e / (kSrcW * kSrcW);
            const int kk = (e / kSrcW) % kSrcW;
            const int ii = e % kSrcW;
            const int ic = J.i0 + ii, kr = J.k0 + kk;
            const double w = (J.param == 0 || J.param == 1)
                                 ? dsource_weight(th, J.kx, J.kz, J.h, ic, kr, c, J.param)
                                 : source_weight(tu, J.kx, J.kz, J.h, ic, kr, c);
            J.srcw[e] = (float)w;
        }
        for (int m = threadIdx.x; m < J.nsteps; m += blockDim.x) {
            const double t = m * J.dt;
            const double S = temporal ? dwavelet(J.stf, t, th[2], th[3], J.param - 2)
                                      : wavelet(J.stf, t, th[2], th[3]);
            J.srcs[m] = (float)S;
        }
        return;
    }
    for (int e = threadIdx.x; e < 2 * kSrcW * kSrcW; e += blockDim.x) {
        const int c = e / (kSrcW * kSrcW);
        const int kk = (e / kSrcW) % kSrcW;
        const int ii = e % kSrcW;
        const int ic = J.i0 + ii, kr = J.k0 + kk;
        double w = source_weight(th, J.kx, J.kz, J.h, ic, kr, c);
        if (J.param >= 0 && spatial)
            w = source_weight(tp, J.kx2, J.kz2, J.h, ic, kr, c) - w;
        J.srcw[e] = (float)w;
    }
    for (int m = threadIdx.x; m < J.nsteps; m += blockDim.x) {
        const double t = m * J.dt;
        double S = wavelet(J.stf, t, th[2], th[3]);
        if (J.param >= 0 && temporal) S = wavelet(J.stf, t, tp[2], tp[3]) - S;
        J.srcs[m] = (float)S;
    }
}

// Depth-only medium: one row of kCoefStride coefficients per depth index,
// the operator of the stencil kernel written out per row (a = lambda+2mu).
__global__ void layered_coef_kernel(const double* __restrict__ rho,
                                    const double* __restrict__ lam,
                                    const double* __restrict__ mu, int nz, double h,
                                    double dt, float* __restrict__ coef) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nz) return;
    double c[kCoefStride];
    for (int j = 0; j < kCoefStride; ++j) c[j] = 0.0;
    if (k < nz - 1) {
        const double s = dt * dt / (rho[k] * h * h);
        const double l0 = lam[k], m0 = mu[k], a0 = l0 + 2.0 * m0;
        const double l1 = lam[k + 1], m1 = mu[k + 1], a1 = l1 + 2.0 * m1;
        c[kCxxU] = s * a0;
        c[kCxxV] = s * m0;
        c[kFco] = dt * dt / rho[k];
        if (k == 0) {
            // traction-free row
            c[kCzpU] = s * (m0 + m1);               // 2 mu_{1/2}
            c[kCmpU] = s * 0.5 * (l0 + m1);
            c[kCm0U] = s * 0.5 * (m0 - l0);
            c[kCzpV] = s * (a0 + a1);               // 2 a_{1/2}
            c[kCmpV] = s * 0.5 * (l1 + m0);
            c[kCm0V] = s * 0.5 * (l0 - m0);
        } else {
            const double lm = lam[k - 1], mm = mu[k - 1], am = lm + 2.0 * mm;
            c[kCzpU] = s * 0.5 * (m0 + m1);
            c[kCzmU] = s * 0.5 * (mm + m0);
            c[kCmpU] = s * 0.25 * (l0 + m1);
            c[kCmmU] = s * 0.25 * (l0 + mm);
            c[kCzpV] = s * 0.5 * (a0 + a1);
            c[kCzmV] = s * 0.5 * (am + a0);
            c[kCmpV] = s * 0.25 * (l1 + m0);
            c[kCmmV] = s * 0.25 * (lm + m0);
        }
    }
    // absorbing-edge coefficients, every row (the bottom row included)
    {
        const double a = lam[k] + 2.0 * mu[k];
        const double cp = sqrt(a / rho[k]), cs = sqrt(mu[k] / rho[k]);
        c[kCeP] = cp * dt / h;
        c[kCeS] = cs * dt / h;
        c[kCeL] = lam[k] * dt / (rho[k] * cp * h);
    }
    for (int j = 0; j < kCoefStride; ++j) coef[(size_t)k * kCoefStride + j] = (float)c[j];
}

__global__ void nodal_coef_kernel(const double* __restrict__ rho,
                                  const double* __restrict__ lam,
                                  const double* __restrict__ mu, int nx, int nz,
                                  int pitch, double h, double dt,
                                  float* __restrict__ coef) {
    const size_t plane = (size_t)nz * pitch;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < plane;
         e += (size_t)gridDim.x * blockDim.x) {
        const int k = (int)(e / pitch), i = (int)(e % pitch);
        float l = 0.f, m = 0.f, sc = 0.f;
        if (i < nx) {
            const size_t p = (size_t)k * nx + i;
            l = (float)lam[p];
            m = (float)mu[p];
            sc = (float)(dt * dt / (rho[p] * h * h));
        }
        coef[e] = l;
        coef[plane + e] = m;
        coef[2 * plane + e] = sc;
    }
}

// H_2 of one sample from the dual field on the forcing window.  Threads
// 0..97 own a (component, node) of the window and accumulate, over the
// levels, the six time-series projections Psi_b = sum_n b(t_n) psi^{N-n}
// (b = S, dS/dt0, dS/dp and the three second derivatives); then one thread
// per (j, k) sums W_i a_jk(i) Psi_{b(jk)} over the window (fixed order).
__global__ void __launch_bounds__(128) h2_kernel(const H2Job* __restrict__ jobs) {
    const H2Job& J = jobs[blockIdx.x];
    constexpr int kWin = kSrcW * kSrcW;
    __shared__ double psi[2 * kWin][6];
    const int e = threadIdx.x;
    const int N = J.nsteps;
    if (e < 2 * kWin) {
        const int comp = e / kWin, node = e % kWin;
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int n = 0; n < N; ++n) {
            const float2 pv = J.wrec[(size_t)(N - 1 - n) * kWin + node];  // psi^{N-n}
            const double p = comp == 0 ? pv.x : pv.y;
            const double t = n * J.dt;
            acc[0] += p * wavelet(J.stf, t, J.theta[2], J.theta[3]);
            acc[1] += p * dwavelet(J.stf, t, J.theta[2], J.theta[3], 0);
            acc[2] += p * dwavelet(J.stf, t, J.theta[2], J.theta[3], 1);
            acc[3] += p * d2wavelet(J.stf, t, J.theta[2], J.theta[3], 0);
            acc[4] += p * d2wavelet(J.stf, t, J.theta[2], J.theta[3], 1);
            acc[5] += p * d2wavelet(J.stf, t, J.theta[2], J.theta[3], 2);
        }
        for (int b = 0; b < 6; ++b) psi[e][b] = acc[b];
    }
    __syncthreads();
    if (threadIdx.x < kNT * kNT) {
        const int j = threadIdx.x / kNT, k = threadIdx.x % kNT;
        if (j > k) return;
        // spatial orders, moments and time series of d^2 F / dtheta_j dtheta_k
        int ox = 0, oz = 0, b = -1;
        double m[3] = {J.theta[4], J.theta[5], J.theta[6]};
        const int a0 = j, a1 = k;
        auto spatial = [](int q) { return q == 0 || q == 1; };
        auto temporal = [](int q) { return q == 2 || q == 3; };
        auto moment = [](int q) { return q >= 4; };
        if (moment(a0) && moment(a1)) {
            b = -1;
        } else {
            int tcount = 0, tfirst = -1;
            for (int qi = 0; qi < 2; ++qi) {
                const int q = qi == 0 ? a0 : a1;
                if (spatial(q)) (q == 0 ? ox : oz) += 1;
                if (temporal(q)) {
                    if (tcount == 0) tfirst = q;
                    ++tcount;
                }
                if (moment(q)) {
                    m[0] = m[1] = m[2] = 0.0;
                    m[q - 4] = 1.0;
                }
            }
            if (tcount == 0) b = 0;
            else if (tcount == 1) b = tfirst == 2 ? 1 : 2;
            else b = (a0 == 2 && a1 == 2) ? 3 : (a0 == 3 && a1 == 3) ? 5 : 4;
        }
        double v = 0.0;
        if (b >= 0) {
            for (int q = 0; q < 2 * kWin; ++q) {
                const int comp = q / kWin, node = q % kWin;
                const int ic = J.i0 + node % kSrcW, kr = J.k0 + node / kSrcW;
                const double Wq = J.h * J.h * (kr == 0 ? 0.5 : 1.0);
                v += Wq * window_weight(J.theta, m, J.kx, J.kz, J.h, ic, kr, comp, ox, oz) *
                     psi[q][b];
            }
            v = -v;
        }
        J.H2[j * kNT + k] = v;
        J.H2[k * kNT + j] = v;
    }
}

__global__ void dual_force_kernel(const DualJob* __restrict__ jobs, int njobs) {
    for (int j = blockIdx.y; j < njobs; j += gridDim.y) {
        const DualJob& J = jobs[j];
        const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
        if (e >= (size_t)J.nsteps * J.nrec) continue;
        const int s = (int)(e / J.nrec), r = (int)(e % J.nrec);
        const size_t src = (size_t)(J.nsteps - s) * J.nrec + r;   // level N - s
        const float2 y = J.ystar[src], g = J.ghat[src], z = J.noise[src];
        const double sigma = J.sigma, sc = J.w_inv / (sigma * sigma);
        float2 o;
        o.x = (float)((((double)y.x - (double)g.x) + sigma * (double)z.x) * sc);
        o.y = (float)((((double)y.y - (double)g.y) + sigma * (double)z.y) * sc);
        J.rforce[e] = o;
    }
}

}  // namespace

void launch_source_tables(const SourceJob* jobs, int njobs, int /*max_nsteps*/,
                          hipStream_t s) {
    if (njobs <= 0) return;
    source_kernel<<<njobs, 256, 0, s>>>(jobs);
}

void launch_layered_coef(const double* rho, const double* lam, const double* mu,
                         int nz, double h, double dt, float* coef, hipStream_t s) {
    layered_coef_kernel<<<(nz + 127) / 128, 128, 0, s>>>(rho, lam, mu, nz, h, dt, coef);
}

void launch_nodal_coef(const double* rho, const double* lam, const double* mu,
                       int nx, int nz, int pitch, double h, double dt, float* coef,
                       hipStream_t s) {
    const size_t plane = (size_t)nz * pitch;
    size_t blocks = (plane + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    nodal_coef_kernel<<<(unsigned)blocks, 256, 0, s>>>(rho, lam, mu, nx, nz, pitch, h,
                                                        dt, coef);
}

void launch_h2(const H2Job* jobs, int njobs, hipStream_t s) {
    if (njobs > 0) h2_kernel<<<njobs, 128, 0, s>>>(jobs);
}

void launch_dual_force(const DualJob* jobs, int njobs, size_t max_elems, hipStream_t s) {
    if (njobs <= 0 || max_elems == 0) return;
    const dim3 grid((unsigned)((max_elems + 255) / 256), (unsigned)(njobs < 65535 ? njobs : 65535));
    dual_force_kernel<<<grid, 256, 0, s>>>(jobs, njobs);
}

}  // namespace eig
