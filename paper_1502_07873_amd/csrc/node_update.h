// Per-node leapfrog updates shared by every stencil kernel (the tiled
// kernels and the LDS-resident one): the same operands pass through the
// same inline code, so all of them produce bitwise-identical fields.  Also
// the explicit global-memory accessors the kernels use.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace eig {

namespace {

// Pointers read out of a descriptor are generic; loads through them would be
// FLAT instructions.  These accessors address global memory explicitly.
#if defined(__HIP_DEVICE_COMPILE__)
#define GAS __attribute__((address_space(1)))
#else
#define GAS
#endif
typedef float fv2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float2 ld2(const float2* p, size_t i) {
    const fv2 v = ((const GAS fv2*)p)[i];
    return make_float2(v.x, v.y);
}
__device__ __forceinline__ void st2(float2* p, size_t i, float2 v) {
    fv2 w;
    w.x = v.x;
    w.y = v.y;
    ((GAS fv2*)p)[i] = w;
}
typedef float fv4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld4(const float2* p, size_t i) {  // i even
    const fv4 v = *(const GAS fv4*)((const GAS fv2*)p + i);
    return make_float4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st4(float2* p, size_t i, float4 v) {  // i even
    fv4 w;
    w.x = v.x;
    w.y = v.y;
    w.z = v.z;
    w.w = v.w;
    *(GAS fv4*)((GAS fv2*)p + i) = w;
}
__device__ __forceinline__ float ld1(const float* p, size_t i) {
    return ((const GAS float*)p)[i];
}
__device__ __forceinline__ int ldi(const int32_t* p, size_t i) {
    return ((const GAS int32_t*)p)[i];
}

// One row of u^m seen from one node: centre values and the sum and
// difference of the x-neighbours.
struct NodeRow {
    float u, v;      // centre
    float dxu, dxv;  // w_{i+1} - w_{i-1}
    float sxu, sxv;  // w_{i+1} + w_{i-1}
};

__device__ __forceinline__ NodeRow node_row(float u, float v, float lu, float lv,
                                            float ru, float rv) {
    NodeRow r;
    r.u = u;
    r.v = v;
    r.dxu = ru - lu;
    r.dxv = rv - lv;
    r.sxu = ru + lu;
    r.sxv = rv + lv;
    return r;
}

struct LayerCoef {
    float c[kFco + 1];
};

// Row k of a depth-only coefficient table (wave-uniform: scalar loads).
__device__ __forceinline__ LayerCoef load_coef(const float* coef, int k) {
    LayerCoef r;
    const size_t cb = (size_t)k * kCoefStride;
#pragma unroll
    for (int j = 0; j <= kFco; ++j) r.c[j] = ld1(coef, cb + j);
    return r;
}

// u^{m+1} at one node of a depth-only medium.  Every stencil variant calls
// this, so all of them produce bitwise-identical fields.
__device__ __forceinline__ float2 layered_update(const LayerCoef& c, const NodeRow& rm,
                                                 const NodeRow& rc, const NodeRow& rn,
                                                 float upu, float upv, bool src, float fsv,
                                                 float wu, float wv) {
    float au = c.c[kCxxU] * (rc.sxu - 2.f * rc.u) + c.c[kCzpU] * (rn.u - rc.u)
             - c.c[kCzmU] * (rc.u - rm.u) + c.c[kCmpU] * rn.dxv
             - c.c[kCmmU] * rm.dxv + c.c[kCm0U] * rc.dxv;
    float av = c.c[kCxxV] * (rc.sxv - 2.f * rc.v) + c.c[kCzpV] * (rn.v - rc.v)
             - c.c[kCzmV] * (rc.v - rm.v) + c.c[kCmpV] * rn.dxu
             - c.c[kCmmV] * rm.dxu + c.c[kCm0V] * rc.dxu;
    if (src) {
        au += fsv * wu;
        av += fsv * wv;
    }
    float2 nw;
    nw.x = rc.u + ((rc.u - upu) + au);
    nw.y = rc.v + ((rc.v - upv) + av);
    return nw;
}

// An opaque copy: the compiler may not fuse the product that made x into a
// later addition, so x enters every use rounded, as it does after a DPP move.
__device__ __forceinline__ float pinned(float x) {
    __asm__ volatile("" : "+v"(x));
    return x;
}

// Nodal media: coef = three planes (lambda, mu, s = dt^2/(rho h^2)).
//
// Operands of the nodal operator at one node (i, k): the node's own values,
// its x-neighbours on row k, rows k+1 and k-1 (centre values and the
// x-difference w_{i+1} - w_{i-1}), and the x-neighbours' products
// p = lambda Dz v and q = mu Dz u (Dz over rows k+1, k-1, or k+1, k on the
// free surface).  Every nodal variant hands nodal_accel / nodal_new the same
// operand values, so all of them produce bitwise-identical fields.
struct NodalView {
    float u, v, lam, mu;                   // node (i, k)
    float uL, uR, vL, vR, aL, aR, mL, mR;  // x-neighbours on row k (a = lambda + 2 mu)
    float un, vn, lamn, mun, dxun, dxvn;   // row k+1
    float um, vm, lamm, mum, dxum, dxvm;   // row k-1 (unused on the free surface)
    float pR, pL, qR, qL;                  // the x-neighbours' p and q
};

// Acceleration terms at one node, before the scaling by s.  Every product
// that is fused into a sum is written as an fmaf and nothing else is fused
// (contraction off here), so the rounding does not depend on how the caller's
// code around it is laid out: a kernel that knows the row's branch at compile
// time rounds exactly as one that branches at run time.
__device__ __forceinline__ float2 nodal_accel(const NodalView& n, bool top) {
#pragma clang fp contract(off)
    const float ac = __builtin_fmaf(2.f, n.mu, n.lam);
    const float an = __builtin_fmaf(2.f, n.mun, n.lamn);
    // a b - c d as fma(a, b, -(c d)).  The factors 1/2 and 1/4 are exact, so
    // c (x + y) = c x + c y and c x + z = fma(c, x, z) bit for bit.
    const float xu = __builtin_fmaf(ac + n.aR, n.uR - n.u, -((n.aL + ac) * (n.u - n.uL)));
    const float xv = __builtin_fmaf(n.mu + n.mR, n.vR - n.v, -((n.mL + n.mu) * (n.v - n.vL)));
    float au, av;
    if (top) {
        const float dxu_c = n.uR - n.uL, dxv_c = n.vR - n.vL;
        au = __builtin_fmaf(n.mu + n.mun, n.un - n.u, 0.5f * xu);
        av = __builtin_fmaf(ac + an, n.vn - n.v, 0.5f * xv);
        // 1/2 [lam_{i+1,0} (v_{i+1,1}-v_{i+1,0}) - lam_{i-1,0} (...)]
        au = __builtin_fmaf(0.5f, (n.pR - n.pL) + __builtin_fmaf(n.mu, dxv_c, n.mun * n.dxvn), au);
        av = __builtin_fmaf(0.5f, __builtin_fmaf(n.lam, dxu_c, n.lamn * n.dxun) + (n.qR - n.qL), av);
    } else {
        const float am = __builtin_fmaf(2.f, n.mum, n.lamm);
        au = 0.5f * (xu + __builtin_fmaf(n.mu + n.mun, n.un - n.u, -((n.mum + n.mu) * (n.u - n.um))));
        av = 0.5f * (xv + __builtin_fmaf(ac + an, n.vn - n.v, -((am + ac) * (n.v - n.vm))));
        // 1/4 [lam_{i+1,k} Dz v_{i+1} - lam_{i-1,k} Dz v_{i-1}], Dz w = w_{k+1} - w_{k-1}
        au = __builtin_fmaf(0.25f, (n.pR - n.pL) + __builtin_fmaf(n.mun, n.dxvn, -(n.mum * n.dxvm)), au);
        av = __builtin_fmaf(0.25f, __builtin_fmaf(n.lamn, n.dxun, -(n.lamm * n.dxum)) + (n.qR - n.qL), av);
    }
    return make_float2(au, av);
}

// u^{m+1} from the acceleration terms, s, u^m, u^{m-1} and the forcing:
// inj 1 adds a receiver force density (w0, w1) (dual solves), inj 2 the
// source window weights (w0, w1) times the series value; dt^2/rho f = s h^2 f.
// Fused products explicit, as in nodal_accel.
__device__ __forceinline__ float2 nodal_new(float2 acc, float sc, float u, float v, float upu,
                                           float upv, int inj, float h2, float sval,
                                           float w0, float w1) {
#pragma clang fp contract(off)
    float au = acc.x * sc, av = acc.y * sc;
    if (inj == 1) {
        au = __builtin_fmaf(sc * h2, w0, au);
        av = __builtin_fmaf(sc * h2, w1, av);
    } else if (inj == 2) {
        const float f = sc * h2 * sval;
        au = __builtin_fmaf(f, w0, au);
        av = __builtin_fmaf(f, w1, av);
    }
    float2 nw;
    nw.x = u + ((u - upu) + au);
    nw.y = v + ((v - upv) + av);
    return nw;
}

// U(i, k) gives u^m, L(i, k) and M(i, k) lambda and mu, S() the node's
// dt^2/(rho h^2) (each from device memory or LDS); up is u^{m-1} at the node.
// ROW: 0 any row, 1 a row below the surface, 2 the surface row (a caller
// that knows which drops the other branch; the arithmetic is the same).
template <int ROW = 0, class UF, class LF, class MF, class SF>
__device__ __forceinline__ float2 nodal_node_gen(UF U, LF L, MF M, SF S, float2 up, int i, int k,
                                                 int inj, float h2, float sval, float w0,
                                                 float w1) {
    const bool top = ROW == 0 ? k == 0 : ROW == 2;
    NodalView n;
    const float2 c = U(i, k), l = U(i - 1, k), r = U(i + 1, k);
    n.u = c.x;
    n.v = c.y;
    n.lam = L(i, k);
    n.mu = M(i, k);
    n.uL = l.x;
    n.uR = r.x;
    n.vL = l.y;
    n.vR = r.y;
    const float lL = L(i - 1, k), mL = M(i - 1, k), lR = L(i + 1, k), mR = M(i + 1, k);
    n.aL = pinned(lL + 2.f * mL);
    n.aR = pinned(lR + 2.f * mR);
    n.mL = mL;
    n.mR = mR;
    const float2 cn = U(i, k + 1), ln = U(i - 1, k + 1), rn = U(i + 1, k + 1);
    n.un = cn.x;
    n.vn = cn.y;
    n.lamn = L(i, k + 1);
    n.mun = M(i, k + 1);
    n.dxun = rn.x - ln.x;
    n.dxvn = rn.y - ln.y;
    float pR, pL, qR, qL;
    if (top) {
        n.um = n.vm = n.lamm = n.mum = n.dxum = n.dxvm = 0.f;
        pR = lR * (rn.y - r.y);
        pL = lL * (ln.y - l.y);
        qR = mR * (rn.x - r.x);
        qL = mL * (ln.x - l.x);
    } else {
        const float2 cm = U(i, k - 1), lm = U(i - 1, k - 1), rm = U(i + 1, k - 1);
        n.um = cm.x;
        n.vm = cm.y;
        n.lamm = L(i, k - 1);
        n.mum = M(i, k - 1);
        n.dxum = rm.x - lm.x;
        n.dxvm = rm.y - lm.y;
        pR = lR * (rn.y - rm.y);
        pL = lL * (ln.y - lm.y);
        qR = mR * (rn.x - rm.x);
        qL = mL * (ln.x - lm.x);
    }
    n.pR = pinned(pR);
    n.pL = pinned(pL);
    n.qR = pinned(qR);
    n.qL = pinned(qL);
    const float2 acc = nodal_accel(n, top);
    return nodal_new(acc, S(), n.u, n.v, up.x, up.y, inj, h2, sval, w0, w1);
}

// The same with the coefficient planes in device memory, row pitch `pitch`.
template <class UF>
__device__ __forceinline__ float2 nodal_node_at(UF U, float2 up, const float* LAM,
                                                const float* MU, const float* SC, int pitch,
                                                int i, int k, int inj, float h2, float sval,
                                                float w0, float w1) {
    auto L = [&](int ii, int kk) { return ld1(LAM, (size_t)kk * pitch + ii); };
    auto M = [&](int ii, int kk) { return ld1(MU, (size_t)kk * pitch + ii); };
    auto S = [&]() { return ld1(SC, (size_t)k * pitch + i); };
    return nodal_node_gen(U, L, M, S, up, i, k, inj, h2, sval, w0, w1);
}

}  // namespace

}  // namespace eig
