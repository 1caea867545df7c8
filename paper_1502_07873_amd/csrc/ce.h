// First-order Clayton-Engquist updates of absorbing edge nodes, shared by the
// edge kernel and by the one-step stencils that update the edges of their
// own tiles: the same operands give the same bits in both.
//
// Every component w of an edge node takes the form
//   w^{m+1} = ((1 - a) w^{m-1} + 2 (a w_in + T)) / (1 + a)
// with w_in the same component one node inside, T a tangential difference
// (times h) of the other component, a = c dt / h for that component's wave
// speed, and T's factor a or lambda dt / (rho c_p h) (the relation and its
// time-centred reading are set out in boundary.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace eig {

// The two sums are explicit FMAs: which product a compiler would otherwise
// fuse depends on the surrounding code, and the edge kernel and the stencils
// must round alike.
__device__ __forceinline__ float ce_new(float a, float prev, float in, float tang) {
    return __builtin_fmaf(1.f - a, prev, 2.f * __builtin_fmaf(a, in, tang)) / (1.f + a);
}

// Node of a side column (sg = 1 at i = 0, -1 at i = nx-1) at row k: up and dn
// are u^m at rows min(k+1, nz-1) and max(k-1, 0) of the column, half is 1 at
// the ends of the column and 1/2 elsewhere, in is u^m one node inside the
// grid on row k, old is u^{m-1} at the node.
__device__ __forceinline__ float2 ce_side(float ap, float as, float l, float sg, float half,
                                          float2 up, float2 dn, float2 in, float2 old) {
    const float dzu = half * (up.x - dn.x), dzv = half * (up.y - dn.y);
    float2 nw;
    nw.x = ce_new(ap, old.x, in.x, sg * l * dzv);
    nw.y = ce_new(as, old.y, in.y, sg * as * dzu);
    return nw;
}

// Node of the bottom row (1 <= i <= nx-2): ddu, ddv are u^m(i+1) - u^m(i-1)
// on the bottom row, in is u^m one row up, old is u^{m-1} at the node.
__device__ __forceinline__ float2 ce_bottom(float ap, float as, float l, float ddu, float ddv,
                                            float2 in, float2 old) {
    const float dxu = 0.5f * ddu, dxv = 0.5f * ddv;
    float2 nw;
    nw.x = ce_new(as, old.x, in.x, -as * dxv);
    nw.y = ce_new(ap, old.y, in.y, -l * dxu);
    return nw;
}

struct CeCoef {
    float ap, as, l;
};

// a_p = c_p dt / h, a_s = c_s dt / h and lambda dt / (rho c_p h) at node (i, k)
__device__ __forceinline__ CeCoef ce_coef(const SolveDesc& d, int i, int k) {
    CeCoef c;
    if (d.medium_kind == EIG_MEDIUM_NODAL) {
        const size_t plane = (size_t)d.nz * d.pitch, o = (size_t)k * d.pitch + i;
        const float lam = d.coef[o], mu = d.coef[plane + o], sc = d.coef[2 * plane + o];
        c.ap = sqrtf((lam + 2.f * mu) * sc);   // sc = dt^2 / (rho h^2)
        c.as = sqrtf(mu * sc);
        c.l = lam * sc / c.ap;
    } else {
        const float* r = d.coef + (size_t)k * kCoefStride;
        c.ap = r[kCeP];
        c.as = r[kCeS];
        c.l = r[kCeL];
    }
    return c;
}

// Grid node (i, k) of edge node e: nodes 0..nz-1 are the left column,
// nz..2nz-1 the right column (corners included), then the bottom row's inner
// nodes i = 1..nx-2.
__device__ __forceinline__ int2 ce_edge_pos(int nx, int nz, int e) {
    if (e < 2 * nz) return make_int2(e < nz ? 0 : nx - 1, e < nz ? e : e - nz);
    return make_int2(e - 2 * nz + 1, nz - 1);
}

// Edge node e of solve d with coefficients c, u^m in Q and u^{m-1} in P
// (overwritten with u^{m+1}), rows `pitch` nodes apart (device memory or
// LDS).
__device__ __forceinline__ void ce_edge_update(const SolveDesc& d, const float2* Q, float2* P,
                                               int pitch, int e, const CeCoef& c) {
    const int nx = d.nx, nz = d.nz;
    if (e < 2 * nz) {
        const bool left = e < nz;
        const int k = left ? e : e - nz;
        const int i = left ? 0 : nx - 1, ii = left ? 1 : nx - 2;
        const int ka = k == 0 ? 0 : k - 1, kb = k == nz - 1 ? nz - 1 : k + 1;
        const float half = (k == 0 || k == nz - 1) ? 1.f : 0.5f;
        const float2 up = Q[(size_t)kb * pitch + i], dn = Q[(size_t)ka * pitch + i];
        const float2 in = Q[(size_t)k * pitch + ii];
        const float2 old = P[(size_t)k * pitch + i];
        P[(size_t)k * pitch + i] =
            ce_side(c.ap, c.as, c.l, left ? 1.f : -1.f, half, up, dn, in, old);
    } else {
        const int i = e - 2 * nz + 1, k = nz - 1;
        const float2 r = Q[(size_t)k * pitch + i + 1], l = Q[(size_t)k * pitch + i - 1];
        const float2 in = Q[(size_t)(k - 1) * pitch + i];
        const float2 old = P[(size_t)k * pitch + i];
        P[(size_t)k * pitch + i] = ce_bottom(c.ap, c.as, c.l, r.x - l.x, r.y - l.y, in, old);
    }
}

__device__ __forceinline__ void ce_edge_node_at(const SolveDesc& d, const float2* Q, float2* P,
                                                int pitch, int e) {
    const int2 ik = ce_edge_pos(d.nx, d.nz, e);
    ce_edge_update(d, Q, P, pitch, e, ce_coef(d, ik.x, ik.y));
}

// Edge node e of solve d at its step m, fields in the solve's buffers.
__device__ __forceinline__ void ce_edge_node(const SolveDesc& d, int m, int e) {
    const float2* Q = (m & 1) ? d.buf1 : d.buf0;  // u^m
    float2* P = (m & 1) ? d.buf0 : d.buf1;        // u^{m-1} -> u^{m+1}
    ce_edge_node_at(d, Q, P, d.pitch, e);
}

// Absorbing edges as extra wavefronts of a stencil launch: tile entries
// (solve, kEdgeStrip << 16 | part) ask a wave for edge nodes
// part * kEdgeTileNodes .. +kEdgeTileNodes of that solve.  The edge relation
// reads only u^m and the node's own u^{m-1}, and the interior waves never
// write edge nodes, so both kinds of wave share one launch.
__device__ __forceinline__ bool ce_edge_tile(const SolveDesc* descs, int2 te, int step,
                                             int lane) {
    const int sc = __builtin_amdgcn_readfirstlane(te.y);
    if ((sc >> 16) != kEdgeStrip) return false;
    const SolveDesc& d = descs[__builtin_amdgcn_readfirstlane(te.x)];
    const int m = step - d.start;
    if (m < 0 || m >= d.nsteps) return true;
    const int nb = 2 * d.nz + d.nx - 2;
    const int e0 = (sc & 0xffff) * kEdgeTileNodes, e1 = min(nb, e0 + kEdgeTileNodes);
    for (int e = e0 + lane; e < e1; e += 64) ce_edge_node(d, m, e);
    return true;
}

}  // namespace eig
