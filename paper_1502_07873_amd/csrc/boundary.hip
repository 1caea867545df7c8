// Absorbing edges: the first-order Clayton-Engquist relation on the left,
// right and bottom edges (the paper's condition on the artificial boundary,
// discretised with the centred time difference of Section 3.3.1).
//
// At an edge node with outward normal n and tangent t the relation is
//   u_t = -(1/rho) (n n^T / c_p + t t^T / c_s) sigma(u) n.
// Written out with the normal derivative one-sided into the grid, the
// tangential one central (one-sided at the ends of the edge), and the node's
// own same-component term at the mean of levels m+1 and m-1, every component
// w of an edge node takes the form
//   w^{m+1} = ((1 - a) w^{m-1} + 2 (a w_in + b T)) / (1 + a)
// with w_in the same component on the neighbour one node inside, T a
// tangential difference (times h) of the other component, a = c dt / h for
// the wave speed of that component's direction and b = a or
// lambda dt / (rho c_p h):
//   left   (i = 0):    u: a_p, u_{1},     + l Dz v      v: a_s, v_{1},     + a_s Dz u
//   right  (i = nx-1): u: a_p, u_{nx-2},  - l Dz v      v: a_s, v_{nx-2},  - a_s Dz u
//   bottom (k = nz-1): u: a_s, u_{nz-2},  - a_s Dx v    v: a_p, v_{nz-2},  - l Dx u
// (Dz w = (w_{k+1} - w_{k-1}) / 2, or the one-sided difference at the top and
// bottom of a side column; Dx likewise along the bottom row.)  Corners take
// their column's relation.  The interior kernels never write edge nodes, so
// this kernel and the interior step of the same level are independent.
#include "internal.h"

namespace eig {

namespace {

struct CeCoef {
    float ap, as, l;
};

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

__device__ __forceinline__ float ce_new(float a, float prev, float in, float tang) {
    return ((1.f - a) * prev + 2.f * (a * in + tang)) / (1.f + a);
}

// One block per running solve; threads stride over its edge nodes.
__global__ void __launch_bounds__(256) ce_edge_kernel(const SolveDesc* __restrict__ descs,
                                                      int step) {
    const SolveDesc& d = descs[blockIdx.x];
    const int m = step - d.start;
    if (m < 0 || m >= d.nsteps) return;
    const int nx = d.nx, nz = d.nz, pitch = d.pitch;
    const float2* Q = (m & 1) ? d.buf1 : d.buf0;  // u^m
    float2* P = (m & 1) ? d.buf0 : d.buf1;        // u^{m-1} -> u^{m+1}
    const int nb = 2 * nz + nx - 2;
    for (int e = threadIdx.x; e < nb; e += blockDim.x) {
        if (e < 2 * nz) {
            const bool left = e < nz;
            const int k = left ? e : e - nz;
            const int i = left ? 0 : nx - 1, ii = left ? 1 : nx - 2;
            const int ka = k == 0 ? 0 : k - 1, kb = k == nz - 1 ? nz - 1 : k + 1;
            const float half = (k == 0 || k == nz - 1) ? 1.f : 0.5f;
            const float2 up = Q[(size_t)kb * pitch + i], dn = Q[(size_t)ka * pitch + i];
            const float dzu = half * (up.x - dn.x), dzv = half * (up.y - dn.y);
            const float2 in = Q[(size_t)k * pitch + ii];
            const float2 old = P[(size_t)k * pitch + i];
            const CeCoef c = ce_coef(d, i, k);
            const float sg = left ? 1.f : -1.f;
            float2 nw;
            nw.x = ce_new(c.ap, old.x, in.x, sg * c.l * dzv);
            nw.y = ce_new(c.as, old.y, in.y, sg * c.as * dzu);
            P[(size_t)k * pitch + i] = nw;
        } else {
            const int i = e - 2 * nz + 1, k = nz - 1;
            const float2 r = Q[(size_t)k * pitch + i + 1], l = Q[(size_t)k * pitch + i - 1];
            const float dxu = 0.5f * (r.x - l.x), dxv = 0.5f * (r.y - l.y);
            const float2 in = Q[(size_t)(k - 1) * pitch + i];
            const float2 old = P[(size_t)k * pitch + i];
            const CeCoef c = ce_coef(d, i, k);
            float2 nw;
            nw.x = ce_new(c.as, old.x, in.x, -c.as * dxv);
            nw.y = ce_new(c.ap, old.y, in.y, -c.l * dxu);
            P[(size_t)k * pitch + i] = nw;
        }
    }
}

}  // namespace

void launch_ce_edges(const SolveDesc* descs, int n, int step, hipStream_t s) {
    if (n > 0) ce_edge_kernel<<<n, 256, 0, s>>>(descs, step);
}

}  // namespace eig
