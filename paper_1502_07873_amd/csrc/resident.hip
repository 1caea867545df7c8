// Leapfrog solves resident in LDS: small grids advanced through their whole
// time loop by one workgroup each, in one launch.
#include "ce.h"
#include "internal.h"
#include "node_update.h"

namespace eig {

namespace {

// Resident solves (variants 21, 22): a grid whose two field levels fit one
// workgroup's LDS (2 nx nz float2, rows nx nodes apart) is advanced through
// its whole time loop by one workgroup of 16 waves, so the fields never
// leave the CU; one barrier per step separates the levels.  Level m sits in
// LDS half m & 1 and u^{m+1} overwrites u^{m-1} in place (every node is
// read at the old level and written only by its owner).
//
// Work split: the W = nx-2 free columns times the nz-1 free rows are cut
// into nb = floor(1024 / W) row bands, and thread t takes column t mod W of
// band t div W (threads past nb W rest; a grid wider than 1024 columns takes
// several passes of one band).  Lanes are thus packed across band
// boundaries instead of rounding each band up to whole waves: 99 columns
// leave 34 of 1024 lanes idle rather than 29 of every 128.  A thread
// streams down its band keeping rows k-1, k, k+1 as in the one-node
// kernels.  Nothing inside a step waits on device memory: the forcing
// window weights and, for depth-only media, the coefficient table (nz rows
// of kCoefStride floats, read per lane) are staged in LDS after the
// fields, the edge nodes' coefficients are held in registers, the receiver
// map is read once and the series value one step ahead.  Absorbing edge
// nodes follow in the same phase: their relation reads only u^m and the
// node's own u^{m-1}.  The per-node arithmetic is that of the one-node
// kernels (layered_update, nodal_node_at, ce_edge_update), so the fields
// are bitwise those of every variant.
constexpr int kResWaves = 16;
constexpr int kResThreads = 64 * kResWaves;
constexpr int kResEdgePerThread = kResidentMaxEdge / kResThreads;

template <int KIND>
__global__ void __launch_bounds__(kResThreads)
stencil_resident(const SolveDesc* __restrict__ descs, const int2* __restrict__ tiles,
                 int ntiles) {
    extern __shared__ float2 res_lds[];
    if ((int)blockIdx.x >= ntiles) return;
    const int2 te = tiles[blockIdx.x];
    const SolveDesc* d = descs + __builtin_amdgcn_readfirstlane(te.x);
    const bool absorbing = __builtin_amdgcn_readfirstlane(te.y) != 0;
    const int nx = d->nx, nz = d->nz, nsteps = d->nsteps;
    const int plane = nx * nz;
    for (int j = threadIdx.x; j < 2 * plane; j += kResThreads)
        res_lds[j] = make_float2(0.f, 0.f);
    float* const srcw_lds = (float*)(res_lds + 2 * plane);     // 2 kSrcW^2 floats
    float* const coef_lds = srcw_lds + kResSrcwFloats;         // depth-only media
    for (int j = threadIdx.x; j < 2 * kSrcW * kSrcW; j += kResThreads)
        srcw_lds[j] = ld1(d->srcw, j);
    if constexpr (KIND == EIG_MEDIUM_LAYERED)
        for (int j = threadIdx.x; j < nz * kCoefStride; j += kResThreads)
            coef_lds[j] = ld1(d->coef, j);
    const int W = nx - 2;           // free columns 1..nx-2
    const int nrow = nz - 1;        // free rows 0..nz-2
    const int nb = max(1, kResThreads / W);
    const int npair = nb * W;       // (band, column) pairs
    const int nedge = 2 * nz + nx - 2;
    const int si0 = d->src_i0, sk0 = d->src_k0;
    const float* srcs = d->srcs;
    float2* traces = d->traces;
    const int nrec = d->nrec;
    const float2* rfz = d->rforce;
    float2* wrec = d->wrec;
    const float* coef = d->coef;
    const int cpitch = d->pitch;
    const size_t cplane = (size_t)nz * cpitch;
    const float h2 = d->h2;
    CeCoef ecoef[kResEdgePerThread];
#pragma unroll
    for (int q = 0; q < kResEdgePerThread; ++q) {
        const int e = threadIdx.x + q * kResThreads;
        ecoef[q] = CeCoef{0.f, 0.f, 0.f};
        if (absorbing && e < nedge) {
            const int2 ik = ce_edge_pos(nx, nz, e);
            ecoef[q] = ce_coef(*d, ik.x, ik.y);
        }
    }
    // the thread's (band, column) pair of its first pass and its receiver,
    // fixed over the time loop
    const int b_first = (int)threadIdx.x / W;
    const int i_first = (int)threadIdx.x - b_first * W + 1;
    const int kb_first = b_first * nrow / nb, ke_first = (b_first + 1) * nrow / nb;
    int rec_first = -1;   // only read where the band starts at the surface
    if ((int)threadIdx.x < npair && kb_first == 0) rec_first = ldi(d->recmap, i_first);
    __syncthreads();
    float sval_next = nsteps > 0 ? ld1(srcs, 0) : 0.f;
    for (int m = 0; m < nsteps; ++m) {
        const float2* Q = res_lds + ((m & 1) ? plane : 0);  // u^m
        float2* P = res_lds + ((m & 1) ? 0 : plane);        // u^{m-1} -> u^{m+1}
        const float sval = sval_next;
        if (m + 1 < nsteps) sval_next = ld1(srcs, m + 1);
        for (int v = threadIdx.x; v < npair; v += kResThreads) {
            const bool first = v == (int)threadIdx.x;
            int i = i_first, kb = kb_first, ke = ke_first;
            if (!first) {  // grids wider than one pass
                const int b = v / W;
                i = v - b * W + 1;
                kb = b * nrow / nb;
                ke = (b + 1) * nrow / nb;
            }
            const int di = i - si0;
            const bool src_lane = di >= 0 && di < kSrcW;
            int rec = -1;
            if (kb == 0) rec = first ? rec_first : ldi(d->recmap, i);
            if constexpr (KIND == EIG_MEDIUM_LAYERED) {
                auto row = [&](int k) {
                    const float2* r = Q + k * nx + i;
                    const float2 l = r[-1], c = r[0], rr = r[1];
                    return node_row(c.x, c.y, l.x, l.y, rr.x, rr.y);
                };
                // rows of the source window and the surface row take the
                // forcing and receiver paths; the other rows are the plain
                // update
                auto update = [&](int k, const NodeRow& rm, const NodeRow& rc,
                                  const NodeRow& rn) {
                    LayerCoef cf;
#pragma unroll
                    for (int j = 0; j <= kFco; ++j) cf.c[j] = coef_lds[k * kCoefStride + j];
                    const float2 up = P[k * nx + i];
                    const int dk = k - sk0;
                    if (k != 0 && (unsigned)dk >= (unsigned)kSrcW) {
                        P[k * nx + i] = layered_update(cf, rm, rc, rn, up.x, up.y, false, 0.f,
                                                       0.f, 0.f);
                        return;
                    }
                    const bool in_win = src_lane && dk >= 0 && dk < kSrcW;
                    bool src = in_win;
                    float wu = 0.f, wv = 0.f, fsv = cf.c[kFco] * sval;
                    if (src) {
                        wu = srcw_lds[(0 * kSrcW + dk) * kSrcW + di];
                        wv = srcw_lds[(1 * kSrcW + dk) * kSrcW + di];
                    }
                    if (rfz && k == 0 && rec >= 0) {  // dual solve: receiver injection
                        const float2 rf = ld2(rfz, (size_t)m * nrec + rec);
                        src = true;
                        fsv = cf.c[kFco];
                        wu = rf.x;
                        wv = rf.y;
                    }
                    const float2 nw = layered_update(cf, rm, rc, rn, up.x, up.y, src, fsv, wu, wv);
                    P[k * nx + i] = nw;
                    if (k == 0 && rec >= 0) st2(traces, (size_t)(m + 1) * nrec + rec, nw);
                    if (wrec && in_win)
                        st2(wrec, (size_t)m * (kSrcW * kSrcW) + dk * kSrcW + di, nw);
                };
                NodeRow r0 = NodeRow{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
                if (kb > 0) r0 = row(kb - 1);
                NodeRow r1 = row(kb);
                int k = kb;
                // three rows per trip: the rows rotate through registers
                for (; k + 3 <= ke; k += 3) {
                    const NodeRow r2 = row(k + 1);
                    update(k, r0, r1, r2);
                    const NodeRow r3 = row(k + 2);
                    update(k + 1, r1, r2, r3);
                    const NodeRow r4 = row(k + 3);
                    update(k + 2, r2, r3, r4);
                    r0 = r3;
                    r1 = r4;
                }
                for (; k < ke; ++k) {
                    const NodeRow r2 = row(k + 1);
                    update(k, r0, r1, r2);
                    r0 = r1;
                    r1 = r2;
                }
            } else {
                const float* LAM = coef;
                const float* MU = coef + cplane;
                const float* SC = coef + 2 * cplane;
                auto U = [&](int ii, int kk) { return Q[kk * nx + ii]; };
                for (int k = kb; k < ke; ++k) {
                    const int dk = k - sk0;
                    const bool in_win = src_lane && dk >= 0 && dk < kSrcW;
                    int inj = 0;
                    float w0 = 0.f, w1 = 0.f;
                    if (rfz && k == 0 && rec >= 0) {  // dual solve: receiver injection
                        const float2 rf = ld2(rfz, (size_t)m * nrec + rec);
                        inj = 1;
                        w0 = rf.x;
                        w1 = rf.y;
                    } else if (in_win) {
                        inj = 2;
                        w0 = srcw_lds[(0 * kSrcW + dk) * kSrcW + di];
                        w1 = srcw_lds[(1 * kSrcW + dk) * kSrcW + di];
                    }
                    const float2 nw = nodal_node_at(U, P[k * nx + i], LAM, MU, SC, cpitch, i, k,
                                                    inj, h2, sval, w0, w1);
                    P[k * nx + i] = nw;
                    if (k == 0 && rec >= 0) st2(traces, (size_t)(m + 1) * nrec + rec, nw);
                    if (wrec && in_win)
                        st2(wrec, (size_t)m * (kSrcW * kSrcW) + dk * kSrcW + di, nw);
                }
            }
        }
        if (absorbing) {
#pragma unroll
            for (int q = 0; q < kResEdgePerThread; ++q) {
                const int e = threadIdx.x + q * kResThreads;
                if (e < nedge) ce_edge_update(*d, Q, P, nx, e, ecoef[q]);
            }
        }
        __syncthreads();
    }
}

}  // namespace

void launch_resident(const SolveDesc* descs, const int2* tiles, int ntiles, int kind,
                     size_t lds_bytes, hipStream_t s) {
    if (ntiles <= 0) return;
    // allow dynamic LDS up to the whole 160 KiB of a CU for this kernel (on
    // the current device; idempotent, once per wave)
    const void* fn = kind == EIG_MEDIUM_NODAL ? (const void*)stencil_resident<EIG_MEDIUM_NODAL>
                                              : (const void*)stencil_resident<EIG_MEDIUM_LAYERED>;
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kResidentLdsBytes);
    (void)hipGetLastError();
    if (kind == EIG_MEDIUM_NODAL)
        stencil_resident<EIG_MEDIUM_NODAL><<<ntiles, kResThreads, lds_bytes, s>>>(
            descs, tiles, ntiles);
    else
        stencil_resident<EIG_MEDIUM_LAYERED><<<ntiles, kResThreads, lds_bytes, s>>>(
            descs, tiles, ntiles);
}

}  // namespace eig
