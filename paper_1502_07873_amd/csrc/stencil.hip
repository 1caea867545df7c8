// Leapfrog step of the 2-D elastic wave equation for many solves at once,
// with the point-source forcing and the surface receivers fused in.
//
// Scheme (paper Section 3.3.1, full-discrete formulas): at every free node
//   u^{m+1} = 2 u^m - u^{m-1} + dt^2/rho (A_h u^m + f^m),
// A_h the second-order operator made of D+(a D-) terms for the normal
// second derivatives and D0(c D0) terms for the mixed ones, with a
// traction-free top row (depth 0) and rigid left, right and bottom edges.
// The top-row closure is the one that makes A_h the negative gradient of a
// discrete elastic energy with trapezoid weights (so the scheme conserves a
// discrete energy); derived per node, it reads, with a = lambda + 2 mu and
// Dx w_k = w_{i+1,k} - w_{i-1,k}:
//   h^2 (A_h u)_x = a (u_{i+1} - 2u + u_{i-1}) + 2 mu_{1/2} (u_1 - u_0)
//                   + 1/2 (lambda_0 + mu_1) Dx v_1 + 1/2 (mu_0 - lambda_0) Dx v_0
//   h^2 (A_h u)_z = mu (v_{i+1} - 2v + v_{i-1}) + 2 a_{1/2} (v_1 - v_0)
//                   + 1/2 (lambda_1 + mu_0) Dx u_1 + 1/2 (lambda_0 - mu_0) Dx u_0
// (depth-only media; the nodal variant keeps every coefficient per node).
//
// Work decomposition: one wavefront owns a tile of 64 columns and up to
// kTileRows rows of one solve and streams down the rows, keeping the rows
// k-1, k, k+1 of u^m in registers; x-neighbours come from cross-lane moves,
// the two edge lanes fetch the halo columns.  Every u^m value is read from
// HBM once per step (tile halos hit L2), u^{m-1} is read once and u^{m+1}
// written in place of it: 24 bytes of field traffic per grid-point update.
// Depth-only coefficients are per-row scalars (SGPR loads).
#include "ce.h"
#include "internal.h"
#include "node_update.h"
#include "tile.h"

namespace eig {

namespace {

// Variant 0: one node per lane (64 columns per wave), one row of prefetch.
__device__ __forceinline__ void load_row(const float2* Q, size_t off, int i,
                                         int hc, bool hl, float2& c, float2& h) {
    c = ld2(Q, off + i);
    const float2 hv = ld2(Q, off + (hl ? hc : i));
    h.x = hl ? hv.x : 0.f;
    h.y = hl ? hv.y : 0.f;
}

__device__ __forceinline__ NodeRow make_row(float2 c, float2 h) {
    return node_row(c.x, c.y, from_left(c.x, h.x), from_left(c.y, h.y),
                    from_right(c.x, h.x), from_right(c.y, h.y));
}

__global__ void __launch_bounds__(256)
stencil_layered_w1(const SolveDesc* __restrict__ descs, const int2* __restrict__ tiles,
                   int ntiles, int step) {
    TileInfo t;
    if (!decode_tile(descs, tiles, ntiles, step, 64, 32, t)) return;
    const SolveDesc* d = t.d;
    const int lane = threadIdx.x & 63;
    const int m = t.m, x0 = t.x0, kb = t.kb, ke = t.ke;
    const int nx = d->nx, nz = d->nz, pitch = d->pitch;
    const int i = x0 + lane;
    const float2* Q = (m & 1) ? d->buf1 : d->buf0;  // u^m
    float2* P = (m & 1) ? d->buf0 : d->buf1;        // u^{m-1} -> u^{m+1}
    const float* coef = d->coef;
    const bool upd = (i >= 1) && (i <= nx - 2);
    const bool hl = (lane == 0 && x0 > 0) || (lane == 63 && x0 + 64 < nx);
    const int hc = (lane == 0) ? x0 - 1 : x0 + 64;
    const int si0 = d->src_i0, sk0 = d->src_k0;
    const bool src_cols = (si0 < x0 + 64) && (si0 + kSrcW > x0);
    const int di = i - si0;
    const bool src_lane = src_cols && di >= 0 && di < kSrcW;
    const float sval = src_cols ? ld1(d->srcs, m) : 0.0f;
    const float* srcw = d->srcw;
    float2* traces = d->traces;
    const int nrec = d->nrec;
    int rec = -1;
    if (kb == 0) rec = ldi(d->recmap, i);
    const float2* rfz = d->rforce;
    float2* wrec = d->wrec;

    NodeRow rm, rc, rn;
    if (kb == 0) {
        rm = NodeRow{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    } else {
        float2 c, h;
        load_row(Q, (size_t)(kb - 1) * pitch, i, hc, hl, c, h);
        rm = make_row(c, h);
    }
    float2 cc, ch, cn, chn;
    load_row(Q, (size_t)kb * pitch, i, hc, hl, cc, ch);
    load_row(Q, (size_t)(kb + 1) * pitch, i, hc, hl, cn, chn);
    float2 up = ld2(P, (size_t)kb * pitch + i);
    rc = make_row(cc, ch);

    for (int k = kb; k < ke; ++k) {
        float2 cnn = make_float2(0.f, 0.f), chnn = cnn, upn = cnn;
        if (k + 2 <= nz - 1) load_row(Q, (size_t)(k + 2) * pitch, i, hc, hl, cnn, chnn);
        if (k + 1 < ke) upn = ld2(P, (size_t)(k + 1) * pitch + i);
        rn = make_row(cn, chn);
        const LayerCoef cf = load_coef(coef, k);
        const int dk = k - sk0;
        const bool in_win = src_lane && dk >= 0 && dk < kSrcW;
        bool src = in_win;
        float wu = 0.f, wv = 0.f, fsv = cf.c[kFco] * sval;
        if (src) {
            wu = ld1(srcw, (0 * kSrcW + dk) * kSrcW + di);
            wv = ld1(srcw, (1 * kSrcW + dk) * kSrcW + di);
        }
        if (rfz && k == 0 && rec >= 0) {  // dual solve: receiver injection
            const float2 rf = ld2(rfz, (size_t)m * nrec + rec);
            src = true;
            fsv = cf.c[kFco];
            wu = rf.x;
            wv = rf.y;
        }
        const float2 nw = layered_update(cf, rm, rc, rn, up.x, up.y, src, fsv, wu, wv);
        if (upd) {
            st2(P, (size_t)k * pitch + i, nw);
            if (k == 0 && rec >= 0) st2(traces, (size_t)(m + 1) * nrec + rec, nw);
            if (wrec && in_win) st2(wrec, (size_t)m * (kSrcW * kSrcW) + dk * kSrcW + di, nw);
        }
        rm = rc;
        rc = rn;
        cn = cnn;
        chn = chnn;
        up = upn;
    }
}

// Variants 1..: two nodes per lane (128 columns per wave) with 16-byte loads,
// R rows per wave and D rows of prefetch.  Lane l owns columns x0+2l and
// x0+2l+1; the left neighbour of the first and the right neighbour of the
// second come from the adjacent lanes (DPP), lanes 0 and 63 load the halo.
struct Raw2 {
    float4 c;  // (u, v) of the two columns
    float2 h;  // halo column (edge lanes only)
};

// live: the lane's first column lies inside the grid.  Lanes past nx hold
// only padding columns, which stay zero in memory and feed no updated node,
// so their loads are skipped (zeros) and their stores left out.
__device__ __forceinline__ Raw2 load_raw2(const float2* Q, size_t off, int i0, int hc,
                                          bool hl, bool live = true) {
    Raw2 r;
    r.c = make_float4(0.f, 0.f, 0.f, 0.f);
    if (live) r.c = ld4(Q, off + i0);
    r.h = make_float2(0.f, 0.f);
    if (hl) r.h = ld2(Q, off + hc);
    return r;
}

__device__ __forceinline__ void make_rows2(const Raw2& r, NodeRow& a, NodeRow& b) {
    const float lu = from_left(r.c.z, r.h.x), lv = from_left(r.c.w, r.h.y);
    const float ru = from_right(r.c.x, r.h.x), rv = from_right(r.c.y, r.h.y);
    a = node_row(r.c.x, r.c.y, lu, lv, r.c.z, r.c.w);
    b = node_row(r.c.z, r.c.w, r.c.x, r.c.y, ru, rv);
}

template <int R, int D>
__global__ void __launch_bounds__(256)
stencil_layered_w2(const SolveDesc* __restrict__ descs, const int2* __restrict__ tiles,
                   int ntiles, int step) {
    if (edge_wave(descs, tiles, ntiles, step)) return;
    TileInfo t;
    if (!decode_tile(descs, tiles, ntiles, step, 128, R, t)) return;
    const SolveDesc* d = t.d;
    const int lane = threadIdx.x & 63;
    const int m = t.m, x0 = t.x0, kb = t.kb, ke = t.ke;
    const int nx = d->nx, nz = d->nz, pitch = d->pitch;
    const int i0 = x0 + 2 * lane;
    const float2* Q = (m & 1) ? d->buf1 : d->buf0;
    float2* P = (m & 1) ? d->buf0 : d->buf1;
    const float* coef = d->coef;
    const bool upd0 = (i0 >= 1) && (i0 <= nx - 2);
    const bool upd1 = (i0 + 1 <= nx - 2);
    const bool live = i0 < nx;
    const bool hl = (lane == 0 && x0 > 0) || (lane == 63 && x0 + 128 < nx);
    const int hc = (lane == 0) ? x0 - 1 : x0 + 128;
    const int si0 = d->src_i0, sk0 = d->src_k0;
    const bool src_cols = (si0 < x0 + 128) && (si0 + kSrcW > x0);
    const int di0 = i0 - si0, di1 = di0 + 1;
    const bool s0 = src_cols && di0 >= 0 && di0 < kSrcW;
    const bool s1 = src_cols && di1 >= 0 && di1 < kSrcW;
    const float sval = src_cols ? ld1(d->srcs, m) : 0.0f;
    const float* srcw = d->srcw;
    float2* traces = d->traces;
    const int nrec = d->nrec;
    int rec0 = -1, rec1 = -1;
    if (kb == 0) {
        rec0 = ldi(d->recmap, i0);
        rec1 = ldi(d->recmap, i0 + 1);
    }
    const float2* rfz = d->rforce;
    float2* wrec = d->wrec;

    NodeRow am, bm, ac, bc, an, bn;
    if (kb == 0) {
        am = bm = NodeRow{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    } else {
        make_rows2(load_raw2(Q, (size_t)(kb - 1) * pitch, i0, hc, hl, live), am, bm);
    }
    make_rows2(load_raw2(Q, (size_t)kb * pitch, i0, hc, hl, live), ac, bc);
    // prefetch ring: raw rows k+1..k+D of u^m, rows k..k+D-1 of u^{m-1}
    Raw2 q1, q2;
    float4 p0, p1;
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    q1 = load_raw2(Q, (size_t)(kb + 1) * pitch, i0, hc, hl, live);
    p0 = z4;
    if (live) p0 = ld4(P, (size_t)kb * pitch + i0);
    if (D == 2) {
        q2.c = z4;
        q2.h = make_float2(0.f, 0.f);
        if (kb + 2 <= nz - 1) q2 = load_raw2(Q, (size_t)(kb + 2) * pitch, i0, hc, hl, live);
        p1 = z4;
        if (live && kb + 1 < ke) p1 = ld4(P, (size_t)(kb + 1) * pitch + i0);
    }

    for (int k = kb; k < ke; ++k) {
        Raw2 qn;
        qn.c = z4;
        qn.h = make_float2(0.f, 0.f);
        float4 pn = z4;
        if (k + 1 + D <= nz - 1) qn = load_raw2(Q, (size_t)(k + 1 + D) * pitch, i0, hc, hl, live);
        if (live && k + D < ke) pn = ld4(P, (size_t)(k + D) * pitch + i0);
        make_rows2(q1, an, bn);
        const LayerCoef cf = load_coef(coef, k);
        float fsa = cf.c[kFco] * sval, fsb = fsa;
        const int dk = k - sk0;
        const bool row_src = dk >= 0 && dk < kSrcW;
        const bool wa = s0 && row_src, wb = s1 && row_src;
        bool sa = wa, sb = wb;
        float wua = 0.f, wva = 0.f, wub = 0.f, wvb = 0.f;
        if (sa) {
            wua = ld1(srcw, (0 * kSrcW + dk) * kSrcW + di0);
            wva = ld1(srcw, (1 * kSrcW + dk) * kSrcW + di0);
        }
        if (sb) {
            wub = ld1(srcw, (0 * kSrcW + dk) * kSrcW + di1);
            wvb = ld1(srcw, (1 * kSrcW + dk) * kSrcW + di1);
        }
        if (rfz && k == 0) {  // dual solve: receiver injection
            if (rec0 >= 0) {
                const float2 rf = ld2(rfz, (size_t)m * nrec + rec0);
                sa = true;
                fsa = cf.c[kFco];
                wua = rf.x;
                wva = rf.y;
            }
            if (rec1 >= 0) {
                const float2 rf = ld2(rfz, (size_t)m * nrec + rec1);
                sb = true;
                fsb = cf.c[kFco];
                wub = rf.x;
                wvb = rf.y;
            }
        }
        const float2 na = layered_update(cf, am, ac, an, p0.x, p0.y, sa, fsa, wua, wva);
        const float2 nb = layered_update(cf, bm, bc, bn, p0.z, p0.w, sb, fsb, wub, wvb);
        if (wrec) {
            const size_t wb0 = (size_t)m * (kSrcW * kSrcW) + dk * kSrcW;
            if (wa && upd0) st2(wrec, wb0 + di0, na);
            if (wb && upd1) st2(wrec, wb0 + di1, nb);
        }
        // edge and padding columns are never written: rigid edges stay zero,
        // absorbing ones belong to the edge waves of this launch (or to the
        // edge kernel); the u^{m-1} an edge wave may already have replaced
        // feeds only edge results that are discarded here
        if (upd0 && upd1) {
            st4(P, (size_t)k * pitch + i0, make_float4(na.x, na.y, nb.x, nb.y));
        } else if (upd0) {
            st2(P, (size_t)k * pitch + i0, na);
        } else if (upd1) {
            st2(P, (size_t)k * pitch + i0 + 1, nb);
        }
        if (k == 0) {
            if (rec0 >= 0) st2(traces, (size_t)(m + 1) * nrec + rec0, na);
            if (rec1 >= 0) st2(traces, (size_t)(m + 1) * nrec + rec1, nb);
        }
        am = ac;
        bm = bc;
        ac = an;
        bc = bn;
        if (D == 2) {
            q1 = q2;
            q2 = qn;
            p0 = p1;
            p1 = pn;
        } else {
            q1 = qn;
            p0 = pn;
        }
    }
}

// Two leapfrog steps per launch (temporal blocking), depth-only media.
// Pass p takes u^{m-1}, u^m (m = 2p) to u^{m+1} and u^{m+2}; level l lives in
// buffer (l + 1) mod 4, so a pass reads two buffers and writes the other
// two, and no wave ever overwrites data a neighbouring wave still reads.
// Each wave recomputes u^{m+1} on a one-node halo around its 128 x R tile
// (the rows kb-1 and ke, and the columns x0-1 / x0+128 handled as a third
// node by lanes 0 / 63), so field traffic is 32 bytes per node per two
// updates instead of 48.  Both steps use the same per-node update as the
// one-step kernels: the fields are bitwise identical.
struct RawTB {
    float4 c;  // (u, v) of the lane's two columns
    float4 h;  // lanes 0 / 63: the two columns beyond the tile edge
};

__device__ __forceinline__ RawTB load_raw_tb(const float2* Q, size_t off, int i0, int hcol,
                                             bool hl, bool live) {
    RawTB r;
    r.c = make_float4(0.f, 0.f, 0.f, 0.f);
    if (live) r.c = ld4(Q, off + i0);
    r.h = make_float4(0.f, 0.f, 0.f, 0.f);
    if (hl) r.h = ld4(Q, off + hcol);
    return r;
}

// Node rows of the lane's columns A = x0+2l, B = x0+2l+1 and of the halo
// node T (lane 0: x0-1 with neighbours x0-2 | x0; lane 63: x0+128 with
// neighbours x0+127 | x0+129; other lanes: unused).
struct RowTB {
    NodeRow a, b, t;
};

__device__ __forceinline__ RowTB make_row_tb(const RawTB& r, bool first) {
    RowTB o;
    const float eu = first ? r.h.z : r.h.x, ev = first ? r.h.w : r.h.y;
    const float lu = from_left(r.c.z, eu), lv = from_left(r.c.w, ev);
    const float ru = from_right(r.c.x, eu), rv = from_right(r.c.y, ev);
    o.a = node_row(r.c.x, r.c.y, lu, lv, r.c.z, r.c.w);
    o.b = node_row(r.c.z, r.c.w, r.c.x, r.c.y, ru, rv);
    o.t = node_row(eu, ev, first ? r.h.x : r.c.z, first ? r.h.y : r.c.w,
                   first ? r.c.x : r.h.z, first ? r.c.y : r.h.w);
    return o;
}

__device__ __forceinline__ void make_rows_x(float2 xa, float2 xb, float2 xt, NodeRow& a,
                                            NodeRow& b) {
    a = node_row(xa.x, xa.y, from_left(xb.x, xt.x), from_left(xb.y, xt.y), xb.x, xb.y);
    b = node_row(xb.x, xb.y, xa.x, xa.y, from_right(xa.x, xt.x), from_right(xa.y, xt.y));
}

// PART: the tile's strip runs past nx (lanes beyond it are not live); full
// strips compile without the lane predicate.
template <int R, int D, bool PART>
__device__ __forceinline__ void tb2_tile(const SolveDesc* __restrict__ descs,
                                         const int2* __restrict__ tiles, int tile, int pass) {
    const int2 te = tiles[tile];
    const SolveDesc* d = descs + __builtin_amdgcn_readfirstlane(te.x);
    const int sc = __builtin_amdgcn_readfirstlane(te.y);
    const int m = 2 * (pass - d->start);
    if (m < 0 || m >= d->nsteps) return;
    const bool two = m + 1 < d->nsteps;
    const int lane = threadIdx.x & 63;
    const bool first = lane == 0;
    const int nx = d->nx, nz = d->nz, pitch = d->pitch;
    const int x0 = (sc >> 16) * 128;
    const int kb = (sc & 0xffff) * R;
    const int ke = min(kb + R, nz - 1);
    const int i0 = x0 + 2 * lane;
    float2* const bufs[4] = {d->buf0, d->buf1, d->buf2, d->buf3};
    const float2* prev = bufs[m & 3];
    const float2* cur = bufs[(m + 1) & 3];
    float2* out1 = bufs[(m + 2) & 3];
    float2* out2 = bufs[(m + 3) & 3];
    const float* coef = d->coef;
    const bool updA = (i0 >= 1) && (i0 <= nx - 2);
    const bool updB = (i0 + 1 <= nx - 2);
    const bool live = !PART || i0 < nx;
    const int tcol = first ? x0 - 1 : x0 + 128;
    const bool edge = (first && x0 > 0) || (lane == 63 && x0 + 128 < nx);
    const bool updT = edge && tcol >= 1 && tcol <= nx - 2;
    const int hcol = first ? x0 - 2 : x0 + 128;
    // sources (windows tested per row; the halo node may be in the window)
    const int si0 = d->src_i0, sk0 = d->src_k0;
    const bool src_cols = (si0 < x0 + 130) && (si0 + kSrcW > x0 - 1);
    const int dA = i0 - si0, dB = dA + 1, dT = tcol - si0;
    const bool sA = src_cols && dA >= 0 && dA < kSrcW;
    const bool sB = src_cols && dB >= 0 && dB < kSrcW;
    const bool sT = src_cols && dT >= 0 && dT < kSrcW;
    const float sval1 = src_cols ? ld1(d->srcs, m) : 0.f;
    const float sval2 = (src_cols && two) ? ld1(d->srcs, m + 1) : 0.f;
    const float* srcw = d->srcw;
    float2* traces = d->traces;
    const int nrec = d->nrec;
    int recA = -1, recB = -1;
    if (kb == 0) {
        recA = ldi(d->recmap, i0);
        recB = ldi(d->recmap, i0 + 1);
    }
    const NodeRow z = NodeRow{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const float2 z2 = make_float2(0.f, 0.f);

    // step-1 rows [j0, j1] (tile rows plus a one-row halo inside the free rows)
    const int j0 = kb > 0 ? kb - 1 : 0;
    const int j1 = min(ke, nz - 2);
    RowTB um, uc, un;
    if (j0 >= 1) {
        um = make_row_tb(load_raw_tb(cur, (size_t)(j0 - 1) * pitch, i0, hcol, edge, live), first);
    } else {
        um.a = um.b = um.t = z;
    }
    uc = make_row_tb(load_raw_tb(cur, (size_t)j0 * pitch, i0, hcol, edge, live), first);
    // prefetch ring: raw u^m rows j+1..j+D, u^{m-1} rows j..j+D-1 (one row
    // measured fastest: deeper rings cost more than the latency they hide)
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    RawTB rq[D];
    float4 pq[D];
    float2 tq[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
        rq[q].c = z4;
        rq[q].h = z4;
        pq[q] = z4;
        tq[q] = z2;
        if (j0 + 1 + q <= nz - 1) rq[q] = load_raw_tb(cur, (size_t)(j0 + 1 + q) * pitch, i0, hcol, edge, live);
        if (live && j0 + q <= j1) {
            pq[q] = ld4(prev, (size_t)(j0 + q) * pitch + i0);
            if (edge) tq[q] = ld2(prev, (size_t)(j0 + q) * pitch + tcol);
        }
    }
    // u^{m+1} rows k-1 and k for the second step
    NodeRow a2m = z, b2m = z, a2c = z, b2c = z;

    for (int j = j0; j <= j1; ++j) {
        RawTB rnn;
        rnn.c = z4;
        rnn.h = z4;
        float4 pvn = z4;
        float2 ptn = z2;
        if (j + 1 + D <= nz - 1) rnn = load_raw_tb(cur, (size_t)(j + 1 + D) * pitch, i0, hcol, edge, live);
        if (live && j + D <= j1) {
            pvn = ld4(prev, (size_t)(j + D) * pitch + i0);
            if (edge) ptn = ld2(prev, (size_t)(j + D) * pitch + tcol);
        }
        const RawTB rn = rq[0];
        const float4 pv = pq[0];
        const float2 pt = tq[0];
#pragma unroll
        for (int q = 0; q + 1 < D; ++q) {
            rq[q] = rq[q + 1];
            pq[q] = pq[q + 1];
            tq[q] = tq[q + 1];
        }
        rq[D - 1] = rnn;
        pq[D - 1] = pvn;
        tq[D - 1] = ptn;
        un = make_row_tb(rn, first);
        // first step at row j: u^{m+1} at A, B and the halo node
        const LayerCoef cj = load_coef(coef, j);
        const float f1 = cj.c[kFco] * sval1;
        const int dk1 = j - sk0;
        const bool row1 = dk1 >= 0 && dk1 < kSrcW;
        float wua = 0.f, wva = 0.f, wub = 0.f, wvb = 0.f, wut = 0.f, wvt = 0.f;
        if (sA && row1) {
            wua = ld1(srcw, (0 * kSrcW + dk1) * kSrcW + dA);
            wva = ld1(srcw, (1 * kSrcW + dk1) * kSrcW + dA);
        }
        if (sB && row1) {
            wub = ld1(srcw, (0 * kSrcW + dk1) * kSrcW + dB);
            wvb = ld1(srcw, (1 * kSrcW + dk1) * kSrcW + dB);
        }
        if (sT && row1) {
            wut = ld1(srcw, (0 * kSrcW + dk1) * kSrcW + dT);
            wvt = ld1(srcw, (1 * kSrcW + dk1) * kSrcW + dT);
        }
        float2 xa = layered_update(cj, um.a, uc.a, un.a, pv.x, pv.y, sA && row1, f1, wua, wva);
        float2 xb = layered_update(cj, um.b, uc.b, un.b, pv.z, pv.w, sB && row1, f1, wub, wvb);
        float2 xt = layered_update(cj, um.t, uc.t, un.t, pt.x, pt.y, sT && row1, f1, wut, wvt);
        if (!updA) xa = z2;
        if (!updB) xb = z2;
        if (!updT) xt = z2;
        if (j >= kb && j < ke) {
            if (live) st4(out1, (size_t)j * pitch + i0, make_float4(xa.x, xa.y, xb.x, xb.y));
            if (j == 0) {
                if (recA >= 0) st2(traces, (size_t)(m + 1) * nrec + recA, xa);
                if (recB >= 0) st2(traces, (size_t)(m + 1) * nrec + recB, xb);
            }
        }
        NodeRow a2n, b2n;
        make_rows_x(xa, xb, xt, a2n, b2n);
        // second step at row k = j - 1
        const int k = j - 1;
        if (two && k >= kb) {
            const LayerCoef ck = load_coef(coef, k);
            const float f2 = ck.c[kFco] * sval2;
            const int dk2 = k - sk0;
            const bool row2 = dk2 >= 0 && dk2 < kSrcW;
            float qua = 0.f, qva = 0.f, qub = 0.f, qvb = 0.f;
            if (sA && row2) {
                qua = ld1(srcw, (0 * kSrcW + dk2) * kSrcW + dA);
                qva = ld1(srcw, (1 * kSrcW + dk2) * kSrcW + dA);
            }
            if (sB && row2) {
                qub = ld1(srcw, (0 * kSrcW + dk2) * kSrcW + dB);
                qvb = ld1(srcw, (1 * kSrcW + dk2) * kSrcW + dB);
            }
            float2 ya = layered_update(ck, a2m, a2c, a2n, um.a.u, um.a.v, sA && row2, f2, qua, qva);
            float2 yb = layered_update(ck, b2m, b2c, b2n, um.b.u, um.b.v, sB && row2, f2, qub, qvb);
            if (!updA) ya = z2;
            if (!updB) yb = z2;
            if (live) st4(out2, (size_t)k * pitch + i0, make_float4(ya.x, ya.y, yb.x, yb.y));
            if (k == 0) {
                if (recA >= 0) st2(traces, (size_t)(m + 2) * nrec + recA, ya);
                if (recB >= 0) st2(traces, (size_t)(m + 2) * nrec + recB, yb);
            }
        }
        um = uc;
        uc = un;
        a2m = a2c;
        b2m = b2c;
        a2c = a2n;
        b2c = b2n;
    }
    // bottom tile: the last free row's second step sees the rigid row (zeros)
    if (two && ke == nz - 1 && ke - 1 >= kb) {
        const int k = ke - 1;
        const LayerCoef ck = load_coef(coef, k);
        const float f2 = ck.c[kFco] * sval2;
        const int dk2 = k - sk0;
        const bool row2 = dk2 >= 0 && dk2 < kSrcW;
        float qua = 0.f, qva = 0.f, qub = 0.f, qvb = 0.f;
        if (sA && row2) {
            qua = ld1(srcw, (0 * kSrcW + dk2) * kSrcW + dA);
            qva = ld1(srcw, (1 * kSrcW + dk2) * kSrcW + dA);
        }
        if (sB && row2) {
            qub = ld1(srcw, (0 * kSrcW + dk2) * kSrcW + dB);
            qvb = ld1(srcw, (1 * kSrcW + dk2) * kSrcW + dB);
        }
        float2 ya = layered_update(ck, a2m, a2c, z, um.a.u, um.a.v, sA && row2, f2, qua, qva);
        float2 yb = layered_update(ck, b2m, b2c, z, um.b.u, um.b.v, sB && row2, f2, qub, qvb);
        if (!updA) ya = z2;
        if (!updB) yb = z2;
        if (live) st4(out2, (size_t)k * pitch + i0, make_float4(ya.x, ya.y, yb.x, yb.y));
        if (k == 0) {
            if (recA >= 0) st2(traces, (size_t)(m + 2) * nrec + recA, ya);
            if (recB >= 0) st2(traces, (size_t)(m + 2) * nrec + recB, yb);
        }
    }
}

template <int R, int D>
__global__ void __launch_bounds__(256)
stencil_layered_tb2(const SolveDesc* __restrict__ descs, const int2* __restrict__ tiles,
                    int ntiles, int pass) {
    const int tile = __builtin_amdgcn_readfirstlane(
        xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    if (tile >= ntiles) return;
    const int2 te = tiles[tile];
    const int nx = descs[__builtin_amdgcn_readfirstlane(te.x)].nx;
    const int x0 = (__builtin_amdgcn_readfirstlane(te.y) >> 16) * 128;
    if (x0 + 128 <= nx)
        tb2_tile<R, D, false>(descs, tiles, tile, pass);
    else
        tb2_tile<R, D, true>(descs, tiles, tile, pass);
}

// Two leapfrog steps per launch with the halo columns computed up front.
// Same scheme and buffer rotation as stencil_layered_tb2, but u^{m+1} at the
// columns x0-1 and x0+128 (needed by the second step of the tile's edge
// nodes) is formed once per launch for the R+2 first-step rows, one lane per
// (column, row), and parked in LDS; the row loop then carries only the two
// nodes each lane owns (22 % fewer vector instructions, 114 instead of 140
// VGPRs).  The halo nodes go through the same per-node update with the same
// operands, so the fields are bitwise those of every variant.  At 512^2 it
// is 3 % slower than stencil_layered_tb2 (both sit at the machine's copy
// bandwidth; a deeper prefetch ring was slower still); it stays a tuner
// candidate.
template <int R, int D>
__global__ void __launch_bounds__(256)
stencil_layered_tb2h(const SolveDesc* __restrict__ descs, const int2* __restrict__ tiles,
                     int ntiles, int pass) {
    __shared__ float2 halo[kWavesPerBlock][2][R + 2];
    const int tile = __builtin_amdgcn_readfirstlane(
        xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    if (tile >= ntiles) return;
    const int2 te = tiles[tile];
    const SolveDesc* d = descs + __builtin_amdgcn_readfirstlane(te.x);
    const int sc = __builtin_amdgcn_readfirstlane(te.y);
    const int m = 2 * (pass - d->start);
    if (m < 0 || m >= d->nsteps) return;
    const bool two = m + 1 < d->nsteps;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nx = d->nx, nz = d->nz, pitch = d->pitch;
    const int x0 = (sc >> 16) * 128;
    const int kb = (sc & 0xffff) * R;
    const int ke = min(kb + R, nz - 1);
    const int i0 = x0 + 2 * lane;
    float2* const bufs[4] = {d->buf0, d->buf1, d->buf2, d->buf3};
    const float2* prev = bufs[m & 3];
    const float2* cur = bufs[(m + 1) & 3];
    float2* out1 = bufs[(m + 2) & 3];
    float2* out2 = bufs[(m + 3) & 3];
    const float* coef = d->coef;
    const bool updA = (i0 >= 1) && (i0 <= nx - 2);
    const bool updB = (i0 + 1 <= nx - 2);
    const bool live = i0 < nx;
    const bool hl = (lane == 0 && x0 > 0) || (lane == 63 && x0 + 128 < nx);
    const int hc = (lane == 0) ? x0 - 1 : x0 + 128;
    const int si0 = d->src_i0, sk0 = d->src_k0;
    const float sval1 = ld1(d->srcs, m);
    const float sval2 = two ? ld1(d->srcs, m + 1) : 0.f;
    const float* srcw = d->srcw;
    float2* traces = d->traces;
    const int nrec = d->nrec;
    const NodeRow z = NodeRow{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const float2 z2 = make_float2(0.f, 0.f);
    const int j0 = kb > 0 ? kb - 1 : 0;
    const int j1 = min(ke, nz - 2);
    const int nrow = j1 - j0 + 1;

    // u^{m+1} at the halo columns, rows j0..j1 (zero where not a free node)
    for (int it = lane; it < 2 * nrow; it += 64) {
        const int side = it & 1, r = it >> 1, j = j0 + r;
        const int c = side == 0 ? x0 - 1 : x0 + 128;
        float2 xt = z2;
        if (c >= 1 && c <= nx - 2) {
            NodeRow rows[3];
            for (int q = 0; q < 3; ++q) {
                const int jj = j - 1 + q;
                if (jj < 0) {
                    rows[q] = z;
                    continue;
                }
                const size_t o = (size_t)jj * pitch;
                const float2 l = ld2(cur, o + c - 1), ce = ld2(cur, o + c), rr = ld2(cur, o + c + 1);
                rows[q] = node_row(ce.x, ce.y, l.x, l.y, rr.x, rr.y);
            }
            const float2 pt = ld2(prev, (size_t)j * pitch + c);
            const LayerCoef cj = load_coef(coef, j);
            const int dT = c - si0, dk1 = j - sk0;
            const bool s1 = dT >= 0 && dT < kSrcW && dk1 >= 0 && dk1 < kSrcW;
            float wut = 0.f, wvt = 0.f;
            if (s1) {
                wut = ld1(srcw, (0 * kSrcW + dk1) * kSrcW + dT);
                wvt = ld1(srcw, (1 * kSrcW + dk1) * kSrcW + dT);
            }
            xt = layered_update(cj, rows[0], rows[1], rows[2], pt.x, pt.y, s1,
                                cj.c[kFco] * sval1, wut, wvt);
        }
        halo[wave][side][r] = xt;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    const bool src_cols = (si0 < x0 + 128) && (si0 + kSrcW > x0);
    const int dA = i0 - si0, dB = dA + 1;
    const bool sA = src_cols && dA >= 0 && dA < kSrcW;
    const bool sB = src_cols && dB >= 0 && dB < kSrcW;
    int recA = -1, recB = -1;
    if (kb == 0) {
        recA = ldi(d->recmap, i0);
        recB = ldi(d->recmap, i0 + 1);
    }
    const int side_me = lane == 63 ? 1 : 0;

    NodeRow am, bm, ac, bc, an, bn;
    if (j0 >= 1) {
        make_rows2(load_raw2(cur, (size_t)(j0 - 1) * pitch, i0, hc, hl, live), am, bm);
    } else {
        am = bm = z;
    }
    make_rows2(load_raw2(cur, (size_t)j0 * pitch, i0, hc, hl, live), ac, bc);
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    // prefetch ring: raw u^m rows j+1..j+D, u^{m-1} rows j..j+D-1
    Raw2 rq[D];
    float4 pq[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
        rq[q].c = z4;
        rq[q].h = z2;
        pq[q] = z4;
        if (j0 + 1 + q <= nz - 1) rq[q] = load_raw2(cur, (size_t)(j0 + 1 + q) * pitch, i0, hc, hl, live);
        if (live && j0 + q <= j1) pq[q] = ld4(prev, (size_t)(j0 + q) * pitch + i0);
    }
    // u^{m+1} rows k-1 and k for the second step
    NodeRow a2m = z, b2m = z, a2c = z, b2c = z;
    for (int j = j0; j <= j1; ++j) {
        Raw2 qn;
        qn.c = z4;
        qn.h = z2;
        float4 pn = z4;
        if (j + 1 + D <= nz - 1) qn = load_raw2(cur, (size_t)(j + 1 + D) * pitch, i0, hc, hl, live);
        if (live && j + D <= j1) pn = ld4(prev, (size_t)(j + D) * pitch + i0);
        const Raw2 q1 = rq[0];
        const float4 p0 = pq[0];
#pragma unroll
        for (int q = 0; q + 1 < D; ++q) {
            rq[q] = rq[q + 1];
            pq[q] = pq[q + 1];
        }
        rq[D - 1] = qn;
        pq[D - 1] = pn;
        make_rows2(q1, an, bn);
        // first step at row j
        const LayerCoef cj = load_coef(coef, j);
        const float f1 = cj.c[kFco] * sval1;
        const int dk1 = j - sk0;
        const bool row1 = dk1 >= 0 && dk1 < kSrcW;
        float wua = 0.f, wva = 0.f, wub = 0.f, wvb = 0.f;
        if (sA && row1) {
            wua = ld1(srcw, (0 * kSrcW + dk1) * kSrcW + dA);
            wva = ld1(srcw, (1 * kSrcW + dk1) * kSrcW + dA);
        }
        if (sB && row1) {
            wub = ld1(srcw, (0 * kSrcW + dk1) * kSrcW + dB);
            wvb = ld1(srcw, (1 * kSrcW + dk1) * kSrcW + dB);
        }
        float2 xa = layered_update(cj, am, ac, an, p0.x, p0.y, sA && row1, f1, wua, wva);
        float2 xb = layered_update(cj, bm, bc, bn, p0.z, p0.w, sB && row1, f1, wub, wvb);
        if (!updA) xa = z2;
        if (!updB) xb = z2;
        if (j >= kb && j < ke) {
            if (live) st4(out1, (size_t)j * pitch + i0, make_float4(xa.x, xa.y, xb.x, xb.y));
            if (j == 0) {
                if (recA >= 0) st2(traces, (size_t)(m + 1) * nrec + recA, xa);
                if (recB >= 0) st2(traces, (size_t)(m + 1) * nrec + recB, xb);
            }
        }
        const float2 xt = halo[wave][side_me][j - j0];
        NodeRow a2n, b2n;
        make_rows_x(xa, xb, xt, a2n, b2n);
        // second step at row k = j - 1
        const int k = j - 1;
        if (two && k >= kb) {
            const LayerCoef ck = load_coef(coef, k);
            const float f2 = ck.c[kFco] * sval2;
            const int dk2 = k - sk0;
            const bool row2 = dk2 >= 0 && dk2 < kSrcW;
            float qua = 0.f, qva = 0.f, qub = 0.f, qvb = 0.f;
            if (sA && row2) {
                qua = ld1(srcw, (0 * kSrcW + dk2) * kSrcW + dA);
                qva = ld1(srcw, (1 * kSrcW + dk2) * kSrcW + dA);
            }
            if (sB && row2) {
                qub = ld1(srcw, (0 * kSrcW + dk2) * kSrcW + dB);
                qvb = ld1(srcw, (1 * kSrcW + dk2) * kSrcW + dB);
            }
            float2 ya = layered_update(ck, a2m, a2c, a2n, am.u, am.v, sA && row2, f2, qua, qva);
            float2 yb = layered_update(ck, b2m, b2c, b2n, bm.u, bm.v, sB && row2, f2, qub, qvb);
            if (!updA) ya = z2;
            if (!updB) yb = z2;
            if (live) st4(out2, (size_t)k * pitch + i0, make_float4(ya.x, ya.y, yb.x, yb.y));
            if (k == 0) {
                if (recA >= 0) st2(traces, (size_t)(m + 2) * nrec + recA, ya);
                if (recB >= 0) st2(traces, (size_t)(m + 2) * nrec + recB, yb);
            }
        }
        am = ac;
        bm = bc;
        ac = an;
        bc = bn;
        a2m = a2c;
        b2m = b2c;
        a2c = a2n;
        b2c = b2n;
    }
    // bottom tile: the last free row's second step sees the rigid row (zeros)
    if (two && ke == nz - 1 && ke - 1 >= kb) {
        const int k = ke - 1;
        const LayerCoef ck = load_coef(coef, k);
        const float f2 = ck.c[kFco] * sval2;
        const int dk2 = k - sk0;
        const bool row2 = dk2 >= 0 && dk2 < kSrcW;
        float qua = 0.f, qva = 0.f, qub = 0.f, qvb = 0.f;
        if (sA && row2) {
            qua = ld1(srcw, (0 * kSrcW + dk2) * kSrcW + dA);
            qva = ld1(srcw, (1 * kSrcW + dk2) * kSrcW + dA);
        }
        if (sB && row2) {
            qub = ld1(srcw, (0 * kSrcW + dk2) * kSrcW + dB);
            qvb = ld1(srcw, (1 * kSrcW + dk2) * kSrcW + dB);
        }
        float2 ya = layered_update(ck, a2m, a2c, z, am.u, am.v, sA && row2, f2, qua, qva);
        float2 yb = layered_update(ck, b2m, b2c, z, bm.u, bm.v, sB && row2, f2, qub, qvb);
        if (!updA) ya = z2;
        if (!updB) yb = z2;
        if (live) st4(out2, (size_t)k * pitch + i0, make_float4(ya.x, ya.y, yb.x, yb.y));
        if (k == 0) {
            if (recA >= 0) st2(traces, (size_t)(m + 2) * nrec + recA, ya);
            if (recB >= 0) st2(traces, (size_t)(m + 2) * nrec + recB, yb);
        }
    }
}

// Three leapfrog steps per launch (temporal blocking), depth-only media.
// Levels alternate between two buffer pairs: a launch reads u^{m-1}, u^m
// from one pair and writes u^{m+2}, u^{m+3} to the other (u^{m+1} only
// reaches the receivers), so field traffic is 32 bytes per node per three
// updates.  A wave streams down its 128 x R tile doing step 1 at row j,
// step 2 at row j-1 and step 3 at row j-2; the values its edge nodes need
// from the neighbouring strips (u^{m+1} and u^{m+2} one column beyond the
// tile) come from a side buffer that stencil_tb3_halo fills first, one lane
// per (strip boundary, row).  Every node goes through the same per-node
// update as all other variants: the fields are bitwise identical.
// Measured at 3840 x 512^2: 12.64 ms per launch (4.21 ms per step) against
// 3.48 ms per step for stencil_layered_tb2 -- with a third of the field
// traffic per step it is bound by vector issue (396 instructions per row
// pass, 144 of them register moves; unrolling the row rotation needed 206
// VGPRs), so it is offered ("temporal_blocking" 3) but not the default.

// side[b][k][4]: u^{m+1} at columns b-1 and b, then u^{m+2} at b-1 and b,
// for the strip boundary b = 128 (bi + 1) and free row k.
__global__ void __launch_bounds__(256)
stencil_tb3_halo(const SolveDesc* __restrict__ descs, const int2* __restrict__ htiles,
                 int nhtiles, int pass) {
    const int tile = __builtin_amdgcn_readfirstlane(
        xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    if (tile >= nhtiles) return;
    const int2 te = htiles[tile];
    const SolveDesc* d = descs + __builtin_amdgcn_readfirstlane(te.x);
    const int hc = __builtin_amdgcn_readfirstlane(te.y);
    const int m = 3 * (pass - d->start);
    if (m < 0 || m >= d->nsteps) return;
    const int nx = d->nx, nz = d->nz, pitch = d->pitch;
    const int bi = hc >> 16;
    const int b = 128 * (bi + 1);
    const int k = (hc & 0xffff) * 64 + (threadIdx.x & 63);
    if (k > nz - 2) return;
    const float2* prev = ((pass - d->start) & 1) ? d->buf2 : d->buf0;
    const float2* cur = ((pass - d->start) & 1) ? d->buf3 : d->buf1;
    const float* coef = d->coef;
    const int si0 = d->src_i0, sk0 = d->src_k0;
    const float sval1 = ld1(d->srcs, m);
    const float sval2 = m + 1 < d->nsteps ? ld1(d->srcs, m + 1) : 0.f;
    const float* srcw = d->srcw;
    const NodeRow z = NodeRow{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const float2 z2 = make_float2(0.f, 0.f);
    // u^m on rows k-2..k+2, columns b-3..b+2 (zero outside the grid)
    float2 U[5][6];
#pragma unroll
    for (int r = 0; r < 5; ++r)
#pragma unroll
        for (int c = 0; c < 6; ++c) {
            const int rr = k - 2 + r, cc = b - 3 + c;
            U[r][c] = (rr >= 0 && rr <= nz - 1 && cc >= 0 && cc <= nx - 1)
                          ? ld2(cur, (size_t)rr * pitch + cc) : z2;
        }
    // step 1 on rows k-1..k+1, columns b-2..b+1
    float2 X1[3][4];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int rr = k - 1 + r, cc = b - 2 + c;
            float2 x = z2;
            if (rr >= 0 && rr <= nz - 2 && cc >= 1 && cc <= nx - 2) {
                const NodeRow rm = rr >= 1 ? node_row(U[r][c + 1].x, U[r][c + 1].y, U[r][c].x,
                                                      U[r][c].y, U[r][c + 2].x, U[r][c + 2].y)
                                           : z;
                const NodeRow rc = node_row(U[r + 1][c + 1].x, U[r + 1][c + 1].y, U[r + 1][c].x,
                                            U[r + 1][c].y, U[r + 1][c + 2].x, U[r + 1][c + 2].y);
                const NodeRow rn = node_row(U[r + 2][c + 1].x, U[r + 2][c + 1].y, U[r + 2][c].x,
                                            U[r + 2][c].y, U[r + 2][c + 2].x, U[r + 2][c + 2].y);
                const float2 p = ld2(prev, (size_t)rr * pitch + cc);
                const LayerCoef cf = load_coef(coef, rr);
                const int di = cc - si0, dk = rr - sk0;
                const bool src = di >= 0 && di < kSrcW && dk >= 0 && dk < kSrcW;
                float wu = 0.f, wv = 0.f;
                if (src) {
                    wu = ld1(srcw, (0 * kSrcW + dk) * kSrcW + di);
                    wv = ld1(srcw, (1 * kSrcW + dk) * kSrcW + di);
                }
                x = layered_update(cf, rm, rc, rn, p.x, p.y, src, cf.c[kFco] * sval1, wu, wv);
            }
            X1[r][c] = x;
        }
    // step 2 at row k, columns b-1 and b
    float2 X2[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int cc = b - 1 + c;
        float2 x = z2;
        if (cc >= 1 && cc <= nx - 2 && m + 1 < d->nsteps) {
            const NodeRow rm = k >= 1 ? node_row(X1[0][c + 1].x, X1[0][c + 1].y, X1[0][c].x,
                                                 X1[0][c].y, X1[0][c + 2].x, X1[0][c + 2].y)
                                      : z;
            const NodeRow rc = node_row(X1[1][c + 1].x, X1[1][c + 1].y, X1[1][c].x, X1[1][c].y,
                                        X1[1][c + 2].x, X1[1][c + 2].y);
            const NodeRow rn = node_row(X1[2][c + 1].x, X1[2][c + 1].y, X1[2][c].x, X1[2][c].y,
                                        X1[2][c + 2].x, X1[2][c + 2].y);
            const float2 p = U[2][c + 2];   // u^m at (k, cc)
            const LayerCoef cf = load_coef(coef, k);
            const int di = cc - si0, dk = k - sk0;
            const bool src = di >= 0 && di < kSrcW && dk >= 0 && dk < kSrcW;
            float wu = 0.f, wv = 0.f;
            if (src) {
                wu = ld1(srcw, (0 * kSrcW + dk) * kSrcW + di);
                wv = ld1(srcw, (1 * kSrcW + dk) * kSrcW + di);
            }
            x = layered_update(cf, rm, rc, rn, p.x, p.y, src, cf.c[kFco] * sval2, wu, wv);
        }
        X2[c] = x;
    }
    float2* out = d->side + ((size_t)bi * nz + k) * 4;
    st4(out, 0, make_float4(X1[1][1].x, X1[1][1].y, X1[1][2].x, X1[1][2].y));
    st4(out, 2, make_float4(X2[0].x, X2[0].y, X2[1].x, X2[1].y));
}

template <int R>
__global__ void __launch_bounds__(256)
stencil_layered_tb3(const SolveDesc* __restrict__ descs, const int2* __restrict__ tiles,
                    int ntiles, int pass) {
    const int tile = __builtin_amdgcn_readfirstlane(
        xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    if (tile >= ntiles) return;
    const int2 te = tiles[tile];
    const SolveDesc* d = descs + __builtin_amdgcn_readfirstlane(te.x);
    const int sc = __builtin_amdgcn_readfirstlane(te.y);
    const int lp = pass - d->start;
    const int m = 3 * lp;
    if (m < 0 || m >= d->nsteps) return;
    const int nsub = min(3, d->nsteps - m);
    const int lane = threadIdx.x & 63;
    const int nx = d->nx, nz = d->nz, pitch = d->pitch;
    const int x0 = (sc >> 16) * 128;
    const int kb = (sc & 0xffff) * R;
    const int ke = min(kb + R, nz - 1);
    const int i0 = x0 + 2 * lane;
    const bool odd = lp & 1;
    const float2* prev = odd ? d->buf2 : d->buf0;
    const float2* cur = odd ? d->buf3 : d->buf1;
    float2* outA = odd ? d->buf0 : d->buf2;   // u^{m+2}
    float2* outB = odd ? d->buf1 : d->buf3;   // u^{m+3}
    const float* coef = d->coef;
    const bool updA = (i0 >= 1) && (i0 <= nx - 2);
    const bool updB = (i0 + 1 <= nx - 2);
    const bool hl = (lane == 0 && x0 > 0) || (lane == 63 && x0 + 128 < nx);
    const int hc = (lane == 0) ? x0 - 1 : x0 + 128;
    // side-buffer column of this lane's halo node (lanes 0 and 63 only)
    const float2* side = nullptr;
    int sofs = 0;
    if (lane == 0 && x0 > 0) {
        side = d->side + (size_t)(x0 / 128 - 1) * nz * 4;
        sofs = 0;   // column b - 1 with b = x0
    } else if (lane == 63 && x0 + 128 < nx) {
        side = d->side + (size_t)(x0 / 128) * nz * 4;
        sofs = 1;   // column b with b = x0 + 128
    }
    const int si0 = d->src_i0, sk0 = d->src_k0;
    const bool src_cols = (si0 < x0 + 128) && (si0 + kSrcW > x0);
    const int dA = i0 - si0, dB = dA + 1;
    const bool sA = src_cols && dA >= 0 && dA < kSrcW;
    const bool sB = src_cols && dB >= 0 && dB < kSrcW;
    const float sv1 = ld1(d->srcs, m);
    const float sv2 = nsub > 1 ? ld1(d->srcs, m + 1) : 0.f;
    const float sv3 = nsub > 2 ? ld1(d->srcs, m + 2) : 0.f;
    const float* srcw = d->srcw;
    float2* traces = d->traces;
    const int nrec = d->nrec;
    int recA = -1, recB = -1;
    if (kb == 0) {
        recA = ldi(d->recmap, i0);
        recB = ldi(d->recmap, i0 + 1);
    }
    const NodeRow z = NodeRow{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const float2 z2 = make_float2(0.f, 0.f);
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const int j0 = kb >= 2 ? kb - 2 : 0;
    const int j1 = min(ke + 1, nz - 2);                 // last step-1 row
    const int s2lo = kb >= 1 ? kb - 1 : 0, s2hi = min(ke, nz - 2);

    auto wts = [&](bool s, int dk, int di, float& wu, float& wv) {
        wu = 0.f;
        wv = 0.f;
        if (s && dk >= 0 && dk < kSrcW) {
            wu = ld1(srcw, (0 * kSrcW + dk) * kSrcW + di);
            wv = ld1(srcw, (1 * kSrcW + dk) * kSrcW + di);
        }
    };

    NodeRow am, bm, ac, bc, an, bn;
    if (j0 >= 1) {
        make_rows2(load_raw2(cur, (size_t)(j0 - 1) * pitch, i0, hc, hl), am, bm);
    } else {
        am = bm = z;
    }
    make_rows2(load_raw2(cur, (size_t)j0 * pitch, i0, hc, hl), ac, bc);
    Raw2 q1;
    q1.c = z4;
    q1.h = z2;
    if (j0 + 1 <= nz - 1) q1 = load_raw2(cur, (size_t)(j0 + 1) * pitch, i0, hc, hl);
    float4 p0 = ld4(prev, (size_t)j0 * pitch + i0);
    NodeRow a1m = z, b1m = z, a1c = z, b1c = z;   // u^{m+1} rows j-2, j-1
    NodeRow a2m = z, b2m = z, a2c = z, b2c = z;   // u^{m+2} rows j-3, j-2
    for (int j = j0; j <= ke + 1; ++j) {
        Raw2 qn;
        qn.c = z4;
        qn.h = z2;
        float4 pn = z4;
        if (j + 2 <= nz - 1 && j + 1 <= j1) qn = load_raw2(cur, (size_t)(j + 2) * pitch, i0, hc, hl);
        if (j + 1 <= j1) pn = ld4(prev, (size_t)(j + 1) * pitch + i0);
        // step 1 at row j
        NodeRow a1n = z, b1n = z;
        if (j <= j1) {
            make_rows2(q1, an, bn);
            const LayerCoef cj = load_coef(coef, j);
            float wua, wva, wub, wvb;
            wts(sA, j - sk0, dA, wua, wva);
            wts(sB, j - sk0, dB, wub, wvb);
            const bool r1 = j - sk0 >= 0 && j - sk0 < kSrcW;
            float2 xa = layered_update(cj, am, ac, an, p0.x, p0.y, sA && r1, cj.c[kFco] * sv1,
                                       wua, wva);
            float2 xb = layered_update(cj, bm, bc, bn, p0.z, p0.w, sB && r1, cj.c[kFco] * sv1,
                                       wub, wvb);
            if (!updA) xa = z2;
            if (!updB) xb = z2;
            if (j == 0) {
                if (recA >= 0) st2(traces, (size_t)(m + 1) * nrec + recA, xa);
                if (recB >= 0) st2(traces, (size_t)(m + 1) * nrec + recB, xb);
            }
            const float2 xt = side ? ld2(side, (size_t)j * 4 + sofs) : z2;
            make_rows_x(xa, xb, xt, a1n, b1n);
        } else {
            an = bn = z;
        }
        // step 2 at row j - 1
        NodeRow a2n = z, b2n = z;
        const int k2 = j - 1;
        if (nsub > 1 && k2 >= s2lo && k2 <= s2hi) {
            const LayerCoef ck = load_coef(coef, k2);
            float wua, wva, wub, wvb;
            wts(sA, k2 - sk0, dA, wua, wva);
            wts(sB, k2 - sk0, dB, wub, wvb);
            const bool r2 = k2 - sk0 >= 0 && k2 - sk0 < kSrcW;
            float2 ya = layered_update(ck, a1m, a1c, a1n, am.u, am.v, sA && r2,
                                       ck.c[kFco] * sv2, wua, wva);
            float2 yb = layered_update(ck, b1m, b1c, b1n, bm.u, bm.v, sB && r2,
                                       ck.c[kFco] * sv2, wub, wvb);
            if (!updA) ya = z2;
            if (!updB) yb = z2;
            if (k2 >= kb && k2 < ke)
                st4(outA, (size_t)k2 * pitch + i0, make_float4(ya.x, ya.y, yb.x, yb.y));
            if (k2 == 0) {
                if (recA >= 0) st2(traces, (size_t)(m + 2) * nrec + recA, ya);
                if (recB >= 0) st2(traces, (size_t)(m + 2) * nrec + recB, yb);
            }
            const float2 xt = side ? ld2(side, (size_t)k2 * 4 + 2 + sofs) : z2;
            make_rows_x(ya, yb, xt, a2n, b2n);
        }
        // step 3 at row j - 2
        const int k3 = j - 2;
        if (nsub > 2 && k3 >= kb && k3 < ke) {
            const LayerCoef ck = load_coef(coef, k3);
            float wua, wva, wub, wvb;
            wts(sA, k3 - sk0, dA, wua, wva);
            wts(sB, k3 - sk0, dB, wub, wvb);
            const bool r3 = k3 - sk0 >= 0 && k3 - sk0 < kSrcW;
            float2 za = layered_update(ck, a2m, a2c, a2n, a1m.u, a1m.v, sA && r3,
                                       ck.c[kFco] * sv3, wua, wva);
            float2 zb = layered_update(ck, b2m, b2c, b2n, b1m.u, b1m.v, sB && r3,
                                       ck.c[kFco] * sv3, wub, wvb);
            if (!updA) za = z2;
            if (!updB) zb = z2;
            st4(outB, (size_t)k3 * pitch + i0, make_float4(za.x, za.y, zb.x, zb.y));
            if (k3 == 0) {
                if (recA >= 0) st2(traces, (size_t)(m + 3) * nrec + recA, za);
                if (recB >= 0) st2(traces, (size_t)(m + 3) * nrec + recB, zb);
            }
        }
        am = ac;
        bm = bc;
        ac = an;
        bc = bn;
        a1m = a1c;
        b1m = b1c;
        a1c = a1n;
        b1c = b1n;
        a2m = a2c;
        b2m = b2c;
        a2c = a2n;
        b2c = b2n;
        q1 = qn;
        p0 = pn;
    }
}

__global__ void fill_zero_kernel(uint4* p, size_t n16, uint8_t* tail, size_t ntail) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x; j < n16; j += stride)
        p[j] = make_uint4(0, 0, 0, 0);
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < ntail) tail[t] = 0;
}

__global__ void zero_level0_kernel(const SolveDesc* __restrict__ descs) {
    const SolveDesc& d = descs[blockIdx.x];
    for (int r = threadIdx.x; r < d.nrec; r += blockDim.x) d.traces[r] = make_float2(0.f, 0.f);
}

}  // namespace

void launch_tb3_halo(const SolveDesc* descs, const int2* htiles, int nhtiles, int pass,
                     hipStream_t s) {
    if (nhtiles <= 0) return;
    const int blocks = (nhtiles + kWavesPerBlock - 1) / kWavesPerBlock;
    stencil_tb3_halo<<<blocks, 64 * kWavesPerBlock, 0, s>>>(descs, htiles, nhtiles, pass);
}

void launch_zero_level0(const SolveDesc* descs, int n, hipStream_t s) {
    if (n > 0) zero_level0_kernel<<<n, 64, 0, s>>>(descs);
}

void launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return;
    // callers pass 16-byte aligned buffers; the remainder is cleared bytewise
    const size_t n16 = bytes / 16;
    const size_t ntail = bytes - n16 * 16;
    size_t blocks = (n16 + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 8192) blocks = 8192;
    fill_zero_kernel<<<(unsigned)blocks, 256, 0, s>>>(
        (uint4*)p, n16, (uint8_t*)p + n16 * 16, ntail);
}

void launch_layered_stencil(const SolveDesc* descs, const int2* tiles, int ntiles, int step,
                            int variant, hipStream_t s) {
    const int blocks = (ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int threads = 64 * kWavesPerBlock;
    switch (variant) {
        case 0: stencil_layered_w1<<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 1: stencil_layered_w2<32, 1><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 2: stencil_layered_w2<32, 2><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 3: stencil_layered_w2<64, 2><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 4: stencil_layered_w2<16, 2><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 5: stencil_layered_w2<64, 1><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 7: stencil_layered_w2<8, 2><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 8: stencil_layered_w2<16, 1><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 9: stencil_layered_tb2<16, 1><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 10: stencil_layered_tb2<32, 1><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 11: stencil_layered_tb2<64, 1><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 12: stencil_layered_tb2<128, 1><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 13: stencil_layered_tb2h<64, 1><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 14: stencil_layered_tb2h<32, 1><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 15: stencil_layered_tb3<64><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 16: stencil_layered_tb3<32><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        default: break;
    }
}

}  // namespace eig
