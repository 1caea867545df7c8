// Leapfrog step for nodal media (every coefficient per node): the one-node
// kernel (variant 6), two nodes per lane (17, 18) and two steps per launch
// (19, 20).  The per-node arithmetic is shared with every other kernel
// (node_update.h), so all of them produce bitwise-identical fields.
#include "ce.h"
#include "internal.h"
#include "node_update.h"
#include "tile.h"

namespace eig {

namespace {

struct RowN {
    float u, v, hu, hv;   // centre and halo-column values of u^m
    float lam, mu;        // centre nodal coefficients
    float hlam, hmu;      // halo-column coefficients
};

// Variant 6: one node per lane (64 columns per wave), 32 rows per wave.
__global__ void __launch_bounds__(256)
stencil_nodal(const SolveDesc* __restrict__ descs, const int2* __restrict__ tiles,
              int ntiles, int step) {
    TileInfo t;
    if (!decode_tile(descs, tiles, ntiles, step, 64, 32, t)) return;
    const SolveDesc* d = t.d;
    const int lane = threadIdx.x & 63;
    const int m = t.m, x0 = t.x0, kb = t.kb, ke = t.ke;
    const int nx = d->nx, nz = d->nz, pitch = d->pitch;
    const int i = x0 + lane;
    const float2* Q = (m & 1) ? d->buf1 : d->buf0;
    float2* P = (m & 1) ? d->buf0 : d->buf1;
    const size_t plane = (size_t)nz * pitch;
    const float* LAM = d->coef;
    const float* MU = LAM + plane;
    const float* SC = LAM + 2 * plane;

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
    const float h2 = d->h2;
    int rec = -1;
    if (kb == 0) rec = ldi(d->recmap, i);
    const float2* rfz = d->rforce;
    float2* wrec = d->wrec;

    auto load = [=](int k) {
        RowN r;
        const size_t o = (size_t)k * pitch;
        const int j = hl ? hc : i;
        const float2 c = ld2(Q, o + i);
        const float2 h = ld2(Q, o + j);
        r.u = c.x; r.v = c.y;
        r.lam = ld1(LAM, o + i);
        r.mu = ld1(MU, o + i);
        const float hlam = ld1(LAM, o + j), hmu = ld1(MU, o + j);
        r.hu = hl ? h.x : 0.f;
        r.hv = hl ? h.y : 0.f;
        r.hlam = hl ? hlam : 0.f;
        r.hmu = hl ? hmu : 0.f;
        return r;
    };

    RowN rm, rc, rn;
    if (kb == 0) {
        rm = RowN{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    } else {
        rm = load(kb - 1);
    }
    rc = load(kb);
    rn = load(kb + 1);
    float2 up = ld2(P, (size_t)kb * pitch + i);
    float sc = ld1(SC, (size_t)kb * pitch + i);

    for (int k = kb; k < ke; ++k) {
        RowN rnn = RowN{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float2 upn = make_float2(0.f, 0.f);
        float scn = 0.f;
        if (k + 2 <= nz - 1) rnn = load(k + 2);
        if (k + 1 < ke) {
            upn = ld2(P, (size_t)(k + 1) * pitch + i);
            scn = ld1(SC, (size_t)(k + 1) * pitch + i);
        }
        NodalView n;
        n.u = rc.u;
        n.v = rc.v;
        n.lam = rc.lam;
        n.mu = rc.mu;
        n.uL = from_left(rc.u, rc.hu);
        n.uR = from_right(rc.u, rc.hu);
        n.vL = from_left(rc.v, rc.hv);
        n.vR = from_right(rc.v, rc.hv);
        const float ac = rc.lam + 2.f * rc.mu;
        const float ah = rc.hlam + 2.f * rc.hmu;
        n.aL = from_left(ac, ah);
        n.aR = from_right(ac, ah);
        n.mL = from_left(rc.mu, rc.hmu);
        n.mR = from_right(rc.mu, rc.hmu);
        n.un = rn.u;
        n.vn = rn.v;
        n.lamn = rn.lam;
        n.mun = rn.mu;
        n.dxun = from_right(rn.u, rn.hu) - from_left(rn.u, rn.hu);
        n.dxvn = from_right(rn.v, rn.hv) - from_left(rn.v, rn.hv);
        const bool top = k == 0;
        float p, ph, q, qh;
        if (top) {
            n.um = n.vm = n.lamm = n.mum = n.dxum = n.dxvm = 0.f;
            p = rc.lam * (rn.v - rc.v);
            ph = rc.hlam * (rn.hv - rc.hv);
            q = rc.mu * (rn.u - rc.u);
            qh = rc.hmu * (rn.hu - rc.hu);
        } else {
            n.um = rm.u;
            n.vm = rm.v;
            n.lamm = rm.lam;
            n.mum = rm.mu;
            n.dxum = from_right(rm.u, rm.hu) - from_left(rm.u, rm.hu);
            n.dxvm = from_right(rm.v, rm.hv) - from_left(rm.v, rm.hv);
            p = rc.lam * (rn.v - rm.v);
            ph = rc.hlam * (rn.hv - rm.hv);
            q = rc.mu * (rn.u - rm.u);
            qh = rc.hmu * (rn.hu - rm.hu);
        }
        n.pR = from_right(p, ph);
        n.pL = from_left(p, ph);
        n.qR = from_right(q, qh);
        n.qL = from_left(q, qh);
        const float2 acc = nodal_accel(n, top);
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
            w0 = ld1(srcw, (0 * kSrcW + dk) * kSrcW + di);
            w1 = ld1(srcw, (1 * kSrcW + dk) * kSrcW + di);
        }
        const float2 nw = nodal_new(acc, sc, rc.u, rc.v, up.x, up.y, inj, h2, sval, w0, w1);
        if (upd) {
            st2(P, (size_t)k * pitch + i, nw);
            if (k == 0 && rec >= 0) st2(traces, (size_t)(m + 1) * nrec + rec, nw);
            if (wrec && in_win) st2(wrec, (size_t)m * (kSrcW * kSrcW) + dk * kSrcW + di, nw);
        }
        rm = rc;
        rc = rn;
        rn = rnn;
        up = upn;
        sc = scn;
    }
}

// Nodal media, two nodes per lane (128 columns per wave) with 16- and 8-byte
// loads, R rows per wave.  Lane l owns columns x0+2l (A) and x0+2l+1 (B);
// each x-neighbour quantity needs one cross-lane move per node pair instead
// of one per node, and lanes 0 / 63 load the halo column.
struct RawN2 {
    float4 c;                     // (u, v) of A and B
    float lamA, lamB, muA, muB;   // their coefficients
    float hu, hv, hlam, hmu;      // halo column (lanes 0 / 63), else 0
};

__device__ __forceinline__ float2 ld2f(const float* p, size_t i) {  // i even
    const fv2 v = *(const GAS fv2*)((const GAS float*)p + i);
    return make_float2(v.x, v.y);
}

__device__ __forceinline__ RawN2 load_rawn2(const float2* Q, const float* LAM,
                                            const float* MU, size_t o, int i0, int hc,
                                            bool hl) {
    RawN2 r;
    r.c = ld4(Q, o + i0);
    const float2 l = ld2f(LAM, o + i0), mu = ld2f(MU, o + i0);
    r.lamA = l.x;
    r.lamB = l.y;
    r.muA = mu.x;
    r.muB = mu.y;
    r.hu = r.hv = r.hlam = r.hmu = 0.f;
    if (hl) {
        const float2 h = ld2(Q, o + hc);
        r.hu = h.x;
        r.hv = h.y;
        r.hlam = ld1(LAM, o + hc);
        r.hmu = ld1(MU, o + hc);
    }
    return r;
}

// u at the next level on the lane's two nodes A = x0+2l and B = x0+2l+1 of
// row k, from rows k-1 (rm), k (rc) and k+1 (rn) of the current level (with
// the halo-column values held by lanes 0 / 63, zeros elsewhere), the scaled
// mass s of A and B (sc), the previous level at row k (up) and the forcing
// (injA/B, weights, series value).  The two-node one-step kernel and both
// steps of the two-step kernel call it, so they produce the same bits.
struct PairInj {
    int injA, injB;
    float wa0, wa1, wb0, wb1;
};

__device__ __forceinline__ void nodal_pair(const RawN2& rm, const RawN2& rc, const RawN2& rn,
                                           bool top, float2 sc, float4 up, const PairInj& in,
                                           float h2, float sval, float2& na, float2& nb) {
    NodalView A, B;
    A.u = rc.c.x;
    A.v = rc.c.y;
    A.lam = rc.lamA;
    A.mu = rc.muA;
    B.u = rc.c.z;
    B.v = rc.c.w;
    B.lam = rc.lamB;
    B.mu = rc.muB;
    // the in-lane neighbour values are pinned: A's right flux and B's left
    // flux are then separate products with one use each, as in the
    // one-node kernel, so the compiler fuses them into the same FMAs
    A.uL = from_left(rc.c.z, rc.hu);
    A.uR = pinned(rc.c.z);
    A.vL = from_left(rc.c.w, rc.hv);
    A.vR = pinned(rc.c.w);
    B.uL = pinned(rc.c.x);
    B.uR = from_right(rc.c.x, rc.hu);
    B.vL = pinned(rc.c.y);
    B.vR = from_right(rc.c.y, rc.hv);
    const float aA = pinned(rc.lamA + 2.f * rc.muA);
    const float aB = pinned(rc.lamB + 2.f * rc.muB);
    const float ah = rc.hlam + 2.f * rc.hmu;
    A.aL = from_left(aB, ah);
    A.aR = aB;
    B.aL = aA;
    B.aR = from_right(aA, ah);
    A.mL = from_left(rc.muB, rc.hmu);
    A.mR = pinned(rc.muB);
    B.mL = pinned(rc.muA);
    B.mR = from_right(rc.muA, rc.hmu);
    A.un = rn.c.x;
    A.vn = rn.c.y;
    A.lamn = rn.lamA;
    A.mun = rn.muA;
    B.un = rn.c.z;
    B.vn = rn.c.w;
    B.lamn = rn.lamB;
    B.mun = rn.muB;
    A.dxun = rn.c.z - from_left(rn.c.z, rn.hu);
    A.dxvn = rn.c.w - from_left(rn.c.w, rn.hv);
    B.dxun = from_right(rn.c.x, rn.hu) - rn.c.x;
    B.dxvn = from_right(rn.c.y, rn.hv) - rn.c.y;
    float pA, pB, ph, qA, qB, qh;
    if (top) {
        A.um = A.vm = A.lamm = A.mum = A.dxum = A.dxvm = 0.f;
        B.um = B.vm = B.lamm = B.mum = B.dxum = B.dxvm = 0.f;
        pA = rc.lamA * (rn.c.y - rc.c.y);
        pB = rc.lamB * (rn.c.w - rc.c.w);
        ph = rc.hlam * (rn.hv - rc.hv);
        qA = rc.muA * (rn.c.x - rc.c.x);
        qB = rc.muB * (rn.c.z - rc.c.z);
        qh = rc.hmu * (rn.hu - rc.hu);
    } else {
        A.um = rm.c.x;
        A.vm = rm.c.y;
        A.lamm = rm.lamA;
        A.mum = rm.muA;
        B.um = rm.c.z;
        B.vm = rm.c.w;
        B.lamm = rm.lamB;
        B.mum = rm.muB;
        A.dxum = rm.c.z - from_left(rm.c.z, rm.hu);
        A.dxvm = rm.c.w - from_left(rm.c.w, rm.hv);
        B.dxum = from_right(rm.c.x, rm.hu) - rm.c.x;
        B.dxvm = from_right(rm.c.y, rm.hv) - rm.c.y;
        pA = rc.lamA * (rn.c.y - rm.c.y);
        pB = rc.lamB * (rn.c.w - rm.c.w);
        ph = rc.hlam * (rn.hv - rm.hv);
        qA = rc.muA * (rn.c.x - rm.c.x);
        qB = rc.muB * (rn.c.z - rm.c.z);
        qh = rc.hmu * (rn.hu - rm.hu);
    }
    pA = pinned(pA);
    pB = pinned(pB);
    qA = pinned(qA);
    qB = pinned(qB);
    A.pR = pB;
    A.pL = from_left(pB, ph);
    B.pL = pA;
    B.pR = from_right(pA, ph);
    A.qR = qB;
    A.qL = from_left(qB, qh);
    B.qL = qA;
    B.qR = from_right(qA, qh);
    const float2 accA = nodal_accel(A, top), accB = nodal_accel(B, top);
    na = nodal_new(accA, sc.x, A.u, A.v, up.x, up.y, in.injA, h2, sval, in.wa0, in.wa1);
    nb = nodal_new(accB, sc.y, B.u, B.v, up.z, up.w, in.injB, h2, sval, in.wb0, in.wb1);
}

template <int R>
__global__ void __launch_bounds__(256)
stencil_nodal_w2(const SolveDesc* __restrict__ descs, const int2* __restrict__ tiles,
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
    const size_t plane = (size_t)nz * pitch;
    const float* LAM = d->coef;
    const float* MU = LAM + plane;
    const float* SC = LAM + 2 * plane;
    const bool upd0 = (i0 >= 1) && (i0 <= nx - 2);
    const bool upd1 = (i0 + 1 <= nx - 2);
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
    const float h2 = d->h2;
    int rec0 = -1, rec1 = -1;
    if (kb == 0) {
        rec0 = ldi(d->recmap, i0);
        rec1 = ldi(d->recmap, i0 + 1);
    }
    const float2* rfz = d->rforce;
    float2* wrec = d->wrec;
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const RawN2 zr = RawN2{z4, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    RawN2 rm = zr, rc, rn;
    if (kb > 0) rm = load_rawn2(Q, LAM, MU, (size_t)(kb - 1) * pitch, i0, hc, hl);
    rc = load_rawn2(Q, LAM, MU, (size_t)kb * pitch, i0, hc, hl);
    rn = load_rawn2(Q, LAM, MU, (size_t)(kb + 1) * pitch, i0, hc, hl);
    float4 up = ld4(P, (size_t)kb * pitch + i0);
    float2 sc = ld2f(SC, (size_t)kb * pitch + i0);

    for (int k = kb; k < ke; ++k) {
        RawN2 rnn = zr;
        float4 upn = z4;
        float2 scn = make_float2(0.f, 0.f);
        if (k + 2 <= nz - 1) rnn = load_rawn2(Q, LAM, MU, (size_t)(k + 2) * pitch, i0, hc, hl);
        if (k + 1 < ke) {
            upn = ld4(P, (size_t)(k + 1) * pitch + i0);
            scn = ld2f(SC, (size_t)(k + 1) * pitch + i0);
        }
        const bool top = k == 0;
        const int dk = k - sk0;
        const bool row_src = dk >= 0 && dk < kSrcW;
        const bool wa = s0 && row_src, wb = s1 && row_src;
        int injA = 0, injB = 0;
        float wa0 = 0.f, wa1 = 0.f, wb0 = 0.f, wb1 = 0.f;
        if (rfz && k == 0 && rec0 >= 0) {  // dual solve: receiver injection
            const float2 rf = ld2(rfz, (size_t)m * nrec + rec0);
            injA = 1;
            wa0 = rf.x;
            wa1 = rf.y;
        } else if (wa) {
            injA = 2;
            wa0 = ld1(srcw, (0 * kSrcW + dk) * kSrcW + di0);
            wa1 = ld1(srcw, (1 * kSrcW + dk) * kSrcW + di0);
        }
        if (rfz && k == 0 && rec1 >= 0) {
            const float2 rf = ld2(rfz, (size_t)m * nrec + rec1);
            injB = 1;
            wb0 = rf.x;
            wb1 = rf.y;
        } else if (wb) {
            injB = 2;
            wb0 = ld1(srcw, (0 * kSrcW + dk) * kSrcW + di1);
            wb1 = ld1(srcw, (1 * kSrcW + dk) * kSrcW + di1);
        }
        float2 na, nb;
        nodal_pair(rm, rc, rn, top, sc, up, PairInj{injA, injB, wa0, wa1, wb0, wb1}, h2, sval,
                   na, nb);
        if (wrec) {
            const size_t w0 = (size_t)m * (kSrcW * kSrcW) + dk * kSrcW;
            if (wa && upd0) st2(wrec, w0 + di0, na);
            if (wb && upd1) st2(wrec, w0 + di1, nb);
        }
        // edge and padding columns are never written
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
        rm = rc;
        rc = rn;
        rn = rnn;
        up = upn;
        sc = scn;
    }
}

// u at the next level at one node (i, k) of a nodal medium with every
// operand read from memory (Q: current level, P: previous level): the halo
// columns of the two-step kernel.  The neighbours' quantities are formed as
// the one-node kernel forms them in the neighbouring lanes, and the products
// among them are pinned, as a cross-lane move leaves them rounded, so the
// result is bitwise that of every nodal variant.
__device__ float2 nodal_node(const float2* Q, const float2* P, const float* LAM,
                             const float* MU, const float* SC, int pitch, int i, int k,
                             int inj, float h2, float sval, float w0, float w1) {
    auto U = [&](int ii, int kk) { return ld2(Q, (size_t)kk * pitch + ii); };
    return nodal_node_at(U, ld2(P, (size_t)k * pitch + i), LAM, MU, SC, pitch, i, k, inj, h2,
                         sval, w0, w1);
}

// Two leapfrog steps per launch for nodal media (rigid edges, no receiver
// injection).  Same buffer rotation as the depth-only two-step kernels
// (level l in buffer (l + 1) mod 4): a launch reads u^{m-1} and u^m and
// writes u^{m+1} and u^{m+2}, 16 bytes of fields per update instead of 24.
// A wave owns 128 columns x R rows.  First, u^{m+1} at the two halo columns
// x0-1 and x0+128 is formed for the rows kb-1..ke (one lane per node, into
// LDS).  Then the row loop takes step one at row j for the lane's two nodes
// (rows kb-1..ke, the halo rows included) and step two at row j-1 from the
// three u^{m+1} rows it holds; the lambda and mu rows it needs stay from the
// u^m rows already loaded.  Both steps go through nodal_pair and the halo
// nodes through nodal_node, so the fields are bitwise those of the one-step
// nodal kernels.
// Measured at 2048 x 1024 x 4000 (30 solves per launch): 2.25e11 updates/s
// with 32-row tiles against 1.96e11 for the best one-step kernel.  With a
// third less field traffic (3.6 TB/s here) the kernel is bound by vector
// issue: about 135 vector instructions per update, two fifths of them
// register moves that the edge-lane cross-lane moves (old value = halo) and
// the pinned operands need, at ~84 % of the device's non-packed FP32 issue
// rate.  Unrolling the row loop over fixed register slots (no row copies)
// took 244 VGPRs for no fewer moves; 64- and 30-row tiles, and cache-sized
// chunks of two or three solves, were slower or equal.
template <int R>
__global__ void __launch_bounds__(256)
stencil_nodal_tb2(const SolveDesc* __restrict__ descs, const int2* __restrict__ tiles,
                  int ntiles, int pass) {
    __shared__ float2 halo[kWavesPerBlock][2][R + 2];
    const int tile = __builtin_amdgcn_readfirstlane(
        xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + (threadIdx.x >> 6));
    if (tile >= ntiles) return;
    const int2 te = tiles[tile];
    const SolveDesc* d = descs + __builtin_amdgcn_readfirstlane(te.x);
    const int sc0 = __builtin_amdgcn_readfirstlane(te.y);
    const int m = 2 * (pass - d->start);
    if (m < 0 || m >= d->nsteps) return;
    const bool two = m + 1 < d->nsteps;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nx = d->nx, nz = d->nz, pitch = d->pitch;
    const int x0 = (sc0 >> 16) * 128;
    const int kb = (sc0 & 0xffff) * R;
    const int ke = min(kb + R, nz - 1);
    const int i0 = x0 + 2 * lane;
    float2* const bufs[4] = {d->buf0, d->buf1, d->buf2, d->buf3};
    const float2* prev = bufs[m & 3];        // u^{m-1}
    const float2* cur = bufs[(m + 1) & 3];   // u^m
    float2* out1 = bufs[(m + 2) & 3];        // u^{m+1}
    float2* out2 = bufs[(m + 3) & 3];        // u^{m+2}
    const size_t plane = (size_t)nz * pitch;
    const float* LAM = d->coef;
    const float* MU = LAM + plane;
    const float* SC = LAM + 2 * plane;
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
    const float h2 = d->h2;
    const float2 z2 = make_float2(0.f, 0.f);
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const RawN2 zr = RawN2{z4, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    const int j0 = kb > 0 ? kb - 1 : 0;
    const int j1 = min(ke, nz - 2);
    const int nrow = j1 - j0 + 1;

    // u^{m+1} at the halo columns, rows j0..j1 (zero where not a free node)
    for (int it = lane; it < 2 * nrow; it += 64) {
        const int side = it & 1, r = it >> 1, j = j0 + r;
        const int c = side == 0 ? x0 - 1 : x0 + 128;
        float2 xt = z2;
        if (c >= 1 && c <= nx - 2) {
            const int dT = c - si0, dk1 = j - sk0;
            const bool s1 = dT >= 0 && dT < kSrcW && dk1 >= 0 && dk1 < kSrcW;
            float w0 = 0.f, w1 = 0.f;
            if (s1) {
                w0 = ld1(srcw, (0 * kSrcW + dk1) * kSrcW + dT);
                w1 = ld1(srcw, (1 * kSrcW + dk1) * kSrcW + dT);
            }
            xt = nodal_node(cur, prev, LAM, MU, SC, pitch, c, j, s1 ? 2 : 0, h2, sval1, w0, w1);
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
    auto inj_of = [&](int row, float sv, float& fs) {
        PairInj in{0, 0, 0.f, 0.f, 0.f, 0.f};
        const int dk = row - sk0;
        const bool rs = dk >= 0 && dk < kSrcW;
        if (sA && rs) {
            in.injA = 2;
            in.wa0 = ld1(srcw, (0 * kSrcW + dk) * kSrcW + dA);
            in.wa1 = ld1(srcw, (1 * kSrcW + dk) * kSrcW + dA);
        }
        if (sB && rs) {
            in.injB = 2;
            in.wb0 = ld1(srcw, (0 * kSrcW + dk) * kSrcW + dB);
            in.wb1 = ld1(srcw, (1 * kSrcW + dk) * kSrcW + dB);
        }
        fs = sv;
        return in;
    };
    // u^{m+1} row j as a pair row: the lane's nodes, the halo column from
    // LDS for lanes 0 / 63, and the coefficients of the u^m row j
    auto next_row = [&](float2 na, float2 nb, const RawN2& coefrow, int j) {
        RawN2 x = coefrow;
        x.c = make_float4(na.x, na.y, nb.x, nb.y);
        x.hu = x.hv = 0.f;
        if (hl) {
            const float2 hv = halo[wave][lane == 0 ? 0 : 1][j - j0];
            x.hu = hv.x;
            x.hv = hv.y;
        }
        return x;
    };

    // u^m rows j-1, j, j+1 (and the prefetched j+2), u^{m-1} and s of row j
    RawN2 rm = zr, rc, rn;
    if (j0 > 0) rm = load_rawn2(cur, LAM, MU, (size_t)(j0 - 1) * pitch, i0, hc, hl);
    rc = load_rawn2(cur, LAM, MU, (size_t)j0 * pitch, i0, hc, hl);
    rn = load_rawn2(cur, LAM, MU, (size_t)(j0 + 1) * pitch, i0, hc, hl);
    float4 up = ld4(prev, (size_t)j0 * pitch + i0);
    float2 sc = ld2f(SC, (size_t)j0 * pitch + i0);
    // u^{m+1} rows j-2, j-1 as pair rows; u^m and s of row j-1
    RawN2 xm = zr, xc = zr;
    float4 um_prev = z4;
    float2 sc_prev = make_float2(0.f, 0.f);

    for (int j = j0; j <= j1; ++j) {
        RawN2 rnn = zr;
        float4 upn = z4;
        float2 scn = make_float2(0.f, 0.f);
        if (j + 2 <= nz - 1) rnn = load_rawn2(cur, LAM, MU, (size_t)(j + 2) * pitch, i0, hc, hl);
        if (j + 1 <= j1) {
            upn = ld4(prev, (size_t)(j + 1) * pitch + i0);
            scn = ld2f(SC, (size_t)(j + 1) * pitch + i0);
        }
        // step one at row j
        float fs1;
        const PairInj in1 = inj_of(j, sval1, fs1);
        float2 na, nb;
        nodal_pair(rm, rc, rn, j == 0, sc, up, in1, h2, fs1, na, nb);
        if (!updA) na = z2;
        if (!updB) nb = z2;
        if (j >= kb && j < ke) {
            if (live) st4(out1, (size_t)j * pitch + i0, make_float4(na.x, na.y, nb.x, nb.y));
            if (j == 0) {
                if (recA >= 0) st2(traces, (size_t)(m + 1) * nrec + recA, na);
                if (recB >= 0) st2(traces, (size_t)(m + 1) * nrec + recB, nb);
            }
        }
        const RawN2 xn = next_row(na, nb, rc, j);
        // step two at row k = j - 1 (u^m of row k is the previous level)
        const int k = j - 1;
        if (two && k >= kb) {
            float fs2;
            const PairInj in2 = inj_of(k, sval2, fs2);
            float2 ya, yb;
            nodal_pair(xm, xc, xn, k == 0, sc_prev, um_prev, in2, h2, fs2, ya, yb);
            if (!updA) ya = z2;
            if (!updB) yb = z2;
            if (live) st4(out2, (size_t)k * pitch + i0, make_float4(ya.x, ya.y, yb.x, yb.y));
            if (k == 0) {
                if (recA >= 0) st2(traces, (size_t)(m + 2) * nrec + recA, ya);
                if (recB >= 0) st2(traces, (size_t)(m + 2) * nrec + recB, yb);
            }
        }
        xm = xc;
        xc = xn;
        um_prev = rc.c;
        sc_prev = sc;
        rm = rc;
        rc = rn;
        rn = rnn;
        up = upn;
        sc = scn;
    }
    // bottom tile: the last free row's second step sees the rigid row, whose
    // displacement is zero but whose lambda and mu enter the operator (rc
    // holds that row of u^m after the loop)
    if (two && ke == nz - 1 && ke - 1 >= kb) {
        const int k = ke - 1;
        float fs2;
        const PairInj in2 = inj_of(k, sval2, fs2);
        RawN2 xb = rc;
        xb.c = z4;
        xb.hu = xb.hv = 0.f;
        float2 ya, yb;
        nodal_pair(xm, xc, xb, k == 0, sc_prev, um_prev, in2, h2, fs2, ya, yb);
        if (!updA) ya = z2;
        if (!updB) yb = z2;
        if (live) st4(out2, (size_t)k * pitch + i0, make_float4(ya.x, ya.y, yb.x, yb.y));
        if (k == 0) {
            if (recA >= 0) st2(traces, (size_t)(m + 2) * nrec + recA, ya);
            if (recB >= 0) st2(traces, (size_t)(m + 2) * nrec + recB, yb);
        }
    }
}

}  // namespace

void launch_nodal_stencil(const SolveDesc* descs, const int2* tiles, int ntiles, int step,
                          int variant, hipStream_t s) {
    const int blocks = (ntiles + kWavesPerBlock - 1) / kWavesPerBlock;
    const int threads = 64 * kWavesPerBlock;
    switch (variant) {
        case 17: stencil_nodal_w2<16><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 18: stencil_nodal_w2<32><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 19: stencil_nodal_tb2<16><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        case 20: stencil_nodal_tb2<32><<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
        default: stencil_nodal<<<blocks, threads, 0, s>>>(descs, tiles, ntiles, step); break;
    }
}

}  // namespace eig
