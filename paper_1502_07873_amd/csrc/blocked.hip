// Depth-only media, K leapfrog steps per launch with the tile kept in LDS
// (variant 23: 58 x 58 tiles, K = 4; the temporal_blocking 4 family, the
// default for rigid edges).
//
// A workgroup of 512 threads owns a TW x TH tile of one solve (two share a
// CU).  It loads u^{m-1} and u^m on the tile and a K-node halo around it
// (clipped to the grid) into LDS, then takes K steps there: step j forms
// u^{m+j} on the tile grown by K - j nodes, so the region shrinks by one
// node per step as the halo's values go stale from the outside in, and
// writes it over u^{m+j-2} in place (a node is read at the old level and
// written only by its owner).  Last it stores u^{m+K-1} and u^{m+K} of the
// tile.  Passes alternate between the two buffer pairs of a solve: pass L
// reads levels m-1 and m (m = K L) from pair L & 1 and writes its two last
// levels to the other pair, slot = level & 1, so no workgroup overwrites a
// value another one still loads.
//
// Per update a workgroup loads (tile + halo) x 2 levels and stores the tile
// x 2 levels: (66 x 66 + 58 x 58) x 16 B / (58 x 58 x 4) = 9.2 B; the halos
// neighbouring tiles share come from L2, so past L2 a launch moves each
// node's two levels once in and once out, 8 B per update (16 for the
// two-step kernels).  The halo costs 11 % more updates (the region of step j
// is (58 + 2(K-j))^2).  All loads of a thread are issued before its first
// LDS store (blk_load), so a workgroup waits for memory once; loading row by
// row, a wave waited for each row's loads in turn, and the kernel ran no
// faster than the two-step one (3.3e11 updates/s on the 512^2 Monte Carlo
// query, against 4.4-4.5e11 now).
//
// Work split: threads are packed over (band, column) pairs of the first
// step's region, fixed for a tile; at step j a thread clips its column and
// band to that step's region.  With 58-column tiles the first region is 64
// columns wide, so each wave is one band (blk_lane) and its lanes share their
// rows.  A thread streams down its rows keeping rows k-1, k, k+1 in
// registers.  Coefficient rows, forcing weights and the forcing series
// values sit in LDS.  Receivers are recorded by the tile that owns their
// column; forcing is added at every computed node of the window, halo
// included, so every tile that computes a node computes it alike.  The
// per-node arithmetic is layered_update, so the fields are bitwise those of
// every variant.  Rigid edges only, no receiver injection (dual solves run
// one step per launch).
#include "internal.h"
#include "node_update.h"
#include "tile.h"

namespace eig {

namespace {

// Where one tile of one pass sits.
struct BlkTile {
    const SolveDesc* d;
    int m, nst;                  // first level of the pass, steps taken
    int x0, z0, x1, z1;          // tile [x0, x1) x [z0, z1)
    int rx0, rz0, rw, rh;        // region (tile + halo, clipped)
    int pin, pout;               // buffer pairs read / written
};

template <int TW, int TH, int K>
__device__ __forceinline__ bool blk_setup(const SolveDesc* __restrict__ descs, int2 te, int pass,
                                          BlkTile& t) {
    t.d = descs + __builtin_amdgcn_readfirstlane(te.x);
    const int sc = __builtin_amdgcn_readfirstlane(te.y);
    const int L = pass - t.d->start;
    t.m = K * L;
    if (L < 0 || t.m >= t.d->nsteps) return false;
    t.nst = min(K, t.d->nsteps - t.m);
    const int nx = t.d->nx, nz = t.d->nz;
    t.x0 = (sc >> 16) * TW;
    t.z0 = (sc & 0xffff) * TH;
    t.x1 = min(t.x0 + TW, nx);
    t.z1 = min(t.z0 + TH, nz - 1);  // free rows < nz-1
    t.rx0 = max(t.x0 - K, 0);
    t.rz0 = max(t.z0 - K, 0);
    t.rw = min(t.x1 + K, nx) - t.rx0;
    t.rh = min(t.z1 + K, nz) - t.rz0;
    t.pin = 2 * (L & 1);
    t.pout = 2 - t.pin;
    return true;
}

__device__ __forceinline__ const float2* blk_buf(const SolveDesc* d, int i) {
    return i == 0 ? d->buf0 : (i == 1 ? d->buf1 : (i == 2 ? d->buf2 : d->buf3));
}

// The thread's (band, column) of a tile's first-step region.  A region at
// most 64 columns wide (tiles of 64 - 2 (K - 1) columns) gives each wave one
// band: lane l takes column c0 + l, so a wave's lanes share their rows and
// every lane of an interior tile's wave is busy in the first step.
struct BlkLane {
    int col, kb, ke;
    bool active;
};

template <int K, int NT>
__device__ __forceinline__ BlkLane blk_lane(const BlkTile& tl) {
    const int nx = tl.d->nx, nz = tl.d->nz;
    const int c0 = max(tl.x0 - (K - 1), 1), c1 = min(tl.x1 + (K - 1), nx - 1);
    const int r0 = max(tl.z0 - (K - 1), 0), r1 = min(tl.z1 + (K - 1), nz - 1);
    const int W = c1 - c0, nrow = r1 - r0;
    const int Wl = W <= 64 ? 64 : W;  // lanes per band
    const int nb = max(1, NT / Wl);
    const int band = (int)threadIdx.x / Wl;
    const int lane = (int)threadIdx.x - band * Wl;
    BlkLane ln;
    ln.active = band < nb && lane < W;
    ln.col = c0 + lane;
    ln.kb = r0 + band * nrow / nb;
    ln.ke = r0 + (band + 1) * nrow / nb;
    return ln;
}

// Receiver recorded by this thread (its column on the tile's surface row),
// or -1.  Read before a prefetch is issued: vector loads retire in order.
__device__ __forceinline__ int blk_rec(const BlkTile& tl, const BlkLane& ln) {
    if (ln.active && ln.kb == 0 && ln.col >= tl.x0 && ln.col < tl.x1)
        return ldi(tl.d->recmap, ln.col);
    return -1;
}

// Loads the region's two field levels (and, for nodal media, lambda, mu and
// s at its nodes) into LDS rows RW nodes apart.  Each thread issues all of
// its loads before its first LDS store, so a workgroup waits for memory once
// rather than once per row.
template <int NT, int RW, int NQ, bool NODAL>
__device__ __forceinline__ void blk_load(const BlkTile& tl, const float2* prev, const float2* cur,
                                         float2* Fp, float2* Fc, float* C0, float* C1,
                                         float* C2) {
    const int n = tl.rh * tl.rw, rw = tl.rw, pitch = tl.d->pitch;
    const size_t plane = (size_t)tl.d->nz * pitch;
    const float* coef = tl.d->coef;
    float2 a[NQ], b[NQ];
    float cl[NODAL ? NQ : 1], cm[NODAL ? NQ : 1], cs[NODAL ? NQ : 1];
    int off[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int e = (int)threadIdx.x + q * NT;
        off[q] = -1;
        if (e < n) {
            const int r = e / rw, c = e - r * rw;
            const size_t g = (size_t)(tl.rz0 + r) * pitch + tl.rx0 + c;
            a[q] = ld2(prev, g);
            b[q] = ld2(cur, g);
            if constexpr (NODAL) {
                cl[q] = ld1(coef, g);
                cm[q] = ld1(coef, plane + g);
                cs[q] = ld1(coef, 2 * plane + g);
            }
            off[q] = r * RW + c;
        }
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (off[q] < 0) continue;
        Fp[off[q]] = a[q];
        Fc[off[q]] = b[q];
        if constexpr (NODAL) {
            C0[off[q]] = cl[q];
            C1[off[q]] = cm[q];
            C2[off[q]] = cs[q];
        }
    }
}

// The K steps of one tile whose region, coefficient rows, forcing weights and
// series values are in LDS (barrier before the first step is the caller's).
template <int TW, int TH, int K, int NT, int RW>
__device__ __forceinline__ void blk_steps(const BlkTile& tl, const BlkLane& ln, int rec,
                                          float2 (*fld)[RW * (TH + 2 * K)],
                                          const float* cf_lds, const float* sw_lds,
                                          const float* sv_lds) {
    static_assert(TW + 2 * (K - 1) <= 64, "one band per wave");
    const SolveDesc* d = tl.d;
    const int nx = d->nx, nz = d->nz;
    const int m = tl.m, x0 = tl.x0, x1 = tl.x1, z0 = tl.z0, z1 = tl.z1;
    const int rz0 = tl.rz0;
    const bool active = ln.active;
    // a wave is one band: its rows are wave-uniform
    const int col = ln.col, kb = __builtin_amdgcn_readfirstlane(ln.kb),
              ke = __builtin_amdgcn_readfirstlane(ln.ke);
    const int si0 = d->src_i0, sk0 = d->src_k0;
    const int di = col - si0;
    const bool src_lane = di >= 0 && di < kSrcW;
    float2* traces = d->traces;
    const int nrec = d->nrec;
    const int lc = col - tl.rx0;  // LDS column
    for (int j = 1; j <= tl.nst; ++j) {
        const int lvl = m + j;
        const float2* Q = fld[(lvl - 1) & 1];
        float2* P = fld[lvl & 1];
        const int g = K - j;  // this step's region: the tile grown by g
        const int cj0 = max(x0 - g, 1), cj1 = min(x1 + g, nx - 1);
        const int rj0 = max(z0 - g, 0), rj1 = min(z1 + g, nz - 1);
        const int ka = max(kb, rj0), kz = min(ke, rj1);
        if (active && col >= cj0 && col < cj1 && ka < kz) {
            const float sval = sv_lds[j - 1];
            auto row = [&](int k) {
                const float2* rr = Q + (k - rz0) * RW + lc;
                const float2 l = rr[-1], c = rr[0], r = rr[1];
                return node_row(c.x, c.y, l.x, l.y, r.x, r.y);
            };
            auto update = [&](int k, const NodeRow& rm, const NodeRow& rc, const NodeRow& rn) {
                LayerCoef cf;
#pragma unroll
                for (int q = 0; q <= kFco; ++q) cf.c[q] = cf_lds[(k - rz0) * kCoefStride + q];
                float2* pp = P + (k - rz0) * RW + lc;
                const float2 up = *pp;
                const int dk = k - sk0;
                if (k != 0 && (unsigned)dk >= (unsigned)kSrcW) {
                    *pp = layered_update(cf, rm, rc, rn, up.x, up.y, false, 0.f, 0.f, 0.f);
                    return;
                }
                const bool in_win = src_lane && dk >= 0 && dk < kSrcW;
                float wu = 0.f, wv = 0.f;
                const float fsv = cf.c[kFco] * sval;
                if (in_win) {
                    wu = sw_lds[(0 * kSrcW + dk) * kSrcW + di];
                    wv = sw_lds[(1 * kSrcW + dk) * kSrcW + di];
                }
                const float2 nw = layered_update(cf, rm, rc, rn, up.x, up.y, in_win, fsv, wu, wv);
                *pp = nw;
                if (k == 0 && rec >= 0) st2(traces, (size_t)lvl * nrec + rec, nw);
            };
            NodeRow ra = NodeRow{0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (ka > 0) ra = row(ka - 1);
            NodeRow rb = row(ka);
            int k = ka;
            for (; k + 3 <= kz; k += 3) {
                const NodeRow r2 = row(k + 1);
                update(k, ra, rb, r2);
                const NodeRow r3 = row(k + 2);
                update(k + 1, rb, r2, r3);
                const NodeRow r4 = row(k + 3);
                update(k + 2, r2, r3, r4);
                ra = r3;
                rb = r4;
            }
            for (; k < kz; ++k) {
                const NodeRow r2 = row(k + 1);
                update(k, ra, rb, r2);
                ra = rb;
                rb = r2;
            }
        }
        __syncthreads();
    }
}

// Store the tile's last two levels to the other pair.
template <int TH, int K, int NT, int RW>
__device__ __forceinline__ void blk_store(const BlkTile& tl, float2 (*fld)[RW * (TH + 2 * K)]) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int pitch = tl.d->pitch;
    for (int q = 0; q < 2; ++q) {
        const int lvl = tl.m + tl.nst - 1 + q;
        float2* out = const_cast<float2*>(blk_buf(tl.d, tl.pout + (lvl & 1)));
        const float2* F = fld[lvl & 1];
        for (int r = tl.z0 + wave; r < tl.z1; r += NT / 64)
            for (int c = tl.x0 + lane; c < tl.x1; c += 64)
                st2(out, (size_t)r * pitch + c, F[(r - tl.rz0) * RW + (c - tl.rx0)]);
    }
}

template <int TW, int TH, int K, int NT, int WPC>
__global__ void __launch_bounds__(NT, NT / 256 * WPC)  // waves per SIMD for WPC per CU
stencil_layered_lds(const SolveDesc* __restrict__ descs, const int2* __restrict__ tiles,
                    int ntiles, int pass) {
    constexpr int RW = TW + 2 * K, RH = TH + 2 * K;  // largest region
    __shared__ float2 fld[2][RH * RW];
    __shared__ float cf_lds[RH * kCoefStride];
    __shared__ float sw_lds[2 * kSrcW * kSrcW];
    __shared__ float sv_lds[K];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    if (b >= ntiles) return;
    BlkTile tl;
    if (!blk_setup<TW, TH, K>(descs, tiles[b], pass, tl)) return;  // uniform
    const SolveDesc* d = tl.d;
    const int m = tl.m;
    const float2* prev = blk_buf(d, tl.pin + ((m - 1) & 1));  // u^{m-1}
    const float2* cur = blk_buf(d, tl.pin + (m & 1));         // u^m
    // the small tables' loads go out with the region's (stored after it)
    constexpr int NCF = (RH * kCoefStride + NT - 1) / NT;
    static_assert(NT >= 2 * kSrcW * kSrcW && NT >= K, "one table entry per thread");
    const int t = threadIdx.x;
    float cfv[NCF], swv = 0.f, svv = 0.f;
#pragma unroll
    for (int q = 0; q < NCF; ++q)
        if (t + q * NT < tl.rh * kCoefStride)
            cfv[q] = ld1(d->coef, (size_t)tl.rz0 * kCoefStride + t + q * NT);
    if (t < 2 * kSrcW * kSrcW) swv = ld1(d->srcw, t);
    if (t < tl.nst) svv = ld1(d->srcs, m + t);
    blk_load<NT, RW, (RH * RW + NT - 1) / NT, false>(tl, prev, cur, fld[(m - 1) & 1], fld[m & 1],
                                                     nullptr, nullptr, nullptr);
#pragma unroll
    for (int q = 0; q < NCF; ++q)
        if (t + q * NT < tl.rh * kCoefStride) cf_lds[t + q * NT] = cfv[q];
    if (t < 2 * kSrcW * kSrcW) sw_lds[t] = swv;
    if (t < tl.nst) sv_lds[t] = svv;
    const BlkLane ln = blk_lane<K, NT>(tl);
    const int rec = blk_rec(tl, ln);
    __syncthreads();
    blk_steps<TW, TH, K, NT, RW>(tl, ln, rec, fld, cf_lds, sw_lds, sv_lds);
    blk_store<TH, K, NT, RW>(tl, fld);
}

// u, v, lambda and mu of one row at columns i-1, i, i+1.
struct NodalRow3 {
    float2 ul, uc, ur;
    float ll, lc, lr, ml, mc, mr;
};

// Step j of a tile whose region, medium and forcing are in LDS, each thread
// streaming down its band of one column (variant 24).
template <int K, int RW, class FLD, class CL>
__device__ __forceinline__ void nodal_lds_stream(const BlkTile& tl, const BlkLane& ln, int rec,
                                                 int j, FLD fld, CL cl, const float* sw_lds,
                                                 float sval) {
    const SolveDesc* d = tl.d;
    const int nx = d->nx, nz = d->nz;
    const int lvl = tl.m + j;
    const float2* Q = fld[(lvl - 1) & 1];
    float2* P = fld[lvl & 1];
    const int gq = K - j;
    const int cj0 = max(tl.x0 - gq, 1), cj1 = min(tl.x1 + gq, nx - 1);
    const int rj0 = max(tl.z0 - gq, 0), rj1 = min(tl.z1 + gq, nz - 1);
    const int col = ln.col;
    // a wave is one band (the caller's tiles keep the first region within
    // 64 columns): its rows are wave-uniform
    const int ka = max(__builtin_amdgcn_readfirstlane(ln.kb), rj0);
    const int kz = min(__builtin_amdgcn_readfirstlane(ln.ke), rj1);
    if (!(ln.active && col >= cj0 && col < cj1 && ka < kz)) return;
    const int lc = col - tl.rx0, rz0 = tl.rz0;
    const int sk0 = d->src_k0, di = col - d->src_i0;
    const bool src_col = (unsigned)di < (unsigned)kSrcW;
    const float h2 = d->h2;
    auto row = [&](int k) {
        const int o = (k - rz0) * RW + lc;
        NodalRow3 r;
        r.ul = Q[o - 1];
        r.uc = Q[o];
        r.ur = Q[o + 1];
        r.ll = cl[0][o - 1];
        r.lc = cl[0][o];
        r.lr = cl[0][o + 1];
        r.ml = cl[1][o - 1];
        r.mc = cl[1][o];
        r.mr = cl[1][o + 1];
        return r;
    };
    // node (col, k) from rows k-1 (a), k (b), k+1 (c)
    auto update = [&](auto row_kind, int k, const NodalRow3& a, const NodalRow3& b,
                      const NodalRow3& c) {
        constexpr int RK = decltype(row_kind)::value;
        auto pick = [&](int kk) -> const NodalRow3& { return kk < k ? a : (kk == k ? b : c); };
        auto U = [&](int ii, int kk) {
            const NodalRow3& r = pick(kk);
            return ii < col ? r.ul : (ii == col ? r.uc : r.ur);
        };
        auto L = [&](int ii, int kk) {
            const NodalRow3& r = pick(kk);
            return ii < col ? r.ll : (ii == col ? r.lc : r.lr);
        };
        auto M = [&](int ii, int kk) {
            const NodalRow3& r = pick(kk);
            return ii < col ? r.ml : (ii == col ? r.mc : r.mr);
        };
        const int o = (k - rz0) * RW + lc;
        auto S = [&]() { return cl[2][o]; };
        const int wk = k - sk0;
        int inj = 0;
        float w0 = 0.f, w1 = 0.f;
        if (src_col && (unsigned)wk < (unsigned)kSrcW) {
            inj = 2;
            w0 = sw_lds[(0 * kSrcW + wk) * kSrcW + di];
            w1 = sw_lds[(1 * kSrcW + wk) * kSrcW + di];
        }
        const float2 nw = nodal_node_gen<RK>(U, L, M, S, P[o], col, k, inj, h2, sval, w0, w1);
        P[o] = nw;
        if (RK == 2 && rec >= 0) st2(d->traces, (size_t)lvl * d->nrec + rec, nw);
    };
    constexpr std::integral_constant<int, 1> below{};
    NodalRow3 ra, rb;
    int k = ka;
    if (k == 0) {
        rb = row(0);
        const NodalRow3 r1 = row(1);
        update(std::integral_constant<int, 2>(), 0, rb, rb, r1);
        ra = rb;
        rb = r1;
        k = 1;
    } else {
        ra = row(k - 1);
        rb = row(k);
    }
    for (; k + 3 <= kz; k += 3) {
        const NodalRow3 r2 = row(k + 1);
        update(below, k, ra, rb, r2);
        const NodalRow3 r3 = row(k + 2);
        update(below, k + 1, rb, r2, r3);
        const NodalRow3 r4 = row(k + 3);
        update(below, k + 2, r2, r3, r4);
        ra = r3;
        rb = r4;
    }
    for (; k < kz; ++k) {
        const NodalRow3 r2 = row(k + 1);
        update(below, k, ra, rb, r2);
        ra = rb;
        rb = r2;
    }
}

// Nodal media, K steps per launch (variant 24: 58 x 34 tiles; the
// forced-only variant 25: 64 x 24; two 512-thread workgroups per CU).  Same
// passes, buffer pairs, regions and receiver ownership as the depth-only
// kernel above; LDS also holds lambda, mu and dt^2/(rho h^2) over the region
// (28 B per region node with both field levels: 78 KB at 66 x 42, the
// tallest region two workgroups per CU can hold: each wave's band gets 5
// rows of the first step, 4 with 26-row tiles, which ran 8 % slower).  Variant
// 24 (STREAM) gives each wave one band of the 64-column first region and
// streams down its rows with u, v, lambda and mu of rows k-1, k, k+1 and
// columns i-1, i, i+1 in registers; variant 25 gives thread t the nodes t,
// t + NT, ... of a step's region in row-major order and reads every operand
// from LDS.  Both form each node through nodal_node_gen, the per-node update
// every nodal kernel uses, with the surface row's branch chosen at compile
// time; its fused products are explicit, so the fields are bitwise those of
// every nodal variant.  Rigid edges only, no receiver injection.
template <int TW, int TH, int K, int NT, int WPC, bool STREAM>
__global__ void __launch_bounds__(NT, NT / 256 * WPC)
stencil_nodal_lds(const SolveDesc* __restrict__ descs, const int2* __restrict__ tiles,
                  int ntiles, int pass) {
    constexpr int RW = TW + 2 * K, RH = TH + 2 * K;  // largest region
    static_assert(!STREAM || TW + 2 * (K - 1) <= 64, "one band per wave");
    __shared__ float2 fld[2][RH * RW];
    __shared__ float cl[3][RH * RW];  // lambda, mu, s
    __shared__ float sw_lds[2 * kSrcW * kSrcW];
    __shared__ float sv_lds[K];
    const int b = xcd_block(blockIdx.x, gridDim.x);
    if (b >= ntiles) return;
    BlkTile tl;
    if (!blk_setup<TW, TH, K>(descs, tiles[b], pass, tl)) return;  // uniform
    const SolveDesc* d = tl.d;
    const int m = tl.m, nx = d->nx, nz = d->nz;
    const float2* prev = blk_buf(d, tl.pin + ((m - 1) & 1));  // u^{m-1}
    const float2* cur = blk_buf(d, tl.pin + (m & 1));         // u^m
    static_assert(NT >= 2 * kSrcW * kSrcW && NT >= K, "one table entry per thread");
    const int t = threadIdx.x;
    float swv = 0.f, svv = 0.f;
    if (t < 2 * kSrcW * kSrcW) swv = ld1(d->srcw, t);
    if (t < tl.nst) svv = ld1(d->srcs, m + t);
    blk_load<NT, RW, (RH * RW + NT - 1) / NT, true>(tl, prev, cur, fld[(m - 1) & 1], fld[m & 1],
                                                    cl[0], cl[1], cl[2]);
    if (t < 2 * kSrcW * kSrcW) sw_lds[t] = swv;
    if (t < tl.nst) sv_lds[t] = svv;
    const BlkLane ln = blk_lane<K, NT>(tl);
    const int rec = STREAM ? blk_rec(tl, ln) : -1;
    __syncthreads();
    const int si0 = d->src_i0, sk0 = d->src_k0;
    float2* traces = d->traces;
    const int nrec = d->nrec;
    const float h2 = d->h2;
    for (int j = 1; j <= tl.nst; ++j) {
        if constexpr (STREAM) {
            nodal_lds_stream<K, RW>(tl, ln, rec, j, fld, cl, sw_lds, sv_lds[j - 1]);
            __syncthreads();
            continue;
        }
        const int lvl = m + j;
        const float2* Q = fld[(lvl - 1) & 1];
        float2* P = fld[lvl & 1];
        const int gq = K - j;  // this step's region: the tile grown by gq
        const int cj0 = max(tl.x0 - gq, 1), cj1 = min(tl.x1 + gq, nx - 1);
        const int rj0 = max(tl.z0 - gq, 0), rj1 = min(tl.z1 + gq, nz - 1);
        const int w = cj1 - cj0;
        const float sval = sv_lds[j - 1];
        // the surface row first (its own branch of the update), then the rows
        // below it, thread t taking nodes t, t + NT, ... in row-major order
        auto node = [&](auto row_kind, int i, int k, int o) {
            constexpr int RK = decltype(row_kind)::value;
            const float2* Qo = Q + o;
            const float* Lo = cl[0] + o;
            const float* Mo = cl[1] + o;
            auto U = [&](int ii, int kk) { return Qo[(kk - k) * RW + (ii - i)]; };
            auto L = [&](int ii, int kk) { return Lo[(kk - k) * RW + (ii - i)]; };
            auto M = [&](int ii, int kk) { return Mo[(kk - k) * RW + (ii - i)]; };
            auto S = [&]() { return cl[2][o]; };
            const int wk = k - sk0, wi = i - si0;
            int inj = 0;
            float w0 = 0.f, w1 = 0.f;
            if ((unsigned)wk < (unsigned)kSrcW && (unsigned)wi < (unsigned)kSrcW) {
                inj = 2;
                w0 = sw_lds[(0 * kSrcW + wk) * kSrcW + wi];
                w1 = sw_lds[(1 * kSrcW + wk) * kSrcW + wi];
            }
            const float2 nw = nodal_node_gen<RK>(U, L, M, S, P[o], i, k, inj, h2, sval, w0, w1);
            P[o] = nw;
            return nw;
        };
        int r0 = rj0;
        if (w > 0 && rj0 == 0 && rj1 > 0) {
            for (int i = cj0 + (int)threadIdx.x; i < cj1; i += NT) {
                const float2 nw = node(std::integral_constant<int, 2>(), i, 0, i - tl.rx0 - tl.rz0 * RW);
                if (i >= tl.x0 && i < tl.x1) {
                    const int rec = ldi(d->recmap, i);
                    if (rec >= 0) st2(traces, (size_t)lvl * nrec + rec, nw);
                }
            }
            r0 = 1;
        }
        if (w > 0 && rj1 > r0) {
            const int dk = NT / w, di = NT - dk * w;
            const int t0 = (int)threadIdx.x / w;
            int k = r0 + t0, i = cj0 + ((int)threadIdx.x - t0 * w);
            int o = (k - tl.rz0) * RW + (i - tl.rx0);
            const int dox = dk * RW + di, dow = RW - w;
            while (k < rj1) {
                node(std::integral_constant<int, 1>(), i, k, o);
                i += di;
                k += dk;
                o += dox;
                if (i >= cj1) {
                    i -= w;
                    ++k;
                    o += dow;
                }
            }
        }
        __syncthreads();
    }
    blk_store<TH, K, NT, RW>(tl, fld);
}

}  // namespace

void launch_blocked_stencil(const SolveDesc* descs, const int2* tiles, int ntiles, int pass,
                            int variant, hipStream_t s) {
    switch (variant) {
        case 24:
            stencil_nodal_lds<58, 34, 4, 512, 2, true><<<ntiles, 512, 0, s>>>(descs, tiles,
                                                                              ntiles, pass);
            break;
        case 25:
            stencil_nodal_lds<64, 24, 4, 512, 2, false><<<ntiles, 512, 0, s>>>(descs, tiles,
                                                                               ntiles, pass);
            break;
        default:
            stencil_layered_lds<58, 58, 4, 512, 2><<<ntiles, 512, 0, s>>>(descs, tiles, ntiles,
                                                                          pass);
            break;
    }
}

}  // namespace eig
