// Host-side pieces shared by the C-ABI entry points and the serving engine:
// the context, its budgeted workspace and pinned staging, descriptor blobs,
// argument checks and sizing helpers.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

namespace eig {
int set_error(int code, const std::string& msg);
}  // namespace eig

using namespace eig;

#define HIP_TRY(expr)                                                                 \
    do {                                                                              \
        hipError_t e_ = (expr);                                                       \
        if (e_ != hipSuccess)                                                         \
            return set_error(EIG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

namespace {

constexpr int kStageRing = 4;
constexpr size_t kAlign = 256;

inline size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

}  // namespace

struct eig_ctx {
    int device = 0;
    size_t budget = 0;
    char* ws = nullptr;      // device workspace
    size_t ws_size = 0;
    void* stage[kStageRing] = {};  // pinned staging blobs
    size_t stage_size[kStageRing] = {};
    hipEvent_t stage_ev[kStageRing] = {};
    bool stage_used[kStageRing] = {};
    int stage_next = 0;
    // stencil timing: event pairs per wave, launch / update / byte counters
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timing;
    int64_t launches = 0;
    double updates = 0.0, bytes = 0.0;
    double resolved_ms = 0.0;
    // stencil variant selection: forced (EIG_STENCIL_VARIANT), or tuned
    // online per (medium kind, nx, nz) and cached here
    int forced_variant = -1;
    int default_variant = 4;      // one step per launch
    int default_variant_tb = 11;  // two steps per launch
    int default_variant_tb3 = 15; // three steps per launch
    int temporal_blocking = 4;    // steps per launch for rigid edges: 1, 2, 3 or 4
    bool autotune = true;
    std::map<std::tuple<int, int, int, int, int>, int> tuned;
    int last_variant = -1;  // variant of the most recent stencil launch
    int64_t max_wave_solves = 0;  // 0: no limit (all solves of a wave per launch)
    // live field bytes per wave chunk (0: no limit); 192 MiB leaves room in
    // the device's 256 MB last-level cache for everything else a launch reads
    size_t wave_cache_bytes = (size_t)192 << 20;
    // waves are split for the cache only if at least this many solves fit a
    // chunk (fewer leave too few tiles per launch)
    int cache_chunk_min_solves = 16;
    // nodal media: solves on one medium whose tiles are interleaved by
    // position (coefficient reuse in L2); 1 keeps solve-major order
    int coef_interleave = 8;
    // grids whose two field levels fit one workgroup's LDS run resident
    // (their whole time loop in one launch)
    bool resident = true;
    // absorbing edges updated inside the one-step kernels that can (else by
    // the separate edge kernel after every step)
    bool fused_edges = true;
    // serving engines created on this context: live field bytes their
    // admitted groups may hold (0: no limit)
    size_t serve_cache_bytes = (size_t)192 << 20;
    // time loops captured as HIP graphs and replayed when a wave repeats
    // exactly (same descriptor blob at the same device address, same variants)
    bool graphs = true;
    hipStream_t capture_stream = nullptr;  // capture only; never runs work
    std::map<std::tuple<uint64_t, uintptr_t, size_t>, hipGraphExec_t> graph_cache;
    std::vector<std::tuple<uint64_t, uintptr_t, size_t>> graph_order;
    int64_t graph_captures = 0, graph_replays = 0;
};

namespace {

// Make the device workspace at least `bytes` large (never above budget).
inline int ensure_ws(eig_ctx* c, size_t bytes) {
    if (bytes <= c->ws_size) return EIG_OK;
    if (bytes > c->budget)
        return set_error(EIG_EBUDGET, "request needs " + std::to_string(bytes) +
                                          " bytes of device workspace, budget is " +
                                          std::to_string(c->budget));
    if (c->ws) {
        HIP_TRY(hipDeviceSynchronize());
        HIP_TRY(hipFree(c->ws));
        c->ws = nullptr;
        c->ws_size = 0;
    }
    size_t want = std::min(c->budget, std::max(bytes, bytes + bytes / 4));
    if (hipMalloc((void**)&c->ws, want) != hipSuccess) {
        (void)hipGetLastError();
        if (hipMalloc((void**)&c->ws, bytes) != hipSuccess) {
            (void)hipGetLastError();
            c->ws = nullptr;
            return set_error(EIG_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
        }
        want = bytes;
    }
    c->ws_size = want;
    return EIG_OK;
}

// Upload a host blob into device memory `dst` through a pinned staging
// buffer; a staging buffer is reused only after its previous copy finished.
inline int upload(eig_ctx* c, void* dst, const std::vector<char>& blob, hipStream_t s) {
    if (blob.empty()) return EIG_OK;
    const int r = c->stage_next;
    c->stage_next = (r + 1) % kStageRing;
    if (c->stage_used[r]) HIP_TRY(hipEventSynchronize(c->stage_ev[r]));
    if (c->stage_size[r] < blob.size()) {
        if (c->stage[r]) HIP_TRY(hipHostFree(c->stage[r]));
        c->stage[r] = nullptr;
        c->stage_size[r] = 0;
        const size_t sz = align_up(blob.size(), 1 << 20);
        HIP_TRY(hipHostMalloc(&c->stage[r], sz, hipHostMallocDefault));
        c->stage_size[r] = sz;
    }
    std::memcpy(c->stage[r], blob.data(), blob.size());
    HIP_TRY(hipMemcpyAsync(dst, c->stage[r], blob.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(c->stage_ev[r], s));
    c->stage_used[r] = true;
    return EIG_OK;
}

// Host-side image of a device region: record (offset, bytes) pieces first,
// fill them, then place the blob at a device base address.
struct Blob {
    std::vector<char> data;
    size_t put(const void* p, size_t bytes) {
        const size_t off = align_up(data.size());
        data.resize(off + bytes);
        if (bytes) std::memcpy(data.data() + off, p, bytes);
        return off;
    }
};

// Device workspace carving for one wave.
struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = align_up(off);
        off = o + bytes;
        return o;
    }
};

inline int floor_cell(double x, double h) { return (int)std::floor(x / h); }

inline bool valid_grid(const eig_grid& g) {
    return g.nx >= 8 && g.nz >= 8 && g.nx <= 65536 && g.nz <= 65536 && g.h > 0 &&
           g.dt > 0 && std::isfinite(g.h) && std::isfinite(g.dt) && g.nsteps >= 0 &&
           g.nsteps < (1 << 28) && (g.bc == EIG_BC_RIGID || g.bc == EIG_BC_ABSORBING);
}

// Source stencil rows/columns kx-2..kx+3 must stay on free nodes.
inline bool source_inside(double x, double z, const eig_grid& g) {
    if (!std::isfinite(x) || !std::isfinite(z)) return false;
    const int kx = floor_cell(x, g.h), kz = floor_cell(z, g.h);
    return kx - 2 >= 1 && kx + 3 <= g.nx - 2 && kz - 2 >= 0 && kz + 3 <= g.nz - 2;
}

// A deviation solve is forced on the union of the nominal and the perturbed
// 6x6 stencils, a window kSrcW = 7 nodes wide: the perturbed coordinate may
// leave the nominal cell by at most one cell either way.
inline bool deviation_in_window(double coord, double step, double h) {
    const int a = floor_cell(coord, h), b = floor_cell(coord + step, h);
    return std::abs(a - b) <= kSrcW - 6;
}

inline int pitch_of(int nx) { return (nx + kPitchAlign - 1) / kPitchAlign * kPitchAlign; }

struct SolveSpec {
    int grid;      // index into caller's grid array
    int medium;    // index into the deduplicated media
    int recset;    // index into the receiver sets
    double theta[kNT];
    int param;     // -1 nominal
    double step;
    int deriv;     // 1: forcing dF/dtheta_param (sensitivity solve)
    int stf;
    float2* traces;  // destination (device)
    const float2* rforce = nullptr;  // dual solve: receiver injection [nsteps][nrec]
    float2* wrec = nullptr;          // dual solve: window record [nsteps][49]
};

struct MediumKey {
    int kind;
    const double *rho, *lam, *mu;
    int nx, nz;
    double h, dt;
    bool operator<(const MediumKey& o) const {
        return std::tie(kind, rho, lam, mu, nx, nz, h, dt) <
               std::tie(o.kind, o.rho, o.lam, o.mu, o.nx, o.nz, o.h, o.dt);
    }
};

struct RecSet {
    std::vector<int32_t> ix;
    int nx;
};

inline int check_receivers(const eig_receivers& r, const eig_grid& g) {
    if (r.n < 0 || (r.n > 0 && !r.ix))
        return set_error(EIG_EINVAL, "receivers: n < 0 or ix NULL");
    std::vector<int32_t> v(r.ix, r.ix + r.n);
    for (int32_t x : v)
        if (x < 1 || x > g.nx - 2)
            return set_error(EIG_EINVAL, "receiver index outside the free surface 1..nx-2");
    std::sort(v.begin(), v.end());
    if (std::adjacent_find(v.begin(), v.end()) != v.end())
        return set_error(EIG_EINVAL, "receivers must be distinct");
    return EIG_OK;
}

// Device bytes for one solve (fields + forcing tables), excluding traces.
inline size_t solve_bytes(const eig_grid& g) {
    const size_t field = (size_t)g.nz * pitch_of(g.nx) * sizeof(float2);
    return align_up(field) * 4 + align_up(2 * kSrcW * kSrcW * sizeof(float)) +
           align_up((size_t)std::max(g.nsteps, 1) * sizeof(float)) + 4 * kAlign;
}

inline size_t medium_bytes(const MediumKey& k) {
    if (k.kind == EIG_MEDIUM_NODAL)
        return align_up((size_t)3 * k.nz * pitch_of(k.nx) * sizeof(float)) + kAlign;
    return align_up((size_t)k.nz * kCoefStride * sizeof(float)) + kAlign;
}


}  // namespace
