// C-ABI layer: argument checks, planning, device workspace and launches.
//
// Solve engine.  A call turns into a list of solves (grid, medium, forcing,
// receivers, trace destination).  Solves are grouped in waves that fit the
// context's HBM budget; for each wave the host builds descriptor tables
// (solve descriptors, a tile-to-solve map, forcing-table jobs, receiver maps)
// in one pinned staging blob, uploads it with a single copy, builds the
// medium coefficient and forcing tables on the device, clears the wavefields,
// and then enqueues one stencil launch per time step over all tiles of the
// solves still running (solves sorted by step count, so the running ones are
// a prefix).  Nothing is copied back; everything is ordered on the caller's
// stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "internal.h"

namespace eig {

static thread_local std::string g_error;

int set_error(int code, const std::string& msg) {
    g_error = msg;
    return code;
}

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

size_t align_up(size_t v, size_t a = kAlign) { return (v + a - 1) / a * a; }

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
};

namespace {

// Make the device workspace at least `bytes` large (never above budget).
int ensure_ws(eig_ctx* c, size_t bytes) {
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
int upload(eig_ctx* c, void* dst, const std::vector<char>& blob, hipStream_t s) {
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

int floor_cell(double x, double h) { return (int)std::floor(x / h); }

bool valid_grid(const eig_grid& g) {
    return g.nx >= 8 && g.nz >= 8 && g.nx <= 65536 && g.nz <= 65536 && g.h > 0 &&
           g.dt > 0 && std::isfinite(g.h) && std::isfinite(g.dt) && g.nsteps >= 0 &&
           g.nsteps < (1 << 28);
}

// Source stencil rows/columns kx-2..kx+3 must stay on free nodes.
bool source_inside(double x, double z, const eig_grid& g) {
    if (!std::isfinite(x) || !std::isfinite(z)) return false;
    const int kx = floor_cell(x, g.h), kz = floor_cell(z, g.h);
    return kx - 2 >= 1 && kx + 3 <= g.nx - 2 && kz - 2 >= 0 && kz + 3 <= g.nz - 2;
}

int pitch_of(int nx) { return (nx + kTileW - 1) / kTileW * kTileW; }

struct SolveSpec {
    int grid;      // index into caller's grid array
    int medium;    // index into the deduplicated media
    int recset;    // index into the receiver sets
    double theta[kNT];
    int param;     // -1 nominal
    double step;
    int stf;
    float2* traces;  // destination (device)
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

int check_receivers(const eig_receivers& r, const eig_grid& g) {
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
size_t solve_bytes(const eig_grid& g) {
    const size_t field = (size_t)g.nz * pitch_of(g.nx) * sizeof(float2);
    return align_up(field) * 2 + align_up(2 * kSrcW * kSrcW * sizeof(float)) +
           align_up((size_t)std::max(g.nsteps, 1) * sizeof(float)) + 4 * kAlign;
}

size_t medium_bytes(const MediumKey& k) {
    if (k.kind == EIG_MEDIUM_NODAL)
        return align_up((size_t)3 * k.nz * pitch_of(k.nx) * sizeof(float)) + kAlign;
    return align_up((size_t)k.nz * kCoefStride * sizeof(float)) + kAlign;
}

// Run a set of solves that fits the workspace region [base, base+cap).
// `extra_off` bytes at the start of the region are reserved by the caller.
int run_wave(eig_ctx* c, const std::vector<SolveSpec>& solves,
             const std::vector<eig_grid>& grids, const std::vector<MediumKey>& media,
             const std::vector<RecSet>& recsets, char* base, size_t cap,
             hipStream_t s) {
    const int n = (int)solves.size();
    if (n == 0) return EIG_OK;
    Carve cv;
    // which media / recsets this wave uses
    std::vector<int> med_used, rec_used;
    for (const auto& sp : solves) {
        med_used.push_back(sp.medium);
        rec_used.push_back(sp.recset);
    }
    std::sort(med_used.begin(), med_used.end());
    med_used.erase(std::unique(med_used.begin(), med_used.end()), med_used.end());
    std::sort(rec_used.begin(), rec_used.end());
    rec_used.erase(std::unique(rec_used.begin(), rec_used.end()), rec_used.end());
    std::map<int, size_t> med_off;
    for (int m : med_used) med_off[m] = cv.take(medium_bytes(media[m]));
    // fields: one contiguous block for all solves (cleared with one launch)
    std::vector<size_t> f0(n), f1(n), sw(n), ss(n);
    const size_t fields_begin = align_up(cv.off);
    cv.off = fields_begin;
    for (int i = 0; i < n; ++i) {
        const eig_grid& g = grids[solves[i].grid];
        const size_t field = (size_t)g.nz * pitch_of(g.nx) * sizeof(float2);
        f0[i] = cv.take(field);
        f1[i] = cv.take(field);
    }
    const size_t fields_end = cv.off;
    for (int i = 0; i < n; ++i) {
        const eig_grid& g = grids[solves[i].grid];
        sw[i] = cv.take(2 * kSrcW * kSrcW * sizeof(float));
        ss[i] = cv.take((size_t)std::max(g.nsteps, 1) * sizeof(float));
    }
    // order: medium kind, then steps descending
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        const int ka = media[solves[a].medium].kind, kb = media[solves[b].medium].kind;
        if (ka != kb) return ka < kb;
        return grids[solves[a].grid].nsteps > grids[solves[b].grid].nsteps;
    });
    // the staging blob (receiver maps, descriptors, tile map, forcing jobs)
    // gets its device place first so descriptors can point into it
    size_t ntiles_total = 0;
    for (int i = 0; i < n; ++i) {
        const eig_grid& g = grids[solves[i].grid];
        ntiles_total += (size_t)(pitch_of(g.nx) / kTileW) * ((g.nz - 1 + kTileRows - 1) / kTileRows);
    }
    size_t blob_bound = align_up((size_t)n * sizeof(SolveDesc)) +
                        align_up(ntiles_total * sizeof(int32_t)) +
                        align_up((size_t)n * sizeof(SourceJob)) + 4 * kAlign;
    for (int r : rec_used) blob_bound += align_up((size_t)pitch_of(recsets[r].nx) * sizeof(int32_t));
    const size_t blob_dev = cv.take(blob_bound);
    if (cv.off > cap) return set_error(EIG_EBUDGET, "wave does not fit the workspace");
    char* bd = base + blob_dev;
    Blob blob;
    std::map<int, size_t> o_rec;
    for (int r : rec_used) {
        std::vector<int32_t> map(pitch_of(recsets[r].nx), -1);
        for (size_t q = 0; q < recsets[r].ix.size(); ++q) map[recsets[r].ix[q]] = (int32_t)q;
        o_rec[r] = blob.put(map.data(), map.size() * sizeof(int32_t));
    }
    // descriptors and tiles
    std::vector<SolveDesc> desc(n);
    std::vector<int32_t> tiles;
    std::vector<SourceJob> jobs(n);
    struct Group { int kind; int first_tile; std::vector<std::pair<int, int>> steps_tiles; };
    std::vector<Group> groups;
    for (int oi = 0; oi < n; ++oi) {
        const int i = ord[oi];
        const SolveSpec& sp = solves[i];
        const eig_grid& g = grids[sp.grid];
        const MediumKey& mk = media[sp.medium];
        SolveDesc& d = desc[oi];
        d.buf0 = (float2*)(base + f0[i]);
        d.buf1 = (float2*)(base + f1[i]);
        d.coef = (const float*)(base + med_off[sp.medium]);
        d.srcw = (const float*)(base + sw[i]);
        d.srcs = (const float*)(base + ss[i]);
        d.recmap = (const int32_t*)(bd + o_rec[sp.recset]);
        d.traces = sp.traces;
        d.nx = g.nx;
        d.nz = g.nz;
        d.pitch = pitch_of(g.nx);
        d.nsteps = g.nsteps;
        d.start = 0;
        d.nrec = (int32_t)recsets[sp.recset].ix.size();
        d.nstrip = d.pitch / kTileW;
        d.nchunk = (g.nz - 1 + kTileRows - 1) / kTileRows;
        d.medium_kind = mk.kind;
        d.h2 = (float)(g.h * g.h);
        // forcing window: union of the nominal and perturbed 6x6 stencils
        SourceJob& J = jobs[oi];
        std::memcpy(J.theta, sp.theta, sizeof(J.theta));
        J.step = sp.step;
        J.h = g.h;
        J.dt = g.dt;
        J.param = sp.param;
        J.kx = floor_cell(sp.theta[0], g.h);
        J.kz = floor_cell(sp.theta[1], g.h);
        double tp[kNT];
        std::memcpy(tp, sp.theta, sizeof(tp));
        if (sp.param >= 0) tp[sp.param] = sp.theta[sp.param] + sp.step;
        J.kx2 = floor_cell(tp[0], g.h);
        J.kz2 = floor_cell(tp[1], g.h);
        J.i0 = std::min(J.kx, J.kx2) - 2;
        J.k0 = std::min(J.kz, J.kz2) - 2;
        // keep the 7-wide window inside the grid (the extra column/row is 0)
        J.i0 = std::min(J.i0, g.nx - kSrcW);
        J.k0 = std::min(J.k0, g.nz - kSrcW);
        J.nsteps = g.nsteps;
        J.stf = sp.stf;
        J.srcw = (float*)(base + sw[i]);
        J.srcs = (float*)(base + ss[i]);
        d.src_i0 = J.i0;
        d.src_k0 = J.k0;
        if (groups.empty() || groups.back().kind != mk.kind)
            groups.push_back(Group{mk.kind, (int)tiles.size(), {}});
        d.tile0 = (int)tiles.size() - groups.back().first_tile;
        const int nt = d.nstrip * d.nchunk;
        for (int t = 0; t < nt; ++t) tiles.push_back(oi);
        groups.back().steps_tiles.push_back({g.nsteps, (int)tiles.size() - groups.back().first_tile});
    }
    const size_t o_desc = blob.put(desc.data(), desc.size() * sizeof(SolveDesc));
    const size_t o_tile = blob.put(tiles.data(), tiles.size() * sizeof(int32_t));
    const size_t o_jobs = blob.put(jobs.data(), jobs.size() * sizeof(SourceJob));
    if (blob.data.size() > blob_bound) return set_error(EIG_EBUDGET, "descriptor blob overflow");
    int rc = upload(c, bd, blob.data, s);
    if (rc) return rc;
    // tables
    for (int m : med_used) {
        const MediumKey& mk = media[m];
        float* coef = (float*)(base + med_off[m]);
        if (mk.kind == EIG_MEDIUM_NODAL)
            launch_nodal_coef(mk.rho, mk.lam, mk.mu, mk.nx, mk.nz, pitch_of(mk.nx), mk.h,
                              mk.dt, coef, s);
        else
            launch_layered_coef(mk.rho, mk.lam, mk.mu, mk.nz, mk.h, mk.dt, coef, s);
    }
    launch_source_tables((const SourceJob*)(bd + o_jobs), n, 0, s);
    launch_fill_zero(base + fields_begin, fields_end - fields_begin, s);
    const SolveDesc* ddesc = (const SolveDesc*)(bd + o_desc);
    launch_zero_level0(ddesc, n, s);  // traces at t_0 (zero initial state)
    HIP_TRY(hipGetLastError());
    // time loop
    const int32_t* dtile = (const int32_t*)(bd + o_tile);
    int max_steps = 0;
    for (const auto& g : groups)
        for (const auto& st : g.steps_tiles) max_steps = std::max(max_steps, st.first);
    // per group and solve: grid-point updates per step, in launch order
    std::vector<std::vector<double>> upd_per_solve(groups.size());
    {
        int oi = 0;
        for (size_t gi = 0; gi < groups.size(); ++gi)
            for (size_t q = 0; q < groups[gi].steps_tiles.size(); ++q, ++oi)
                upd_per_solve[gi].push_back((double)desc[oi].nx * desc[oi].nz);
    }
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (max_steps > 0) {
        HIP_TRY(hipEventCreate(&ev0));
        HIP_TRY(hipEventCreate(&ev1));
        HIP_TRY(hipEventRecord(ev0, s));
    }
    for (int step = 0; step < max_steps; ++step) {
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            const auto& g = groups[gi];
            // running solves form a prefix (steps descending within a group)
            int ntile = 0;
            double upd = 0.0;
            for (size_t q = 0; q < g.steps_tiles.size(); ++q) {
                const auto& st = g.steps_tiles[q];
                if (st.first > step) {
                    ntile = st.second;
                    upd += upd_per_solve[gi][q];
                } else {
                    break;
                }
            }
            if (ntile > 0) {
                launch_stencil(ddesc, dtile + g.first_tile, ntile, step, g.kind, s);
                c->launches += 1;
                c->updates += upd;
                c->bytes += upd * (g.kind == EIG_MEDIUM_NODAL ? 36.0 : 24.0);
            }
        }
    }
    if (max_steps > 0) {
        HIP_TRY(hipEventRecord(ev1, s));
        c->timing.push_back({ev0, ev1});
    }
    HIP_TRY(hipGetLastError());
    return EIG_OK;
}

// Incremental upper bound of the workspace a wave needs.
struct WaveSizer {
    const std::vector<eig_grid>& grids;
    const std::vector<MediumKey>& media;
    const std::vector<RecSet>& recsets;
    std::vector<char> med_seen, rec_seen;
    size_t bytes = 64 * kAlign;
    WaveSizer(const std::vector<eig_grid>& g, const std::vector<MediumKey>& m,
              const std::vector<RecSet>& r)
        : grids(g), media(m), recsets(r), med_seen(m.size(), 0), rec_seen(r.size(), 0) {}
    size_t cost(const SolveSpec& sp) const {
        const eig_grid& g = grids[sp.grid];
        size_t b = solve_bytes(g) + sizeof(SolveDesc) + sizeof(SourceJob) + 64;
        b += (size_t)((g.nz - 1 + kTileRows - 1) / kTileRows) * (pitch_of(g.nx) / kTileW) * 4;
        if (!med_seen[sp.medium]) b += medium_bytes(media[sp.medium]);
        if (!rec_seen[sp.recset]) b += 2 * align_up((size_t)pitch_of(recsets[sp.recset].nx) * 4);
        return b;
    }
    void add(const SolveSpec& sp) {
        bytes += cost(sp);
        med_seen[sp.medium] = 1;
        rec_seen[sp.recset] = 1;
    }
};

int validate_medium(const eig_medium& m) {
    if (m.kind != EIG_MEDIUM_LAYERED && m.kind != EIG_MEDIUM_NODAL)
        return set_error(EIG_EINVAL, "medium kind");
    if (!m.rho || !m.lam || !m.mu) return set_error(EIG_EINVAL, "medium arrays NULL");
    return EIG_OK;
}

int medium_index(std::vector<MediumKey>& media, std::map<MediumKey, int>& seen,
                 const eig_medium& m, const eig_grid& g) {
    MediumKey k{m.kind, m.rho, m.lam, m.mu, g.nx, g.nz, g.h, g.dt};
    auto it = seen.find(k);
    if (it != seen.end()) return it->second;
    const int id = (int)media.size();
    media.push_back(k);
    seen[k] = id;
    return id;
}

}  // namespace

extern "C" {

const char* eig_last_error(void) { return g_error.c_str(); }

int eig_ctx_create(int device, size_t hbm_budget_bytes, eig_ctx** out) {
    if (!out) return set_error(EIG_EINVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return set_error(EIG_EINVAL, "no such device");
    HIP_TRY(hipSetDevice(device));
    eig_ctx* c = new eig_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    for (int r = 0; r < kStageRing; ++r) {
        if (hipEventCreateWithFlags(&c->stage_ev[r], hipEventDisableTiming) != hipSuccess) {
            delete c;
            return set_error(EIG_EHIP, "hipEventCreate failed");
        }
    }
    *out = c;
    return EIG_OK;
}

void eig_ctx_destroy(eig_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    if (c->ws) (void)hipFree(c->ws);
    for (auto& pr : c->timing) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    for (int r = 0; r < kStageRing; ++r) {
        if (c->stage[r]) (void)hipHostFree(c->stage[r]);
        if (c->stage_ev[r]) (void)hipEventDestroy(c->stage_ev[r]);
    }
    delete c;
}

size_t eig_ctx_workspace_bytes(const eig_ctx* c) { return c ? c->ws_size : 0; }

int eig_ctx_stencil_stats(eig_ctx* c, int32_t reset, double* ms, int64_t* launches,
                          double* updates, double* bytes) {
    if (!c) return set_error(EIG_EINVAL, "ctx is NULL");
    HIP_TRY(hipSetDevice(c->device));
    for (auto& pr : c->timing) {
        float t = 0.f;
        HIP_TRY(hipEventSynchronize(pr.second));
        HIP_TRY(hipEventElapsedTime(&t, pr.first, pr.second));
        c->resolved_ms += t;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    c->timing.clear();
    if (ms) *ms = c->resolved_ms;
    if (launches) *launches = c->launches;
    if (updates) *updates = c->updates;
    if (bytes) *bytes = c->bytes;
    if (reset) {
        c->resolved_ms = 0.0;
        c->launches = 0;
        c->updates = 0.0;
        c->bytes = 0.0;
    }
    return EIG_OK;
}

int forward_solve_batch(eig_ctx* c, int32_t nsolve, const eig_grid* grid,
                        const eig_medium* medium, const double* theta,
                        const int32_t* dev_param, const double* dev_step,
                        int32_t stf_kind, const eig_receivers* rec,
                        float* const* traces, void* stream) {
    if (!c) return set_error(EIG_EINVAL, "ctx is NULL");
    if (nsolve < 0) return set_error(EIG_EINVAL, "nsolve < 0");
    if (nsolve == 0) return EIG_OK;
    if (!grid || !medium || !theta || !rec || !traces)
        return set_error(EIG_EINVAL, "NULL array argument");
    if (stf_kind != EIG_STF_GAUSS && stf_kind != EIG_STF_GAUSS_DERIV)
        return set_error(EIG_EINVAL, "stf_kind");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<eig_grid> grids(grid, grid + nsolve);
    std::vector<MediumKey> media;
    std::map<MediumKey, int> seen;
    std::vector<RecSet> recsets;
    std::vector<SolveSpec> solves;
    for (int i = 0; i < nsolve; ++i) {
        const eig_grid& g = grid[i];
        if (!valid_grid(g)) return set_error(EIG_EINVAL, "grid " + std::to_string(i));
        int rc = validate_medium(medium[i]);
        if (rc) return rc;
        rc = check_receivers(rec[i], g);
        if (rc) return rc;
        if (!traces[i]) return set_error(EIG_EINVAL, "traces pointer NULL");
        SolveSpec sp{};
        sp.grid = i;
        sp.medium = medium_index(media, seen, medium[i], g);
        sp.recset = (int)recsets.size();
        recsets.push_back(RecSet{std::vector<int32_t>(rec[i].ix, rec[i].ix + rec[i].n), g.nx});
        std::memcpy(sp.theta, theta + (size_t)i * kNT, sizeof(sp.theta));
        sp.param = dev_param ? dev_param[i] : -1;
        sp.step = (sp.param >= 0 && dev_step) ? dev_step[i] : 0.0;
        if (sp.param < -1 || sp.param >= kNT) return set_error(EIG_EINVAL, "dev_param");
        if (sp.param >= 0 && (!(sp.step != 0.0) || !std::isfinite(sp.step)))
            return set_error(EIG_EINVAL, "dev_step must be finite and nonzero");
        for (int j = 0; j < kNT; ++j)
            if (!std::isfinite(sp.theta[j])) return set_error(EIG_EINVAL, "theta not finite");
        if (!source_inside(sp.theta[0], sp.theta[1], g))
            return set_error(EIG_EINVAL, "source stencil touches a rigid node");
        if (sp.param == 0 || sp.param == 1) {
            double x = sp.theta[0], z = sp.theta[1];
            (sp.param == 0 ? x : z) += sp.step;
            if (!source_inside(x, z, g))
                return set_error(EIG_EINVAL, "perturbed source stencil touches a rigid node");
        }
        sp.stf = stf_kind;
        sp.traces = (float2*)traces[i];
        solves.push_back(sp);
    }
    // waves within the budget
    size_t i0 = 0;
    while (i0 < solves.size()) {
        WaveSizer ws(grids, media, recsets);
        std::vector<SolveSpec> wave;
        size_t i1 = i0;
        while (i1 < solves.size()) {
            const size_t add = ws.cost(solves[i1]);
            if (!wave.empty() && ws.bytes + add > c->budget) break;
            ws.add(solves[i1]);
            wave.push_back(solves[i1]);
            ++i1;
        }
        int rc = ensure_ws(c, ws.bytes);
        if (rc) return rc;
        rc = run_wave(c, wave, grids, media, recsets, c->ws, c->ws_size, s);
        if (rc) return rc;
        i0 = i1;
    }
    return EIG_OK;
}

int jacobian_fd(eig_ctx* c, int32_t nsample, const eig_grid* grid,
                const eig_medium* medium, const double* theta, double rel_step,
                int32_t stf_kind, const eig_receivers* rec, int32_t sigma_mode,
                const double* sigma, int32_t per_receiver, float* const* nominal,
                double* const* J, double* H1, int32_t* status, void* stream) {
    if (!c) return set_error(EIG_EINVAL, "ctx is NULL");
    if (nsample < 0) return set_error(EIG_EINVAL, "nsample < 0");
    if (nsample == 0) return EIG_OK;
    if (!grid || !medium || !theta || !rec || !sigma || !H1)
        return set_error(EIG_EINVAL, "NULL array argument");
    if (!(rel_step > 0) || !std::isfinite(rel_step) || rel_step > 0.1)
        return set_error(EIG_EINVAL, "rel_step must be in (0, 0.1]");
    if (stf_kind != EIG_STF_GAUSS && stf_kind != EIG_STF_GAUSS_DERIV)
        return set_error(EIG_EINVAL, "stf_kind");
    if (sigma_mode != EIG_SIGMA_GIVEN && sigma_mode != EIG_SIGMA_NOMINAL_PEAK)
        return set_error(EIG_EINVAL, "sigma_mode");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const int nrec0 = rec[0].n;
    for (int i = 0; i < nsample; ++i) {
        const eig_grid& g = grid[i];
        if (!valid_grid(g)) return set_error(EIG_EINVAL, "grid " + std::to_string(i));
        int rc = validate_medium(medium[i]);
        if (rc) return rc;
        rc = check_receivers(rec[i], g);
        if (rc) return rc;
        if (rec[i].n < 1) return set_error(EIG_EINVAL, "at least one receiver");
        if (per_receiver && rec[i].n != nrec0)
            return set_error(EIG_EINVAL, "per_receiver needs equal receiver counts");
        if (!(sigma[i] > 0) || !std::isfinite(sigma[i]))
            return set_error(EIG_EINVAL, "sigma must be positive");
        const double* th = theta + (size_t)i * kNT;
        for (int j = 0; j < kNT; ++j) {
            if (!std::isfinite(th[j]) || th[j] == 0.0)
                return set_error(EIG_EINVAL, "theta entries must be finite and nonzero");
        }
        for (int j = 0; j < 2; ++j)
            for (int sg = -1; sg <= 1; ++sg) {
                double x = th[0], z = th[1];
                const double d = rel_step * std::fabs(th[j]);
                (j == 0 ? x : z) += sg * d;
                if (!source_inside(x, z, g))
                    return set_error(EIG_EINVAL, "source stencil touches a rigid node");
            }
    }
    std::vector<eig_grid> grids(grid, grid + nsample);
    std::vector<MediumKey> media;
    std::map<MediumKey, int> seen;
    std::vector<RecSet> recsets;
    std::vector<int> med_of(nsample), rec_of(nsample);
    std::map<std::pair<int, std::vector<int32_t>>, int> rec_seen;
    for (int i = 0; i < nsample; ++i) {
        med_of[i] = medium_index(media, seen, medium[i], grid[i]);
        std::vector<int32_t> ix(rec[i].ix, rec[i].ix + rec[i].n);
        auto key = std::make_pair(grid[i].nx, ix);
        auto it = rec_seen.find(key);
        if (it == rec_seen.end()) {
            rec_seen[key] = (int)recsets.size();
            rec_of[i] = (int)recsets.size();
            recsets.push_back(RecSet{ix, grid[i].nx});
        } else {
            rec_of[i] = it->second;
        }
    }
    const int ngroup = per_receiver ? nrec0 : 1;
    // bytes of one sample beyond its solves: 15 trace arrays + descriptors
    auto sample_trace_bytes = [&](int i) {
        return 15 * align_up((size_t)(grid[i].nsteps + 1) * rec[i].n * sizeof(float2));
    };
    int s0 = 0;
    while (s0 < nsample) {
        // grow the wave sample by sample while it fits the budget
        int s1 = s0;
        size_t need = 0;
        WaveSizer wsz(grids, media, recsets);
        size_t extra = 4 * kAlign;
        while (s1 < nsample) {
            SolveSpec sp{};
            sp.grid = s1;
            sp.medium = med_of[s1];
            sp.recset = rec_of[s1];
            const size_t one = wsz.cost(sp);
            const size_t more = 15 * one + sample_trace_bytes(s1) + sizeof(SampleDesc) +
                                3 * kAlign + 2 * sizeof(double);
            if (s1 > s0 && wsz.bytes + extra + more > c->budget) break;
            for (int q = 0; q < 15; ++q) wsz.add(sp);
            extra += sample_trace_bytes(s1) + sizeof(SampleDesc) + 3 * kAlign + 2 * sizeof(double);
            need = wsz.bytes + extra;
            ++s1;
        }
        int rc = ensure_ws(c, need);
        if (rc) return rc;
        // carve: [traces | sample descs | sigma given | sigma | solve region]
        Carve cv;
        const int ns = s1 - s0;
        std::vector<std::array<size_t, 15>> toff(ns);
        for (int q = 0; q < ns; ++q)
            for (int k = 0; k < 15; ++k)
                toff[q][k] = cv.take((size_t)(grid[s0 + q].nsteps + 1) * rec[s0 + q].n * sizeof(float2));
        const size_t o_sd = cv.take(ns * sizeof(SampleDesc));
        const size_t o_given = cv.take(ns * sizeof(double));
        const size_t o_sig = cv.take(ns * sizeof(double));
        const size_t solve_base = align_up(cv.off);
        std::vector<SolveSpec> solves;
        std::vector<SampleDesc> sds(ns);
        for (int q = 0; q < ns; ++q) {
            const int i = s0 + q;
            const double* th = theta + (size_t)i * kNT;
            SampleDesc& sd = sds[q];
            std::memset(&sd, 0, sizeof(sd));
            sd.nt = grid[i].nsteps + 1;
            sd.nrec = rec[i].n;
            sd.J = J ? J[i] : nullptr;
            float2* nom = (nominal && nominal[i]) ? (float2*)nominal[i]
                                                  : (float2*)(c->ws + toff[q][0]);
            sd.nominal = nom;
            SolveSpec sp{};
            sp.grid = i;
            sp.medium = med_of[i];
            sp.recset = rec_of[i];
            std::memcpy(sp.theta, th, sizeof(sp.theta));
            sp.stf = stf_kind;
            sp.param = -1;
            sp.step = 0.0;
            sp.traces = nom;
            solves.push_back(sp);
            for (int j = 0; j < kNT; ++j) {
                const double d = rel_step * std::fabs(th[j]);
                sd.inv2d[j] = 1.0 / (2.0 * d);
                for (int sg = 0; sg < 2; ++sg) {
                    SolveSpec pj = sp;
                    pj.param = j;
                    pj.step = sg == 0 ? d : -d;
                    pj.traces = (float2*)(c->ws + toff[q][1 + 2 * j + sg]);
                    sd.dev[2 * j + sg] = pj.traces;
                    solves.push_back(pj);
                }
            }
        }
        rc = run_wave(c, solves, grids, media, recsets, c->ws + solve_base,
                      c->ws_size - solve_base, s);
        if (rc) return rc;
        // upload descriptors and sigma values to their carved places
        std::vector<char> part1(ns * sizeof(SampleDesc));
        std::memcpy(part1.data(), sds.data(), part1.size());
        rc = upload(c, c->ws + o_sd, part1, s);
        if (rc) return rc;
        std::vector<char> part2(ns * sizeof(double));
        std::memcpy(part2.data(), sigma + s0, part2.size());
        rc = upload(c, c->ws + o_given, part2, s);
        if (rc) return rc;
        const SampleDesc* dsd = (const SampleDesc*)(c->ws + o_sd);
        double* dsig = (double*)(c->ws + o_sig);
        launch_sample_check(dsd, ns, (const double*)(c->ws + o_given), sigma_mode, dsig,
                            status ? status + s0 : nullptr, s);
        launch_hessian(dsd, ns, per_receiver ? 1 : 0, ngroup, dsig,
                       H1 + (size_t)s0 * ngroup * kNT * kNT, s);
        HIP_TRY(hipGetLastError());
        s0 = s1;
    }
    return EIG_OK;
}

static int upload_small(eig_ctx* c, size_t off, const void* p, size_t bytes, hipStream_t s) {
    std::vector<char> v(bytes);
    std::memcpy(v.data(), p, bytes);
    return upload(c, c->ws + off, v, s);
}

static int check_prior(const eig_prior* prior) {
    if (!prior) return set_error(EIG_EINVAL, "prior is NULL");
    if (prior->kind == EIG_PRIOR_UNIFORM) {
        for (int j = 0; j < kNT; ++j)
            if (!(prior->hi[j] > prior->lo[j])) return set_error(EIG_EINVAL, "prior box lo < hi");
    } else if (prior->kind != EIG_PRIOR_GAUSSIAN) {
        return set_error(EIG_EINVAL, "prior kind");
    }
    return EIG_OK;
}

int laplace_eig(eig_ctx* c, int32_t nsample, const double* H1, const eig_prior* prior,
                const double* theta, const double* w, double* dkl, double* logdet,
                double* eig, int32_t* status, void* stream) {
    if (!c) return set_error(EIG_EINVAL, "ctx is NULL");
    if (nsample <= 0 || !H1 || !w || !dkl || !eig)
        return set_error(EIG_EINVAL, "laplace_eig arguments");
    int rc = check_prior(prior);
    if (rc) return rc;
    if (prior->kind == EIG_PRIOR_GAUSSIAN && !theta)
        return set_error(EIG_EINVAL, "gaussian prior needs theta");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Carve cv;
    const size_t o_pr = cv.take(sizeof(eig_prior));
    const size_t o_th = cv.take((size_t)nsample * kNT * sizeof(double));
    const size_t o_w = cv.take((size_t)nsample * sizeof(double));
    rc = ensure_ws(c, cv.off);
    if (rc) return rc;
    std::vector<double> th((size_t)nsample * kNT, 0.0);
    if (theta) std::memcpy(th.data(), theta, th.size() * sizeof(double));
    if ((rc = upload_small(c, o_pr, prior, sizeof(eig_prior), s))) return rc;
    if ((rc = upload_small(c, o_th, th.data(), th.size() * sizeof(double), s))) return rc;
    if ((rc = upload_small(c, o_w, w, (size_t)nsample * sizeof(double), s))) return rc;
    launch_laplace(H1, nsample, (const eig_prior*)(c->ws + o_pr), (const double*)(c->ws + o_th),
                   (const double*)(c->ws + o_w), dkl, logdet, status, eig, s);
    HIP_TRY(hipGetLastError());
    return EIG_OK;
}

int design_eval(eig_ctx* c, int32_t nsample, int32_t ncand, const double* H1r,
                int32_t ndesign, const uint8_t* mask, const eig_prior* prior,
                const double* theta, const double* w, double* eig, void* stream) {
    if (!c) return set_error(EIG_EINVAL, "ctx is NULL");
    if (nsample <= 0 || ncand <= 0 || ndesign <= 0 || !H1r || !mask || !w || !eig)
        return set_error(EIG_EINVAL, "design_eval arguments");
    int rc = check_prior(prior);
    if (rc) return rc;
    if (prior->kind == EIG_PRIOR_GAUSSIAN && !theta)
        return set_error(EIG_EINVAL, "gaussian prior needs theta");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Carve cv;
    const size_t o_pr = cv.take(sizeof(eig_prior));
    const size_t o_th = cv.take((size_t)nsample * kNT * sizeof(double));
    const size_t o_w = cv.take((size_t)nsample * sizeof(double));
    const size_t o_work = cv.take((size_t)nsample * ndesign * sizeof(double));
    rc = ensure_ws(c, cv.off);
    if (rc) return rc;
    std::vector<double> th((size_t)nsample * kNT, 0.0);
    if (theta) std::memcpy(th.data(), theta, th.size() * sizeof(double));
    if ((rc = upload_small(c, o_pr, prior, sizeof(eig_prior), s))) return rc;
    if ((rc = upload_small(c, o_th, th.data(), th.size() * sizeof(double), s))) return rc;
    if ((rc = upload_small(c, o_w, w, (size_t)nsample * sizeof(double), s))) return rc;
    launch_design_eval(H1r, nsample, ncand, mask, ndesign, (const eig_prior*)(c->ws + o_pr),
                       (const double*)(c->ws + o_th), (const double*)(c->ws + o_w),
                       (double*)(c->ws + o_work), eig, s);
    HIP_TRY(hipGetLastError());
    return EIG_OK;
}

int design_greedy(eig_ctx* c, int32_t nsample, int32_t ncand, const double* H1r,
                  const eig_prior* prior, const double* theta, const double* w,
                  int32_t kmax, int32_t* order, double* curve, void* stream) {
    if (!c) return set_error(EIG_EINVAL, "ctx is NULL");
    if (nsample <= 0 || ncand <= 0 || kmax <= 0 || !H1r || !w || !order || !curve)
        return set_error(EIG_EINVAL, "design_greedy arguments");
    int rc = check_prior(prior);
    if (rc) return rc;
    if (prior->kind == EIG_PRIOR_GAUSSIAN && !theta)
        return set_error(EIG_EINVAL, "gaussian prior needs theta");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    Carve cv;
    const size_t o_pr = cv.take(sizeof(eig_prior));
    const size_t o_th = cv.take((size_t)nsample * kNT * sizeof(double));
    const size_t o_w = cv.take((size_t)nsample * sizeof(double));
    const size_t o_work = cv.take((size_t)nsample * ncand * sizeof(double));
    const size_t o_ival = cv.take((size_t)ncand * sizeof(double));
    const size_t o_H = cv.take((size_t)nsample * kNT * kNT * sizeof(double));
    const size_t o_ch = cv.take((size_t)ncand);
    rc = ensure_ws(c, cv.off);
    if (rc) return rc;
    std::vector<double> th((size_t)nsample * kNT, 0.0);
    if (theta) std::memcpy(th.data(), theta, th.size() * sizeof(double));
    if ((rc = upload_small(c, o_pr, prior, sizeof(eig_prior), s))) return rc;
    if ((rc = upload_small(c, o_th, th.data(), th.size() * sizeof(double), s))) return rc;
    if ((rc = upload_small(c, o_w, w, (size_t)nsample * sizeof(double), s))) return rc;
    launch_fill_zero(c->ws + o_H, (size_t)nsample * kNT * kNT * sizeof(double), s);
    launch_fill_zero(c->ws + o_ch, (size_t)ncand, s);
    for (int k = 0; k < kmax; ++k)
        launch_greedy_step(H1r, nsample, ncand, (const eig_prior*)(c->ws + o_pr),
                           (const double*)(c->ws + o_th), (const double*)(c->ws + o_w),
                           (double*)(c->ws + o_H), (uint8_t*)(c->ws + o_ch),
                           (double*)(c->ws + o_work), (double*)(c->ws + o_ival), k, order,
                           curve, s);
    HIP_TRY(hipGetLastError());
    return EIG_OK;
}

int noise_sigma_peak(eig_ctx* c, const eig_grid* grid, const eig_medium* medium,
                     const double* theta, int32_t stf_kind, double rel, double* sigma_out,
                     void* stream) {
    if (!c || !grid || !medium || !theta || !sigma_out || !(rel > 0))
        return set_error(EIG_EINVAL, "noise_sigma_peak arguments");
    if (!valid_grid(*grid)) return set_error(EIG_EINVAL, "grid");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    const int nrec = grid->nx - 2;
    std::vector<int32_t> ix(nrec);
    for (int r = 0; r < nrec; ++r) ix[r] = r + 1;
    eig_receivers rv{nrec, ix.data()};
    const size_t tbytes = (size_t)(grid->nsteps + 1) * nrec * sizeof(float2);
    float2* tr = nullptr;
    double* dout = nullptr;
    HIP_TRY(hipMalloc((void**)&tr, tbytes));
    if (hipMalloc((void**)&dout, sizeof(double)) != hipSuccess) {
        (void)hipFree(tr);
        return set_error(EIG_ENOMEM, "hipMalloc");
    }
    float* tp = (float*)tr;
    int rc = forward_solve_batch(c, 1, grid, medium, theta, nullptr, nullptr, stf_kind, &rv,
                                 &tp, stream);
    if (rc == EIG_OK) {
        launch_surface_peak(tr, (grid->nsteps + 1) * nrec, rel, dout, s);
        if (hipMemcpyAsync(sigma_out, dout, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            rc = set_error(EIG_EHIP, "noise_sigma_peak copy");
    }
    (void)hipFree(tr);
    (void)hipFree(dout);
    return rc;
}

}  // extern "C"
