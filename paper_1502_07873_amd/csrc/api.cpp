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
#include <cstdlib>
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

#include "host.h"

namespace {

int run_chunk(eig_ctx* c, const std::vector<SolveSpec>& solves,
              const std::vector<eig_grid>& grids, const std::vector<MediumKey>& media,
              const std::vector<RecSet>& recsets, char* base, size_t cap, hipStream_t s,
              bool allow_graph);

// A solve whose two field levels fit one workgroup's LDS runs resident
// (variants 21, 22: its whole time loop in one launch, fields never in HBM),
// unless that is switched off or a tiled variant is forced.
bool resident_ok(const eig_ctx* c, const eig_grid& g, int kind) {
    if (!c->resident) return false;
    if (c->forced_variant >= 0 && !kVariants[c->forced_variant].resident) return false;
    return resident_lds_bytes(kind, g.nx, g.nz) <= kResidentLdsBytes &&
           2 * g.nz + g.nx - 2 <= kResidentMaxEdge;
}
// Steps a resident launch stands for in the launch-count arithmetic: above
// any grid's nsteps (valid grids have nsteps < 2^28).
constexpr int kResidentSpan = 1 << 28;

// Leapfrog steps per launch of the kernels a solve class runs: absorbing
// edges and dual solves one; depth-only media temporal_blocking (1, 2, 3 or
// 4); nodal media two unless temporal_blocking is 1 or 4.
int family_steps_of(const eig_ctx* c, int kind, bool one_step) {
    if (one_step) return 1;
    if (kind == EIG_MEDIUM_LAYERED || c->temporal_blocking == 4) return c->temporal_blocking;
    return std::min(c->temporal_blocking, 2);
}

// Leapfrog steps per launch of a tiled solve (a forced variant's, else its
// family's).
int tiled_steps_of(const eig_ctx* c, const SolveSpec& sp, const eig_grid& g,
                   const MediumKey& mk) {
    const bool one_step = g.bc == EIG_BC_ABSORBING || sp.rforce != nullptr;
    int steps = family_steps_of(c, mk.kind, one_step);
    if (c->forced_variant >= 0 && kVariants[c->forced_variant].medium_kind == mk.kind &&
        !kVariants[c->forced_variant].resident &&
        !(one_step && kVariants[c->forced_variant].steps != 1))
        steps = kVariants[c->forced_variant].steps;
    return steps;
}

// Field bytes one solve keeps live from launch to launch: four buffers when
// a solve with rigid edges advances several steps per launch, two
// otherwise.
size_t live_field_bytes(const eig_ctx* c, const SolveSpec& sp, const eig_grid& g,
                        const MediumKey& mk) {
    if (resident_ok(c, g, mk.kind)) return 0;  // fields in LDS
    const size_t field = (size_t)g.nz * pitch_of(g.nx) * sizeof(float2);
    return (tiled_steps_of(c, sp, g, mk) >= 2 ? 4 : 2) * field;
}

// A wave's solves advance together, but not necessarily in one set of
// launches.  When their live fields exceed wave_cache_bytes (sized to the
// device's last-level cache), the wave runs as consecutive chunks of about
// that many bytes each, so that every chunk's fields stay in that cache from
// one launch to the next instead of streaming through HBM; the chunks reuse
// the same workspace in stream order.  For the split the solves are ordered
// by kind, grid and length, so that each chunk is one or two uniform groups
// of launches.  Waves where fewer than cache_chunk_min_solves solves would
// fit are not split for the cache (too few tiles per launch to pay).  Solves
// that take four steps per launch with the tile in LDS move a quarter of the
// two-step kernels' field bytes per step and run faster as one wave through
// HBM (all their tiles in every launch) than in cache-sized chunks, so their
// fields do not count towards the limit.  A chunk also holds at most
// max_wave_solves solves when that is set.

int run_wave(eig_ctx* c, const std::vector<SolveSpec>& solves,
             const std::vector<eig_grid>& grids, const std::vector<MediumKey>& media,
             const std::vector<RecSet>& recsets, char* base, size_t cap, hipStream_t s) {
    const size_t n = solves.size();
    if (n == 0) return EIG_OK;
    std::vector<size_t> live(n), order(n);
    double total = 0.0;
    for (size_t i = 0; i < n; ++i) {
        const SolveSpec& sp = solves[i];
        const eig_grid& g = grids[sp.grid];
        const MediumKey& mk = media[sp.medium];
        live[i] = tiled_steps_of(c, sp, g, mk) == 4 ? 0 : live_field_bytes(c, sp, g, mk);
        total += (double)live[i];
        order[i] = i;
    }
    // chunk boundaries: every change of kind, edges, grid or length (so a
    // chunk is uniform and its tuned variant suits the chunks that share its
    // tuning key), and within a uniform segment its live bytes cut into
    // equal spans of at most the limit
    std::vector<size_t> cut{0};
    const double lim = (double)c->wave_cache_bytes;
    if (lim > 0 && total > lim && (double)c->cache_chunk_min_solves * total / (double)n <= lim) {
        auto key = [&](size_t i) {
            const SolveSpec& sp = solves[i];
            const eig_grid& g = grids[sp.grid];
            return std::make_tuple(media[sp.medium].kind, g.bc, sp.rforce != nullptr, g.nx,
                                   g.nz, -g.nsteps, sp.medium);
        };
        auto uniform = [&](size_t a, size_t b) {
            const auto ka = key(a), kb = key(b);
            return std::get<0>(ka) == std::get<0>(kb) && std::get<1>(ka) == std::get<1>(kb) &&
                   std::get<2>(ka) == std::get<2>(kb) && std::get<3>(ka) == std::get<3>(kb) &&
                   std::get<4>(ka) == std::get<4>(kb) && std::get<5>(ka) == std::get<5>(kb);
        };
        std::stable_sort(order.begin(), order.end(),
                         [&](size_t a, size_t b) { return key(a) < key(b); });
        size_t q0 = 0;
        while (q0 < n) {
            size_t q1 = q0 + 1;
            double seg = (double)live[order[q0]];
            while (q1 < n && uniform(order[q0], order[q1])) seg += (double)live[order[q1++]];
            const size_t nch = std::max<size_t>(1, (size_t)std::ceil(seg / lim));
            const double span = seg / (double)nch;
            double acc = 0.0;
            size_t made = 1;
            for (size_t q = q0; q < q1; ++q) {
                const double b = (double)live[order[q]];
                if (q > cut.back() && acc + 0.5 * b > span * (double)made) {
                    cut.push_back(q);
                    ++made;
                }
                acc += b;
            }
            if (q1 < n) cut.push_back(q1);
            q0 = q1;
        }
    }
    cut.push_back(n);
    std::vector<std::pair<size_t, size_t>> parts;
    const size_t per = c->max_wave_solves > 0 ? (size_t)c->max_wave_solves : n;
    for (size_t k = 0; k + 1 < cut.size(); ++k)
        for (size_t q0 = cut[k]; q0 < cut[k + 1]; q0 += per)
            parts.push_back({q0, std::min(cut[k + 1], q0 + per)});
    // captured time loops are cached eight at a time: a wave of more chunks
    // could never replay them
    const bool allow_graph = parts.size() <= 8;
    std::vector<SolveSpec> part;
    for (const auto& pr : parts) {
        part.clear();
        for (size_t q = pr.first; q < pr.second; ++q) part.push_back(solves[order[q]]);
        const int rc = run_chunk(c, part, grids, media, recsets, base, cap, s, allow_graph);
        if (rc) return rc;
    }
    return EIG_OK;
}

size_t tiles_of(const eig_grid& g, const StencilVariant& v) {
    if (v.resident) return 1;  // one workgroup per solve
    return (size_t)((g.nx + v.cols - 1) / v.cols) * ((g.nz - 1 + v.rows - 1) / v.rows);
}

// Variants a wave may run for a medium kind: the forced one, else all of
// that kind (tuned online per grid class).  Grids with absorbing edges run
// one step per launch (their edge nodes are updated between steps).
void stencil_candidates(const eig_ctx* c, int kind, bool one_step, std::vector<int>& out) {
    out.clear();
    if (c->forced_variant >= 0 && kVariants[c->forced_variant].medium_kind == kind &&
        !kVariants[c->forced_variant].resident &&
        !(one_step && kVariants[c->forced_variant].steps != 1)) {
        out.push_back(c->forced_variant);
        return;
    }
    // one family per wave: two or three steps per launch (four field
    // buffers) or one
    const int steps = family_steps_of(c, kind, one_step);
    for (int v = 1; v < kNumVariants; ++v)
        if (kVariants[v].medium_kind == kind && kVariants[v].steps == steps &&
            !kVariants[v].resident && !kVariants[v].forced_only)
            out.push_back(v);
    if (out.empty()) out.push_back(kind == EIG_MEDIUM_NODAL ? 6 : 0);
    if (!c->autotune) {
        const int want = steps == 3 ? c->default_variant_tb3
                                    : (steps == 2 ? c->default_variant_tb : c->default_variant);
        int keep = out[0];
        for (int v : out)
            if (v == want) keep = v;
        out.assign(1, keep);
    }
}

// Run a set of solves that fits the workspace region [base, base+cap).
int run_chunk(eig_ctx* c, const std::vector<SolveSpec>& solves,
             const std::vector<eig_grid>& grids, const std::vector<MediumKey>& media,
             const std::vector<RecSet>& recsets, char* base, size_t cap,
             hipStream_t s, bool allow_graph) {
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
    // stencil variants this wave may use, per solve class (medium kind,
    // absorbing edges, dual solve): the last two need one step per launch
    std::vector<int> cands[2][2];
    for (int kind = 0; kind < 2; ++kind)
        for (int one = 0; one < 2; ++one) stencil_candidates(c, kind, one != 0, cands[kind][one]);
    auto one_step = [&](int i) {
        return grids[solves[i].grid].bc == EIG_BC_ABSORBING || solves[i].rforce != nullptr;
    };
    // grids that fit one workgroup's LDS run resident (variants 21, 22)
    static const std::vector<int> res_cand[2] = {{21}, {22}};
    std::vector<char> res(n);
    for (int i = 0; i < n; ++i)
        res[i] = resident_ok(c, grids[solves[i].grid], media[solves[i].medium].kind);
    auto cand_of = [&](int i) -> const std::vector<int>& {
        if (res[i]) return res_cand[media[solves[i].medium].kind];
        return cands[media[solves[i].medium].kind][one_step(i) ? 1 : 0];
    };
    auto family_steps = [&](int i) { return kVariants[cand_of(i)[0]].steps; };
    // fields: one contiguous block for all solves (cleared with one launch);
    // two-steps-per-launch kernels rotate over four buffers per solve
    std::vector<size_t> f0(n), f1(n), f2(n, 0), f3(n, 0), sw(n), ss(n);
    const size_t fields_begin = align_up(cv.off);
    cv.off = fields_begin;
    for (int i = 0; i < n; ++i) {
        if (res[i]) continue;  // fields in LDS only
        const eig_grid& g = grids[solves[i].grid];
        const size_t field = (size_t)g.nz * pitch_of(g.nx) * sizeof(float2);
        f0[i] = cv.take(field);
        f1[i] = cv.take(field);
        if (family_steps(i) >= 2) {
            f2[i] = cv.take(field);
            f3[i] = cv.take(field);
        }
    }
    const size_t fields_end = cv.off;
    // three-steps-per-launch halo side buffers (written before every read)
    auto nbound = [&](const eig_grid& g) { return (g.nx + 127) / 128 - 1; };
    std::vector<size_t> side_off(n, 0);
    for (int i = 0; i < n; ++i) {
        const eig_grid& g = grids[solves[i].grid];
        if (family_steps(i) == 3 && nbound(g) > 0)
            side_off[i] = cv.take((size_t)nbound(g) * g.nz * 4 * sizeof(float2));
    }
    for (int i = 0; i < n; ++i) {
        const eig_grid& g = grids[solves[i].grid];
        sw[i] = cv.take(2 * kSrcW * kSrcW * sizeof(float));
        ss[i] = cv.take((size_t)std::max(g.nsteps, 1) * sizeof(float));
    }
    // order: solve class (medium kind, edges), then steps descending
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    auto class_of = [&](int i) {
        return 8 * res[i] + 4 * media[solves[i].medium].kind +
               2 * (solves[i].rforce != nullptr) + grids[solves[i].grid].bc;
    };
    std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
        const int ka = class_of(a), kb = class_of(b);
        if (ka != kb) return ka < kb;
        return grids[solves[a].grid].nsteps > grids[solves[b].grid].nsteps;
    });
    // the staging blob (receiver maps, descriptors, tile maps, forcing jobs)
    // gets its device place first so descriptors can point into it
    size_t ntiles_total = 0;
    for (int i = 0; i < n; ++i) {
        const eig_grid& g = grids[solves[i].grid];
        for (int v : cand_of(i)) {
            ntiles_total += tiles_of(g, kVariants[v]);
            if (kVariants[v].edges) ntiles_total += edge_tiles_of(g.nx, g.nz);
            if (kVariants[v].steps == 3)
                ntiles_total += (size_t)std::max(nbound(g), 0) * ((g.nz - 1 + 63) / 64);
        }
    }
    // one aligned piece per descriptor table, job table, receiver map and
    // (halo) tile map: at most 4 solve classes x 2 maps x every variant
    const size_t npieces = 4 + 8 * (size_t)kNumVariants;
    size_t blob_bound = align_up((size_t)n * sizeof(SolveDesc)) +
                        align_up(ntiles_total * sizeof(int2)) + npieces * kAlign +
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
    // descriptors, and per medium kind a group of solves with one tile map
    // per candidate variant
    std::vector<SolveDesc> desc(n);
    std::vector<SourceJob> jobs(n);
    struct Group {
        int kind, bc, cls;
        int first, last;               // solve range in launch order
        size_t lds = 0;                // resident groups: dynamic LDS bytes
        std::vector<int> cand;         // candidate variants
        std::vector<std::vector<int2>> tiles;                     // per candidate
        std::vector<std::vector<std::pair<int, int>>> steps_tiles;  // per candidate
        std::vector<std::vector<int2>> htiles;                    // three-step halo
        std::vector<std::vector<std::pair<int, int>>> steps_htiles;
    };
    std::vector<Group> groups;
    for (int oi = 0; oi < n; ++oi) {
        const int i = ord[oi];
        const SolveSpec& sp = solves[i];
        const eig_grid& g = grids[sp.grid];
        const MediumKey& mk = media[sp.medium];
        SolveDesc& d = desc[oi];
        d.buf0 = res[i] ? nullptr : (float2*)(base + f0[i]);
        d.buf1 = res[i] ? nullptr : (float2*)(base + f1[i]);
        d.buf2 = f2[i] ? (float2*)(base + f2[i]) : nullptr;
        d.buf3 = f3[i] ? (float2*)(base + f3[i]) : nullptr;
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
        d.medium_kind = mk.kind;
        d.h2 = (float)(g.h * g.h);
        d.rforce = sp.rforce;
        d.wrec = sp.wrec;
        d.side = side_off[i] ? (float2*)(base + side_off[i]) : nullptr;
        // forcing window: union of the nominal and perturbed 6x6 stencils
        SourceJob& J = jobs[oi];
        std::memcpy(J.theta, sp.theta, sizeof(J.theta));
        J.step = sp.step;
        J.h = g.h;
        J.dt = g.dt;
        J.param = sp.param;
        J.deriv = sp.deriv;
        J.kx = floor_cell(sp.theta[0], g.h);
        J.kz = floor_cell(sp.theta[1], g.h);
        double tp[kNT];
        std::memcpy(tp, sp.theta, sizeof(tp));
        if (sp.param >= 0 && !sp.deriv) tp[sp.param] = sp.theta[sp.param] + sp.step;
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
        if (groups.empty() || groups.back().cls != class_of(i)) {
            Group gr;
            gr.kind = mk.kind;
            gr.bc = g.bc;
            gr.cls = class_of(i);
            gr.first = oi;
            gr.cand = cand_of(i);
            gr.tiles.resize(gr.cand.size());
            gr.steps_tiles.resize(gr.cand.size());
            gr.htiles.resize(gr.cand.size());
            gr.steps_htiles.resize(gr.cand.size());
            groups.push_back(gr);
        }
        Group& gr = groups.back();
        gr.last = oi + 1;
        for (size_t v = 0; v < gr.cand.size(); ++v) {
            const StencilVariant& sv = kVariants[gr.cand[v]];
            if (sv.resident) {
                gr.tiles[v].push_back(make_int2(oi, g.bc == EIG_BC_ABSORBING ? 1 : 0));
                gr.steps_tiles[v].push_back({g.nsteps, (int)gr.tiles[v].size()});
                gr.lds = std::max(gr.lds, resident_lds_bytes(mk.kind, g.nx, g.nz));
                continue;
            }
            const int nstrip = (g.nx + sv.cols - 1) / sv.cols;
            const int nchunk = (g.nz - 1 + sv.rows - 1) / sv.rows;
            for (int ch = 0; ch < nchunk; ++ch)
                for (int st = 0; st < nstrip; ++st)
                    gr.tiles[v].push_back(make_int2(oi, (st << 16) | ch));
            if (sv.edges && g.bc == EIG_BC_ABSORBING && c->fused_edges)
                for (int part = 0; part < edge_tiles_of(g.nx, g.nz); ++part)
                    gr.tiles[v].push_back(make_int2(oi, (kEdgeStrip << 16) | part));
            gr.steps_tiles[v].push_back({g.nsteps, (int)gr.tiles[v].size()});
            if (sv.steps == 3) {
                const int nhch = (g.nz - 1 + 63) / 64;
                for (int bi = 0; bi < nbound(g); ++bi)
                    for (int ch = 0; ch < nhch; ++ch)
                        gr.htiles[v].push_back(make_int2(oi, (bi << 16) | ch));
                gr.steps_htiles[v].push_back({g.nsteps, (int)gr.htiles[v].size()});
            }
        }
    }
    // Nodal media: the kernels read 12 B of coefficients per node for every
    // solve.  Within a set of up to coef_interleave consecutive solves on one
    // medium and grid, order the tiles by position first and solve second,
    // so that the solves' tiles at one position run together and share the
    // coefficient rows in L2.  Tiles of one launch are independent, so the
    // order changes no result; members of a set share nsteps, so running
    // solves still form a prefix of whole sets.
    if (c->coef_interleave > 1)
        for (Group& gr : groups) {
            if (gr.kind != EIG_MEDIUM_NODAL) continue;
            for (size_t v = 0; v < gr.cand.size(); ++v) {
                auto& tv = gr.tiles[v];
                auto& stv = gr.steps_tiles[v];
                std::vector<int2> out;
                out.reserve(tv.size());
                int q = 0;
                const int nq = (int)stv.size();
                while (q < nq) {
                    const SolveDesc& a = desc[gr.first + q];
                    int e = q + 1;
                    while (e < nq && e - q < c->coef_interleave) {
                        const SolveDesc& b = desc[gr.first + e];
                        if (b.coef != a.coef || b.nx != a.nx || b.nz != a.nz ||
                            b.nsteps != a.nsteps)
                            break;
                        ++e;
                    }
                    const int lo = q ? stv[q - 1].second : 0;
                    const int per = stv[q].second - lo;  // equal for all members
                    for (int t = 0; t < per; ++t)
                        for (int r = q; r < e; ++r) out.push_back(tv[lo + (r - q) * per + t]);
                    for (int r = q; r < e; ++r) stv[r].second = (int)out.size();
                    q = e;
                }
                tv.swap(out);
            }
        }
    const size_t o_desc = blob.put(desc.data(), desc.size() * sizeof(SolveDesc));
    std::vector<std::vector<size_t>> o_tiles(groups.size()), o_htiles(groups.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        for (auto& tv : groups[gi].tiles)
            o_tiles[gi].push_back(blob.put(tv.data(), tv.size() * sizeof(int2)));
        for (auto& hv : groups[gi].htiles)
            o_htiles[gi].push_back(hv.empty() ? 0 : blob.put(hv.data(), hv.size() * sizeof(int2)));
    }
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
    // launches: ceil(steps / steps-per-launch) per group
    int max_steps = 0;
    for (const auto& g : groups) {
        const int spl = kVariants[g.cand[0]].resident ? kResidentSpan : kVariants[g.cand[0]].steps;
        for (const auto& st : g.steps_tiles[0])
            max_steps = std::max(max_steps, (st.first + spl - 1) / spl);
    }
    // per group: variant in use, and an online tuning window if this grid
    // class has not been tuned yet (the tuning launches are real steps)
    struct Tune {
        bool active = false;
        int begin = 0, reps = 4;
        std::vector<hipEvent_t> ev;  // 2 per tuning launch
        std::tuple<int, int, int, int, int> key;
    };
    std::vector<int> use(groups.size(), 0);
    std::vector<Tune> tune(groups.size());
    for (size_t gi = 0; gi < groups.size(); ++gi) {
        Group& g = groups[gi];
        const SolveDesc& d0 = desc[g.first];
        // grid class and batch size (log2 of the solve count) both matter
        int bucket = 0;
        while ((2 << bucket) <= g.last - g.first) ++bucket;
        tune[gi].key = std::make_tuple(g.cls, d0.nx, d0.nz, kVariants[g.cand[0]].steps, bucket);
        use[gi] = 0;
        if (g.cand.size() > 1) {
            auto it = c->tuned.find(tune[gi].key);
            if (it != c->tuned.end() &&
                std::find(g.cand.begin(), g.cand.end(), it->second) != g.cand.end()) {
                for (size_t v = 0; v < g.cand.size(); ++v)
                    if (g.cand[v] == it->second) use[gi] = (int)v;
            } else {
                const int need = 1 + (int)g.cand.size() * tune[gi].reps;
                for (size_t v = 0; v < g.cand.size(); ++v)
                    if (g.cand[v] == c->default_variant || g.cand[v] == c->default_variant_tb)
                        use[gi] = (int)v;
                if (max_steps >= need) {
                    tune[gi].active = true;
                    tune[gi].begin = 1;
                    tune[gi].ev.resize(2 * g.cand.size() * tune[gi].reps);
                    for (auto& e : tune[gi].ev) HIP_TRY(hipEventCreate(&e));
                }
            }
        }
    }
    // graph capture: only without an open tuning window (no events inside)
    bool any_tuning = false;
    for (const auto& tn : tune) any_tuning = any_tuning || tn.active;
    const bool use_graph = c->graphs && allow_graph && !any_tuning && max_steps > 0;
    std::tuple<uint64_t, uintptr_t, size_t> gkey{0, 0, 0};
    hipGraphExec_t gexec = nullptr;
    bool capturing = false;
    if (use_graph) {
        uint64_t hsh = 1469598103934665603ull;   // FNV-1a over the blob and the variants
        for (char ch : blob.data) hsh = (hsh ^ (uint8_t)ch) * 1099511628211ull;
        for (int u : use) hsh = (hsh ^ (uint64_t)(u + 1)) * 1099511628211ull;
        gkey = std::make_tuple(hsh, (uintptr_t)bd, blob.data.size());
        auto it = c->graph_cache.find(gkey);
        if (it != c->graph_cache.end()) {
            gexec = it->second;
        } else {
            if (!c->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&c->capture_stream,
                                                                      hipStreamNonBlocking));
            capturing = hipStreamBeginCapture(c->capture_stream,
                                              hipStreamCaptureModeThreadLocal) == hipSuccess;
        }
    }
    const bool replay = gexec != nullptr;
    hipStream_t ls = capturing ? c->capture_stream : s;   // where launches go
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (max_steps > 0) {
        HIP_TRY(hipEventCreate(&ev0));
        HIP_TRY(hipEventCreate(&ev1));
        HIP_TRY(hipEventRecord(ev0, s));
    }
    for (int step = 0; step < max_steps; ++step) {
        for (size_t gi = 0; gi < groups.size(); ++gi) {
            Group& g = groups[gi];
            Tune& tn = tune[gi];
            int vi = use[gi];
            int slot = -1;
            const int ncand = (int)g.cand.size();
            if (tn.active && step >= tn.begin && step < tn.begin + ncand * tn.reps) {
                slot = step - tn.begin;
                vi = slot % ncand;
            }
            // running solves form a prefix (steps descending within a group);
            // a resident group takes all its steps in the first launch
            const bool resident = kVariants[g.cand[vi]].resident != 0;
            if (resident && step > 0) continue;
            const int spl = resident ? kResidentSpan : kVariants[g.cand[vi]].steps;
            int ntile = 0, nrun = 0;
            double upd = 0.0;
            const auto& stv = g.steps_tiles[vi];
            for (size_t q = 0; q < stv.size(); ++q) {
                if (stv[q].first > step * spl) {
                    ntile = stv[q].second;
                    nrun = (int)q + 1;
                    const SolveDesc& dq = desc[g.first + q];
                    upd += (double)dq.nx * dq.nz * std::min(spl, stv[q].first - step * spl);
                } else {
                    break;
                }
            }
            if (ntile > 0) {
                c->last_variant = g.cand[vi];
                if (slot >= 0) HIP_TRY(hipEventRecord(tn.ev[2 * slot], s));
                if (spl == 3 && !replay) {
                    int nh = 0;
                    for (const auto& hs : g.steps_htiles[vi]) {
                        if (hs.first > step * spl) nh = hs.second;
                        else break;
                    }
                    launch_tb3_halo(ddesc, (const int2*)(bd + o_htiles[gi][vi]), nh, step, ls);
                }
                if (!replay && resident)
                    launch_resident(ddesc, (const int2*)(bd + o_tiles[gi][vi]), ntile, g.kind,
                                    g.lds, ls);
                else if (!replay)
                    launch_stencil(ddesc, (const int2*)(bd + o_tiles[gi][vi]), ntile, step,
                                   g.cand[vi], ls);
                if (slot >= 0) HIP_TRY(hipEventRecord(tn.ev[2 * slot + 1], s));
                if (g.bc == EIG_BC_ABSORBING && !replay && !resident &&
                    !(kVariants[g.cand[vi]].edges && c->fused_edges))
                    launch_ce_edges(ddesc + g.first, nrun, step, ls);
                c->launches += 1;
                c->updates += upd;
                c->bytes += upd * (g.kind == EIG_MEDIUM_NODAL ? 36.0 : 24.0);
            }
            if (slot == ncand * tn.reps - 1) {
                // end of the tuning window: pick the fastest variant
                HIP_TRY(hipEventSynchronize(tn.ev.back()));
                // each candidate's fastest launch: robust to a launch slowed
                // by something else on the device
                std::vector<double> tot(ncand, 1e30);
                for (int q = 0; q < ncand * tn.reps; ++q) {
                    float ms = 0.f;
                    HIP_TRY(hipEventElapsedTime(&ms, tn.ev[2 * q], tn.ev[2 * q + 1]));
                    tot[q % ncand] = std::min(tot[q % ncand], (double)ms);
                }
                int best = 0;
                for (int v = 1; v < ncand; ++v)
                    if (tot[v] < tot[best]) best = v;
                use[gi] = best;
                c->tuned[tn.key] = g.cand[best];
                for (auto& e : tn.ev) (void)hipEventDestroy(e);
                tn.ev.clear();
                tn.active = false;
            }
        }
    }
    if (capturing) {
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(c->capture_stream, &graph);
        if (e == hipSuccess && graph) {
            e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
        }
        if (e != hipSuccess || !gexec) {
            (void)hipGetLastError();
            return set_error(EIG_EHIP, "graph capture of the time loop failed");
        }
        if (c->graph_order.size() >= 8) {   // keep the eight most recent graphs
            auto old_key = c->graph_order.front();
            c->graph_order.erase(c->graph_order.begin());
            auto it = c->graph_cache.find(old_key);
            if (it != c->graph_cache.end()) {
                (void)hipGraphExecDestroy(it->second);
                c->graph_cache.erase(it);
            }
        }
        c->graph_cache[gkey] = gexec;
        c->graph_order.push_back(gkey);
        c->graph_captures += 1;
    } else if (replay) {
        c->graph_replays += 1;
    }
    if (gexec) HIP_TRY(hipGraphLaunch(gexec, s));
    if (max_steps > 0) {
        HIP_TRY(hipEventRecord(ev1, s));
        c->timing.push_back({ev0, ev1});
    }
    for (auto& tn : tune)
        for (auto& e : tn.ev) (void)hipEventDestroy(e);
    HIP_TRY(hipGetLastError());
    return EIG_OK;
}

// Incremental upper bound of the workspace a wave needs.
struct WaveSizer {
    const std::vector<eig_grid>& grids;
    const std::vector<MediumKey>& media;
    const std::vector<RecSet>& recsets;
    std::vector<char> med_seen, rec_seen;
    size_t bytes = (64 + 8 * kNumVariants) * kAlign;
    WaveSizer(const std::vector<eig_grid>& g, const std::vector<MediumKey>& m,
              const std::vector<RecSet>& r)
        : grids(g), media(m), recsets(r), med_seen(m.size(), 0), rec_seen(r.size(), 0) {}
    size_t cost(const SolveSpec& sp) const {
        const eig_grid& g = grids[sp.grid];
        size_t b = solve_bytes(g) + sizeof(SolveDesc) + sizeof(SourceJob) + 64;
        for (int v = 0; v < kNumVariants; ++v)
            b += (tiles_of(g, kVariants[v]) + edge_tiles_of(g.nx, g.nz)) * sizeof(int2);
        // three-step halo: side buffer and halo tile maps (upper bound)
        const size_t nb = (size_t)(g.nx + 127) / 128;
        b += nb * g.nz * 4 * sizeof(float2) + 2 * nb * ((g.nz + 63) / 64) * sizeof(int2) + kAlign;
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
    // device address of this device's no-alloc scratch array; a failure is
    // reported by the entry point that needs it (it retries the lookup)
    (void)noalloc_scratch_init(device);
    eig_ctx* c = new eig_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes;
    if (const char* e = std::getenv("EIG_STENCIL_VARIANT")) {
        const int v = std::atoi(e);
        if (v >= 0 && v < kNumVariants) c->forced_variant = v;
    }
    if (const char* e = std::getenv("EIG_AUTOTUNE")) c->autotune = std::atoi(e) != 0;
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
    for (auto& kv : c->graph_cache) (void)hipGraphExecDestroy(kv.second);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    delete c;
}

size_t eig_ctx_workspace_bytes(const eig_ctx* c) { return c ? c->ws_size : 0; }

int eig_ctx_set_option(eig_ctx* c, const char* name, int64_t value) {
    if (!c || !name) return set_error(EIG_EINVAL, "ctx or name is NULL");
    const std::string n(name);
    if (n == "stencil_variant") {
        if (value < -1 || value >= kNumVariants) return set_error(EIG_EINVAL, "variant");
        c->forced_variant = (int)value;
    } else if (n == "autotune") {
        c->autotune = value != 0;
        if (!c->autotune) c->tuned.clear();
    } else if (n == "default_variant") {
        if (value < 0 || value >= kNumVariants || kVariants[value].resident)
            return set_error(EIG_EINVAL, "variant");
        c->default_variant = (int)value;
    } else if (n == "temporal_blocking") {
        if (value < 0 || value > 4) return set_error(EIG_EINVAL, "temporal_blocking: 0..4");
        c->temporal_blocking = value == 0 ? 1 : (value == 1 ? 2 : (int)value);
    } else if (n == "max_wave_solves") {
        if (value < 0) return set_error(EIG_EINVAL, "max_wave_solves < 0");
        c->max_wave_solves = value;
    } else if (n == "graphs") {
        c->graphs = value != 0;
    } else if (n == "serve_cache_bytes") {
        if (value < 0) return set_error(EIG_EINVAL, "serve_cache_bytes < 0");
        c->serve_cache_bytes = (size_t)value;
    } else if (n == "fused_edges") {
        c->fused_edges = value != 0;
    } else if (n == "wave_cache_bytes") {
        if (value < 0) return set_error(EIG_EINVAL, "wave_cache_bytes < 0");
        c->wave_cache_bytes = (size_t)value;
    } else if (n == "cache_chunk_min_solves") {
        if (value < 1) return set_error(EIG_EINVAL, "cache_chunk_min_solves < 1");
        c->cache_chunk_min_solves = (int)value;
    } else if (n == "coef_interleave") {
        if (value < 1 || value > 4096) return set_error(EIG_EINVAL, "coef_interleave outside 1..4096");
        c->coef_interleave = (int)value;
    } else if (n == "resident") {
        c->resident = value != 0;
    } else {
        return set_error(EIG_EINVAL, "unknown option " + n);
    }
    return EIG_OK;
}

int eig_ctx_get_option(const eig_ctx* c, const char* name, int64_t* value) {
    if (!c || !name || !value) return set_error(EIG_EINVAL, "NULL argument");
    const std::string n(name);
    if (n == "stencil_variant") *value = c->forced_variant;
    else if (n == "autotune") *value = c->autotune;
    else if (n == "default_variant") *value = c->default_variant;
    else if (n == "temporal_blocking") *value = c->temporal_blocking;
    else if (n == "max_wave_solves") *value = c->max_wave_solves;
    else if (n == "graphs") *value = c->graphs;
    else if (n == "wave_cache_bytes") *value = (int64_t)c->wave_cache_bytes;
    else if (n == "cache_chunk_min_solves") *value = c->cache_chunk_min_solves;
    else if (n == "coef_interleave") *value = c->coef_interleave;
    else if (n == "resident") *value = c->resident ? 1 : 0;
    else if (n == "fused_edges") *value = c->fused_edges;
    else if (n == "serve_cache_bytes") *value = (int64_t)c->serve_cache_bytes;
    else if (n == "graph_captures") *value = c->graph_captures;
    else if (n == "graph_replays") *value = c->graph_replays;
    else if (n == "last_variant") *value = c->last_variant;
    else return set_error(EIG_EINVAL, "unknown option " + n);
    return EIG_OK;
}

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
    // host-side argument checks first (they need no device), then the context
    if (nsolve < 0) return set_error(EIG_EINVAL, "nsolve < 0");
    if (nsolve == 0) return c ? EIG_OK : set_error(EIG_EINVAL, "ctx is NULL");
    if (!grid || !medium || !theta || !rec || !traces)
        return set_error(EIG_EINVAL, "NULL array argument");
    if (stf_kind != EIG_STF_GAUSS && stf_kind != EIG_STF_GAUSS_DERIV)
        return set_error(EIG_EINVAL, "stf_kind");
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
            if (!deviation_in_window(sp.theta[sp.param], sp.step, g.h))
                return set_error(EIG_EINVAL,
                                 "dev_step moves the source by more than one cell");
        }
        sp.stf = stf_kind;
        sp.traces = (float2*)traces[i];
        solves.push_back(sp);
    }
    if (!c) return set_error(EIG_EINVAL, "ctx is NULL");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
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

// Jacobian columns of every sample and H_1, either from 2*7 central-difference
// deviation solves (sensitivity == 0) or from 7 solves driven by dF/dtheta_j
// (sensitivity == 1); both share waves, tables, checks and the Hessian pass.
static int jacobian_core(eig_ctx* c, int32_t nsample, const eig_grid* grid,
                         const eig_medium* medium, const double* theta, double rel_step,
                         int sensitivity, int32_t stf_kind, const eig_receivers* rec,
                         int32_t sigma_mode, const double* sigma, int32_t per_receiver,
                         float* const* nominal, double* const* J, double* H1,
                         int32_t* status, void* stream) {
    // host-side argument checks first (they need no device), then the context
    if (nsample < 0) return set_error(EIG_EINVAL, "nsample < 0");
    if (nsample == 0) return c ? EIG_OK : set_error(EIG_EINVAL, "ctx is NULL");
    if (!grid || !medium || !theta || !rec || !sigma || !H1)
        return set_error(EIG_EINVAL, "NULL array argument");
    if (!sensitivity && (!(rel_step > 0) || !std::isfinite(rel_step) || rel_step > 0.1))
        return set_error(EIG_EINVAL, "rel_step must be in (0, 0.1]");
    const int per = sensitivity ? 1 + kNT : 1 + 2 * kNT;  // solves per sample
    if (stf_kind != EIG_STF_GAUSS && stf_kind != EIG_STF_GAUSS_DERIV)
        return set_error(EIG_EINVAL, "stf_kind");
    if (sigma_mode != EIG_SIGMA_GIVEN && sigma_mode != EIG_SIGMA_NOMINAL_PEAK)
        return set_error(EIG_EINVAL, "sigma_mode");
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
            if (!std::isfinite(th[j]) || (!sensitivity && th[j] == 0.0))
                return set_error(EIG_EINVAL, "theta entries must be finite and nonzero");
        }
        if (sensitivity && !source_inside(th[0], th[1], g))
            return set_error(EIG_EINVAL, "source stencil touches a rigid node");
        for (int j = 0; j < 2 && !sensitivity; ++j)
            for (int sg = -1; sg <= 1; ++sg) {
                double x = th[0], z = th[1];
                const double d = rel_step * std::fabs(th[j]);
                (j == 0 ? x : z) += sg * d;
                if (!source_inside(x, z, g))
                    return set_error(EIG_EINVAL, "source stencil touches a rigid node");
                if (!deviation_in_window(th[j], sg * d, g.h))
                    return set_error(EIG_EINVAL,
                                     "rel_step * |theta| moves the source by more than one "
                                     "cell (the forcing window covers one)");
            }
    }
    if (!c) return set_error(EIG_EINVAL, "ctx is NULL");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
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
    // bytes of one sample beyond its solves: one trace array per solve + descriptors
    auto sample_trace_bytes = [&](int i) {
        return per * align_up((size_t)(grid[i].nsteps + 1) * rec[i].n * sizeof(float2));
    };
    int s0 = 0;
    while (s0 < nsample) {
        // grow the wave sample by sample while it fits the budget
        int s1 = s0;
        size_t need = 0;
        WaveSizer wsz(grids, media, recsets);
        size_t extra = 4 * kAlign;
        size_t rstride = 0;  // per-receiver partials: doubles per sample (largest)
        while (s1 < nsample) {
            SolveSpec sp{};
            sp.grid = s1;
            sp.medium = med_of[s1];
            sp.recset = rec_of[s1];
            const size_t one = wsz.cost(sp);
            const size_t rs = per_receiver
                                  ? std::max(rstride, receiver_work_doubles(grid[s1].nsteps + 1,
                                                                            rec[s1].n))
                                  : 0;
            const size_t rwork = (size_t)(s1 - s0 + 1) * rs * sizeof(double);
            // one alignment pad each before sigma given, sigma, the partials
            // and the solve region
            const size_t more = per * one + sample_trace_bytes(s1) + sizeof(SampleDesc) +
                                4 * kAlign + 2 * sizeof(double) + sample_work_bytes(1);
            if (s1 > s0 && wsz.bytes + extra + more + rwork > c->budget) break;
            for (int q = 0; q < per; ++q) wsz.add(sp);
            extra += sample_trace_bytes(s1) + sizeof(SampleDesc) + 4 * kAlign + 2 * sizeof(double) +
                     sample_work_bytes(1);
            rstride = rs;
            need = wsz.bytes + extra + rwork;
            ++s1;
        }
        int rc = ensure_ws(c, need);
        if (rc) return rc;
        // carve: [traces | sample descs | sigma given | sigma | per-sample
        // partials | solve region]
        Carve cv;
        const int ns = s1 - s0;
        std::vector<std::array<size_t, 1 + 2 * kNT>> toff(ns);
        for (int q = 0; q < ns; ++q)
            for (int k = 0; k < per; ++k)
                toff[q][k] = cv.take((size_t)(grid[s0 + q].nsteps + 1) * rec[s0 + q].n * sizeof(float2));
        const size_t o_sd = cv.take(ns * sizeof(SampleDesc));
        const size_t o_given = cv.take(ns * sizeof(double));
        const size_t o_sig = cv.take(ns * sizeof(double));
        const size_t o_work =
            cv.take(std::max(sample_work_bytes(ns), (size_t)ns * rstride * sizeof(double)));
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
            sd.rho = medium[i].rho;
            sd.lam = medium[i].lam;
            sd.mu = medium[i].mu;
            sd.med_kind = medium[i].kind;
            sd.nx = grid[i].nx;
            sd.nz = grid[i].nz;
            sd.dt2_h2 = (grid[i].dt / grid[i].h) * (grid[i].dt / grid[i].h);
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
            for (int j = 0; j < kNT && sensitivity; ++j) {
                SolveSpec pj = sp;
                pj.param = j;
                pj.deriv = 1;
                pj.traces = (float2*)(c->ws + toff[q][1 + j]);
                sd.dev[2 * j] = pj.traces;  // dev[2j+1] stays NULL: direct column
                sd.inv2d[j] = 1.0;
                solves.push_back(pj);
            }
            for (int j = 0; j < kNT && !sensitivity; ++j) {
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
        double* dwork = (double*)(c->ws + o_work);
        launch_sample_check(dsd, ns, (const double*)(c->ws + o_given), sigma_mode, dsig,
                            status ? status + s0 : nullptr, dwork, s);
        launch_hessian(dsd, ns, per_receiver ? 1 : 0, ngroup, dsig,
                       H1 + (size_t)s0 * ngroup * kNT * kNT, dwork, s, rstride);
        HIP_TRY(hipGetLastError());
        s0 = s1;
    }
    return EIG_OK;
}

int jacobian_fd(eig_ctx* c, int32_t nsample, const eig_grid* grid,
                const eig_medium* medium, const double* theta, double rel_step,
                int32_t stf_kind, const eig_receivers* rec, int32_t sigma_mode,
                const double* sigma, int32_t per_receiver, float* const* nominal,
                double* const* J, double* H1, int32_t* status, void* stream) {
    return jacobian_core(c, nsample, grid, medium, theta, rel_step, 0, stf_kind, rec,
                         sigma_mode, sigma, per_receiver, nominal, J, H1, status, stream);
}

int jacobian_sensitivity(eig_ctx* c, int32_t nsample, const eig_grid* grid,
                         const eig_medium* medium, const double* theta, int32_t stf_kind,
                         const eig_receivers* rec, int32_t sigma_mode, const double* sigma,
                         int32_t per_receiver, float* const* nominal, double* const* J,
                         double* H1, int32_t* status, void* stream) {
    return jacobian_core(c, nsample, grid, medium, theta, 0.0, 1, stf_kind, rec, sigma_mode,
                         sigma, per_receiver, nominal, J, H1, status, stream);
}

int nested_mc_eig(eig_ctx* c, int32_t nouter, int32_t ninner, int32_t nobs,
                  const float* g_outer, const float* noise, const float* g_inner,
                  double sigma, double* logratio, double* eig, void* stream) {
    if (!c) return set_error(EIG_EINVAL, "ctx is NULL");
    if (nouter <= 0 || ninner <= 0 || nobs <= 0)
        return set_error(EIG_EINVAL, "nested_mc_eig sizes must be positive");
    if (!g_outer || !noise || !g_inner || !logratio)
        return set_error(EIG_EINVAL, "NULL array argument");
    if (!(sigma > 0) || !std::isfinite(sigma)) return set_error(EIG_EINVAL, "sigma");
    HIP_TRY(hipSetDevice(c->device));
    const int rc = ensure_ws(c, nested_workspace(nouter, ninner, nobs));
    if (rc) return rc;
    launch_nested(g_outer, noise, g_inner, nouter, ninner, nobs, sigma, logratio, eig,
                  (double*)c->ws, (hipStream_t)stream);
    HIP_TRY(hipGetLastError());
    return EIG_OK;
}

static int upload_small(eig_ctx* c, size_t off, const void* p, size_t bytes, hipStream_t s) {
    std::vector<char> v(bytes);
    std::memcpy(v.data(), p, bytes);
    return upload(c, c->ws + off, v, s);
}

static int check_prior(const eig_prior* prior) {
    if (!prior) return set_error(EIG_EINVAL, "prior is NULL");
    if (prior->active < 0 || prior->active >= (1 << kNT))
        return set_error(EIG_EINVAL, "prior active mask");
    if (prior->kind == EIG_PRIOR_UNIFORM) {
        for (int j = 0; j < kNT; ++j)
            if (!(prior->hi[j] > prior->lo[j])) return set_error(EIG_EINVAL, "prior box lo < hi");
    } else if (prior->kind != EIG_PRIOR_GAUSSIAN) {
        return set_error(EIG_EINVAL, "prior kind");
    }
    return EIG_OK;
}

// Host side of the Gauss-Newton step on the active parameters:
// (H_1 - grad grad h) step = -grad_data + grad h, through the diagonal
// scaling of Section 3.3.3.  Returns false if the system is not SPD.
static bool gn_step(const double* H1, const double* grad, const eig_prior& pr,
                    const double* th, double* step) {
    const int act = pr.active ? pr.active : (1 << kNT) - 1;
    int idx[kNT], n = 0;
    for (int j = 0; j < kNT; ++j)
        if ((act >> j) & 1) idx[n++] = j;
    double A[kNT][kNT], b[kNT];
    for (int a = 0; a < n; ++a) {
        b[a] = -grad[idx[a]];
        for (int c = 0; c < n; ++c) A[a][c] = H1[idx[a] * kNT + idx[c]];
    }
    if (pr.kind == EIG_PRIOR_GAUSSIAN) {
        // grad h = -Gamma^-1 (theta - mean), grad grad h = -Gamma^-1 (active block)
        double C[kNT][kNT], Ci[kNT][kNT];
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < n; ++c) C[a][c] = pr.cov[idx[a] * kNT + idx[c]];
        // invert C by Gauss-Jordan (n <= 7, SPD)
        double M[kNT][2 * kNT];
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < 2 * n; ++c) M[a][c] = c < n ? C[a][c] : (c - n == a ? 1.0 : 0.0);
        for (int p = 0; p < n; ++p) {
            const double d = M[p][p];
            if (!(d > 0.0)) return false;
            for (int c = 0; c < 2 * n; ++c) M[p][c] /= d;
            for (int r = 0; r < n; ++r)
                if (r != p) {
                    const double f = M[r][p];
                    for (int c = 0; c < 2 * n; ++c) M[r][c] -= f * M[p][c];
                }
        }
        for (int a = 0; a < n; ++a)
            for (int c = 0; c < n; ++c) Ci[a][c] = M[a][c + n];
        for (int a = 0; a < n; ++a) {
            double g = 0.0;
            for (int c = 0; c < n; ++c) {
                A[a][c] += Ci[a][c];
                g -= Ci[a][c] * (th[idx[c]] - pr.mean[idx[c]]);
            }
            b[a] += g;
        }
    }
    double s[kNT];
    for (int a = 0; a < n; ++a) {
        if (!(A[a][a] > 0.0) || !std::isfinite(A[a][a])) return false;
        s[a] = std::sqrt(A[a][a]);
    }
    double L[kNT][kNT];
    for (int j = 0; j < n; ++j) {
        double v = A[j][j] / (s[j] * s[j]);
        for (int k = 0; k < j; ++k) v -= L[j][k] * L[j][k];
        if (!(v > 0.0)) return false;
        L[j][j] = std::sqrt(v);
        for (int i = j + 1; i < n; ++i) {
            double w = A[i][j] / (s[i] * s[j]);
            for (int k = 0; k < j; ++k) w -= L[i][k] * L[j][k];
            L[i][j] = w / L[j][j];
        }
    }
    double y[kNT], x[kNT];
    for (int i = 0; i < n; ++i) {
        double v = b[i] / s[i];
        for (int k = 0; k < i; ++k) v -= L[i][k] * y[k];
        y[i] = v / L[i][i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double v = y[i];
        for (int k = i + 1; k < n; ++k) v -= L[k][i] * x[k];
        x[i] = v / L[i][i];
    }
    for (int j = 0; j < kNT; ++j) step[j] = 0.0;
    for (int a = 0; a < n; ++a) step[idx[a]] = x[a] / s[a];
    return true;
}

int theorem3_eig(eig_ctx* c, int32_t nsample, const eig_grid* grid, const eig_medium* medium,
                 const double* theta_star, int32_t stf_kind, const eig_receivers* rec,
                 const float* const* noise, double sigma, const eig_prior* prior,
                 const double* w, int32_t iters, double* theta_hat, double* H1out,
                 double* H2out, double* val, double* eig, int32_t* status, void* stream) {
    if (!c) return set_error(EIG_EINVAL, "ctx is NULL");
    if (nsample <= 0) return set_error(EIG_EINVAL, "nsample must be positive");
    if (!grid || !medium || !theta_star || !rec || !noise || !w || !theta_hat || !H1out ||
        !H2out || !val)
        return set_error(EIG_EINVAL, "NULL array argument");
    if (!(sigma > 0) || !std::isfinite(sigma)) return set_error(EIG_EINVAL, "sigma");
    if (iters < 0 || iters > 64) return set_error(EIG_EINVAL, "iters must be in 0..64");
    if (stf_kind != EIG_STF_GAUSS && stf_kind != EIG_STF_GAUSS_DERIV)
        return set_error(EIG_EINVAL, "stf_kind");
    int rc = check_prior(prior);
    if (rc) return rc;
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<eig_grid> grids(grid, grid + nsample);
    std::vector<MediumKey> media;
    std::map<MediumKey, int> seen;
    std::vector<RecSet> recsets;
    std::vector<int> med_of(nsample);
    for (int i = 0; i < nsample; ++i) {
        const eig_grid& g = grid[i];
        if (!valid_grid(g)) return set_error(EIG_EINVAL, "grid " + std::to_string(i));
        if (g.bc != EIG_BC_RIGID)
            return set_error(EIG_EUNSUPPORTED,
                             "theorem3_eig: the dual solve is the time-reversed stencil only "
                             "with rigid edges");
        if ((rc = validate_medium(medium[i]))) return rc;
        if ((rc = check_receivers(rec[i], g))) return rc;
        if (rec[i].n < 1) return set_error(EIG_EINVAL, "at least one receiver");
        if (!noise[i]) return set_error(EIG_EINVAL, "noise pointer NULL");
        const double* th = theta_star + (size_t)i * kNT;
        for (int j = 0; j < kNT; ++j)
            if (!std::isfinite(th[j])) return set_error(EIG_EINVAL, "theta not finite");
        if (!source_inside(th[0], th[1], g))
            return set_error(EIG_EINVAL, "source stencil touches a rigid node");
        med_of[i] = medium_index(media, seen, medium[i], g);
        recsets.push_back(RecSet{std::vector<int32_t>(rec[i].ix, rec[i].ix + rec[i].n), g.nx});
    }
    std::vector<double> th_cur(theta_star, theta_star + (size_t)nsample * kNT);
    // per-sample device region: truth, nominal and 7 sensitivity traces, the
    // dual's traces, injection and window record, descriptors, H1, grad, H2
    // (the last three as rows of chunk-wide arrays)
    auto sample_bytes = [&](int i) {
        const size_t tr = align_up((size_t)(grid[i].nsteps + 1) * rec[i].n * sizeof(float2));
        return 10 * tr + align_up((size_t)grid[i].nsteps * rec[i].n * sizeof(float2)) +
               align_up((size_t)grid[i].nsteps * kSrcW * kSrcW * sizeof(float2)) +
               align_up(sizeof(SampleDesc)) + align_up(sizeof(H2Job)) + align_up(sizeof(DualJob)) +
               align_up(sample_work_bytes(1)) +
               3 * align_up(kNT * kNT * sizeof(double)) + 4 * kAlign;
    };
    int s0 = 0;
    while (s0 < nsample) {
        int s1 = s0;
        size_t need = 0;
        WaveSizer wsz(grids, media, recsets);
        size_t extra = 8 * kAlign + align_up(sizeof(eig_prior));
        while (s1 < nsample) {
            SolveSpec sp{};
            sp.grid = s1;
            sp.medium = med_of[s1];
            sp.recset = s1;
            const size_t one = wsz.cost(sp);
            if (s1 > s0 && wsz.bytes + extra + 8 * one + sample_bytes(s1) > c->budget) break;
            for (int q = 0; q < 8; ++q) wsz.add(sp);
            extra += sample_bytes(s1) + 2 * sizeof(double);
            need = wsz.bytes + extra;
            ++s1;
        }
        if ((rc = ensure_ws(c, need))) return rc;
        const int ns = s1 - s0;
        Carve cv;
        struct Off {
            size_t ystar, nominal, sens[kNT], dtr, rf, wrec;
        };
        std::vector<Off> off(ns);
        for (int q = 0; q < ns; ++q) {
            const int i = s0 + q;
            const size_t tr = (size_t)(grid[i].nsteps + 1) * rec[i].n * sizeof(float2);
            off[q].ystar = cv.take(tr);
            off[q].nominal = cv.take(tr);
            for (int j = 0; j < kNT; ++j) off[q].sens[j] = cv.take(tr);
            off[q].dtr = cv.take(tr);
            off[q].rf = cv.take((size_t)grid[i].nsteps * rec[i].n * sizeof(float2));
            off[q].wrec = cv.take((size_t)grid[i].nsteps * kSrcW * kSrcW * sizeof(float2));
        }
        // H1 [ns][7][7], gradients [ns][7], H2 [ns][7][7]: one Hessian launch
        // and one copy each per chunk
        const size_t o_H1 = cv.take((size_t)ns * kNT * kNT * sizeof(double));
        const size_t o_grad = cv.take((size_t)ns * kNT * sizeof(double));
        const size_t o_H2 = cv.take((size_t)ns * kNT * kNT * sizeof(double));
        const size_t o_sd = cv.take(ns * sizeof(SampleDesc));
        const size_t o_h2 = cv.take(ns * sizeof(H2Job));
        const size_t o_dj = cv.take(ns * sizeof(DualJob));
        const size_t o_sig = cv.take(ns * sizeof(double));
        const size_t o_work = cv.take(sample_work_bytes(ns));
        const size_t solve_base = align_up(cv.off);
        char* ws = c->ws;
        auto tp = [&](size_t o) { return (float2*)(ws + o); };
        // sigma per sample (given)
        {
            std::vector<double> sg(ns, sigma);
            if ((rc = upload_small(c, o_sig, sg.data(), ns * sizeof(double), s))) return rc;
        }
        auto base_spec = [&](int i, const double* th) {
            SolveSpec sp{};
            sp.grid = i;
            sp.medium = med_of[i];
            sp.recset = i;
            std::memcpy(sp.theta, th, sizeof(sp.theta));
            sp.param = -1;
            sp.stf = stf_kind;
            return sp;
        };
        // 1. truth traces g(theta*)
        {
            std::vector<SolveSpec> sol;
            for (int q = 0; q < ns; ++q) {
                SolveSpec sp = base_spec(s0 + q, theta_star + (size_t)(s0 + q) * kNT);
                sp.traces = tp(off[q].ystar);
                sol.push_back(sp);
            }
            if ((rc = run_wave(c, sol, grids, media, recsets, ws + solve_base,
                               c->ws_size - solve_base, s)))
                return rc;
        }
        // 2./3. Gauss-Newton from theta*, then H_1 and g at theta^
        std::vector<double> hbuf((size_t)ns * (kNT * kNT + kNT));
        for (int it = 0; it <= iters; ++it) {
            std::vector<SolveSpec> sol;
            std::vector<SampleDesc> sds(ns);
            for (int q = 0; q < ns; ++q) {
                const int i = s0 + q;
                for (int j = 0; j < kNT; ++j)
                    if (!std::isfinite(th_cur[(size_t)i * kNT + j]))
                        return set_error(EIG_ENONFINITE, "Gauss-Newton diverged");
                if (!source_inside(th_cur[(size_t)i * kNT], th_cur[(size_t)i * kNT + 1], grid[i]))
                    return set_error(EIG_EINVAL,
                                     "Gauss-Newton iterate left the grid's source region");
                SolveSpec sp = base_spec(i, &th_cur[(size_t)i * kNT]);
                sp.traces = tp(off[q].nominal);
                sol.push_back(sp);
                SampleDesc& sd = sds[q];
                std::memset(&sd, 0, sizeof(sd));
                sd.nt = grid[i].nsteps + 1;
                sd.nrec = rec[i].n;
                sd.nominal = tp(off[q].nominal);
                sd.ystar = tp(off[q].ystar);
                sd.noise = (const float2*)noise[i];
                sd.grad = (double*)(ws + o_grad) + (size_t)q * kNT;
                for (int j = 0; j < kNT; ++j) {
                    SolveSpec pj = sp;
                    pj.param = j;
                    pj.deriv = 1;
                    pj.traces = tp(off[q].sens[j]);
                    sd.dev[2 * j] = pj.traces;
                    sd.inv2d[j] = 1.0;
                    sol.push_back(pj);
                }
            }
            if ((rc = run_wave(c, sol, grids, media, recsets, ws + solve_base,
                               c->ws_size - solve_base, s)))
                return rc;
            std::vector<char> blob(ns * sizeof(SampleDesc));
            std::memcpy(blob.data(), sds.data(), blob.size());
            if ((rc = upload(c, ws + o_sd, blob, s))) return rc;
            // H1 and the gradient of every sample (row q of the chunk arrays)
            launch_hessian((const SampleDesc*)(ws + o_sd), ns, 0, 1, (const double*)(ws + o_sig),
                           (double*)(ws + o_H1), (double*)(ws + o_work), s);
            HIP_TRY(hipGetLastError());
            if (it == iters) break;
            HIP_TRY(hipMemcpyAsync(hbuf.data(), ws + o_H1, (size_t)ns * kNT * kNT * sizeof(double),
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipMemcpyAsync(hbuf.data() + (size_t)ns * kNT * kNT, ws + o_grad,
                                   (size_t)ns * kNT * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            for (int q = 0; q < ns; ++q) {
                const double* Hq = &hbuf[(size_t)q * kNT * kNT];
                const double* gq = &hbuf[(size_t)ns * kNT * kNT + (size_t)q * kNT];
                double* th = &th_cur[(size_t)(s0 + q) * kNT];
                double step[kNT];
                if (!gn_step(Hq, gq, *prior, th, step))
                    return set_error(EIG_ENOTPD, "Gauss-Newton system not positive definite");
                for (int j = 0; j < kNT; ++j) th[j] += step[j];
            }
        }
        // 4. dual solves driven by the weighted residuals at the receivers
        {
            std::vector<SolveSpec> sol;
            std::vector<H2Job> jobs(ns);
            std::vector<DualJob> djobs(ns);
            size_t max_elems = 0;
            for (int q = 0; q < ns; ++q) {
                const int i = s0 + q;
                const eig_grid& g = grid[i];
                djobs[q] = DualJob{tp(off[q].ystar), (const float2*)noise[i], tp(off[q].nominal),
                                   tp(off[q].rf), sigma, 2.0 / (g.h * g.h), g.nsteps, rec[i].n};
                max_elems = std::max(max_elems, (size_t)g.nsteps * rec[i].n);
                double th0[kNT];
                std::memcpy(th0, &th_cur[(size_t)i * kNT], sizeof(th0));
                SolveSpec sp = base_spec(i, th0);
                sp.theta[4] = sp.theta[5] = sp.theta[6] = 0.0;  // no window forcing
                sp.traces = tp(off[q].dtr);
                sp.rforce = tp(off[q].rf);
                sp.wrec = tp(off[q].wrec);
                sol.push_back(sp);
                H2Job& J = jobs[q];
                std::memcpy(J.theta, th0, sizeof(J.theta));
                J.h = g.h;
                J.dt = g.dt;
                J.nsteps = g.nsteps;
                J.stf = stf_kind;
                J.kx = floor_cell(th0[0], g.h);
                J.kz = floor_cell(th0[1], g.h);
                J.i0 = J.kx - 2;
                J.k0 = J.kz - 2;
                J.wrec = tp(off[q].wrec);
                J.H2 = (double*)(ws + o_H2) + (size_t)q * kNT * kNT;
            }
            {
                std::vector<char> dblob(ns * sizeof(DualJob));
                std::memcpy(dblob.data(), djobs.data(), dblob.size());
                if ((rc = upload(c, ws + o_dj, dblob, s))) return rc;
                launch_dual_force((const DualJob*)(ws + o_dj), ns, max_elems, s);
            }
            HIP_TRY(hipGetLastError());
            if ((rc = run_wave(c, sol, grids, media, recsets, ws + solve_base,
                               c->ws_size - solve_base, s)))
                return rc;
            std::vector<char> blob(ns * sizeof(H2Job));
            std::memcpy(blob.data(), jobs.data(), blob.size());
            if ((rc = upload(c, ws + o_h2, blob, s))) return rc;
            launch_h2((const H2Job*)(ws + o_h2), ns, s);
        }
        // 5. outputs of the chunk
        HIP_TRY(hipMemcpyAsync(H1out + (size_t)s0 * kNT * kNT, ws + o_H1,
                               (size_t)ns * kNT * kNT * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(H2out + (size_t)s0 * kNT * kNT, ws + o_H2,
                               (size_t)ns * kNT * kNT * sizeof(double), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));  // the next chunk reuses the workspace
        s0 = s1;
    }
    std::memcpy(theta_hat, th_cur.data(), th_cur.size() * sizeof(double));
    // 6. Theorem 3 integrand and the weighted average
    Carve cv;
    const size_t o_pr = cv.take(sizeof(eig_prior));
    const size_t o_th = cv.take((size_t)nsample * kNT * sizeof(double));
    const size_t o_w = cv.take((size_t)nsample * sizeof(double));
    if ((rc = ensure_ws(c, cv.off))) return rc;
    if ((rc = upload_small(c, o_pr, prior, sizeof(eig_prior), s))) return rc;
    if ((rc = upload_small(c, o_th, th_cur.data(), th_cur.size() * sizeof(double), s))) return rc;
    if ((rc = upload_small(c, o_w, w, (size_t)nsample * sizeof(double), s))) return rc;
    launch_theorem3(H1out, H2out, nsample, (const eig_prior*)(c->ws + o_pr),
                    (const double*)(c->ws + o_th), (const double*)(c->ws + o_w), val, status,
                    eig, s);
    HIP_TRY(hipGetLastError());
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
