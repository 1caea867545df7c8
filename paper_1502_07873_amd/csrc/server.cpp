// Serving engine: continuous batching of design queries on one GPU.
//
// A query is the per-sample Jacobian/H_1 work of jacobian_fd followed by
// laplace_eig.  Its samples are admitted in groups of `group_samples` as
// device memory frees up (first-fit arena inside the server's HBM budget)
// and as descriptor slots allow, so queries that arrive while others run
// join at the next segment boundary.  Work is scheduled by segments: at each
// boundary the admitted groups are ranked by their query's remaining
// grid-point updates (shortest first, then arrival order); all groups of
// the first query run, and those of the next queries are added while a
// launch stays within max(the first query's points, kFillPoints), the size
// at which a launch already keeps the device busy.  A short query that
// arrives behind a long one therefore runs at once, alone or beside other
// short ones, and the long one resumes when it is done.  Every launch
// advances each scheduled solve by one leapfrog step (two or four for the
// multi-step kernels): a solve with `done` launches behind it that is scheduled at
// launch L has SolveDesc::start = L - done, rewritten when a paused group
// resumes.  Segment boundaries also fall where a scheduled group finishes;
// there finished groups get their Hessian kernels and free their memory and
// waiting groups are admitted.  Per-sample arithmetic does not depend on the
// batch or the schedule, so each query's result is the same alone and in the
// mix.
#include <deque>
#include <memory>

#include "host.h"

namespace {

// First-fit allocator over [0, size) with coalescing.
struct Arena {
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size = 0, align = kAlign;
    size_t used = 0, peak = 0;       // bytes handed out now / at most
    void init(size_t sz, size_t al) {
        size = sz;
        align = al;
        free_.clear();
        used = peak = 0;
        if (sz) free_[0] = sz;
    }
    size_t round(size_t b) const { return (b + align - 1) / align * align; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = round(std::max<size_t>(bytes, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, noff = it->first + bytes;
            free_.erase(it);
            if (rest) free_[noff] = rest;
            used += bytes;
            peak = std::max(peak, used);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = round(std::max<size_t>(bytes, 1));
        used -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

struct SrvQuery {
    int64_t id = 0;
    eig_grid grid{};
    eig_medium medium{};
    int nsample = 0;
    std::vector<double> theta;
    double rel_step = 1e-4;
    int stf = EIG_STF_GAUSS_DERIV;
    std::vector<int32_t> rec;
    int sigma_mode = EIG_SIGMA_GIVEN;
    double sigma = 1.0;
    eig_prior prior{};
    std::vector<double> w;
    double *H1 = nullptr, *dkl = nullptr, *eig = nullptr;
    int32_t *status = nullptr, *chol_status = nullptr;
    int next_sample = 0;
    int groups_running = 0;
    double waited = 0.0;     // updates others did while its groups sat paused
    double queued_at = 0.0;  // the server's update count when it was submitted
    bool finished = false;
    hipEvent_t done_ev = nullptr;
    size_t tail_off = 0, tail_bytes = 0;  // prior, theta, weights for laplace
};

struct SrvGroup {
    SrvQuery* q = nullptr;
    int s0 = 0, s1 = 0;      // samples [s0, s1) of the query
    size_t slot0 = 0, nslot = 0;
    size_t off = 0, bytes = 0;
    size_t live = 0;         // field bytes its solves keep live between launches
    int64_t start = 0;       // launch index of step 0 in the descriptors on the device
    int64_t done = 0;        // launches this group has taken
    bool on = false;         // in the current tile map
    int nsteps = 0;
    size_t o_sd = 0, o_given = 0, o_sig = 0, o_work = 0;
    std::vector<SolveDesc> desc;  // host copy of its descriptors (start rewritten)
};

// Grid points per launch at which one launch already keeps the device busy
// (the two-step kernel's cache-sized chunks hold 6.3 million).
constexpr double kFillPoints = 16.0 * (1 << 20);

size_t trace_bytes(const eig_grid& g, int nrec) {
    return align_up((size_t)(g.nsteps + 1) * nrec * sizeof(float2));
}

// Arena bytes of a group of G samples of query q (one allocation).
size_t group_bytes(const SrvQuery& q, int G) {
    const eig_grid& g = q.grid;
    MediumKey mk{q.medium.kind, q.medium.rho, q.medium.lam, q.medium.mu, g.nx, g.nz, g.h, g.dt};
    size_t b = medium_bytes(mk) + align_up((size_t)pitch_of(g.nx) * sizeof(int32_t));
    b += (size_t)15 * G * (solve_bytes(g) + trace_bytes(g, (int)q.rec.size()));
    b += align_up((size_t)G * sizeof(SampleDesc)) + 2 * align_up((size_t)G * sizeof(double));
    b += align_up(sample_work_bytes(G));
    b += align_up((size_t)15 * G * sizeof(SourceJob));
    return b + 16 * kAlign;
}

// Arena bytes of a query's laplace inputs (prior, theta, weights), reserved
// with its first group and released when the query finishes.
size_t tail_bytes(const SrvQuery& q) {
    return align_up(sizeof(eig_prior)) + align_up(q.theta.size() * 8) + align_up(q.w.size() * 8) +
           4 * kAlign;
}

}  // namespace

struct eig_server {
    eig_ctx* ctx = nullptr;
    char* mem = nullptr;
    size_t mem_size = 0;
    Arena arena;
    SolveDesc* descs = nullptr;  // device slot array
    size_t nslot_cap = 0;
    Arena slots;                 // unit: one slot
    int2* tiles = nullptr;
    size_t tile_cap = 0;
    int64_t launch = 0;
    int group_samples = 16;
    int variant_layered = 4;
    int variant_nodal = 18;
    // cache-limited admission: the admitted groups' live fields stay within
    // cache_bytes (the device's last-level cache), so launches read and write
    // that cache instead of HBM; 0: admit whatever memory and slots allow
    size_t cache_bytes = 0;
    size_t live = 0;
    int spl_layered = 1, spl_nodal = 1;  // leapfrog steps per launch of each kind's variant
    std::deque<SrvQuery*> queue;
    std::map<int64_t, std::unique_ptr<SrvQuery>> queries;
    std::vector<SrvGroup> groups;
    std::vector<std::pair<int, size_t>> kind_tiles;  // (variant, ntiles) per kind range
    std::vector<size_t> kind_tile_off;
    bool tiles_dirty = true;
    int64_t next_id = 1;
    double work_done = 0.0;  // grid-point updates of all launches so far
};

namespace {

int spl_of(const eig_server* v, int kind) {
    return kind == EIG_MEDIUM_NODAL ? v->spl_nodal : v->spl_layered;
}

// Admits one sample group of queued query q if memory, slots and the cache
// limit allow (*ok), else leaves everything as it was.
int srv_admit_group(eig_server* v, SrvQuery& q, hipStream_t s, bool* ok) {
    eig_ctx* c = v->ctx;
    *ok = false;
    {
        int G = std::min(v->group_samples, q.nsample - q.next_sample);
        G = std::min<int>(G, (int)(v->nslot_cap / 15));
        const int spl = spl_of(v, q.medium.kind);
        const size_t sample_live = (size_t)15 * (spl >= 2 ? 4 : 2) * q.grid.nz *
                                   pitch_of(q.grid.nx) * sizeof(float2);
        // the cache limit applies to queries one of whose samples fits it;
        // larger ones gain nothing from it and are admitted by memory alone,
        // and so are four-step kinds, which stream HBM at their floor
        const bool cached = v->cache_bytes && spl < 4 && sample_live <= v->cache_bytes;
        if (cached) {
            G = std::min<int>(G, (int)(v->cache_bytes / sample_live));
            if (!v->groups.empty() && v->live + (size_t)G * sample_live > v->cache_bytes)
                return EIG_OK;
        }
        size_t off = 0, slot0 = 0;
        if (q.next_sample == 0 && q.tail_bytes == 0) {
            // the query's small laplace inputs are reserved with its first group
            const size_t tb = tail_bytes(q);
            if (!v->arena.alloc(tb, &q.tail_off)) return EIG_OK;
            q.tail_bytes = tb;
        }
        // a full group when memory allows; with nothing running, halve the
        // group until it fits (submit guaranteed that one sample does), so
        // the head of the queue never waits for memory that cannot free up
        size_t bytes = group_bytes(q, G);
        bool got = v->arena.alloc(bytes, &off);
        while (!got && v->groups.empty() && G > 1) {
            G = (G + 1) / 2;
            bytes = group_bytes(q, G);
            got = v->arena.alloc(bytes, &off);
        }
        if (!got) return EIG_OK;
        if (!v->slots.alloc((size_t)15 * G, &slot0)) {
            v->arena.release(off, bytes);
            return EIG_OK;
        }
        SrvGroup gr;
        gr.q = &q;
        gr.s0 = q.next_sample;
        gr.s1 = q.next_sample + G;
        gr.slot0 = slot0;
        gr.nslot = (size_t)15 * G;
        gr.off = off;
        gr.bytes = bytes;
        gr.live = cached ? (size_t)G * sample_live : 0;
        gr.start = v->launch;
        gr.nsteps = q.grid.nsteps;
        const bool four = spl >= 2;
        // carve the group's region
        char* base = v->mem + off;
        const eig_grid& g = q.grid;
        const int nrec = (int)q.rec.size();
        MediumKey mk{q.medium.kind, q.medium.rho, q.medium.lam, q.medium.mu, g.nx, g.nz, g.h, g.dt};
        Carve cv;
        const size_t o_coef = cv.take(medium_bytes(mk));
        const size_t o_map = cv.take((size_t)pitch_of(g.nx) * sizeof(int32_t));
        const size_t field = (size_t)g.nz * pitch_of(g.nx) * sizeof(float2);
        const size_t fields_begin = align_up(cv.off);
        cv.off = fields_begin;
        std::vector<size_t> f0(gr.nslot), f1(gr.nslot), f2(gr.nslot, 0), f3(gr.nslot, 0);
        std::vector<size_t> sw(gr.nslot), ss(gr.nslot), tr(gr.nslot);
        for (size_t k = 0; k < gr.nslot; ++k) {
            f0[k] = cv.take(field);
            f1[k] = cv.take(field);
            if (four) {
                f2[k] = cv.take(field);
                f3[k] = cv.take(field);
            }
        }
        const size_t fields_end = cv.off;
        for (size_t k = 0; k < gr.nslot; ++k) {
            sw[k] = cv.take(2 * kSrcW * kSrcW * sizeof(float));
            ss[k] = cv.take((size_t)std::max(g.nsteps, 1) * sizeof(float));
            tr[k] = cv.take((size_t)(g.nsteps + 1) * nrec * sizeof(float2));
        }
        gr.o_sd = cv.take((size_t)G * sizeof(SampleDesc));
        gr.o_given = cv.take((size_t)G * sizeof(double));
        gr.o_sig = cv.take((size_t)G * sizeof(double));
        gr.o_work = cv.take(sample_work_bytes(G));
        const size_t o_jobs = cv.take(gr.nslot * sizeof(SourceJob));
        if (cv.off > bytes) return set_error(EIG_EBUDGET, "server group carve overflow");
        // descriptors, forcing jobs, sample descriptors
        std::vector<SolveDesc> desc(gr.nslot);
        std::vector<SourceJob> jobs(gr.nslot);
        std::vector<SampleDesc> sds(G);
        std::vector<double> given(G, q.sigma);
        for (int gs = 0; gs < G; ++gs) {
            const double* th = q.theta.data() + (size_t)(gr.s0 + gs) * kNT;
            SampleDesc& sd = sds[gs];
            std::memset(&sd, 0, sizeof(sd));
            sd.nt = g.nsteps + 1;
            sd.nrec = nrec;
            sd.rho = q.medium.rho;
            sd.lam = q.medium.lam;
            sd.mu = q.medium.mu;
            sd.med_kind = q.medium.kind;
            sd.nx = g.nx;
            sd.nz = g.nz;
            sd.dt2_h2 = (g.dt / g.h) * (g.dt / g.h);
            for (int q15 = 0; q15 < 15; ++q15) {
                const size_t k = (size_t)gs * 15 + q15;
                const int param = q15 == 0 ? -1 : (q15 - 1) / 2;
                const double d = param >= 0 ? q.rel_step * std::fabs(th[param]) : 0.0;
                const double step = q15 == 0 ? 0.0 : ((q15 - 1) % 2 == 0 ? d : -d);
                SolveDesc& dd = desc[k];
                std::memset(&dd, 0, sizeof(dd));
                dd.buf0 = (float2*)(base + f0[k]);
                dd.buf1 = (float2*)(base + f1[k]);
                dd.buf2 = four ? (float2*)(base + f2[k]) : nullptr;
                dd.buf3 = four ? (float2*)(base + f3[k]) : nullptr;
                dd.coef = (const float*)(base + o_coef);
                dd.srcw = (const float*)(base + sw[k]);
                dd.srcs = (const float*)(base + ss[k]);
                dd.recmap = (const int32_t*)(base + o_map);
                dd.traces = (float2*)(base + tr[k]);
                dd.nx = g.nx;
                dd.nz = g.nz;
                dd.pitch = pitch_of(g.nx);
                dd.nsteps = g.nsteps;
                dd.start = (int32_t)gr.start;
                dd.nrec = nrec;
                dd.medium_kind = q.medium.kind;
                dd.h2 = (float)(g.h * g.h);
                SourceJob& J = jobs[k];
                std::memcpy(J.theta, th, sizeof(J.theta));
                J.step = step;
                J.h = g.h;
                J.dt = g.dt;
                J.param = param;
                J.kx = floor_cell(th[0], g.h);
                J.kz = floor_cell(th[1], g.h);
                double tp[kNT];
                std::memcpy(tp, th, sizeof(tp));
                if (param >= 0) tp[param] = th[param] + step;
                J.kx2 = floor_cell(tp[0], g.h);
                J.kz2 = floor_cell(tp[1], g.h);
                J.i0 = std::min(std::min(J.kx, J.kx2) - 2, g.nx - kSrcW);
                J.k0 = std::min(std::min(J.kz, J.kz2) - 2, g.nz - kSrcW);
                J.nsteps = g.nsteps;
                J.stf = q.stf;
                J.srcw = (float*)(base + sw[k]);
                J.srcs = (float*)(base + ss[k]);
                dd.src_i0 = J.i0;
                dd.src_k0 = J.k0;
                if (q15 == 0) sd.nominal = dd.traces;
                else sd.dev[q15 - 1] = dd.traces;
                if (param >= 0) sd.inv2d[param] = 1.0 / (2.0 * d);
            }
        }
        std::vector<int32_t> map(pitch_of(g.nx), -1);
        for (int r = 0; r < nrec; ++r) map[q.rec[r]] = r;
        // uploads: receiver map, sample descriptors, sigma, jobs (group
        // region) and descriptors (slot range)
        auto put = [&](size_t o, const void* p, size_t nb) -> int {
            std::vector<char> b(nb);
            std::memcpy(b.data(), p, nb);
            return upload(c, base + o, b, s);
        };
        int rc;
        if ((rc = put(o_map, map.data(), map.size() * sizeof(int32_t)))) return rc;
        if ((rc = put(gr.o_sd, sds.data(), sds.size() * sizeof(SampleDesc)))) return rc;
        if ((rc = put(gr.o_given, given.data(), given.size() * sizeof(double)))) return rc;
        if ((rc = put(o_jobs, jobs.data(), jobs.size() * sizeof(SourceJob)))) return rc;
        {
            std::vector<char> b(desc.size() * sizeof(SolveDesc));
            std::memcpy(b.data(), desc.data(), b.size());
            if ((rc = upload(c, v->descs + gr.slot0, b, s))) return rc;
        }
        gr.desc = std::move(desc);
        if (q.medium.kind == EIG_MEDIUM_NODAL)
            launch_nodal_coef(q.medium.rho, q.medium.lam, q.medium.mu, g.nx, g.nz,
                              pitch_of(g.nx), g.h, g.dt, (float*)(base + o_coef), s);
        else
            launch_layered_coef(q.medium.rho, q.medium.lam, q.medium.mu, g.nz, g.h, g.dt,
                                (float*)(base + o_coef), s);
        launch_source_tables((const SourceJob*)(base + o_jobs), (int)gr.nslot, 0, s);
        launch_fill_zero(base + fields_begin, fields_end - fields_begin, s);
        launch_zero_level0(v->descs + gr.slot0, (int)gr.nslot, s);
        HIP_TRY(hipGetLastError());
        v->live += gr.live;
        q.next_sample += G;
        q.groups_running += 1;
        if (q.next_sample >= q.nsample)
            v->queue.erase(std::find(v->queue.begin(), v->queue.end(), &q));
        v->groups.push_back(std::move(gr));
        v->tiles_dirty = true;
    }
    *ok = true;
    return EIG_OK;
}

double query_work_left(const eig_server* v, const SrvQuery& q);
int64_t group_launches(const eig_server* v, const SrvGroup& gr);

// Admission in the scheduler's order: queued queries by remaining work
// (shortest first, then arrival), each taking as many groups as fit; a query
// that cannot take a group now is skipped, unless others have done more than
// twice its remaining work since it arrived, in which case it is admitted
// first and nothing queued behind it is (so large queries are not starved).
int srv_admit(eig_server* v, hipStream_t s) {
    for (;;) {
        std::vector<SrvQuery*> order(v->queue.begin(), v->queue.end());
        auto overdue = [&](const SrvQuery* q) {
            return v->work_done - q->queued_at > 2.0 * query_work_left(v, *q);
        };
        std::stable_sort(order.begin(), order.end(), [&](SrvQuery* a, SrvQuery* b) {
            const bool oa = overdue(a), ob = overdue(b);
            if (oa != ob) return oa;
            if (oa) return a->id < b->id;
            const double wa = query_work_left(v, *a), wb = query_work_left(v, *b);
            return wa != wb ? wa < wb : a->id < b->id;
        });
        bool any = false;
        for (SrvQuery* q : order) {
            bool ok = false;
            const int rc = srv_admit_group(v, *q, s, &ok);
            if (rc) return rc;
            if (ok) {
                any = true;
                break;   // priorities may change: rank again
            }
            if (overdue(q)) break;
        }
        if (!any) return EIG_OK;
    }
}



int srv_finish_query(eig_server* v, SrvQuery& q, hipStream_t s) {
    eig_ctx* c = v->ctx;
    // laplace_eig over the whole query (prior, theta, weights reserved with
    // the first group)
    char* base = v->mem + q.tail_off;
    Blob blob;
    const size_t o_pr = blob.put(&q.prior, sizeof(eig_prior));
    const size_t o_th = blob.put(q.theta.data(), q.theta.size() * sizeof(double));
    const size_t o_w = blob.put(q.w.data(), q.w.size() * sizeof(double));
    int rc = upload(c, base, blob.data, s);
    if (rc) return rc;
    launch_laplace(q.H1, q.nsample, (const eig_prior*)(base + o_pr),
                   (const double*)(base + o_th), (const double*)(base + o_w), q.dkl, nullptr,
                   q.chol_status, q.eig, s);
    HIP_TRY(hipEventRecord(q.done_ev, s));
    HIP_TRY(hipGetLastError());
    v->arena.release(q.tail_off, q.tail_bytes);  // later users are ordered after this work
    q.tail_bytes = 0;
    q.finished = true;
    return EIG_OK;
}

// launches a group needs in total
int64_t group_launches(const eig_server* v, const SrvGroup& gr) {
    const int spl = spl_of(v, gr.q->medium.kind);
    return (gr.nsteps + spl - 1) / spl;
}

int srv_retire(eig_server* v, hipStream_t s) {
    std::vector<SrvGroup> keep;
    for (auto& gr : v->groups) {
        if (gr.done < group_launches(v, gr)) {
            keep.push_back(std::move(gr));
            continue;
        }
        SrvQuery& q = *gr.q;
        char* base = v->mem + gr.off;
        const int G = gr.s1 - gr.s0;
        const SampleDesc* dsd = (const SampleDesc*)(base + gr.o_sd);
        double* dsig = (double*)(base + gr.o_sig);
        double* dwork = (double*)(base + gr.o_work);
        launch_sample_check(dsd, G, (const double*)(base + gr.o_given), q.sigma_mode, dsig,
                            q.status ? q.status + gr.s0 : nullptr, dwork, s);
        launch_hessian(dsd, G, 0, 1, dsig, q.H1 + (size_t)gr.s0 * kNT * kNT, dwork, s);
        HIP_TRY(hipGetLastError());
        v->arena.release(gr.off, gr.bytes);
        v->slots.release(gr.slot0, gr.nslot);
        v->live -= gr.live;
        v->tiles_dirty = true;
        q.groups_running -= 1;
        if (q.next_sample >= q.nsample && q.groups_running == 0) {
            const int rc = srv_finish_query(v, q, s);
            if (rc) return rc;
        }
    }
    v->groups.swap(keep);
    return EIG_OK;
}

// Grid-point updates a query still needs (admitted and waiting samples).
double query_work_left(const eig_server* v, const SrvQuery& q) {
    const double pts = (double)q.grid.nx * q.grid.nz;
    double w = 15.0 * (q.nsample - q.next_sample) * pts * q.grid.nsteps;
    for (const auto& gr : v->groups) {
        if (gr.q != &q) continue;
        const int spl = spl_of(v, q.medium.kind);
        w += (double)gr.nslot * pts * std::max<int64_t>(0, gr.nsteps - spl * gr.done);
    }
    return w;
}

// Chooses the groups of the next segment (see the file comment) and brings
// the device descriptors of resumed groups up to date.
int srv_schedule(eig_server* v, hipStream_t s) {
    std::vector<std::pair<double, SrvQuery*>> qs;
    for (const auto& gr : v->groups) {
        bool seen = false;
        for (const auto& e : qs) seen = seen || e.second == gr.q;
        if (!seen) qs.push_back({query_work_left(v, *gr.q), gr.q});
    }
    std::stable_sort(qs.begin(), qs.end(), [](const auto& a, const auto& b) {
        return a.first != b.first ? a.first < b.first : a.second->id < b.second->id;
    });
    auto points = [](const SrvGroup& gr) {
        return (double)gr.nslot * gr.q->grid.nx * gr.q->grid.nz;
    };
    std::map<const SrvQuery*, bool> run;
    double acc = 0.0, cap = 0.0;
    for (size_t k = 0; k < qs.size(); ++k) {
        const SrvQuery* q = qs[k].second;
        double pts = 0.0;
        for (const auto& gr : v->groups)
            if (gr.q == q) pts += points(gr);
        if (k == 0) cap = std::max(pts, kFillPoints);
        // no starvation: a query while paused for which the others have done
        // as much work as it still needs runs whatever its rank (its
        // slowdown stays below about 2x)
        if (k > 0 && acc + pts > cap && q->waited < qs[k].first) continue;
        run[q] = true;
        acc += pts;
    }
    for (const auto& e : qs)
        if (run.count(e.second)) e.second->waited = 0.0;
    for (auto& gr : v->groups) {
        const bool on = run.count(gr.q) != 0;
        if (on != gr.on) v->tiles_dirty = true;
        gr.on = on;
        if (!on || gr.start == v->launch - gr.done) continue;
        // resumed (or first scheduled): step done at launch L = start + done
        gr.start = v->launch - gr.done;
        for (auto& d : gr.desc) d.start = (int32_t)gr.start;
        std::vector<char> b(gr.desc.size() * sizeof(SolveDesc));
        std::memcpy(b.data(), gr.desc.data(), b.size());
        const int rc = upload(v->ctx, v->descs + gr.slot0, b, s);
        if (rc) return rc;
    }
    return EIG_OK;
}

int srv_rebuild_tiles(eig_server* v, hipStream_t s) {
    if (!v->tiles_dirty) return EIG_OK;
    v->tiles_dirty = false;
    std::vector<int2> all;
    v->kind_tiles.clear();
    v->kind_tile_off.clear();
    for (int kind : {EIG_MEDIUM_LAYERED, EIG_MEDIUM_NODAL}) {
        const int var = kind == EIG_MEDIUM_NODAL ? v->variant_nodal : v->variant_layered;
        const StencilVariant& sv = kVariants[var];
        const size_t begin = all.size();
        for (const auto& gr : v->groups) {
            if (gr.q->medium.kind != kind || !gr.on) continue;
            const eig_grid& g = gr.q->grid;
            const int nstrip = (g.nx + sv.cols - 1) / sv.cols;
            const int nchunk = (g.nz - 1 + sv.rows - 1) / sv.rows;
            // a group's solves share one medium: on nodal media, sets of
            // coef_interleave solves run position-major (coefficients read
            // from L2 once per set; the order changes no result)
            const size_t set = kind == EIG_MEDIUM_NODAL
                                   ? (size_t)std::max(v->ctx->coef_interleave, 1) : 1;
            for (size_t k0 = 0; k0 < gr.nslot; k0 += set) {
                const size_t k1 = std::min(gr.nslot, k0 + set);
                for (int ch = 0; ch < nchunk; ++ch)
                    for (int st = 0; st < nstrip; ++st)
                        for (size_t k = k0; k < k1; ++k)
                            all.push_back(make_int2((int)(gr.slot0 + k), (st << 16) | ch));
            }
        }
        v->kind_tiles.push_back({var, all.size() - begin});
        v->kind_tile_off.push_back(begin);
    }
    if (all.size() > v->tile_cap) {
        HIP_TRY(hipStreamSynchronize(s));
        if (v->tiles) HIP_TRY(hipFree(v->tiles));
        v->tiles = nullptr;
        v->tile_cap = all.size() + all.size() / 2 + 1024;
        HIP_TRY(hipMalloc((void**)&v->tiles, v->tile_cap * sizeof(int2)));
    }
    std::vector<char> b(all.size() * sizeof(int2));
    if (!b.empty()) std::memcpy(b.data(), all.data(), b.size());
    return upload(v->ctx, v->tiles, b, s);
}

}  // namespace

extern "C" {

int eig_server_create(eig_ctx* c, size_t budget, int32_t group_samples, eig_server** out) {
    if (!c || !out || budget < ((size_t)64 << 20))
        return set_error(EIG_EINVAL, "eig_server_create arguments");
    HIP_TRY(hipSetDevice(c->device));
    auto v = std::make_unique<eig_server>();
    v->ctx = c;
    v->group_samples = group_samples > 0 ? group_samples : 16;
    // the server advances groups launch by launch: resident variants (a
    // whole time loop per launch) are not used here.  Rigid edges only, so
    // with temporal_blocking 4 (the default) both kinds take four steps per
    // launch with the tile in LDS (variants 23, 24); otherwise depth-only
    // media take two steps (16-row tiles under the cache limit) and nodal
    // media one, with two nodes per lane
    const int fv = c->forced_variant;
    const bool forced = fv >= 0 && !kVariants[fv].resident;
    const bool forced_layered = forced && kVariants[fv].medium_kind == EIG_MEDIUM_LAYERED;
    const bool forced_nodal = forced && kVariants[fv].medium_kind == EIG_MEDIUM_NODAL;
    v->cache_bytes = c->serve_cache_bytes;
    if (forced_layered)
        v->variant_layered = fv;
    else if (c->temporal_blocking == 4)
        v->variant_layered = 23;
    else if (v->cache_bytes)
        v->variant_layered = c->temporal_blocking >= 2 ? 9 : c->default_variant;
    else
        v->variant_layered = c->temporal_blocking >= 2 ? c->default_variant_tb : c->default_variant;
    if (forced_nodal)
        v->variant_nodal = fv;
    else if (c->temporal_blocking == 4)
        v->variant_nodal = 24;
    v->spl_layered = kVariants[v->variant_layered].steps;
    v->spl_nodal = kVariants[v->variant_nodal].steps;
    v->nslot_cap = 1 << 17;
    if (hipMalloc((void**)&v->mem, budget) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(EIG_ENOMEM, "server arena allocation failed");
    }
    v->mem_size = budget;
    v->arena.init(budget, kAlign);
    if (hipMalloc((void**)&v->descs, v->nslot_cap * sizeof(SolveDesc)) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(v->mem);
        return set_error(EIG_ENOMEM, "server descriptor allocation failed");
    }
    v->slots.init(v->nslot_cap, 1);
    *out = v.release();
    return EIG_OK;
}

void eig_server_destroy(eig_server* v) {
    if (!v) return;
    (void)hipSetDevice(v->ctx->device);
    (void)hipDeviceSynchronize();
    for (auto& kv : v->queries)
        if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
    if (v->tiles) (void)hipFree(v->tiles);
    if (v->descs) (void)hipFree(v->descs);
    if (v->mem) (void)hipFree(v->mem);
    delete v;
}

int eig_server_submit(eig_server* v, const eig_grid* grid, const eig_medium* medium,
                      int32_t nsample, const double* theta, double rel_step,
                      int32_t stf_kind, const eig_receivers* rec, int32_t sigma_mode,
                      double sigma, const eig_prior* prior, const double* w, double* H1,
                      double* dkl, double* eig, int32_t* status, int32_t* chol_status,
                      int64_t* id) {
    if (!v || !grid || !medium || !theta || !rec || !prior || !w || !H1 || !dkl || !eig || !id)
        return set_error(EIG_EINVAL, "eig_server_submit: NULL argument");
    if (nsample < 1) return set_error(EIG_EINVAL, "nsample < 1");
    if (!valid_grid(*grid)) return set_error(EIG_EINVAL, "grid");
    if (grid->bc != EIG_BC_RIGID)
        return set_error(EIG_EUNSUPPORTED, "the server runs rigid-edge grids only");
    if (medium->kind != EIG_MEDIUM_LAYERED && medium->kind != EIG_MEDIUM_NODAL)
        return set_error(EIG_EINVAL, "medium kind");
    if (!medium->rho || !medium->lam || !medium->mu)
        return set_error(EIG_EINVAL, "medium arrays NULL");
    int rc = check_receivers(*rec, *grid);
    if (rc) return rc;
    if (rec->n < 1) return set_error(EIG_EINVAL, "at least one receiver");
    if (!(rel_step > 0) || rel_step > 0.1) return set_error(EIG_EINVAL, "rel_step");
    if (stf_kind != EIG_STF_GAUSS && stf_kind != EIG_STF_GAUSS_DERIV)
        return set_error(EIG_EINVAL, "stf_kind");
    if (sigma_mode != EIG_SIGMA_GIVEN && sigma_mode != EIG_SIGMA_NOMINAL_PEAK)
        return set_error(EIG_EINVAL, "sigma_mode");
    if (!(sigma > 0) || !std::isfinite(sigma)) return set_error(EIG_EINVAL, "sigma");
    if (prior->kind == EIG_PRIOR_UNIFORM) {
        for (int j = 0; j < kNT; ++j)
            if (!(prior->hi[j] > prior->lo[j])) return set_error(EIG_EINVAL, "prior box");
    } else if (prior->kind != EIG_PRIOR_GAUSSIAN) {
        return set_error(EIG_EINVAL, "prior kind");
    }
    for (int s = 0; s < nsample; ++s) {
        const double* th = theta + (size_t)s * kNT;
        for (int j = 0; j < kNT; ++j)
            if (!std::isfinite(th[j]) || th[j] == 0.0)
                return set_error(EIG_EINVAL, "theta entries must be finite and nonzero");
        for (int j = 0; j < 2; ++j)
            for (int sg = -1; sg <= 1; ++sg) {
                double x = th[0], z = th[1];
                (j == 0 ? x : z) += sg * rel_step * std::fabs(th[j]);
                if (!source_inside(x, z, *grid))
                    return set_error(EIG_EINVAL, "source stencil touches a rigid node");
                if (!deviation_in_window(th[j], sg * rel_step * std::fabs(th[j]), grid->h))
                    return set_error(EIG_EINVAL,
                                     "rel_step * |theta| moves the source by more than one "
                                     "cell (the forcing window covers one)");
            }
    }
    auto q = std::make_unique<SrvQuery>();
    q->id = v->next_id++;
    q->grid = *grid;
    q->medium = *medium;
    q->nsample = nsample;
    q->theta.assign(theta, theta + (size_t)nsample * kNT);
    q->rel_step = rel_step;
    q->stf = stf_kind;
    q->rec.assign(rec->ix, rec->ix + rec->n);
    q->sigma_mode = sigma_mode;
    q->sigma = sigma;
    q->prior = *prior;
    q->w.assign(w, w + nsample);
    q->H1 = H1;
    q->dkl = dkl;
    q->eig = eig;
    q->status = status;
    q->chol_status = chol_status;
    // an idle server always admits at least one sample of the query at the
    // head of the queue: its one-sample group and its laplace inputs must
    // fit the arena together
    if (group_bytes(*q, 1) + tail_bytes(*q) > v->mem_size)
        return set_error(EIG_EBUDGET, "one sample of this query exceeds the server budget");
    HIP_TRY(hipEventCreateWithFlags(&q->done_ev, hipEventDisableTiming));
    *id = q->id;
    q->queued_at = v->work_done;
    v->queue.push_back(q.get());
    v->queries[q->id] = std::move(q);
    return EIG_OK;
}

int eig_server_step(eig_server* v, int32_t max_launches, void* stream, int32_t* running) {
    if (!v || max_launches < 0) return set_error(EIG_EINVAL, "eig_server_step arguments");
    HIP_TRY(hipSetDevice(v->ctx->device));
    hipStream_t s = (hipStream_t)stream;
    eig_ctx* c = v->ctx;
    int rc;
    if ((rc = srv_retire(v, s))) return rc;
    if ((rc = srv_admit(v, s))) return rc;
    int done = 0;
    while (done < max_launches && !v->groups.empty()) {
        if ((rc = srv_schedule(v, s))) return rc;
        if ((rc = srv_rebuild_tiles(v, s))) return rc;
        int64_t seg = max_launches - done;
        for (const auto& gr : v->groups)
            if (gr.on) seg = std::min(seg, group_launches(v, gr) - gr.done);
        // queries none of whose admitted groups run in this segment
        std::vector<SrvQuery*> paused;
        for (const auto& gr : v->groups) {
            bool any_on = false;
            for (const auto& g2 : v->groups) any_on = any_on || (g2.q == gr.q && g2.on);
            if (!any_on && std::find(paused.begin(), paused.end(), gr.q) == paused.end())
                paused.push_back(gr.q);
        }
        for (int64_t l = 0; l < seg; ++l) {
            double upd = 0.0;
            for (auto& gr : v->groups) {
                if (!gr.on) continue;
                const int spl = spl_of(v, gr.q->medium.kind);
                const int64_t left = gr.nsteps - spl * gr.done;
                upd += (double)gr.q->grid.nx * gr.q->grid.nz * gr.nslot *
                       (double)std::min<int64_t>(spl, left);
                gr.done += 1;
            }
            c->updates += upd;
            v->work_done += upd;
            for (SrvQuery* q : paused) q->waited += upd;
            for (size_t kk = 0; kk < v->kind_tiles.size(); ++kk) {
                const size_t nt = v->kind_tiles[kk].second;
                if (nt == 0) continue;
                launch_stencil(v->descs, v->tiles + v->kind_tile_off[kk], (int)nt,
                               (int)v->launch, v->kind_tiles[kk].first, s);
                c->launches += 1;
            }
            ++v->launch;
        }
        done += (int)seg;
        if ((rc = srv_retire(v, s))) return rc;
        if ((rc = srv_admit(v, s))) return rc;
    }
    HIP_TRY(hipGetLastError());
    if (running) *running = (int32_t)v->groups.size();
    if (v->groups.empty() && !v->queue.empty())
        return set_error(EIG_EBUDGET, "the query at the head of the queue cannot be admitted");
    return EIG_OK;
}

int eig_server_poll(eig_server* v, int64_t id, int32_t* done) {
    if (!v || !done) return set_error(EIG_EINVAL, "eig_server_poll arguments");
    auto it = v->queries.find(id);
    if (it == v->queries.end()) return set_error(EIG_EINVAL, "unknown query id");
    SrvQuery& q = *it->second;
    *done = 0;
    if (!q.finished) return EIG_OK;
    const hipError_t e = hipEventQuery(q.done_ev);
    if (e == hipSuccess) {
        *done = 1;
        (void)hipEventDestroy(q.done_ev);
        v->queries.erase(it);
        return EIG_OK;
    }
    if (e == hipErrorNotReady) return EIG_OK;
    return set_error(EIG_EHIP, std::string("hipEventQuery: ") + hipGetErrorString(e));
}

int eig_server_memory(eig_server* v, size_t* budget, size_t* in_use, size_t* peak) {
    if (!v) return set_error(EIG_EINVAL, "server is NULL");
    if (budget) *budget = v->mem_size;
    if (in_use) *in_use = v->arena.used;
    if (peak) *peak = v->arena.peak;
    return EIG_OK;
}

int eig_server_pending(eig_server* v, int32_t* queued, int32_t* running) {
    if (!v) return set_error(EIG_EINVAL, "server is NULL");
    if (queued) *queued = (int32_t)v->queue.size();
    if (running) *running = (int32_t)v->groups.size();
    return EIG_OK;
}

}  // extern "C"
