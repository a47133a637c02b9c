// Request server: many MCMC chains submit f + g requests for data sets kept
// resident in HBM; a scheduler thread batches requests of the same data set
// into one several-beta pass over X and keeps up to n_slots launches in
// flight on n_streams streams (continuous batching: requests that arrive
// while passes run are packed into the next free slot).  Data sets are
// admitted to device memory on first use within an HBM budget, evicting the
// least recently used idle ones when needed.
//
// The offload cost of a host-driven call is the reason for this design
// (Sec. 4.5): one transfer + launch pays for up to NB evaluations.  A small
// data set's pass is bound by latency (a few dependent memory round trips
// and the cross-block merge), not by its bytes, so the passes of every data
// set of one kernel geometry that has requests queued share one launch (a
// fleet launch): each keeps its own blocks, rows and merge order, so its
// results are bitwise those of a launch of its own.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <thread>
#include <unordered_map>

#include "fg_kernel.hpp"
#include "runtime.hpp"

using Clock = std::chrono::steady_clock;

namespace glmrt {
namespace {

struct Request {
    uint64_t ticket;
    int64_t ds;
    double prec;
    bool has_mean;
    std::vector<double> beta, mean;
    Clock::time_point t_submit;
};

enum { R_PENDING = 0, R_DONE = 1, R_CANCELLED = 2, R_FAILED = 3 };

struct Result {
    int state = R_PENDING;
    double f = 0.0;
    std::vector<double> g;
};

struct SDataset {
    glm_dataset_desc src;     // as given (host or device pointers)
    bool on_device = false;   // caller-owned device buffers: always resident, never evicted
    bool resident = false;
    glm_dataset_desc dev{};   // device copy in use
    void* mem = nullptr;      // server allocation (host-sourced data sets)
    size_t bytes = 0;
    uint64_t last_use = 0;
    int inflight = 0;
    Plan plan;
    MultiInst mi;             // several-beta instance (or plan.fn with NB = 1)
};

// One data set's pass within a launch.
struct SlotJob {
    int64_t ds;
    int nb;
    int K;
    size_t out_off;   // doubles into the slot's result area
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<SlotJob> jobs;
    std::vector<uint64_t> tickets;            // in job order
    std::vector<Clock::time_point> t_submit;
    // staging in: [fleet jobs][block -> job table][per job: betas nb x K,
    // precisions nb, means nb x K if any request has one]; out: per job
    // nb x (K + 1) doubles, written by the kernel into coherent pinned host
    // memory (no device-to-host copy per launch)
    unsigned char* h_in = nullptr;
    unsigned char* d_in = nullptr;
    double* h_out = nullptr;
    size_t cap_in = 0, cap_out = 0;   // bytes, doubles
    Scratch scratch;
};

}  // namespace
}  // namespace glmrt

using namespace glmrt;

struct glm_server {
    glm_ctx* ctx = nullptr;
    glm_server_config cfg{};
    std::thread th;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    bool accepting = true;
    std::map<int64_t, std::deque<Request>> pending;   // queued requests per data set
    size_t queued = 0;
    std::unordered_map<uint64_t, Result> results;
    std::map<int64_t, SDataset> datasets;   // references stay valid as sets are added
    int64_t next_ds = 1;
    std::atomic<uint64_t> next_ticket{1};
    std::vector<Slot> slots;
    std::vector<hipStream_t> streams;
    uint64_t use_clock = 0;
    size_t resident_bytes = 0;
    // statistics
    uint64_t submitted = 0, completed = 0, cancelled = 0, failed = 0;
    uint64_t passes = 0, betas_in_passes = 0, admissions = 0, evictions = 0, launches = 0;
    int max_sets = 32;   // data sets per launch at most
    uint64_t hist[9] = {0};
    std::vector<float> lat_us;   // submit -> completion of finished requests
    std::string sched_error;
};

namespace glmrt {
namespace {

size_t data_bytes(const glm_dataset_desc& d) {
    const size_t es = elem_size(d.dtype);
    size_t b = (size_t)d.N * d.ldx * es + (size_t)d.N;
    if (d.col_scale) b += (size_t)d.K * 4;
    return b;
}

// Frees the server's copy of an idle host-sourced data set.
void evict(glm_server* s, SDataset& ds) {
    if (ds.mem) (void)hipFree(ds.mem);
    ds.mem = nullptr;
    ds.resident = false;
    s->resident_bytes -= ds.bytes;
    s->evictions++;
}

// 1: resident now, 0: must wait (budget held by busy data sets), -1: error.
int admit(glm_server* s, SDataset& ds) {
    if (ds.resident) return 1;
    while (s->resident_bytes + ds.bytes > s->cfg.hbm_budget_bytes) {
        SDataset* lru = nullptr;
        for (auto& kv : s->datasets) {
            SDataset& o = kv.second;
            if (o.resident && !o.on_device && o.inflight == 0 && (!lru || o.last_use < lru->last_use))
                lru = &o;
        }
        if (!lru) return 0;
        evict(s, *lru);
    }
    const size_t es = elem_size(ds.src.dtype);
    const size_t xb = (size_t)ds.src.N * ds.src.ldx * es;
    const size_t xb_al = (xb + 255) / 256 * 256;
    const size_t yb_al = ((size_t)ds.src.N + 255) / 256 * 256;
    const size_t sb = ds.src.col_scale ? (size_t)ds.src.K * 4 : 0;
    void* mem = nullptr;
    if (hipMalloc(&mem, xb_al + yb_al + sb + 256) != hipSuccess) {
        s->sched_error = "device allocation for a data set failed";
        return -1;
    }
    char* base = (char*)mem;
    ds.dev = ds.src;
    ds.dev.X = base;
    ds.dev.y = (const uint8_t*)(base + xb_al);
    ds.dev.col_scale = sb ? (const float*)(base + xb_al + yb_al) : nullptr;
    hipError_t e = hipSuccess;
    if (xb) e = hipMemcpy((void*)ds.dev.X, ds.src.X, xb, hipMemcpyHostToDevice);
    if (e == hipSuccess && ds.src.N) e = hipMemcpy((void*)ds.dev.y, ds.src.y, ds.src.N, hipMemcpyHostToDevice);
    if (e == hipSuccess && sb) e = hipMemcpy((void*)ds.dev.col_scale, ds.src.col_scale, sb, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipFree(mem);
        s->sched_error = hipGetErrorString(e);
        return -1;
    }
    ds.mem = mem;
    ds.resident = true;
    s->resident_bytes += ds.bytes;
    s->admissions++;
    return 1;
}

// Grows the slot's staging areas and scratch to at least the given sizes
// (with headroom, so that growth is rare; the slot is idle when called).
bool ensure_slot_capacity(Slot& sl, size_t in_bytes, size_t out_doubles, size_t np, size_t ng,
                          size_t nc) {
    if (sl.cap_in < in_bytes) {
        const size_t cap = std::max(in_bytes + in_bytes / 2, (size_t)1 << 16);
        if (sl.h_in) (void)hipHostFree(sl.h_in);
        if (sl.d_in) (void)hipFree(sl.d_in);
        sl.h_in = sl.d_in = nullptr;
        sl.cap_in = 0;
        if (hipHostMalloc((void**)&sl.h_in, cap) != hipSuccess) return false;
        if (hipMalloc((void**)&sl.d_in, cap) != hipSuccess) return false;
        sl.cap_in = cap;
    }
    if (sl.cap_out < out_doubles) {
        const size_t cap = std::max(out_doubles + out_doubles / 2, (size_t)4096);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        sl.h_out = nullptr;
        sl.cap_out = 0;
        if (hipHostMalloc((void**)&sl.h_out, cap * 8, hipHostMallocCoherent) != hipSuccess)
            return false;
        sl.cap_out = cap;
    }
    Scratch& sc = sl.scratch;
    if (!sc.base || sc.cap_partials < np || sc.cap_gpart < ng || sc.cap_counters < nc) {
        if (sc.base) (void)hipFree(sc.base);
        sc = Scratch{};
        np += np / 2;
        ng += ng / 2;
        nc += nc / 2 + 64;
        const size_t bytes = (np + ng) * 8 + nc * 4;
        if (hipMalloc(&sc.base, bytes) != hipSuccess) return false;
        sc.partials = (double*)sc.base;
        sc.gpart = sc.partials + np;
        sc.counters = (unsigned*)(sc.gpart + ng);
        sc.cap_partials = np;
        sc.cap_gpart = ng;
        sc.cap_counters = nc;
        // tickets start at zero; every launch leaves the ones it used at zero
        if (hipMemsetAsync(sc.counters, 0, nc * 4, sl.stream) != hipSuccess) return false;
    }
    return true;
}

// Completes finished launches; returns true if any finished.
bool reap(glm_server* s) {
    bool any = false;
    for (Slot& sl : s->slots) {
        if (!sl.busy || hipEventQuery(sl.done) != hipSuccess) continue;
        const Clock::time_point now = Clock::now();
        std::lock_guard<std::mutex> lk(s->mu);
        size_t t = 0;
        for (const SlotJob& j : sl.jobs) {
            const double* o = sl.h_out + j.out_off;
            for (int i = 0; i < j.nb; ++i, ++t) {
                Result& r = s->results[sl.tickets[t]];
                r.state = R_DONE;
                r.f = o[(size_t)i * (j.K + 1)];
                r.g.assign(o + (size_t)i * (j.K + 1) + 1, o + (size_t)(i + 1) * (j.K + 1));
                s->lat_us.push_back(
                    (float)std::chrono::duration<double, std::micro>(now - sl.t_submit[t]).count());
            }
            s->datasets[j.ds].inflight--;
        }
        s->completed += t;
        sl.busy = false;
        any = true;
    }
    if (any) s->cv.notify_all();
    return any;
}

// Fails every queued request of a data set (its admission failed).
void fail_queue(glm_server* s, int64_t dsid) {
    auto& q = s->pending[dsid];
    for (Request& r : q) {
        s->results[r.ticket].state = R_FAILED;
        s->failed++;
    }
    s->queued -= q.size();
    q.clear();
    s->cv.notify_all();
}

// A data set chosen for a launch with the requests it takes.
struct Pick {
    int64_t id;
    SDataset* ds;
    std::vector<Request> reqs;
};

// Starts at most one launch on a free slot; returns true if it did (or if it
// failed requests).  The data set whose oldest queued request is oldest goes
// first (FIFO across data sets); the other data sets of its kernel geometry
// with queued requests join it in the same order, up to max_sets_per_pass;
// data sets that must wait for memory are skipped.
bool dispatch(glm_server* s) {
    Slot* sl = nullptr;
    for (Slot& c : s->slots)
        if (!c.busy) {
            sl = &c;
            break;
        }
    if (!sl) return false;
    std::vector<Pick> picks;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->queued == 0) return false;
        std::vector<std::pair<Clock::time_point, int64_t>> heads;
        for (auto& kv : s->pending)
            if (!kv.second.empty()) heads.push_back({kv.second.front().t_submit, kv.first});
        std::sort(heads.begin(), heads.end());
        const void* fleet = nullptr;
        bool failed = false;
        for (auto& h : heads) {
            SDataset& ds = s->datasets[h.second];
            if (!picks.empty() && !fleet) break;
            if (!picks.empty() && ds.mi.fleet != fleet) continue;
            const int a = admit(s, ds);
            if (a < 0) {
                fail_queue(s, h.second);
                failed = true;
                continue;
            }
            if (a == 0) continue;
            const int NB = ds.mi.fn ? ds.mi.NB : 1;
            Pick pk{h.second, &ds, {}};
            auto& q = s->pending[h.second];
            while (!q.empty() && (int)pk.reqs.size() < NB) {
                pk.reqs.push_back(std::move(q.front()));
                q.pop_front();
            }
            s->queued -= pk.reqs.size();
            ds.inflight++;   // also keeps it from being evicted by a later admission
            ds.last_use = ++s->use_clock;
            if (picks.empty()) fleet = s->max_sets > 1 ? ds.mi.fleet : nullptr;
            picks.push_back(std::move(pk));
            if ((int)picks.size() >= s->max_sets) break;
        }
        if (picks.empty()) return failed;
    }
    // small grids first: their dependent round trips start at once
    std::stable_sort(picks.begin(), picks.end(), [](const Pick& a, const Pick& b) {
        return a.ds->plan.nblocks < b.ds->plan.nblocks;
    });
    const int nj = (int)picks.size();
    const bool use_fleet = nj > 1;
    const SDataset& d0 = *picks[0].ds;
    const int NB = d0.mi.fn ? d0.mi.NB : 1;

    // layout of the staging and scratch areas
    std::vector<size_t> in_off(nj), out_off(nj), p_off(nj), g_off(nj), c_off(nj);
    std::vector<bool> has_mean(nj, false);
    int grid = 0;
    for (int j = 0; j < nj; ++j) grid += picks[j].ds->plan.nblocks;
    size_t in_bytes = use_fleet ? (size_t)nj * sizeof(glmk::FleetJob) : 0;
    if (use_fleet) in_bytes += ((size_t)grid * 2 + 7) / 8 * 8;
    size_t out_d = 0, np = 0, ng = 0, nc = 0;
    for (int j = 0; j < nj; ++j) {
        const Pick& pk = picks[j];
        const int K = pk.ds->src.K, nb = (int)pk.reqs.size();
        for (const Request& r : pk.reqs) has_mean[j] = has_mean[j] || r.has_mean;
        in_off[j] = in_bytes;
        in_bytes += ((size_t)nb * K + nb + (has_mean[j] ? (size_t)nb * K : 0)) * 8;
        out_off[j] = out_d;
        out_d += (size_t)nb * (K + 1);
        size_t a, b, c;
        scratch_need(pk.ds->plan, K, NB, &a, &b, &c);
        p_off[j] = np;
        g_off[j] = ng;
        c_off[j] = nc;
        np += a;
        ng += b;
        nc += c;
    }
    bool ok = ensure_slot_capacity(*sl, in_bytes, out_d, np, ng, nc);
    if (ok) {
        unsigned char* h = sl->h_in;
        std::vector<glmk::FgParams> prm(nj);
        for (int j = 0; j < nj; ++j) {
            const Pick& pk = picks[j];
            const int K = pk.ds->src.K, nb = (int)pk.reqs.size();
            double* hb = (double*)(h + in_off[j]);
            double* hp = hb + (size_t)nb * K;
            double* hm = hp + nb;
            for (int i = 0; i < nb; ++i) {
                const Request& r = pk.reqs[i];
                std::memcpy(hb + (size_t)i * K, r.beta.data(), K * 8);
                hp[i] = r.prec;
                if (has_mean[j]) {
                    if (r.has_mean)
                        std::memcpy(hm + (size_t)i * K, r.mean.data(), K * 8);
                    else
                        std::fill(hm + (size_t)i * K, hm + (size_t)(i + 1) * K, 0.0);
                }
            }
            const double* db = (const double*)(sl->d_in + in_off[j]);
            fused_params(pk.ds->dev, pk.ds->plan, NB, db, has_mean[j] ? db + (size_t)nb * K + nb : nullptr,
                         db + (size_t)nb * K, 0.0, nb, sl->h_out + out_off[j],
                         sl->scratch.partials + p_off[j], sl->scratch.gpart + g_off[j],
                         sl->scratch.counters + c_off[j], nullptr, nullptr, &prm[j]);
        }
        if (use_fleet) {
            glmk::FleetJob* fj = (glmk::FleetJob*)h;
            uint16_t* bj = (uint16_t*)(h + (size_t)nj * sizeof(glmk::FleetJob));
            int b = 0;
            for (int j = 0; j < nj; ++j) {
                fj[j].p = prm[j];
                fj[j].blk0 = b;
                fj[j].pad_ = 0;
                for (int k = 0; k < prm[j].nblocks; ++k) bj[b++] = (uint16_t)j;
            }
        }
        ok = hipMemcpyAsync(sl->d_in, h, in_bytes, hipMemcpyHostToDevice, sl->stream) == hipSuccess;
        if (ok) {
            if (use_fleet) {
                ok = launch_fleet(d0.mi.fleet, grid, d0.mi.wpb, (const glmk::FleetJob*)sl->d_in,
                                  (const uint16_t*)(sl->d_in + (size_t)nj * sizeof(glmk::FleetJob)),
                                  sl->stream) == GLM_OK;
            } else {
                const void* fn = d0.mi.fn ? d0.mi.fn : d0.plan.fn;
                const int wpb = d0.mi.fn ? d0.mi.wpb : d0.plan.wpb;
                void* args[] = {&prm[0]};
                ok = hipLaunchKernel(fn, dim3(d0.plan.nblocks), dim3(wpb * 64), args, 0,
                                     sl->stream) == hipSuccess;
            }
        }
        if (ok) ok = hipEventRecord(sl->done, sl->stream) == hipSuccess;
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (!ok) {
        for (Pick& pk : picks) {
            for (const Request& r : pk.reqs) s->results[r.ticket].state = R_FAILED;
            s->failed += pk.reqs.size();
            pk.ds->inflight--;
        }
        s->sched_error = "launch failed";
        s->cv.notify_all();
        return true;
    }
    sl->busy = true;
    sl->jobs.clear();
    sl->tickets.clear();
    sl->t_submit.clear();
    for (int j = 0; j < nj; ++j) {
        const Pick& pk = picks[j];
        const int nb = (int)pk.reqs.size();
        sl->jobs.push_back(SlotJob{pk.id, nb, pk.ds->src.K, out_off[j]});
        for (const Request& r : pk.reqs) {
            sl->tickets.push_back(r.ticket);
            sl->t_submit.push_back(r.t_submit);
        }
        s->passes++;
        s->betas_in_passes += nb;
        s->hist[std::min(nb, 8)]++;
    }
    s->launches++;
    return true;
}

void scheduler(glm_server* s) {
    (void)hipSetDevice(s->ctx->device);
    while (true) {
        bool progress = reap(s);
        while (dispatch(s)) progress = true;
        bool busy = false;
        for (Slot& sl : s->slots) busy |= sl.busy;
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && !busy && (s->queued == 0 || !s->accepting)) break;
        if (!progress) {
            if (busy)
                s->cv.wait_for(lk, std::chrono::microseconds(5));
            else
                s->cv.wait_for(lk, std::chrono::milliseconds(2),
                               [&] { return s->stop || s->queued > 0; });
        }
    }
}

}  // namespace
}  // namespace glmrt

extern "C" {

glm_status glm_server_create(glm_ctx* ctx, const glm_server_config* cfg, glm_server** out) {
    clear_error();
    if (!ctx || !cfg || !out) GLM_FAIL(GLM_EINVAL, "glm_server_create: NULL argument");
    *out = nullptr;
    if (cfg->max_beta_per_pass < 1 || cfg->n_streams < 1 || cfg->n_slots < 1 || cfg->queue_capacity < 1)
        GLM_FAIL(GLM_EINVAL, "glm_server_create: counts must be >= 1");
    if (cfg->max_sets_per_pass < 0 || cfg->max_sets_per_pass > 256)
        GLM_FAIL(GLM_EINVAL, "glm_server_create: max_sets_per_pass = %d not in 0..256",
                 cfg->max_sets_per_pass);
    glm_status st = use_device(ctx);
    if (st != GLM_OK) return st;
    std::unique_ptr<glm_server> s(new glm_server);
    s->ctx = ctx;
    s->cfg = *cfg;
    s->max_sets = cfg->max_sets_per_pass ? cfg->max_sets_per_pass : 32;
    s->streams.resize(cfg->n_streams);
    for (auto& st_ : s->streams) GLM_HIP_CHECK(hipStreamCreateWithFlags(&st_, hipStreamNonBlocking));
    s->slots.resize(cfg->n_slots);
    for (int i = 0; i < cfg->n_slots; ++i) {
        s->slots[i].stream = s->streams[i % cfg->n_streams];
        GLM_HIP_CHECK(hipEventCreateWithFlags(&s->slots[i].done, hipEventDisableTiming));
    }
    glm_server* raw = s.get();
    s->th = std::thread(scheduler, raw);
    *out = s.release();
    return GLM_OK;
}

glm_status glm_server_add_dataset(glm_server* s, const glm_dataset_desc* d, int32_t on_device,
                                  glm_dataset_id* out) {
    clear_error();
    if (!s || !d || !out) GLM_FAIL(GLM_EINVAL, "glm_server_add_dataset: NULL argument");
    glm_status st = validate_desc(*d);
    if (st != GLM_OK) return st;
    SDataset ds;
    ds.src = *d;
    ds.on_device = on_device != 0;
    ds.bytes = data_bytes(*d);
    std::lock_guard<std::mutex> lk(s->mu);
    if (ds.bytes > s->cfg.hbm_budget_bytes ||
        (ds.on_device && s->resident_bytes + ds.bytes > s->cfg.hbm_budget_bytes))
        GLM_FAIL(GLM_EBUDGET, "glm_server_add_dataset: %zu bytes exceed the HBM budget", ds.bytes);
    // plan on the device layout (16-byte alignment of the server's copy holds)
    glm_dataset_desc probe = *d;
    if (!ds.on_device) probe.X = nullptr;
    st = make_plan(s->ctx, probe, &ds.plan);
    if (st != GLM_OK) return st;
    ds.mi = multi_instance(d->dtype, ds.plan.lpr, ds.plan.cpl, s->cfg.max_beta_per_pass);
    if (ds.on_device) {
        ds.dev = *d;
        ds.resident = true;
        s->resident_bytes += ds.bytes;
    }
    const int64_t id = s->next_ds++;
    s->datasets[id] = ds;
    *out = id;
    return GLM_OK;
}

glm_status glm_server_submit(glm_server* s, glm_dataset_id ds, const double* beta_host, double prec,
                             const double* mean_host, uint64_t* ticket) {
    clear_error();
    if (!s || !beta_host || !ticket) GLM_FAIL(GLM_EINVAL, "glm_server_submit: NULL argument");
    if (!(prec >= 0.0)) GLM_FAIL(GLM_EINVAL, "glm_server_submit: prior precision < 0");
    Request r;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->accepting) GLM_FAIL(GLM_ECANCELLED, "glm_server_submit: server is shutting down");
        auto it = s->datasets.find(ds);
        if (it == s->datasets.end())
            GLM_FAIL(GLM_ENOTFOUND, "glm_server_submit: unknown data set %lld", (long long)ds);
        if ((int64_t)s->queued >= s->cfg.queue_capacity)
            GLM_FAIL(GLM_EAGAIN, "glm_server_submit: request queue full");
        const int K = it->second.src.K;
        r.beta.assign(beta_host, beta_host + K);
        r.has_mean = mean_host != nullptr;
        if (mean_host) r.mean.assign(mean_host, mean_host + K);
        r.ds = ds;
        r.prec = prec;
        r.ticket = s->next_ticket++;
        r.t_submit = Clock::now();
        s->results[r.ticket] = Result{};
        *ticket = r.ticket;
        s->pending[ds].push_back(std::move(r));
        s->queued++;
        s->submitted++;
    }
    s->cv.notify_all();
    return GLM_OK;
}

glm_status glm_server_submit_many(glm_server* s, int32_t n, const glm_dataset_id* ds,
                                  const double* const* betas, const double* precs, uint64_t* tickets) {
    clear_error();
    if (!s || n < 0 || (n > 0 && (!ds || !betas || !precs || !tickets)))
        GLM_FAIL(GLM_EINVAL, "glm_server_submit_many: bad argument");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (!s->accepting) GLM_FAIL(GLM_ECANCELLED, "glm_server_submit_many: server is shutting down");
        if ((int64_t)s->queued + n > s->cfg.queue_capacity)
            GLM_FAIL(GLM_EAGAIN, "glm_server_submit_many: request queue full");
        for (int i = 0; i < n; ++i) {
            auto it = s->datasets.find(ds[i]);
            if (it == s->datasets.end())
                GLM_FAIL(GLM_ENOTFOUND, "glm_server_submit_many: unknown data set %lld", (long long)ds[i]);
            if (!betas[i] || !(precs[i] >= 0.0)) GLM_FAIL(GLM_EINVAL, "glm_server_submit_many: request %d", i);
        }
        const Clock::time_point now = Clock::now();
        for (int i = 0; i < n; ++i) {
            const int K = s->datasets[ds[i]].src.K;
            Request r;
            r.beta.assign(betas[i], betas[i] + K);
            r.has_mean = false;
            r.ds = ds[i];
            r.prec = precs[i];
            r.ticket = s->next_ticket++;
            r.t_submit = now;
            s->results[r.ticket] = Result{};
            tickets[i] = r.ticket;
            s->pending[ds[i]].push_back(std::move(r));
        }
        s->queued += n;
        s->submitted += n;
    }
    s->cv.notify_all();
    return GLM_OK;
}

glm_status glm_server_wait_many(glm_server* s, int32_t n, const uint64_t* tickets, double* f_out) {
    clear_error();
    if (!s || n < 0 || (n > 0 && !tickets)) GLM_FAIL(GLM_EINVAL, "glm_server_wait_many: bad argument");
    glm_status first = GLM_OK;
    std::unique_lock<std::mutex> lk(s->mu);
    for (int i = 0; i < n; ++i) {
        while (true) {
            auto it = s->results.find(tickets[i]);
            if (it == s->results.end() || it->second.state != R_PENDING) break;
            s->cv.wait_for(lk, std::chrono::milliseconds(1));
        }
        auto it = s->results.find(tickets[i]);
        if (it == s->results.end()) {
            if (first == GLM_OK) {
                first = GLM_ENOTFOUND;
                set_error("glm_server_wait_many: unknown ticket %llu", (unsigned long long)tickets[i]);
            }
            if (f_out) f_out[i] = NAN;
            continue;
        }
        const int state = it->second.state;
        if (f_out) f_out[i] = state == R_DONE ? it->second.f : NAN;
        if (state != R_DONE && first == GLM_OK) {
            first = state == R_CANCELLED ? GLM_ECANCELLED : GLM_EHIP;
            set_error("glm_server_wait_many: request %d did not finish", i);
        }
        s->results.erase(it);
    }
    return first;
}

static glm_status take_result(glm_server* s, uint64_t ticket, double* f, double* g_host) {
    auto it = s->results.find(ticket);
    if (it == s->results.end()) GLM_FAIL(GLM_ENOTFOUND, "glm_server: unknown ticket %llu", (unsigned long long)ticket);
    Result& r = it->second;
    if (r.state == R_PENDING) return GLM_PENDING;
    const int state = r.state;
    if (state == R_DONE) {
        if (f) *f = r.f;
        if (g_host) std::memcpy(g_host, r.g.data(), r.g.size() * 8);
    }
    s->results.erase(it);
    if (state == R_CANCELLED) GLM_FAIL(GLM_ECANCELLED, "glm_server: request cancelled by shutdown");
    if (state == R_FAILED) GLM_FAIL(GLM_EHIP, "glm_server: request failed: %s", s->sched_error.c_str());
    return GLM_OK;
}

glm_status glm_server_poll(glm_server* s, uint64_t ticket, double* f, double* g_host) {
    clear_error();
    if (!s) GLM_FAIL(GLM_EINVAL, "glm_server_poll: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    return take_result(s, ticket, f, g_host);
}

glm_status glm_server_wait(glm_server* s, uint64_t ticket, double* f, double* g_host) {
    clear_error();
    if (!s) GLM_FAIL(GLM_EINVAL, "glm_server_wait: NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    while (true) {
        auto it = s->results.find(ticket);
        if (it == s->results.end() || it->second.state != R_PENDING) break;
        s->cv.wait_for(lk, std::chrono::milliseconds(1));
    }
    return take_result(s, ticket, f, g_host);
}

glm_status glm_server_stats(glm_server* s, glm_server_metrics* out) {
    clear_error();
    if (!s || !out) GLM_FAIL(GLM_EINVAL, "glm_server_stats: NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    std::memset(out, 0, sizeof(*out));
    out->submitted = s->submitted;
    out->completed = s->completed;
    out->cancelled = s->cancelled;
    out->failed = s->failed;
    out->passes = s->passes;
    out->launches = s->launches;
    out->betas_in_passes = s->betas_in_passes;
    out->admissions = s->admissions;
    out->evictions = s->evictions;
    out->resident_bytes = s->resident_bytes;
    int nres = 0;
    for (auto& kv : s->datasets) nres += kv.second.resident;
    out->resident_datasets = nres;
    out->queue_depth = (int32_t)s->queued;
    for (int i = 0; i < 9; ++i) out->pass_width_hist[i] = s->hist[i];
    if (!s->lat_us.empty()) {
        std::vector<float> v = s->lat_us;
        auto pct = [&](double q) {
            const size_t k = std::min(v.size() - 1, (size_t)(q * (v.size() - 1)));
            std::nth_element(v.begin(), v.begin() + k, v.end());
            return (double)v[k];
        };
        out->latency_p50_us = pct(0.50);
        out->latency_p99_us = pct(0.99);
        double sum = 0;
        for (float x : s->lat_us) sum += x;
        out->latency_mean_us = sum / s->lat_us.size();
    }
    return GLM_OK;
}

glm_status glm_server_reset_stats(glm_server* s) {
    clear_error();
    if (!s) GLM_FAIL(GLM_EINVAL, "glm_server_reset_stats: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    s->submitted = s->completed = s->cancelled = s->failed = 0;
    s->passes = s->betas_in_passes = s->admissions = s->evictions = s->launches = 0;
    std::memset(s->hist, 0, sizeof(s->hist));
    s->lat_us.clear();
    return GLM_OK;
}

glm_status glm_server_shutdown(glm_server* s) {
    clear_error();
    if (!s) GLM_FAIL(GLM_EINVAL, "glm_server_shutdown: NULL server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->accepting = false;
        for (auto& kv : s->pending) {
            for (Request& r : kv.second) {
                s->results[r.ticket].state = R_CANCELLED;
                s->cancelled++;
            }
            kv.second.clear();
        }
        s->queued = 0;
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    return GLM_OK;
}

glm_status glm_server_destroy(glm_server* s) {
    clear_error();
    if (!s) return GLM_OK;
    glm_server_shutdown(s);
    (void)hipSetDevice(s->ctx->device);
    for (Slot& sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.h_in) (void)hipHostFree(sl.h_in);
        if (sl.h_out) (void)hipHostFree(sl.h_out);
        if (sl.d_in) (void)hipFree(sl.d_in);
        if (sl.scratch.base) (void)hipFree(sl.scratch.base);
    }
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    for (auto& kv : s->datasets)
        if (kv.second.mem) (void)hipFree(kv.second.mem);
    delete s;
    return GLM_OK;
}

}  // extern "C"
