// Request server: many MCMC chains submit f + g requests for data sets kept
// resident in HBM; a scheduler thread batches requests of the same data set
// into one several-beta pass over X and keeps up to n_slots launches in
// flight on n_streams streams (continuous batching: requests that arrive
// while passes run are packed into the next free slot).  Data sets are
// admitted to device memory on first use within an HBM budget, evicting the
// least recently used idle ones when needed.  Admission is asynchronous: the
// scheduler only reserves the budget; an admission thread obtains the memory
// (reusing evicted allocations, or the stream-ordered allocator) and copies
// the data set on a copy stream of its own (through pinned staging buffers
// when the source is pageable), so passes over resident data sets keep
// running while a data set is loaded, and no call synchronises the device.
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

enum { DS_OUT = 0, DS_LOADING = 1, DS_RESIDENT = 2 };

struct SDataset {
    glm_dataset_desc src;     // as given (host or device pointers)
    bool on_device = false;   // caller-owned device buffers: always resident, never evicted
    int state = DS_OUT;       // loading: budget reserved, copy in progress
    glm_dataset_desc dev{};   // device copy in use
    void* mem = nullptr;      // server allocation (host-sourced data sets)
    size_t mem_bytes = 0;     // its size
    size_t bytes = 0;         // budget charge (data_bytes)
    size_t pass_bytes = 0;    // algorithmic bytes of one pass: N (K size + 1)
    size_t held = 0;          // budget collected while waiting to be admitted
    int fresh = 0;            // passes still owed to the requests queued at admission:
                              // until they ran, the data set is not evicted
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

// Latency record in O(1) memory: counts per bucket of a 2 % geometric grid
// from 0.1 us to about 10^4 s (quantiles to within one bucket, 2 %), plus
// the exact sum for the mean.
struct LatHist {
    static constexpr int NB = 1300;
    static constexpr double LO = 0.1, STEP = 1.02;
    uint64_t cnt[NB] = {};
    uint64_t n = 0;
    double sum = 0.0;
    void add(double us) {
        int b = us <= LO ? 0 : (int)(std::log(us / LO) / std::log(STEP));
        b = std::min(std::max(b, 0), NB - 1);
        cnt[b]++;
        n++;
        sum += us;
    }
    // the geometric middle of the bucket holding the q-quantile
    double quantile(double q) const {
        if (!n) return 0.0;
        const uint64_t want = std::min(n - 1, (uint64_t)(q * (double)(n - 1))) + 1;
        uint64_t c = 0;
        for (int b = 0; b < NB; ++b) {
            c += cnt[b];
            if (c >= want) return LO * std::pow(STEP, b + 0.5);
        }
        return LO * std::pow(STEP, NB - 0.5);
    }
    void clear() { *this = LatHist(); }
};

// An allocation kept after its data set was evicted, for reuse.
struct CachedMem {
    void* p;
    size_t bytes;
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
    uint64_t wake = 0;          // bumped by every event the scheduler may wait for
    size_t resident_bytes = 0;  // budget charge of resident and loading data sets (and
                                // of what the holder has collected)
    int64_t holder = -1;        // the data set collecting budget for its admission
    size_t device_bytes = 0;    // of those, caller-owned device data sets (never evicted)
    // admission
    std::thread admit_th;
    std::condition_variable admit_cv;
    std::deque<int64_t> admit_q;        // data sets whose copy is to start, in order
    std::vector<CachedMem> cache;       // evicted allocations kept for reuse
    size_t cached_bytes = 0;
    hipStream_t copy_stream = nullptr;
    unsigned char* stage[2] = {nullptr, nullptr};   // pinned staging for pageable sources
    hipEvent_t stage_ev[2] = {nullptr, nullptr};
    hipEvent_t copy_done = nullptr;
    bool pools = false;         // stream-ordered allocator available
    // statistics
    uint64_t submitted = 0, completed = 0, cancelled = 0, failed = 0;
    uint64_t passes = 0, betas_in_passes = 0, admissions = 0, evictions = 0, launches = 0;
    uint64_t bytes_streamed = 0, bytes_admitted = 0, bytes_staged = 0;
    double admit_seconds = 0.0;
    int max_sets = 32;   // data sets per launch at most
    uint64_t hist[9] = {0};
    LatHist lat;   // submit -> completion of finished requests
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

size_t pass_bytes(const glm_dataset_desc& d) {
    return (size_t)d.N * ((size_t)d.K * elem_size(d.dtype) + 1);
}

// Evicts an idle host-sourced data set: its budget charge is released and
// its allocation kept for reuse (freeing it here would synchronise the
// device).  Called with s->mu held.
void evict(glm_server* s, SDataset& ds) {
    if (ds.mem) {
        s->cache.push_back(CachedMem{ds.mem, ds.mem_bytes});
        s->cached_bytes += ds.mem_bytes;
    }
    ds.mem = nullptr;
    ds.mem_bytes = 0;
    ds.state = DS_OUT;
    s->resident_bytes -= ds.bytes;
    s->evictions++;
}

// Called with s->mu held.  1: resident; 0: wait; -1: it can never fit
// (nothing that holds budget beside it could ever be evicted).
//
// Admission is first come, first served: one data set at a time (the
// holder) collects budget, taking free budget and evicting idle host-sourced
// data sets (those with no request queued first, least recently used first).
// When that is not enough it keeps what it took and waits: no other data set
// is admitted and no new pass starts on an evictable one (dispatch checks
// the holder) until the passes in flight finish and their data sets can be
// evicted too, so a large data set cannot be starved by smaller ones that
// keep taking the budget it frees.  A fully reserved data set is queued for
// the admission thread and counts as just used.  Once loaded it owes passes
// to the requests queued for it then (fresh): it is not evicted, and takes
// passes even while a holder waits, until those have run.
int admit(glm_server* s, int64_t id, SDataset& ds) {
    if (ds.state == DS_RESIDENT) return 1;
    if (ds.state == DS_LOADING) return 0;
    if (s->holder >= 0 && s->holder != id) return 0;
    const size_t need = ds.bytes - ds.held;
    size_t free = s->cfg.hbm_budget_bytes > s->resident_bytes
                      ? (size_t)(s->cfg.hbm_budget_bytes - s->resident_bytes)
                      : 0;
    bool busy = false;
    while (free < need) {
        SDataset* lru = nullptr;
        bool lru_wanted = true;
        busy = false;
        for (auto& kv : s->datasets) {
            SDataset& o = kv.second;
            if (&o == &ds || o.on_device || o.state == DS_OUT) continue;
            if (o.state == DS_LOADING || o.inflight > 0 || o.fresh > 0) {
                busy = true;
                continue;
            }
            auto q = s->pending.find(kv.first);
            const bool wanted = q != s->pending.end() && !q->second.empty();
            if (!lru || (lru_wanted && !wanted) ||
                (wanted == lru_wanted && o.last_use < lru->last_use)) {
                lru = &o;
                lru_wanted = wanted;
            }
        }
        if (!lru) break;
        evict(s, *lru);
        free += lru->bytes;
    }
    const size_t take = std::min(free, need);
    ds.held += take;
    s->resident_bytes += take;
    if (ds.held < ds.bytes) {
        if (!busy) {   // cannot happen when every set fits beside the device-resident ones
            s->resident_bytes -= ds.held;
            ds.held = 0;
            s->holder = -1;
            return -1;
        }
        s->holder = id;
        return 0;
    }
    ds.held = 0;   // now the data set's own charge in resident_bytes
    s->holder = -1;
    ds.last_use = ++s->use_clock;
    ds.state = DS_LOADING;
    s->admit_q.push_back(id);
    s->admit_cv.notify_all();
    return 0;
}

// Copies n bytes from a host source to device memory on the copy stream:
// directly when the source is pinned, else through the two pinned staging
// buffers (a buffer is refilled once its previous copy has finished).
constexpr size_t kStageBytes = size_t(32) << 20;

hipError_t copy_in(glm_server* s, void* dst, const void* src, size_t n, int& turn,
                   size_t& staged) {
    if (!n) return hipSuccess;
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, src);
    if (e != hipSuccess) (void)hipGetLastError();   // pageable memory on some runtimes
    const bool pinned = e == hipSuccess && attr.type == hipMemoryTypeHost;
    if (pinned) return hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s->copy_stream);
    staged += n;
    for (size_t off = 0; off < n; off += kStageBytes) {
        const size_t len = std::min(kStageBytes, n - off);
        const int b = turn++ & 1;
        e = hipEventSynchronize(s->stage_ev[b]);
        if (e != hipSuccess) return e;
        std::memcpy(s->stage[b], (const char*)src + off, len);
        e = hipMemcpyAsync((char*)dst + off, s->stage[b], len, hipMemcpyHostToDevice, s->copy_stream);
        if (e != hipSuccess) return e;
        e = hipEventRecord(s->stage_ev[b], s->copy_stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Fails every queued request of a data set (with s->mu held).
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

// The admission thread: for each data set queued by admit(), takes an
// evicted allocation that fits (at most twice the size), else releases
// cached allocations beyond the budget and allocates on the copy stream;
// copies X, y and the FP8 scales; waits for the copy; marks the data set
// resident and wakes the scheduler.
void admitter(glm_server* s) {
    (void)hipSetDevice(s->ctx->device);
    int turn = 0;
    while (true) {
        int64_t id;
        SDataset* ds;
        void* mem = nullptr;
        size_t mem_bytes = 0, need = 0;
        std::vector<CachedMem> release;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->admit_cv.wait(lk, [&] { return s->stop || !s->admit_q.empty(); });
            if (s->stop) return;   // queued requests are cancelled by the shutdown
            id = s->admit_q.front();
            s->admit_q.pop_front();
            ds = &s->datasets[id];
            const size_t es = elem_size(ds->src.dtype);
            const size_t xb_al = ((size_t)ds->src.N * ds->src.ldx * es + 255) / 256 * 256;
            const size_t yb_al = ((size_t)ds->src.N + 255) / 256 * 256;
            const size_t sb = ds->src.col_scale ? (size_t)ds->src.K * 4 : 0;
            need = xb_al + yb_al + sb + 256;
            int best = -1;
            for (int i = 0; i < (int)s->cache.size(); ++i) {
                const size_t b = s->cache[i].bytes;
                if (b >= need && b <= 2 * need && (best < 0 || b < s->cache[best].bytes)) best = i;
            }
            if (best >= 0) {
                mem = s->cache[best].p;
                mem_bytes = s->cache[best].bytes;
                s->cached_bytes -= mem_bytes;
                s->cache.erase(s->cache.begin() + best);
            }
            // keep what the server holds (resident, loading and cached) within the budget
            while (!s->cache.empty() &&
                   s->resident_bytes + s->cached_bytes > s->cfg.hbm_budget_bytes) {
                release.push_back(s->cache.back());
                s->cached_bytes -= s->cache.back().bytes;
                s->cache.pop_back();
            }
        }
        const auto t0 = Clock::now();
        size_t staged = 0;
        hipError_t e = hipSuccess;
        for (const CachedMem& c : release)
            if (e == hipSuccess) e = s->pools ? hipFreeAsync(c.p, s->copy_stream) : hipFree(c.p);
        if (e == hipSuccess && !mem) {
            e = s->pools ? hipMallocAsync(&mem, need, s->copy_stream) : hipMalloc(&mem, need);
            mem_bytes = need;
            if (e != hipSuccess) mem = nullptr;
        }
        glm_dataset_desc dev = ds->src;
        if (e == hipSuccess) {
            const size_t es = elem_size(ds->src.dtype);
            const size_t xb = (size_t)ds->src.N * ds->src.ldx * es;
            const size_t xb_al = (xb + 255) / 256 * 256;
            const size_t yb_al = ((size_t)ds->src.N + 255) / 256 * 256;
            const size_t sb = ds->src.col_scale ? (size_t)ds->src.K * 4 : 0;
            char* base = (char*)mem;
            dev.X = base;
            dev.y = (const uint8_t*)(base + xb_al);
            dev.col_scale = sb ? (const float*)(base + xb_al + yb_al) : nullptr;
            e = copy_in(s, (void*)dev.X, ds->src.X, xb, turn, staged);
            if (e == hipSuccess)
                e = copy_in(s, (void*)dev.y, ds->src.y, (size_t)ds->src.N, turn, staged);
            if (e == hipSuccess && sb)
                e = copy_in(s, (void*)dev.col_scale, ds->src.col_scale, sb, turn, staged);
            if (e == hipSuccess) e = hipEventRecord(s->copy_done, s->copy_stream);
            if (e == hipSuccess) e = hipEventSynchronize(s->copy_done);
        }
        const double sec = std::chrono::duration<double>(Clock::now() - t0).count();
        std::lock_guard<std::mutex> lk(s->mu);
        if (e != hipSuccess) {
            if (mem) {
                s->cache.push_back(CachedMem{mem, mem_bytes});
                s->cached_bytes += mem_bytes;
            }
            s->resident_bytes -= ds->bytes;
            ds->state = DS_OUT;
            s->sched_error = std::string("data set admission failed: ") + hipGetErrorString(e);
            fail_queue(s, id);
        } else {
            ds->dev = dev;
            ds->mem = mem;
            ds->mem_bytes = mem_bytes;
            ds->state = DS_RESIDENT;
            {
                const int NB = ds->mi.fn ? ds->mi.NB : 1;
                auto q = s->pending.find(id);
                const size_t nq = q == s->pending.end() ? 0 : q->second.size();
                ds->fresh = (int)((nq + NB - 1) / NB);   // 0 if nothing waits for it
            }
            s->admissions++;
            s->bytes_admitted += ds->bytes;
            s->bytes_staged += staged;
            s->admit_seconds += sec;
        }
        s->wake++;
        s->cv.notify_all();
    }
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
                s->lat.add(std::chrono::duration<double, std::micro>(now - sl.t_submit[t]).count());
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
            // while a data set waits for budget, evictable ones take no new
            // passes (their passes in flight finish and free it)
            if (s->holder >= 0 && !ds.on_device && ds.state == DS_RESIDENT && ds.fresh == 0)
                continue;
            const int a = admit(s, h.second, ds);
            if (a < 0) {
                s->sched_error = "data set can never fit the HBM budget beside the device-resident ones";
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
            if (ds.fresh > 0) ds.fresh--;
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
        s->bytes_streamed += pk.ds->pass_bytes;
        s->betas_in_passes += nb;
        s->hist[std::min(nb, 8)]++;
    }
    s->launches++;
    return true;
}

void scheduler(glm_server* s) {
    (void)hipSetDevice(s->ctx->device);
    uint64_t seen = 0;
    while (true) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            seen = s->wake;
        }
        bool progress = reap(s);
        while (dispatch(s)) progress = true;
        bool busy = false;
        for (Slot& sl : s->slots) busy |= sl.busy;
        std::unique_lock<std::mutex> lk(s->mu);
        if (s->stop && !busy && (s->queued == 0 || !s->accepting)) break;
        if (!progress) {
            if (busy)   // poll the slots' events
                s->cv.wait_for(lk, std::chrono::microseconds(5));
            else        // wait for a request, an admitted data set or the stop
                s->cv.wait_for(lk, std::chrono::milliseconds(2),
                               [&] { return s->stop || s->wake != seen; });
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
    int pools = 0;
    GLM_HIP_CHECK(hipDeviceGetAttribute(&pools, hipDeviceAttributeMemoryPoolsSupported, ctx->device));
    s->pools = pools != 0;
    GLM_HIP_CHECK(hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking));
    GLM_HIP_CHECK(hipEventCreateWithFlags(&s->copy_done, hipEventDisableTiming));
    for (int b = 0; b < 2; ++b) {
        GLM_HIP_CHECK(hipHostMalloc((void**)&s->stage[b], kStageBytes));
        GLM_HIP_CHECK(hipEventCreateWithFlags(&s->stage_ev[b], hipEventDisableTiming));
    }
    glm_server* raw = s.get();
    s->th = std::thread(scheduler, raw);
    s->admit_th = std::thread(admitter, raw);
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
    ds.pass_bytes = pass_bytes(*d);
    std::lock_guard<std::mutex> lk(s->mu);
    // Device-resident data sets are never evicted, so every data set must fit
    // beside all of them: then admission can always make room by evicting
    // idle host-sourced ones.
    if (s->device_bytes + ds.bytes > s->cfg.hbm_budget_bytes)
        GLM_FAIL(GLM_EBUDGET,
                 "glm_server_add_dataset: %zu bytes do not fit the HBM budget of %llu beside the "
                 "%zu bytes of device-resident data sets",
                 ds.bytes, (unsigned long long)s->cfg.hbm_budget_bytes, s->device_bytes);
    // plan on the device layout (16-byte alignment of the server's copy holds)
    glm_dataset_desc probe = *d;
    if (!ds.on_device) probe.X = nullptr;
    st = make_plan(s->ctx, probe, &ds.plan);
    if (st != GLM_OK) return st;
    ds.mi = multi_instance(d->dtype, ds.plan.lpr, ds.plan.cpl, s->cfg.max_beta_per_pass,
                           s->ctx->matrix_cores);
    if (ds.on_device) {
        ds.dev = *d;
        ds.state = DS_RESIDENT;
        s->resident_bytes += ds.bytes;
        s->device_bytes += ds.bytes;
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
        s->wake++;
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
        s->wake++;
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
    for (auto& kv : s->datasets) nres += kv.second.state == DS_RESIDENT;
    out->resident_datasets = nres;
    out->queue_depth = (int32_t)s->queued;
    for (int i = 0; i < 9; ++i) out->pass_width_hist[i] = s->hist[i];
    if (s->lat.n) {
        out->latency_p50_us = s->lat.quantile(0.50);
        out->latency_p99_us = s->lat.quantile(0.99);
        out->latency_mean_us = s->lat.sum / (double)s->lat.n;
    }
    out->bytes_streamed = s->bytes_streamed;
    out->bytes_admitted = s->bytes_admitted;
    out->admit_seconds = s->admit_seconds;
    out->cached_bytes = s->cached_bytes;
    out->bytes_staged = s->bytes_staged;
    return GLM_OK;
}

glm_status glm_server_reset_stats(glm_server* s) {
    clear_error();
    if (!s) GLM_FAIL(GLM_EINVAL, "glm_server_reset_stats: NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    s->submitted = s->completed = s->cancelled = s->failed = 0;
    s->passes = s->betas_in_passes = s->admissions = s->evictions = s->launches = 0;
    s->bytes_streamed = s->bytes_admitted = s->bytes_staged = 0;
    s->admit_seconds = 0.0;
    std::memset(s->hist, 0, sizeof(s->hist));
    s->lat.clear();
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
        s->wake++;
    }
    s->cv.notify_all();
    s->admit_cv.notify_all();
    if (s->th.joinable()) s->th.join();
    if (s->admit_th.joinable()) s->admit_th.join();
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
    if (s->copy_stream) {
        (void)hipStreamSynchronize(s->copy_stream);
        auto release = [&](void* p) {
            if (s->pools)
                (void)hipFreeAsync(p, s->copy_stream);
            else
                (void)hipFree(p);
        };
        for (auto& kv : s->datasets)
            if (kv.second.mem) release(kv.second.mem);
        for (const CachedMem& c : s->cache) release(c.p);
        (void)hipStreamSynchronize(s->copy_stream);
        (void)hipStreamDestroy(s->copy_stream);
    }
    for (int b = 0; b < 2; ++b) {
        if (s->stage[b]) (void)hipHostFree(s->stage[b]);
        if (s->stage_ev[b]) (void)hipEventDestroy(s->stage_ev[b]);
    }
    if (s->copy_done) (void)hipEventDestroy(s->copy_done);
    delete s;
    return GLM_OK;
}

}  // extern "C"
