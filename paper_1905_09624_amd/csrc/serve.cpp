// Continuous-batching server over a resident COBS index.
//
// The score budget is one device pool of per-query score buffers (one
// query's counts over every document, the memory a query split over several
// work items accumulates into).  Requests are copied at submit time and
// admitted in arrival order while a buffer is free; each holds its buffer
// until its result is ready.  Each of num_streams workers owns a HIP stream
// and a workspace sized at start for the batch limits; a free worker takes
// every admitted request that shares the head request's options (K, top-k),
// up to the batch limits, and runs them as one device batch.  While one
// worker's batch is on the GPU the next worker collects the requests that
// arrived meanwhile, so new arrivals join the next batch instead of waiting
// for a queue to drain.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.h"

using namespace cobs;

namespace {

struct Request {
    uint64_t ticket = 0;
    std::vector<uint8_t> bytes;
    uint32_t k_num = 0, k_den = 1, topk = 0;
    uint64_t arrival_ns = 0, done_ns = 0;
    uint32_t slot = 0;                 // score buffer held while admitted
    bool done = false;
    cobs_status status = COBS_OK;
    std::string error;
    cobs_hits hits{};
};

}  // namespace

struct cobs_server {
    cobs_index *ix = nullptr;
    cobs_serve_opts opts{};
    DevBuf pool;                       // n_slots score buffers, zero between batches
    uint64_t n_slots = 0;
    std::vector<uint32_t> free_slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> waiting;    // not yet admitted
    std::deque<std::shared_ptr<Request>> ready;      // admitted, not yet batched
    std::unordered_map<uint64_t, std::shared_ptr<Request>> all;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams;
    std::vector<Workspace *> spaces;
    uint64_t next_ticket = 1;
    bool stopping = false;
    uint64_t submitted = 0, completed = 0, rejected = 0, cancelled = 0, batches = 0, lookups = 0;
    uint64_t first_arrival = ~0ull, last_done = 0;
    std::vector<uint64_t> latencies;

    void admit_locked()
    {
        while (!waiting.empty() && !free_slots.empty()) {
            waiting.front()->slot = free_slots.back();
            free_slots.pop_back();
            ready.push_back(waiting.front());
            waiting.pop_front();
        }
    }

    void worker(int lane);
};

void cobs_server::worker(int lane)
{
    (void)hipSetDevice(ix->device);
    hipStream_t st = streams[lane];
    Workspace *ws = spaces[lane];
    const uint32_t q = ix->prm.q;
    std::vector<std::shared_ptr<Request>> batch;
    std::vector<uint8_t> bytes;
    std::vector<uint64_t> off;
    std::vector<uint32_t> slots;
    for (;;) {
        batch.clear();
        {
            std::unique_lock<std::mutex> lk(mu);
            // while stopping, requests still waiting for a score buffer are
            // admitted when a batch in flight frees one (its worker then
            // notifies): sleep until then instead of polling
            cv_work.wait(lk, [&] { return !ready.empty() || (stopping && waiting.empty()); });
            if (ready.empty()) return;
            const Request &head = *ready.front();
            const uint32_t kn = head.k_num, kd = head.k_den, tk = head.topk;
            uint64_t windows = 0;
            for (auto it = ready.begin(); it != ready.end() && batch.size() < opts.max_batch_queries;) {
                Request &r = **it;
                const uint64_t w = r.bytes.size() >= q ? r.bytes.size() - q + 1 : 0;
                if (r.k_num == kn && r.k_den == kd && r.topk == tk &&
                    (batch.empty() || windows + w <= opts.max_batch_terms)) {
                    windows += w;
                    batch.push_back(*it);
                    it = ready.erase(it);
                } else {
                    ++it;
                }
            }
        }
        bytes.clear();
        off.assign(1, 0);
        slots.clear();
        for (auto &r : batch) {
            bytes.insert(bytes.end(), r->bytes.begin(), r->bytes.end());
            off.push_back(bytes.size());
            slots.push_back(r->slot);
        }
        BatchSpec spec;
        spec.bytes = bytes.data();
        spec.q_off = off.data();
        spec.n = (uint32_t)batch.size();
        spec.mem = COBS_MEM_HOST;
        spec.k_num = batch[0]->k_num;
        spec.k_den = batch[0]->k_den;
        spec.topk = batch[0]->topk;
        spec.score_bits = opts.score_bits;
        spec.slots = slots.data();
        spec.accum = pool.as<uint32_t>();
        BatchOut bo;
        cobs_status s = run_batch(ix, *ws, spec, st, bo);
        std::string err = s == COBS_OK ? "" : cobs_last_error();
        std::vector<cobs_status> per(batch.size(), s);
        if (s == COBS_OK)
            for (size_t i = 0; i < batch.size(); ++i)
                per[i] = make_hits(bo, (uint32_t)i, 1, &batch[i]->hits);
        const uint64_t t = now_ns();
        {
            std::lock_guard<std::mutex> lk(mu);
            ++batches;
            for (size_t i = 0; i < batch.size(); ++i) {
                Request &r = *batch[i];
                r.status = per[i];
                r.error = err;
                r.done = true;
                r.done_ns = t;
                free_slots.push_back(r.slot);
                if (per[i] == COBS_OK) {
                    ++completed;
                    lookups += r.hits.num_terms;
                    latencies.push_back(t > r.arrival_ns ? t - r.arrival_ns : 0);
                    last_done = std::max(last_done, t);
                }
            }
            admit_locked();
        }
        cv_done.notify_all();
        cv_work.notify_all();
    }
}

extern "C" {

cobs_status cobs_serve(cobs_index *ix, const cobs_serve_opts *opts, cobs_server **out)
{
    if (!ix || !out) return set_error(COBS_EINVAL, "NULL argument");
    *out = nullptr;
    auto *s = new cobs_server();
    s->ix = ix;
    if (opts) s->opts = *opts;
    if (s->opts.num_streams == 0) s->opts.num_streams = 2;
    if (s->opts.num_streams > 8) {
        delete s;
        return set_error(COBS_EINVAL, "num_streams must be <= 8");
    }
    if (s->opts.max_batch_queries == 0) s->opts.max_batch_queries = 4096;
    if (s->opts.max_batch_terms == 0) s->opts.max_batch_terms = 1ull << 23;
    if (s->opts.score_bits == 0) s->opts.score_bits = 32;
    if (s->opts.score_bits != 16 && s->opts.score_bits != 32) {
        delete s;
        return set_error(COBS_EINVAL, "score_bits must be 16 or 32");
    }
    (void)hipSetDevice(ix->device);
    const uint64_t slot_bytes = std::max<uint64_t>(ix->acc_words * 4, 4);
    uint64_t budget = s->opts.score_budget_bytes;
    if (budget == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 1ull << 32;
        budget = std::min<uint64_t>(4096 * slot_bytes, fr / 4);
    }
    s->n_slots = std::min<uint64_t>(budget / slot_bytes, 1u << 30);
    if (s->opts.max_inflight) s->n_slots = std::min<uint64_t>(s->n_slots, s->opts.max_inflight);
    auto fail = [&](cobs_status st) {
        for (hipStream_t x : s->streams) (void)hipStreamDestroy(x);
        for (Workspace *w : s->spaces) delete w;
        delete s;
        return st;
    };
    for (uint32_t i = 0; i < s->opts.num_streams; ++i) {
        hipStream_t st;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(hip_error(e, "hipStreamCreateWithFlags"));
        s->streams.push_back(st);
        s->spaces.push_back(new Workspace());
    }
    if (s->n_slots) {
        hipError_t e = s->pool.ensure(s->n_slots * slot_bytes, true, s->streams[0]);
        if (e != hipSuccess) return fail(hip_error(e, "score buffer pool"));
        s->free_slots.reserve(s->n_slots);
        for (uint64_t i = s->n_slots; i-- > 0;) s->free_slots.push_back((uint32_t)i);
    }
    for (uint32_t i = 0; i < s->opts.num_streams; ++i) {
        const uint64_t w = s->opts.max_batch_terms;
        const uint32_t nq = (uint32_t)std::min<uint64_t>(s->opts.max_batch_queries, s->n_slots + 1);
        cobs_status st = reserve_workspace(ix, *s->spaces[i], w, nq, s->streams[i]);
        if (st != COBS_OK) return fail(st);
    }
    if (hipStreamSynchronize(s->streams[0]) != hipSuccess)
        return fail(set_error(COBS_EDEVICE, "stream synchronisation failed"));
    for (uint32_t i = 0; i < s->opts.num_streams; ++i)
        s->workers.emplace_back(&cobs_server::worker, s, (int)i);
    *out = s;
    return COBS_OK;
}

cobs_status cobs_submit(cobs_server *s, const uint8_t *query, uint64_t len, uint32_t k_num,
                        uint32_t k_den, uint32_t topk, uint64_t arrival_ns, uint64_t *ticket)
{
    if (!s || !ticket || (len && !query)) return set_error(COBS_EINVAL, "NULL argument");
    if (k_den == 0) return set_error(COBS_EINVAL, "k_den must be > 0");
    auto r = std::make_shared<Request>();
    r->bytes.assign(query, query + len);
    r->k_num = k_num;
    r->k_den = k_den;
    r->topk = topk;
    r->arrival_ns = arrival_ns ? arrival_ns : now_ns();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stopping) return set_error(COBS_ECANCELLED, "server is stopping");
        ++s->submitted;
        if (s->n_slots == 0) {
            ++s->rejected;
            return set_error(COBS_EBUDGET, "the score memory budget holds no score buffer");
        }
        r->ticket = s->next_ticket++;
        s->first_arrival = std::min(s->first_arrival, r->arrival_ns);
        s->all[r->ticket] = r;
        s->waiting.push_back(r);
        s->admit_locked();
        *ticket = r->ticket;
    }
    s->cv_work.notify_one();
    return COBS_OK;
}

cobs_status cobs_wait(cobs_server *s, uint64_t ticket, cobs_hits **out, uint64_t *latency_ns)
{
    if (!s || !out) return set_error(COBS_EINVAL, "NULL argument");
    *out = nullptr;
    std::shared_ptr<Request> r;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return set_error(COBS_EINVAL, "unknown ticket");
        r = it->second;
        s->cv_done.wait(lk, [&] { return r->done; });
        s->all.erase(ticket);
    }
    if (latency_ns) *latency_ns = r->done_ns > r->arrival_ns ? r->done_ns - r->arrival_ns : 0;
    if (r->status != COBS_OK) return set_error(r->status, r->error);
    cobs_hits *h = (cobs_hits *)std::malloc(sizeof(cobs_hits));
    if (!h) return set_error(COBS_ENOMEM, "out of host memory");
    *h = r->hits;
    r->hits.doc_id = nullptr;
    r->hits.score = nullptr;
    *out = h;
    return COBS_OK;
}

cobs_status cobs_serve_replay(cobs_server *s, const uint8_t *bytes, const uint64_t *q_off,
                              uint32_t n, const uint64_t *arrival_ns, uint32_t k_num,
                              uint32_t k_den, uint32_t topk, uint64_t *latency_ns,
                              uint32_t *n_hits)
{
    if (!s || (n && (!q_off || !arrival_ns))) return set_error(COBS_EINVAL, "NULL argument");
    std::vector<std::atomic<uint64_t>> tickets(n);
    for (auto &t : tickets) t.store(0);
    std::atomic<int> sub_err{COBS_OK};
    std::string sub_msg;
    const uint64_t start = now_ns() + 1000000ull;
    std::thread submitter([&] {
        for (uint32_t i = 0; i < n; ++i) {
            const uint64_t at = start + arrival_ns[i];
            for (;;) {
                const uint64_t t = now_ns();
                if (t >= at) break;
                if (at - t > 200000) std::this_thread::sleep_for(std::chrono::nanoseconds(at - t - 100000));
            }
            uint64_t tk = 0;
            cobs_status st = cobs_submit(s, bytes + q_off[i], q_off[i + 1] - q_off[i], k_num,
                                         k_den, topk, at, &tk);
            if (st != COBS_OK) {
                sub_err.store(st);
                sub_msg = cobs_last_error();
                tickets[i].store(~0ull);
                continue;
            }
            tickets[i].store(tk);
        }
    });
    cobs_status first = COBS_OK;
    std::string first_msg;
    for (uint32_t i = 0; i < n; ++i) {
        uint64_t tk;
        while ((tk = tickets[i].load()) == 0) std::this_thread::sleep_for(std::chrono::microseconds(50));
        if (tk == ~0ull) {
            if (latency_ns) latency_ns[i] = 0;
            if (n_hits) n_hits[i] = 0;
            continue;
        }
        cobs_hits *h = nullptr;
        uint64_t lat = 0;
        cobs_status st = cobs_wait(s, tk, &h, &lat);
        if (st != COBS_OK && first == COBS_OK) {
            first = st;
            first_msg = cobs_last_error();
        }
        if (latency_ns) latency_ns[i] = lat;
        if (n_hits) n_hits[i] = h ? h->n : 0;
        if (h) cobs_hits_free(h, 1);
    }
    submitter.join();
    if (first == COBS_OK && sub_err.load() != COBS_OK)
        return set_error((cobs_status)sub_err.load(), sub_msg);
    if (first != COBS_OK) return set_error(first, first_msg);
    return COBS_OK;
}

cobs_status cobs_serve_stop(cobs_server *s, cobs_serve_stats *stats)
{
    if (!s) return set_error(COBS_EINVAL, "server is NULL");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    for (auto &t : s->workers) t.join();
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->submitted = s->submitted;
        stats->completed = s->completed;
        stats->rejected = s->rejected;
        stats->cancelled = s->cancelled;
        stats->batches = s->batches;
        stats->lookups = s->lookups;
        std::vector<uint64_t> l = s->latencies;
        std::sort(l.begin(), l.end());
        if (!l.empty()) {
            stats->p50_ns = l[(l.size() - 1) / 2];
            stats->p99_ns = l[std::min(l.size() - 1, (size_t)((l.size() - 1) * 0.99 + 0.5))];
            stats->max_ns = l.back();
        }
        if (s->completed && s->last_done > s->first_arrival) {
            stats->wall_s = (double)(s->last_done - s->first_arrival) * 1e-9;
            stats->queries_per_s = (double)s->completed / stats->wall_s;
            stats->lookups_per_s = (double)s->lookups / stats->wall_s;
        }
    }
    for (auto &kv : s->all) {
        std::free(kv.second->hits.doc_id);
        std::free(kv.second->hits.score);
    }
    for (hipStream_t st : s->streams) (void)hipStreamDestroy(st);
    for (Workspace *w : s->spaces) delete w;
    delete s;
    return COBS_OK;
}

}  // extern "C"
