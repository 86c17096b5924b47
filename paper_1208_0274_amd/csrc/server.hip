// Request loop with continuous batching over a resident index.
//
// Several slots (a workspace, a stream and a worker thread each) run searches
// at the same time, so the kernels of different requests overlap on the
// device.  A free slot admits the requests at the head of the queue while the
// device-memory budget allows: consecutive requests with the same scoring and
// threshold are taken together and run as one batched search (their queries
// end to end, split again afterwards), so requests that arrive while others
// are on the device join the next batch as soon as a slot and memory free up.
// Each request retires as soon as its own batch is done.
#include <hip/hip_runtime.h>

#include <cmath>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "alae_internal.h"

namespace alae {
alae_status download_hits(alae_workspace *ws, hipStream_t s, alae_hits *out);
}

using namespace alae;

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
    uint64_t id = 0;
    std::vector<uint8_t> codes;
    alae_scoring scoring{};
    std::vector<int8_t> matrix;
    int32_t H = 0;
    uint64_t need = 0;  // admission estimate (device bytes)
    Clock::time_point t_submit;
    bool done = false;
    alae_status status = ALAE_OK;
    alae_hits result{};
    std::string error;
};

// Device bytes a request's search is expected to hold at its widest level:
// two frontier levels of 20-byte entries (with the slack of buffers that grow
// by doubling), with about max(64, 2000 (n/1e9)^0.6)
// live entries per query column at the widest one (the frontier of a trie
// level grows with the text roughly as the entry count of Section 6 does;
// 2000 is what i.i.d. DNA of 1e9 bases shows), the profile and the query.
uint64_t row_memory_estimate(uint64_t m, int sigma, uint64_t n) {
    const double per_col = std::max(64.0, 2000.0 * std::pow((double)n / 1e9, 0.6));
    // buffers grow by doubling: up to twice what the rows need
    return (uint64_t)((double)m * 80.0 * per_col) + (uint64_t)sigma * m + 16ull * m;
}

bool same_scheme(const Request &a, const Request &b) {
    if (a.H != b.H || a.scoring.use_matrix != b.scoring.use_matrix || a.scoring.sg != b.scoring.sg ||
        a.scoring.ss != b.scoring.ss)
        return false;
    if (a.scoring.use_matrix) return a.matrix == b.matrix;
    return a.scoring.sa == b.scoring.sa && a.scoring.sb == b.scoring.sb;
}

struct Slot {
    alae_workspace *ws = nullptr;
    hipStream_t stream = nullptr;
    uint8_t *d_query = nullptr;
    uint64_t cap = 0;
    std::thread th;
};

constexpr uint64_t kBatchColumns = 1ull << 20;  // query columns of one batched search

}  // namespace

struct alae_server {
    const alae_index *idx = nullptr;
    uint64_t budget = 0;
    int max_batch = 16;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> requests;
    uint64_t next_id = 1;
    uint64_t reserved_bytes = 0;
    bool stop = false;
    // statistics
    uint64_t submitted = 0, completed = 0, batches = 0, batched = 0, rejected = 0;
    std::vector<double> latencies_ms;
    Clock::time_point t_first{}, t_last{};
};

// Run one batch on a slot; fills each request's result and status.
static void run_batch(alae_server *srv, Slot &slot, std::vector<std::shared_ptr<Request>> &batch) {
    alae_status st = ALAE_OK;
    uint64_t m = 0;
    for (auto &r : batch) m += r->codes.size();
    if (m > slot.cap) {
        if (slot.d_query) hipFree(slot.d_query);
        slot.d_query = nullptr;
        slot.cap = 0;
        if (hipMalloc(&slot.d_query, m) != hipSuccess) {
            hipGetLastError();
            set_error("device allocation of %llu query bytes failed", (unsigned long long)m);
            st = ALAE_E_NOMEM;
        } else {
            slot.cap = m;
        }
    }
    std::vector<uint8_t> cat;
    std::vector<size_t> lens;
    if (st == ALAE_OK) {
        cat.reserve(m);
        for (auto &r : batch) {
            cat.insert(cat.end(), r->codes.begin(), r->codes.end());
            lens.push_back(r->codes.size());
        }
        if (hipMemcpyAsync(slot.d_query, cat.data(), m, hipMemcpyHostToDevice, slot.stream) != hipSuccess ||
            hipStreamSynchronize(slot.stream) != hipSuccess) {
            set_error("query upload failed");
            st = ALAE_E_DEVICE;
        }
    }
    alae_scoring sc = batch[0]->scoring;
    if (sc.use_matrix) sc.matrix = batch[0]->matrix.data();
    alae_hits all{};
    std::vector<size_t> off(batch.size() + 1, 0);
    if (st == ALAE_OK) {
        size_t cnt = 0;
        if (batch.size() == 1) {
            st = alae_search_device(slot.ws, slot.d_query, m, &sc, batch[0]->H, nullptr, slot.stream, &cnt);
            off[1] = cnt;
        } else {
            st = alae_search_device_batch(slot.ws, slot.d_query, lens.data(), lens.size(), &sc, batch[0]->H, nullptr,
                                          slot.stream, &cnt);
            if (st == ALAE_OK) st = alae_workspace_batch_offsets(slot.ws, off.data(), batch.size());
        }
        if (st == ALAE_OK) st = download_hits(slot.ws, slot.stream, &all);
    }
    const std::string err = st == ALAE_OK ? std::string() : std::string(alae_last_error());
    for (size_t i = 0; i < batch.size(); ++i) {
        Request &r = *batch[i];
        r.status = st;
        if (st != ALAE_OK) {
            r.error = err;
            continue;
        }
        const size_t n = off[i + 1] - off[i], alloc = n ? n : 1;
        alae_hits h{};
        h.count = n;
        h.query_end = (uint32_t *)malloc(alloc * sizeof(uint32_t));
        h.text_end = (uint64_t *)malloc(alloc * sizeof(uint64_t));
        h.score = (int32_t *)malloc(alloc * sizeof(int32_t));
        if (!h.query_end || !h.text_end || !h.score) {
            alae_hits_free(&h);
            r.status = ALAE_E_NOMEM;
            r.error = "out of host memory for a result";
            continue;
        }
        if (n) {
            memcpy(h.query_end, all.query_end + off[i], n * sizeof(uint32_t));
            memcpy(h.text_end, all.text_end + off[i], n * sizeof(uint64_t));
            memcpy(h.score, all.score + off[i], n * sizeof(int32_t));
        }
        r.result = h;
    }
    alae_hits_free(&all);
}

static void worker_loop(alae_server *srv, size_t si) {
    Slot &slot = srv->slots[si];
    hipSetDevice(srv->idx->device);
    for (;;) {
        std::vector<std::shared_ptr<Request>> batch;
        uint64_t need = 0;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            // the head request waits until the budget has room for it (no overtaking, so a
            // large request is never starved by small ones)
            srv->cv_work.wait(lk, [&] {
                return srv->stop ||
                       (!srv->queue.empty() && srv->reserved_bytes + srv->queue.front()->need <= srv->budget);
            });
            if (srv->stop && srv->queue.empty()) return;
            uint64_t cols = 0;
            while (!srv->queue.empty() && (int)batch.size() < srv->max_batch) {
                auto &r = srv->queue.front();
                // a batch holds at most a slot's share of the budget (the head request alone may hold more)
                if (!batch.empty() && (!same_scheme(*batch[0], *r) || cols + r->codes.size() > kBatchColumns ||
                                       srv->reserved_bytes + need + r->need > srv->budget ||
                                       need + r->need > srv->budget / srv->slots.size()))
                    break;
                cols += r->codes.size();
                need += r->need;
                batch.push_back(r);
                srv->queue.pop_front();
            }
            srv->reserved_bytes += need;
            srv->batches += 1;
            srv->batched += batch.size();
        }
        run_batch(srv, slot, batch);
        // a slot's workspace keeps what its largest search grew (freeing synchronises the
        // device, which stalls the other slots); only a search beyond a slot's share of the
        // budget (a single request larger than that) gives its memory back
        if (need > srv->budget / srv->slots.size()) workspace_trim(slot.ws);
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            const auto now = Clock::now();
            for (auto &r : batch) {
                r->done = true;
                srv->completed += 1;
                srv->latencies_ms.push_back(std::chrono::duration<double, std::milli>(now - r->t_submit).count());
            }
            srv->t_last = now;
            srv->reserved_bytes -= need;
        }
        srv->cv_done.notify_all();
        srv->cv_work.notify_all();
    }
}

static void destroy_server(alae_server *srv) {
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    for (auto &s : srv->slots)
        if (s.th.joinable()) s.th.join();
    for (auto &kv : srv->requests) alae_hits_free(&kv.second->result);
    hipSetDevice(srv->idx->device);
    for (auto &s : srv->slots) {
        if (s.d_query) hipFree(s.d_query);
        if (s.stream) hipStreamDestroy(s.stream);
        alae_workspace_free(s.ws);
    }
    delete srv;
}

extern "C" {

alae_status alae_server_create(const alae_index *index, const alae_server_opts *opts, alae_server **out) {
    if (!index || !out) {
        set_error("alae_server_create: null argument");
        return ALAE_E_ARG;
    }
    alae_server *srv = new (std::nothrow) alae_server();
    if (!srv) {
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    srv->idx = index;
    // a search over a large text fills the GPU by itself: two slots there, four otherwise
    const int nslots = (opts && opts->max_inflight > 0) ? std::min(opts->max_inflight, 16)
                                                          : (index->n >= (1ull << 28) ? 2 : 4);
    srv->max_batch = (opts && opts->max_batch > 0) ? opts->max_batch : 16;
    srv->slots.resize((size_t)nslots);
    for (auto &s : srv->slots) {
        alae_status st = alae_workspace_create(index, &s.ws);
        if (st == ALAE_OK && hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) {
            set_error("stream creation failed");
            st = ALAE_E_DEVICE;
        }
        if (st != ALAE_OK) {
            destroy_server(srv);
            return st;
        }
    }
    size_t free_b = 0, total_b = 0;
    hipMemGetInfo(&free_b, &total_b);
    srv->budget = (opts && opts->memory_budget) ? opts->memory_budget : (uint64_t)(free_b / 2);
    for (size_t i = 0; i < srv->slots.size(); ++i) srv->slots[i].th = std::thread(worker_loop, srv, i);
    *out = srv;
    return ALAE_OK;
}

alae_status alae_server_submit(alae_server *srv, const char *query, size_t m, const alae_scoring *scoring,
                               int32_t H, uint64_t *req_id) {
    if (!srv || !query || !scoring || !req_id || m == 0) {
        set_error("alae_server_submit: null argument or empty query");
        return ALAE_E_ARG;
    }
    auto req = std::make_shared<Request>();
    try {
        req->codes.resize(m);
    } catch (const std::bad_alloc &) {
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    if (!encode(query, m, srv->idx->alphabet, req->codes.data())) {
        set_error("alae_server_submit: query character outside the alphabet");
        return ALAE_E_ALPHABET;
    }
    req->scoring = *scoring;
    if (scoring->use_matrix) {
        if (!scoring->matrix) {
            set_error("alae_server_submit: matrix is NULL");
            return ALAE_E_ARG;
        }
        const int s = srv->idx->sigma;
        req->matrix.assign(scoring->matrix, scoring->matrix + s * s);
    }
    req->scoring.matrix = nullptr;
    req->H = H;
    req->need = row_memory_estimate(m, srv->idx->sigma, srv->idx->n);
    req->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(srv->mu);
    if (req->need > srv->budget) {
        srv->rejected += 1;
        set_error("request needs about %llu device bytes, budget is %llu", (unsigned long long)req->need,
                  (unsigned long long)srv->budget);
        return ALAE_E_ADMISSION;
    }
    req->id = srv->next_id++;
    if (srv->submitted == 0) srv->t_first = req->t_submit;
    srv->submitted += 1;
    srv->requests[req->id] = req;
    srv->queue.push_back(req);
    *req_id = req->id;
    srv->cv_work.notify_all();
    return ALAE_OK;
}

alae_status alae_server_poll(alae_server *srv, uint64_t req_id, int wait, alae_hits *out) {
    if (!srv || !out) {
        set_error("alae_server_poll: null argument");
        return ALAE_E_ARG;
    }
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->requests.find(req_id);
    if (it == srv->requests.end()) {
        set_error("alae_server_poll: unknown request %llu", (unsigned long long)req_id);
        return ALAE_E_NOT_FOUND;
    }
    std::shared_ptr<Request> req = it->second;
    if (!req->done) {
        if (!wait) {
            memset(out, 0, sizeof(*out));
            out->count = SIZE_MAX;
            return ALAE_OK;
        }
        srv->cv_done.wait(lk, [&] { return req->done; });
    }
    srv->requests.erase(req_id);
    if (req->status != ALAE_OK) {
        set_error("%s", req->error.c_str());
        return req->status;
    }
    *out = req->result;
    req->result = alae_hits{};
    return ALAE_OK;
}

alae_status alae_server_get_stats(alae_server *srv, alae_server_stats *out) {
    if (!srv || !out) {
        set_error("alae_server_get_stats: null argument");
        return ALAE_E_ARG;
    }
    std::lock_guard<std::mutex> lk(srv->mu);
    memset(out, 0, sizeof(*out));
    out->submitted = srv->submitted;
    out->completed = srv->completed;
    out->rejected = srv->rejected;
    out->batches = srv->batches;
    out->mean_batch = srv->batches ? (double)srv->batched / (double)srv->batches : 0.0;
    out->queued = srv->queue.size();
    if (!srv->latencies_ms.empty()) {
        std::vector<double> v = srv->latencies_ms;
        std::sort(v.begin(), v.end());
        auto pct = [&](double p) { return v[std::min(v.size() - 1, (size_t)(p * (double)(v.size() - 1) + 0.5))]; };
        out->p50_ms = pct(0.50);
        out->p99_ms = pct(0.99);
        out->max_ms = v.back();
        double s = 0;
        for (double x : v) s += x;
        out->mean_ms = s / (double)v.size();
        out->span_s = std::chrono::duration<double>(srv->t_last - srv->t_first).count();
    }
    return ALAE_OK;
}

void alae_server_reset_stats(alae_server *srv) {
    if (!srv) return;
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->submitted = srv->completed = srv->batches = srv->batched = srv->rejected = 0;
    srv->latencies_ms.clear();
}

void alae_server_destroy(alae_server *srv) {
    if (!srv) return;
    destroy_server(srv);
}

}  // extern "C"
