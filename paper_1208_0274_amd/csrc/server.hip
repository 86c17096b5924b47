// Request loop that keeps the index resident on the device.
//
// Requests are admitted by the device memory their frontier rows are
// expected to need (a bound from the query length), queued, and run by a
// worker thread on one workspace; each request retires as soon as its result
// is on the host.  Polling returns the result and releases it.
#include <hip/hip_runtime.h>

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

struct Request {
    uint64_t id = 0;
    std::vector<uint8_t> codes;
    alae_scoring scoring{};
    std::vector<int8_t> matrix;
    int32_t H = 0;
    bool done = false;
    alae_status status = ALAE_OK;
    alae_hits result{};
    std::string error;
};

// Device bytes a request's search is expected to hold at its widest level:
// entries of about 20 bytes for a few rows of width m, plus the query
// profile.  Used only for admission.
uint64_t row_memory_estimate(uint64_t m, int sigma) {
    return 64ull * m * 20ull + (uint64_t)sigma * m + 16ull * m;
}

}  // namespace

struct alae_server {
    const alae_index *idx = nullptr;
    uint64_t budget = 0;
    int max_inflight = 1;
    alae_workspace *ws = nullptr;
    uint8_t *d_query = nullptr;
    uint64_t d_query_cap = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<std::shared_ptr<Request>> queue;
    std::map<uint64_t, std::shared_ptr<Request>> requests;
    uint64_t next_id = 1;
    uint64_t reserved_bytes = 0;
    bool stop = false;
    std::thread worker;
};

static void server_loop(alae_server *srv) {
    for (;;) {
        std::shared_ptr<Request> req;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->cv_work.wait(lk, [&] { return srv->stop || !srv->queue.empty(); });
            if (srv->stop && srv->queue.empty()) return;
            req = srv->queue.front();
            srv->queue.pop_front();
        }
        alae_status st = ALAE_OK;
        const uint64_t m = req->codes.size();
        if (m > srv->d_query_cap) {
            if (srv->d_query) hipFree(srv->d_query);
            srv->d_query = nullptr;
            srv->d_query_cap = 0;
            if (hipMalloc(&srv->d_query, m) != hipSuccess) {
                st = ALAE_E_NOMEM;
            } else {
                srv->d_query_cap = m;
            }
        }
        if (st == ALAE_OK && hipMemcpy(srv->d_query, req->codes.data(), m, hipMemcpyHostToDevice) != hipSuccess)
            st = ALAE_E_DEVICE;
        if (st == ALAE_OK) {
            alae_scoring sc = req->scoring;
            if (sc.use_matrix) sc.matrix = req->matrix.data();
            size_t cnt = 0;
            st = alae_search_device(srv->ws, srv->d_query, m, &sc, req->H, nullptr, nullptr, &cnt);
            if (st == ALAE_OK) st = download_hits(srv->ws, nullptr, &req->result);
        }
        {
            std::lock_guard<std::mutex> lk(srv->mu);
            req->status = st;
            if (st != ALAE_OK) req->error = alae_last_error();
            req->done = true;
            srv->reserved_bytes -= row_memory_estimate(m, srv->idx->sigma);
        }
        srv->cv_done.notify_all();
    }
}

extern "C" {

alae_status alae_server_create(const alae_index *index, const alae_server_opts *opts, alae_server **out) {
    if (!index || !out) {
        set_error("alae_server_create: null argument");
        return ALAE_E_ARG;
    }
    std::unique_ptr<alae_server> srv(new (std::nothrow) alae_server());
    if (!srv) {
        set_error("out of host memory");
        return ALAE_E_NOMEM;
    }
    srv->idx = index;
    alae_status st = alae_workspace_create(index, &srv->ws);
    if (st != ALAE_OK) return st;
    size_t free_b = 0, total_b = 0;
    hipMemGetInfo(&free_b, &total_b);
    srv->budget = (opts && opts->memory_budget) ? opts->memory_budget : (uint64_t)(free_b / 2);
    srv->max_inflight = (opts && opts->max_inflight > 0) ? opts->max_inflight : 64;
    srv->worker = std::thread(server_loop, srv.get());
    *out = srv.release();
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
    const uint64_t need = row_memory_estimate(m, srv->idx->sigma);
    std::lock_guard<std::mutex> lk(srv->mu);
    if (need > srv->budget) {
        set_error("request needs about %llu device bytes, budget is %llu", (unsigned long long)need,
                  (unsigned long long)srv->budget);
        return ALAE_E_ADMISSION;
    }
    req->id = srv->next_id++;
    srv->reserved_bytes += need;
    srv->requests[req->id] = req;
    srv->queue.push_back(req);
    *req_id = req->id;
    srv->cv_work.notify_one();
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

void alae_server_destroy(alae_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    for (auto &kv : srv->requests) alae_hits_free(&kv.second->result);
    if (srv->d_query) hipFree(srv->d_query);
    alae_workspace_free(srv->ws);
    delete srv;
}

}  // extern "C"
