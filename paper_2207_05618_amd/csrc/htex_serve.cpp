// htex_serve.cpp -- continuous-batching server over resident meshes.
//
// One scheduler thread owns every HIP call of the server.  Its loop:
//   1. admission: pending requests, in arrival order, take a request slot
//      and an arena block (32 bytes per query) while both are available;
//   2. uploads: admitted requests' queries go to the device in chunks of
//      copy_chunk_queries, taken round-robin over the requests still
//      uploading (a whole request at a time when the chunk size is 0), with
//      a few chunks in flight per copy stream;
//   3. batching: when a compute stream is free, the requests not yet
//      launched whose uploads are complete or all issued (in order, up to
//      max_batch_queries) become one tile list and one k_serve launch, which
//      waits on the device for the upload chunks still in flight;
//   4. downloads: whole results are queued behind the launch; with chunks,
//      requests whose batch has finished copy their results back
//      round-robin like the uploads;
//   5. completion: a request whose last result chunk has arrived is
//      complete: its arena block and slot are released and its latency
//      recorded.
// Requests that arrive while batches run are admitted and launched as soon
// as a slot, memory and a stream free up, so their work overlaps on the
// device with the batches in flight.  Round-robin chunks share the PCIe
// link among the requests in flight (processor sharing): a small request
// no longer waits behind a large one's copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "htex.h"
#include "htex_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

#define fail htex::set_error

// First-fit allocator over [0, size) in 256-byte units.
class Arena {
  public:
    explicit Arena(int64_t size) : size_(size) { free_[0] = size; }
    int64_t alloc(int64_t bytes)
    {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest > 0) free_[off + bytes] = rest;
                used_ += bytes;
                if (used_ > peak_) peak_ = used_;
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off, int64_t bytes)
    {
        bytes = (bytes + 255) / 256 * 256;
        used_ -= bytes;
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
    int64_t peak() const { return peak_; }
    int64_t size() const { return size_; }

  private:
    int64_t size_, used_ = 0, peak_ = 0;
    std::map<int64_t, int64_t> free_;
};

struct Request {
    int64_t id;
    int32_t mesh;
    int64_t Q;
    const int32_t *h;
    const float *u, *v, *f;
    float *out;
    Clock::time_point t_submit;
    int64_t arena_off = -1, arena_bytes = 0;
    // device arrays inside the arena
    int32_t *dh = nullptr;
    float *du = nullptr, *dv = nullptr, *df = nullptr, *dout = nullptr;
    // queries whose upload / download has been issued, and completed
    int64_t up_sent = 0, up_done = 0, down_sent = 0, down_done = 0;
    bool batched = false;   // in a batch (possibly before its upload is seen complete)
};

// A copy of one request's queries [q0, q0 + n) in flight on a copy stream.
struct Chunk {
    hipEvent_t ev;
    Request *r;
    int64_t n;
};

struct Batch {
    hipEvent_t ev_done = nullptr;
    bool busy = false;
    std::vector<Request *> reqs;
    htex::ServeTile *tiles_host = nullptr;   // page-locked
    htex::ServeTile *tiles_dev = nullptr;
    hipStream_t stream = nullptr;
};

}  // namespace

struct htex_server {
    htex_server_config cfg{};
    int channels = 4;          // values per texel and per result row
    int device = 0;
    int grid = 0;
    int tiles_cap = 0;
    char *arena_dev = nullptr;
    Arena *arena = nullptr;
    htex::ServeMesh *meshes_dev = nullptr;
    std::vector<htex::ServeMesh> meshes;
    int32_t *err_dev = nullptr;
    std::vector<hipStream_t> s_up, s_down;   // copy streams (both directions run at once)
    int up_rr = 0, down_rr = 0;
    std::vector<Batch> batches;

    std::mutex mu;                 // guards inbox, done, counters, meshes
    std::condition_variable cv;
    std::deque<Request *> inbox;   // submitted, not yet seen by the scheduler
    std::deque<std::pair<int64_t, double>> done;
    int64_t next_id = 0;
    int64_t submitted = 0, completed = 0, rejected = 0, n_batches = 0, queries_done = 0;
    int32_t invalid = 0;
    std::atomic<bool> stop{false};
    std::thread worker;
    std::string worker_error;

    // scheduler-thread state
    std::deque<Request *> pending;      // waiting for admission
    std::deque<Request *> uploading;    // admitted, upload chunks left to issue
    std::deque<Request *> admitted;     // uploaded, not launched
    std::deque<Request *> downloading;  // batch finished, result chunks left to issue
    std::vector<Chunk> up_chunks, down_chunks;   // copies in flight
    std::vector<hipEvent_t> free_events;
    int inflight = 0;

    void run();
    bool step();
    bool idle() const;
};

namespace {

// Places a request's device arrays inside its arena block.
void carve_arrays(htex_server *S, Request *r)
{
    const bool tri = S->cfg.filter == HTEX_TRILINEAR;
    const int64_t Q = r->Q;
    char *base = S->arena_dev + r->arena_off;
    auto carve = [&](int64_t bytes) {
        char *p = base;
        base += (bytes + 255) / 256 * 256;
        return p;
    };
    r->dh = reinterpret_cast<int32_t *>(carve(4 * Q));
    r->du = reinterpret_cast<float *>(carve(4 * Q));
    r->dv = reinterpret_cast<float *>(carve(4 * Q));
    r->df = tri ? reinterpret_cast<float *>(carve(4 * Q)) : nullptr;
    r->dout = reinterpret_cast<float *>(carve(4 * S->channels * Q));
}

hipError_t take_event(htex_server *S, hipEvent_t *ev)
{
    if (!S->free_events.empty()) {
        *ev = S->free_events.back();
        S->free_events.pop_back();
        return hipSuccess;
    }
    return hipEventCreateWithFlags(ev, hipEventDisableTiming);
}

// Issues the next upload chunk of r: queries [up_sent, up_sent + n).
hipError_t upload_chunk(htex_server *S, Request *r, int64_t n, Chunk *c)
{
    hipStream_t su = S->s_up[S->up_rr++ % S->s_up.size()];
    const int64_t q0 = r->up_sent;
    hipError_t e = hipMemcpyAsync(r->dh + q0, r->h + q0, 4 * n, hipMemcpyHostToDevice, su);
    if (!e) e = hipMemcpyAsync(r->du + q0, r->u + q0, 4 * n, hipMemcpyHostToDevice, su);
    if (!e) e = hipMemcpyAsync(r->dv + q0, r->v + q0, 4 * n, hipMemcpyHostToDevice, su);
    if (!e && r->df) e = hipMemcpyAsync(r->df + q0, r->f + q0, 4 * n, hipMemcpyHostToDevice, su);
    if (!e) e = take_event(S, &c->ev);
    if (!e) e = hipEventRecord(c->ev, su);
    c->r = r;
    c->n = n;
    r->up_sent += n;
    return e;
}

// Issues the next result chunk of r: rows [down_sent, down_sent + n).
hipError_t download_chunk(htex_server *S, Request *r, int64_t n, Chunk *c)
{
    hipStream_t sd = S->s_down[S->down_rr++ % S->s_down.size()];
    const int64_t q0 = r->down_sent, row = S->channels;
    hipError_t e = hipMemcpyAsync(r->out + row * q0, r->dout + row * q0, 4 * row * n,
                                  hipMemcpyDeviceToHost, sd);
    if (!e) e = take_event(S, &c->ev);
    if (!e) e = hipEventRecord(c->ev, sd);
    c->r = r;
    c->n = n;
    r->down_sent += n;
    return e;
}

int64_t request_bytes(const htex_server *S, int64_t Q)
{
    const int64_t a = (4 * Q + 255) / 256 * 256;
    const int64_t arrays = S->cfg.filter == HTEX_TRILINEAR ? 4 : 3;
    return arrays * a + (4 * S->channels * Q + 255) / 256 * 256;
}

}  // namespace

// One pass of the scheduler; returns true if it did any work.
bool htex_server::step()
{
    bool worked = false;
    {
        std::lock_guard<std::mutex> lk(mu);
        while (!inbox.empty()) {
            pending.push_back(inbox.front());
            inbox.pop_front();
        }
    }
    auto check = [](hipError_t e, const char *what) {
        if (e) throw std::runtime_error(std::string(what) + ": " + hipGetErrorString(e));
    };
    // 1. admission in arrival order
    while (!pending.empty() && inflight < cfg.max_inflight) {
        Request *r = pending.front();
        const int64_t bytes = request_bytes(this, r->Q);
        const int64_t off = arena->alloc(bytes);
        if (off < 0) break;
        r->arena_off = off;
        r->arena_bytes = bytes;
        pending.pop_front();
        ++inflight;
        carve_arrays(this, r);
        uploading.push_back(r);
        worked = true;
    }
    const int64_t chunk = cfg.copy_chunk_queries > 0 ? cfg.copy_chunk_queries : INT64_MAX;
    // a few chunks queued per copy stream keep its DMA engine busy between
    // two passes of this loop
    const size_t max_up = 4 * s_up.size(), max_down = 4 * s_down.size();
    // 2. upload chunks, round-robin over the requests still uploading
    while (!uploading.empty() && up_chunks.size() < max_up) {
        Request *r = uploading.front();
        uploading.pop_front();
        const int64_t left = r->Q - r->up_sent;
        Chunk c;
        check(upload_chunk(this, r, left < chunk ? left : chunk, &c), "upload");
        up_chunks.push_back(c);
        if (r->up_sent < r->Q) uploading.push_back(r);
        worked = true;
    }
    for (size_t i = 0; i < up_chunks.size();) {
        const Chunk c = up_chunks[i];
        if (hipEventQuery(c.ev) != hipSuccess) {
            ++i;
            continue;
        }
        free_events.push_back(c.ev);
        up_chunks[i] = up_chunks.back();
        up_chunks.pop_back();
        c.r->up_done += c.n;
        if (c.r->up_done == c.r->Q && !c.r->batched) admitted.push_back(c.r);
        worked = true;
    }
    // 3. batching on free compute streams
    for (Batch &b : batches) {
        if (b.busy) {
            if (hipEventQuery(b.ev_done) == hipSuccess) {
                b.busy = false;
                for (Request *r : b.reqs) downloading.push_back(r);
                b.reqs.clear();
                worked = true;
            } else {
                continue;
            }
        }
        // requests whose upload has completed; and, while no admitted
        // request waits for an upload slot, also those whose last chunk is
        // in flight: the launch then waits for those chunks on the device,
        // so at light load no host round trip sits between an upload and
        // its launch.  Under overload the copy queue is the bottleneck and
        // such launches would hold the compute stream idle behind it (the
        // sustained rate measured 1.4-1.5e9 samples/s that way, against
        // 1.7-2.4e9 when launches take completed uploads only).
        std::vector<Request *> cand(admitted.begin(), admitted.end());
        if (uploading.empty()) for (const Chunk &c : up_chunks)
            if (c.r->up_sent == c.r->Q && !c.r->batched &&
                std::find(cand.begin(), cand.end(), c.r) == cand.end())
                cand.push_back(c.r);
        if (cand.empty()) continue;
        int ntiles = 0;
        int64_t nq = 0;
        for (Request *r : cand) {
            const int t = (int)((r->Q + htex::kTileQueries - 1) / htex::kTileQueries);
            if (!b.reqs.empty() && (nq + r->Q > cfg.max_batch_queries || ntiles + t > tiles_cap))
                break;
            if (ntiles + t > tiles_cap) break;   // cannot happen: submit bounds Q
            for (int i = 0; i < t; ++i) {
                htex::ServeTile &T = b.tiles_host[ntiles + i];
                T.h = r->dh;
                T.u = r->du;
                T.v = r->dv;
                T.f = r->df;
                T.out = r->dout;
                T.q0 = (int64_t)i * htex::kTileQueries;
                T.mesh = r->mesh;
                const int64_t left = r->Q - T.q0;
                T.count = (int32_t)(left < htex::kTileQueries ? left : htex::kTileQueries);
            }
            ntiles += t;
            nq += r->Q;
            r->batched = true;
            for (const Chunk &c : up_chunks)
                if (c.r == r) check(hipStreamWaitEvent(b.stream, c.ev, 0), "wait");
            b.reqs.push_back(r);
        }
        if (b.reqs.empty()) continue;
        while (!admitted.empty() && admitted.front()->batched) admitted.pop_front();
        hipError_t e = hipMemcpyAsync(b.tiles_dev, b.tiles_host, sizeof(htex::ServeTile) * ntiles,
                                      hipMemcpyHostToDevice, b.stream);
        if (!e) e = htex::launch_serve(meshes_dev, b.tiles_dev, ntiles, grid, cfg.dtype, channels,
                                       cfg.filter, err_dev, b.stream);
        if (!e) e = hipEventRecord(b.ev_done, b.stream);
        check(e, "launch");
        if (cfg.copy_chunk_queries == 0) {
            // whole-request results: queued now behind the launch, so no host
            // round trip sits between the batch's end and its downloads
            for (hipStream_t sd : s_down) check(hipStreamWaitEvent(sd, b.ev_done, 0), "wait");
            for (Request *r : b.reqs) {
                Chunk c;
                check(download_chunk(this, r, r->Q, &c), "download");
                down_chunks.push_back(c);
            }
            b.reqs.clear();   // the download chunks own the requests now
        }
        b.busy = true;
        {
            std::lock_guard<std::mutex> lk(mu);
            ++n_batches;
        }
        worked = true;
    }
    // 4. result chunks, round-robin over the requests whose batch finished
    while (!downloading.empty() && down_chunks.size() < max_down) {
        Request *r = downloading.front();
        downloading.pop_front();
        const int64_t left = r->Q - r->down_sent;
        Chunk c;
        check(download_chunk(this, r, left < chunk ? left : chunk, &c), "download");
        down_chunks.push_back(c);
        if (r->down_sent < r->Q) downloading.push_back(r);
        worked = true;
    }
    // 5. completion
    for (size_t i = 0; i < down_chunks.size();) {
        const Chunk c = down_chunks[i];
        if (hipEventQuery(c.ev) != hipSuccess) {
            ++i;
            continue;
        }
        free_events.push_back(c.ev);
        down_chunks[i] = down_chunks.back();
        down_chunks.pop_back();
        Request *r = c.r;
        r->down_done += c.n;
        worked = true;
        if (r->down_done < r->Q) continue;
        const double lat = std::chrono::duration<double>(Clock::now() - r->t_submit).count();
        arena->release(r->arena_off, r->arena_bytes);
        --inflight;
        {
            std::lock_guard<std::mutex> lk(mu);
            done.emplace_back(r->id, lat);
            ++completed;
            queries_done += r->Q;
        }
        delete r;
    }
    if (worked) cv.notify_all();
    return worked;
}

bool htex_server::idle() const
{
    if (!pending.empty() || !uploading.empty() || !admitted.empty() || !downloading.empty() ||
        !up_chunks.empty() || !down_chunks.empty())
        return false;
    for (const Batch &b : batches)
        if (b.busy) return false;
    return true;
}

void htex_server::run()
{
    if (hipSetDevice(device) != hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        worker_error = "hipSetDevice failed in the scheduler";
        return;
    }
    try {
        for (;;) {
            const bool worked = step();
            const bool quiet = idle();
            if (stop.load() && quiet) {
                bool empty;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    empty = inbox.empty();
                }
                if (empty) break;
            }
            if (!worked) {
                if (quiet) {
                    std::unique_lock<std::mutex> lk(mu);
                    cv.wait_for(lk, std::chrono::microseconds(200),
                                [&] { return !inbox.empty() || stop.load(); });
                } else {
                    std::this_thread::sleep_for(std::chrono::microseconds(5));
                }
            }
        }
    } catch (const std::exception &ex) {
        std::lock_guard<std::mutex> lk(mu);
        worker_error = ex.what();
    }
    int32_t bad = 0;
    if (hipMemcpy(&bad, err_dev, sizeof bad, hipMemcpyDeviceToHost) == hipSuccess) {
        std::lock_guard<std::mutex> lk(mu);
        invalid = bad;
    }
    cv.notify_all();
}

extern "C" {

htex_status htex_server_create(const htex_server_config *cfg, htex_server **out)
{
    if (!cfg || !out) return fail(HTEX_E_ARG, "NULL argument");
    if (cfg->dtype < HTEX_F32 || cfg->dtype > HTEX_FP8_E4M3) return fail(HTEX_E_ARG, "bad dtype");
    if (cfg->filter != HTEX_BILINEAR && cfg->filter != HTEX_TRILINEAR)
        return fail(HTEX_E_ARG, "bad filter");
    if (cfg->max_inflight <= 0 || cfg->compute_streams < 1 || cfg->compute_streams > 4 ||
        cfg->copy_streams < 1 || cfg->copy_streams > 4 ||
        cfg->arena_bytes <= 0 || cfg->max_batch_queries <= 0 || cfg->max_meshes <= 0 ||
        cfg->grid_blocks < 0 || cfg->copy_chunk_queries < 0 || cfg->reserved != 0)
        return fail(HTEX_E_ARG, "bad server configuration");
    if (cfg->channels != 0 && cfg->channels != 1 && cfg->channels != 4)
        return fail(HTEX_E_ARG, "channels must be 0 (RGBA), 1 or 4");
    htex_server *S = new htex_server();
    S->cfg = *cfg;
    S->channels = cfg->channels ? cfg->channels : 4;
    hipError_t e = hipGetDevice(&S->device);
    int cus = 0;
    if (!e) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, S->device);
    S->grid = cfg->grid_blocks ? cfg->grid_blocks : 4 * (cus > 0 ? cus : 256);
    // tile capacity: the largest admissible request plus a full batch
    const int64_t max_q = cfg->arena_bytes / 32 + 1;
    const int64_t cap_q = (cfg->max_batch_queries > max_q ? cfg->max_batch_queries : max_q);
    S->tiles_cap = (int)(cap_q / htex::kTileQueries + 2 + cfg->max_inflight);
    if (!e) e = hipMalloc(&S->arena_dev, cfg->arena_bytes);
    if (!e) e = hipMalloc(&S->meshes_dev, sizeof(htex::ServeMesh) * cfg->max_meshes);
    if (!e) e = hipMalloc(&S->err_dev, sizeof(int32_t));
    if (!e) e = hipMemset(S->err_dev, 0, sizeof(int32_t));
    const int ncopy = cfg->copy_streams;
    S->s_up.assign(ncopy, nullptr);
    S->s_down.assign(ncopy, nullptr);
    for (int i = 0; i < ncopy; ++i) {
        if (!e) e = hipStreamCreateWithFlags(&S->s_up[i], hipStreamNonBlocking);
        if (!e) e = hipStreamCreateWithFlags(&S->s_down[i], hipStreamNonBlocking);
    }
    S->batches.resize(cfg->compute_streams);
    for (Batch &b : S->batches) {
        if (!e) e = hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking);
        if (!e) e = hipEventCreateWithFlags(&b.ev_done, hipEventDisableTiming);
        if (!e) e = hipHostMalloc(&b.tiles_host, sizeof(htex::ServeTile) * S->tiles_cap);
        if (!e) e = hipMalloc(&b.tiles_dev, sizeof(htex::ServeTile) * S->tiles_cap);
    }
    if (e) {
        htex_server_destroy(S);
        return fail(HTEX_E_DEVICE, "server setup: %s", hipGetErrorString(e));
    }
    S->arena = new Arena(cfg->arena_bytes);
    S->worker = std::thread([S] { S->run(); });
    *out = S;
    htex::clear_error();
    return HTEX_OK;
}

htex_status htex_server_add_mesh(htex_server *S, int32_t H, const void *prep, const htex_pool *pool,
                                 int32_t *mesh_id)
{
    if (!S || !prep || !pool || !mesh_id || H <= 0) return fail(HTEX_E_ARG, "bad argument");
    if (pool->dtype != S->cfg.dtype) return fail(HTEX_E_ARG, "pool dtype differs from the server's");
    if (pool->channels != S->channels)
        return fail(HTEX_E_ARG, "pool has %d channels, the server %d", pool->channels, S->channels);
    if (S->cfg.filter == HTEX_TRILINEAR && !pool->has_mips)
        return fail(HTEX_E_ARG, "trilinear serving needs pools with mips");
    if (!pool->texels || (pool->dtype == HTEX_FP8_E4M3 && !pool->scale))
        return fail(HTEX_E_ARG, "pool arrays missing");
    std::lock_guard<std::mutex> lk(S->mu);
    if ((int)S->meshes.size() >= S->cfg.max_meshes) return fail(HTEX_E_RANGE, "mesh table full");
    htex::ServeMesh m{prep, pool->texels, pool->scale, pool->total_texels, H, pool->has_mips};
    const int id = (int)S->meshes.size();
    // the scheduler only reads entries of meshes already registered, and a
    // request can name a mesh only after this call returns
    hipError_t e = hipMemcpy(S->meshes_dev + id, &m, sizeof m, hipMemcpyHostToDevice);
    if (e) return fail(HTEX_E_DEVICE, "mesh table: %s", hipGetErrorString(e));
    S->meshes.push_back(m);
    *mesh_id = id;
    htex::clear_error();
    return HTEX_OK;
}

htex_status htex_server_submit(htex_server *S, int32_t mesh_id, int64_t Q, const int32_t *h,
                               const float *u, const float *v, const float *footprint, float *out,
                               int64_t *request_id)
{
    if (!S || !request_id) return fail(HTEX_E_ARG, "NULL argument");
    if (Q <= 0 || !h || !u || !v || !out) return fail(HTEX_E_ARG, "bad query arrays");
    if (S->cfg.filter == HTEX_TRILINEAR && !footprint)
        return fail(HTEX_E_ARG, "trilinear serving needs footprints");
    std::lock_guard<std::mutex> lk(S->mu);
    if (mesh_id < 0 || mesh_id >= (int)S->meshes.size())
        return fail(HTEX_E_ARG, "unknown mesh %d", mesh_id);
    if (request_bytes(S, Q) > S->arena->size()) {
        ++S->rejected;
        return fail(HTEX_E_NOMEM, "request of %lld queries exceeds the arena", (long long)Q);
    }
    if (!S->worker_error.empty()) return fail(HTEX_E_DEVICE, "scheduler stopped: %s",
                                              S->worker_error.c_str());
    Request *r = new Request();
    r->id = S->next_id++;
    r->mesh = mesh_id;
    r->Q = Q;
    r->h = h;
    r->u = u;
    r->v = v;
    r->f = footprint;
    r->out = out;
    r->t_submit = Clock::now();
    S->inbox.push_back(r);
    ++S->submitted;
    *request_id = r->id;
    S->cv.notify_all();
    htex::clear_error();
    return HTEX_OK;
}

htex_status htex_server_poll(htex_server *S, int32_t max, int64_t *ids, double *latency_s, int32_t *n)
{
    if (!S || !n || max < 0 || (max > 0 && (!ids || !latency_s))) return fail(HTEX_E_ARG, "bad argument");
    std::lock_guard<std::mutex> lk(S->mu);
    int k = 0;
    while (k < max && !S->done.empty()) {
        ids[k] = S->done.front().first;
        latency_s[k] = S->done.front().second;
        S->done.pop_front();
        ++k;
    }
    *n = k;
    if (!S->worker_error.empty()) return fail(HTEX_E_DEVICE, "scheduler stopped: %s",
                                              S->worker_error.c_str());
    htex::clear_error();
    return HTEX_OK;
}

htex_status htex_server_drain(htex_server *S, double timeout_s)
{
    if (!S) return fail(HTEX_E_ARG, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    const auto until = Clock::now() + std::chrono::duration_cast<Clock::duration>(
                                          std::chrono::duration<double>(timeout_s));
    while (S->completed < S->submitted) {
        if (!S->worker_error.empty())
            return fail(HTEX_E_DEVICE, "scheduler stopped: %s", S->worker_error.c_str());
        if (S->cv.wait_until(lk, until) == std::cv_status::timeout && S->completed < S->submitted)
            return fail(HTEX_E_BUSY, "%lld requests still in flight",
                        (long long)(S->submitted - S->completed));
    }
    // every launch has finished: refresh the invalid-query counter
    int32_t bad = 0;
    if (hipMemcpy(&bad, S->err_dev, sizeof bad, hipMemcpyDeviceToHost) == hipSuccess)
        S->invalid = bad;
    htex::clear_error();
    return HTEX_OK;
}

htex_status htex_server_stats_get(htex_server *S, htex_server_stats *st)
{
    if (!S || !st) return fail(HTEX_E_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    st->submitted = S->submitted;
    st->completed = S->completed;
    st->rejected = S->rejected;
    st->batches = S->n_batches;
    st->queries_done = S->queries_done;
    st->arena_peak_bytes = S->arena ? S->arena->peak() : 0;
    st->invalid_queries = S->invalid;
    st->pad = 0;
    htex::clear_error();
    return HTEX_OK;
}

htex_status htex_server_destroy(htex_server *S)
{
    if (!S) return fail(HTEX_E_ARG, "NULL server");
    if (S->worker.joinable()) {
        S->stop.store(true);
        S->cv.notify_all();
        S->worker.join();
    }
    for (Batch &b : S->batches) {
        if (b.stream) (void)hipStreamSynchronize(b.stream);
        if (b.ev_done) (void)hipEventDestroy(b.ev_done);
        if (b.tiles_host) (void)hipHostFree(b.tiles_host);
        if (b.tiles_dev) (void)hipFree(b.tiles_dev);
        if (b.stream) (void)hipStreamDestroy(b.stream);
    }
    for (hipStream_t st : S->s_up)
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    for (hipStream_t st : S->s_down)
        if (st) {
            (void)hipStreamSynchronize(st);
            (void)hipStreamDestroy(st);
        }
    if (S->arena_dev) (void)hipFree(S->arena_dev);
    if (S->meshes_dev) (void)hipFree(S->meshes_dev);
    if (S->err_dev) (void)hipFree(S->err_dev);
    // requests left behind only if the scheduler stopped on an error; one
    // request may sit in several lists (uploading and a chunk in flight)
    std::set<Request *> left;
    for (Request *r : S->inbox) left.insert(r);
    for (Request *r : S->pending) left.insert(r);
    for (Request *r : S->uploading) left.insert(r);
    for (Request *r : S->admitted) left.insert(r);
    for (Request *r : S->downloading) left.insert(r);
    for (const Batch &b : S->batches)
        for (Request *r : b.reqs) left.insert(r);
    for (const Chunk &c : S->up_chunks) {
        left.insert(c.r);
        (void)hipEventDestroy(c.ev);
    }
    for (const Chunk &c : S->down_chunks) {
        left.insert(c.r);
        (void)hipEventDestroy(c.ev);
    }
    for (hipEvent_t ev : S->free_events) (void)hipEventDestroy(ev);
    for (Request *r : left) delete r;
    delete S->arena;
    delete S;
    htex::clear_error();
    return HTEX_OK;
}

}  // extern "C"
