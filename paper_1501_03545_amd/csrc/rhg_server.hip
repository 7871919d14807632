// rhg_server.hip -- a request server for graph generation on one GPU:
// continuous batching with device-resident state.
//
// Requests (n, average degree, gamma, seed) are planned on the host when
// they are submitted and queued first come, first served.  The head of the
// queue is admitted as soon as a slot (a HIP stream of its own) is free and
// its expected device memory fits beside what admitted requests hold; its
// whole pipeline then runs asynchronously on its slot's stream, so requests
// that arrive while others run overlap with them on the device.  Device
// memory comes from one arena the server allocates at creation and hands
// out by first fit on the host, so admission never calls the allocator.
// A request's result (points and CSR) stays in the arena until the caller
// releases it; its index workspace goes back as soon as it completes.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "rhg_internal.h"

namespace {

using clock_type = std::chrono::steady_clock;

// First-fit allocator over [0, size) of the arena, 256-byte granules.
struct Arena {
    std::map<size_t, size_t> free_;  // offset -> length
    size_t size = 0;
    void init(size_t n)
    {
        size = n;
        free_.clear();
        if (n) free_[0] = n;
    }
    bool take(size_t bytes, size_t *off)
    {
        bytes = rhg::align_up(bytes ? bytes : 1, 256);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            return true;
        }
        return false;
    }
    void give(size_t off, size_t bytes)
    {
        bytes = rhg::align_up(bytes ? bytes : 1, 256);
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

struct Block {
    size_t off = 0, bytes = 0;
    bool live = false;
};

struct Req {
    int64_t id = 0;
    rhg_params p;
    rhg_tuning t;
    bool has_t = false;
    size_t ws_bytes = 0, res_bytes = 0;  // workspace; points + row_ptr + col_idx
    int64_t col_cap = 0;
    Block ws, res;
    int slot = -1;
    int attempts = 0;
    clock_type::time_point submitted;
    double latency_ms = 0.0;
    rhg_status status = RHG_OK;
    int64_t nnz = 0;
};

}  // namespace

struct rhg_server {
    size_t budget = 0, reserved = 0;
    char *arena_base = nullptr;
    Arena arena;
    int slots = 0;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    int64_t *tail = nullptr;  // pinned host: per slot (2m, overflow flag)
    std::vector<int> slot_req_free;
    std::map<int64_t, Req> reqs;         // every request not yet released
    std::deque<int64_t> queue;           // submitted, not admitted
    std::vector<int64_t> inflight;       // per slot: request id or -1
    std::deque<int64_t> finished;        // completed, not yet handed out by poll
    rhg_server_stats st;
};

namespace {

// Device bytes of a request: (r, theta), row_ptr and col_idx slots for the
// target degree times n with slack (the result), and the index workspace.
void size_request(Req &q)
{
    const int64_t n = q.p.n;
    const double k = q.p.avg_degree == q.p.avg_degree ? q.p.avg_degree : 16.0;
    q.col_cap = (int64_t)((double)n * k * 1.3) + 4096;
    const size_t N = (size_t)(n > 0 ? n : 1);
    q.res_bytes = rhg::align_up(16 * N, 256) + rhg::align_up(8 * (size_t)(n + 1), 256) +
                  rhg::align_up(4 * (size_t)q.col_cap, 256) + 256;
    q.ws_bytes = rhg_index_workspace_bytes(&q.p, q.has_t ? &q.t : nullptr);
}

struct Views {
    double *r, *theta;
    int64_t *row_ptr;
    int32_t *col;
    int32_t *flag;
};

Views views(rhg_server *s, const Req &q)
{
    char *b = s->arena_base + q.res.off;
    const int64_t n = q.p.n;
    const size_t N = (size_t)(n > 0 ? n : 1);
    Views v;
    v.r = (double *)b;
    v.theta = v.r + N;
    b += rhg::align_up(16 * N, 256);
    v.row_ptr = (int64_t *)b;
    b += rhg::align_up(8 * (size_t)(n + 1), 256);
    v.col = (int32_t *)b;
    b += rhg::align_up(4 * (size_t)q.col_cap, 256);
    v.flag = (int32_t *)b;
    return v;
}

__global__ void server_tail_kernel(const int64_t *row_ptr, int64_t n, const int32_t *flag, int64_t *out)
{
    if (threadIdx.x == 0) {
        out[0] = row_ptr[n];
        out[1] = *flag;
    }
}

// Launch q's whole pipeline on its slot's stream, then copy (2m, flag) to
// the slot's pinned host pair and record the slot's event.
rhg_status launch(rhg_server *s, Req &q)
{
    const Views v = views(s, q);
    hipStream_t st = s->streams[q.slot];
    rhg_status r = rhg_generate_async(&q.p, q.has_t ? &q.t : nullptr, v.r, v.theta, s->arena_base + q.ws.off,
                                      q.ws.bytes, v.row_ptr, v.col, q.col_cap, v.flag, st);
    if (r != RHG_OK) return r;
    int64_t *dtail = (int64_t *)(s->arena_base + q.ws.off);  // the index is done with its workspace by then
    hipLaunchKernelGGL(server_tail_kernel, dim3(1), dim3(64), 0, st, v.row_ptr, q.p.n, v.flag, dtail);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpyAsync(s->tail + 2 * q.slot, dtail, 16, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipEventRecord(s->events[q.slot], st);
    if (e != hipSuccess) return rhg::check_hip(e, "rhg_server (launch)");
    ++q.attempts;
    return RHG_OK;
}

void give(rhg_server *s, Block &b)
{
    if (!b.live) return;
    s->arena.give(b.off, b.bytes);
    s->reserved -= rhg::align_up(b.bytes ? b.bytes : 1, 256);
    b.live = false;
}

bool take(rhg_server *s, Block &b, size_t bytes)
{
    size_t off = 0;
    if (!s->arena.take(bytes, &off)) return false;
    b.off = off;
    b.bytes = bytes;
    b.live = true;
    s->reserved += rhg::align_up(bytes ? bytes : 1, 256);
    s->st.max_reserved_bytes = std::max<int64_t>(s->st.max_reserved_bytes, (int64_t)s->reserved);
    return true;
}

// Admit the head of the queue while a slot and arena room are free.
rhg_status admit(rhg_server *s)
{
    while (!s->queue.empty()) {
        int slot = -1;
        for (int k = 0; k < s->slots; ++k)
            if (s->inflight[k] < 0) { slot = k; break; }
        if (slot < 0) break;
        Req &q = s->reqs[s->queue.front()];
        if (!take(s, q.res, q.res_bytes)) break;  // first come, first served: the head waits
        if (!take(s, q.ws, q.ws_bytes)) {
            give(s, q.res);
            break;
        }
        s->queue.pop_front();
        q.slot = slot;
        s->inflight[slot] = q.id;
        const rhg_status r = launch(s, q);
        if (r != RHG_OK) {
            q.status = r;
            s->inflight[slot] = -1;
            give(s, q.ws);
            q.slot = -1;
            s->finished.push_back(q.id);
            continue;
        }
        int busy = 0;
        for (int k = 0; k < s->slots; ++k) busy += s->inflight[k] >= 0;
        s->st.max_inflight = std::max<int64_t>(s->st.max_inflight, busy);
    }
    return RHG_OK;
}

}  // namespace

using rhg::check_hip;
using rhg::fail;

extern "C" {

rhg_status rhg_server_create(size_t budget_bytes, int slots, rhg_server **out)
{
    if (!out) return fail(RHG_EINVAL, "rhg_server_create: out is NULL");
    *out = nullptr;
    if (slots < 1 || slots > 64) return fail(RHG_EINVAL, "rhg_server_create: slots must be 1 .. 64");
    if (budget_bytes < (1u << 20)) return fail(RHG_EINVAL, "rhg_server_create: budget below 1 MiB");
    rhg_server *s = new (std::nothrow) rhg_server;
    if (!s) return fail(RHG_ENOMEM, "rhg_server_create: host allocation failed");
    s->budget = rhg::align_up(budget_bytes, 256);
    s->slots = slots;
    memset(&s->st, 0, sizeof(s->st));
    hipError_t e = hipMalloc((void **)&s->arena_base, s->budget);
    if (e != hipSuccess) {
        delete s;
        return fail(RHG_ENOMEM, "rhg_server_create: the device arena of " + std::to_string(budget_bytes) +
                                    " bytes could not be allocated");
    }
    s->arena.init(s->budget);
    e = hipHostMalloc((void **)&s->tail, sizeof(int64_t) * 2 * slots, hipHostMallocDefault);
    s->streams.assign(slots, nullptr);
    s->events.assign(slots, nullptr);
    s->inflight.assign(slots, -1);
    for (int k = 0; k < slots && e == hipSuccess; ++k) {
        e = hipStreamCreateWithFlags(&s->streams[k], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&s->events[k], hipEventDisableTiming);
    }
    if (e != hipSuccess) {
        rhg_server_destroy(s);
        return check_hip(e, "rhg_server_create");
    }
    *out = s;
    return RHG_OK;
}

rhg_status rhg_server_submit(rhg_server *s, int64_t req_id, int64_t n, double avg_degree, double gamma,
                             uint64_t seed, const rhg_tuning *t)
{
    if (!s) return fail(RHG_EINVAL, "rhg_server_submit: NULL server");
    if (s->reqs.count(req_id)) return fail(RHG_EINVAL, "rhg_server_submit: request id in use");
    Req q;
    q.id = req_id;
    q.submitted = clock_type::now();
    rhg_status r = rhg_plan(n, avg_degree, gamma, seed, &q.p);
    if (r != RHG_OK) return r;
    if (t) {
        q.t = *t;
        q.has_t = true;
    }
    size_request(q);
    const size_t need = rhg::align_up(q.res_bytes, 256) + rhg::align_up(q.ws_bytes, 256);
    if (need > s->budget) {
        ++s->st.rejected;
        return fail(RHG_ECAPACITY, "rhg_server_submit: the request needs " + std::to_string(need) +
                                       " bytes of device memory, the budget is " + std::to_string(s->budget));
    }
    s->reqs[req_id] = q;
    s->queue.push_back(req_id);
    ++s->st.submitted;
    return admit(s);
}

rhg_status rhg_server_poll(rhg_server *s, rhg_completion *out, int cap, int *count)
{
    if (!s || !count || (cap > 0 && !out)) return fail(RHG_EINVAL, "rhg_server_poll: NULL argument");
    *count = 0;
    for (int k = 0; k < s->slots; ++k) {
        const int64_t id = s->inflight[k];
        if (id < 0) continue;
        const hipError_t e = hipEventQuery(s->events[k]);
        if (e == hipErrorNotReady) continue;
        Req &q = s->reqs[id];
        if (e != hipSuccess) {
            q.status = check_hip(e, "rhg_server_poll");
        } else {
            const int64_t nnz = s->tail[2 * k], flag = s->tail[2 * k + 1];
            if (flag & 2) {
                q.status = fail(RHG_EINTERNAL, "rhg_server: the emit pass disagreed with the count pass");
            } else if (flag & 1) {
                // more edges than the reserved col_idx slots: run again with
                // exactly 2m slots (a new result block; the old one returns)
                ++s->st.refills;
                Block old = q.res;
                q.col_cap = nnz;
                const int64_t N = q.p.n > 0 ? q.p.n : 1;
                q.res_bytes = rhg::align_up(16 * (size_t)N, 256) + rhg::align_up(8 * (size_t)(q.p.n + 1), 256) +
                              rhg::align_up(4 * (size_t)(nnz > 0 ? nnz : 1), 256) + 256;
                if (take(s, q.res, q.res_bytes)) {
                    give(s, old);
                    const rhg_status r = launch(s, q);
                    if (r == RHG_OK) continue;
                    q.status = r;
                } else {
                    q.res = old;
                    q.status = fail(RHG_ECAPACITY, "rhg_server: no room for the request's edges");
                }
            } else {
                q.nnz = nnz;
            }
        }
        q.latency_ms = std::chrono::duration<double, std::milli>(clock_type::now() - q.submitted).count();
        s->inflight[k] = -1;
        q.slot = -1;
        give(s, q.ws);  // the index is no part of the result
        s->finished.push_back(id);
    }
    admit(s);
    while (!s->finished.empty() && *count < cap) {
        Req &q = s->reqs[s->finished.front()];
        s->finished.pop_front();
        rhg_completion &c = out[(*count)++];
        memset(&c, 0, sizeof(c));
        c.req_id = q.id;
        c.status = q.status;
        c.params = q.p;
        c.n = q.p.n;
        c.latency_ms = q.latency_ms;
        if (q.status == RHG_OK) {
            const Views v = views(s, q);
            c.nnz = q.nnz;
            c.row_ptr = v.row_ptr;
            c.col_idx = v.col;
            c.r = v.r;
            c.theta = v.theta;
            ++s->st.completed;
            s->st.edges += q.nnz / 2;
        } else {
            ++s->st.failed;
        }
    }
    return RHG_OK;
}

rhg_status rhg_server_release(rhg_server *s, int64_t req_id)
{
    if (!s) return fail(RHG_EINVAL, "rhg_server_release: NULL server");
    auto it = s->reqs.find(req_id);
    if (it == s->reqs.end()) return fail(RHG_EINVAL, "rhg_server_release: unknown request id");
    Req &q = it->second;
    if (q.slot >= 0) return fail(RHG_EBUSY, "rhg_server_release: the request is still running");
    for (auto f = s->finished.begin(); f != s->finished.end(); ++f)
        if (*f == req_id) return fail(RHG_EBUSY, "rhg_server_release: the request's completion was not polled yet");
    auto qi = std::find(s->queue.begin(), s->queue.end(), req_id);
    if (qi != s->queue.end()) s->queue.erase(qi);  // withdrawn before admission
    give(s, q.ws);
    give(s, q.res);
    s->reqs.erase(it);
    return admit(s);
}

rhg_status rhg_server_get_stats(rhg_server *s, rhg_server_stats *out)
{
    if (!s || !out) return fail(RHG_EINVAL, "rhg_server_get_stats: NULL argument");
    *out = s->st;
    out->reserved_bytes = (int64_t)s->reserved;
    int busy = 0;
    for (int k = 0; k < s->slots; ++k) busy += s->inflight[k] >= 0;
    out->inflight = busy;
    out->queued = (int64_t)s->queue.size();
    return RHG_OK;
}

void rhg_server_destroy(rhg_server *s)
{
    if (!s) return;
    for (int k = 0; k < (int)s->streams.size(); ++k)
        if (s->streams[k]) (void)hipStreamSynchronize(s->streams[k]);
    for (int k = 0; k < (int)s->streams.size(); ++k) {
        if (s->events[k]) (void)hipEventDestroy(s->events[k]);
        if (s->streams[k]) (void)hipStreamDestroy(s->streams[k]);
    }
    if (s->tail) (void)hipHostFree(s->tail);
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
}

}  // extern "C"
