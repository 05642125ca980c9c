// vmt_serve.cpp -- serving loop over device-resident V-states.
//
// Requests (generate n elements from state s, or jump state s by 2^k) arrive
// over time. The loop admits them in arrival order while keeping at most one
// request per state in flight (a state's requests run in order) and the
// outputs in flight within a memory budget, and launches everything admitted
// so far whenever one of its streams is free: one persistent generation
// launch plus one jump launch per stream (continuous batching). Each task
// raises a completion flag in host memory when its outputs and state are
// written, so memory and the state are released per request, not per launch.
// With a chunk size, a large generation request is served as a run of
// bounded tasks in successive launches (its state and output space stay held
// until the last one), so a launch never grows long and requests arriving
// meanwhile join the next launch instead of waiting behind it.
// The plain form launches every request on its own as soon as it is
// admitted, with the same kernels.
#include <hip/hip_runtime_api.h>
#include <immintrin.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <list>
#include <map>
#include <vector>

#include "vmt.h"
#include "vmt_common.hpp"
#include "vmt_internal.hpp"
#include "vmt_launch.hpp"

namespace {

// Output placement within the arena plus the in-flight budget. Reuse mode:
// first fit with coalescing (space is recycled as requests complete). Retain
// mode: bump allocation, nothing is overwritten during a run. 256-byte granules.
class Arena {
public:
    Arena(uint64_t capacity, uint64_t budget, bool retain) : capacity_(capacity), budget_(budget), retain_(retain) {
        free_[0] = capacity;
    }
    bool alloc(uint64_t bytes, uint64_t* off) {
        bytes = (bytes + 255) / 256 * 256;
        if (inflight_ + bytes > budget_) return false;
        if (retain_) {
            if (bump_ + bytes > capacity_) return false;
            *off = bump_;
            bump_ += bytes;
            inflight_ += bytes;
            return true;
        }
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const uint64_t rest = it->second - bytes, start = it->first + bytes;
                free_.erase(it);
                if (rest) free_[start] = rest;
                inflight_ += bytes;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        inflight_ -= bytes;
        if (retain_) return;
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

private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t capacity_, budget_, inflight_ = 0, bump_ = 0;
    bool retain_;
};

using Clock = std::chrono::steady_clock;

}  // namespace

struct vmt_server {
    vmt_ctx* ctx = nullptr;
    int variant = 0;
    uint32_t M = 0;
    int out_kind = 0;
    size_t elem = 4;
    int mode = 0;  // 0 continuous batching, 1 plain
    bool retain = false;
    uint64_t budget = 0;
    uint64_t chunk = 0;  // elements per generation task (0: whole request)
    std::vector<uint8_t*> states;
    uint8_t* arena = nullptr;
    uint64_t capacity = 0;
    vmt::BatchShape shape;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    // batching mode: per stream, room for one task per state of each kind
    std::vector<uint8_t*> d_buf;            // [gen tasks][jump tasks][2 counters]
    std::vector<vmt::BatchTask*> h_gen;     // pinned staging
    std::vector<vmt::JumpTask*> h_jump;
};

namespace {

int server_fail(int code, const char* msg) { return vmt::set_error(code, "%s", msg); }

void destroy_server(vmt_server* s) {
    for (auto st : s->streams) (void)hipStreamSynchronize(st);
    for (auto e : s->events) (void)hipEventDestroy(e);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    for (auto p : s->d_buf) (void)hipFree(p);
    for (auto p : s->h_gen) (void)hipHostFree(p);
    for (auto p : s->h_jump) (void)hipHostFree(p);
    delete s;
}

}  // namespace

extern "C" {

vmt_server* vmt_server_create(vmt_ctx* ctx, void* const* d_states, size_t n_states, void* d_arena, size_t arena_bytes,
                              uint64_t budget_bytes, int out_kind, uint32_t n_streams, int mode, uint64_t chunk_elems,
                              int* status) {
    auto fail = [&](int code, const char* msg) -> vmt_server* {
        int c = server_fail(code, msg);
        if (status) *status = c;
        return nullptr;
    };
    if (!ctx || vmt::ctx_device(ctx) < 0) return fail(VMT_EDEVICE, "server needs a device context");
    if (!d_states || n_states == 0 || !d_arena || arena_bytes == 0) return fail(VMT_EINVAL, "empty states or arena");
    if (n_streams < 1 || n_streams > 16) return fail(VMT_EINVAL, "1 <= streams <= 16");
    if (mode < 0 || mode > 3) return fail(VMT_EINVAL, "mode: bit 0 plain launches, bit 1 retain outputs");
    if ((uintptr_t)d_arena % 256) return fail(VMT_EINVAL, "arena must be 256-byte aligned");
    if (hipSetDevice(vmt::ctx_device(ctx)) != hipSuccess) return fail(VMT_EDEVICE, "hipSetDevice");
    vmt_server* s = new vmt_server;
    s->ctx = ctx;
    s->out_kind = out_kind;
    s->elem = (out_kind == VMT_OUT_U64 || out_kind == VMT_OUT_F64) ? 8 : 4;
    s->retain = (mode & 2) != 0;
    s->chunk = chunk_elems;
    mode &= 1;
    s->mode = mode;
    for (size_t i = 0; i < n_states; i++) {
        int v;
        uint32_t M;
        int st = vmt::ctx_state_info(ctx, d_states[i], &v, &M);
        if (st) {
            if (status) *status = st;
            delete s;
            return nullptr;
        }
        if (i == 0) {
            s->variant = v;
            s->M = M;
        } else if (v != s->variant || M != s->M) {
            delete s;
            return fail(VMT_EINVAL, "server states must share variant and M");
        }
        s->states.push_back(static_cast<uint8_t*>(d_states[i]));
    }
    if (!vmt::batch_supported(s->variant, s->M, out_kind)) {
        delete s;
        return fail(VMT_EVARIANT, "output kind not available for batched generation of these states");
    }
    s->arena = static_cast<uint8_t*>(d_arena);
    s->capacity = s->retain ? arena_bytes : std::min<uint64_t>(arena_bytes, budget_bytes);
    s->budget = std::min<uint64_t>(arena_bytes, budget_bytes);
    vmt::ctx_batch_shape(ctx, s->variant, s->M, out_kind, &s->shape);
    const size_t cap = n_states;
    for (uint32_t i = 0; i < n_streams; i++) {
        hipStream_t st;
        hipEvent_t ev;
        uint8_t* d = nullptr;
        vmt::BatchTask* hg = nullptr;
        vmt::JumpTask* hj = nullptr;
        bool ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) s->streams.push_back(st);
        ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (ok) s->events.push_back(ev);
        if (mode == 0) {
            ok = ok && hipMalloc(&d, cap * (sizeof(vmt::BatchTask) + sizeof(vmt::JumpTask)) + 256) == hipSuccess;
            if (ok) s->d_buf.push_back(d);
            ok = ok && hipHostMalloc(&hg, cap * sizeof(vmt::BatchTask), hipHostMallocDefault) == hipSuccess;
            if (ok) s->h_gen.push_back(hg);
            ok = ok && hipHostMalloc(&hj, cap * sizeof(vmt::JumpTask), hipHostMallocDefault) == hipSuccess;
            if (ok) s->h_jump.push_back(hj);
            ok = ok && vmt::reset_counters(reinterpret_cast<uint32_t*>(
                                               d + cap * (sizeof(vmt::BatchTask) + sizeof(vmt::JumpTask))),
                                           st) == hipSuccess;
        }
        if (!ok) {
            destroy_server(s);
            return fail(VMT_ENOMEM, "stream, event or task buffer allocation failed");
        }
    }
    for (auto st : s->streams) (void)hipStreamSynchronize(st);
    if (status) *status = VMT_OK;
    return s;
}

int vmt_server_run(vmt_server* s, const vmt_request* reqs, size_t n, vmt_result* res, int realtime, double* wall_s) {
    if (!s || (!reqs && n) || (!res && n)) return server_fail(VMT_EINVAL, "null argument");
    if (hipSetDevice(vmt::ctx_device(s->ctx)) != hipSuccess) return server_fail(VMT_EDEVICE, "hipSetDevice");
    const size_t ns = s->states.size();
    // jump polynomials for every k in the trace, on the device before the clock starts
    std::map<uint32_t, std::pair<const uint64_t*, uint32_t>> polys;
    for (size_t i = 0; i < n; i++) {
        res[i] = vmt_result{0, 0, 0, 0, VMT_OK, -1};
        if (reqs[i].state >= ns) {
            res[i].status = VMT_EINVAL;
            continue;
        }
        if (reqs[i].kind == 1) {
            if (reqs[i].k > 65536) {
                res[i].status = VMT_EINVAL;
                continue;
            }
            if (!polys.count(reqs[i].k)) {
                const uint64_t* p;
                uint32_t deg;
                int st = vmt::ctx_pow2_poly(s->ctx, s->variant, reqs[i].k, &p, &deg);
                if (st) return st;
                polys[reqs[i].k] = {p, deg};
            }
        } else if (reqs[i].kind == 0) {
            if (reqs[i].count * s->elem > s->budget) res[i].status = VMT_EINVAL;  // can never be admitted
        } else {
            res[i].status = VMT_EINVAL;
        }
    }
    uint32_t* flags = nullptr;
    vmt::BatchTask* d_one = nullptr;  // plain mode: one task slot and counter pair per request
    if (hipHostMalloc(&flags, std::max<size_t>(n, 1) * sizeof(uint32_t), hipHostMallocCoherent) != hipSuccess)
        return server_fail(VMT_ENOMEM, "flags");
    std::memset(flags, 0, std::max<size_t>(n, 1) * sizeof(uint32_t));
    vmt::BatchTask* h_one = nullptr;
    vmt::JumpTask* h_onej = nullptr;
    uint8_t* d_plain = nullptr;
    if (s->mode == 1) {
        const size_t per = sizeof(vmt::BatchTask) + sizeof(vmt::JumpTask) + 8;
        if (hipMalloc(&d_plain, std::max<size_t>(n, 1) * per) != hipSuccess ||
            hipHostMalloc(&h_one, std::max<size_t>(n, 1) * sizeof(vmt::BatchTask), hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&h_onej, std::max<size_t>(n, 1) * sizeof(vmt::JumpTask), hipHostMallocDefault) != hipSuccess) {
            (void)hipFree(d_plain);
            (void)hipHostFree(h_one);
            (void)hipHostFree(h_onej);
            (void)hipHostFree(flags);
            return server_fail(VMT_ENOMEM, "plain-mode task slots");
        }
        d_one = reinterpret_cast<vmt::BatchTask*>(d_plain);
        uint32_t* ctrs = reinterpret_cast<uint32_t*>(d_plain + n * (sizeof(vmt::BatchTask) + sizeof(vmt::JumpTask)));
        (void)hipMemset(ctrs, 0, n * 8);
        (void)hipDeviceSynchronize();
    }
    const size_t cap = ns;
    const size_t jump_off = cap * sizeof(vmt::BatchTask);
    const size_t ctr_off = cap * (sizeof(vmt::BatchTask) + sizeof(vmt::JumpTask));

    Arena arena(s->capacity, s->budget, s->retain);
    std::vector<uint8_t> busy(ns, 0);
    std::list<uint32_t> queued;   // arrived, not admitted, in arrival order
    std::vector<uint32_t> ready;  // admitted (or continuing), not launched
    std::list<uint32_t> inflight;  // continuous batching: tasks complete in any order
    std::vector<std::deque<uint32_t>> fifo(s->streams.size());  // plain: a stream completes in launch order
    std::vector<uint64_t> produced(n, 0), cur(n, 0);  // elements written so far / in the task in flight
    std::vector<uint32_t> home(n, UINT32_MAX);         // plain: the stream a request's launches go to
    std::vector<int> stream_busy(s->streams.size(), 0);
    auto chunk_len = [&](uint32_t r) {
        const uint64_t left = reqs[r].count - produced[r];
        return s->chunk && left > s->chunk ? s->chunk : left;
    };
    size_t next = 0, done = 0, launches = 0;
    uint32_t rr = 0;
    int err = VMT_OK;
    // order of arrival (the trace is expected sorted, but do not rely on it)
    std::vector<uint32_t> order(n);
    for (size_t i = 0; i < n; i++) order[i] = (uint32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return reqs[a].t_arrival < reqs[b].t_arrival; });
    for (size_t i = 0; i < n; i++)
        if (res[i].status != VMT_OK) done++;
    const auto t0 = Clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(Clock::now() - t0).count(); };
    double last_progress = 0.0;
    const double watchdog_s = 30.0;  // no completion for this long with work in flight: give up

    while (done < n && err == VMT_OK) {
        const double t = now_s();
        bool progress = false;
        bool any_inflight = !inflight.empty();
        for (auto& q : fifo) any_inflight = any_inflight || !q.empty();
        if (any_inflight && t - last_progress > watchdog_s) {
            err = vmt::set_error(VMT_EBUSY, "serving watchdog: no request completed for %.0f s", watchdog_s);
            break;
        }
        // completions: a finished chunk either continues its request or completes it
        auto finish = [&](uint32_t r) {
            if (reqs[r].kind == 0) produced[r] += cur[r];
            if (reqs[r].kind == 0 && produced[r] < reqs[r].count) {
                __atomic_store_n(&flags[r], 0u, __ATOMIC_RELEASE);  // the next chunk raises it again
                ready.push_back(r);
            } else {
                res[r].t_done = now_s();
                if (reqs[r].kind == 0) arena.release(res[r].out_offset, reqs[r].count * s->elem);
                busy[reqs[r].state] = 0;
                done++;
            }
            progress = true;
        };
        for (auto it = inflight.begin(); it != inflight.end();) {
            if (__atomic_load_n(&flags[*it], __ATOMIC_ACQUIRE)) {
                const uint32_t r = *it;
                it = inflight.erase(it);
                finish(r);
            } else {
                ++it;
            }
        }
        for (auto& q : fifo)
            while (!q.empty() && __atomic_load_n(&flags[q.front()], __ATOMIC_ACQUIRE)) {
                const uint32_t r = q.front();
                q.pop_front();
                finish(r);
            }
        for (size_t i = 0; i < s->streams.size(); i++)
            if (stream_busy[i] && hipEventQuery(s->events[i]) == hipSuccess) stream_busy[i] = 0;
        // arrivals
        while (next < n && (!realtime || reqs[order[next]].t_arrival <= t)) {
            const uint32_t r = order[next++];
            if (res[r].status == VMT_OK) queued.push_back(r);
        }
        // admission: arrival order, one request per state in flight, outputs within the budget
        std::vector<uint8_t> blocked;
        for (auto it = queued.begin(); it != queued.end();) {
            const uint32_t r = *it;
            const uint32_t st = reqs[r].state;
            if (busy[st] || (!blocked.empty() && blocked[st])) {
                if (blocked.empty()) blocked.assign(ns, 0);
                blocked[st] = 1;
                ++it;
                continue;
            }
            if (reqs[r].kind == 0) {
                uint64_t off;
                if (!arena.alloc(reqs[r].count * s->elem, &off)) break;  // memory is admitted first come, first served
                res[r].out_offset = off;
            }
            busy[st] = 1;
            res[r].t_admit = now_s();
            ready.push_back(r);
            it = queued.erase(it);
            progress = true;
        }
        // launches
        if (!ready.empty()) {
            if (s->mode == 0) {
                for (size_t si = 0; si < s->streams.size() && !ready.empty(); si++) {
                    if (stream_busy[si]) continue;
                    hipStream_t st = s->streams[si];
                    uint32_t ng = 0, nj = 0;
                    for (uint32_t r : ready) {
                        if (reqs[r].kind == 0) {
                            cur[r] = chunk_len(r);
                            s->h_gen[si][ng++] = vmt::BatchTask{
                                s->states[reqs[r].state], s->arena + res[r].out_offset + produced[r] * s->elem, cur[r],
                                &flags[r]};
                        } else {
                            auto pp = polys[reqs[r].k];
                            s->h_jump[si][nj++] =
                                vmt::JumpTask{s->states[reqs[r].state], pp.first, 0u, pp.second, &flags[r]};
                        }
                        if (res[r].launch < 0) {
                            res[r].t_launch = now_s();
                            res[r].launch = (int)launches;
                        }
                        inflight.push_back(r);
                    }
                    // longest first for the persistent kernel
                    std::stable_sort(s->h_gen[si], s->h_gen[si] + ng,
                                     [](const vmt::BatchTask& a, const vmt::BatchTask& b) { return a.len > b.len; });
                    ready.clear();
                    uint8_t* d = s->d_buf[si];
                    hipError_t e = hipSuccess;
                    if (nj) {
                        e = hipMemcpyAsync(d + jump_off, s->h_jump[si], nj * sizeof(vmt::JumpTask), hipMemcpyHostToDevice, st);
                        if (e == hipSuccess)
                            e = vmt::launch_jump(s->variant, s->M, reinterpret_cast<vmt::JumpTask*>(d + jump_off),
                                                 s->h_jump[si][0], nj, st);
                    }
                    if (ng && e == hipSuccess) {
                        e = hipMemcpyAsync(d, s->h_gen[si], ng * sizeof(vmt::BatchTask), hipMemcpyHostToDevice, st);
                        if (e == hipSuccess)
                            e = vmt::launch_batch(s->variant, s->M, s->out_kind, s->shape,
                                                  reinterpret_cast<vmt::BatchTask*>(d), ng,
                                                  reinterpret_cast<uint32_t*>(d + ctr_off), st);
                    }
                    if (e == hipSuccess) e = hipEventRecord(s->events[si], st);
                    if (e != hipSuccess) {
                        err = vmt::set_error(VMT_EDEVICE, "serving launch: %s", hipGetErrorString(e));
                        break;
                    }
                    stream_busy[si] = 1;
                    launches++;
                    progress = true;
                }
            } else {
                for (uint32_t r : ready) {
                    // a continuing request stays on its stream: its counter pair may still be in use by the
                    // previous launch's last workgroup after the flag is raised, and stream order covers that
                    if (home[r] == UINT32_MAX) home[r] = rr++ % (uint32_t)s->streams.size();
                    const uint32_t si = home[r];
                    hipStream_t st = s->streams[si];
                    hipError_t e;
                    uint8_t* base = d_plain;
                    if (reqs[r].kind == 0) {
                        cur[r] = chunk_len(r);
                        h_one[r] = vmt::BatchTask{s->states[reqs[r].state],
                                                  s->arena + res[r].out_offset + produced[r] * s->elem, cur[r], &flags[r]};
                        vmt::BatchTask* dt = reinterpret_cast<vmt::BatchTask*>(base) + r;
                        uint32_t* ctr = reinterpret_cast<uint32_t*>(
                                            base + n * (sizeof(vmt::BatchTask) + sizeof(vmt::JumpTask))) + 2 * (size_t)r;
                        e = hipMemcpyAsync(dt, &h_one[r], sizeof(vmt::BatchTask), hipMemcpyHostToDevice, st);
                        if (e == hipSuccess) {
                            vmt::BatchShape one = s->shape;
                            one.grid = 1;
                            e = vmt::launch_batch(s->variant, s->M, s->out_kind, one, dt, 1, ctr, st);
                        }
                    } else {
                        auto pp = polys[reqs[r].k];
                        h_onej[r] = vmt::JumpTask{s->states[reqs[r].state], pp.first, 0u, pp.second, &flags[r]};
                        vmt::JumpTask* dj = reinterpret_cast<vmt::JumpTask*>(base + n * sizeof(vmt::BatchTask)) + r;
                        e = hipMemcpyAsync(dj, &h_onej[r], sizeof(vmt::JumpTask), hipMemcpyHostToDevice, st);
                        if (e == hipSuccess) e = vmt::launch_jump(s->variant, s->M, dj, h_onej[r], 1, st);
                    }
                    if (e != hipSuccess) {
                        err = vmt::set_error(VMT_EDEVICE, "serving launch: %s", hipGetErrorString(e));
                        break;
                    }
                    if (res[r].launch < 0) {
                        res[r].t_launch = now_s();
                        res[r].launch = (int)launches;
                    }
                    launches++;
                    fifo[si].push_back(r);
                }
                ready.clear();
                progress = true;
            }
        }
        if (progress) last_progress = now_s();
        else _mm_pause();
    }
    const double wall = now_s();
    for (auto st : s->streams) (void)hipStreamSynchronize(st);
    (void)hipHostFree(flags);
    if (d_plain) {
        (void)hipFree(d_plain);
        (void)hipHostFree(h_one);
        (void)hipHostFree(h_onej);
    }
    if (wall_s) *wall_s = wall;
    return err;
}

int vmt_server_destroy(vmt_server* s) {
    if (!s) return server_fail(VMT_EINVAL, "null server");
    (void)hipSetDevice(vmt::ctx_device(s->ctx));
    destroy_server(s);
    return VMT_OK;
}

}  // extern "C"
