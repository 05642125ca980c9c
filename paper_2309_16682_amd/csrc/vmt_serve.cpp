// vmt_serve.cpp -- serving loop over device-resident V-states.
//
// Requests (generate n elements from state s, or jump state s by 2^k) arrive
// over time. The loop admits them in arrival order while keeping at most one
// request per state in flight (a state's requests run in order) and the
// outputs in flight within a memory budget. Continuous batching: whenever a
// generation stream is free, every generation task ready so far goes into one
// persistent launch on it (longest first); whenever a jump stream is free,
// every ready jump goes into one jump launch. Tasks add to a completion
// counter in host memory when their outputs and state are written, so memory
// and states are released per request, not per launch.
//
// Large generation requests (more than the chunk size) are either served as
// a run of bounded tasks in successive launches, or -- with splitting -- cut
// into C chunks that run side by side: chunk c starts from the state jumped
// by c * 2^v lane steps (Sec. 3.1; a jump of d steps on every lane skips d * M
// words of the interleaved stream, eq. (combseq)). Chunks 0 .. C-2 run on
// copies of the state held in scratch slots, the state itself is jumped to
// the last chunk, so it ends where the request ends. The copies and jumps are
// a preparation phase on a jump stream; the chunks then join the next
// generation launch.
//
// The plain form launches every request on its own as soon as it is
// admitted, with the same kernels.
#include <hip/hip_runtime_api.h>
#include <immintrin.h>

#include <algorithm>
#include <chrono>
#include <cmath>
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

constexpr uint32_t kJumpStreams = 2;
constexpr uint32_t kSlots = 2048;  // scratch states for split requests

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
int ceil_log2(uint64_t x) { return x <= 1 ? 0 : 64 - __builtin_clzll(x - 1); }

}  // namespace

struct vmt_server {
    vmt_ctx* ctx = nullptr;
    int variant = 0;
    uint32_t M = 0;
    int out_kind = 0;
    size_t elem = 4;
    int mode = 0;  // 0 continuous batching, 1 plain
    bool retain = false;
    bool split = false;
    uint64_t budget = 0;
    uint64_t chunk = 0;  // elements per generation task (0: whole request)
    double watchdog_s = 30.0;  // a run gives up after this long with work in flight and no completion
    std::vector<uint8_t*> states;
    uint8_t* arena = nullptr;
    uint64_t capacity = 0;
    vmt::BatchShape shape;
    // streams [0, n_gen) generate, [n_gen, n_gen + n_jump) jump (batching mode)
    uint32_t n_gen = 0, n_jump = 0;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    size_t task_cap = 0;                // tasks of one kind per launch
    std::vector<uint8_t*> d_buf;        // gen: [tasks][2 counters]; jump: [jump tasks][copy tasks]
    std::vector<uint8_t*> h_buf;        // pinned staging, same layout
    uint8_t* slots = nullptr;           // kSlots scratch states (splitting)
    size_t slot_bytes = 0, state_bytes = 0;
};

namespace {

int server_fail(int code, const char* msg) { return vmt::set_error(code, "%s", msg); }

void destroy_server(vmt_server* s) {
    for (auto st : s->streams) (void)hipStreamSynchronize(st);
    for (auto e : s->events) (void)hipEventDestroy(e);
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    for (auto p : s->d_buf) (void)hipFree(p);
    for (auto p : s->h_buf) (void)hipHostFree(p);
    if (s->slots) (void)hipFree(s->slots);
    delete s;
}

size_t gen_buf_bytes(size_t cap) { return (cap * sizeof(vmt::BatchTask) + 255) / 256 * 256 + 256; }
size_t jump_buf_bytes(size_t cap) {
    return (cap * sizeof(vmt::JumpTask) + 255) / 256 * 256 + cap * sizeof(vmt::CopyTask);
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
    if (!ctx) return fail(VMT_EINVAL, "null context");
    if (!d_states || n_states == 0 || !d_arena || arena_bytes == 0) return fail(VMT_EINVAL, "empty states or arena");
    if (vmt::reject_duplicate_states(d_states, n_states)) {  // two requests could then run one state at once
        if (status) *status = VMT_EINVAL;
        return nullptr;
    }
    if (vmt::ctx_device(ctx) < 0) return fail(VMT_EDEVICE, "server needs a device context");
    if (n_streams < 1 || n_streams > 16) return fail(VMT_EINVAL, "1 <= streams <= 16");
    if (mode < 0 || mode > 7) return fail(VMT_EINVAL, "mode: bit 0 plain launches, bit 1 retain outputs, bit 2 split");
    if ((mode & 1) && (mode & 4)) return fail(VMT_EINVAL, "the plain form does not split requests");
    if ((mode & 4) && chunk_elems == 0) return fail(VMT_EINVAL, "splitting needs a chunk size");
    if ((uintptr_t)d_arena % 256) return fail(VMT_EINVAL, "arena must be 256-byte aligned");
    if (hipSetDevice(vmt::ctx_device(ctx)) != hipSuccess) return fail(VMT_EDEVICE, "hipSetDevice");
    vmt_server* s = new vmt_server;
    s->ctx = ctx;
    s->out_kind = out_kind;
    s->elem = (out_kind == VMT_OUT_U64 || out_kind == VMT_OUT_F64) ? 8 : 4;
    s->retain = (mode & 2) != 0;
    s->split = (mode & 4) != 0;
    s->chunk = chunk_elems;
    s->mode = mode & 1;
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
    s->state_bytes = vmt_state_bytes(s->variant, s->M);
    s->slot_bytes = (s->state_bytes + 255) / 256 * 256;
    vmt::ctx_batch_shape(ctx, s->variant, s->M, out_kind, &s->shape);
    s->n_gen = n_streams;
    s->n_jump = s->mode == 0 ? kJumpStreams : 0;
    s->task_cap = n_states + (s->split ? kSlots : 0);
    bool ok = true;
    if (s->split) ok = hipMalloc(&s->slots, kSlots * s->slot_bytes) == hipSuccess;
    for (uint32_t i = 0; ok && i < s->n_gen + s->n_jump; i++) {
        hipStream_t st;
        hipEvent_t ev;
        ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
        if (ok) s->streams.push_back(st);
        ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
        if (ok) s->events.push_back(ev);
        if (s->mode == 0) {
            const size_t bytes = i < s->n_gen ? gen_buf_bytes(s->task_cap) : jump_buf_bytes(s->task_cap);
            uint8_t* d = nullptr;
            uint8_t* h = nullptr;
            ok = ok && hipMalloc(&d, bytes) == hipSuccess;
            if (ok) s->d_buf.push_back(d);
            ok = ok && hipHostMalloc(&h, bytes, hipHostMallocDefault) == hipSuccess;
            if (ok) s->h_buf.push_back(h);
            if (ok && i < s->n_gen)
                ok = vmt::reset_counters(reinterpret_cast<uint32_t*>(d + bytes - 256), st) == hipSuccess;
        }
    }
    if (!ok) {
        destroy_server(s);
        return fail(VMT_ENOMEM, "stream, event, task buffer or scratch state allocation failed");
    }
    for (auto st : s->streams) (void)hipStreamSynchronize(st);
    if (status) *status = VMT_OK;
    return s;
}

int vmt_server_run(vmt_server* s, const vmt_request* reqs, size_t n, vmt_result* res, int realtime, double* wall_s) {
    if (!s || (!reqs && n) || (!res && n)) return server_fail(VMT_EINVAL, "null argument");
    if (hipSetDevice(vmt::ctx_device(s->ctx)) != hipSuccess) return server_fail(VMT_EDEVICE, "hipSetDevice");
    const size_t ns = s->states.size();
    const uint32_t M = s->M;
    // per request: chunks when split (0: not split) and log2 of the chunk length in lane steps
    std::vector<uint32_t> nchunks(n, 0);
    std::vector<int> vlog(n, -1);
    // jump polynomials for every k and every split in the trace, on the device before the clock starts
    std::map<uint32_t, std::pair<const uint64_t*, uint32_t>> polys;
    std::map<int, size_t> split_need;  // v -> chunks - 1
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
            if (reqs[i].count * s->elem > s->budget) {
                res[i].status = VMT_EINVAL;  // can never be admitted
            } else if (s->split && reqs[i].count > s->chunk) {
                // chunks of 2^v lane steps, at least the chunk size, at most kSlots + 1 of them
                const uint64_t steps = ceil_div(reqs[i].count, M);
                int v = std::max(ceil_log2(ceil_div(s->chunk, M)), 4);
                while (ceil_div(steps, 1ull << v) > kSlots + 1) v++;
                const uint64_t C = ceil_div(steps, 1ull << v);
                if (C >= 2) {
                    nchunks[i] = (uint32_t)C;
                    vlog[i] = v;
                    split_need[v] = std::max<size_t>(split_need[v], C - 1);
                }
            }
        } else {
            res[i].status = VMT_EINVAL;
        }
    }
    std::map<int, std::pair<const uint64_t*, std::vector<uint32_t>>> split_polys;
    for (auto& kv : split_need) {
        auto& e = split_polys[kv.first];
        int st = vmt::ctx_split_polys(s->ctx, s->variant, kv.first, kv.second, &e.first, &e.second);
        if (st) return st;
    }
    uint32_t* flags = nullptr;  // completion counts, one per request
    if (hipHostMalloc(&flags, std::max<size_t>(n, 1) * sizeof(uint32_t), hipHostMallocCoherent) != hipSuccess)
        return server_fail(VMT_ENOMEM, "flags");
    std::memset(flags, 0, std::max<size_t>(n, 1) * sizeof(uint32_t));
    vmt::BatchTask* h_one = nullptr;  // plain mode: one task slot and counter pair per request
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
        uint32_t* ctrs = reinterpret_cast<uint32_t*>(d_plain + n * (sizeof(vmt::BatchTask) + sizeof(vmt::JumpTask)));
        (void)hipMemset(ctrs, 0, n * 8);
        (void)hipDeviceSynchronize();
    }

    Arena arena(s->capacity, s->budget, s->retain);
    std::vector<uint8_t> busy(ns, 0);
    std::list<uint32_t> queued;       // arrived, not admitted, in arrival order
    std::vector<uint32_t> ready_gen;  // generation tasks ready to launch (a split request: all its chunks)
    std::vector<uint32_t> ready_jump; // jumps and split preparations ready to launch
    std::list<uint32_t> inflight;     // batching: requests with tasks in flight (they complete in any order)
    std::vector<std::deque<uint32_t>> fifo(s->streams.size());  // plain: a stream completes in launch order
    std::vector<uint64_t> produced(n, 0), cur(n, 0);  // elements written so far / in the task in flight
    std::vector<uint32_t> target(n, 0);               // completion count that ends the tasks in flight
    std::vector<uint8_t> prepared(n, 0);              // split: copies and jumps done
    std::vector<uint32_t> home(n, UINT32_MAX);        // plain: the stream a request's launches go to
    std::vector<std::vector<uint32_t>> slot_of(n);    // split: scratch slots of chunks 0 .. C-2
    std::vector<uint32_t> free_slots;
    for (uint32_t i = 0; s->split && i < kSlots; i++) free_slots.push_back(kSlots - 1 - i);
    std::vector<int> stream_busy(s->streams.size(), 0);
    auto chunk_len = [&](uint32_t r) {
        const uint64_t left = reqs[r].count - produced[r];
        return s->chunk && left > s->chunk ? s->chunk : left;
    };
    auto slot_ptr = [&](uint32_t slot) { return s->slots + (size_t)slot * s->slot_bytes; };
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
    const double watchdog_s = s->watchdog_s;
    std::vector<uint8_t> completed(n, 0);
    auto mark_launch = [&](uint32_t r) {
        if (res[r].launch < 0) {
            res[r].t_launch = now_s();
            res[r].launch = (int)launches;
        }
    };

    while (done < n && err == VMT_OK) {
        const double t = now_s();
        bool progress = false;
        bool any_inflight = !inflight.empty();
        for (auto& q : fifo) any_inflight = any_inflight || !q.empty();
        if (any_inflight && t - last_progress >= watchdog_s) {
            err = vmt::set_error(VMT_EBUSY, "serving watchdog: no request completed for %.0f s", watchdog_s);
            break;
        }
        // completions: a finished phase either leads to the next one or completes the request
        auto finish = [&](uint32_t r) {
            progress = true;
            if (reqs[r].kind == 0 && nchunks[r] && !prepared[r]) {
                prepared[r] = 1;  // copies and jumps done: the chunks can run
                ready_gen.push_back(r);
                return;
            }
            if (reqs[r].kind == 0 && !nchunks[r]) {
                produced[r] += cur[r];
                if (produced[r] < reqs[r].count) {  // the next task of a long request
                    ready_gen.push_back(r);
                    return;
                }
            }
            res[r].t_done = now_s();
            completed[r] = 1;
            if (reqs[r].kind == 0) arena.release(res[r].out_offset, reqs[r].count * s->elem);
            for (uint32_t sl : slot_of[r]) free_slots.push_back(sl);
            slot_of[r].clear();
            busy[reqs[r].state] = 0;
            done++;
        };
        for (auto it = inflight.begin(); it != inflight.end();) {
            if (__atomic_load_n(&flags[*it], __ATOMIC_ACQUIRE) == target[*it]) {
                const uint32_t r = *it;
                it = inflight.erase(it);
                finish(r);
            } else {
                ++it;
            }
        }
        for (auto& q : fifo)
            while (!q.empty() && __atomic_load_n(&flags[q.front()], __ATOMIC_ACQUIRE) == target[q.front()]) {
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
        // admission: arrival order, one request per state in flight, outputs within the budget, scratch
        // states for split requests (memory and slots are granted first come, first served)
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
            if (nchunks[r] && free_slots.size() < nchunks[r] - 1) break;
            if (reqs[r].kind == 0) {
                uint64_t off;
                if (!arena.alloc(reqs[r].count * s->elem, &off)) break;
                res[r].out_offset = off;
            }
            for (uint32_t c = 0; c + 1 < nchunks[r]; c++) {
                slot_of[r].push_back(free_slots.back());
                free_slots.pop_back();
            }
            busy[st] = 1;
            res[r].t_admit = now_s();
            if (reqs[r].kind == 1 || nchunks[r]) ready_jump.push_back(r);
            else ready_gen.push_back(r);
            it = queued.erase(it);
            progress = true;
        }
        // launches
        if (s->mode == 0) {
            // jumps and split preparations, on the jump streams
            for (uint32_t si = s->n_gen; si < s->n_gen + s->n_jump && !ready_jump.empty(); si++) {
                if (stream_busy[si]) continue;
                hipStream_t st = s->streams[si];
                uint8_t* h = s->h_buf[si];
                uint8_t* d = s->d_buf[si];
                const size_t copy_off = (s->task_cap * sizeof(vmt::JumpTask) + 255) / 256 * 256;
                auto* hj = reinterpret_cast<vmt::JumpTask*>(h);
                auto* hc = reinterpret_cast<vmt::CopyTask*>(h + copy_off);
                uint32_t nj = 0, nc = 0;
                for (uint32_t r : ready_jump) {
                    uint8_t* X = s->states[reqs[r].state];
                    if (reqs[r].kind == 1) {
                        auto pp = polys[reqs[r].k];
                        hj[nj++] = vmt::JumpTask{X, pp.first, 0u, pp.second, &flags[r]};
                        target[r] += 1;
                    } else {
                        // chunk c < C-1 on a copy jumped by c 2^v, the state itself jumped to the last chunk
                        const auto& sp = split_polys[vlog[r]];
                        const uint32_t C = nchunks[r];
                        for (uint32_t c = 0; c + 1 < C; c++) hc[nc++] = vmt::CopyTask{X, slot_ptr(slot_of[r][c])};
                        for (uint32_t c = 1; c < C; c++) {
                            uint8_t* stc = c + 1 == C ? X : slot_ptr(slot_of[r][c]);
                            hj[nj++] = vmt::JumpTask{stc, sp.first + (size_t)(c - 1) * vmt::kPolyWords, 0u,
                                                     sp.second[c - 1], &flags[r]};
                        }
                        target[r] += C - 1;
                    }
                    mark_launch(r);
                    inflight.push_back(r);
                }
                ready_jump.clear();
                hipError_t e = hipSuccess;
                if (nj) e = hipMemcpyAsync(d, h, nj * sizeof(vmt::JumpTask), hipMemcpyHostToDevice, st);
                if (e == hipSuccess && nc)
                    e = hipMemcpyAsync(d + copy_off, h + copy_off, nc * sizeof(vmt::CopyTask), hipMemcpyHostToDevice, st);
                if (e == hipSuccess && nc)
                    e = vmt::launch_copy_states(reinterpret_cast<vmt::CopyTask*>(d + copy_off), nc,
                                                (uint32_t)s->state_bytes, st);
                if (e == hipSuccess && nj)
                    e = vmt::launch_jump(s->variant, M, reinterpret_cast<vmt::JumpTask*>(d), hj[0], nj, st);
                if (e == hipSuccess) e = hipEventRecord(s->events[si], st);
                if (e != hipSuccess) {
                    err = vmt::set_error(VMT_EDEVICE, "serving jump launch: %s", hipGetErrorString(e));
                    break;
                }
                stream_busy[si] = 1;
                launches++;
                progress = true;
            }
            // generation, on the generation streams
            for (uint32_t si = 0; si < s->n_gen && !ready_gen.empty() && err == VMT_OK; si++) {
                if (stream_busy[si]) continue;
                hipStream_t st = s->streams[si];
                auto* hg = reinterpret_cast<vmt::BatchTask*>(s->h_buf[si]);
                uint32_t ng = 0;
                for (uint32_t r : ready_gen) {
                    uint8_t* X = s->states[reqs[r].state];
                    uint8_t* out = s->arena + res[r].out_offset;
                    if (nchunks[r]) {
                        const uint32_t C = nchunks[r];
                        const uint64_t E = (1ull << vlog[r]) * M;
                        for (uint32_t c = 0; c < C; c++) {
                            uint8_t* stc = c + 1 == C ? X : slot_ptr(slot_of[r][c]);
                            const uint64_t len = c + 1 < C ? E : reqs[r].count - (uint64_t)c * E;
                            hg[ng++] = vmt::BatchTask{stc, out + (uint64_t)c * E * s->elem, len, &flags[r]};
                        }
                        target[r] += C;
                    } else {
                        cur[r] = chunk_len(r);
                        hg[ng++] = vmt::BatchTask{X, out + produced[r] * s->elem, cur[r], &flags[r]};
                        target[r] += 1;
                    }
                    mark_launch(r);
                    inflight.push_back(r);
                }
                ready_gen.clear();
                // longest first for the persistent kernel
                std::stable_sort(hg, hg + ng, [](const vmt::BatchTask& a, const vmt::BatchTask& b) { return a.len > b.len; });
                uint8_t* d = s->d_buf[si];
                hipError_t e = hipMemcpyAsync(d, hg, ng * sizeof(vmt::BatchTask), hipMemcpyHostToDevice, st);
                if (e == hipSuccess)
                    e = vmt::launch_batch(s->variant, M, s->out_kind, s->shape, reinterpret_cast<vmt::BatchTask*>(d), ng,
                                          reinterpret_cast<uint32_t*>(d + gen_buf_bytes(s->task_cap) - 256), st);
                if (e == hipSuccess) e = hipEventRecord(s->events[si], st);
                if (e != hipSuccess) {
                    err = vmt::set_error(VMT_EDEVICE, "serving launch: %s", hipGetErrorString(e));
                    break;
                }
                stream_busy[si] = 1;
                launches++;
                progress = true;
            }
        } else if (!ready_gen.empty() || !ready_jump.empty()) {
            std::vector<uint32_t> ready(ready_jump);
            ready.insert(ready.end(), ready_gen.begin(), ready_gen.end());
            ready_jump.clear();
            ready_gen.clear();
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
                        e = vmt::launch_batch(s->variant, M, s->out_kind, one, dt, 1, ctr, st);
                    }
                } else {
                    auto pp = polys[reqs[r].k];
                    h_onej[r] = vmt::JumpTask{s->states[reqs[r].state], pp.first, 0u, pp.second, &flags[r]};
                    vmt::JumpTask* dj = reinterpret_cast<vmt::JumpTask*>(base + n * sizeof(vmt::BatchTask)) + r;
                    e = hipMemcpyAsync(dj, &h_onej[r], sizeof(vmt::JumpTask), hipMemcpyHostToDevice, st);
                    if (e == hipSuccess) e = vmt::launch_jump(s->variant, M, dj, h_onej[r], 1, st);
                }
                if (e != hipSuccess) {
                    err = vmt::set_error(VMT_EDEVICE, "serving launch: %s", hipGetErrorString(e));
                    break;
                }
                target[r] += 1;
                mark_launch(r);
                launches++;
                fifo[si].push_back(r);
            }
            progress = true;
        }
        if (progress) last_progress = now_s();
        else _mm_pause();
    }
    const double wall = now_s();
    for (auto st : s->streams) (void)hipStreamSynchronize(st);
    if (err != VMT_OK)  // the run gave up: what it launched has run (the streams are drained), the rest has not
        for (size_t i = 0; i < n; i++)
            if (res[i].status == VMT_OK && !completed[i]) res[i].status = err;
    (void)hipHostFree(flags);
    if (d_plain) {
        (void)hipFree(d_plain);
        (void)hipHostFree(h_one);
        (void)hipHostFree(h_onej);
    }
    if (wall_s) *wall_s = wall;
    return err;
}

int vmt_server_set_watchdog(vmt_server* s, double seconds) {
    if (!s) return server_fail(VMT_EINVAL, "null server");
    if (!(seconds >= 0.0) || !std::isfinite(seconds)) return server_fail(VMT_EINVAL, "watchdog: 0 <= seconds < inf");
    s->watchdog_s = seconds;
    return VMT_OK;
}

int vmt_server_destroy(vmt_server* s) {
    if (!s) return server_fail(VMT_EINVAL, "null server");
    (void)hipSetDevice(vmt::ctx_device(s->ctx));
    destroy_server(s);
    return VMT_OK;
}

}  // extern "C"
