// vmt_tune.cpp -- the launch-shape autotuner.
//
// Every candidate shape of a kernel family is run on scratch states and
// outputs (one untimed launch, then `reps` timed ones, fastest counts); the
// fastest shape is stored in the context through vmt_shape_set. Shapes
// change the speed only: the kernels write the same bits whatever the shape.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "vmt.h"
#include "vmt_common.hpp"
#include "vmt_internal.hpp"
#include "vmt_launch.hpp"

namespace {

size_t elem_bytes(int out_kind) { return out_kind == VMT_OUT_U64 || out_kind == VMT_OUT_F64 ? 8 : 4; }

// Scratch device memory released on every exit path.
struct Scratch {
    std::vector<void*> ptrs;
    void* get(size_t bytes) {
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
        ptrs.push_back(p);
        return p;
    }
    ~Scratch() {
        (void)hipDeviceSynchronize();
        for (void* p : ptrs) (void)hipFree(p);
    }
};

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
};

// Fastest of `reps` timed runs of `launch` after one untimed run, in ms.
template <class F>
int time_best(F launch, int reps, hipStream_t stream, double* best_ms) {
    Timer t;
    if (!t.a || !t.b) return vmt::set_error(VMT_EDEVICE, "hipEventCreate failed");
    hipError_t e = launch();
    if (e != hipSuccess) return vmt::set_error(VMT_EDEVICE, "autotune launch: %s", hipGetErrorString(e));
    double best = 1e300;
    for (int r = 0; r < reps; r++) {
        e = hipEventRecord(t.a, stream);
        if (e == hipSuccess) e = launch();
        if (e == hipSuccess) e = hipEventRecord(t.b, stream);
        if (e == hipSuccess) e = hipEventSynchronize(t.b);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t.a, t.b);
        if (e != hipSuccess) return vmt::set_error(VMT_EDEVICE, "autotune timing: %s", hipGetErrorString(e));
        best = std::min(best, (double)ms);
    }
    *best_ms = best;
    return VMT_OK;
}

}  // namespace

extern "C" {

int vmt_autotune(vmt_ctx* ctx, int family, int variant, uint32_t M, int out_kind, const uint64_t* lens, size_t count,
                 int reps, vmt_shape* best, vmt_shape* tried, size_t tried_cap, size_t* n_tried, hipStream_t stream) {
    if (!ctx || !lens || count == 0 || reps < 1) return vmt::set_error(VMT_EINVAL, "bad autotune arguments");
    if (family != VMT_FAMILY_GENERATE && family != VMT_FAMILY_BATCH)
        return vmt::set_error(VMT_EINVAL, "unknown family %d", family);
    if (family == VMT_FAMILY_GENERATE && count != 1)
        return vmt::set_error(VMT_EINVAL, "the generate family takes one length");
    const int device = vmt::ctx_device(ctx);
    if (device < 0) return vmt::set_error(VMT_EDEVICE, "host-only context");
    if (hipSetDevice(device) != hipSuccess) return vmt::set_error(VMT_EDEVICE, "hipSetDevice");
    const size_t sb = vmt_state_bytes(variant, M);
    if (sb == 0) return vmt::set_error(VMT_EINVAL, "bad variant or M");
    if (family == VMT_FAMILY_BATCH ? !vmt::batch_supported(variant, M, out_kind)
                                   : !vmt::generate_supported(variant, M, M < 16 ? M : 16, out_kind))
        return vmt::set_error(VMT_EVARIANT, "output kind %d not available for variant %d, M=%u", out_kind, variant, M);

    const size_t eb = elem_bytes(out_kind);
    std::vector<uint64_t> offs(count);
    uint64_t total = 0, out_bytes = 0;
    for (size_t i = 0; i < count; i++) {
        offs[i] = total;
        total += (lens[i] * eb + 255) / 256 * 256;
        out_bytes += lens[i] * eb;
    }
    Scratch scratch;
    uint8_t* states = static_cast<uint8_t*>(scratch.get(sb * count));
    uint8_t* out = static_cast<uint8_t*>(scratch.get(std::max<uint64_t>(total, 256)));
    if (!states || !out) return vmt::set_error(VMT_ENOMEM, "autotune scratch (%zu states, %llu output bytes)", count,
                                               (unsigned long long)total);
    // one seeded state, copied to every slot (timing does not depend on the values)
    int st = vmt_init_genrand(ctx, variant, 1, M, states, stream);
    if (st) return st;
    for (size_t i = 1; i < count; i++)
        if (hipMemcpyAsync(states + i * sb, states, sb, hipMemcpyDeviceToDevice, stream) != hipSuccess)
            return vmt::set_error(VMT_EDEVICE, "autotune state copy");
    if (hipStreamSynchronize(stream) != hipSuccess) return vmt::set_error(VMT_EDEVICE, "autotune set-up");

    std::vector<vmt_shape> cand;
    if (family == VMT_FAMILY_GENERATE) {
        // Single launches: lanes per workgroup, timed on at most 2^22 elements (their rate does not depend
        // on the length). Split calls: every chunk length giving 2 to 4096 chunks, timed on the full length.
        const uint64_t n = lens[0];
        const uint64_t epw = vmt::is_sfmt(variant) ? 4 : 1;
        const uint64_t steps = (n + M * epw - 1) / (M * epw);
        auto call = [&](uint64_t len) -> hipError_t {
            int r = out_kind == VMT_OUT_U32   ? vmt_generate_u32(ctx, states, len, (uint32_t*)out, stream)
                    : out_kind == VMT_OUT_U64 ? vmt_generate_u64(ctx, states, len, (uint64_t*)out, stream)
                    : out_kind == VMT_OUT_F32 ? vmt_uniform_f32(ctx, states, len, (float*)out, stream)
                                              : vmt_uniform_f64(ctx, states, len, (double*)out, stream);
            return r == VMT_OK ? hipSuccess : hipErrorLaunchFailure;
        };
        std::vector<vmt_shape> shapes;
        for (uint32_t lpw = 1; lpw <= M && lpw <= 16; lpw *= 2) {
            if (!vmt::generate_supported(variant, M, lpw, out_kind)) continue;
            vmt_shape sh{};
            sh.lanes_per_wg = lpw;
            sh.store_bytes = 16;
            sh.split_log2 = 255;
            shapes.push_back(sh);
        }
        const bool can_split = vmt::is_sfmt(variant) || vmt::batch_supported(variant, M, out_kind);
        // MT chunks run whole (lanes_per_wg = M, the persistent batch kernel) or by lane groups of 1 .. M/2
        // lanes; SFMT chunks always run 16 lanes per workgroup (or M if fewer)
        std::vector<uint32_t> split_lpw{M < 16 ? M : 16};
        for (uint32_t lpw = 1; !vmt::is_sfmt(variant) && lpw < M && lpw <= 16; lpw *= 2)
            if (vmt::generate_supported(variant, M, lpw, out_kind)) split_lpw.push_back(lpw);
        for (uint32_t v = 4; can_split && v <= 40; v++) {
            const uint64_t chunks = (steps + (1ull << v) - 1) >> v;
            if (chunks < 2) break;
            if (chunks > 4096 || (1ull << v) * M * epw * eb < (16u << 10)) continue;
            for (uint32_t lpw : split_lpw) {
                vmt_shape sh{};
                sh.lanes_per_wg = lpw;
                sh.store_bytes = 16;
                sh.split_log2 = v;
                shapes.push_back(sh);
            }
        }
        for (vmt_shape sh : shapes) {
            st = vmt_shape_set(ctx, family, variant, M, out_kind, &sh);
            if (st) break;
            const uint64_t len = sh.split_log2 == 255 ? std::min<uint64_t>(n, 1ull << 22) : n;
            double ms = 0;
            st = time_best([&] { return call(len); }, reps, stream, &ms);
            if (st) break;
            sh.gbps = len * eb / (ms * 1e-3) / 1e9;
            cand.push_back(sh);
        }
        (void)vmt_state_release(ctx, states);
        if (st) {
            (void)vmt_shape_set(ctx, family, variant, M, out_kind, nullptr);
            return st;
        }
    } else {
        (void)vmt_state_release(ctx, states);
        std::vector<uint32_t> order(count);
        std::iota(order.begin(), order.end(), 0u);
        std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return lens[a] > lens[b]; });
        std::vector<vmt::BatchTask> tasks;
        for (uint32_t i : order) tasks.push_back(vmt::BatchTask{states + i * sb, out + offs[i], lens[i], nullptr});
        uint8_t* d_buf = static_cast<uint8_t*>(scratch.get(count * sizeof(vmt::BatchTask) + 512));
        if (!d_buf) return vmt::set_error(VMT_ENOMEM, "autotune task list");
        auto* d_tasks = reinterpret_cast<vmt::BatchTask*>(d_buf);
        auto* d_counter = reinterpret_cast<uint32_t*>(d_buf + (count * sizeof(vmt::BatchTask) + 255) / 256 * 256);
        if (hipMemcpy(d_tasks, tasks.data(), count * sizeof(vmt::BatchTask), hipMemcpyHostToDevice) != hipSuccess ||
            vmt::reset_counters(d_counter, stream) != hipSuccess)
            return vmt::set_error(VMT_EDEVICE, "autotune task upload");
        const uint32_t cus = vmt::device_cus(device);
        for (uint32_t tv = 0; tv <= 2; tv++)
            for (uint32_t sw : {16u, 8u}) {
                if (!vmt::batch_shape_supported(variant, M, out_kind, tv, sw)) continue;
                const uint32_t fit = vmt::batch_max_per_cu(variant, M, out_kind, tv, sw);
                for (uint32_t per_cu = 1; per_cu <= fit; per_cu++) {
                    vmt::BatchShape shape;
                    shape.tv = tv;
                    shape.sw = sw;
                    shape.grid = per_cu * cus;
                    double ms = 0;
                    st = time_best([&] { return vmt::launch_batch(variant, M, out_kind, shape, d_tasks, (uint32_t)count,
                                                                  d_counter, stream); },
                                   reps, stream, &ms);
                    if (st) return st;
                    vmt_shape sh{};
                    sh.lanes_per_wg = M;
                    sh.threads_variant = tv;
                    sh.store_bytes = sw;
                    sh.wg_per_cu = per_cu;
                    sh.threads = vmt::batch_threads(variant, M, out_kind, tv, sw);
                    sh.gbps = out_bytes / (ms * 1e-3) / 1e9;
                    cand.push_back(sh);
                }
            }
    }
    if (cand.empty()) return vmt::set_error(VMT_EVARIANT, "no shape available");
    size_t bi = 0;
    for (size_t i = 1; i < cand.size(); i++)
        if (cand[i].gbps > cand[bi].gbps) bi = i;
    st = vmt_shape_set(ctx, family, variant, M, out_kind, &cand[bi]);
    if (st) return st;
    if (best) *best = cand[bi];
    if (tried)
        for (size_t i = 0; i < cand.size() && i < tried_cap; i++) tried[i] = cand[i];
    if (n_tried) *n_tried = cand.size();
    return VMT_OK;
}

}  // extern "C"
