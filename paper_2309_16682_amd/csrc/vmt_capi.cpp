// vmt_capi.cpp -- the C ABI declared in include/vmt.h.
//
// Host side of the runtime: argument checks, the state registry, the jump
// polynomials (computed here on the CPU with gf2poly, applied on the GPU),
// task lists for batched calls, and kernel launches on the caller's stream.
#include "vmt.h"

#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "gf2poly.hpp"
#include "vmt_common.hpp"
#include "vmt_internal.hpp"
#include "vmt_launch.hpp"

using vmt::Words;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(VMT_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool valid_M(uint32_t M) { return M >= 1 && M <= 64 && (M & (M - 1)) == 0; }
bool valid_variant(int v) { return v >= VMT_MT32 && v < (int)vmt::kVariants; }
int log2u(uint32_t M) { return 31 - __builtin_clz(M); }

struct StateInfo {
    int variant;
    uint32_t M;
};

struct DevPoly {
    uint64_t* d = nullptr;  // kPolyWords words on the device
    uint32_t deg = 0;
};

// Jump polynomials for splitting one stream into chunks of 2^v lane steps:
// slot c - 1 holds t^(c 2^v) mod mu.
struct SplitTable {
    std::vector<Words> host;
    std::vector<uint32_t> deg;
    uint64_t* d = nullptr;      // cap slots of kPolyWords words
    uint32_t* d_deg = nullptr;  // their degrees
    size_t cap = 0, uploaded = 0;
};

struct LaneTable {
    uint64_t* d = nullptr;  // M slots of kPolyWords words
    uint32_t max_deg = 0;
};

// Recurrence polynomial of each bit of a V-stream (linear-complexity check).
struct CheckPoly {
    Words host;
    uint32_t deg = 0;
    uint32_t* d = nullptr;  // one device block: bit pattern, coefficient list, chunk offsets
    vmt::CheckPolyDev dev;
};

}  // namespace

// A stream's workspace (see vmt_ctx::split_ws); `mu` is held from taking the
// workspace until the call's last launch is enqueued, so that calls issued on
// one stream from several host threads do not interleave their launches over it.
struct StreamWorkspace {
    uint8_t* buf = nullptr;
    size_t cap = 0;
    std::mutex mu;
};

struct vmt_ctx {
    int device = -1;
    std::mutex mu;
    std::unordered_map<const void*, StateInfo> reg;
    std::unique_ptr<vmt::PolyMod> ring[vmt::kVariants];
    std::map<uint64_t, Words> pow2[vmt::kVariants];                 // k -> t^(2^k) mod mu
    std::map<uint32_t, LaneTable> lanes[vmt::kVariants];            // M -> lane polynomials on the device
    std::map<std::vector<uint64_t>, DevPoly> jumps[vmt::kVariants];  // distance -> jump polynomial on the device (bounded)
    std::map<uint32_t, DevPoly> pow2_dev[vmt::kVariants];            // k -> t^(2^k) on the device (k <= 65536, never evicted:
                                                         // servers and batches hold these pointers)
    std::map<uint32_t, vmt_shape> shapes;  // shape_key -> launch shape set by the caller or the autotuner
    std::map<uint32_t, SplitTable> split[vmt::kVariants];  // log2 chunk -> t^(c 2^v) mod mu, c = 1, 2, ...
    std::map<uint32_t, CheckPoly> check[vmt::kVariants];   // M -> recurrence polynomial of the V-stream's bits
    std::vector<void*> retired;                 // replaced device tables (queued kernels may still read them)
    // Workspace per stream of split calls and jumps (copies, task lists, counters, jump parts): calls on one stream
    // use it in stream order, and everything in it that a call reads is written by the call's own launches, so it
    // is reused from call to call without a stream-ordered allocation and free each time (those leave the GPU idle
    // between calls).
    std::unordered_map<hipStream_t, std::unique_ptr<StreamWorkspace>> split_ws;
};

struct vmt_batch_plan {
    vmt_ctx* ctx;
    int variant;
    uint32_t M;
    int out_kind;
    uint32_t count;
    vmt::BatchShape shape;
    vmt::BatchTask* d_tasks;
    uint32_t* d_counter;
};

namespace {

int set_device(vmt_ctx* ctx) {
    if (!ctx) return fail(VMT_EINVAL, "null context");
    if (ctx->device < 0) return fail(VMT_EDEVICE, "host-only context (created with device -1)");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    return VMT_OK;
}

// ---- polynomials (caller holds ctx->mu) ---------------------------------------

vmt::PolyMod& ring(vmt_ctx* ctx, int variant) {
    if (!ctx->ring[variant]) ctx->ring[variant].reset(new vmt::PolyMod(vmt::generator_minpoly(variant)));
    return *ctx->ring[variant];
}

// t^(2^k) mod mu, extending the cached squaring chain from the nearest k below.
// MT19937-32/-64: mu is irreducible of degree D = 19937 (2^D - 1, the period,
// is prime), so t^(2^D) = t (Frobenius): t^(2^k) = t^(2^(k mod D)), and for
// k mod D close to D it is D - (k mod D) square roots of t -- the lane
// distances 2^(19937 - log2 M) cost a few square roots instead of ~19,930
// squarings.
const Words& pow2(vmt_ctx* ctx, int variant, uint64_t k) {
    auto& cache = ctx->pow2[variant];
    auto it = cache.find(k);
    if (it != cache.end()) return it->second;
    vmt::PolyMod& R = ring(ctx, variant);
    constexpr uint64_t kD = 19937;
    if (!vmt::is_sfmt(variant) && R.degree() == (int)kD) {
        const uint64_t e = k % kD;
        if (e != k) {
            Words v = pow2(ctx, variant, e);
            return cache[k] = std::move(v);
        }
        if (kD - e <= 64) {
            Words cur(R.words(), 0);
            cur[0] = 2;  // t
            for (uint64_t i = 0; i < kD - e; i++) cur = R.sqrt(cur);
            return cache[k] = std::move(cur);
        }
    }
    auto below = cache.lower_bound(k);
    Words cur;
    uint64_t from = 0;
    if (below != cache.begin()) {
        --below;
        cur = below->second;
        from = below->first;
    } else {
        cur.assign(R.words(), 0);
        cur[0] = 2;  // t
    }
    for (uint64_t i = from; i < k; i++) {
        cur = R.sqr(cur);
        if (i + 1 <= 512 || (i + 1) % 1024 == 0) cache[i + 1] = cur;  // keep small k and checkpoints
    }
    cache[k] = cur;
    return cache[k];
}

int upload_poly(const Words& p, DevPoly* out) {
    std::vector<uint64_t> buf(vmt::kPolyWords, 0);
    const int deg = vmt::poly_degree(p);
    if (deg >= vmt::kPolyWords * 64) return fail(VMT_EINVAL, "polynomial too large");
    std::copy(p.begin(), p.begin() + std::min(p.size(), buf.size()), buf.begin());
    hipError_t e = hipMalloc(&out->d, buf.size() * 8);
    if (e != hipSuccess) return fail(VMT_ENOMEM, "hipMalloc(poly): %s", hipGetErrorString(e));
    e = hipMemcpy(out->d, buf.data(), buf.size() * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(poly)");
    out->deg = deg < 0 ? 0 : uint32_t(deg);
    return VMT_OK;
}

// Recurrence polynomial A of every bit of the V-stream of M lanes (caller
// holds ctx->mu). Lane t starts t J steps after lane 0, J = 2^(19937 - log2 M)
// (Sec. 3). For a root alpha of the degree-19937 factor phi of mu,
// alpha^(2^19937) = alpha, so alpha^J is the M-th root of alpha: the
// interleaved sequence of a bit is a trace sequence of alpha^J, a conjugate
// of alpha, and obeys phi again. MT19937: mu = phi, A = mu. SFMT19937:
// mu = phi psi (psi of degree 31); the psi part of lane t is a sequence of
// psi shifted by t J, the interleave of M of them obeys psi(t^M) = psi^M,
// so A = phi psi^M for the sequence of 128-bit words.
CheckPoly& check_poly(vmt_ctx* ctx, int variant, uint32_t M) {
    auto it = ctx->check[variant].find(M);
    if (it != ctx->check[variant].end()) return it->second;
    vmt::PolyMod& R = ring(ctx, variant);
    Words A = R.modulus();
    if (vmt::is_sfmt(variant)) {
        Words f = pow2(ctx, variant, vmt::mexp(variant));  // t^(2^MEXP) mod mu
        f[0] ^= 2;                            // - t
        const Words phi = vmt::poly_gcd(R.modulus(), f);
        Words rem;
        Words psiM = vmt::poly_div(R.modulus(), phi, &rem);
        for (uint32_t m = 1; m < M; m *= 2) psiM = vmt::poly_mul(psiM, psiM);
        A = vmt::poly_mul(phi, psiM);
    }
    vmt::poly_trim(A);
    CheckPoly& c = ctx->check[variant][M];
    c.host = A;
    c.deg = (uint32_t)vmt::poly_degree(A);
    return c;
}

// Lane polynomials t^(t J) mod mu, t = 0..M-1, J = 2^(19937 - log2 M) (Sec. 3, Table jvalues).
int lane_table(vmt_ctx* ctx, int variant, uint32_t M, LaneTable** out) {
    auto it = ctx->lanes[variant].find(M);
    if (it != ctx->lanes[variant].end()) {
        *out = &it->second;
        return VMT_OK;
    }
    vmt::PolyMod& R = ring(ctx, variant);
    std::vector<uint64_t> host((size_t)M * vmt::kPolyWords, 0);
    host[0] = 1;  // lane 0: t^0
    uint32_t max_deg = 0;
    if (M > 1) {
        const Words gJ = pow2(ctx, variant, vmt::mexp(variant) - (uint32_t)log2u(M));
        Words g = gJ;
        for (uint32_t t = 1; t < M; t++) {
            if (t > 1) g = R.mul(g, gJ);
            const int d = vmt::poly_degree(g);
            max_deg = std::max<uint32_t>(max_deg, d < 0 ? 0 : uint32_t(d));
            std::copy(g.begin(), g.begin() + std::min<size_t>(g.size(), vmt::kPolyWords),
                      host.begin() + (size_t)t * vmt::kPolyWords);
        }
    }
    LaneTable lt;
    lt.max_deg = max_deg;
    hipError_t e = hipMalloc(&lt.d, host.size() * 8);
    if (e != hipSuccess) return fail(VMT_ENOMEM, "hipMalloc(lane table): %s", hipGetErrorString(e));
    e = hipMemcpy(lt.d, host.data(), host.size() * 8, hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(lane table)");
    auto res = ctx->lanes[variant].emplace(M, lt);
    *out = &res.first->second;
    return VMT_OK;
}

// Device copy of t^(2^k) mod mu (k <= 65536), kept for the context's lifetime.
int pow2_dev(vmt_ctx* ctx, int variant, uint32_t k, DevPoly** out) {
    auto& cache = ctx->pow2_dev[variant];
    auto it = cache.find(k);
    if (it == cache.end()) {
        DevPoly dp;
        int st = upload_poly(pow2(ctx, variant, k), &dp);
        if (st) return st;
        it = cache.emplace(k, dp).first;
    }
    *out = &it->second;
    return VMT_OK;
}

// Device copy of t^d mod mu, cached per distance.
int jump_table(vmt_ctx* ctx, int variant, const std::vector<uint64_t>& dist, const Words* known, DevPoly** out) {
    auto& cache = ctx->jumps[variant];
    auto it = cache.find(dist);
    if (it != cache.end()) {
        *out = &it->second;
        return VMT_OK;
    }
    if (cache.size() >= 4096) {  // bound the cache (entries are used only by the call that looked them up)
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
        for (auto& kv : cache) (void)hipFree(kv.second.d);
        cache.clear();
    }
    Words g = known ? *known : ring(ctx, variant).t_pow(dist.data(), dist.size());
    DevPoly dp;
    int st = upload_poly(g, &dp);
    if (st) return st;
    auto res = cache.emplace(dist, dp);
    *out = &res.first->second;
    return VMT_OK;
}

int lookup(vmt_ctx* ctx, const void* d_state, StateInfo* info) {
    if (!d_state) return fail(VMT_EINVAL, "null state");
    auto it = ctx->reg.find(d_state);
    if (it == ctx->reg.end())
        return fail(VMT_ESTATE, "state %p was not initialised or imported through this context", d_state);
    *info = it->second;
    return VMT_OK;
}

uint32_t shape_key(int family, int variant, uint32_t M, int out_kind) {
    return (uint32_t)family | (uint32_t)variant << 1 | (uint32_t)out_kind << 4 | (uint32_t)log2u(M) << 6;
}

// Shape in force for (family, variant, M, out_kind): the stored one, else the
// default (caller holds ctx->mu).
vmt_shape current_shape(vmt_ctx* ctx, int family, int variant, uint32_t M, int out_kind) {
    auto it = ctx->shapes.find(shape_key(family, variant, M, out_kind));
    if (it != ctx->shapes.end()) return it->second;
    vmt_shape d{};  // lanes_per_wg 0: chosen per call (auto_lpw)
    d.store_bytes = 16;
    return d;
}

// Lanes per workgroup for one launch when the shape leaves it open: MT19937
// calls of 256 KiB or more run one lane per workgroup (M workgroups write
// side by side, about twice the rate of one workgroup for all lanes);
// smaller calls and SFMT19937 keep whole groups of up to 16 lanes.
uint32_t auto_lpw(int variant, uint32_t M, uint64_t n, size_t eb) {
    if (!vmt::is_sfmt(variant) && n * eb >= (256u << 10)) return 1;
    return M < 16 ? M : 16;
}

size_t out_elem_bytes(int out_kind) { return out_kind == VMT_OUT_U64 || out_kind == VMT_OUT_F64 ? 8 : 4; }

// ---- splitting one stream over many workgroups --------------------------------
//
// A call for n elements is cut into C chunks of 2^v lane steps (2^v * M
// stream words). Chunk c starts from the state jumped by c * 2^v steps: a
// jump of d steps on every lane skips exactly d * M words of the interleaved
// stream (Sec. 3, eq. (combseq)), so chunk c is elements [c E, (c + 1) E) of
// the request. Chunks 0 .. C-2 run on copies of the state; the state itself
// is jumped to the last chunk and runs it, so it ends where the call ends.
// All chunks run as one batched launch.

constexpr uint32_t kNeverSplit = 255;
constexpr uint64_t kMaxChunks = 65535;  // chunks are a grid dimension

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }
int ceil_log2(uint64_t x) { return x <= 1 ? 0 : 64 - __builtin_clzll(x - 1); }

// log2 of the chunk length in lane steps, or -1 for a single launch.
int split_log2(const vmt_shape& sh, int variant, uint32_t M, uint64_t n, size_t eb, int out_kind) {
    if (sh.split_log2 == kNeverSplit) return -1;
    const uint64_t epw = vmt::is_sfmt(variant) ? 4 : 1;  // stream elements per word
    if (!vmt::is_sfmt(variant) && !vmt::batch_supported(variant, M, out_kind)) return -1;
    const uint64_t steps = ceil_div(n, M * epw);
    int v;
    if (sh.split_log2) {
        v = (int)sh.split_log2;
    } else {
        // Automatic. The jumps of a split call take 0.17 / 0.25 / 0.40 ms for up to 256 / 512 / 1024 MT lane
        // jumps (each lane jump sliced over a workgroup), and one launch writes a few tens of GB/s, so MT calls
        // split from 8 MiB, into at most 256 lane jumps up to 32 MiB, 512 up to 256 MiB and 1024 beyond, with
        // chunks of at least 256 KiB. SFMT19937 splits from M MiB into chunks of 2^14 lane steps (its serial
        // chains run at about 0.25 GB/s per lane, so many chunks pay off; beyond 1024 lane jumps the chunks
        // share each lane's raw rows).
        if (vmt::is_sfmt(variant)) {
            if (n * eb < (uint64_t)M << 20) return -1;
            v = 14;
        } else {
            const uint64_t bytes = n * eb;
            if (bytes < (8ull << 20)) return -1;
            const uint64_t lanes = bytes <= (32ull << 20) ? 256 : bytes <= (256ull << 20) ? 512 : 1024;
            const uint64_t cmax = std::max<uint64_t>(lanes / M, 2);
            v = std::max(ceil_log2(ceil_div(steps, cmax)), ceil_log2(ceil_div(256u << 10, M * epw * eb)));
        }
        while (ceil_div(steps, 1ull << v) > 4096) v++;
    }
    while (ceil_div(steps, 1ull << v) > kMaxChunks) v++;
    if (steps <= (1ull << v)) return -1;
    return v;
}

// Table of t^(c 2^v) mod mu for c = 1..need on the device (caller holds ctx->mu).
int split_table(vmt_ctx* ctx, int variant, int v, size_t need, SplitTable** out) {
    SplitTable& T = ctx->split[variant][(uint32_t)v];
    if (T.host.size() < need) {
        vmt::PolyMod& R = ring(ctx, variant);
        const Words g1 = pow2(ctx, variant, (uint64_t)v);
        while (T.host.size() < need) {
            Words g = T.host.empty() ? g1 : R.mul(T.host.back(), g1);
            const int d = vmt::poly_degree(g);
            if (d >= vmt::kPolyWords * 64) return fail(VMT_EINVAL, "polynomial too large");
            T.deg.push_back(d < 0 ? 0u : (uint32_t)d);
            T.host.push_back(std::move(g));
        }
    }
    if (T.cap < need) {
        const size_t cap = std::max<size_t>({need, 2 * T.cap, 16});
        uint64_t* d = nullptr;
        uint32_t* dd = nullptr;
        hipError_t e = hipMalloc((void**)&d, cap * vmt::kPolyWords * 8);
        if (e != hipSuccess) return fail(VMT_ENOMEM, "hipMalloc(split table): %s", hipGetErrorString(e));
        e = hipMalloc((void**)&dd, cap * sizeof(uint32_t));
        if (e != hipSuccess) {
            (void)hipFree(d);
            return fail(VMT_ENOMEM, "hipMalloc(split degrees): %s", hipGetErrorString(e));
        }
        if (T.d) ctx->retired.push_back(T.d);
        if (T.d_deg) ctx->retired.push_back(T.d_deg);
        T.d = d;
        T.d_deg = dd;
        T.cap = cap;
        T.uploaded = 0;
    }
    if (T.uploaded < need) {
        std::vector<uint64_t> buf((need - T.uploaded) * vmt::kPolyWords, 0);
        for (size_t c = T.uploaded; c < need; c++)
            std::copy(T.host[c].begin(), T.host[c].begin() + std::min<size_t>(T.host[c].size(), vmt::kPolyWords),
                      buf.begin() + (c - T.uploaded) * vmt::kPolyWords);
        hipError_t e = hipMemcpy(T.d + T.uploaded * vmt::kPolyWords, buf.data(), buf.size() * 8, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(T.d_deg + T.uploaded, T.deg.data() + T.uploaded, (need - T.uploaded) * sizeof(uint32_t),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy(split table)");
        T.uploaded = need;
    }
    *out = &T;
    return VMT_OK;
}

// Device scratch of `bytes` for one call on `stream`: the context's workspace
// for the stream (grown stream-ordered when too small, the old one freed
// behind the work queued on the stream), with the stream's lock taken into
// `lock` (hold it until the call's launches are enqueued), or, under stream
// capture, a stream-ordered allocation of the call's own (*own = true; the
// caller frees it stream-ordered), so that a graph owns its memory. Calls on
// one stream use the workspace in stream order; each must write every byte of
// it that it reads.
hipError_t stream_workspace(vmt_ctx* ctx, hipStream_t stream, size_t bytes, uint8_t** buf, bool* own,
                            std::unique_lock<std::mutex>* lock) {
    hipStreamCaptureStatus capturing = hipStreamCaptureStatusNone;
    hipError_t e = hipStreamIsCapturing(stream, &capturing);
    if (e != hipSuccess) return e;
    *own = capturing != hipStreamCaptureStatusNone;
    if (*own) return hipMallocAsync((void**)buf, bytes, stream);
    StreamWorkspace* ws = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto& slot = ctx->split_ws[stream];
        if (!slot) slot = std::make_unique<StreamWorkspace>();
        ws = slot.get();
    }
    *lock = std::unique_lock<std::mutex>(ws->mu);
    if (ws->cap < bytes) {
        const size_t cap = std::max(bytes, 2 * ws->cap);
        uint8_t* p = nullptr;
        e = hipMallocAsync((void**)&p, cap, stream);
        if (e != hipSuccess) return e;
        if (ws->buf) (void)hipFreeAsync(ws->buf, stream);
        ws->buf = p;
        ws->cap = cap;
    }
    *buf = ws->buf;
    return hipSuccess;
}

int generate_split(vmt_ctx* ctx, const StateInfo& info, uint8_t* d_state, uint64_t n, uint8_t* d_out, int out_kind,
                   int v, uint32_t lpw, hipStream_t stream) {
    const uint32_t M = info.M;
    const uint64_t epw = vmt::is_sfmt(info.variant) ? 4 : 1;
    const uint64_t E = (1ull << v) * M * epw;  // elements per chunk
    const uint64_t C = ceil_div(n, E);
    const size_t eb = out_elem_bytes(out_kind);
    const uint64_t* polys = nullptr;
    const uint32_t* d_deg = nullptr;
    uint32_t deg0 = 0;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        SplitTable* T = nullptr;
        int st = split_table(ctx, info.variant, v, C - 1, &T);
        if (st) return st;
        polys = T->d;
        d_deg = T->d_deg;
        deg0 = C > 1 ? T->deg[0] : 0u;
    }
    const size_t sb = vmt_state_bytes(info.variant, M);
    const size_t sbs = (sb + 255) / 256 * 256;
    const size_t off_bt = (C - 1) * sbs;
    const size_t off_jt = off_bt + (C * sizeof(vmt::BatchTask) + 255) / 256 * 256;
    const size_t off_ctr = off_jt + ((C - 1) * sizeof(vmt::JumpTask) + 255) / 256 * 256;
    const size_t off_done = off_ctr + 256;  // one counter per chunk for the lane-group generation
    const size_t off_parts = off_done + (C * sizeof(uint32_t) + 255) / 256 * 256;
    const size_t parts_bytes = vmt::split_jump_parts_bytes(info.variant, M, C - 1);
    const size_t total = off_parts + parts_bytes;
    uint8_t* buf = nullptr;
    bool own = false;
    std::unique_lock<std::mutex> ws_lock;
    hipError_t e = stream_workspace(ctx, stream, total, &buf, &own, &ws_lock);
    if (e != hipSuccess)
        return e == hipErrorOutOfMemory ? fail(VMT_ENOMEM, "split workspace: %s", hipGetErrorString(e))
                                        : hip_fail(e, "split workspace");
    auto* d_bt = reinterpret_cast<vmt::BatchTask*>(buf + off_bt);
    auto* d_jt = reinterpret_cast<vmt::JumpTask*>(buf + off_jt);
    auto* d_ctr = reinterpret_cast<uint32_t*>(buf + off_ctr);
    auto* d_done = reinterpret_cast<uint32_t*>(buf + off_done);
    // copies for chunks 0 .. C-2, the state itself for the last; the task lists are written on the device
    e = vmt::launch_split_setup(d_state, buf, (uint32_t)sb, sbs, (uint32_t)C, d_out, E, n, (uint32_t)eb, polys, d_deg,
                                d_bt, d_jt, d_done, stream);
    // copy 0 is chunk 0: it is not jumped and holds the window every other chunk starts from
    const vmt::JumpTask jt0{C > 2 ? buf + sbs : d_state, polys, 0u, deg0, nullptr};  // the first jump task, as written
    if (e == hipSuccess)
        e = vmt::launch_split_jump(info.variant, M, buf, d_jt, jt0, (uint32_t)(C - 1), stream,
                                   parts_bytes ? buf + off_parts : nullptr);
    if (e == hipSuccess) {
        if (vmt::is_sfmt(info.variant)) {
            e = vmt::launch_batch_sfmt(info.variant, M, M < 16 ? M : 16, out_kind, d_bt, (uint32_t)C, stream);
        } else if (lpw < M) {  // each chunk's lanes spread over M / lpw workgroups
            e = vmt::launch_batch_gen_mt(info.variant, M, lpw, out_kind, d_bt, (uint32_t)C, stream, d_done);
        } else {
            vmt::BatchShape shape;
            vmt::ctx_batch_shape(ctx, info.variant, M, out_kind, &shape);
            e = vmt::reset_counters(d_ctr, stream);
            if (e == hipSuccess)
                e = vmt::launch_batch(info.variant, M, out_kind, shape, d_bt, (uint32_t)C, d_ctr, stream);
        }
    }
    if (own) (void)hipFreeAsync(buf, stream);
    if (e != hipSuccess) return hip_fail(e, "split generate");
    return VMT_OK;
}

int generate(vmt_ctx* ctx, void* d_state, size_t n, void* d_out, int out_kind, hipStream_t stream) {
    int st = set_device(ctx);
    if (st) return st;
    StateInfo info;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        st = lookup(ctx, d_state, &info);
        if (st) return st;
    }
    if (n == 0) return VMT_OK;
    if (!d_out) return fail(VMT_EINVAL, "null output");
    if ((uintptr_t)d_out % out_elem_bytes(out_kind))
        return fail(VMT_EINVAL, "output must be aligned to its element size");
    vmt_shape sh;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        sh = current_shape(ctx, VMT_FAMILY_GENERATE, info.variant, info.M, out_kind);
    }
    const uint32_t lpw = sh.lanes_per_wg ? sh.lanes_per_wg : auto_lpw(info.variant, info.M, n, out_elem_bytes(out_kind));
    if (!vmt::generate_supported(info.variant, info.M, lpw, out_kind))
        return fail(VMT_EVARIANT, "output kind %d not defined for variant %d", out_kind, info.variant);
    const int v = split_log2(sh, info.variant, info.M, n, out_elem_bytes(out_kind), out_kind);
    if (v >= 0)  // a split call runs its MT chunks by lane groups only with a tuned lanes-per-workgroup below M
        return generate_split(ctx, info, static_cast<uint8_t*>(d_state), n, static_cast<uint8_t*>(d_out), out_kind, v,
                              sh.lanes_per_wg ? sh.lanes_per_wg : info.M, stream);
    hipError_t e = vmt::launch_generate(info.variant, info.M, lpw, out_kind, static_cast<uint8_t*>(d_state), d_out,
                                        n, stream);
    if (e != hipSuccess) return hip_fail(e, "generate launch");
    return VMT_OK;
}

int init_common(vmt_ctx* ctx, int variant, uint32_t M, void* d_state, const vmt::InitTask& task, hipStream_t stream) {
    LaneTable* lt = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        int st = lane_table(ctx, variant, M, &lt);
        if (st) return st;
    }
    hipError_t e = vmt::launch_init(variant, M, nullptr, task, 1, lt->d, lt->max_deg, stream);
    if (e != hipSuccess) return hip_fail(e, "init launch");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->reg[d_state] = StateInfo{variant, M};
    return VMT_OK;
}

// A jump launch with, where it applies, the scratch for lane sums split over
// several workgroups (stream-ordered, freed behind the launches).
// A jump launch with, where it applies, scratch for lane sums split over
// several workgroups (the stream's workspace).
hipError_t jump_launch(vmt_ctx* ctx, uint32_t variant, uint32_t M, const vmt::JumpTask* d_tasks,
                       const vmt::JumpTask& one, uint32_t count, hipStream_t stream) {
    const size_t pb = vmt::jump_parts_bytes(variant, M, count);
    uint8_t* d_parts = nullptr;
    bool own = false;
    std::unique_lock<std::mutex> ws_lock;
    if (pb) {
        hipError_t e = stream_workspace(ctx, stream, pb, &d_parts, &own, &ws_lock);
        if (e != hipSuccess) return e;
    }
    hipError_t e = vmt::launch_jump(variant, M, d_tasks, one, count, stream, d_parts);
    if (own) (void)hipFreeAsync(d_parts, stream);
    return e;
}

int jump_with(vmt_ctx* ctx, void* d_state, const std::vector<uint64_t>& dist, const Words* known, hipStream_t stream) {
    int st = set_device(ctx);
    if (st) return st;
    StateInfo info;
    DevPoly* dp = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        st = lookup(ctx, d_state, &info);
        if (st) return st;
        st = jump_table(ctx, info.variant, dist, known, &dp);
        if (st) return st;
    }
    vmt::JumpTask task{static_cast<uint8_t*>(d_state), dp->d, 0u, dp->deg, nullptr};
    hipError_t e = jump_launch(ctx, info.variant, info.M, nullptr, task, 1, stream);
    if (e != hipSuccess) return hip_fail(e, "jump launch");
    return VMT_OK;
}

int check_batch(vmt_ctx* ctx, void* const* d_states, size_t count, StateInfo* common) {
    if (!d_states) return fail(VMT_EINVAL, "null state array");
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (size_t i = 0; i < count; i++) {
        StateInfo info;
        int st = lookup(ctx, d_states[i], &info);
        if (st) return st;
        if (i == 0) *common = info;
        else if (info.variant != common->variant || info.M != common->M)
            return fail(VMT_EINVAL, "batch mixes variants or lane counts (state %zu)", i);
    }
    return VMT_OK;
}

// Task list sorted longest first (LPT order for the persistent kernel).
std::vector<vmt::BatchTask> batch_tasks(void* const* d_states, const uint64_t* lens, void* const* d_outs, size_t count) {
    std::vector<uint32_t> order(count);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return lens[a] > lens[b]; });
    std::vector<vmt::BatchTask> tasks;
    tasks.reserve(count);
    for (uint32_t i : order) tasks.push_back(vmt::BatchTask{static_cast<uint8_t*>(d_states[i]), d_outs[i], lens[i], nullptr});
    return tasks;
}

int validate_batch_args(vmt_ctx* ctx, void* const* d_states, const uint64_t* lens, void* const* d_outs, size_t count,
                        int out_kind, StateInfo* info) {
    if (count == 0) return VMT_OK;
    if (!lens || !d_outs) return fail(VMT_EINVAL, "null lens or output array");
    if (count > 0xFFFFFFFFull) return fail(VMT_EINVAL, "too many tasks");
    int st = check_batch(ctx, d_states, count, info);
    if (st) return st;
    const bool ok = vmt::is_sfmt(info->variant)
                        ? vmt::generate_supported(info->variant, info->M, info->M < 16 ? info->M : 16, out_kind)
                        : vmt::batch_supported(info->variant, info->M, out_kind);
    if (!ok)
        return fail(VMT_EVARIANT, "batched output kind %d not available for variant %d with M=%u", out_kind,
                    info->variant, info->M);
    st = vmt::reject_duplicate_states(d_states, count);
    if (st) return st;
    for (size_t i = 0; i < count; i++) {
        if (lens[i] && !d_outs[i]) return fail(VMT_EINVAL, "null output for task %zu", i);
        if ((uintptr_t)d_outs[i] % out_elem_bytes(out_kind))
            return fail(VMT_EINVAL, "output %zu is not aligned to its element size", i);
    }
    return VMT_OK;
}

// One batched launch: the persistent queue for MT19937; for SFMT19937 one
// workgroup per task and lane group (its serial chains leave no room for a
// queue to balance), in slices of at most 65535 tasks (a grid dimension).
hipError_t launch_tasks(int variant, uint32_t M, int out_kind, const vmt::BatchShape& shape,
                        const vmt::BatchTask* d_tasks, uint32_t count, uint32_t* d_counter, hipStream_t stream) {
    if (!vmt::is_sfmt(variant)) return vmt::launch_batch(variant, M, out_kind, shape, d_tasks, count, d_counter, stream);
    for (uint32_t i = 0; i < count; i += 65535) {
        hipError_t e = vmt::launch_batch_sfmt(variant, M, M < 16 ? M : 16, out_kind, d_tasks + i, std::min(65535u, count - i),
                                              stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

namespace vmt {

int set_error(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ctx_state_info(vmt_ctx* ctx, const void* d_state, int* variant, uint32_t* M) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    StateInfo info;
    int st = lookup(ctx, d_state, &info);
    if (st) return st;
    *variant = info.variant;
    *M = info.M;
    return VMT_OK;
}

int ctx_pow2_poly(vmt_ctx* ctx, int variant, uint32_t k, const uint64_t** d_poly, uint32_t* degree) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    DevPoly* dp = nullptr;
    int st = pow2_dev(ctx, variant, k, &dp);
    if (st) return st;
    *d_poly = dp->d;
    *degree = dp->deg;
    return VMT_OK;
}

int ctx_device(vmt_ctx* ctx) { return ctx->device; }

int reject_duplicate_states(void* const* d_states, size_t count) {
    if (count < 2) return VMT_OK;
    std::vector<const void*> seen(d_states, d_states + count);
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
        return set_error(VMT_EINVAL, "a state appears twice in one call");
    return VMT_OK;
}

int ctx_split_polys(vmt_ctx* ctx, int variant, int v, size_t need, const uint64_t** d_table,
                    std::vector<uint32_t>* degrees) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    SplitTable* T = nullptr;
    int st = split_table(ctx, variant, v, need, &T);
    if (st) return st;
    *d_table = T->d;
    degrees->assign(T->deg.begin(), T->deg.begin() + need);
    return VMT_OK;
}

void ctx_batch_shape(vmt_ctx* ctx, int variant, uint32_t M, int out_kind, BatchShape* out) {
    vmt_shape sh;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        sh = current_shape(ctx, VMT_FAMILY_BATCH, variant, M, out_kind);
    }
    out->tv = sh.threads_variant;
    out->sw = sh.store_bytes;
    const uint32_t fit = batch_max_per_cu(variant, M, out_kind, out->tv, out->sw);
    const uint32_t per_cu = sh.wg_per_cu && sh.wg_per_cu < fit ? sh.wg_per_cu : fit;
    out->grid = per_cu * device_cus(ctx->device);
}

}  // namespace vmt

extern "C" {

const char* vmt_last_error(void) { return g_err.c_str(); }

const char* vmt_version(void) { return "vmt-mi355x 0.1 (gfx950)"; }

vmt_ctx* vmt_ctx_create(int device, int* status) {
    std::unique_ptr<vmt_ctx> ctx(new (std::nothrow) vmt_ctx);
    if (!ctx) {
        if (status) *status = fail(VMT_ENOMEM, "out of host memory");
        return nullptr;
    }
    ctx->device = device;
    if (device >= 0) {
        int n = 0;
        hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess || device >= n) {
            if (status) *status = fail(VMT_EDEVICE, "no HIP device %d (%s)", device, hipGetErrorString(e));
            return nullptr;
        }
        e = hipSetDevice(device);
        if (e != hipSuccess) {
            if (status) *status = hip_fail(e, "hipSetDevice");
            return nullptr;
        }
        // the device address of the allocation-free call's scratch array, looked up once per device
        e = vmt::noalloc_scratch_init(device);
        if (e != hipSuccess) {
            if (status) *status = hip_fail(e, "scratch array address");
            return nullptr;
        }
    }
    if (status) *status = VMT_OK;
    return ctx.release();
}

int vmt_ctx_destroy(vmt_ctx* ctx) {
    if (!ctx) return fail(VMT_EINVAL, "null context");
    if (ctx->device >= 0) {
        (void)hipSetDevice(ctx->device);
        (void)hipDeviceSynchronize();
        for (int v = 0; v < (int)vmt::kVariants; v++) {
            for (auto& kv : ctx->lanes[v]) (void)hipFree(kv.second.d);
            for (auto& kv : ctx->jumps[v]) (void)hipFree(kv.second.d);
            for (auto& kv : ctx->pow2_dev[v]) (void)hipFree(kv.second.d);
            for (auto& kv : ctx->split[v]) {
                (void)hipFree(kv.second.d);
                (void)hipFree(kv.second.d_deg);
            }
            for (auto& kv : ctx->check[v]) (void)hipFree(kv.second.d);
        }
        for (void* p : ctx->retired) (void)hipFree(p);
        // stream-ordered allocations: freed on the null stream (their own streams may be gone), then waited for
        for (auto& kv : ctx->split_ws) (void)hipFreeAsync(kv.second->buf, nullptr);
        (void)hipDeviceSynchronize();
    }
    delete ctx;
    return VMT_OK;
}

size_t vmt_state_bytes(int variant, uint32_t M) {
    if (!valid_variant(variant) || !valid_M(M)) return 0;
    return vmt::kHeaderBytes + (size_t)vmt::words_per_lane(variant) * M * vmt::word_bytes(variant);
}

int vmt_init_genrand(vmt_ctx* ctx, int variant, uint64_t seed, uint32_t M, void* d_state, hipStream_t stream) {
    int st = set_device(ctx);
    if (st) return st;
    if (!valid_variant(variant)) return fail(VMT_EINVAL, "unknown variant %d", variant);
    if (!valid_M(M)) return fail(VMT_EINVAL, "M must be a power of two in [1, 64], got %u", M);
    if (!d_state || (uintptr_t)d_state % 256) return fail(VMT_EINVAL, "state must be non-null and 256-byte aligned");
    vmt::InitTask task{static_cast<uint8_t*>(d_state), nullptr, seed, vmt::kSeedGenrand, 0};
    return init_common(ctx, variant, M, d_state, task, stream);
}

int vmt_init_by_array(vmt_ctx* ctx, int variant, const uint32_t* key, size_t key_len, uint32_t M, void* d_state,
                      hipStream_t stream) {
    int st = set_device(ctx);
    if (st) return st;
    if (variant != VMT_MT32) return fail(VMT_EVARIANT, "init_by_array is defined for MT19937-32 only");
    if (!valid_M(M)) return fail(VMT_EINVAL, "M must be a power of two in [1, 64], got %u", M);
    if (!key || key_len == 0 || key_len > 4096) return fail(VMT_EINVAL, "key must have 1..4096 words");
    if (!d_state || (uintptr_t)d_state % 256) return fail(VMT_EINVAL, "state must be non-null and 256-byte aligned");
    void* d_key = nullptr;
    hipError_t e = hipMallocAsync(&d_key, key_len * 4, stream);
    if (e != hipSuccess) return fail(VMT_ENOMEM, "hipMallocAsync(key): %s", hipGetErrorString(e));
    e = hipMemcpyAsync(d_key, key, key_len * 4, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
        (void)hipFreeAsync(d_key, stream);
        return hip_fail(e, "hipMemcpyAsync(key)");
    }
    vmt::InitTask task{static_cast<uint8_t*>(d_state), static_cast<const uint32_t*>(d_key), 0, vmt::kSeedByArray,
                       (uint32_t)key_len};
    st = init_common(ctx, variant, M, d_state, task, stream);
    (void)hipFreeAsync(d_key, stream);
    return st;
}

int vmt_init_genrand_batch(vmt_ctx* ctx, int variant, const uint64_t* seeds, size_t count, uint32_t M,
                           void* const* d_states, hipStream_t stream) {
    if (!valid_variant(variant)) return fail(VMT_EINVAL, "unknown variant %d", variant);
    if (!valid_M(M)) return fail(VMT_EINVAL, "M must be a power of two in [1, 64], got %u", M);
    if (count == 0) return set_device(ctx);
    if (!seeds || !d_states) return fail(VMT_EINVAL, "null seeds or states");
    if (count > (1u << 24)) return fail(VMT_EINVAL, "too many states");
    for (size_t i = 0; i < count; i++)
        if (!d_states[i] || (uintptr_t)d_states[i] % 256) return fail(VMT_EINVAL, "state %zu null or misaligned", i);
    int st = vmt::reject_duplicate_states(d_states, count);  // two seedings of one window would race
    if (st) return st;
    st = set_device(ctx);
    if (st) return st;
    LaneTable* lt = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        st = lane_table(ctx, variant, M, &lt);
        if (st) return st;
    }
    std::vector<vmt::InitTask> tasks(count);
    for (size_t i = 0; i < count; i++)
        tasks[i] = vmt::InitTask{static_cast<uint8_t*>(d_states[i]), nullptr, seeds[i], vmt::kSeedGenrand, 0};
    const size_t task_bytes = count * sizeof(vmt::InitTask);
    vmt::InitTask* d_tasks = nullptr;
    hipError_t e = hipMallocAsync((void**)&d_tasks, task_bytes, stream);
    if (e != hipSuccess) return fail(VMT_ENOMEM, "hipMallocAsync(init batch): %s", hipGetErrorString(e));
    e = hipMemcpyAsync(d_tasks, tasks.data(), task_bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = vmt::launch_init(variant, M, d_tasks, tasks[0], (uint32_t)count, lt->d, lt->max_deg, stream);
    (void)hipFreeAsync(d_tasks, stream);
    if (e != hipSuccess) return hip_fail(e, "init batch");
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (size_t i = 0; i < count; i++) ctx->reg[d_states[i]] = StateInfo{variant, M};
    return VMT_OK;
}

int vmt_init_by_array_batch(vmt_ctx* ctx, const uint32_t* keys, size_t key_len, size_t count, uint32_t M,
                            void* const* d_states, hipStream_t stream) {
    if (!valid_M(M)) return fail(VMT_EINVAL, "M must be a power of two in [1, 64], got %u", M);
    if (count == 0) return set_device(ctx);
    if (!keys || !d_states || key_len == 0 || key_len > 4096) return fail(VMT_EINVAL, "bad keys");
    if (count > (1u << 24)) return fail(VMT_EINVAL, "too many states");
    for (size_t i = 0; i < count; i++)
        if (!d_states[i] || (uintptr_t)d_states[i] % 256) return fail(VMT_EINVAL, "state %zu null or misaligned", i);
    int st = vmt::reject_duplicate_states(d_states, count);  // two seedings of one window would race
    if (st) return st;
    st = set_device(ctx);
    if (st) return st;
    LaneTable* lt = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        st = lane_table(ctx, VMT_MT32, M, &lt);
        if (st) return st;
    }
    const size_t key_bytes = count * key_len * 4, task_bytes = count * sizeof(vmt::InitTask);
    uint8_t* d_buf = nullptr;
    hipError_t e = hipMallocAsync((void**)&d_buf, key_bytes + task_bytes + 16, stream);
    if (e != hipSuccess) return fail(VMT_ENOMEM, "hipMallocAsync(init batch): %s", hipGetErrorString(e));
    const uint32_t* d_keys = reinterpret_cast<const uint32_t*>(d_buf);
    vmt::InitTask* d_tasks = reinterpret_cast<vmt::InitTask*>(d_buf + ((key_bytes + 15) / 16) * 16);
    std::vector<vmt::InitTask> tasks(count);
    for (size_t i = 0; i < count; i++)
        tasks[i] = vmt::InitTask{static_cast<uint8_t*>(d_states[i]), d_keys + i * key_len, 0, vmt::kSeedByArray,
                                 (uint32_t)key_len};
    e = hipMemcpyAsync(d_buf, keys, key_bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(d_tasks, tasks.data(), task_bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
        e = vmt::launch_init(VMT_MT32, M, d_tasks, tasks[0], (uint32_t)count, lt->d, lt->max_deg, stream);
    (void)hipFreeAsync(d_buf, stream);
    if (e != hipSuccess) return hip_fail(e, "init batch");
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (size_t i = 0; i < count; i++) ctx->reg[d_states[i]] = StateInfo{VMT_MT32, M};
    return VMT_OK;
}

int vmt_jump(vmt_ctx* ctx, void* d_state, const uint64_t* dist_le, size_t dist_words, hipStream_t stream) {
    if (!dist_le || dist_words == 0 || dist_words > 320) return fail(VMT_EINVAL, "distance needs 1..320 words");
    std::vector<uint64_t> d(dist_le, dist_le + dist_words);
    while (d.size() > 1 && d.back() == 0) d.pop_back();
    if (d.size() == 1 && d[0] == 0) {
        int st = set_device(ctx);
        if (st) return st;
        StateInfo info;
        std::lock_guard<std::mutex> lk(ctx->mu);
        return lookup(ctx, d_state, &info);  // jump by 0: nothing to do
    }
    return jump_with(ctx, d_state, d, nullptr, stream);
}

int vmt_jump_pow2(vmt_ctx* ctx, void* d_state, uint32_t k, hipStream_t stream) {
    if (k > 65536) return fail(VMT_EINVAL, "k must be <= 65536");
    int st = set_device(ctx);
    if (st) return st;
    StateInfo info;
    DevPoly* dp = nullptr;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        st = lookup(ctx, d_state, &info);
        if (st) return st;
        st = pow2_dev(ctx, info.variant, k, &dp);
        if (st) return st;
    }
    vmt::JumpTask task{static_cast<uint8_t*>(d_state), dp->d, 0u, dp->deg, nullptr};
    hipError_t e = jump_launch(ctx, info.variant, info.M, nullptr, task, 1, stream);
    if (e != hipSuccess) return hip_fail(e, "jump launch");
    return VMT_OK;
}

int vmt_jump_pow2_batch(vmt_ctx* ctx, void* const* d_states, const uint32_t* ks, size_t count, hipStream_t stream) {
    if (count == 0) return set_device(ctx);
    if (!ks || !d_states) return fail(VMT_EINVAL, "null ks or states");
    int st = vmt::reject_duplicate_states(d_states, count);  // two jumps of one window in place would race
    if (st) return st;
    st = set_device(ctx);
    if (st) return st;
    StateInfo info;
    st = check_batch(ctx, d_states, count, &info);
    if (st) return st;
    std::vector<vmt::JumpTask> tasks(count);
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (size_t i = 0; i < count; i++) {
            if (ks[i] > 65536) return fail(VMT_EINVAL, "k must be <= 65536");
            DevPoly* dp = nullptr;
            st = pow2_dev(ctx, info.variant, ks[i], &dp);
            if (st) return st;
            tasks[i] = vmt::JumpTask{static_cast<uint8_t*>(d_states[i]), dp->d, 0u, dp->deg, nullptr};
        }
    }
    vmt::JumpTask* d_tasks = nullptr;
    hipError_t e = hipMallocAsync((void**)&d_tasks, count * sizeof(vmt::JumpTask), stream);
    if (e != hipSuccess) return fail(VMT_ENOMEM, "hipMallocAsync(jump tasks): %s", hipGetErrorString(e));
    e = hipMemcpyAsync(d_tasks, tasks.data(), count * sizeof(vmt::JumpTask), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = jump_launch(ctx, info.variant, info.M, d_tasks, tasks[0], (uint32_t)count, stream);
    (void)hipFreeAsync(d_tasks, stream);
    if (e != hipSuccess) return hip_fail(e, "jump batch");
    return VMT_OK;
}

int vmt_generate_u32(vmt_ctx* ctx, void* d_state, size_t n, uint32_t* d_out, hipStream_t stream) {
    return generate(ctx, d_state, n, d_out, vmt::kOutU32, stream);
}
int vmt_generate_u64(vmt_ctx* ctx, void* d_state, size_t n, uint64_t* d_out, hipStream_t stream) {
    return generate(ctx, d_state, n, d_out, vmt::kOutU64, stream);
}
int vmt_uniform_f32(vmt_ctx* ctx, void* d_state, size_t n, float* d_out, hipStream_t stream) {
    return generate(ctx, d_state, n, d_out, vmt::kOutF32, stream);
}
int vmt_uniform_f64(vmt_ctx* ctx, void* d_state, size_t n, double* d_out, hipStream_t stream) {
    return generate(ctx, d_state, n, d_out, vmt::kOutF64, stream);
}

int vmt_batch_generate(vmt_ctx* ctx, void* const* d_states, const uint64_t* lens, void* const* d_outs, size_t count,
                       int out_kind, hipStream_t stream) {
    int st = set_device(ctx);
    if (st) return st;
    StateInfo info{};
    st = validate_batch_args(ctx, d_states, lens, d_outs, count, out_kind, &info);
    if (st || count == 0) return st;
    std::vector<vmt::BatchTask> tasks = batch_tasks(d_states, lens, d_outs, count);
    const size_t bytes = count * sizeof(vmt::BatchTask);
    uint8_t* d_buf = nullptr;
    hipError_t e = hipMallocAsync((void**)&d_buf, bytes + 256, stream);
    if (e != hipSuccess) return fail(VMT_ENOMEM, "hipMallocAsync(batch): %s", hipGetErrorString(e));
    vmt::BatchTask* d_tasks = reinterpret_cast<vmt::BatchTask*>(d_buf);
    uint32_t* d_counter = reinterpret_cast<uint32_t*>(d_buf + ((bytes + 255) / 256) * 256);
    e = hipMemcpyAsync(d_tasks, tasks.data(), bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = vmt::reset_counters(d_counter, stream);
    if (e == hipSuccess) {
        vmt::BatchShape shape;
        if (!vmt::is_sfmt(info.variant)) vmt::ctx_batch_shape(ctx, info.variant, info.M, out_kind, &shape);
        e = launch_tasks(info.variant, info.M, out_kind, shape, d_tasks, (uint32_t)count, d_counter, stream);
    }
    (void)hipFreeAsync(d_buf, stream);
    if (e != hipSuccess) return hip_fail(e, "batch launch");
    return VMT_OK;
}

static_assert(VMT_NOALLOC_MAX_TASKS == vmt::kNoAllocMaxTasks, "header and library agree on the scratch size");

int vmt_batch_generate_noalloc(vmt_ctx* ctx, void* const* d_states, const uint64_t* lens, void* const* d_outs,
                               size_t count, int out_kind, hipStream_t stream) {
    if (!ctx) return fail(VMT_EINVAL, "null context");
    if (count > VMT_NOALLOC_MAX_TASKS)
        return fail(VMT_EINVAL, "%zu states in one allocation-free batch call; at most %u", count,
                    (unsigned)VMT_NOALLOC_MAX_TASKS);
    int st = set_device(ctx);
    if (st) return st;
    StateInfo info{};
    st = validate_batch_args(ctx, d_states, lens, d_outs, count, out_kind, &info);
    if (st || count == 0) return st;
    vmt::BatchTask* d_tasks = nullptr;
    uint32_t* d_counter = nullptr;
    hipError_t e = vmt::noalloc_scratch(ctx->device, &d_tasks, &d_counter);
    if (e != hipSuccess) return hip_fail(e, "scratch array");
    std::vector<vmt::BatchTask> tasks = batch_tasks(d_states, lens, d_outs, count);
    e = hipMemcpyAsync(d_tasks, tasks.data(), count * sizeof(vmt::BatchTask), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = vmt::reset_counters(d_counter, stream);  // a kernel, not a memset
    if (e == hipSuccess) {
        vmt::BatchShape shape;
        if (!vmt::is_sfmt(info.variant)) vmt::ctx_batch_shape(ctx, info.variant, info.M, out_kind, &shape);
        e = launch_tasks(info.variant, info.M, out_kind, shape, d_tasks, (uint32_t)count, d_counter, stream);
    }
    if (e != hipSuccess) return hip_fail(e, "allocation-free batch launch");
    return VMT_OK;
}

vmt_batch_plan* vmt_batch_plan_create(vmt_ctx* ctx, void* const* d_states, const uint64_t* lens, void* const* d_outs,
                                      size_t count, int out_kind, int* status) {
    int st = set_device(ctx);
    StateInfo info{};
    if (!st && count == 0) st = fail(VMT_EINVAL, "empty plan");
    if (!st) st = validate_batch_args(ctx, d_states, lens, d_outs, count, out_kind, &info);
    if (st) {
        if (status) *status = st;
        return nullptr;
    }
    std::vector<vmt::BatchTask> tasks = batch_tasks(d_states, lens, d_outs, count);
    const size_t bytes = count * sizeof(vmt::BatchTask);
    uint8_t* d_buf = nullptr;
    hipError_t e = hipMalloc((void**)&d_buf, bytes + 256);
    if (e != hipSuccess) {
        if (status) *status = fail(VMT_ENOMEM, "hipMalloc(plan): %s", hipGetErrorString(e));
        return nullptr;
    }
    e = hipMemcpy(d_buf, tasks.data(), bytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = vmt::reset_counters(reinterpret_cast<uint32_t*>(d_buf + ((bytes + 255) / 256) * 256), nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(d_buf);
        if (status) *status = hip_fail(e, "hipMemcpy(plan)");
        return nullptr;
    }
    vmt_batch_plan* plan = new vmt_batch_plan;
    plan->ctx = ctx;
    plan->variant = info.variant;
    plan->M = info.M;
    plan->out_kind = out_kind;
    plan->count = (uint32_t)count;
    if (!vmt::is_sfmt(info.variant)) vmt::ctx_batch_shape(ctx, info.variant, info.M, out_kind, &plan->shape);
    plan->d_tasks = reinterpret_cast<vmt::BatchTask*>(d_buf);
    plan->d_counter = reinterpret_cast<uint32_t*>(d_buf + ((bytes + 255) / 256) * 256);
    if (status) *status = VMT_OK;
    return plan;
}

int vmt_batch_plan_launch(vmt_batch_plan* plan, hipStream_t stream) {
    if (!plan) return fail(VMT_EINVAL, "null plan");
    int st = set_device(plan->ctx);
    if (st) return st;
    hipError_t e = launch_tasks(plan->variant, plan->M, plan->out_kind, plan->shape, plan->d_tasks, plan->count,
                                plan->d_counter, stream);
    if (e != hipSuccess) return hip_fail(e, "plan launch");
    return VMT_OK;
}

int vmt_batch_plan_write_pattern(vmt_batch_plan* plan, hipStream_t stream) {
    if (!plan) return fail(VMT_EINVAL, "null plan");
    int st = set_device(plan->ctx);
    if (st) return st;
    if (!vmt::pattern_supported(plan->variant, plan->M, plan->out_kind))
        return fail(VMT_EVARIANT, "write pattern: only V-MT19937-32 M=16 uint32 and V-MT19937-64 M=8 uint64 plans");
    hipError_t e = vmt::launch_write_pattern(plan->variant, plan->M, plan->out_kind, plan->shape, plan->d_tasks,
                                             plan->count, plan->d_counter, stream);
    if (e != hipSuccess) return hip_fail(e, "write pattern launch");
    return VMT_OK;
}

int vmt_calib_fill(vmt_ctx* ctx, void* d_buf, size_t bytes, int mode, hipStream_t stream) {
    int st = set_device(ctx);
    if (st) return st;
    if (!d_buf || bytes % 16 || (uintptr_t)d_buf % 16) return fail(VMT_EINVAL, "fill: buffer and size must be 16-byte aligned");
    if (mode < 0 || mode > 3) return fail(VMT_EINVAL, "fill mode must be 0..3");
    hipError_t e = vmt::launch_fill(d_buf, bytes, mode, vmt::device_cus(ctx->device), stream);
    if (e != hipSuccess) return hip_fail(e, "fill launch");
    return VMT_OK;
}

int vmt_batch_plan_destroy(vmt_batch_plan* plan) {
    if (!plan) return fail(VMT_EINVAL, "null plan");
    (void)hipSetDevice(plan->ctx->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(plan->d_tasks);
    delete plan;
    return VMT_OK;
}

int vmt_state_export(vmt_ctx* ctx, const void* d_state, void* h_buf, size_t bytes, hipStream_t stream) {
    int st = set_device(ctx);
    if (st) return st;
    StateInfo info;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        st = lookup(ctx, d_state, &info);
        if (st) return st;
    }
    if (!h_buf || bytes != vmt_state_bytes(info.variant, info.M))
        return fail(VMT_EINVAL, "buffer must hold exactly vmt_state_bytes = %zu bytes",
                    vmt_state_bytes(info.variant, info.M));
    hipError_t e = hipMemcpyAsync(h_buf, d_state, bytes, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "export");
    return VMT_OK;
}

int vmt_state_import(vmt_ctx* ctx, void* d_state, const void* h_buf, size_t bytes, hipStream_t stream) {
    int st = set_device(ctx);
    if (st) return st;
    if (!d_state || !h_buf || (uintptr_t)d_state % 256) return fail(VMT_EINVAL, "null or misaligned buffer");
    if (bytes < vmt::kHeaderBytes) return fail(VMT_EINVAL, "buffer smaller than a header");
    vmt::StateHeader h;
    std::memcpy(&h, h_buf, sizeof h);
    if (h.magic != vmt::kMagic || h.version != vmt::kVersion) return fail(VMT_ESTATE, "not a vmt state (magic/version)");
    if (!valid_variant((int)h.variant) || !valid_M(h.M)) return fail(VMT_ESTATE, "bad variant or M in header");
    if (h.n != vmt::words_per_lane(h.variant) || h.word_bytes != vmt::word_bytes(h.variant) ||
        h.block != h.n * h.M * vmt::elems_per_word(h.variant) || h.pos > h.block)
        return fail(VMT_ESTATE, "inconsistent header");
    if (bytes != vmt_state_bytes((int)h.variant, h.M)) return fail(VMT_EINVAL, "size does not match header");
    hipError_t e = hipMemcpyAsync(d_state, h_buf, bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "import");
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->reg[d_state] = StateInfo{(int)h.variant, h.M};
    return VMT_OK;
}

int vmt_state_release(vmt_ctx* ctx, const void* d_state) {
    if (!ctx || !d_state) return fail(VMT_EINVAL, "null argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->reg.erase(d_state) == 0) return fail(VMT_ESTATE, "state %p is not registered", d_state);
    return VMT_OK;
}

int vmt_minpoly(vmt_ctx* ctx, int variant, uint64_t* out, size_t cap, int* degree) {
    if (!ctx || !out) return fail(VMT_EINVAL, "null argument");
    if (!valid_variant(variant)) return fail(VMT_EINVAL, "unknown variant %d", variant);
    std::lock_guard<std::mutex> lk(ctx->mu);
    const Words& mu = ring(ctx, variant).modulus();
    if (cap < mu.size()) return fail(VMT_EINVAL, "need %zu words", mu.size());
    std::fill(out, out + cap, 0);
    std::copy(mu.begin(), mu.end(), out);
    if (degree) *degree = vmt::poly_degree(mu);
    return VMT_OK;
}

int vmt_jump_poly(vmt_ctx* ctx, int variant, const uint64_t* dist_le, size_t dist_words, uint64_t* out, size_t cap,
                  int* degree) {
    if (!ctx || !out || !dist_le || dist_words == 0) return fail(VMT_EINVAL, "null argument");
    if (!valid_variant(variant)) return fail(VMT_EINVAL, "unknown variant %d", variant);
    std::lock_guard<std::mutex> lk(ctx->mu);
    vmt::PolyMod& R = ring(ctx, variant);
    Words g;
    // a single set bit: use the cached squaring chain
    int bits = 0, top = -1;
    for (size_t i = 0; i < dist_words; i++) {
        bits += __builtin_popcountll(dist_le[i]);
        if (dist_le[i]) top = int(i * 64 + 63 - __builtin_clzll(dist_le[i]));
    }
    if (bits == 1) g = pow2(ctx, variant, (uint64_t)top);
    else g = R.t_pow(dist_le, dist_words);
    if (cap < g.size()) return fail(VMT_EINVAL, "need %zu words", g.size());
    std::fill(out, out + cap, 0);
    std::copy(g.begin(), g.end(), out);
    if (degree) *degree = vmt::poly_degree(g);
    return VMT_OK;
}

int vmt_check_poly(vmt_ctx* ctx, int variant, uint32_t M, uint64_t* out, size_t cap, int* degree) {
    if (!ctx || !out) return fail(VMT_EINVAL, "null argument");
    if (!valid_variant(variant)) return fail(VMT_EINVAL, "unknown variant %d", variant);
    if (!valid_M(M)) return fail(VMT_EINVAL, "M must be a power of two in [1, 64], got %u", M);
    std::lock_guard<std::mutex> lk(ctx->mu);
    const CheckPoly& c = check_poly(ctx, variant, M);
    if (cap < c.host.size()) return fail(VMT_EINVAL, "need %zu words", c.host.size());
    std::fill(out, out + cap, 0);
    std::copy(c.host.begin(), c.host.end(), out);
    if (degree) *degree = (int)c.deg;
    return VMT_OK;
}

int vmt_check_stream(vmt_ctx* ctx, int variant, uint32_t M, int out_kind, const void* d_out, uint64_t n,
                     uint64_t* d_count, hipStream_t stream) {
    int st = set_device(ctx);
    if (st) return st;
    if (!valid_variant(variant)) return fail(VMT_EINVAL, "unknown variant %d", variant);
    if (!valid_M(M)) return fail(VMT_EINVAL, "M must be a power of two in [1, 64], got %u", M);
    if (!d_out || !d_count) return fail(VMT_EINVAL, "null argument");
    if (out_kind < VMT_OUT_U32 || out_kind > VMT_OUT_F64) return fail(VMT_EINVAL, "unknown output kind %d", out_kind);
    // 32-bit words per element and per recurrence step (one base-generator word)
    const bool wide = out_kind == VMT_OUT_U64 || out_kind == VMT_OUT_F64;
    if (variant != VMT_MT64 && wide)
        return fail(VMT_EVARIANT, "variant %d produces no 64-bit output kind %d", variant, out_kind);
    const uint32_t wpe = wide ? 2 : 1;
    const uint32_t S = vmt::is_sfmt(variant) ? 4 : wpe;
    if ((uintptr_t)d_out % (4 * wpe) || (uintptr_t)d_count % 8)
        return fail(VMT_EINVAL, "misaligned stream or count pointer");
    if (n > (UINT64_MAX >> 2)) return fail(VMT_EINVAL, "stream too long");
    const uint64_t nw = n * wpe;
    vmt::CheckPolyDev dev;
    uint32_t deg = 0;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        CheckPoly& c = check_poly(ctx, variant, M);
        deg = c.deg;
        if (nw <= (uint64_t)deg * S)
            return fail(VMT_EINVAL, "stream of %llu words is too short for a recurrence of degree %u (stride %u)",
                        (unsigned long long)nw, deg, S);
        if (!c.d) {
            // bit pattern (dense form) and set coefficients with per-chunk offsets (sparse form)
            const uint32_t C = vmt::kCheckChunkBits;
            const size_t n_bitw = ((size_t)deg + C) / C * C / 32;
            std::vector<uint32_t> blob(n_bitw, 0), terms, off;
            for (size_t i = 0; i < c.host.size() && 2 * i < n_bitw; i++) {
                blob[2 * i] = (uint32_t)c.host[i];
                if (2 * i + 1 < n_bitw) blob[2 * i + 1] = (uint32_t)(c.host[i] >> 32);
            }
            for (uint32_t ch = 0; ch <= deg / C; ch++) {
                off.push_back((uint32_t)terms.size());
                for (uint32_t i = ch * C; i < (ch + 1) * C && i <= deg; i++)
                    if ((blob[i / 32] >> (i % 32)) & 1u) terms.push_back(i);
            }
            off.push_back((uint32_t)terms.size());
            const size_t at_terms = blob.size(), at_off = at_terms + terms.size();
            blob.insert(blob.end(), terms.begin(), terms.end());
            blob.insert(blob.end(), off.begin(), off.end());
            void* d = nullptr;
            hipError_t e = hipMalloc(&d, blob.size() * 4);
            if (e != hipSuccess) return fail(VMT_ENOMEM, "hipMalloc(check polynomial): %s", hipGetErrorString(e));
            e = hipMemcpy(d, blob.data(), blob.size() * 4, hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                (void)hipFree(d);
                return hip_fail(e, "hipMemcpy(check polynomial)");
            }
            c.d = static_cast<uint32_t*>(d);
            c.dev.deg = deg;
            // Sparse costs one LDS word per coefficient and offset, dense one 40-word window per 32
            // coefficients (8 offsets) plus the XORs: the coefficient list wins below ~4 per 32.
            c.dev.dense = terms.size() * 8 > (size_t)deg;
            c.dev.bits = c.d;
            c.dev.terms = c.d + at_terms;
            c.dev.term_off = c.d + at_off;
        }
        dev = c.dev;
    }
    hipError_t e = vmt::launch_check(out_kind, d_out, nw, S, dev, reinterpret_cast<unsigned long long*>(d_count),
                                     vmt::device_cus(ctx->device), stream);
    if (e != hipSuccess) return hip_fail(e, "check kernel launch");
    return VMT_OK;
}

int vmt_shape_get(vmt_ctx* ctx, int family, int variant, uint32_t M, int out_kind, vmt_shape* shape) {
    if (!ctx || !shape) return fail(VMT_EINVAL, "null argument");
    if (family != VMT_FAMILY_GENERATE && family != VMT_FAMILY_BATCH) return fail(VMT_EINVAL, "unknown family %d", family);
    if (!valid_variant(variant) || !valid_M(M) || out_kind < 0 || out_kind > 3)
        return fail(VMT_EINVAL, "bad variant, M or output kind");
    std::lock_guard<std::mutex> lk(ctx->mu);
    *shape = current_shape(ctx, family, variant, M, out_kind);
    if (family == VMT_FAMILY_BATCH) shape->threads = vmt::batch_threads(variant, M, out_kind, shape->threads_variant,
                                                                         shape->store_bytes);
    return VMT_OK;
}

int vmt_shape_set(vmt_ctx* ctx, int family, int variant, uint32_t M, int out_kind, const vmt_shape* shape) {
    if (!ctx) return fail(VMT_EINVAL, "null context");
    if (family != VMT_FAMILY_GENERATE && family != VMT_FAMILY_BATCH) return fail(VMT_EINVAL, "unknown family %d", family);
    if (!valid_variant(variant) || !valid_M(M) || out_kind < 0 || out_kind > 3)
        return fail(VMT_EINVAL, "bad variant, M or output kind");
    const uint32_t key = shape_key(family, variant, M, out_kind);
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (!shape) {
        ctx->shapes.erase(key);
        return VMT_OK;
    }
    vmt_shape sh = current_shape(ctx, family, variant, M, out_kind);
    if (family == VMT_FAMILY_GENERATE) {
        if (shape->lanes_per_wg && !vmt::generate_supported(variant, M, shape->lanes_per_wg, out_kind))
            return fail(VMT_EINVAL, "lanes per workgroup %u not available for variant %d, M=%u, output kind %d",
                        shape->lanes_per_wg, variant, M, out_kind);
        if (shape->split_log2 && shape->split_log2 != kNeverSplit && (shape->split_log2 < 4 || shape->split_log2 > 40))
            return fail(VMT_EINVAL, "split_log2 must be 0 (automatic), 255 (never) or in [4, 40]");
        sh.lanes_per_wg = shape->lanes_per_wg;
        sh.split_log2 = shape->split_log2;
    } else {
        if (!vmt::batch_shape_supported(variant, M, out_kind, shape->threads_variant, shape->store_bytes))
            return fail(VMT_EINVAL, "batch shape (threads variant %u, %u-byte stores) not available for variant %d, "
                        "M=%u, output kind %d", shape->threads_variant, shape->store_bytes, variant, M, out_kind);
        sh.threads_variant = shape->threads_variant;
        sh.store_bytes = shape->store_bytes;
        sh.wg_per_cu = shape->wg_per_cu;
    }
    sh.gbps = shape->gbps;
    ctx->shapes[key] = sh;
    return VMT_OK;
}

}  // extern "C"
