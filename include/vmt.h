/*
 * vmt.h -- C ABI of libvmt: V-family Mersenne Twister generators on MI355X.
 *
 * Implements the generators of F. Cannizzo, "VMT19937: A SIMD-Friendly Pseudo
 * Random Number Generator based on Mersenne Twister 19937" (arXiv 2309.16682):
 * M copies of a base generator (MT19937-32, MT19937-64 or SFMT19937), copy t
 * started t*J steps into the base sequence by jump-ahead, polled round robin
 * into one stream (Sec. 3, eq. combseq; J = 2^(19937 - log2 M), Table jvalues).
 *
 * Conventions for every call
 *   - Status: every function returning int returns VMT_OK (0) or a negative
 *     VMT_E* code. Nothing aborts and no exception crosses the ABI. The
 *     message for the last failure on the calling thread is vmt_last_error().
 *   - Memory: the caller owns state and output buffers (device memory, e.g.
 *     torch tensors). The context owns only its polynomial tables and the
 *     registry that records the variant and lane count of each state it has
 *     initialised or imported. A state must be initialised (vmt_init_*) or
 *     imported (vmt_state_import) through a context before other calls use it.
 *   - Streams: device work is enqueued on the caller's hipStream_t (NULL =
 *     the null stream) and is stream-ordered; results are valid once the
 *     stream has reached the call. Calls return before the GPU work ends.
 *   - Failure: arguments are checked on the host before anything is
 *     enqueued; a call that returns an argument error (VMT_EINVAL,
 *     VMT_EVARIANT, VMT_ESTATE) has enqueued nothing and left the state
 *     unchanged. After VMT_EDEVICE or VMT_ENOMEM from the HIP runtime part of
 *     the call's work may have been enqueued: the state is then undefined.
 *   - Allocation: batched calls and batched jumps allocate their task lists
 *     stream-ordered (hipMallocAsync on the call's stream). Split generation
 *     and jumps of few MT lanes use a workspace per stream owned by the
 *     context (copies of the state, task lists, partial sums), grown
 *     stream-ordered when a call needs more and kept until vmt_ctx_destroy;
 *     under stream capture they allocate their own, stream-ordered. Plans and
 *     servers allocate once, at creation.
 *     vmt_batch_generate_noalloc allocates nothing (its task list goes into a
 *     fixed device scratch array).
 *   - Concurrency: calls on different states may overlap on different
 *     streams. Calls on one state must be ordered by the caller (one stream).
 *
 * Stream elements. MT19937-32: uint32. MT19937-64: uint64. SFMT19937: the
 * uint32 sub-words of its 128-bit words (sub-word 0 first), the round robin
 * over lanes taken per 128-bit word.
 */
#ifndef VMT_H
#define VMT_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define VMT_OK 0
#define VMT_EINVAL (-1)   /* bad argument: NULL pointer, unsupported M, size  */
#define VMT_EVARIANT (-2) /* operation not defined for this generator variant */
#define VMT_ENOMEM (-3)   /* host or device allocation failed                 */
#define VMT_EDEVICE (-4)  /* HIP runtime error                                 */
#define VMT_EBUSY (-5)    /* resource in use                                   */
#define VMT_ESTATE (-6)   /* state not registered or header inconsistent      */

/* generator variants (Sec. 2.2, 2.3, 2.4) */
#define VMT_MT32 0
#define VMT_MT64 1
#define VMT_SFMT 2
/* SFMT with the generator authors' parameter sets for other Mersenne
 * exponents: the recurrence of eq. (sfmt_step) with other shifts, masks and
 * N = MEXP / 128 + 1 words of 128 bits; the paper's claim that the method
 * carries over to any F2-linear generator (Sec. 3.1, Sec. 5). Everything
 * below that holds for VMT_SFMT holds for these, with 19937 replaced by the
 * exponent (period multiple of 2^MEXP - 1, lane distance J = 2^(MEXP - log2 M)). */
#define VMT_SFMT607 3
#define VMT_SFMT1279 4
#define VMT_SFMT2281 5
#define VMT_SFMT4253 6
#define VMT_SFMT11213 7

/* output kinds for vmt_batch_generate */
#define VMT_OUT_U32 0
#define VMT_OUT_U64 1
#define VMT_OUT_F32 2
#define VMT_OUT_F64 3

typedef struct vmt_ctx vmt_ctx;

/* Thread-local text of the last error on this thread ("" if none).
 * Cite: paper silent; error reporting of this C ABI.
 */
const char* vmt_last_error(void);

/* Library version string.
 * Cite: paper silent; library identification.
 */
const char* vmt_version(void);

/* Create a context on HIP device `device`. On failure returns NULL and, if
 * status is not NULL, stores the error code there. The context computes the
 * minimal polynomials of the three base generators and the lane polynomials
 * it needs lazily, on the host, and keeps them for its lifetime.
 * Cite: paper silent on contexts; it holds the minimal polynomials of Sec. 3.1 (jump polynomial t^d
 * mod mu) and the lane polynomials t^(tJ) of eq. (jumpahead). No cache directory: the host
 * polynomials of a context take about 0.03 s.
 */
vmt_ctx* vmt_ctx_create(int device, int* status);

/* Destroy a context: frees its device tables. Waits for the device.
 * Cite: paper silent; releases what vmt_ctx_create built.
 */
int vmt_ctx_destroy(vmt_ctx* ctx);

/* Bytes of device memory a state of `variant` with M lanes occupies: a
 * 256-byte header plus the lane-interleaved window, n words x M lanes
 * (word k of lane t at index k*M + t). M must be a power of two in [1, 64].
 * Returns 0 for an invalid variant or M.
 * Cite: Sec. 3, eq. (msmt19937) (the interleaved state of M instances) with the n words per
 * instance of Sec. 2.2-2.4 and the circular buffer of Sec. 2.5, eq. (staterec).
 */
size_t vmt_state_bytes(int variant, uint32_t M);

/* Initialise a V-state (Sec. 3, Sec. 3.1). The base state X_0 comes from
 * `seed` by the base generator's published init_genrand rule (the paper
 * leaves seeding open): MT19937-32 and SFMT19937 take the low 32 bits of
 * seed, SFMT then applies its period certification. Lane t becomes X_0
 * advanced by t*J steps, J = 2^(19937 - log2 M). The first element of the
 * stream is the base generator's first output. d_state must hold
 * vmt_state_bytes(variant, M) bytes of device memory, 256-byte aligned.
 * Cite: Sec. 3 eq. (subseq) and Sec. 3.1 eq. (jumpahead) (lane t = X_0 advanced t J steps, J from
 * Table jvalues); seeding itself: paper silent, the generators' published init_genrand.
 */
int vmt_init_genrand(vmt_ctx* ctx, int variant, uint64_t seed, uint32_t M, void* d_state,
                     hipStream_t stream);

/* As vmt_init_genrand, with X_0 from init_by_array(key[0..key_len-1]) of the
 * MT19937 release (host array). MT19937-32 only (VMT_EVARIANT otherwise);
 * 1 <= key_len <= 4096.
 * Cite: as vmt_init_genrand; the key expansion is paper silent (MT19937's published init_by_array).
 */
int vmt_init_by_array(vmt_ctx* ctx, int variant, const uint32_t* key, size_t key_len, uint32_t M,
                      void* d_state, hipStream_t stream);

/* Batched vmt_init_genrand: count states of one variant with M lanes, state
 * i seeded init_genrand(seeds[i]) (host array of count seeds); d_states is a
 * host array of count device pointers (256-byte aligned), each state at most
 * once (VMT_EINVAL otherwise). One launch seeds and de-phases every lane of
 * every state; the result equals count vmt_init_genrand calls.
 * Cite: as vmt_init_genrand; batching many generators: paper silent.
 */
int vmt_init_genrand_batch(vmt_ctx* ctx, int variant, const uint64_t* seeds, size_t count, uint32_t M,
                           void* const* d_states, hipStream_t stream);

/* Batched vmt_init_by_array: count states, state i keyed by
 * keys[i*key_len .. i*key_len + key_len - 1] (host array), all MT19937-32
 * with M lanes; d_states is a host array of count device pointers, each
 * state at most once (VMT_EINVAL otherwise).
 * Cite: as vmt_init_by_array; batching many generators: paper silent.
 */
int vmt_init_by_array_batch(vmt_ctx* ctx, const uint32_t* keys, size_t key_len, size_t count,
                            uint32_t M, void* const* d_states, hipStream_t stream);

/* Jump ahead (Sec. 3.1): every lane advances d base steps, i.e. the stream
 * skips d*M elements (4*d*M uint32 for SFMT19937). d is the little-endian
 * multiword integer dist_le[0..dist_words-1] (host array; dist_words <= 320).
 * The jump polynomial t^d mod (minimal polynomial) is computed on the host
 * and cached per distance; the state is updated on the device.
 * Cite: Sec. 3.1, eq. (jumpahead) and the polynomial jump the paper cites as the alternative to eq.
 * (transmat); on a V-state: every lane advances d steps (eq. (subseq)), so eq. (combseq)'s stream
 * skips d M elements.
 */
int vmt_jump(vmt_ctx* ctx, void* d_state, const uint64_t* dist_le, size_t dist_words,
             hipStream_t stream);

/* vmt_jump with d = 2^k, k <= 65536.
 * Cite: as vmt_jump.
 */
int vmt_jump_pow2(vmt_ctx* ctx, void* d_state, uint32_t k, hipStream_t stream);

/* Batched jump by 2^k: count states (host array of device pointers), state i
 * jumped by 2^ks[i]; all states must share variant and M, each state at most
 * once (VMT_EINVAL otherwise).
 * Cite: as vmt_jump; batching: paper silent.
 */
int vmt_jump_pow2_batch(vmt_ctx* ctx, void* const* d_states, const uint32_t* ks, size_t count,
                        hipStream_t stream);

/* Next n stream elements into d_out (device, aligned to the element size).
 * generate_u32: MT19937-32 and SFMT19937. generate_u64: MT19937-64. n may be
 * 0. A long call may run split over many workgroups (see "Splitting" below):
 * the outputs are the same; the state afterwards is the same point of the
 * stream, possibly on a shifted block grid (as after any jump).
 * Cite: Sec. 2.1 eq. (formula) (a generator yields w-bit words), Sec. 3 eq. (combseq) (the round
 * robin of the M instances), the bulk (vectorial) query mode of Sec. 4.3.
 */
int vmt_generate_u32(vmt_ctx* ctx, void* d_state, size_t n, uint32_t* d_out, hipStream_t stream);
int vmt_generate_u64(vmt_ctx* ctx, void* d_state, size_t n, uint64_t* d_out, hipStream_t stream);

/* Uniform floats in [0, 1) by fixed exact maps of the stream elements, one
 * element per output: f32 = (u32 >> 8) * 2^-24 for MT19937-32 and SFMT19937,
 * (u64 >> 40) * 2^-24 for MT19937-64; f64 = (u64 >> 11) * 2^-53 for
 * MT19937-64 (VMT_EVARIANT for the 32-bit generators).
 * Cite: paper silent (it generates integers only); the maps are the fixed exact integer-to-float
 * conversions of the workloads measured here, applied to the eq. (combseq) stream.
 */
int vmt_uniform_f32(vmt_ctx* ctx, void* d_state, size_t n, float* d_out, hipStream_t stream);
int vmt_uniform_f64(vmt_ctx* ctx, void* d_state, size_t n, double* d_out, hipStream_t stream);

/* Batched generation: state i writes lens[i] elements of kind out_kind into
 * d_outs[i]. d_states, lens and d_outs are host arrays of count entries; all
 * states must share variant and M. MT19937-32/-64 (M <= 16): one persistent
 * kernel processes the states longest first from a device work queue.
 * SFMT19937: one workgroup per state and group of up to 16 lanes. Each state
 * must appear at most once per call.
 * Cite: paper silent (the paper runs one generator at a time); each state is the V-generator of
 * Sec. 3, eq. (combseq).
 */
int vmt_batch_generate(vmt_ctx* ctx, void* const* d_states, const uint64_t* lens, void* const* d_outs,
                       size_t count, int out_kind, hipStream_t stream);

/* Allocation-free form of vmt_batch_generate: same arguments, same results,
 * same kernels, but the task list and the work-queue counters go into a
 * fixed scratch array in device memory (a file-scope array of the library,
 * one per GPU, held until the process ends) instead of memory allocated per
 * call. The call itself allocates no device memory: no hipMalloc, hipFree or
 * stream-ordered allocation. The host task list is copied in with
 * hipMemcpyAsync on `stream`. At most VMT_NOALLOC_MAX_TASKS states per call
 * (VMT_EINVAL beyond, nothing enqueued). The scratch array of a GPU is
 * shared by every call of this function on that GPU and keeps the last
 * call's task list: calls that overlap on one GPU (on different streams, or
 * from different threads without ordering) race and may produce wrong
 * outputs; the caller orders them, e.g. on one stream. The context must have
 * been created for a device (vmt_ctx_create looks the array's device address
 * up then, once per GPU).
 * Cite: for callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not allocate, harnesses that forbid it);
 * the operation is vmt_batch_generate's.
 */
#define VMT_NOALLOC_MAX_TASKS 32768
int vmt_batch_generate_noalloc(vmt_ctx* ctx, void* const* d_states, const uint64_t* lens, void* const* d_outs,
                               size_t count, int out_kind, hipStream_t stream);

/* Plan form of vmt_batch_generate for repeated replay: uploads the task list
 * once and returns a handle whose launch reuses it (the same states, lengths
 * and outputs each time; states advance on every launch). The launch can be
 * captured into a HIP graph by the caller.
 * Cite: as vmt_batch_generate.
 */
typedef struct vmt_batch_plan vmt_batch_plan;
vmt_batch_plan* vmt_batch_plan_create(vmt_ctx* ctx, void* const* d_states, const uint64_t* lens,
                                      void* const* d_outs, size_t count, int out_kind, int* status);
int vmt_batch_plan_launch(vmt_batch_plan* plan, hipStream_t stream);
int vmt_batch_plan_destroy(vmt_batch_plan* plan);

/* Measurement only (paper silent; the write ceiling the generation rate is
 * compared with). vmt_batch_plan_write_pattern enqueues the plan's batch
 * kernel with the twist left out: the same task queue, launch shape, window
 * reads and writes and output stores of the same lengths to the same
 * addresses, so its rate is what the plan's output pattern allows. The
 * outputs receive tempered words of the unchanged windows (not stream
 * values) and the states are left as they were. V-MT19937-32 M=16 uint32 and
 * V-MT19937-64 M=8 uint64 plans (VMT_EVARIANT otherwise). Must not overlap a
 * launch of the same plan (they share its queue counter).
 * vmt_calib_fill writes `bytes` (a multiple of 16, 16-byte aligned buffer)
 * with 16-byte stores. mode bit 0 = 0: one-shot workgroups each storing one
 * 4 KiB piece, in address order (a plain fill, the sequential write
 * ceiling); bit 0 = 1: two persistent workgroups per compute unit, each
 * writing its own contiguous region in order (the pattern of many
 * independent output streams, as batched generation writes). mode bit 1:
 * nontemporal stores. VMT_EINVAL for a mode outside 0..3.
 * Cite: paper silent; a measurement aid.
 */
int vmt_batch_plan_write_pattern(vmt_batch_plan* plan, hipStream_t stream);
int vmt_calib_fill(vmt_ctx* ctx, void* d_buf, size_t bytes, int mode, hipStream_t stream);

/* Copy a state to or from host memory (bytes = vmt_state_bytes). Import
 * validates the header and registers the state with the context. Both
 * synchronise `stream`.
 * Cite: Sec. 3, eq. (msmt19937): the state is the interleaved window of the M instances; the copy
 * format itself: paper silent.
 */
int vmt_state_export(vmt_ctx* ctx, const void* d_state, void* h_buf, size_t bytes, hipStream_t stream);
int vmt_state_import(vmt_ctx* ctx, void* d_state, const void* h_buf, size_t bytes, hipStream_t stream);

/* ---- serving loop ------------------------------------------------------------
 * A server owns S streams and serves requests against a fixed list of
 * registered states (same variant and M) with outputs placed in a caller-owned
 * device arena. Requests are admitted in arrival order while (a) each state has
 * at most one request in flight, so a state's requests run in order, and (b)
 * the outputs in flight fit in min(arena_bytes, budget_bytes). Mode 0
 * (continuous batching): whenever a stream is free, everything admitted so far
 * is launched on it as one persistent generation launch (longest first) and
 * one jump launch; launches on different streams overlap. Mode 1 (plain): each
 * admitted request is its own launch, streams taken round robin. Every task
 * counts into a completion flag in host memory, so outputs and states are
 * released per request. The output of request i lives at d_arena + results[i].out_offset;
 * by default later requests of the same run reuse the space of completed ones.
 * Mode bit 1 (retain) places outputs one after another instead, so all outputs
 * of a run stay in the arena (the budget still bounds the bytes in flight). */
typedef struct {
    double t_arrival; /* seconds from the start of the run */
    uint32_t state;   /* index into the server's state list */
    uint32_t kind;    /* 0: generate `count` elements, 1: jump by 2^k */
    uint64_t count;
    uint32_t k;
    uint32_t reserved;
} vmt_request;

typedef struct {
    double t_admit, t_launch, t_done; /* seconds from the start of the run (host clock) */
    uint64_t out_offset;              /* byte offset of the output in the arena (generate) */
    int32_t status;                   /* VMT_OK, or VMT_EINVAL for a request that cannot be served */
    int32_t launch;                   /* index of the launch that ran it */
} vmt_result;

typedef struct vmt_server vmt_server;

/* d_states: host array of n_states registered device states (each at most
 * once, VMT_EINVAL otherwise); d_arena:
 * 256-byte aligned device memory; out_kind: VMT_OUT_* of the generated
 * elements; 1 <= n_streams <= 16 generation streams (mode 0 adds two jump
 * streams); mode: bit 0 plain launches, bit 1 retain, bit 2 split.
 * chunk_elems > 0 bounds the elements of one generation task. A larger
 * request is served either as tasks of at most chunk_elems elements, one per
 * launch, back to back (the state stays reserved and the output space is held
 * for the whole request), so that no launch is long and newly arrived
 * requests are not queued behind large ones; or, with bit 2 (batching mode
 * only), cut into C chunks of 2^v lane steps (2^v >= chunk_elems / M) that
 * run side by side: chunk c from the state jumped by c * 2^v steps (Sec. 3.1;
 * a jump of d steps skips d * M stream words), chunks 0 .. C-2 on copies in
 * scratch states of the server (2048 of them; a request waits for enough
 * free ones), the last on the state itself. 0 = one task per request.
 * Cite: paper silent (no serving in the paper); requests are generation (Sec. 3, eq. (combseq)) and
 * jumps by 2^k (Sec. 3.1).
 */
vmt_server* vmt_server_create(vmt_ctx* ctx, void* const* d_states, size_t n_states, void* d_arena,
                              size_t arena_bytes, uint64_t budget_bytes, int out_kind, uint32_t n_streams,
                              int mode, uint64_t chunk_elems, int* status);
/* Serve n requests. realtime = 1: request i becomes visible at its
 * t_arrival (host clock from the start of the call); 0: all at once.
 * results (host array of n) receives the timeline of each request; *wall_s
 * the duration of the run. Blocks until every request has completed.
 * Cite: as vmt_server_create.
 */
int vmt_server_run(vmt_server* server, const vmt_request* reqs, size_t n, vmt_result* results, int realtime,
                   double* wall_s);
/* Bound on how long a run may go with work in flight and no request
 * completing (default 30 s; 0 <= seconds < inf, else VMT_EINVAL). When it is
 * reached the run gives up: it drains its streams and returns VMT_EBUSY, and
 * every request that had not completed gets status VMT_EBUSY. Of those, a
 * request with launch >= 0 had tasks launched, which have all run by the time
 * the call returns; one with launch = -1 never started and left its state
 * untouched. A generation request served by one task (no chunking or
 * splitting) with launch >= 0 has therefore written its whole output and
 * advanced its state past it; a chunked or split one may stop part-way.
 * seconds = 0 gives up at the first check with anything in flight, which
 * forces this path from the host. The server stays usable.
 * Cite: paper silent; failure handling of the serving loop.
 */
int vmt_server_set_watchdog(vmt_server* server, double seconds);
int vmt_server_destroy(vmt_server* server);

/* Forget a state: the context's registry is keyed by device address, so a
 * caller that frees a state's memory should release it first (a later
 * allocation at the same address must be initialised or imported again).
 * Cite: paper silent; registry bookkeeping.
 */
int vmt_state_release(vmt_ctx* ctx, const void* d_state);

/* Host helpers (no device work). Minimal polynomial of the one-step map of a
 * base generator and t^d mod it, as little-endian bit arrays (bit i of the
 * uint64 array = coefficient of t^i); cap = words available in out.
 * Cite: Sec. 3.1 (the jump polynomial is t^d modulo the minimal polynomial of the one-step map, eq.
 * (matmult)); computing mu by Berlekamp-Massey: paper silent.
 */
int vmt_minpoly(vmt_ctx* ctx, int variant, uint64_t* out, size_t cap, int* degree);
int vmt_jump_poly(vmt_ctx* ctx, int variant, const uint64_t* dist_le, size_t dist_words, uint64_t* out,
                  size_t cap, int* degree);

/* ---- linear-complexity self-check ----------------------------------------------
 * Every output bit of an F2-linear generator, read along its stream, obeys a
 * fixed linear recurrence; its length is the sequence's linear complexity,
 * which the paper reports as the one statistical test every MT-based
 * generator fails (Sec. 4.1, LinearComp). For the V-stream the recurrence is
 * known in closed form, so a generated buffer can be checked against it on
 * the device at any size:
 *
 *   MT19937-32/-64: A = mu, the minimal polynomial (irreducible, degree
 *     19937). Lane t is lane 0 advanced t J steps with J = 2^(19937 - log2 M);
 *     since alpha^(2^19937) = alpha for every root alpha of mu, the
 *     interleaved bit sequence is again a trace sequence of a root of mu (a
 *     conjugate), so each bit of the V-stream obeys mu itself: the linear
 *     complexity stays 19937 for every M (eq. combseq). Any other lane spacing
 *     gives 19937 M.
 *   SFMT19937: mu = phi psi with phi of degree 19937 (the period part) and psi
 *     of degree 31; the phi part collapses as above, the psi part does not, so
 *     each bit of the sequence of 128-bit words obeys A = phi(t) psi(t^M)
 *     (degree 19937 + 31 M).
 *
 * vmt_check_poly writes A (bit i of out = coefficient of t^i; cap words
 * available) and its degree; host only.
 * Cite: Sec. 4.1 (LinearComp, the test every MT-based generator fails) and eq. (combseq) with J
 * from Table jvalues.
 */
int vmt_check_poly(vmt_ctx* ctx, int variant, uint32_t M, uint64_t* out, size_t cap, int* degree);

/* Count the offsets at which a generated stream breaks its recurrence. The
 * stream (n elements of out_kind, as the generate, uniform or batch calls
 * write them for this variant and M) is read as the sequence w of 32-bit
 * words it carries: uint32 as is, float as its integer f 2^24, uint64 as
 * (low, high) halves, double as the halves of its integer f 2^53. With
 * S = words per recurrence step (MT19937-32: 1 (u32, f32); MT19937-64: 2
 * (u64, f64), 1 (f32); SFMT19937: 4 (u32, f32), one 128-bit word), every
 * offset x with x + deg(A) S < n_words must satisfy
 * XOR_{i : A_i = 1} w[x + i S] = 0. *d_count (one uint64 in device memory,
 * overwritten) receives the number of offsets where it does not: 0 for an
 * intact stream; a single flipped bit gives one failing offset per set
 * coefficient of A within range, a wrong lane spacing almost every offset.
 * The stream may start anywhere in the V-stream. Enqueued on `stream`;
 * VMT_EINVAL if n_words <= deg(A) S (nothing to check), VMT_EVARIANT for an
 * out kind the variant does not produce (u64 or f64 of the 32-bit
 * generators). Allocates nothing after the first call for a (variant, M):
 * the device copy of A stays with the context.
 * Cite: as vmt_check_poly.
 */
int vmt_check_stream(vmt_ctx* ctx, int variant, uint32_t M, int out_kind, const void* d_out, uint64_t n,
                     uint64_t* d_count, hipStream_t stream);

/* ---- launch shapes and the autotuner ------------------------------------------
 * Family VMT_FAMILY_GENERATE is generation from one state (vmt_generate_*,
 * vmt_uniform_*): the state's M lanes are split over M / lanes_per_wg
 * workgroups (lanes_per_wg: a power of two dividing M, at most 16; the LDS
 * window of a workgroup is [n][lanes_per_wg]; 0 = chosen per call from its
 * size). Family VMT_FAMILY_BATCH is the
 * persistent kernel of vmt_batch_generate, batch plans and the serving loop,
 * one whole state per workgroup: threads_variant v gives each thread 2^v
 * times the default share of the twist (0, 1, 2; 1 and 2 only for M = 8 and
 * 16), store_bytes is the width of each output store (16 or 8), wg_per_cu
 * the resident workgroups per compute unit (0: as many as fit). The context
 * keeps one shape per (family, variant, M, out_kind); plans and servers take
 * the shape in force when they are created. Every shape produces the same
 * bits; only the speed differs.
 *
 * Splitting (generate family): a long call is cut into chunks of 2^split_log2
 * lane steps (2^split_log2 * M stream words); chunk c runs from the state
 * jumped by c * 2^split_log2 steps (Sec. 3.1; a jump of d steps skips d * M
 * words of the interleaved stream), chunks 0 .. C-2 on copies, the last on
 * the state itself, all in one batched launch, so the state ends where the
 * call ends (on a block grid shifted by the jump). split_log2 = 0 lets the
 * library decide from the call size, 255 never splits, 4..40 fixes the chunk.
 * MT19937-32/-64 split only for M <= 16; their chunks run one workgroup per
 * chunk when lanes_per_wg is 0 or M, and by lane groups (M / lanes_per_wg
 * workgroups per chunk) when lanes_per_wg is below M; SFMT chunks run
 * min(M, 16) lanes per workgroup. Splitting needs the jump tables of the
 * chunk offsets (computed on the host once per chunk length) and a scratch
 * copy of the state per chunk (in the context's workspace for the stream). */
enum { VMT_FAMILY_GENERATE = 0, VMT_FAMILY_BATCH = 1 };

typedef struct {
    uint32_t lanes_per_wg;    /* generate family */
    uint32_t threads_variant; /* batch family */
    uint32_t store_bytes;     /* batch family */
    uint32_t wg_per_cu;       /* batch family */
    uint32_t threads;         /* output: threads per workgroup of the batch shape */
    uint32_t split_log2;      /* generate family, see below */
    double gbps;              /* output: output GB/s measured by vmt_autotune (0 if not measured) */
} vmt_shape;

/* Shape in force; set stores one (NULL: back to the default). VMT_EINVAL for
 * a shape that is not compiled in.
 * Cite: paper silent; launch shapes of this GPU implementation (the paper's analogue is the SIMD
 * width L of Table jvalues).
 */
int vmt_shape_get(vmt_ctx* ctx, int family, int variant, uint32_t M, int out_kind, vmt_shape* shape);
int vmt_shape_set(vmt_ctx* ctx, int family, int variant, uint32_t M, int out_kind, const vmt_shape* shape);

/* Time every available shape of a family on scratch states and outputs that
 * the call allocates and frees (the caller's states are not touched), store
 * the fastest in the context and return it in *best. Generate family:
 * lens[0] elements per trial (count = 1). Batch family: one task per entry of
 * lens (a sample of the lengths the caller will run). Each shape runs once
 * untimed and `reps` times timed with HIP events on `stream`; the fastest
 * repetition counts. tried (optional, tried_cap entries) receives every shape
 * timed, *n_tried their number. Synchronises `stream`; VMT_ENOMEM if the
 * scratch outputs do not fit.
 * Cite: paper silent; chooses among launch shapes that all give the same bits.
 */
int vmt_autotune(vmt_ctx* ctx, int family, int variant, uint32_t M, int out_kind, const uint64_t* lens,
                 size_t count, int reps, vmt_shape* best, vmt_shape* tried, size_t tried_cap, size_t* n_tried,
                 hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
