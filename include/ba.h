/*
 * ba.h -- C ABI of libba, a gfx950 (MI355X) generator of Barabasi-Albert
 * graphs by per-edge recomputation (Sanders & Schulz, "Scalable Generation of
 * Scale-free Graphs", arXiv:1602.07106).
 *
 * The graph (paper Section 2): an empty seed graph, n nodes, d edges per
 * node, m = n*d edges, self-loops and parallel edges allowed.  The edge array
 * E[0 .. 2m-1] holds edge i at positions 2i (first endpoint) and 2i+1
 * (second endpoint):
 *
 *   E[2i]   = floor(i / d)
 *   E[2i+1] = E[x] with x = h(2i+1) in 0..2i              (Batagelj-Brandes)
 *
 * which the library evaluates per edge, without reading E (paper Section 2,
 * figure generateEdge): r = 2i+1, then r = h(r) at least once and until r is
 * even, and edge i is (floor(i/d), floor(r/(2d))).  The keyed hash is
 *
 *   key  = seed * 0x9E3779B97F4A7C15                      (mod 2^64)
 *   h(r) = umul64hi(fmix64(r XOR key), r)                 (a value in 0..r-1)
 *
 * with fmix64 the SplitMix64 output mix and umul64hi the high 64 bits of the
 * 128-bit product.  The result depends only on (n, d, seed): never on the
 * stream, the launch shape or how a range is split (paper Section 2: the graph
 * depends on the hash function, not on the number of processors).
 *
 * Conventions for every entry point:
 *  - Pointers named as device pointers must be device memory of the current
 *    HIP device, owned by the caller.  The library never allocates or frees
 *    device memory: what a call needs beyond its outputs comes from a
 *    caller-owned workspace (the *_ws calls, batches, the server's arena) or
 *    from the fixed static scratch of ba_generate_static.  Host memory is
 *    allocated only by ba_batch_upload (a staging copy of the table),
 *    ba_server_create (pinned staging) and the server's bookkeeping.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  Calls are
 *    asynchronous: outputs are valid once the stream reaches the call.
 *    Execution errors surface at the caller's next synchronisation.
 *  - Argument checks run on the host before any launch; on error nothing is
 *    launched and no output is touched.
 *  - m = 0 (n = 0 or d = 0) is valid; the call then only writes the outputs
 *    that have a defined value (zero degrees, zero checksum).
 *  - Calls on different streams may run concurrently.  Mutable state: a
 *    thread-local last HIP error code, the thread-local records of the timing
 *    hook, the per-device tuned shape of the batched kernel (written only by
 *    ba_batch_autotune, read by ba_batch_launch, atomic) and the static
 *    scratch of ba_generate_static.
 */
#ifndef BA_H
#define BA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define BA_OK 0
#define BA_EINVAL (-1)  /* null or misaligned buffer, range past m, first_k > n */
#define BA_ERANGE (-2)  /* 2*n*d does not fit 64 bits, or IDs or counts do not fit the output type */
#define BA_ENOMEM (-3)  /* a workspace (or the static scratch) too small for the smallest pass */
#define BA_EDEVICE (-4) /* a HIP call failed; ba_last_hip_error() gives its hipError_t */

/*
 * The whole edge array of the graph (n, d, seed), paper Section 2.
 *   edges : device, uint32[2*n*d], written in full: edges[2i] = E[2i],
 *           edges[2i+1] = E[2i+1].  4-byte aligned (16-byte aligned is faster).
 *   deg   : device, uint32[n] or NULL.  When not NULL it is overwritten with
 *           deg[v] = number of positions p with E[p] = v (a self-loop counts
 *           twice; the degrees sum to 2m).  Computed in the same pass: the
 *           first endpoints in closed form (d per node), the second ones by
 *           global atomics from the generator (no workspace, no allocation;
 *           about an order of magnitude slower than ba_generate_ws, whose
 *           partition-and-histogram pipeline is the fast path).
 * Errors: BA_ERANGE if n > 2^32 or 2*n*d >= 2^64, or deg is given and
 * n*d + d >= 2^32 (a count could exceed uint32: node v holds at most its d
 * first endpoints and the second endpoints of edges d*v .. n*d-1);
 * BA_EINVAL if a needed pointer is NULL or misaligned.
 */
int ba_generate(uint64_t n, uint32_t d, uint64_t seed, uint32_t *edges, uint32_t *deg,
                void *stream);

/*
 * Edges edge_begin .. edge_begin+edge_count-1 of the graph (n, d, seed).
 * Chunks of a graph generated in any order and concatenate to ba_generate's
 * array: the per-edge independence of paper Section 2 (and its load
 * balancing by batches of edge IDs).
 *   edges : device, uint32[2*edge_count]; edges[2j], edges[2j+1] = edge
 *           edge_begin+j.
 *   deg   : device, uint32[n] or NULL.  When not NULL the counts of both
 *           endpoints of every edge in the range are ADDED to it (the caller
 *           initialises it, e.g. to zero), so chunks accumulate to the
 *           degrees of the whole graph.
 * Errors: as ba_generate, plus BA_EINVAL if edge_begin+edge_count > n*d.
 */
int ba_generate_range(uint64_t n, uint32_t d, uint64_t seed, uint64_t edge_begin,
                      uint64_t edge_count, uint32_t *edges, uint32_t *deg, void *stream);

/*
 * Device workspace (bytes) that ba_generate_ws / ba_generate_range_ws need to
 * compute degrees over edge_count edges of (n, d) in one pass; 0 when
 * edge_count is 0 or the graph does not fit.  A smaller workspace (at least
 * what 2^20 edges need) is accepted and processed in several passes.
 * The degree pipeline (a radix partition of second endpoints in HBM followed
 * by LDS histograms) keeps its lists there: about 6.5 bytes per edge.
 */
uint64_t ba_generate_workspace_bytes(uint64_t n, uint32_t d, uint64_t edge_count);

/*
 * ba_generate / ba_generate_range with a caller-provided workspace for the
 * degree computation (ignored when deg is NULL).
 *   workspace : device, 256-byte aligned, workspace_bytes long, owned by the
 *               caller; its contents are scratch (not preserved).  Calls that
 *               share a workspace must be ordered (same stream).
 * Errors: as the calls without workspace, plus BA_EINVAL if deg != NULL and
 * the workspace is NULL or misaligned, and BA_ENOMEM if it is smaller than
 * the smallest pass (2^20 edges) needs.
 */
int ba_generate_ws(uint64_t n, uint32_t d, uint64_t seed, uint32_t *edges, uint32_t *deg,
                   void *workspace, uint64_t workspace_bytes, void *stream);
int ba_generate_range_ws(uint64_t n, uint32_t d, uint64_t seed, uint64_t edge_begin,
                         uint64_t edge_count, uint32_t *edges, uint32_t *deg, void *workspace,
                         uint64_t workspace_bytes, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * ba_generate_ws with the degree pipeline's workspace taken from a fixed
 * static device array of BA_STATIC_SCRATCH_BYTES (256 MiB) instead of the
 * caller.  Nothing is allocated or freed by the call.  Each GPU the library
 * runs on holds its own copy of that array from the moment the library's
 * code is loaded on it until the process ends; the first call on a device
 * looks up the copy's address (a HIP call that allocates nothing).
 *   edges, deg : as ba_generate_ws (deg may be NULL: then no scratch is used).
 * The graph is processed in passes of as many edges as the scratch holds
 * (about 2.26e7 edges a pass at n = 2^26, so the n = 2^26, d = 16 graph
 * takes 48 passes; slower than ba_generate_ws with a whole workspace, same
 * result).  Every call on one GPU shares that GPU's scratch and the scratch
 * keeps whatever the last call left there (each pass initialises what it
 * reads): calls with deg that overlap on one GPU (on different streams,
 * or from different host threads without ordering) race and give wrong
 * degrees; order them on one stream.
 * Errors: as ba_generate_ws, with BA_ENOMEM (checked on the host, before
 * any device call) when deg is given and not even a pass of 2^20 edges fits
 * the scratch, i.e. for n above about 2.29e8.
 */
#define BA_STATIC_SCRATCH_BYTES ((uint64_t)256 << 20)
int ba_generate_static(uint64_t n, uint32_t d, uint64_t seed, uint32_t *edges, uint32_t *deg,
                       void *stream);

/*
 * Test hook (not needed to generate graphs): ba_generate_ws with the
 * partition's region capacities scaled by cap_scale in (0, 1], so that most
 * second endpoints take the overflow path (direct atomics) instead of the
 * regions.  The result is the same for every scale; tests use it to check
 * that path.  Errors: as ba_generate_ws, plus BA_EINVAL for a scale outside
 * (0, 1] or deg NULL.
 */
int ba_test_generate_ws_scaled(uint64_t n, uint32_t d, uint64_t seed, uint32_t *edges, uint32_t *deg,
                               void *workspace, uint64_t workspace_bytes, double cap_scale, void *stream);

/*
 * As ba_generate_range with 64-bit node IDs (any n with 2*n*d < 2^64).
 *   edges : device, uint64[2*edge_count], 8-byte aligned.
 */
int ba_generate_range_u64(uint64_t n, uint32_t d, uint64_t seed, uint64_t edge_begin,
                          uint64_t edge_count, uint64_t *edges, void *stream);

/*
 * Streaming consumer of paper Section 3: degrees of the first first_k nodes
 * of the graph (n, d, seed) without storing any edge, plus an edge checksum.
 *   deg          : device, uint64[first_k], overwritten with the degrees of
 *                  nodes 0..first_k-1 (same convention as ba_generate).
 *   xor_checksum : device, uint64[1] or NULL; overwritten with the XOR over
 *                  all edges i of w_i = (u_i * 2^32 + v_i) * (2i+1) mod 2^64,
 *                  (u_i, v_i) = edge i.
 * Errors: BA_EINVAL if first_k > n or deg is NULL with first_k > 0;
 * BA_ERANGE if 2*n*d >= 2^64.
 */
int ba_degrees(uint64_t n, uint32_t d, uint64_t seed, uint64_t first_k, uint64_t *deg,
               uint64_t *xor_checksum, void *stream);

/*
 * ba_degrees over the edges edge_begin .. edge_begin+edge_count-1 only,
 * ACCUMULATING: endpoint counts are added to deg[0..first_k-1] and the edge
 * words are XORed into *xor_checksum.  Ranges that partition 0..n*d-1 give
 * exactly ba_degrees' result from zeroed outputs.
 */
int ba_degrees_range(uint64_t n, uint32_t d, uint64_t seed, uint64_t edge_begin,
                     uint64_t edge_count, uint64_t first_k, uint64_t *deg,
                     uint64_t *xor_checksum, void *stream);

/*
 * ba_degrees_range with an explicit choice of the LDS counter tier of the
 * streaming kernel (results are identical on every tier; only speed differs):
 *   BA_TIER_AUTO : what ba_degrees and ba_degrees_range use; BA_TIER_64K
 *                  when first_k > 16384 and the targets expected in
 *                  [16384, min(first_k, 65536)), about
 *                  (sqrt(min(first_k, 65536)) - 128) / sqrt(n) of them,
 *                  exceed 1.5% (all positions of the call below 2^32) or
 *                  1.8% (64-bit positions), i.e. for small n; else
 *                  BA_TIER_16K.
 *   BA_TIER_16K  : 32-bit LDS counters for nodes below 16384 (64 KiB per
 *                  block, two blocks per compute unit); every other target
 *                  below first_k is a global atomic.
 *   BA_TIER_64K  : 16-bit LDS counters for nodes below 65536 (128 KiB per
 *                  block, one block per compute unit), moved to the global
 *                  count 32768 at a time as they fill.
 * Errors: as ba_degrees_range, plus BA_EINVAL for another tier value.
 */
enum { BA_TIER_AUTO = 0, BA_TIER_16K = 16, BA_TIER_64K = 64 };
int ba_degrees_range_tier(uint64_t n, uint32_t d, uint64_t seed, uint64_t edge_begin,
                          uint64_t edge_count, uint64_t first_k, uint64_t *deg,
                          uint64_t *xor_checksum, int tier, void *stream);

/*
 * Measurement hook for benchmarks (not needed to generate graphs).
 * ba_kernel_timing(1) makes every later call on this host thread record a
 * HIP event pair on its stream around each kernel it launches, tagged with
 * the kind of kernel; ba_kernel_timing(0) stops and drops what was recorded.
 * ba_kernel_timing_read waits for the recorded events and fills ms[k] (summed
 * kernel milliseconds) and launches[k] for every kind k < BA_KT_COUNT since
 * the last enable/read, then starts a new accumulation.  Both arrays are
 * caller-owned host memory of BA_KT_COUNT elements.  Events add a little
 * host overhead per launch, so leave timing off outside measurements.
 */
enum {
    BA_KT_GEN = 0,     /* per-edge chain kernels (edge array, target list) */
    BA_KT_PART = 1,    /* degree pipeline: radix partition of targets */
    BA_KT_HIST = 2,    /* degree pipeline: LDS histograms into deg */
    BA_KT_STREAM = 3,  /* streaming first-k degrees and checksum */
    BA_KT_OTHER = 4,   /* fills, plan, totals, scans, tail */
    BA_KT_COUNT = 5
};
int ba_kernel_timing(int enable);
int ba_kernel_timing_read(double *ms, uint64_t *launches);

/*
 * Batched generation: many independent graphs in one persistent launch.
 * The paper computes every edge independently and hands batches of edge IDs
 * to processors for load balancing (Section 2, last paragraph); a batch here
 * is a table of instances j = 0..count-1, each a plain BA graph (n[j], d[j],
 * seed[j]) whose edge array (the same uint32 pairs ba_generate writes) goes
 * to edges + out_offset[j] (offsets in uint32 elements).  Instances may be
 * empty (n or d zero).  Results depend only on each instance's parameters,
 * never on the batch, its order or the launch shape.
 *
 * ba_batch_upload checks the table on the host (BA_ERANGE: an instance with
 * n > 2^32 or 2*n*d beyond 2^64, or more than 2^40 tiles in all; BA_EINVAL:
 * null arrays, or a workspace that is null, not 256-byte aligned or smaller
 * than ba_batch_workspace_bytes(count)), writes the device table into the
 * caller's workspace and waits for that copy (the host arrays may be freed on
 * return).  It fills *info (host memory, caller-owned), including
 * info->edges_len, the uint32 elements the output must hold.
 *
 * ba_batch_launch enqueues the whole batch on `stream` as one kernel launch
 * (no copy, no allocation: it can be captured into a HIP graph).  Outputs of
 * different instances must not overlap; edges must be 4-byte aligned and hold
 * edges_len >= info->edges_len elements, else BA_EINVAL.  The workspace must
 * stay untouched while launches that use it run.
 *
 * ba_batch_autotune times every kernel shape (tile edges x waves per block,
 * shapes 0..BA_BATCH_SHAPES-1) on the given batch and keeps the fastest for
 * the current device; later ba_batch_launch calls on that device use it
 * (ba_batch_current_shape reports its index, ba_batch_shape_dims the tile
 * and block of any index).  Without tuning the shape is 0: 1024-edge tiles,
 * 4 waves per block.  The tuner's own launches write the batch's edges too.
 * ba_batch_launch_shape launches with an explicit shape (same output).
 *
 * ba_batch_plan_rounds (host only) splits a table, in order, into rounds
 * whose outputs fit round_elems uint32 elements each, for tables whose
 * whole output exceeds device memory: round_of[j] and offset_of[j] (host
 * arrays of count) give each instance's round and 16-byte-aligned offset in
 * its round's buffer; *rounds the number of rounds.  BA_EINVAL when a single
 * instance needs more than round_elems.
 */
typedef struct {
    uint32_t count;
    uint32_t reserved;
    uint64_t tiles[3];   /* tiles of 1024, 2048 and 4096 edges */
    uint64_t edges_len;  /* uint32 elements the output must hold */
} ba_batch_info;

uint64_t ba_batch_workspace_bytes(uint32_t count);
int ba_batch_upload(uint32_t count, const uint64_t *n, const uint32_t *d, const uint64_t *seed,
                    const uint64_t *out_offset, void *workspace, uint64_t workspace_bytes,
                    ba_batch_info *info, void *stream);
int ba_batch_launch(const ba_batch_info *info, const void *workspace, uint32_t *edges,
                    uint64_t edges_len, void *stream);
int ba_batch_autotune(const ba_batch_info *info, const void *workspace, uint32_t *edges,
                      uint64_t edges_len, int *shape_out, void *stream);
int ba_batch_launch_shape(const ba_batch_info *info, const void *workspace, uint32_t *edges,
                          uint64_t edges_len, int shape, void *stream);
enum { BA_BATCH_SHAPES = 5 };
int ba_batch_current_shape(int *shape);
int ba_batch_shape_dims(int shape, int *tile_edges, int *waves_per_block);
int ba_batch_plan_rounds(uint32_t count, const uint64_t *n, const uint32_t *d, uint64_t round_elems,
                         uint32_t *round_of, uint64_t *offset_of, uint32_t *rounds);

/*
 * Served generation: continuous batching of requests.
 * A request is a plain BA graph (n, d, seed) and asks either for its whole
 * edge array (kind BA_REQ_EDGES: uint32 pairs as ba_generate writes them,
 * 8*n*d bytes) or for the streamed first-k degrees and edge checksum of
 * ba_degrees (kind BA_REQ_DEGREES: first_k uint64 counts then the uint64
 * checksum, 8*(first_k+1) bytes).  Results are bit-identical to the same
 * request run alone.
 *
 * ba_server_create takes a caller-owned device arena (256-byte aligned, at
 * least 4 KiB; results and batch tables live there) and a stream, and
 * records the server's time origin on that stream.  ba_server_submit
 * queues a request on the host (BA_ERANGE / BA_EINVAL for graphs the
 * matching call refuses; BA_ERANGE when the result's byte count would not
 * fit 64 bits) and returns its ticket.  ba_server_pump retires
 * finished steps and, when fewer than max_inflight steps are in flight,
 * launches one more: it admits queued requests in arrival order while their
 * outputs fit the free arena (admission by HBM bytes), runs every admitted
 * edge request as one batched persistent launch on the caller's stream and
 * the degree requests as batched streaming launches on a stream of the
 * server's own (default priority, ordered after the step's table copy), so
 * the two overlap, and records the step's events (*launched = requests
 * admitted).  A step is complete when both streams have passed it; results
 * are valid once their ticket is BA_JOB_READY, not in stream order.  It
 * never blocks on the GPU.  A request that cannot fit even an empty arena
 * is marked BA_JOB_FAILED.  If a launch of the step fails, pump waits for
 * both streams, marks the step's requests BA_JOB_FAILED, frees their arena
 * space and returns the error.
 * ba_server_poll reports a ticket's state and, once BA_JOB_READY, the GPU
 * completion time of its step in ms after the time origin and the byte
 * offset/size of its result in the arena.  ba_server_completed hands out
 * (up to capacity) the tickets that became ready or failed since its last
 * call, oldest first, so a client need not poll every ticket.
 * ba_server_release returns a ready result's arena space (or drops a
 * failed request); a ticket is valid until it is released, and the
 * server's host memory follows the tickets still held.  ba_server_destroy
 * waits for both streams and frees the server (not the arena).  One host thread per server; calls on
 * one server must not overlap.
 */
enum { BA_REQ_EDGES = 0, BA_REQ_DEGREES = 1 };
enum { BA_JOB_QUEUED = 0, BA_JOB_RUNNING = 1, BA_JOB_READY = 2, BA_JOB_FAILED = 3, BA_JOB_RELEASED = 4 };
typedef struct {
    uint64_t n;
    uint64_t seed;
    uint64_t first_k;  /* BA_REQ_DEGREES: nodes 0..first_k-1 (first_k <= n) */
    uint32_t d;
    uint32_t kind;     /* BA_REQ_EDGES or BA_REQ_DEGREES */
} ba_request;
typedef struct ba_server ba_server;

int ba_server_create(void *arena, uint64_t arena_bytes, void *stream, ba_server **out);
int ba_server_destroy(ba_server *s);
int ba_server_submit(ba_server *s, const ba_request *r, uint64_t *ticket);
int ba_server_pump(ba_server *s, uint32_t max_inflight, uint32_t *launched);
int ba_server_poll(ba_server *s, uint64_t ticket, int *state, double *done_ms, uint64_t *offset,
                   uint64_t *bytes);
int ba_server_completed(ba_server *s, uint64_t *tickets, uint32_t capacity, uint32_t *count);
int ba_server_release(ba_server *s, uint64_t ticket);
int ba_server_stats(ba_server *s, uint64_t *queued, uint32_t *inflight, uint64_t *arena_used);

/*
 * The generalized model (paper Section "Generalizations") and the paper's
 * CRC-based hash.  A seed graph of n0 nodes (IDs 0..n0-1) and m0 edges
 * (seed_edges: device array of 2*m0 node IDs below n0, pairs) occupies the
 * first 2*m0 positions of the edge array; nodes n0..n-1 then join with d
 * edges each.  New edge i (0 <= i < (n-n0)*d) is (n0 + floor(i/d), v_i),
 * where v_i follows positions r = 2*m0 + 2i + 1, x(r), x(x(r)), ... until a
 * seed position (v = seed_edges[r]) or an even position 2*m0 + 2j
 * (v = n0 + floor(j/d)).  The draw x(r) lies below
 *   r                               (default: self-loops allowed), or
 *   2*m0 + 2*d*floor(i/d)           (BA_NO_SELF_LOOPS: positions before the
 *                                    new node's own first edge, so v != u),
 * and is a hash of r itself: umul64hi(fmix64(r ^ key), bound) by default,
 * or with BA_HASH_CRC ((crc32c(0,z) << 32) + crc32c(1,z)) mod bound with
 * z = r ^ key (crc32c: the CRC-32C register update over the 8 bytes of z,
 * as the SSE4.2 crc32 instruction; with seed 0 this is the paper's
 * hash_crc).  With n0 = m0 = 0, no flags, it is ba_generate's graph.
 *
 * ba_generate_model writes new edges edge_begin .. edge_begin+edge_count-1
 * as uint32 pairs to `edges` (device, 2*edge_count, 4-byte aligned).
 * BA_EINVAL: unknown flags, n0 > n, null/misaligned buffers, a range past
 * (n-n0)*d, or BA_NO_SELF_LOOPS with m0 = 0 (node n0 would have nothing to
 * attach to); BA_ERANGE: n > 2^32 or positions beyond 2^63.  The seed
 * graph's IDs are not checked; IDs >= n0 pass through to the output.
 */
enum { BA_NO_SELF_LOOPS = 1, BA_HASH_CRC = 2 };
int ba_generate_model(uint64_t n, uint32_t d, uint64_t seed, uint64_t n0, uint64_t m0,
                      const uint32_t *seed_edges, uint32_t flags, uint64_t edge_begin,
                      uint64_t edge_count, uint32_t *edges, void *stream);

/* Text for a status code (static storage, never NULL). */
const char *ba_strerror(int status);

/* hipError_t of the last failed HIP call made by this thread, 0 if none. */
int ba_last_hip_error(void);

/*
 * Host-side self-test of the exact division by d the kernels use for
 * floor(i/d) and floor(r/(2d)) (multiply-high method of Granlund & Montgomery,
 * PLDI 1994, the round-up form for numerators one bit narrower than the
 * word): x < 2^31 takes the 32-bit form, x < 2^63 the 64-bit form, and
 * x >= 2^63 (never a kernel numerator) is divided plainly.  Writes
 * q[j] = floor(x[j] / d) computed that way, on the host, for count host
 * values.  d >= 1.  Returns BA_OK or BA_EINVAL.
 */
int ba_host_divide(uint32_t d, const uint64_t *x, uint64_t *q, uint64_t count);

/*
 * Host-side self-test of the exact remainder x mod b (1 <= b < 2^32) that the
 * CRC-hash kernels use on 32-bit positions for the paper's hash mod x: two
 * quotient estimates in double precision, each followed by one exact
 * correction.  Writes r[j] = x[j] mod b[j] for count host values, computed
 * that way on the host, from a reciprocal seed with a larger error than the
 * device's (so the self-test covers the device's error bound).  Returns
 * BA_OK, or BA_EINVAL for a NULL array with
 * count > 0 or any b[j] = 0.
 */
int ba_host_mod64(const uint64_t *x, const uint32_t *b, uint32_t *r, uint64_t count);

#ifdef __cplusplus
}
#endif

#endif /* BA_H */
