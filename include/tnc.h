/*
 * tnc.h -- C ABI of the MI355X (gfx950) tensor-network path executor.
 *
 * The library executes a fixed pairwise contraction path over a complex
 * tensor network on one GPU (arXiv 2606.01852, Sec. IV: the method takes as
 * given the leaf tensors, the order of pairwise contractions and which labels
 * are sliced).  Every step is put into GEMM form by
 * the GEMM-oriented mode reordering of Sec. IV-A and runs as a batched
 * complex GEMM on MFMA; operands whose stored order differs from the order
 * the step needs are permuted by an LDS-tiled transpose.
 *
 * Conventions shared by every call
 *   - Tensors are row-major, mode 0 outermost (Sec. IV-B: leading modes are
 *     the outermost memory dimensions).  Complex values are interleaved
 *     (re, im): complex64 = 2 x float32, complex128 = 2 x float64.
 *   - A label is a non-negative int32 below n_labels; extent_of_label[l] >= 1.
 *     A closed label joins exactly two tensors and is summed (Sec. II-A); an
 *     open label survives into the result, in the order of open_labels.  An
 *     open label carried by two or more tensors is a batch label: kept, not
 *     summed, wherever two operands share it.  A closed label held by one
 *     tensor or by three or more is rejected (TNC_E_ARG).
 *   - Path: SSA pairs.  Ids below n_tensors are the leaves; step s creates id
 *     n_tensors + s.  Every id is consumed exactly once and the last step
 *     yields the root (TNC_E_PATH otherwise).  A one-leaf network has no steps.
 *   - Slicing (Sec. II-C): sliced labels must be closed.  Slice s fixes them
 *     to the digits of s, row-major over sliced_labels (first most
 *     significant); a result is the sum over the requested slices.
 *   - Errors: every call returns a tnc_status; nothing throws or aborts
 *     across the ABI.  On error, outputs are left untouched and
 *     tnc_last_error() (thread-local) says why.  Asynchronous device faults
 *     surface as TNC_E_DEVICE at the next synchronising call.
 *   - Threads: tnc_submit / tnc_submit_row / tnc_poll / tnc_wait are
 *     thread-safe; every other call is single-threaded per context.  While
 *     a context serves (tnc_serve_start .. tnc_serve_stop), calls that would
 *     change what its worker threads read return TNC_E_BUSY: replacing
 *     leaves, tnc_plan_set_max_chunk / _autotune / _set_graph /
 *     _set_grouping / _set_profile, tnc_ctx_set_gemm_variant, and direct
 *     contractions (tnc_contract, tnc_contract_async).
 *   - "Device pointer" means memory on the context's GPU (e.g. a torch CUDA
 *     tensor's data_ptr()); "host pointer" means ordinary host memory.
 */
#ifndef TNC_H
#define TNC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TNC_OK = 0,
  TNC_E_ARG = 1,          /* malformed argument or network            */
  TNC_E_PATH = 2,         /* path is not a full binary tree            */
  TNC_E_NOMEM = 3,        /* planned peak exceeds the arena            */
  TNC_E_DEVICE = 4,       /* HIP runtime or kernel error               */
  TNC_E_BUSY = 5,         /* serving queue full                        */
  TNC_E_UNSUPPORTED = 6   /* request needs something not built here    */
} tnc_status;

/* Arithmetic of the GEMMs.  C64: complex64 operands, FP32 MFMA, FP32
 * accumulate (the paper's setting, Sec. V).  BF16X3: each float32 operand
 * plane is split into bf16 hi + lo (round to nearest even) and every real
 * product is a_hi*b_hi + a_hi*b_lo + a_lo*b_hi on bf16 MFMA with FP32
 * accumulate (an extension, not in the paper). */
typedef enum { TNC_PREC_C64 = 0, TNC_PREC_BF16X3 = 1 } tnc_prec;

/* Complex-GEMM form.  4M: four real products (re = ar*br - ai*bi,
 * im = ar*bi + ai*br), 8 real FLOPs per complex MAC.  3M: three real
 * products (T1 = ar*br, T2 = ai*bi, T3 = (ar+ai)(br+bi); re = T1 - T2,
 * im = T3 - T1 - T2), 6 executed FLOPs per complex MAC.  Both compose with
 * either precision on MFMA steps (BF16X3 + 3M: 9 bf16 products per complex
 * product instead of 12, the sums ar+ai and br+bi formed in float32 before
 * their split); the VALU kernels of small steps always use the 4M form. */
typedef enum { TNC_GEMM_4M = 0, TNC_GEMM_3M = 1 } tnc_cgemm;

/* Element type of host leaf data handed to the library. */
typedef enum { TNC_IN_C64 = 0, TNC_IN_C128 = 1 } tnc_in;

/* Entry points take these choices as int32_t holding one of the constants
 * above (any other value is TNC_E_ARG), so that no caller can hand the
 * library an enum value outside its range. */

typedef struct tnc_ctx_s* tnc_ctx;
typedef struct tnc_net_s* tnc_net;
typedef struct tnc_plan_s* tnc_plan;
typedef struct tnc_batcher_s* tnc_batcher;
typedef uint64_t tnc_req;

/* Last error message of the calling thread ("" if none).  Owned by the
 * library; valid until the thread's next tnc_* call. */
const char* tnc_last_error(void);

/* Library version string (static storage). */
const char* tnc_version(void);

/* ---------------------------------------------------------------- context
 * device      : HIP device ordinal, or -1 for a host-only context that can
 *               validate networks and build plans but runs nothing.
 * arena       : device pointer to caller-owned scratch for intermediates,
 *               or NULL to let the library allocate arena_bytes itself.
 * arena_bytes : arena size; all intermediates of a contraction live in it
 *               (plans whose planned peak exceeds it fail with TNC_E_NOMEM).
 * stream      : hipStream_t to launch on, or NULL for a library-owned
 *               stream.  Caller-owned arena/stream must outlive the context
 *               and every network and plan made from it. */
tnc_status tnc_ctx_create(int device, void* arena, size_t arena_bytes, void* stream, tnc_ctx* out);
tnc_status tnc_ctx_destroy(tnc_ctx ctx);
/* Number of HIP devices visible (0 when none); never fails. */
int tnc_device_count(void);

/* ---------------------------------------------------------------- network
 * ranks[n_tensors]; labels = concatenated mode labels of every tensor in its
 * stored order; extent_of_label[n_labels]; open_labels[n_open] = result mode
 * order.  host_data[t] = host pointer to tensor t (row-major, stored order,
 * element type `in`); the library copies every leaf to device memory it owns
 * (complex64), where it stays resident until tnc_net_destroy.  host_data may
 * be NULL on a host-only context (structure only).  All checks of Sec. II-A
 * happen here, on the host, before any device work. */
tnc_status tnc_net_create(tnc_ctx ctx, int32_t n_tensors, const int32_t* ranks,
                          const int32_t* labels, int32_t n_labels,
                          const int64_t* extent_of_label, int32_t n_open,
                          const int32_t* open_labels, const void* const* host_data,
                          int32_t in /* tnc_in */, tnc_net* out);
/* Replace leaf `tensor`'s values (same shape), e.g. a new bitstring's
 * projectors: the network's structure and the path stay, only a leaf's data
 * changes (Sec. II-A: a leaf is a tensor of the network; an amplitude
 * query fixes the output qubits' values through such leaves).
 * Synchronous host-to-device copy.  Plans of the network see
 * the new values from their next run on (cached permuted copies are
 * refreshed then); replacing a leaf while runs of its network are in flight
 * is a race. */
tnc_status tnc_net_set_tensor(tnc_net net, int32_t tensor, const void* host_data, int32_t in /* tnc_in */);
/* Replace leaf `tensor`'s values from a device pointer (complex64, stored
 * order).  Device-to-device copy on the context's stream (same rules). */
tnc_status tnc_net_set_tensor_device(tnc_net net, int32_t tensor, const void* dev_data);
tnc_status tnc_net_destroy(tnc_net net);

/* ---------------------------------------------------------------- plan
 * Builds the execution plan of a path (Sec. IV-A reordering, per-step GEMM
 * groups, permutations, memory plan).  ssa_pairs[2*n_steps].  A plan keeps
 * its network (and the network its context) alive: handles may be destroyed
 * in any order, and a destroyed plan's queued or running served requests
 * still complete. */
tnc_status tnc_plan_create(tnc_net net, int32_t n_steps, const int32_t* ssa_pairs,
                           int32_t n_sliced, const int32_t* sliced_labels,
                           int32_t prec /* tnc_prec */, int32_t cgemm /* tnc_cgemm */, tnc_plan* out);
tnc_status tnc_plan_destroy(tnc_plan plan);

typedef struct {
  double flops_per_slice;        /* 8 * sum_a h m n k (Sec. II-B convention)   */
  double bytes_per_slice;        /* 8 * sum_a C_m^(a): operands + result bytes */
  double transpose_bytes;        /* 16 * elements permuted per slice           */
  int64_t n_slices;              /* product of the sliced extents              */
  int64_t max_intermediate;      /* C_s: largest tensor, elements, one slice   */
  int64_t peak_bytes;            /* arena bytes of one slice                   */
  int64_t max_chunk;             /* slices executed together (batch)           */
  int64_t chunk_peak_bytes;      /* arena bytes of a max_chunk batch           */
  double chunk_flops;            /* FLOPs executed by one max_chunk batch: the
                                    slice-invariant steps run once per batch  */
  int32_t n_steps;
  int32_t n_permutes;            /* leaves permuted before use                 */
  int32_t n_permuted_stores;     /* steps whose output order interleaves M, N  */
  int32_t n_result;              /* elements of the result tensor              */
  int32_t n_cached_leaves;       /* leaves without a per-chunk base offset and
                                    up to 2^22 elements: permuted once into the
                                    plan's leaf cache (refreshed when their
                                    data is replaced), not in every run       */
  int32_t n_inplace_leaves;      /* leaves whose sliced labels are fixed per
                                    chunk, read in place by the GEMM that
                                    consumes them (no gather per batch)      */
  int64_t n_launches;            /* launches of one eager run over all slices
                                    (chunk base copies, leaf preparations,
                                    GEMMs and their epilogues or grouped
                                    launches, reductions)                   */
} tnc_plan_info;
tnc_status tnc_plan_get_info(tnc_plan plan, tnc_plan_info* out);

/* Per-step view of the plan for one slice (chunk of 1).  A, B, C are tensor
 * ids (A is the GEMM's M side); h, m, n, k are the products of the extents
 * of the H (batch), M, N, K groups; natural = 1 if C is stored [H|M|N]. */
typedef struct {
  int32_t A, B, C;
  int32_t nH, nM, nN, nK;
  int64_t h, m, n, k;
  int32_t natural;
  int32_t kernel;                /* 0 = MFMA tiles, 1 = small-shape VALU kernel,
                                    2 = long-K dot kernel (k large, m*n tiny)  */
  int32_t variant;               /* MFMA workgroup shape (autotuned)           */
  int32_t swapped;               /* 1 = the GEMM runs transposed (B supplies
                                    the rows) because that fills MFMA tiles   */
  int32_t split;                 /* K cut into this many parts (split-K)       */
  int64_t hA, hB;                /* batch entries A and B hold (1 = broadcast
                                    over the batch): the algorithmic bytes of
                                    the step are 8 (hA m k + hB n k + h m n)  */
  int32_t presplit;              /* 1 = split-bf16x3 step whose operands are
                                    split once into bf16 planes (in the plan's
                                    arena) and staged global -> LDS directly;
                                    bitwise the result of variant 3 (4M form)
                                    or of the 3M form's tiles (its three real
                                    products as three real GEMMs, then one
                                    combining pass)                          */
  int32_t presplit_fused;        /* bit 0 / bit 1: the permute that prepares
                                    operand A / B' (a leaf) writes its planes
                                    itself, one pass instead of a permute and
                                    a split (4M form)                        */
} tnc_step_info;
tnc_status tnc_plan_get_step(tnc_plan plan, int32_t step, tnc_step_info* out);
/* The same view for the batch of max_chunk slices the executor runs (h then
 * includes the batched slice labels the step's operands hold). */
tnc_status tnc_plan_get_batch_step(tnc_plan plan, int32_t step, tnc_step_info* out);
/* Mode order (labels) tensor `id` is stored in when the plan runs one slice:
 * the target order of the Sec. IV-A backward pass.  Writes min(cap, rank)
 * labels, sets *rank. */
tnc_status tnc_plan_get_order(tnc_plan plan, int32_t id, int32_t* labels, int32_t cap, int32_t* rank);

/* Upper bound on slices per device batch (default: as many as fit the arena). */
tnc_status tnc_plan_set_max_chunk(tnc_plan plan, int64_t max_chunk);
/* Time the candidate MFMA workgroup shapes of every GEMM step shape of the
 * plan on the device and keep the fastest (cached per context, and in the
 * file named by the environment variable TNC_AUTOTUNE_CACHE if set).
 * Untuned steps use a shape-based default.  Synchronous. */
tnc_status tnc_plan_autotune(tnc_plan plan);
/* 1 = capture each chunk's launches in a hipGraph and replay it.  A graph is
 * kept per chunk and set of buffers (arena interval, output, accumulator),
 * at most 64 per plan; runs with further buffer sets are launched eagerly
 * (same results). */
tnc_status tnc_plan_set_graph(tnc_plan plan, int32_t enable);
/* 1 (default) = run the contraction tree level by level (a step's level is
 * one more than the highest of its operands'): the small VALU GEMMs of one
 * level go out as one launch, the plain leaf gathers of one level as another.
 * Results are bitwise those of step-by-step launches (0).  Changing it
 * re-plans the chunks (the arena layout follows the execution order) and
 * drops captured graphs; refused with TNC_E_BUSY while the context serves. */
tnc_status tnc_plan_set_grouping(tnc_plan plan, int32_t enable);
/* Where an interleaved output is put in its consumer's order (Sec. IV-A:
 * the reordering exists so that no transpose runs between steps).  0
 * (default): the GEMM's epilogue stores every element straight to its
 * place in the consumer's order (per-row and per-column offset tables).
 * 1: the GEMM stores [batch | rows | columns] into a scratch buffer of the
 * arena and a separate LDS-tiled transpose writes the consumer's order: the
 * executor without the permuted-store epilogue, kept to measure what the
 * epilogue saves (results are bitwise the same).  Steps with split K keep
 * their epilogue pass.  Re-plans the chunks and drops captured graphs;
 * TNC_E_BUSY while the context serves. */
tnc_status tnc_plan_set_store_order(tnc_plan plan, int32_t mode);
/* 1 = time every kernel with HIP events on the launch stream. */
tnc_status tnc_plan_set_profile(tnc_plan plan, int32_t enable);
/* Per-step accumulated kernel time (ms) and launch count since profiling was
 * enabled; step = -1 gives the leaf permutations and gathers, -2 the FP64
 * reductions, -3 the grouped small-GEMM launches (one per tree level). */
tnc_status tnc_plan_get_profile(tnc_plan plan, int32_t step, double* ms, int64_t* launches);

/* ---------------------------------------------------------------- distribution plan
 * Offline planning of a multi-GPU execution (Sec. IV-B), on the host; the
 * library executes nothing across GPUs.  Steps whose operands or output reach
 * large_bytes start use-chains (the tensor's consumers up the tree, to the
 * last large step); along each chain a DP over the distributed modes
 * (Eq. (4) prefixes, tracked by label) chooses keep or redistribute per
 * equation under the cost model of Eq. (5)-(7), with forced redistribution
 * before an equation that sums a distributed mode, and a gather at the end. */
typedef struct {
  double hbm_bytes_per_s;   /* B_dev: device memory bandwidth              */
  double flops_per_s;       /* F_dev: device peak FLOP rate                */
  double net_bytes_per_s;   /* B_net: interconnect bandwidth per device    */
  double latency_s;         /* lambda: per-message latency                 */
} tnc_dist_hw;
typedef struct {
  int32_t chain;            /* use-chain index                             */
  int32_t step;             /* path step (equation)                        */
  int32_t state;            /* 0 activate, 1 keep, 2 redistribute          */
  int32_t n_dist;           /* distributed modes of the step's output      */
  int32_t dist[16];         /* their labels, in mode order                 */
  double t_gemm_s;          /* Eq. (6) per-device GEMM time                */
  double t_comm_s;          /* Eq. (7) redistribution time (0 if kept)     */
  double out_bytes;         /* |C| of the step                             */
} tnc_dist_step;
/* Writes min(cap, n) chain steps to steps[] (host array), sets *n_steps to
 * n, *total_s to the summed optimal chain time (gathers included) and
 * *redistributed_bytes to the all-to-all volume. */
tnc_status tnc_plan_distribute(tnc_plan plan, int32_t n_gpus, double large_bytes, const tnc_dist_hw* hw,
                               tnc_dist_step* steps, int32_t cap, int32_t* n_steps, double* total_s,
                               double* redistributed_bytes);
/* Measure the context's device: hw->flops_per_s = the FP32 MFMA rate of a
 * max-rate loop (independent accumulator chains, all compute units, no
 * memory traffic), hw->hbm_bytes_per_s = bytes read + written per second by
 * a 16-byte-per-lane copy of 2 GiB (best of three after a warm-up each).
 * net_bytes_per_s and latency_s are left as they are.  Allocates 4 GiB of
 * device memory for the duration of the call; synchronous; TNC_E_ARG on a
 * host-only context. */
tnc_status tnc_device_calibrate(tnc_ctx ctx, tnc_dist_hw* hw);

/* ---------------------------------------------------------------- contract
 * Sum over slices [first_slice, first_slice + n_slices) of the sliced
 * contractions (Sec. II-C: slicing fixes the sliced labels, each slice is an
 * independent contraction, and the result is the sum over all slices; every
 * slice is contracted along the path as in Sec. II-B), accumulated in FP64
 * on the device; out_c128 (host pointer,
 * n_result complex128 values, open-label order) receives the result.  A
 * closed network (n_open = 0) yields one amplitude.  Synchronous. */
tnc_status tnc_contract(tnc_plan plan, int64_t first_slice, int64_t n_slices, double* out_c128);
/* Same, but leaves the result on the device and does not synchronise.
 * out_dev: n_result elements of complex128 (TNC_OUT_C128) or complex64
 * (TNC_OUT_C64).  A single-slice complex64 request whose root order equals
 * the open-label order is written by the last GEMM directly (no FP64 pass);
 * otherwise the FP64 sum is rounded to complex64 at the end. */
typedef enum { TNC_OUT_C128 = 0, TNC_OUT_C64 = 1 } tnc_out;
tnc_status tnc_contract_async(tnc_plan plan, int64_t first_slice, int64_t n_slices, void* out_dev,
                              int32_t out_type /* tnc_out */);
/* Sum of |R|^2 over the last result of this plan, in FP64 on the device. */
tnc_status tnc_plan_result_norm2(tnc_plan plan, double* out);

/* ---------------------------------------------------------------- kernels
 * Operand permutation (a bit copy): out[pi(idx)] = in[idx] for a complex64
 * tensor of `rank` modes with extents in[rank] (input order); perm[j] = the
 * input mode that becomes output mode j.  in/out: device pointers, must not
 * overlap.  Asynchronous on the context's stream.  TNC_E_ARG for an extent
 * below 1, a size past 2^60 elements or a perm that is not a permutation
 * (checked before any device work); TNC_E_UNSUPPORTED on a host-only
 * context or above 64 modes. */
tnc_status tnc_permute(tnc_ctx ctx, const void* in, void* out, int32_t rank,
                       const int64_t* extents, const int32_t* perm);
/* The same permutation for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation): same arguments, checks and result as tnc_permute, but the
 * permutation's index tables go to a fixed device-resident table area of
 * 1 MiB per GPU that the library holds from its first context on that GPU
 * until the process ends, instead of memory the library allocates.
 * TNC_E_NOMEM if the tables need more than 1 MiB (decided on the host
 * before any device work; the tables of a 2^30-element permutation take
 * about 130 KiB).  Every call on one GPU shares that area and leaves its
 * own tables in it: a call first waits for the context's stream (earlier
 * calls on it have finished reading the area), copies its tables and waits
 * for the copy, then launches.  Calls that overlap on one GPU from
 * different streams or threads race on the area.  Small permutations that
 * run as a plain gather use no tables and do not wait. */
tnc_status tnc_permute_noalloc(tnc_ctx ctx, const void* in, void* out, int32_t rank,
                               const int64_t* extents, const int32_t* perm);
/* Batched complex GEMM with both operands K-contiguous:
 *   C[b, i, j] = sum_l A[b, i, l] * B[b, j, l]     (no conjugation)
 * A: h*m*k, B: h*n*k, C: h*m*n complex64 (device pointers, contiguous; a
 * batch stride of 0 for A or B broadcasts it).  Asynchronous. */
tnc_status tnc_batched_cgemm(tnc_ctx ctx, int64_t h, int64_t m, int64_t n, int64_t k,
                             const void* A, int64_t stride_a, const void* B, int64_t stride_b,
                             void* C, int32_t prec /* tnc_prec */, int32_t form /* tnc_cgemm */);
/* Force the MFMA tile variant of every complex GEMM this context launches
 * (0 .. tnc_gemm_variant_count()-1; -1 = the plan's autotuned choice).  For
 * tests and tuning sweeps. */
tnc_status tnc_ctx_set_gemm_variant(tnc_ctx ctx, int32_t variant);
int tnc_gemm_variant_count(void);
/* Synchronise the context's stream; TNC_E_DEVICE if a kernel failed. */
tnc_status tnc_ctx_sync(tnc_ctx ctx);

/* ---------------------------------------------------------------- serving
 * Continuous batching: requests are admitted while others run, as soon as a
 * slot and enough arena for the plan's planned peak are free; admitted
 * requests run concurrently on separate streams.  Requests whose planned
 * work reaches the heavy threshold (default 2^38 FLOP) share a lane of
 * heavy_slots slots (default 1): a heavy request waits only for heavy ones
 * ahead of it, and light requests behind a waiting heavy one are admitted
 * past it.  Otherwise admission is in submission order (a request that does
 * not fit the free arena yet blocks the ones behind it).  out_c128 (host
 * pointer) must stay valid until the request is done.  TNC_E_BUSY if the
 * queue is full or the plan's network has a batcher (see below);
 * TNC_E_NOMEM if the request can never fit.
 * On a host-only context (device -1, with an arena size) the server admits
 * and queues in the same way but executes nothing: every request completes
 * with TNC_E_UNSUPPORTED and leaves its output untouched (a dry run of the
 * admission and queueing). */
tnc_status tnc_serve_start(tnc_ctx ctx, int32_t max_inflight, int32_t queue_cap);
/* Heavy-request lane: threshold in planned FLOPs (<= 0 disables the lane)
 * and the number of heavy requests that may run at once (>= 1).  Applies to
 * admissions from now on; TNC_E_ARG if the context is not serving. */
tnc_status tnc_serve_set_heavy(tnc_ctx ctx, double heavy_flops, int32_t heavy_slots);
/* Fusion of light requests with one structure (an extension): requests
 * below the heavy threshold whose plans have the same network shape, path,
 * slicing, precision, GEMM form, chunking and tile variants, over slice
 * ranges that split into the same chunks (e.g. amplitudes of several
 * circuits of one geometry and depth, or slice ranges of one sliced
 * network), are admitted together as one job of up to max_requests
 * (default 8; 1 disables fusion) and run in lockstep with the launches of
 * one run: every MFMA step is one grouped launch over the requests' GEMMs
 * of that step (one persistent kernel whose workgroups loop over the tiles
 * of all of them; every tile variant in 4M, all but 3 in 3M, 0 and 4-6 in
 * split precision's 4M form, all but 3 in its 3M form, other steps one
 * launch per request), and every tree level's small GEMMs and leaf gathers of
 * all the requests are one launch each.  Only requests that wait on their
 * launches more than on their arithmetic are fused: planned FLOP below
 * flops_per_launch times the launches of the request's own run
 * (tnc_plan_info.n_launches for a whole-range request; default 2^30, set
 * between a measured 1.05x gain at 4.5e8 FLOP per launch and a 0.96x loss
 * at 4.1e9); heavier requests would lose the overlap of separate streams.  A huge flops_per_launch (e.g. 1e300) fuses every
 * light request.  Each request's result is bitwise the one it gets alone:
 * its every output element is computed by the same tile code in the same
 * order.  Applies to admissions from now on; TNC_E_ARG if the context is
 * not serving, max_requests is outside 1..64 or flops_per_launch is not
 * positive. */
tnc_status tnc_serve_set_fusion(tnc_ctx ctx, int32_t max_requests, double flops_per_launch);
/* Counters since tnc_serve_start: jobs run (a fused job or a batch of rows
 * counts once), fused jobs, and requests that ran in fused jobs. */
tnc_status tnc_serve_get_stats(tnc_ctx ctx, int64_t* jobs, int64_t* fused_jobs, int64_t* fused_requests);
tnc_status tnc_serve_stop(tnc_ctx ctx);
tnc_status tnc_submit(tnc_ctx ctx, tnc_plan plan, int64_t first_slice, int64_t n_slices,
                      double* out_c128, tnc_req* id);

/* Dynamic batching of row requests (an extension; the paper serves no
 * requests).  `plan`'s network carries an open label `batch_label` of
 * extent B that is the first label of its open list and the outermost
 * stored mode of each of the n_leaves listed leaves, and no other leaf
 * carries it (e.g. the projector leaves of B amplitude queries of one
 * circuit).  A row request supplies those leaves' values for one batch row;
 * the server takes up to B queued rows of one batcher at once, writes them
 * into rows 0..k-1 of the listed leaves (device copies owned by the network)
 * and runs the plan once over all its slices, so the same-shape steps of k
 * requests run as one launch per step.  Rows k..B-1 keep older values and
 * their results are dropped.  One batch of a batcher runs at a time; rows
 * queued meanwhile go into the next.  A row's result is the row of the
 * plan's result at its batch position (the result without the batch label,
 * R / B complex values).
 * tnc_batcher_create: TNC_E_ARG if the label or the leaves do not have that
 * form, TNC_E_BUSY if the network already has a batcher.  The listed leaves
 * are excluded from the plan's leaf cache (chunks built before are
 * rebuilt); call it when the plan is not running.  While a batcher exists,
 * tnc_submit refuses plans on its network (TNC_E_BUSY): batches overwrite
 * its leaves.  The handle may be destroyed while rows are queued (they still
 * run); the network is released from the batcher when the last row is done. */
tnc_status tnc_batcher_create(tnc_plan plan, int32_t batch_label, int32_t n_leaves, const int32_t* leaves,
                              tnc_batcher* out);
tnc_status tnc_batcher_destroy(tnc_batcher b);
/* Queue one row: row_data[i] = host pointer to the values of leaves[i]
 * without the batch mode (numel / B elements, stored order, element type
 * `in`), copied before the call returns; out_c128 (host, R / B complex128)
 * must stay valid until the request is done.  Heavy classification and
 * admission as for tnc_submit, with the batch's work and arena need. */
tnc_status tnc_submit_row(tnc_ctx ctx, tnc_batcher b, const void* const* row_data, int32_t in /* tnc_in */,
                          double* out_c128, tnc_req* id);
/* done = 1 when finished; latency_s = submit-to-done wall time (else 0);
 * status of the request's execution is returned once done.  tnc_wait
 * collects an id (after it, the id is unknown: TNC_E_ARG); tnc_poll does
 * not.  A finished request no longer holds its plan, but its small record
 * stays until collected or until the server stops. */
tnc_status tnc_poll(tnc_ctx ctx, tnc_req id, int32_t* done, double* latency_s);
tnc_status tnc_wait(tnc_ctx ctx, tnc_req id, double* latency_s);

#ifdef __cplusplus
}
#endif
#endif /* TNC_H */
