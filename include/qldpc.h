/*
 * qldpc.h -- C ABI of the MI355X syndrome min-sum decoder library.
 *
 * The library decodes syndromes of quantum LDPC CSS codes with the
 * normalized min-sum algorithm for syndrome-based decoding (Section 2,
 * Algorithm 1 of "GPU-Accelerated Syndrome Decoding for Quantum LDPC Codes
 * below the 63 us Latency Threshold").  Given one CSS side H (m checks,
 * n variables) and a syndrome s = H e^T over GF(2) (Section 2, problem
 * statement), it returns an estimate e_hat with H e_hat^T = s when the
 * decoder converges.  One CSS side is one code object; decoding X and Z
 * errors means two code objects (Section 2, CSS decoding).
 *
 * Conventions
 *  - Every function returns qldpc_status and never aborts.  On failure,
 *    qldpc_last_error() returns a message for the calling thread; out
 *    parameters are written only on success.
 *  - Host pointers are read during the call only.  Device pointers are
 *    caller-owned device memory (e.g. PyTorch tensors) and must stay valid
 *    until the work enqueued on `stream` has finished.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Decode calls
 *    enqueue work and return without synchronising; they allocate nothing.
 *    Argument checks are synchronous; device faults surface as
 *    QLDPC_ERR_DEVICE from a later call or at stream synchronisation.
 *  - Bit vectors (syndromes, error estimates) are packed per shot: bit i is
 *    bit (i mod 32) of 32-bit word floor(i / 32), least significant first;
 *    each shot's row is padded to whole words.  Pad bits are ignored on
 *    input and written as zero.
 *  - A code object is immutable after creation and may be used from any
 *    host thread and stream concurrently.
 */
#ifndef QLDPC_H
#define QLDPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QLDPC_OK = 0,
    QLDPC_ERR_INVALID_ARG = 1,   /* null pointer, bad size, malformed matrix  */
    QLDPC_ERR_UNSUPPORTED = 2,   /* valid input this build has no kernel for  */
    QLDPC_ERR_OUT_OF_MEMORY = 3, /* device allocation failed at create time   */
    QLDPC_ERR_DEVICE = 4,        /* a HIP call failed                          */
    QLDPC_ERR_CAPACITY = 5,      /* admission refused: over the memory budget  */
    QLDPC_ERR_NOT_READY = 6      /* nothing to return yet                      */
} qldpc_status;

/* Thread-local message describing the last failure of this thread. */
const char *qldpc_last_error(void);

/* Library version as major * 10000 + minor * 100 + patch. */
int32_t qldpc_version(void);

/* ------------------------------------------------------------------------ */
/* Code objects (Section 2: parity-check matrix H, Tanner graph S_v / S_c)   */
/* ------------------------------------------------------------------------ */

typedef struct qldpc_code_s *qldpc_code;

/* One CSS side.  H is given as host CSR: row r holds columns
 * col_idx[row_ptr[r] .. row_ptr[r+1]-1], strictly increasing.  Edge e of
 * the code is CSR position e (row-major, increasing column); it indexes the
 * per-edge neural weights.
 *
 * Quasi-cyclic lift data (optional): H is a base_m x base_n array of L x L
 * blocks, base_exp[R * base_n + C] = a >= 0 for the circulant P^a
 * (P^a[r][(r + a) mod L] = 1) or -1 for a zero block; then m = base_m * L
 * and n = base_n * L, and the CSR must equal the expansion (checked).
 *
 * Two device forms.  A lift with the block pattern of a lifted-product code
 * LP(A, A*) with a 3 x 5 monomial base (H_Z or H_X side) and L in {16, 32,
 * 64, 128, 256, 512} selects the lifted kernels, which read only the
 * circulant shifts (every layout, both schedules).  Any other valid H --
 * lift_L = 0, or a lift without such a pattern -- selects the edge-list
 * decoder: flooding over the CSR (check pass) and CSC (variable pass) edge
 * lists, one wavefront per shot with the messages in LDS, all three message
 * formats, both prior modes, posteriors; the layered schedule, the other
 * layouts, sessions in resident mode, mixed plans, neural min-sum and the
 * server then return QLDPC_ERR_UNSUPPORTED.  The edge-list decoder needs
 * max_dc * m messages (padded rows) plus the packed decisions and syndrome
 * within 64 KB: code_create refuses codes that exceed it even in int8
 * (QLDPC_ERR_UNSUPPORTED) and a decode in a wider format that exceeds it
 * returns QLDPC_ERR_UNSUPPORTED. */
typedef struct {
    int32_t m, n;
    const int32_t *row_ptr;   /* host, m + 1 entries, row_ptr[0] = 0 */
    const int32_t *col_idx;   /* host, row_ptr[m] entries            */
    int32_t lift_L;           /* 0 = no lift data                    */
    int32_t base_m, base_n;
    const int32_t *base_exp;  /* host, base_m * base_n entries       */
} qldpc_code_desc;

/* Validates the description, copies what the kernels need to `device`
 * (allocated once, here), and returns a new code object.  Errors:
 * INVALID_ARG (malformed CSR, lift data disagreeing with the CSR, a check of
 * degree < 2, whose check update in Algorithm 1 would have no other edge to
 * take the minimum over), UNSUPPORTED (a code too large for the edge-list
 * decoder), OUT_OF_MEMORY, DEVICE. */
qldpc_status qldpc_code_create(const qldpc_code_desc *desc, int32_t device, qldpc_code *out);

/* Releases the code object and its device memory.  No work using the code
 * may be pending.  NULL is accepted. */
qldpc_status qldpc_code_destroy(qldpc_code code);

/* m, n, number of edges, maximum check and variable degree (any out pointer
 * may be NULL). */
qldpc_status qldpc_code_info(qldpc_code code, int32_t *m, int32_t *n, int32_t *nnz,
                             int32_t *max_dc, int32_t *max_dv);

/* ------------------------------------------------------------------------ */
/* Batched decoding (Algorithm 1)                                            */
/* ------------------------------------------------------------------------ */

typedef enum {
    QLDPC_F32 = 0,   /* FP32 messages; priors are float LLRs                 */
    QLDPC_I8Q4 = 1,  /* int8 saturating messages in [-127, 127]; priors are
                        int8 Q4 fixed point (LLR * 16, see
                        qldpc_quantize_prior); alpha must be num / 2^sh       */
    QLDPC_I16Q8 = 2  /* int16 saturating messages in [-32767, 32767]; priors
                        are int16 Q8 fixed point (LLR * 256, see
                        qldpc_quantize_prior_q8); alpha must be num / 2^sh.
                        The 8- and 16-bit integer data types are the paper's
                        reduced-precision formats (Section 3, Table 1).  Every
                        layout, lift and pattern supports it; sums are exact
                        in 32-bit integers.                                   */
} qldpc_format;

typedef enum {
    QLDPC_FLOOD = 0,   /* all check nodes, then all variable nodes (Alg. 1)  */
    QLDPC_LAYERED = 1  /* block row by block row, posterior updated in place */
} qldpc_schedule;

typedef enum {
    QLDPC_PRIOR_PER_SHOT = 0,  /* priors [batch]: one LLR for every bit      */
    QLDPC_PRIOR_PER_BIT = 1    /* priors [batch][n]                          */
} qldpc_prior_mode;

typedef enum {
    QLDPC_LAYOUT_AUTO = 0,   /* tuned choice for (code, format, batch) when
                                qldpc_autotune recorded one; otherwise:
                                flooding at L in {64, 128} with batch < 512
                                BLOCK (16 waves); otherwise WAVE_REG for
                                L <= 64 and for flooding at L >= 128, WAVE
                                for layered at L = 128, HBM (unsupported)
                                for layered at L >= 256                    */
    QLDPC_LAYOUT_WAVE = 1,   /* one wavefront decodes one shot (or 64 / L
                                shots when L < 64); throughput layout        */
    QLDPC_LAYOUT_BLOCK = 2,  /* one workgroup of several wavefronts decodes
                                one shot, messages in LDS; flooding, L >= 64;
                                the latency layout                          */
    QLDPC_LAYOUT_HBM = 4,    /* one workgroup decodes one shot with its edge
                                messages in a caller-provided device
                                workspace (qldpc_decode_batch_ws); flooding
                                with L in {128, 256, 512}; never AUTO's
                                choice (the register layout is faster)      */
    QLDPC_LAYOUT_WAVE_REG = 3 /* as WAVE, with every message (and, layered,
                                every a-posteriori value) kept in the lanes'
                                registers and moved between lanes by
                                cross-lane permutes instead of LDS (integer
                                messages as exact values on FP32 lanes);
                                L <= 64, and L in {128, 256, 512} with
                                flooding: one workgroup of L / 64 wavefronts
                                per shot, each holding 64 rows of every
                                circulant, the variable pass exchanging
                                through LDS (otherwise
                                QLDPC_ERR_UNSUPPORTED)                       */
} qldpc_layout;

typedef struct {
    int32_t fmt;          /* qldpc_format                                    */
    int32_t sched;        /* qldpc_schedule                                  */
    float alpha;          /* normalisation factor in (0, 1] (Section 2)      */
    int32_t max_iters;    /* I_max, 1 .. 255                                  */
    int32_t early_stop;   /* 1: stop a shot once H e^(k) = s                 */
    int32_t prior_mode;   /* qldpc_prior_mode                                */
    int32_t layout;       /* qldpc_layout                                    */
    int32_t waves_per_shot; /* block layout: wavefronts per shot, 8 or 16;
                               0 = tuned choice                                */
} qldpc_decode_params;

/* Fills `p` with the defaults: F32, flooding, alpha 0.75, 32 iterations,
 * early stop on, per-shot priors, automatic layout and waves per shot. */
void qldpc_default_params(qldpc_decode_params *p);

/* Decodes `batch` syndromes of one code.
 *   syndromes  device uint32 [batch][ceil(m/32)]
 *   priors     device float [batch] or [batch][n] (F32), int8 likewise (I8Q4),
 *              int16 likewise (I16Q8)
 *   errors     device uint32 [batch][ceil(n/32)], out: e_hat
 *   converged  device uint8 [batch], out: 1 iff H e_hat = s at exit
 *   iters_used device uint8 [batch], out, may be NULL: iterations executed
 *   posterior  device float [batch][n], out, may be NULL: a-posteriori LLR Q
 *              of the returned iteration (I8Q4: Q / 16; I16Q8: Q / 256)
 * For each shot, the iteration k whose decision is returned is the first
 * with H e^(k) = s when early_stop is set, else max_iters.  batch = 0 is a
 * no-op.  Errors: INVALID_ARG, UNSUPPORTED (format/schedule/layout
 * combination without a kernel), DEVICE. */
qldpc_status qldpc_decode_batch(qldpc_code code, const qldpc_decode_params *params, int32_t batch,
                                const uint32_t *syndromes, const void *priors, uint32_t *errors,
                                uint8_t *converged, uint8_t *iters_used, float *posterior,
                                void *stream);

/* Device bytes of message workspace a decode of `batch` shots with these
 * parameters needs when called through qldpc_decode_batch_ws: batch * 120
 * * L * (4 for F32, 1 for I8Q4, 2 for I16Q8) when the chosen layout keeps messages in
 * device memory (QLDPC_LAYOUT_HBM, asked for explicitly), else 0.  Errors as
 * qldpc_decode_batch. */
qldpc_status qldpc_decode_workspace_bytes(qldpc_code code, const qldpc_decode_params *params, int32_t batch,
                                          size_t *bytes);

/* qldpc_decode_batch with a caller-owned device workspace of
 * `workspace_bytes` (at least qldpc_decode_workspace_bytes; 256-byte
 * aligned; contents need no initialisation and are garbage afterwards).
 * Layouts that keep messages on chip ignore it (it may then be NULL).
 * qldpc_decode_batch on a layout that needs a workspace returns
 * QLDPC_ERR_UNSUPPORTED.  Calls sharing a workspace must not overlap. */
qldpc_status qldpc_decode_batch_ws(qldpc_code code, const qldpc_decode_params *params, int32_t batch,
                                   const uint32_t *syndromes, const void *priors, uint32_t *errors,
                                   uint8_t *converged, uint8_t *iters_used, float *posterior, void *workspace,
                                   size_t workspace_bytes, void *stream);

/* Bytes of the library's own message workspace on each device. */
#define QLDPC_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * decode as qldpc_decode_batch_ws, with the message workspace taken from a
 * buffer of QLDPC_STATIC_WORKSPACE_BYTES (64 MiB) that the library holds on
 * each device until the process ends.  Allocates nothing.  Arguments,
 * layouts and results are those of qldpc_decode_batch; layouts that keep
 * messages on chip use no workspace.  A batch whose workspace
 * (qldpc_decode_workspace_bytes) exceeds the buffer returns
 * QLDPC_ERR_CAPACITY (e.g. at most 546 FP32 or 2184 int8 shots per call at
 * L = 256 in the HBM layout).  The first call on a device looks up that device's buffer
 * (hipGetSymbolAddress) with the device current.  Every call on a device
 * shares its one buffer: calls that overlap on one device (other streams or
 * threads) race, and the caller must serialise them. */
qldpc_status qldpc_decode_batch_static(qldpc_code code, const qldpc_decode_params *params, int32_t batch,
                                       const uint32_t *syndromes, const void *priors, uint32_t *errors,
                                       uint8_t *converged, uint8_t *iters_used, float *posterior,
                                       void *stream);

/* ------------------------------------------------------------------------ */
/* Layout autotuner                                                          */
/* ------------------------------------------------------------------------ */

/* Layout tuning: the thread and block configuration and the choice between
 * on-chip (LDS or register) and device-memory messages are the tuning space
 * the paper lists (Table 1 and Section 3).
 * Times every kernel layout that can run `params` (wavefront per shot; one
 * workgroup of 8 or 16 wavefronts per shot) on the caller's batch -- the
 * buffers are those of qldpc_decode_batch, decoded several times -- and
 * returns the fastest in `best` (layout and waves_per_shot filled in, other
 * fields copied from `params`).  The choice is also recorded in the code
 * object for this (format, schedule, prior mode, batch size class), and
 * later calls with QLDPC_LAYOUT_AUTO use it.  Synchronises `stream`.
 * Batch size classes: 1, 2-64, 65-1024, 1025-16384, > 16384 shots.  Without
 * a recorded choice, AUTO uses the workgroup layout with 16 wavefronts for
 * flooding below 512 shots and the wavefront layout otherwise. */
qldpc_status qldpc_autotune(qldpc_code code, const qldpc_decode_params *params, int32_t batch,
                            const uint32_t *syndromes, const void *priors, uint32_t *errors,
                            uint8_t *converged, uint8_t *iters_used, void *stream,
                            qldpc_decode_params *best);

/* Writes the recorded choices of `code` as one JSON object to `path`, or
 * reads such a file back into `code` (entries for other lift sizes or code
 * patterns are ignored). */
qldpc_status qldpc_tune_save(qldpc_code code, const char *path);
qldpc_status qldpc_tune_load(qldpc_code code, const char *path);

/* ------------------------------------------------------------------------ */
/* Latency sessions: host buffers in, host buffers out                       */
/* ------------------------------------------------------------------------ */

typedef struct qldpc_session_s *qldpc_session;

typedef enum {
    QLDPC_IO_COPY = 0,   /* pinned staging + copy-in, decode, copy-out on a
                            private stream, captured once as a hipGraph per
                            batch size                                          */
    QLDPC_IO_MAPPED = 1, /* the kernel reads syndromes and writes results in
                            pinned host memory directly (no copy commands)     */
    QLDPC_IO_RESIDENT = 2 /* as MAPPED, with the decoder kept resident on the
                            GPU between requests: one workgroup per shot slot
                            polls a doorbell page in host memory, so a request
                            costs no launch and no stream synchronisation.
                            Flooding with L >= 64 only (the workgroup layout;
                            waves_per_shot 8 or 16, default 16); max_batch <=
                            64; no posteriors.  The grid occupies max_batch
                            compute units while it waits; it leaves after
                            200 ms without a request (the next request
                            relaunches it) or when the session is destroyed.
                            A device-wide synchronisation on the same device
                            (hipDeviceSynchronize, torch.cuda.synchronize)
                            therefore waits up to that idle time.  A request
                            with no answer after 10 s fails with
                            QLDPC_ERR_DEVICE; so does qldpc_session_destroy
                            if the grid has not left 10 s after it was asked
                            to (the session is then leaked, not freed under
                            a running kernel).                                  */
} qldpc_io_mode;

/* A session owns device buffers and pinned host staging for up to
 * `max_batch` shots, a private stream, and its captured graphs.  It measures
 * what the paper's latency figure counts: host syndrome to host result,
 * host-to-device and device-to-host transfers included (Section 3 and the
 * caption of Fig. 3; the 63 us target of Section 1). */
qldpc_status qldpc_session_create(qldpc_code code, const qldpc_decode_params *params,
                                  int32_t max_batch, int32_t io_mode, qldpc_session *out);
qldpc_status qldpc_session_destroy(qldpc_session s);

/* A resident session over the two sides of one CSS code (the paper decodes
 * the X and Z syndromes of a round together, Section 2): hz_side has the
 * H_Z block pattern and hx_side the H_X pattern of the same lift (64 or 128),
 * on the same device.  A request item is a syndrome pair: the H_Z syndrome
 * (of X errors) followed by the H_X syndrome (of Z errors); both are decoded
 * at once by workgroups of the same resident grid.  With such a session,
 * qldpc_session_decode and qldpc_session_latency count `batch` in pairs, and
 * every per-shot buffer holds two entries per pair, H_Z side first:
 * syndromes [batch][2][ceil(m/32)], priors [batch][2] (or [batch][2][n]),
 * errors [batch][2][ceil(n/32)], converged and iters_used [batch][2].
 * max_pairs in [1, 32]; FP32 or int8 (else UNSUPPORTED); io mode RESIDENT
 * with its rules.  Errors: INVALID_ARG (null, bad sizes, patterns or lifts
 * that do not pair), UNSUPPORTED, OUT_OF_MEMORY, DEVICE. */
qldpc_status qldpc_session_create_css(qldpc_code hz_side, qldpc_code hx_side, const qldpc_decode_params *params,
                                      int32_t max_pairs, qldpc_session *out);

/* Synchronous decode of `batch` <= max_batch shots from host buffers
 * (syndromes uint32 [batch][ceil(m/32)], priors as in qldpc_decode_batch)
 * into host buffers (errors, converged, iters_used may be NULL); for a CSS
 * pair session, `batch` <= max_pairs pairs as described above. */
qldpc_status qldpc_session_decode(qldpc_session s, int32_t batch, const uint32_t *host_syndromes,
                                  const void *host_priors, uint32_t *host_errors,
                                  uint8_t *host_converged, uint8_t *host_iters);

/* Runs `nreq` back-to-back session decodes of `batch` shots each, taking
 * request i from shot (i * batch) mod pool of the host pools, and writes
 * each request's end-to-end time in microseconds (steady clock) to
 * lat_us[i]. */
qldpc_status qldpc_session_latency(qldpc_session s, int32_t nreq, int32_t batch, int32_t pool,
                                   const uint32_t *host_syndromes, const void *host_priors,
                                   double *lat_us);

/* ------------------------------------------------------------------------ */
/* Mixed-code persistent batches: shots of several lifted codes (L in        */
/* {16, 32, 64, 128}, H_Z or H_X pattern) with per-shot priors decoded in    */
/* one persistent launch sequence (batching of many decoders, Table 1       */
/* "asynchronous kernel execution"; each shot follows Algorithm 1 on its    */
/* own code).  Both sides of a CSS code can share one batch, the paper's    */
/* concatenated X and Z decoding (Section 2).                               */
/* ------------------------------------------------------------------------ */

typedef struct qldpc_mixed_s *qldpc_mixed;

/* Plan over 1..8 code objects on one device for batches of up to
 * max_batch shots (FP32 flooding, per-shot priors; params gives alpha,
 * iterations and early stop; lifts 16, 32, 64 and 128).  Allocates
 * 4 * (max_batch + 24) bytes of device scratch.  One persistent grid per
 * (pattern, lift size) decodes its shots with its messages in registers: a
 * wavefront per tile of 64 / L shots for L <= 64, a workgroup of two
 * wavefronts per shot for L = 128.  use_graph = 1: every distinct argument
 * set is captured once as a hipGraph (bucketing kernels + persistent
 * decoders, each lift size's grids on a parallel branch) and replayed;
 * use_graph = 0: launched directly, the L = 128 grids on a side stream
 * beside the others (the plan owns its side streams). */
qldpc_status qldpc_mixed_create(const qldpc_code *codes, int32_t ncodes, const qldpc_decode_params *params,
                                int32_t max_batch, int32_t use_graph, qldpc_mixed *out);
qldpc_status qldpc_mixed_destroy(qldpc_mixed plan);

/* Shot i belongs to code shot_code[i] (device int32 [batch], index into the
 * plan's codes; other values leave the shot untouched); its packed syndrome
 * starts at syndromes + syn_off[i] words and its error estimate is written
 * at errors + err_off[i] words (device int64 [batch] each; the caller
 * guarantees ceil(m/32) and ceil(n/32) words of room).  priors: device float
 * [batch]; converged / iters_used: device uint8 [batch].  A shot's result
 * equals qldpc_decode_batch of that shot alone.  Calls on one plan must not
 * overlap (the scratch is shared). */
qldpc_status qldpc_mixed_decode(qldpc_mixed plan, int32_t batch, const int32_t *shot_code,
                                const int64_t *syn_off, const int64_t *err_off, const uint32_t *syndromes,
                                const float *priors, uint32_t *errors, uint8_t *converged,
                                uint8_t *iters_used, void *stream);

/* Sets the persistent grid sizes of a plan: `reg_waves` wavefronts for each
 * (pattern, lift) with L <= 64 and `block_workgroups` two-wave workgroups
 * for L = 128 (0 keeps the current value; defaults 12 and 6 per compute
 * unit).  With
 * fewer waves than tiles every wavefront claims several tiles in turn.  The
 * plan's captured graphs are dropped.  Errors: INVALID_ARG. */
qldpc_status qldpc_mixed_set_grid(qldpc_mixed plan, int32_t reg_waves, int32_t block_workgroups);

/* Times the register-resident persistent grid (codes with L <= 64) at 6,
 * 12, 24 and 48 wavefronts per compute unit on the caller's batch, keeps
 * the fastest in the plan and returns it. */
qldpc_status qldpc_mixed_autotune(qldpc_mixed plan, int32_t batch, const int32_t *shot_code,
                                  const int64_t *syn_off, const int64_t *err_off, const uint32_t *syndromes,
                                  const float *priors, uint32_t *errors, uint8_t *converged,
                                  uint8_t *iters_used, void *stream, int32_t *best_waves);

/* ------------------------------------------------------------------------ */
/* Neural min-sum: flooding min-sum whose check rule scales edge e at        */
/* iteration k by a learned weight w[k][e] instead of alpha (Section 2,      */
/* Algorithm 1, check-node update, with alpha generalised per edge and       */
/* iteration).  FP32 messages, per-shot priors, lifted codes with            */
/* L in {32, 64, 128} (H_Z pattern).  Weights are device float [T][nnz],     */
/* edge e = CSR position, 16-byte aligned.  Training runs exactly T          */
/* iterations without early stop.                                            */
/* ------------------------------------------------------------------------ */

/* Device workspace the forward pass fills and the backward pass reads:
 * every iteration's check-node inputs plus per-wavefront gradient slices
 * (about T * batch * nnz * 4 bytes). */
qldpc_status qldpc_nbp_workspace_bytes(qldpc_code code, int32_t batch, int32_t T, size_t *bytes);

/* posteriors: device float [T][batch][n], out: Q^(k) of iterations 1..T.
 * syndromes and priors as in qldpc_decode_batch (priors [batch]).
 * workspace: device, qldpc_nbp_workspace_bytes, caller-owned. */
qldpc_status qldpc_nbp_forward(qldpc_code code, int32_t batch, int32_t T, const float *weights,
                               const uint32_t *syndromes, const float *priors, float *posteriors,
                               void *workspace, void *stream);

/* Reverse-mode derivative of the forward map.  grad_posteriors: device
 * float [T][batch][n] = dL/dQ^(k); grad_weights: device float [T][nnz], out
 * (overwritten) = dL/dw summed over the batch.  workspace must hold the
 * forward pass of the same inputs and weights.  Signs carry no gradient;
 * the minimum routes its gradient to the lowest-index edge on ties.  The
 * result is bit-reproducible (fixed-order reduction, no atomics). */
qldpc_status qldpc_nbp_backward(qldpc_code code, int32_t batch, int32_t T, const float *weights,
                                const uint32_t *syndromes, const void *workspace,
                                const float *grad_posteriors, float *grad_weights, void *stream);

/* Inference: neural min-sum with early stop for at most T iterations; the
 * shots that do not converge are decoded again from scratch with plain
 * min-sum under `fallback` (FP32, per-shot priors; NULL = no fallback).
 * used_fallback: device uint8 [batch], out: 1 where the fallback ran.
 * errors / converged / iters_used describe the returned decode. */
qldpc_status qldpc_nbp_decode(qldpc_code code, int32_t batch, int32_t T, const float *weights,
                              const qldpc_decode_params *fallback, const uint32_t *syndromes,
                              const float *priors, uint32_t *errors, uint8_t *converged,
                              uint8_t *iters_used, uint8_t *used_fallback, void *stream);

/* Inference with a continuing fallback: neural min-sum (weights [T][nnz])
 * in iterations 1..T, then plain min-sum with `alpha` continuing from the
 * neural decoder's messages in iterations T+1..max_iters (T <= max_iters
 * <= 255), early stop throughout, in one pass.  iters_used (required) counts
 * every iteration; used_fallback: device uint8 [batch], out: 1 where plain
 * iterations ran (iters_used > T).  Same codes and buffers as
 * qldpc_nbp_decode.  Errors: INVALID_ARG, UNSUPPORTED, DEVICE. */
qldpc_status qldpc_nbp_decode_continue(qldpc_code code, int32_t batch, int32_t T, const float *weights,
                                       int32_t max_iters, float alpha, const uint32_t *syndromes,
                                       const float *priors, uint32_t *errors, uint8_t *converged,
                                       uint8_t *iters_used, uint8_t *used_fallback, void *stream);

/* ------------------------------------------------------------------------ */
/* Serving: continuous batching of decode requests (several asynchronous     */
/* decoders overlapping copies and kernels, Table 1 and Section 3)           */
/* ------------------------------------------------------------------------ */

typedef struct qldpc_server_s *qldpc_server;

typedef struct {
    const qldpc_code *codes;          /* 1..8 codes served (H_Z or H_X pattern;
                                         neural weights for H_Z ones only)          */
    int32_t ncodes;
    const float *const *nms_weights;  /* per code: device [nms_T][nnz] neural weights
                                         or NULL (plain min-sum only); the array may
                                         itself be NULL                               */
    int32_t nms_T;                    /* neural iterations before the fallback      */
    qldpc_decode_params params;       /* plain min-sum and fallback: FP32 flooding,
                                         per-shot priors                             */
    size_t hbm_budget;                /* device bytes for in-flight work, 0 = no cap;
                                         slots = min(max_inflight, budget / slot)    */
    int32_t max_inflight;             /* micro-batches on the device at once        */
    int32_t max_batch_shots;          /* shots per micro-batch (largest request)    */
    int32_t queue_capacity;           /* queued requests before submit refuses      */
} qldpc_server_config;

typedef struct {
    uint64_t req_id;
    int32_t code_id, decoder, nshots, status;
    int64_t t_submit_ns, t_done_ns;   /* steady clock                               */
} qldpc_completion;

/* Starts the server: allocates every slot (device buffers, pinned staging,
 * stream, mixed-code plan) up front and a scheduler thread.  CAPACITY if the
 * HBM budget is below one slot. */
qldpc_status qldpc_server_create(const qldpc_server_config *cfg, qldpc_server *out);

/* Slot count, device bytes per slot, queued requests, shots on the device. */
qldpc_status qldpc_server_info(qldpc_server srv, int32_t *slots, size_t *slot_bytes, int32_t *pending,
                               int64_t *inflight_shots);

/* Queues a request of nshots syndromes of code code_id (host uint32
 * [nshots][ceil(m/32)]) with per-shot priors (host float [nshots]);
 * decoder 0 = plain min-sum, 1 = neural min-sum with fallback.  Results go
 * to the caller's host buffers (errors [nshots][ceil(n/32)], converged and
 * iters [nshots]; any may be NULL), which must stay valid until the
 * request's completion is polled.  CAPACITY when the queue is full (the
 * request is not queued). */
qldpc_status qldpc_server_submit(qldpc_server srv, int32_t code_id, int32_t decoder, int32_t nshots,
                                 const uint32_t *host_syndromes, const float *host_priors,
                                 uint32_t *host_errors, uint8_t *host_converged, uint8_t *host_iters,
                                 uint64_t req_id);

/* Moves up to `max` completions (oldest first) to `out`; NOT_READY when none. */
qldpc_status qldpc_server_poll(qldpc_server srv, qldpc_completion *out, int32_t max, int32_t *n_out);

/* Stops admitting, waits for the micro-batches on the device, frees all. */
qldpc_status qldpc_server_destroy(qldpc_server srv);

typedef struct {
    double rate_shots_per_s;          /* offered load                               */
    double duration_s;                /* length of the arrival process              */
    uint64_t seed;
    double p_single;                  /* P(request = 1 shot), else 64 shots         */
    double p_neural;                  /* P(neural decoder) where weights exist      */
    int32_t ncodes;                   /* = the server's code count                  */
    const uint32_t *const *pool_syn;  /* per code: host [pool][ceil(m/32)]          */
    const float *const *pool_prior;   /* per code: host [pool]                      */
    const int32_t *pool_size;         /* per code, >= 64                            */
} qldpc_loadgen_config;

typedef struct {
    int64_t requests, shots, rejected;
    double wall_s, offered_s;
    double p50_us, p99_us, p999_us, mean_us, max_us;  /* from scheduled arrival      */
    double shots_per_s;
} qldpc_loadgen_result;

/* Drives an idle server with an open-loop Poisson stream of requests drawn
 * from host pools (uniform code, size 1 or 64, plain or neural) and
 * measures each latency from its scheduled arrival to its completion.
 * lat_us (nullable) receives up to lat_cap per-request latencies. */
qldpc_status qldpc_server_loadgen(qldpc_server srv, const qldpc_loadgen_config *cfg,
                                  qldpc_loadgen_result *result, double *lat_us, int64_t lat_cap);

/* Host helper: int8 Q4 prior clamp(round-half-away-from-zero(16 * llr),
 * -127, 127) for `count` values (host arrays): the quantisation of the
 * 8-bit integer format (Table 1, reduced-precision data types; Section 3). */
qldpc_status qldpc_quantize_prior(const float *llr, int8_t *out, int64_t count);

/* Host helper: int16 Q8 prior clamp(round-half-away-from-zero(256 * llr),
 * -32767, 32767) for `count` values (host arrays): the quantisation of the
 * 16-bit integer format (Table 1; Section 3). */
qldpc_status qldpc_quantize_prior_q8(const float *llr, int16_t *out, int64_t count);

#ifdef __cplusplus
}
#endif

#endif /* QLDPC_H */
