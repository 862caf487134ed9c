/*
 * ldpc.h -- C ABI of libldpc.so: syndrome-form flooding sum-product decoding of
 * quasi-cyclic (QC) LDPC codes on one MI355X (gfx950), in hand-written HIP.
 *
 * Method: Algorithm 1 of Milicevic et al., "Key Reconciliation with LDPC Codes
 * for Long-Distance Quantum Cryptography" (Sec. III-D), applied to the QC
 * codes of Sec. III-C, in the syndrome (Slepian-Wolf, Sec. II-C.4) form: every
 * check c carries a target bit s_c, multiplies its outgoing messages by
 * (-1)^{s_c}, and a frame stops when its hard decisions x satisfy H x = s.
 *
 * Conventions shared by every entry point:
 *  - Status: every function returning int returns LDPC_OK (0) or a negative
 *    LDPC_E* code; nothing throws across the ABI.  ldpc_last_error() gives a
 *    human-readable detail of the calling thread's last failure.
 *  - Memory: pointers named "device" must point into HIP device memory of the
 *    device the code was created on (e.g. torch CUDA tensors); "host" pointers
 *    are ordinary host memory.  The caller owns every data buffer and the
 *    workspace; the library owns the code handle, its small device tables, two
 *    streams of its own with their events, and up to 4 decode graphs.  Inside
 *    ldpc_decode_batch the only allocation is the one the HIP runtime makes
 *    when a repeated small decode is captured into a graph (see
 *    ldpc_decode_opts.graphs; graphs = 1 avoids it, and
 *    ldpc_decode_batch_noalloc never makes graphs).
 *  - Streams: decode and syndrome calls are asynchronous on the given
 *    hipStream_t (NULL = the null stream); outputs are valid after the caller
 *    synchronises that stream.  Launch errors are reported at enqueue; faults
 *    inside kernels surface at the caller's synchronisation.
 *  - Threads: a code handle is immutable after creation and may be used from
 *    several host threads and streams at once, each call with its own
 *    workspace and output buffers.
 */
#ifndef LDPC_H
#define LDPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    LDPC_OK = 0,
    LDPC_EINVAL = -1,       /* bad argument (null pointer, size, range)          */
    LDPC_ENOMEM = -2,       /* host or device allocation failed at code creation */
    LDPC_EDEVICE = -3,      /* HIP runtime error, or wrong current device        */
    LDPC_EUNSUPPORTED = -4, /* valid code the kernels do not handle (degree cap) */
    LDPC_EWORKSPACE = -5    /* workspace null, too small or misaligned           */
};

/* Largest check (row) degree the check-update kernel handles. */
#define LDPC_MAX_ROW_DEGREE 16

typedef struct ldpc_code ldpc_code;

typedef struct {
    int32_t n;              /* code length nb*Z                                  */
    int32_t m;              /* number of checks mb*Z                             */
    int32_t Z;              /* lifting size (circulant order)                    */
    int32_t mb, nb;         /* base matrix shape                                 */
    int32_t blocks;         /* non-zero base entries                             */
    int64_t edges;          /* Tanner-graph edges, blocks*Z                      */
    int64_t state_edges;    /* edges on columns of degree >= 2 (stored messages) */
    int32_t core_cols;      /* base columns of degree >= 2                       */
    int32_t deg1_cols;      /* base columns of degree 1                          */
    int32_t deg0_cols;      /* base columns of degree 0                          */
    int32_t max_row_degree; /* largest number of non-zero blocks in a base row   */
    int64_t owned_edges;    /* edges of owner blocks: per row with two core blocks
                               and one degree-1 block, the core block whose
                               messages the check pass sums per owner group      */
    int32_t owner_groups;   /* owner groups (up to 12 such rows sharing an owner
                               core column); the variable pass reads one partial
                               sum per group instead of the group's messages     */
} ldpc_code_info_t;

/*
 * Create a QC code from its base matrix (Sec. III-C): each non-zero entry is a
 * Z x Z circulant permutation, the identity with every row cyclically shifted
 * right by the entry (0-based; the paper's I_i is shift i-1), so row a of
 * block (r, c) joins check r*Z + a to variable c*Z + ((a + shift) mod Z).
 *   mb, nb  base shape, >= 1
 *   base    host, mb*nb int32 row-major; -1 = zero block, else shift in [0, Z)
 *   Z       lifting size, 1 <= Z; n = nb*Z, m = mb*Z, the stored edges and twice
 *           the core variables (+ padding) of one frame must each stay below
 *           2^30 - 1024 (32-bit byte offsets), else LDPC_EINVAL
 *   out     host; receives the handle (set to NULL on failure)
 * Builds the block tables (row lists, column lists, degree classes) and copies
 * them to the current HIP device, to which the handle is bound.
 * Errors: LDPC_EINVAL (shape, shift range, null), LDPC_EUNSUPPORTED (a row of
 * degree > LDPC_MAX_ROW_DEGREE, a row with no block, or more than 65535 base
 * rows or base columns), LDPC_ENOMEM, LDPC_EDEVICE.
 */
int ldpc_code_create(int32_t mb, int32_t nb, const int32_t *base, int32_t Z, ldpc_code **out);

/* Release a handle and its device tables; NULL is ignored.  The caller must
 * ensure no enqueued call using the handle is still running. */
void ldpc_code_destroy(ldpc_code *code);

/* Sizes and degree classes of a code.  out: host.  LDPC_EINVAL on null. */
int ldpc_code_info(const ldpc_code *code, ldpc_code_info_t *out);

typedef struct {
    int32_t early_stop;      /* 1: a frame stops at the first checked iteration whose
                                decisions satisfy H x = s (Alg. 1 Step 4); 0: every
                                frame runs max_iters iterations                      */
    int32_t check_from_iter; /* the check runs only at iterations t >= this value (the
                                paper's early-termination lookup, Sec. IV-A); 0 = from
                                t = 0, i.e. also on the channel decisions            */
    int32_t msg_fp16;        /* 1: check-to-variable messages stored as IEEE half;
                                all arithmetic and sums stay in float32             */
    int32_t checks_per_thread; /* schedule of the check kernel: checks of one base
                                row per thread, 1, 2 or 4 (0 = library default:
                                1 for Z <= 256, else 4);
                                a block row's Z checks take ceil(Z / (256 *
                                checks_per_thread)) workgroups.  Results do not
                                depend on it                                      */
    float *llr_out;          /* optional device [F][n]: posterior L_v at exit      */
    void **timing_events;    /* optional host array of caller-created hipEvent_t
                                handles, recorded by the launches of the iteration
                                kernels themselves (start and end of execution):
                                events 4(t-1), 4(t-1)+1 at the start and end of the
                                check pass of iteration t, 4(t-1)+2, 4(t-1)+3 at
                                the start and end of its variable pass            */
    int32_t n_timing_events; /* >= 4*max_iters when timing_events is set          */
    int32_t schedule;        /* LDPC_SCHEDULE_*: how the iterations are launched;
                                results are identical on every schedule           */
    int32_t streams;         /* per-iteration launches only (LDPC_SCHEDULE_LAUNCHES):
                                0 = library choice: F >= 2 frames run as two halves
                                on two streams when one iteration visits at least
                                F * (stored + degree-1 blocks) * Z = 24,000,000
                                edges (16,000,000 with msg_fp16), else one stream;
                                1 = one stream; 2 = two halves whenever F >= 2.
                                Ignored with timing_events (one stream).  Results
                                are identical either way                          */
    int32_t graphs;          /* per-iteration launches on one stream, at most
                                F * (stored + degree-1 blocks) * Z = 1,000,000
                                edge visits per iteration (where the host's
                                launches can bound a decode): 0 = library
                                choice: a call that repeats an earlier call's F,
                                max_iters, options and pointers is captured into
                                a HIP graph at its second occurrence and
                                replayed from the third (the code handle keeps 4
                                such graphs, least recently used replaced); not
                                with timing_events, not while `stream` is itself
                                being captured, never in
                                ldpc_decode_batch_noalloc; 1 = launch the
                                kernels one by one every time.  Results are
                                identical either way                             */
} ldpc_decode_opts;

/*
 * Decode schedules.  Both run the flooding schedule of Alg. 1 with the same
 * arithmetic in the same order, so outputs are bit-identical.
 *  LAUNCHES  two launches per iteration (check pass, variable pass) over all
 *            frames, state in HBM: any code, posteriors and timing events.
 *  RESIDENT  one launch for the whole decode, one 1024-thread workgroup per
 *            frame holding the frame's messages, core totals and bit arrays in
 *            LDS: for small liftings, where the per-iteration launches are
 *            latency-bound.  Needs llr_out and timing_events unset and the
 *            frame's state within one workgroup's LDS (160 KB on MI355X:
 *            state edges * (4 or 2 bytes) + core variables * 16 + bit arrays).
 *  SPLIT     one cooperative launch for the whole decode with up to 4
 *            co-resident workgroups per frame: the frame's messages in device
 *            memory (two buffers, by iteration parity), every workgroup holding
 *            the frame's core totals in LDS, one barrier across a frame's
 *            workgroups per iteration: for a few frames of a small code, where
 *            one workgroup per frame leaves most of the chip idle.  Needs
 *            llr_out and timing_events unset, at most 256 frames, and a frame
 *            state of at most 160 KB (as RESIDENT).
 *  AUTO      RESIDENT when it is possible and a cost model of both, fitted
 *            to measurements, favours it (many frames of a small code), else
 *            LAUNCHES.
 */
enum {
    LDPC_SCHEDULE_AUTO = 0,
    LDPC_SCHEDULE_LAUNCHES = 1,
    LDPC_SCHEDULE_RESIDENT = 2,
    LDPC_SCHEDULE_SPLIT = 3
};

/* Fill opts with the defaults {early_stop=1, check_from_iter=0, msg_fp16=0,
 * checks_per_thread=0, llr_out=NULL, timing_events=NULL, n_timing_events=0,
 * schedule=LDPC_SCHEDULE_AUTO, streams=0, graphs=0}. */
void ldpc_decode_opts_init(ldpc_decode_opts *opts);

/* The schedule (LDPC_SCHEDULE_LAUNCHES, _RESIDENT or _SPLIT) that
 * ldpc_decode_batch runs for F frames with these options (NULL = defaults).
 *   schedule_out  host
 * Errors: LDPC_EINVAL (null, F outside [1, 65535], schedule out of range),
 * LDPC_EUNSUPPORTED (RESIDENT or SPLIT requested where it is not possible). */
int ldpc_decode_schedule(const ldpc_code *code, int32_t F, const ldpc_decode_opts *opts,
                         int32_t *schedule_out);

/* Workspace bytes ldpc_decode_batch needs for F frames and max_iters iterations
 * with these options (NULL = defaults).  Returns 0 on an invalid argument. */
size_t ldpc_workspace_bytes(const ldpc_code *code, int32_t F, int32_t max_iters,
                            const ldpc_decode_opts *opts);

/*
 * Decode F frames (Alg. 1, Steps 2-4, flooding schedule, syndrome form).
 *   llr        device [F][n] float32: channel LLR Q_v = ln P(x_v=0)/P(x_v=1)
 *              (Step 1 is done by the caller), frame-major, v = c*Z + j
 *   syndrome   device [F][m] uint8: target bits s_c in {0,1}, c = r*Z + a
 *   max_iters  T >= 0: most iterations per frame
 *   bits_out   device [F][n] uint8: hard decisions x_v = [L_v < 0] at exit
 *   iters_out  device [F] int32: iterations completed at exit; a frame whose
 *              channel decisions already satisfy H x = s reports 0
 *   converged_out device [F] uint8: 1 iff H x = s holds for bits_out
 *   opts       host, NULL = defaults (see ldpc_decode_opts)
 *   workspace  device, >= ldpc_workspace_bytes(code, F, max_iters, opts) bytes,
 *              256-byte aligned; its contents on entry are ignored
 *   stream     hipStream_t or NULL
 * Messages are clamped through the Phi argument range [1e-7, 30].  Frames are
 * independent: frame f's outputs depend only on frame f's inputs, bit for bit,
 * whatever F and the other frames are.  On the per-iteration launches, a
 * decode that opts.streams sends to two streams (by default F >= 2 frames with
 * enough edge visits per iteration, and no timing_events) runs as two halves,
 * the second on a stream the code handle owns, forked from and joined back into
 * `stream` by events: the decode stays ordered on `stream` like any other work
 * there (and can be captured into a graph from it); calls with one code handle
 * from several host threads are safe, and their second halves share that
 * stream.  Two streams double the launches per iteration, so they pay only
 * where each half's iteration outlasts the host's launch rate.
 * Errors: LDPC_EINVAL (F < 1, max_iters < 0, check_from_iter < 0, null
 * pointer, checks_per_thread not 0/1/2/4, schedule out of range, streams not
 * 0/1/2, graphs not 0/1, too few
 * timing events), LDPC_EUNSUPPORTED (RESIDENT requested where it is not
 * possible), LDPC_EWORKSPACE, LDPC_EDEVICE (current device is not the code's
 * device, or a launch failed).
 */
int ldpc_decode_batch(const ldpc_code *code, int32_t F,
                      const float *llr, const uint8_t *syndrome, int32_t max_iters,
                      uint8_t *bits_out, int32_t *iters_out, uint8_t *converged_out,
                      const ldpc_decode_opts *opts, void *workspace, size_t workspace_bytes,
                      void *stream);

/*
 * ldpc_decode_batch for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, semantics and results as ldpc_decode_batch,
 * without the workspace: the decode state lives in a fixed scratch region
 * inside the library, one per device, of LDPC_NOALLOC_SCRATCH_BYTES (part of
 * the library's device code: the loader places it, and each device the
 * library runs on holds it until the process ends).  Its address is looked
 * up at the first ldpc_code_create on a device (again at the first call
 * here if that failed).  This call allocates and frees nothing, host or
 * device.
 * Limit: ldpc_workspace_bytes(code, F, max_iters, opts) must not exceed
 * LDPC_NOALLOC_SCRATCH_BYTES, else LDPC_EWORKSPACE and nothing is enqueued
 * (e.g. up to 4 frames of the n = 1,000,050 rate-0.02 code, any frame count
 * up to about 500 of n = 9,600).
 * Concurrency: all calls on one device share that device's region, which
 * keeps the last call's contents (a decode reads only what it has written
 * itself first).  Calls whose work overlaps on the device -- on different
 * streams, or from several host threads -- race on it and give undefined
 * results; serialise them (one stream, or events between streams).
 * Errors: as ldpc_decode_batch (LDPC_EWORKSPACE for the size limit;
 * LDPC_EDEVICE if the region's address cannot be found).
 */
#define LDPC_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int ldpc_decode_batch_noalloc(const ldpc_code *code, int32_t F,
                              const float *llr, const uint8_t *syndrome, int32_t max_iters,
                              uint8_t *bits_out, int32_t *iters_out, uint8_t *converged_out,
                              const ldpc_decode_opts *opts, void *stream);

/*
 * s = H x mod 2 for F words: the parity check of Alg. 1 Step 4 (Sec. III-D),
 * on the QC lifting of Sec. III-C, as a stand-alone call (Bob's syndrome of his
 * key bits in syndrome reconciliation, Sec. II-C.4).
 *   bits     device [F][n] uint8 (only bit 0 of each byte is used)
 *   syn_out  device [F][m] uint8, values 0/1
 * Errors: LDPC_EINVAL, LDPC_EDEVICE.
 */
int ldpc_syndrome(const ldpc_code *code, int32_t F, const uint8_t *bits, uint8_t *syn_out,
                  void *stream);

/*
 * Multi-dimensional reverse reconciliation front-end (Sec. II-C.3): channel
 * LLRs from Alice's samples X and Bob's public message M.
 * Frames are cut into d-tuples, d in {1, 2, 4, 8} (reals, complex numbers,
 * quaternions, octonions, multiplied by Cayley-Dickson doubling:
 * (a, b)(c, e) = (a c - conj(e) b, e a + b conj(c))).  Per tuple Alice forms
 * R = M X^{-1}; the noise of R has per-coordinate variance d sigma2 / |X|^2,
 * so the LLR of coordinate i is 2 R_i |X|^2 / (d sigma2) = 2 (M conj(X))_i / (d sigma2).
 *   d        1, 2, 4 or 8
 *   F, n     frames and code length; every frame holds n_d = d * ceil(n / d)
 *            samples (the last tuple is padded)
 *   x, m     device [F][n_d] float32: Alice's samples and Bob's message
 *   sigma2   channel noise variance sigma_Z^2 (SNR = 1 / sigma2), > 0
 *   llr_out  device [F][n] float32: LLRs of the first n coordinates, ready for
 *            ldpc_decode_batch
 * Errors: LDPC_EINVAL (d, F, n, sigma2 or a null pointer), LDPC_EDEVICE.
 */
int ldpc_reconciliation_llr(int32_t d, int32_t F, int32_t n, const float *x, const float *m,
                            float sigma2, float *llr_out, void *stream);

/*
 * Bob's side of the same scheme (Sec. II-C.3): M = U Y per d-tuple, with
 * U_i = (-1)^{c_i}; coordinates of the padded last tuple take c = 0.
 *   bits   device [F][n] uint8 key bits c (bit 0 used)
 *   y      device [F][n_d] float32 Bob's samples
 *   m_out  device [F][n_d] float32
 * Errors: LDPC_EINVAL, LDPC_EDEVICE.
 */
int ldpc_reconciliation_message(int32_t d, int32_t F, int32_t n, const uint8_t *bits,
                                const float *y, float *m_out, void *stream);

/*
 * Multi-request engine: iteration-level scheduling of decode requests of mixed
 * codes on one GPU stream (continuous batching).  Each engine step runs one
 * flooding iteration (Alg. 1, Steps 2-4) of every admitted request in a single
 * check launch and a single variable launch that cover all of them; a request
 * submitted while others decode is admitted at the next step once a slot is
 * free and its decode state fits the HBM budget, and leaves as soon as all its
 * frames have stopped (or after its last iteration).  Per frame the engine runs
 * exactly the kernels of ldpc_decode_batch in the same order, so every request's
 * outputs are bit-identical to decoding it alone with the same options.
 *
 * The engine owns its device memory: a cap of hbm_budget_bytes on the state of
 * admitted requests, taken from the device in chunks of up to 1 GiB when first
 * needed.  The chunks together never exceed hbm_budget_bytes: a request that
 * fits the budget but no free range waits in the queue, and chunks with
 * nothing in flight are returned to the device when a request needs the room;
 * the rest are kept until ldpc_engine_destroy.  Calls on one engine must not run
 * concurrently.  Supported codes: every base row of degree <= 6 with at most one
 * degree-1 block (the multi-edge families); others give LDPC_EUNSUPPORTED.
 */
typedef struct ldpc_engine ldpc_engine;

typedef struct {
    size_t hbm_budget_bytes; /* most device bytes of decode state admitted at once   */
    int32_t max_slots;       /* most requests in flight, 1..64                        */
    int32_t msg_fp16;        /* 1: messages stored as IEEE half (as ldpc_decode_opts)  */
    int32_t early_stop;      /* as ldpc_decode_opts.early_stop                         */
    int32_t checks_per_thread; /* check-kernel schedule as in ldpc_decode_opts      */
    void *stream;            /* hipStream_t for all engine work; NULL = null stream    */
    int64_t max_step_edges;  /* latency cap: most edge visits per engine step, the sum
                                over admitted requests of frames x Tanner-graph edges
                                (blocks * Z); a step's time grows with it, and so does
                                every admitted request's latency (iterations x step
                                time).  0 = no cap.  A request above the cap is still
                                admitted when nothing else is in flight.           */
} ldpc_engine_config;

/* Create an engine on the current device.  Errors: LDPC_EINVAL (null, budget 0,
 * max_slots outside 1..64, checks_per_thread not 0/1/2/4), LDPC_ENOMEM, LDPC_EDEVICE. */
int ldpc_engine_create(const ldpc_engine_config *cfg, ldpc_engine **out);

/* Wait for the engine's stream, free its memory; queued requests are dropped.
 * NULL is ignored. */
void ldpc_engine_destroy(ldpc_engine *engine);

/* Device bytes of decode state one request takes from the budget. */
size_t ldpc_engine_request_bytes(const ldpc_code *code, int32_t F, int32_t max_iters,
                                 int32_t msg_fp16);

/*
 * Queue a request of F frames (pointers as in ldpc_decode_batch; device
 * buffers owned by the caller, which must keep them, and the code, alive until
 * the ticket is reported by ldpc_engine_poll).  Nothing is launched here.
 *   ticket_out  host; receives an id > 0 that ldpc_engine_poll reports when the
 *               request's outputs are written
 * Errors: LDPC_EINVAL (argument, or a request larger than the whole budget),
 * LDPC_EUNSUPPORTED (code shape), LDPC_EDEVICE (code on another device).
 */
int ldpc_engine_submit(ldpc_engine *engine, const ldpc_code *code, int32_t F, const float *llr,
                       const uint8_t *syndrome, int32_t max_iters, uint8_t *bits_out,
                       int32_t *iters_out, uint8_t *converged_out, int64_t *ticket_out);

/*
 * One engine step on the engine's stream: retire requests whose frames have all
 * stopped (read-out enqueued), admit queued requests in arrival order while a slot
 * and budget are free, then one iteration of every active request.  Asynchronous.
 *   active_out, queued_out  host, nullable: requests in flight / still queued
 * Errors: LDPC_EDEVICE.
 */
int ldpc_engine_step(ldpc_engine *engine, int32_t *active_out, int32_t *queued_out);

/* Report up to `capacity` tickets whose outputs are complete (each once).
 *   tickets_out host [capacity]; count_out host.  Errors: LDPC_EINVAL. */
int ldpc_engine_poll(ldpc_engine *engine, int64_t *tickets_out, int32_t capacity,
                     int32_t *count_out);

/* Static English text for a status code. */
const char *ldpc_status_string(int status);

/* Detail of the calling thread's most recent failure ("" if none). */
const char *ldpc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LDPC_H */
