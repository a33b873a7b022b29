/*
 * soft.h -- C ABI of the MI355X generalized-stabilizer shot sampler.
 *
 * The library samples noisy Clifford+T circuits with mid-circuit
 * measurements and postselection in the generalized stabilizer (GS)
 * formalism of arXiv 2512.23037: every shot is an independent pure state
 * (v, B(S, D)) -- a stabilizer/destabilizer tableau plus a sparse coefficient
 * vector over destabilizer strings alpha (Sec. II-C, Definition 1, Eq. 3).
 * Cliffords update the tableau, T/T-dagger split coefficients (Eqs. 1-2 with
 * the Pauli-on-basis identity Eq. 4, Theorem 1 part 3), Pauli measurements
 * collapse and renormalise (Theorem 1 part 2), and Pauli noise is drawn per
 * shot (Sec. II-C, pure-state simulation model; uniform depolarizing noise of
 * Sec. III).  All shots of a run execute on one GPU in one persistent,
 * work-stealing kernel.
 *
 * General conventions
 *  - Every call returns 0 on success or a negative SOFT_E* code; the message
 *    of the last failure is available from soft_last_error().  No C++
 *    exception or abort crosses this boundary.
 *  - "_dev" pointers are device pointers (hipMalloc / torch CUDA tensors on
 *    ROCm); the caller owns them and the library never frees them.  Other
 *    pointers are host pointers, owned by the caller, read or written only
 *    during the call.
 *  - A context is not thread-safe; use one per thread.
 *  - Qubit counts are limited to n <= 64.
 */
#ifndef SOFT_H
#define SOFT_H
#include <stddef.h>
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

enum {
    SOFT_OK = 0,
    SOFT_EINVAL = -1,       /* bad argument                                  */
    SOFT_EPARSE = -2,       /* circuit text rejected ("line N: ..." message) */
    SOFT_ECAPACITY = -3,    /* a size limit was exceeded                     */
    SOFT_EDEVICE = -4,      /* HIP runtime error (message has the HIP text)  */
    SOFT_ESTATE = -5,       /* call order (e.g. run before load_circuit)     */
    SOFT_EUNSUPPORTED = -6  /* request outside what the library implements   */
};

/* Per-shot status (soft_run's status_dev). */
enum { SOFT_PASSED = 0, SOFT_DISCARDED = 1, SOFT_OVERFLOW = 2, SOFT_NUMERIC = 3 };

typedef struct soft_ctx soft_ctx;

/* Uniform depolarizing noise model (Sec. III; the per-shot Pauli draws of the
 * pure-state simulation model of Sec. II-C): every probability in [0, 1].
 * p1: DEP1 after each single-qubit gate (H S SDG X Y Z T TDG); p2: DEP2 after
 * each CX/CZ; p_idle: DEP1 on every qubit untouched since the previous TICK,
 * inserted at the TICK; p_meas: X flip before each M; p_reset: X flip after
 * each R; p_mpp: classical flip of each MPP result.  DEP1 applies X, Y or Z
 * with p/3 each; DEP2 one of the 15 non-identity two-qubit Paulis, p/15 each. */
typedef struct {
    double p1, p2, p_idle, p_meas, p_reset, p_mpp;
} soft_noise;

/* Aggregates of the last soft_run: the small statistics the host reads back
 * (Sec. IV-B) -- pass / discard counts and the logical-error count behind the
 * discard rate and logical error rate of Sec. V, plus the work and support
 * sizes |v| (Definition 1) of the shots. */
typedef struct {
    uint64_t shots, passed, discarded, overflow, numeric;
    uint64_t logical_errors;     /* passed shots with a nonzero observable   */
    uint64_t entries_t;          /* coefficient entries written by T/T-dagger */
    uint64_t entries_m;          /* coefficient entries read by measurements */
    uint64_t noise_slots;        /* noise words drawn (256 per Philox refill of a wave) */
    uint64_t events;             /* T/T-dagger and measurements executed      */
    uint64_t support_hist[16];   /* shots by floor(log2(max |v|)), last bin 15+: the
                                    largest support the kernel held (the speculative
                                    lists may hold smaller ones than the circuit's
                                    gate order; with speculation off they are the
                                    circuit order's; a shot that ended with a deferred
                                    T run skipped counts the supports it computed) */
    double max_norm_dev;         /* max over shots of |sum |v|^2 - 1| at the end */
    uint64_t restarts;           /* shots re-run on the full event list: the speculative
                                    list's span truncation found amplitude left (noise
                                    broke a T / T-dagger cancellation) */
    uint64_t prefix_shots;       /* attempts that started from a checkpoint of the noiseless
                                    trajectory (soft_set_shared_prefix); the work fields
                                    above count only the work run */
    uint64_t redo_shots;         /* deferred T runs applied late because an event needed the
                                    tile, and attempts run again to keep a state
                                    (soft_set_deferred_t) */
} soft_counters;

/* Create a context on HIP device `hip_device` (made current for the call):
 * the device memory that holds the compiled circuit, the counters and the
 * per-shot states of Sec. IV-B is owned by it.  *out receives the handle
 * (NULL on failure).  EINVAL: no such device or out == NULL; EDEVICE: a HIP
 * call failed (message via soft_last_error(NULL)). */
int soft_create(soft_ctx **out, int hip_device);

/* Free everything the context owns (the device memory of Sec. IV-B it
 * allocated); waits for its last run first.  NULL is allowed. */
void soft_destroy(soft_ctx *ctx);

/* Message of the last failed call on ctx ("" if none); valid until the next
 * call on ctx.  With ctx == NULL, the message of the last failed
 * soft_create on this thread.  Error reporting of this boundary only: no
 * operation of the paper corresponds to it. */
const char *soft_last_error(const soft_ctx *ctx);

/* Load circuit text (len bytes, need not be NUL-terminated; copied): a
 * Clifford+T circuit with mid-circuit measurements and postselection, the
 * problem of Sec. II-C, with the operations of the MSC circuits of Sec. III
 * (Table II counts them).  One op per line, '#' starts a comment, first line
 * "QUBITS n":
 *   H q | S q | SDG q | X q | Y q | Z q | H_XY q | H_NXY q | T q | TDG q |
 *   CX c t | CZ a b | M q | R q | MX q | RX q | MR q | MRX q |
 *   MPP P0*P1*...  (factors X3, Y0, Z7; distinct qubits) |
 *   CCZ a b c | CCX a b t | CS a b | CSDG a b | CPHASE theta a b | RZ theta q |
 *   DIAG k q_0..q_{k-1} phi_0..phi_{2^k-1}  (k = 1..3) |
 *   XIF r q | YIF r q | ZIF r q | IF r0,r1.. GATE args | IF r0&r1&.. GATE args |
 *   DEP1 p q... | DEP2 p a b [a b...] | XERR p q... | ZERR p q... | TICK |
 *   DETECTOR e r... | OBSERVABLE e r...
 * M and MPP append to the measurement record; R measures Z and flips back
 * to |0> (not recorded); MX / RX are the X-basis forms, MR / MRX record and
 * reset.  The diagonal gates multiply basis state x of their qubits (bit j
 * of x = j-th listed qubit) by e^{i phi_x}: CCZ phi = pi at x = 7, CCX =
 * H_t CCZ H_t, CS / CSDG phi = +-pi/2 at x = 3, CPHASE phi = theta at
 * x = 3, RZ theta = exp(-i theta Z / 2), DIAG the listed phases (radians);
 * each runs in one pass as the sum of its Z-strings (the expansion used in
 * Proposition 1's proof, each term acting by Eq. 4).  XIF/YIF/ZIF r q apply
 * the Pauli to q when record bit r is 1.  IF applies GATE when the XOR of
 * the listed record bits (',') or their AND ('&') is 1: the corrections of
 * gate teleportation, which the conclusion names as the next extension.
 * GATE is X / Y / Z q (sign flips) or a diagonal gate -- S, SDG, T, TDG q,
 * CZ a b or any of the diagonal gates above -- which acts on the
 * coefficients by its Z-string expansion in every shot where it fires (the
 * coefficient span grows in every shot; CCX keeps its H pair unconditional).
 * IF takes no model noise.  DETECTOR ends the shot as
 * DISCARDED when e ^ XOR(record bits r...) != 0; OBSERVABLE stores that
 * parity as an observable bit.  Op indices (used by abort_op) count op lines
 * from 0.
 * EPARSE on malformed text; ECAPACITY when the circuit's coefficient span
 * exceeds the largest tile the library supports. */
int soft_load_circuit(soft_ctx *ctx, const char *text, size_t len);

/* Set the noise model inserted around the circuit's ops (default: none):
 * the uniform depolarizing model of Sec. III, sampled per shot as in the
 * pure-state simulation model of Sec. II-C.  EINVAL: a probability outside
 * [0, 1]; ESTATE while a mixture is loaded (each variant has its own model). */
int soft_load_noise(soft_ctx *ctx, const soft_noise *model);

/* Load a mixture: n_variants (1..64) circuits, each with its own noise model,
 * sampled together in one launch by soft_run (the batching of many shots per
 * launch of Sec. IV-B, across circuits and noise rates as in the noise scans
 * of Sec. V).  Variant v owns the global
 * shot indices [shot_ends[v-1], shot_ends[v]) (shot_ends[-1] = 0; the ends
 * strictly increase), and a shot of variant v has the same result as the
 * same shot index of a context holding only that circuit and model.
 * texts[v] (lens[v] bytes, copied) use the soft_load_circuit format;
 * models[v] as soft_load_noise.  On failure the message names the variant
 * and the previous contents stay loaded.  soft_load_circuit returns the
 * context to a single circuit.  Explicit uniforms (soft_set_uniforms) are
 * not available for mixtures (EUNSUPPORTED at soft_run). */
int soft_load_mixture(soft_ctx *ctx, uint32_t n_variants, const char *const *texts, const size_t *lens,
                      const soft_noise *models, const uint64_t *shot_ends);

/* Key of the per-shot random streams that choose each shot's noise Paulis
 * and measurement branches (the pure-state simulation model of Sec. II-C;
 * the paper seeds shots by hashing, here Philox4x32-10 of Salmon et al.,
 * SC'11, keyed by seed and counted by shot index).  Noise
 * slot s of shot t uses word s%4 of the block at counter
 * (s/4, t low 32 bits, t high 32 bits, 0); measurement slot s uses stream 1.
 * A noise slot hits iff word < floor(p * 2^32); a measurement's outcome is
 * +1 (record bit 0) iff (word + 1/2) 2^-32 < P(+1). */
int soft_set_rng(soft_ctx *ctx, uint64_t seed);

/* Replace Philox by explicit per-shot words (test mode, for the step-by-step
 * validation of Sec. V-B: both sides see identical draws): words_dev holds
 * n_shots rows of noise_slots + meas_slots words, row i used by the shot at
 * position i of the next soft_run.  The counts must match the loaded circuit
 * and noise model.  words_dev == NULL returns to Philox. */
int soft_set_uniforms(soft_ctx *ctx, const uint32_t *words_dev, uint64_t n_shots,
                      uint32_t noise_slots, uint32_t meas_slots);

/* Coefficient precision of the coefficients v of Definition 1 / Eq. 3:
 * 64 (FP64, the paper's precision; default) or 32 (FP32 complex storage and
 * products; outcome probabilities, renormalisation and norms stay FP64).
 * EINVAL for any other value. */
int soft_set_precision(soft_ctx *ctx, int coeff_bits);

/* Pruning threshold tau: after every T and measurement, coefficients with
 * |v|^2 < tau^2 sum|v|^2 are dropped, so that the support of Definition 1
 * (the nonzero entries) keeps the bounds of Theorem 1 when T and T-dagger
 * cancel up to rounding (the paper is silent on pruning).  Default 1e-12
 * (FP64), 1e-6 (FP32); tau < 0 restores the default; EINVAL for tau >= 1. */
int soft_set_prune(soft_ctx *ctx, double tau);

/* Fixed capacities and launch shape (Sec. IV-B: per-shot capacity with an
 * overflow flag).  support_cap: a shot whose support |v| exceeds it after a T
 * ends as OVERFLOW (0 = no cap).  waves_per_block (1..4), blocks_per_cu
 * (1..32), grab (1..64, consecutive shots a wave takes per steal; their
 * outputs are written together): launch shape, 0 = the autotuned or default
 * value.  One wave runs one shot at a time, so shots in flight per block =
 * waves_per_block; the coefficient tile is not a free size (it holds the
 * circuit's whole span, 2^k_max entries) -- where it lives is
 * soft_set_tile_memory.  EINVAL for values out of range. */
int soft_set_caps(soft_ctx *ctx, uint32_t support_cap, uint32_t waves_per_block,
                  uint32_t blocks_per_cu, uint32_t grab);

/* Speculative span truncation (on by default; it rests on the T-layer
 * structure of Sec. IV-A, Observations 1-3 and Proposition 1): where every T
 * of a run since
 * a checkpoint meets its inverse on the same qubit with nothing in between
 * that fails to commute with its Z (T and T-dagger layers around commuting
 * check rounds), the product of the pairs is the identity, so a shot whose
 * noise left the pairs intact has its coefficients back on the checkpoint's
 * span.  The compiler then emits a second event list that truncates the span
 * there, and step by step as the inverse layer proceeds: it runs the
 * commuting T gates of a layer in another order (cheapest first in a layer
 * that opens, latest-opened first in one that closes; each gate's noise stays
 * after it).  On that list, runs of such T gates on spans of at most 6
 * coordinates with nothing between them run as one pass, with the same
 * arithmetic and the same support after every gate.  The kernel verifies
 * that the dropped coordinates hold exact zeros and otherwise restarts the
 * shot on the full list (counted in
 * soft_counters.restarts).  Records, statuses, abort ops and observables are
 * the full list's either way (coefficients up to rounding order); the support
 * histogram is that of the supports the kernel held, which the other gate
 * order can make smaller.  A run with a support cap (soft_set_caps) uses the
 * full list only, so that the cap sees the circuit order's supports.  on = 0
 * runs the full list only. */
int soft_set_speculation(soft_ctx *ctx, int on);

/* How noise hits are drawn (the same distribution either way: every noise
 * location hit independently with its probability, its Pauli uniform over the
 * channel's list, as the uniform depolarizing noise of Sec. III asks).  mode 0 (default): one Philox word of stream 0 per noise
 * location, hit iff word < floor(p 2^32).  mode 1 (gap sampling): candidate
 * locations form a Bernoulli(p_max) process, p_max the largest location
 * probability of the circuit; the gap to the next candidate comes from one
 * word of stream 2 and the gap table floor((1 - p_max)^g 2^32), and a second
 * word accepts the candidate with probability floor(p / p_max 2^32) 2^-32,
 * its Pauli picked from that word.  Mode 1 draws about 2 n p_max words per
 * shot instead of n.  Explicit words (soft_set_words) always use mode 0.
 * Returns SOFT_EINVAL for another mode. */
int soft_set_noise_mode(soft_ctx *ctx, int mode);

/* Checkpoints of the noiseless trajectory (default on).  Up to the first
 * measurement with a random outcome, every event of a circuit is
 * deterministic in a shot that no noise has hit (Sec. II-C's model: the
 * noise Paulis are the only per-shot randomness before it), so every such
 * shot is in the same state at each point there.  The compiler marks up to 16
 * checkpoints per event list (around the check rounds, and before the first
 * random measurement or the end); each run first computes the noiseless
 * trajectory once per variant and list on the GPU (the same per-shot code,
 * noise off) and stores the state at every checkpoint; a shot then starts at
 * the last checkpoint before its first noise hit, and loads that
 * checkpoint's coefficient tile only if an event reads it.  Results are
 * identical bit for bit either way (the same arithmetic on the same values);
 * on = 0 runs every shot from the start.  The counters' work fields count the
 * work run; prefix_shots counts the shots that started from a checkpoint. */
int soft_set_shared_prefix(soft_ctx *ctx, int on);

/* Deferred T runs (default on).  T gates change only the coefficients, never
 * the tableau signs that outcome-fixed measurements, checks and feedback read
 * (Theorem 1: T leaves the tableau alone), so a run of T gates with no noise
 * between them, followed by such events, can be skipped: a shot that a check
 * ends before any event reads the coefficients never needs the run (most
 * shots with an early fault, Sec. V's early stop of discarded shots).  When
 * an event does need them, the run is applied then, with the tableau signs
 * it saw (the events in between changed only signs and records), before that
 * event; when the shot's final state is kept and a run is still skipped at
 * the end, the attempt runs again with every run applied.  The arithmetic
 * is the same either way, so records, statuses, abort ops, observables and
 * kept states are identical.  Off with a support cap (the cap is checked on every T).  What
 * differs: a shot that ended with a run skipped reports, in support_hist,
 * the largest support it computed, and the norm check covers the
 * coefficients it computed.  on = 0 applies every run. */
int soft_set_deferred_t(soft_ctx *ctx, int on);

/* Where the per-wave coefficient tile lives (the GPU memory layout of
 * Sec. IV-B, re-planned for LDS and HBM): 0 = automatic (LDS when one
 * wave's tile takes at most 8 KiB; a split as mode 3 picks it when the tile
 * is larger but fits in a block's LDS; else device memory; soft_autotune also
 * tries device memory and other splits), 1 = LDS, 2 = device memory (HBM; one slab
 * of 2^k_max entries per resident wave, allocated by the library on first
 * use), 3 = split: the low 2^L entries of the tile in LDS, the other
 * 2^k_max - 2^L in a per-wave device-memory slab, with L the autotuned value
 * or by default the largest L < k_max whose LDS part takes at most 8 KiB;
 * 256 * L + 3 = split with that L (7 <= L <= 19; L >= k_max acts as
 * k_max - 1).  A split needs k_max >= 8; below that mode 3 uses LDS.  LDS is
 * the fast place; device memory lifts the LDS size limit on the span
 * dimension (up to k_max = 20); a split keeps the small coordinates in LDS
 * while more waves fit in a CU than with the whole tile there (the support
 * cap 2^12 with HBM spill of the scale run).  EINVAL for other modes. */
int soft_set_tile_memory(soft_ctx *ctx, int mode);

/* Batch-schedule autotuning (Sec. V measures throughput against the batch
 * size; Sec. IV-B launches fixed batches): time the default launch shape and
 * a grid of others (and, in automatic tile
 * mode, both tile placements) on `sample_shots` shots spread over the
 * variants, in one launch each (outputs discarded; the better of two timings
 * counts), and keep the fastest for this circuit, noise model and precision.
 * The result is cached for the process, keyed by the device (architecture
 * name and compute-unit count), the circuit (with a mixture's shot ranges),
 * precision, pruning threshold, support cap, tile placement and noise draws:
 * every context on such a device that loads the same circuit uses it.
 * Samples of 10^6 shots or more rank shapes reliably; small samples measure
 * launch overhead.  Runs on hip_stream and synchronizes it. */
int soft_autotune(soft_ctx *ctx, uint64_t sample_shots, void *hip_stream);

/* Keep the final state (v, B(S, D)) of Definition 1 / Eq. 3 of shots
 * [shot_lo, shot_lo + count) of later runs for soft_read_coeffs /
 * soft_read_tableau (count <= 16384; 0 disables; ECAPACITY above). */
int soft_set_keep(soft_ctx *ctx, uint64_t shot_lo, uint32_t count);

/* Sample shots shot0 .. shot0 + n_shots - 1: each shot is one independent
 * pure-state trajectory of the Monte-Carlo model of Sec. II-C (Cliffords by
 * Theorem 1 part 1, T by Eqs. 1-2 with Eq. 4, measurements by Theorem 1
 * part 2), stopped at the first failed postselection check (Sec. V-A), all in
 * one persistent launch (Sec. IV-B).  Indices are global: a shot's result
 * depends only on seed, shot index, circuit and noise, not on batching.
 * Asynchronous on hip_stream (a hipStream_t; NULL = default stream).
 *   outcomes_dev: uint32 [ceil(records/32)][n_shots], bit r%32 of word r/32
 *                 of shot i = record r (0 after an abort), or NULL;
 *   status_dev:   uint32 [n_shots] SOFT_PASSED/DISCARDED/OVERFLOW/NUMERIC;
 *   abort_op_dev: uint32 [n_shots] op index that ended the shot
 *                 (0xffffffff if it passed), or NULL;
 *   obs_dev:      uint32 [n_shots], bit j = observable j, or NULL.
 * EINVAL if the shots reach past the last variant's range of a mixture. */
int soft_run(soft_ctx *ctx, uint64_t shot0, uint64_t n_shots, uint32_t *outcomes_dev,
             uint32_t *status_dev, uint32_t *abort_op_dev, uint32_t *obs_dev,
             void *hip_stream);

/* soft_run for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, outputs and results as soft_run; the caller owns the outputs.
 * This call allocates nothing: no hipMalloc / hipFree, no graph is built.
 * It launches the counter reset and the sampler directly on hip_stream (so
 * a caller may capture them) and takes its counters, work cursors,
 * checkpoint slots (soft_set_shared_prefix; at most 4 MiB, else shots run
 * from the start with the same results) and any device-memory tiles from a static
 * scratch array of 36 MiB + 64 KiB per GPU, which the library holds on each
 * GPU it runs on until the process ends.
 * Device-memory tiles and the device-memory parts of split tiles
 * (soft_set_tile_memory) get at most 32 MiB of slabs, so such a launch may
 * run fewer waves; ECAPACITY when one block's slabs exceed 32 MiB.
 * The circuit's device tables are uploaded (allocated) by the soft_load_*
 * calls, never here.
 *   ESTATE: no circuit loaded;
 *   EUNSUPPORTED: kept states or a trace are on (they use library buffers).
 * Every call on a GPU, from any context, shares that GPU's scratch and leaves
 * its counters there: soft_read_counters afterwards reads the last such call
 * on the GPU.  Calls that overlap on one GPU (other streams, other contexts)
 * race on the scratch and must be serialized by the caller. */
int soft_run_noalloc(soft_ctx *ctx, uint64_t shot0, uint64_t n_shots, uint32_t *outcomes_dev,
                     uint32_t *status_dev, uint32_t *abort_op_dev, uint32_t *obs_dev,
                     void *hip_stream);

/* Re-run of chosen shots (Sec. IV-B: shots over the fixed capacity are run
 * again under a larger configuration).  Sample an explicit list of global
 * shot indices: shots_dev (device, uint64,
 * 8-byte aligned) holds n_shots indices in any order; output row i (of
 * outcomes_dev, status_dev, ...) belongs to shots_dev[i], with the layout of
 * soft_run.  A shot's result depends only on its index, so this re-runs
 * chosen shots exactly: e.g. the shots a capped run flagged SOFT_OVERFLOW,
 * after raising the cap (soft_set_caps) or moving the tile to device memory
 * (soft_set_tile_memory) -- the overflow re-run of a production sweep.  Kept
 * shots (soft_set_keep) are matched by shot index.  A mixture's index outside
 * every range runs as the last variant.  Explicit uniforms are for soft_run
 * only (EUNSUPPORTED here). */
int soft_run_list(soft_ctx *ctx, const uint64_t *shots_dev, uint64_t n_shots, uint32_t *outcomes_dev,
                  uint32_t *status_dev, uint32_t *abort_op_dev, uint32_t *obs_dev, void *hip_stream);

/* Aggregates of the last run (the statistics the host reads back, Sec. IV-B;
 * discard rate and logical errors as in Sec. V); synchronizes that run's
 * stream.  ESTATE before any run. */
int soft_read_counters(soft_ctx *ctx, soft_counters *out);

/* Aggregates of the last run over the shots of one variant of a mixture
 * (variant 0 of a single circuit is the whole run), as soft_read_counters
 * (Sec. IV-B, Sec. V).  Synchronizes.  EINVAL: no such variant. */
int soft_read_variant_counters(soft_ctx *ctx, uint32_t variant, soft_counters *out);

/* Final coefficients v_alpha of Definition 1 / Eq. 3 of a kept shot of the
 * last run: the state is sum_alpha v_alpha d_alpha |psi_S>, with the exact
 * global phase of Eqs. 1-2.  Sorted by alpha (bit k =
 * destabilizer d_k), entries below the pruning threshold left out.  Up to
 * cap entries are written; *count receives the full number.  Synchronizes. */
int soft_read_coeffs(soft_ctx *ctx, uint64_t shot, uint64_t *alpha, double *re, double *im,
                     uint32_t cap, uint32_t *count);

/* Final tableau B(S, D) of a kept shot (the Aaronson-Gottesman tableau of
 * Sec. II-B, signs included): 2n rows (destabilizers d_0..d_{n-1}, then
 * stabilizers s_0..s_{n-1}); row i is (-1)^r[i] prod_q sigma(x_q, z_q) with
 * x = bit q of x[i], z = bit q of z[i], sigma(1,1) = Y.  Synchronizes. */
int soft_read_tableau(soft_ctx *ctx, uint64_t shot, uint64_t *x, uint64_t *z, uint8_t *r);

/* Trace mode (the step-by-step validation of Sec. V-B): record the state of shot
 * `shot` after each of its first `steps` events (T/T-dagger, measurements,
 * detectors, observables, end) in the next runs; steps = 0 disables it
 * (steps <= 65536).  Cliffords make no event: they reach the state at the next
 * event, so the state recorded for CCX a b t (H_t CCZ H_t) is the one after
 * its CCZ, with the second H_t still to come. */
int soft_set_trace(soft_ctx *ctx, uint64_t shot, uint32_t steps);

/* State (v, B(S, D)) of Definition 1 of the traced shot after event `step`
 * of the last run (Sec. V-B step-by-step validation).  info[0..5] =
 * written (0/1), op index of the event, status at that point, span dimension
 * k, carried FP64 norm (bits of a double), 1 if the shot ended there.
 * x, z, r: 2n tableau rows as in soft_read_tableau; alpha/re/im/count as in
 * soft_read_coeffs.  Any output pointer may be NULL.  Synchronizes. */
int soft_read_trace(soft_ctx *ctx, uint32_t step, uint64_t info[6], uint64_t *x, uint64_t *z, uint8_t *r,
                    uint64_t *alpha, double *re, double *im, uint32_t cap, uint32_t *count);

/* Facts about the loaded circuit, in the terms of Table II (qubits,
 * measurements) and Theorem 2 (the largest span dimension, log2 of the
 * support bound): info[0..7] = qubits, records, noise slots,
 * measurement slots, observables, events, largest span dimension k_max,
 * record words.  For a mixture, each entry is the largest over the variants
 * (the record words size soft_run's outcome planes). */
int soft_circuit_info(soft_ctx *ctx, uint64_t info[8]);

/* The same facts (Table II, Theorem 2) for variant `variant` of a mixture. */
int soft_variant_info(soft_ctx *ctx, uint32_t variant, uint64_t info[8]);

/* Launch shape (Sec. IV-B) used by the next run: out[0..4] = waves_per_block,
 * blocks_per_cu, grab, LDS bytes per wave (tile or its LDS part, plus record
 * words), tile placement (0 LDS, 1 device memory, 2 split). */
int soft_launch_shape(soft_ctx *ctx, uint32_t out[5]);

/* Graph reuse of this context (the persistent launch is a hipGraph of two
 * kernel nodes, Sec. IV-B's batched launches): out[0] = graph
 * instantiations so far, out[1] = graph launches so far.  A run whose
 * precision, noise source, tile placement and launch shape match an existing
 * instantiation only updates the sampler node's arguments (shot range,
 * outputs, ...), so a scan of equal batches instantiates at most twice (two
 * instantiations are used in turn, so that one can be updated while the
 * other runs). */
int soft_graph_info(soft_ctx *ctx, uint64_t out[2]);

#ifdef __cplusplus
}
#endif
#endif
