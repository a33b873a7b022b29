/*
 * oracle.h -- plain CPU FP64 reference for generalized-stabilizer shot sampling.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU sampler.
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the product library never links or calls it, and the
 * two share no code (parser, noise lowering, random generator and simulator are
 * all written separately here).
 *
 * What it computes (arXiv 2512.23037):
 *   - state = stabilizer/destabilizer tableau (S, D) plus a sparse map
 *     alpha -> v_alpha, |phi> = sum_alpha v_alpha d_alpha |psi_S>
 *     (Sec. II-C, Definition 1 / Eq. 3);
 *   - Clifford gates conjugate all 2n rows, signs included; v is untouched
 *     (Theorem 1 part 1);
 *   - T / T-dagger use the Clifford-linear form of Eqs. 1-2 together with the
 *     Pauli-on-basis identity of Eq. 4 (Theorem 1 part 3);
 *   - Pauli measurements use the projectors (I +- P)/2 of Sec. II-A with the
 *     Aaronson-Gottesman pivot (Theorem 1 part 2);
 *   - stochastic Pauli noise and sampled measurement branches give one pure
 *     state per shot (Sec. II-C, "pure-state simulation model"), with the
 *     uniform depolarizing noise model of Sec. III.
 *
 * All arithmetic on coefficients is IEEE double.  Qubit count n <= 64 (one
 * 64-bit word per half-row).
 *
 * Thread safety: a compiled circuit is immutable and may be shared by threads.
 */
#ifndef SOFT_ORACLE_H
#define SOFT_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double p1;      /* DEP1 after every single-qubit gate (H S SDG X Y Z T TDG) */
    double p2;      /* DEP2 after every two-qubit gate (CX CZ)                  */
    double p_idle;  /* DEP1 on each idle qubit at every TICK                    */
    double p_meas;  /* XERR before every M                                       */
    double p_reset; /* XERR after every R                                        */
    double p_mpp;   /* classical flip of every MPP result                        */
} oracle_noise;

typedef struct oracle_circuit oracle_circuit;

/* Parse `text` (NUL-terminated) and insert model noise.  Returns NULL on a
 * parse error, with "line N: message" written to err (errlen bytes). */
oracle_circuit *oracle_compile(const char *text, const oracle_noise *noise,
                               char *err, int errlen);
void oracle_free(oracle_circuit *c);

/* Noise sampling mode: 0 (default) one word per noise slot from stream 0;
 * 1 geometric gaps between candidate slots from stream 2, thinned by
 * p_slot / p_max (the same hit distribution, different draws).  Explicit
 * words always use mode 0.  Returns 0, or -1 for a bad mode. */
int oracle_set_noise_mode(oracle_circuit *c, int mode);

/* counts[0..6] = n_qubits, n_source_ops, n_records, n_noise_slots,
 *                n_meas_slots, n_observables, n_lowered_ops */
void oracle_counts(const oracle_circuit *c, uint64_t counts[7]);

/* Status codes of a shot. */
enum { ORACLE_PASSED = 0, ORACLE_DISCARDED = 1, ORACLE_OVERFLOW = 2, ORACLE_NUMERIC = 3 };

typedef struct {
    uint32_t status;      /* ORACLE_*                                          */
    uint32_t abort_op;    /* source op index that ended the shot, or 0xffffffff */
    uint32_t obs;         /* bit j = value of OBSERVABLE j                      */
    uint32_t max_support; /* largest |v| seen                                    */
    uint64_t t_entries;   /* sum over T/TDG with beta != 0 of |v| after the op  */
    uint64_t t_phase_entries; /* sum over T/TDG with beta == 0 of |v|            */
    uint64_t m_entries;   /* sum over measurements of |v| before the op         */
    uint64_t noise_slots; /* noise slots drawn before the shot ended           */
    uint64_t events;      /* T/TDG + measurements executed                       */
    double   norm2;       /* sum |v|^2 at the end                                */
    uint64_t noise_words; /* random words drawn for noise (one per slot in mode 0) */
    uint64_t m_out_entries; /* sum over measurements of |v| after the op        */
    uint64_t m_pairs;     /* sum over beta != 0 measurements of representative pairs */
    uint64_t t_phase_flips; /* sum over T/TDG with beta == 0 of entries with lambda = -1 */
    uint64_t meas_words;  /* measurement uniforms used (one per measurement)   */
    /* The part of the counters above (t_entries .. meas_words, in the order of
     * oracle_batch's work sums) spent while the shot was still on the
     * noiseless trajectory that every shot of the circuit shares: before its
     * first applied noise hit (a Pauli or a record flip) and before its first
     * measurement whose outcome was not certain (0 < p0 < 1); all of it if the
     * shot never left that trajectory.  noise_slots and noise_words are 0
     * here: each shot draws its own noise whatever its path. */
    uint64_t shared[10];
} oracle_shot_info;

/* Number of work sums oracle_batch reports. */
enum { ORACLE_WORK_COUNT = 10 };

/* Run one shot.  words: NULL for Philox4x32-10 draws keyed by (seed, shot),
 * else explicit 32-bit words, [n_noise_slots] then [n_meas_slots].
 * tau: pruning threshold (relative to the 2-norm); cap: max |v| after a T.
 * record: ceil(n_records/32) words, bit k = measurement record k.
 * tab_x/tab_z/tab_r: 2n rows each (D rows then S rows), may be NULL.
 * alpha/re/im: final coefficients sorted by alpha, up to coeff_cap entries,
 * the full count written to *n_coeff; may be NULL.
 * p0_trace: probability of outcome +1 at each measurement slot; may be NULL.
 * Returns 0, or -1 if the arguments are inconsistent. */
int oracle_shot(const oracle_circuit *c, uint64_t seed, uint64_t shot,
                const uint32_t *words, double tau, uint32_t cap,
                uint32_t *record, oracle_shot_info *info,
                uint64_t *tab_x, uint64_t *tab_z, uint8_t *tab_r,
                uint64_t *alpha, double *re, double *im, uint32_t coeff_cap,
                uint32_t *n_coeff, double *p0_trace);

/* Run shots [shot0, shot0+n) on `threads` host threads.
 * words: NULL, or explicit words laid out [n][n_noise_slots + n_meas_slots].
 * outcomes: bit-planes [ceil(n_records/32)][n]; status/abort_op/obs: [n].
 * max_support: [n] or NULL.  work: NULL or ORACLE_WORK_COUNT sums of the
 * oracle_shot_info counters (t_entries, t_phase_entries, m_entries,
 * noise_slots, events, noise_words, m_out_entries, m_pairs, t_phase_flips,
 * meas_words).  shared_work: NULL or the ORACLE_WORK_COUNT sums of
 * oracle_shot_info.shared, in the same order. */
int oracle_batch(const oracle_circuit *c, uint64_t seed, uint64_t shot0,
                 uint64_t n, const uint32_t *words, double tau, uint32_t cap,
                 int threads, uint32_t *outcomes, uint32_t *status,
                 uint32_t *abort_op, uint32_t *obs, uint32_t *max_support,
                 uint64_t *work, uint64_t *shared_work);

/* Philox4x32-10 block (Salmon, Moraes, Dror, Shaw, SC'11). */
void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Pauli product with phase: {x, z, e} words, e = exponent of i (mod 4);
 * out = a * b. */
void oracle_pauli_mul(const uint64_t a[3], const uint64_t b[3], uint64_t out[3]);

#ifdef __cplusplus
}
#endif
#endif
