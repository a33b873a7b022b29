// program.h -- the compiled form of a circuit that the sampler kernel walks.
//
// The circuit compiler (compile.cpp) turns circuit text into a list of events
// (T/T-dagger, measurements, detectors, observables) and a table of noise
// locations.  Two facts make this form possible:
//
//  * Only the signs of the 2n tableau rows depend on the shot.  Every Clifford
//    rule and the Aaronson-Gottesman measurement update compute the x/z bits
//    from x/z bits alone, noise Paulis only flip signs, and T does not touch
//    the tableau (Theorem 1).  The x/z "frame" is therefore computed once per
//    circuit, and each Clifford between two events folds into one XOR mask on
//    the per-shot sign bits.
//  * The coefficient support of every shot lies in an affine subspace
//    a ^ span(b_0..b_{k-1}) of {0,1}^n whose linear part is also the same for
//    every shot: T adds the index shift beta of Eq. 4 when it is new, and a
//    measurement either cuts the span by the hyperplane gamma.alpha = const or
//    maps it through sigma -> sigma ^ sigma_p beta.  Only the offset a depends
//    on the shot.  The coefficients are then a dense array of 2^k entries
//    indexed by coordinates j, with alpha(j) = a ^ sum_t j_t b_t, and the
//    alpha <-> alpha ^ beta pairing of Eq. 4 becomes j <-> j ^ mu.
//
// A branching T^s multiplies the whole state by e^{i s pi/8} (Eqs. 1-2); that
// factor is kept as an exact per-shot count of eighth turns and applied only
// when a state is read out.  The tile also holds the state up to a real
// per-shot factor: the cos(pi/8) of each branching T joins it (measurements
// renormalise the tile and reset it), so the tile update is
//   v'_j = v_j + tan(pi/8) i^qb (-1)^(...) v_{j^mu}.
//
// Sign vectors are two 64-bit words: bit i of the D word is the sign of
// destabilizer d_i, bit i of the S word the sign of stabilizer s_i (n <= 64).
#pragma once
#include <stdint.h>

namespace soft {

enum EvKind : uint32_t {
    EV_T_PHASE = 0,  // beta = 0: entries with lambda = -1 pick up e^{i s pi/4}
    EV_T_DOUBLE,     // beta outside the span: k -> k+1, new coordinate on top
    EV_T_BFLY,       // beta = sum_t mu_t b_t: butterfly on pairs (j, j ^ mu)
    EV_M_DET,        // beta = 0 and gamma orthogonal to the span: outcome fixed
    EV_M_CUT,        // beta = 0, gamma.b_t not all 0: keep one parity class
    EV_M_SPLIT,      // beta != 0 outside the span: outcome 50/50
    EV_M_MERGE,      // beta != 0 inside the span: pairs merge, k -> k-1
    EV_DETECTOR,     // parity check of record bits, abort on failure
    EV_OBSERVABLE,   // parity of record bits, stored as an observable bit
    EV_FEEDBACK,     // Pauli flip (masks xD/xS) when the XOR of its record bits is 1 (check pairs
                     // dw0/dm0 and the pair table, as a detector reads them), or with EVF_AND
                     // when all of them are 1
    EV_DROP,         // speculative: coordinates >= mu carry no amplitude; k -> mu
    EV_DIAG,         // diagonal gate on <= 3 qubits, all its Z-strings in one pass (DiagInfo `boff`)
    EV_END,
    EV_NOP           // never in a list: the kernel's kind for an event it skips
};

enum EvFlags : uint32_t {
    EVF_TDG = 1u,      // T-dagger (s = -1)
    EVF_RECORD = 2u,   // store the outcome in the measurement record
    EVF_RESET = 4u,    // reset: apply X_q (masks xD/xS) when the outcome is 1
    EVF_CHECK = 8u,    // a detector that directly follows this measurement
    EVF_BATCH = 16u,   // first of `bcnt` outcome-fixed measurements run side by side
    EVF_CLIFF = 32u,   // cliffD or cliffS is nonzero
    EVF_DROP1 = 64u,   // speculative: after this butterfly (mu's top bit k-1) coordinate k-1 must be
                       // empty, i.e. no partner output kept; then k -> k-1
    EVF_TRUN = 128u,   // speculative: first of `bcnt` doublings with nothing between them, run as one
                       // pass (k + bcnt <= 6: one final entry per lane); the others are skipped
    EVF_BRUN = 256u,   // speculative: first of `bcnt` EVF_DROP1 butterflies with nothing between them
                       // (k <= 6), run in registers, one entry per lane; the others are skipped
    EVF_COND = 512u,   // EV_DIAG: classically controlled, applied only when its condition (the check
                       // pairs, as EV_FEEDBACK reads them) holds; otherwise the span still grows and
                       // the new coordinates hold zeros
    EVF_AND = 1024u,   // EV_FEEDBACK / EV_DIAG with EVF_COND: the condition is that every listed
                       // record bit is 1 (each pair's word covers its whole mask), not their XOR
    EVF_MAT = 2048u,   // the first event at or after a checkpoint, or after a deferrable T run, that
                       // reads or writes the tile: a shot started from that checkpoint loads the
                       // checkpoint's tile here, and a shot that deferred the run is redone
    EVF_DEFER = 4096u, // first of `mslot` events that form a deferrable T run (T gates with no noise
                       // slot and no Clifford flip between them, followed by events that do not
                       // touch the tile): a shot may skip them and is redone without skipping only
                       // if an event needs the tile
    EVF_PAIR = 8192u,  // a plain butterfly whose next event is a butterfly (plain or EVF_DROP1) on the
                       // same span with nothing between them: both run in one pass over quads
                       // {j, j^mu, j^mu', j^mu^mu'}, whose two coordinate bits left out of the
                       // pass index are pbit (low byte) and pbit >> 8
};

// One event: 64 dwords, which one wavefront loads with one dword per lane
// and reads field by field with readlane.  The first 16 dwords are used by
// every kind.
struct alignas(16) Event {
    uint32_t kind;
    uint32_t flags;
    uint32_t noise_end;  // noise slots [.., noise_end) precede this event
    uint32_t src;        // index of the circuit op this event came from
    uint64_t cliffD, cliffS;  // sign flips of the Cliffords since the last event
    uint64_t beta, gamma;     // index shift / anticommuting destabilizers
    uint32_t k;          // span dimension before the event
    uint32_t g;          // bit t = parity(gamma & b_t)
    uint32_t cexp;       // c = i^cexp * (-1)^(parity(rD&beta) ^ parity(rS&gamma))
    uint32_t qb;         // branching T: quarter turns of the partner weight i^qb
    uint32_t mu;         // coordinates of beta in the span (BFLY, MERGE)
    uint32_t tstar;      // coordinate removed (CUT, MERGE) / top bit of mu (BFLY)
    uint32_t pm;         // bit t = bit p of b_t (SPLIT, MERGE)
    uint32_t pbit;       // pivot p (SPLIT, MERGE) / EVF_PAIR: the quad's two coordinate bits
    uint32_t mslot;      // measurement slot (M, MPP, R) / EVF_DEFER: events in the run
    uint32_t rec;        // record index (recorded measurements) / observable index
    uint32_t gbeta;      // parity(gamma & beta)
    uint32_t psign;      // sign bit of the measured Pauli (0 for parsed ops)
    uint32_t expect;     // DETECTOR/OBSERVABLE/check: expected parity
    uint32_t det_off;    //   first (word, mask) pair in the pair table
    uint32_t det_cnt;    //   number of pairs
    uint32_t chk_src;    //   op index of a folded detector
    uint32_t dw0, dm0;   //   the first pair, inline
    uint32_t bcnt;       // EVF_BATCH, EVF_TRUN, EVF_BRUN: number of members (events e .. e + bcnt - 1)
    uint32_t boff;       //   BATCH: their first record in the member table; TRUN, BRUN: the run's
                         //   phase8 step
    uint64_t avec;            // offset update: b_{t*} (CUT) or beta (SPLIT, MERGE)
    uint64_t AD, AS;          // rows (besides d_p, s_p) that absorb s_p
    uint64_t PhD, PhS;        // extra sign bits of those products
    uint64_t xD, xS;          // reset / feedback: rows anticommuting with the flip Pauli
    union {
        struct {
            double Are, Aim;  // T_PHASE: e^{i s pi/4}
        };
        struct {
            // EVF_TRUN: bit J of trot0 / trot1 = bit 0 / 1 of the fixed quarter
            // turns of final entry J (sum over the members i whose new
            // coordinate J sets of qb_i + 2 parity(g_i & (J mod 2^(k + i))))
            uint64_t trot0, trot1;
        };
    };
    // Branching T on a tile that carries the state up to a per-shot real
    // factor: v'_j = v_j + tan(pi/8) i^qb c' v_partner, and cos^2(pi/8) joins
    // the factor's square.
    double Tn;                // tan(pi/8)
    double Cs2;               // cos^2(pi/8)
    // Work of the list's events before this one, so a shot's counters come
    // from the event after the last one it ran: tile entries written by
    // branching T, tile entries read by measurement passes, T and measurement
    // events.
    uint64_t cum_t, cum_m;
    float Tnf;                // Tn in single precision
    uint32_t cum_e;
    double iCs2;              // 1 / Cs2
    // Branching T pass shape, fixed by k and the event: the coordinate bit
    // that pairs the pass's 64-lane iterations by sign (0: all signs +1), and
    // (BFLY) the coordinate bits a lane index occupies, ins0(63, tstar).
    uint32_t tpair, lmask;
};
static_assert(sizeof(Event) == 256, "event layout");

// A run of consecutive outcome-fixed measurements (EV_M_DET) whose results do
// not depend on one another is evaluated with one member per lane.  The
// compiler only forms such a run when
//  * no reset inside it anticommutes with a later member's measured Pauli,
//  * each folded detector reads only its own member's record bit and record
//    bits written before the run (one (word, mask) pair at most),
//  * the recorded members sit on consecutive lanes with consecutive record
//    indices, and no record-flip noise falls between the members.
// Member layout: 20 dwords.
enum BatchInfo : uint32_t {
    BM_CSIGN = 1u,    // c = -1 (cexp == 2)
    BM_RECORD = 2u,
    BM_RESET = 4u,
    BM_CHECK = 8u,
    BM_OWN = 16u,     // the check reads this member's own record bit
    BM_EXPECT = 32u,  // expected parity of the check
};
struct alignas(16) BatchMember {
    uint64_t beta, gamma;
    uint64_t cumD, cumS;  // Clifford sign flips from the first member up to this one
    uint64_t xD, xS;      // reset flip masks (0 without reset)
    uint32_t noise_end;   // noise slots [.., noise_end) precede this member
    uint32_t info;        // BatchInfo bits
    uint32_t dw0, dm0;    // check: record word and mask (own bit removed)
    uint32_t chk_src;     // op index of the folded detector
    uint32_t r0;          // first record written by the run
    uint32_t rlane;       // lane of the first recorded member | (recorded count << 8)
    uint32_t pad;
};
static_assert(sizeof(BatchMember) == 80, "batch member layout");
constexpr uint32_t kBatchMax = 64;

// A diagonal gate U = sum_x e^{i phi_x} |x><x| on m <= 3 qubits, applied in
// one pass.  Over the 2^m Z-strings g of its qubits U = sum_g c_g Z^g
// (c_g = 2^-m sum_x e^{i phi_x} (-1)^{g.x}, the expansion behind
// Proposition 1), and Z^g = i^cexp_g (sign part) d_beta_g s_gamma_g acts on
// the basis by Eq. 4.  In span coordinates term g moves entry j to j ^ mu_g
// (the span first grows by the new beta_g).  The shifts mu_g span a subspace
// with a reduced echelon basis e_0..e_{r-1} (top bits lead_i ascending), so
// the tile splits into 2^(knew - r) cosets j0 ^ span, j0 with zeros at the
// lead bits, and element u = j0 ^ E_u of a coset becomes
//   v'[j0 ^ E_u] = sum_g W_g (-1)^(gm_g . j_in) v[j_in],  j_in = j0 ^ E_(u ^ ug_g)
// (v = 0 past the old span), with W_g = D_g (-1)^(parity(rD & beta_g) ^
// parity((rS ^ a) & gamma_g)) per shot and D_g = c_g i^cexp_g.
struct alignas(16) DiagInfo {
    uint64_t beta[8], gamma[8];  // index shift / anticommuting destabilizers of Z^g
    double dre[8], dim[8];       // D_g
    float fre[8], fim[8];        // D_g in single precision
    uint32_t gm[8];              // bit t = parity(gamma_g & b_t), span after the gate
    uint32_t ug[8];              // mu_g in the coset basis (bit i = bit lead_i of mu_g)
    uint32_t E[8];               // coordinates of coset element u (XOR of e_i over the bits of u)
    uint32_t ng, r, knew, lead;  // Z-strings (2^m), coset dimension, span dimension after, lead_i in bits 5i..5i+4
};
static_assert(sizeof(DiagInfo) == 432, "diagonal gate layout");

// A mixture runs several compiled circuits in one launch: global shot indices
// [previous shot_end, shot_end) belong to the variant, whose events, noise
// locations and thresholds sit at the given offsets of the shared tables.
struct alignas(16) VariantDesc {
    uint64_t shot_end;
    uint32_t ev_off, nz_off, tm1_off;  // tm1_off is a multiple of 256
    uint32_t n_noise;
    uint32_t ev_off_full;  // the full event list (ev_off: the speculative one, or the same)
    uint32_t gap_off;      // gap-sampling threshold table of this variant (n_noise entries)
    // checkpoints of the noiseless trajectory (Program::ckpts) of the list at
    // ev_off and of the full list: [ck_off, ck_off + ck_cnt) of the table
    uint32_t ck_off, ck_cnt, ck_off_full, ck_cnt_full;
    // gap sampling: 1 / log2(q) (0 without noise), which puts the gap of a
    // word w within a few slots of log2(w / 2^32) / log2(q); and 1 when
    // every slot accepts every candidate (acc = 2^32: one probability)
    float gap_l2q;
    uint32_t acc_one;
    uint32_t pad_[2];
};
static_assert(sizeof(VariantDesc) == 64, "variant layout");
constexpr uint32_t kMaxVariants = 64;

// A checkpoint of the noiseless trajectory: the point before event `ev` of a
// list, after noise slots [0, nz).  Up to the first measurement with a random
// outcome every event is deterministic in a shot that no noise has hit, so
// every such shot is in the same state there.
struct Checkpoint {
    uint32_t ev, nz;
};
constexpr uint32_t kMaxCheckpoints = 16;

// A checkpoint's state, built once per launch (one slot per checkpoint of the
// table): this header at the slot's start, the record words at byte 128, the
// coefficient tile (2^k entries of the run's precision) after them, 16-byte
// aligned.
struct alignas(16) CkptState {
    uint64_t rD, rS, a;
    double nrm2, itscale2;
    double tnorm;     // sum of |v_j|^2 over the tile, summed as a shot's end sums it
    uint32_t k, phase8, maxsup, obs;
    uint32_t valid;   // 1 once the build reached the checkpoint
    uint32_t pad[3];
};
static_assert(sizeof(CkptState) == 80, "checkpoint layout");
constexpr uint32_t kCkptRecOff = 128;

enum NoiseKind : uint32_t { NZ_NONE = 0, NZ_DEP1, NZ_DEP2, NZ_XERR, NZ_FLIP, NZ_ZERR };

// One noise location (one random word).  masks[0..3] = rows anticommuting
// with X_a (D, S) and with Z_a (D, S); masks[4..7] the same for qubit b.
//
// Two ways to draw the hits, with the same distribution (each slot hit
// independently with its probability p):
//  * per slot: slot s takes word s of stream 0 and is hit iff word < thr;
//  * gap sampling: candidates form a Bernoulli(p_max) process over the slots,
//    p_max the largest slot probability.  The gap G before the next candidate
//    has P(G >= g) = q^g (q = 1 - p_max); one word w of stream 2 gives
//    G = #{g >= 1 : w < floor(q^g 2^32)} from the variant's gap table, and the
//    next word a accepts the candidate iff a < acc = floor(p / p_max 2^32).
//    Words of stream 2 are taken in order, two per candidate (one past the
//    last slot).  A slot with thr = 0 is never hit in either way.
// A hit's Pauli comes from its word the same way in both: w / thr (per slot)
// or a / acc (gap sampling) split into 3 (DEP1) or 15 (DEP2) equal parts.
struct alignas(16) NoiseLoc {
    uint32_t kind;
    uint32_t rec;     // FLIP: record bit to flip
    uint64_t thr;     // floor(p * 2^32), 0..2^32
    uint64_t masks[8];
    uint64_t acc;     // gap sampling: floor(p / p_max * 2^32), 0 when thr = 0
    uint64_t pad;
};
static_assert(sizeof(NoiseLoc) == 96, "noise layout");

// How a launch draws its noise hits (NoiseLoc): per slot, explicit words
// (per slot, words given by the caller) or gap sampling.
enum NoiseSource : uint32_t { NS_SLOTS = 0, NS_EXPLICIT = 1, NS_GAPS = 2 };

// Per-shot status codes (low byte of the status word).
enum Status : uint32_t { ST_PASSED = 0, ST_DISCARDED = 1, ST_OVERFLOW = 2, ST_NUMERIC = 3 };

// Device counters, all 64-bit: one row of C_COUNT per variant.
enum Counter {
    C_SHOTS = 0, C_PASSED, C_DISCARDED, C_OVERFLOW, C_NUMERIC, C_LOGICAL,
    C_ENTRIES_T, C_ENTRIES_M, C_NOISE, C_EVENTS, C_NORMDEV_BITS,
    C_RESTARTS,              // shots restarted on the full list after a failed DROP check
    C_PREFIX,                // attempts that started from a checkpoint of the noiseless trajectory
    C_REDO,                  // attempts redone because a deferred T run's tile was needed
    C_HIST0,                 // 16 buckets of floor(log2(max |v|))
    C_COUNT = C_HIST0 + 16
};

// Per kept shot (and per traced step): meta words, and separately the dense
// coefficient tile as double pairs.  KM_VALID holds kStateValid once written.
enum KeepMeta {
    KM_STATUS = 0, KM_ABORT, KM_TERM_EV, KM_AFTER, KM_RD, KM_RS, KM_A, KM_K, KM_NRM2, KM_VALID, KM_VAR, KM_PROG,
    KM_COUNT
};

constexpr unsigned long long kStateValid = 0x5f7a7e5f7a7e0001ull;

// Measurement-record words a shot keeps in scalar registers; a circuit with
// at most this many words needs no LDS for its record.
constexpr uint32_t kRecSgpr = 4;

}  // namespace soft
