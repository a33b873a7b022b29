// soft_api.cpp -- the C ABI declared in include/soft.h.
//
// Host side of the sampler: owns the compiled circuit and its device copy,
// chooses the launch shape (fixed, default or autotuned), captures the
// reset + sampler launch pair into a hipGraph, and decodes kept final states
// for the readout calls.  No simulation arithmetic runs here; every shot is
// computed by the kernels in sampler.hip.
#include "soft.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "compile.h"
#include "sampler.h"

using namespace soft;

namespace {

thread_local std::string g_create_error;

struct Shape {
    uint32_t wpb = 0, bpc = 0, grab = 0;
    uint32_t gt = TM_LDS;  // tile placement: TM_LDS, TM_MEM or TM_SPLIT
    uint32_t lds_log2 = 0; // TM_SPLIT: log2 of the tile entries held in LDS
};

struct Variant {
    std::string text;
    NoiseModel noise;
    uint64_t shot_end = ~0ull;  // global shots [previous end, shot_end)
    Program prog;               // the full event list
    Program fast;               // the speculative list with DROP events (empty: none found)
    bool has_fast = false;
};

// counter rows, then the sampler's and the prefix build's work cursors
constexpr size_t kCounterWords = (size_t)kMaxVariants * C_COUNT + 2;
static_assert(kCounterWords * sizeof(unsigned long long) <= kScratchCounterBytes, "scratch counter area");

// Kept final states: at most this many shots, and at most kMaxKeepBytes of
// dense tiles (FP64 pairs) for them.
constexpr uint32_t kMaxKeep = 16384;
constexpr uint64_t kMaxKeepBytes = 4ull << 30;

// Autotuned launch shapes, shared by every context of the process: keyed by
// the device (architecture name and compute-unit count) and by what changes
// the timing of a circuit (its hash with the shot ranges, precision, pruning
// threshold, support cap, tile placement and noise draws).
typedef std::tuple<std::string, int, uint64_t, int, double, uint32_t, int, int> TuneKey;
std::mutex g_tune_mu;
std::map<TuneKey, Shape> g_tuned;

template <typename T> struct DevBuf {
    T *p = nullptr;
    size_t n = 0;  // elements allocated
};

}  // namespace

struct soft_ctx {
    int device = 0;
    int num_cus = 0;
    int max_lds_block = 65536;
    std::string err;

    bool have_text = false;
    bool mixture = false;
    NoiseModel noise;            // model of a single loaded circuit
    std::vector<Variant> vars;   // the circuit, or the circuits of a mixture
    bool dirty = true;           // device tables must be rebuilt
    uint32_t kmax = 0, rec_words = 0;  // largest over the variants
    uint64_t hash = 0;           // of every variant and its shot range

    uint64_t seed = 0;
    const uint32_t *words_dev = nullptr;
    uint64_t words_n = 0;
    uint32_t words_noise = 0, words_meas = 0;
    int bits = 64;
    double tau = -1.0;
    uint32_t support_cap = 0;
    int tile_mode = 0;                        // 0 auto, 1 LDS, 2 device memory, 3 split
    uint32_t split_log2 = 0;                  // split: log2 of the LDS part asked for (0: default)
    bool speculate = true;                    // run speculative event lists where compiled
    bool shared_prefix = true;                // start shots at checkpoints of the noiseless trajectory
    bool defer_t = true;                      // skip deferrable T runs until an event needs their tile
    bool any_prefix = false;                  // some variant's lists have checkpoints
    int noise_mode = 0;                       // 0 a word per noise slot, 1 gap sampling
    Shape user;                               // explicit launch shape parts
    std::string arch;                         // gcnArchName of the device (autotune cache key)

    DevBuf<Event> d_ev;
    DevBuf<NoiseLoc> d_nz;
    DevBuf<uint32_t> d_tm1, d_det, d_gap;
    DevBuf<BatchMember> d_bm;
    DevBuf<DiagInfo> d_diag;
    DevBuf<VariantDesc> d_vars;
    DevBuf<unsigned char> d_gtile;            // device-memory tiles
    DevBuf<unsigned char> d_prefix;           // checkpoint state slots (one per table entry)
    DevBuf<Checkpoint> d_ckpt;                // checkpoint table
    uint32_t n_ckpt = 0;                      // its entries
    unsigned long long *d_counters = nullptr;  // kMaxVariants rows of C_COUNT, then the work cursor
    const unsigned long long *last_counters = nullptr;  // counters of the last run
    double *d_phase = nullptr;                 // cos/sin of k pi/8, k = 0..15
    unsigned char *scratch = nullptr;          // this device's static scratch (soft_run_noalloc)

    uint64_t keep_lo = 0;
    uint32_t keep_n = 0;
    DevBuf<unsigned long long> d_keep_meta;
    DevBuf<double> d_keep_v;
    uint32_t keep_tile = 0;  // tile entries of the last run's keep buffer

    uint64_t trace_shot = 0;
    uint32_t trace_n = 0;
    DevBuf<unsigned long long> d_trace_meta;
    DevBuf<double> d_trace_v;
    uint32_t trace_tile = 0;

    // The reset + sampler pair as a graph of two kernel nodes, instantiated
    // twice (two slots used in turn).  A run whose kernel and launch shape
    // match the slot's only updates the sampler node's arguments (shot range,
    // outputs, ...), so one instantiation serves a whole scan; a slot is
    // updated only after its previous launch has finished (its event), since
    // an update may rewrite arguments a running launch still reads.
    struct GraphSlot {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipGraphNode_t sampler = nullptr;
        hipGraphNode_t build = nullptr;  // the prefix build (between reset and sampler), if any
        hipEvent_t done = nullptr;   // recorded after the slot's last launch
        bool launched = false;
        std::vector<unsigned char> key;  // kernel, grid, block, LDS, counters
        RunParams args;                  // argument storage of the sampler node
        RunParams bargs;                 // and of the prefix build node
        unsigned long long *r_counters = nullptr, *r_next = nullptr;  // reset node arguments
        uint32_t r_n = 0;
    };
    GraphSlot slots[2];
    uint32_t next_slot = 0;
    uint64_t graph_instantiations = 0, graph_launches = 0;

    bool ran = false;
    hipStream_t last_stream = nullptr;
    uint64_t last_shot0 = 0, last_n = 0;
    bool last_list = false;  // the last run sampled a shot list
};

namespace {

int fail(soft_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, expr)                                                                          \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail((ctx), SOFT_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <typename T> int ensure(soft_ctx *c, DevBuf<T> &b, size_t n) {
    if (n == 0) n = 1;
    if (b.n >= n) return SOFT_OK;
    if (b.p) HIPCHK(c, hipFree(b.p));
    b.p = nullptr;
    b.n = 0;
    HIPCHK(c, hipMalloc((void **)&b.p, n * sizeof(T)));
    b.n = n;
    return SOFT_OK;
}

template <typename T> void release(DevBuf<T> &b) {
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.n = 0;
}

double tau_of(const soft_ctx *c) { return c->tau >= 0.0 ? c->tau : (c->bits == 32 ? 1e-6 : 1e-12); }

uint32_t tile_entries(const soft_ctx *c) { return 1u << c->kmax; }
uint32_t rec_words(const soft_ctx *c) { return c->rec_words; }
uint32_t entry_bytes(const soft_ctx *c) { return c->bits == 64 ? 16u : 8u; }
uint32_t tile_bytes(const soft_ctx *c) { return tile_entries(c) * entry_bytes(c); }
// Smallest LDS part of a split tile: the passes put up to 128 consecutive
// entries of one iteration on a wave's lanes, and the split keeps them in one
// place.
constexpr uint32_t kSplitMinLog2 = 7;
bool split_possible(const soft_ctx *c) { return c->kmax >= kSplitMinLog2 + 1u; }
// Tile bytes a wave keeps in LDS.
uint32_t lds_tile_bytes(const soft_ctx *c, const Shape &s) {
    if (s.gt == TM_MEM) return 0u;
    if (s.gt == TM_SPLIT) return (1u << s.lds_log2) * entry_bytes(c);
    return tile_bytes(c);
}
// Device-memory slab bytes per wave.
uint32_t slab_bytes(const soft_ctx *c, const Shape &s) { return tile_bytes(c) - lds_tile_bytes(c, s); }
// LDS bytes per wave: the tile or its LDS part, and the record.  A record of
// at most kRecSgpr words stays in scalar registers and takes no LDS.
uint32_t wave_bytes(const soft_ctx *c, const Shape &s) {
    const uint32_t recb = rec_words(c) > kRecSgpr ? (rec_words(c) * 4u + 15u) & ~15u : 0u;
    return std::max<uint32_t>(16u, ((lds_tile_bytes(c, s) + 15u) & ~15u) + recb);
}
// Bytes of one checkpoint slot: the state, the record words and a whole
// tile, 256-aligned.
uint32_t prefix_stride(const soft_ctx *c) {
    return (kCkptRecOff + ((rec_words(c) * 4u + 15u) & ~15u) + tile_bytes(c) + 255u) & ~255u;
}
bool use_prefix(const soft_ctx *c) { return c->shared_prefix && c->any_prefix; }

// The prefix build launch's parameters: item i = variant i / 2, list i & 1,
// no outputs, no kept states or trace, its own work cursor.
RunParams build_params(const RunParams &rp) {
    RunParams b = rp;
    b.prefix_build = 1;
    b.n_shots = 2ull * rp.n_vars;
    b.shot0 = 0;
    b.shot_list = nullptr;
    b.outcomes = nullptr;
    b.status = nullptr;
    b.abort_op = nullptr;
    b.obs = nullptr;
    b.keep_meta = nullptr;
    b.keep_v = nullptr;
    b.keep_n = 0;
    b.trace_meta = nullptr;
    b.trace_v = nullptr;
    b.trace_n = 0;
    b.grab = 1;
    b.next = rp.next + 1;
    return b;
}

// Default LDS part of a split tile: at most 8 KiB, below the whole tile.
uint32_t split_log2_default(const soft_ctx *c) {
    uint32_t L = c->kmax - 1u;
    while (L > kSplitMinLog2 && (1u << L) * entry_bytes(c) > 8192u) --L;
    return L;
}

void drop_slot(soft_ctx *c, soft_ctx::GraphSlot &g) {
    if (g.launched && g.done) (void)hipEventSynchronize(g.done);
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
    g.sampler = nullptr;
    g.build = nullptr;
    g.launched = false;
    g.key.clear();
    (void)c;
}

void drop_graph(soft_ctx *c) {
    for (auto &g : c->slots) drop_slot(c, g);
}

int compile_into(soft_ctx *c, const std::string &text, const NoiseModel &nm, Program &out, bool speculate = false) {
    try {
        compile_circuit(text, nm, out, speculate);
    } catch (const CompileError &e) {
        return fail(c, e.line > 0 ? SOFT_EPARSE : SOFT_ECAPACITY,
                    e.line > 0 ? "line " + std::to_string(e.line) + ": " + e.msg : e.msg);
    } catch (const std::bad_alloc &) {
        return fail(c, SOFT_ECAPACITY, "out of host memory while compiling");
    }
    return SOFT_OK;
}

// Compile a variant's full event list and, when the circuit offers span
// truncations, its speculative list.
int compile_variant(soft_ctx *c, Variant &V) {
    int rc = compile_into(c, V.text, V.noise, V.prog);
    if (rc) return rc;
    V.has_fast = false;
    V.fast = Program();
    if ((rc = compile_into(c, V.text, V.noise, V.fast, true))) return rc;
    for (const Event &E : V.fast.events)
        if (E.kind == EV_DROP || (E.flags & EVF_DROP1)) V.has_fast = true;
    if (!V.has_fast) V.fast = Program();
    return SOFT_OK;
}

// Upload the compiled variants as one set of tables: each variant's events,
// noise locations, thresholds, check pairs and run members are appended, and
// its references into the shared tables are rebased.
int prepare(soft_ctx *c) {
    if (!c->have_text) return fail(c, SOFT_ESTATE, "no circuit loaded");
    if (!c->dirty) return SOFT_OK;
    std::vector<Event> ev;
    std::vector<NoiseLoc> nz;
    std::vector<uint32_t> tm1, det, gap;
    std::vector<BatchMember> bm;
    std::vector<DiagInfo> dg;
    std::vector<VariantDesc> vd;
    std::vector<Checkpoint> ck;
    c->kmax = 0;
    c->rec_words = 0;
    uint64_t h = 1469598103934665603ULL;
    for (const Variant &V : c->vars) {
        const Program &P = V.prog;
        VariantDesc D;
        std::memset(&D, 0, sizeof(D));
        D.shot_end = V.shot_end;
        D.nz_off = (uint32_t)nz.size();
        D.tm1_off = (uint32_t)tm1.size();
        D.n_noise = P.n_noise;
        D.gap_off = (uint32_t)gap.size();
        D.gap_l2q = (P.gap_pmax > 0.0 && P.gap_pmax < 1.0) ? (float)(1.0 / std::log2(1.0 - P.gap_pmax)) : 0.0f;
        D.acc_one = P.noise.empty() ? 0u : 1u;
        for (const NoiseLoc &L : P.noise)
            if (L.acc != (1ull << 32)) D.acc_one = 0u;
        // each event list with its own check pairs and run members
        auto append = [&](const Program &Q) {
            const uint32_t off = (uint32_t)ev.size();
            const uint32_t det_base = (uint32_t)(det.size() / 2), bm_base = (uint32_t)bm.size();
            const uint32_t dg_base = (uint32_t)dg.size();
            for (Event E : Q.events) {
                E.det_off += det_base;
                if (E.flags & EVF_BATCH) E.boff += bm_base;
                if (E.kind == EV_DIAG) E.boff += dg_base;
                ev.push_back(E);
            }
            det.insert(det.end(), Q.det_pairs.begin(), Q.det_pairs.end());
            bm.insert(bm.end(), Q.batch.begin(), Q.batch.end());
            dg.insert(dg.end(), Q.diag.begin(), Q.diag.end());
            return off;
        };
        D.ev_off_full = append(P);
        D.ev_off = V.has_fast ? append(V.fast) : D.ev_off_full;
        // checkpoints of each list (one set when the variant has one list)
        D.ck_off_full = (uint32_t)ck.size();
        D.ck_cnt_full = (uint32_t)P.ckpts.size();
        ck.insert(ck.end(), P.ckpts.begin(), P.ckpts.end());
        D.ck_off = D.ck_off_full;
        D.ck_cnt = D.ck_cnt_full;
        if (V.has_fast) {
            D.ck_off = (uint32_t)ck.size();
            D.ck_cnt = (uint32_t)V.fast.ckpts.size();
            ck.insert(ck.end(), V.fast.ckpts.begin(), V.fast.ckpts.end());
        }
        nz.insert(nz.end(), P.noise.begin(), P.noise.end());
        tm1.insert(tm1.end(), P.noise_tm1.begin(), P.noise_tm1.end());
        gap.insert(gap.end(), P.gap.begin(), P.gap.end());
        vd.push_back(D);
        c->kmax = std::max(c->kmax, P.kmax);
        c->rec_words = std::max(c->rec_words, (P.n_rec + 31u) / 32u);
        h = (h ^ P.hash) * 1099511628211ULL;
        h = (h ^ V.shot_end) * 1099511628211ULL;
    }
    c->hash = h;
    c->any_prefix = !ck.empty();
    c->n_ckpt = (uint32_t)ck.size();
    int rc;
    if ((rc = ensure(c, c->d_ev, ev.size())) || (rc = ensure(c, c->d_nz, std::max<size_t>(nz.size(), 1))) ||
        (rc = ensure(c, c->d_tm1, tm1.size())) || (rc = ensure(c, c->d_det, std::max<size_t>(det.size(), 2))) ||
        (rc = ensure(c, c->d_bm, std::max<size_t>(bm.size(), 1))) || (rc = ensure(c, c->d_vars, vd.size())) ||
        (rc = ensure(c, c->d_diag, std::max<size_t>(dg.size(), 1))) ||
        (rc = ensure(c, c->d_gap, std::max<size_t>(gap.size(), 1))) ||
        (rc = ensure(c, c->d_ckpt, std::max<size_t>(ck.size(), 1))))
        return rc;
    if (!ck.empty()) HIPCHK(c, hipMemcpy(c->d_ckpt.p, ck.data(), ck.size() * sizeof(Checkpoint), hipMemcpyHostToDevice));
    if (!gap.empty()) HIPCHK(c, hipMemcpy(c->d_gap.p, gap.data(), gap.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_ev.p, ev.data(), ev.size() * sizeof(Event), hipMemcpyHostToDevice));
    if (!nz.empty()) HIPCHK(c, hipMemcpy(c->d_nz.p, nz.data(), nz.size() * sizeof(NoiseLoc), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_tm1.p, tm1.data(), tm1.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    if (!det.empty()) HIPCHK(c, hipMemcpy(c->d_det.p, det.data(), det.size() * sizeof(uint32_t), hipMemcpyHostToDevice));
    if (!bm.empty()) HIPCHK(c, hipMemcpy(c->d_bm.p, bm.data(), bm.size() * sizeof(BatchMember), hipMemcpyHostToDevice));
    if (!dg.empty()) HIPCHK(c, hipMemcpy(c->d_diag.p, dg.data(), dg.size() * sizeof(DiagInfo), hipMemcpyHostToDevice));
    HIPCHK(c, hipMemcpy(c->d_vars.p, vd.data(), vd.size() * sizeof(VariantDesc), hipMemcpyHostToDevice));
    c->dirty = false;
    drop_graph(c);
    return SOFT_OK;
}

// Largest LDS a CU offers to resident blocks (gfx950: 160 KiB).
constexpr uint32_t kLdsPerCu = 160u * 1024u;
constexpr uint32_t kMaxWavesPerCu = 32u;

// Untuned launch shape: as many resident waves per CU as the LDS tiles allow
// (at most 32), two waves per block when that still leaves >= 16 waves.
// Device-memory tiles are used when asked for, or (auto) when one wave's LDS
// tile does not fit in a block's LDS.
// Noise source of the next launch (explicit words use the per-slot form).
uint32_t noise_source(const soft_ctx *c) {
    return c->words_dev != nullptr ? NS_EXPLICIT : (c->noise_mode == 1 ? NS_GAPS : NS_SLOTS);
}

// The placement asked for (soft_set_tile_memory), or (auto) LDS when one
// wave's tile fits in a block's LDS, else device memory.  A split needs a
// span of at least 2^8 entries; below that the tile is small and goes to LDS.
Shape placement(const soft_ctx *c) {
    Shape s;
    if (c->tile_mode == 2) {
        s.gt = TM_MEM;
    } else if (c->tile_mode == 3 && split_possible(c)) {
        s.gt = TM_SPLIT;
        s.lds_log2 = c->split_log2 ? std::min<uint32_t>(c->split_log2, c->kmax - 1u) : split_log2_default(c);
    } else if (c->tile_mode == 0) {
        // LDS up to 8 KiB a wave (20 waves a CU, the register-bound
        // occupancy), a split above that while the tile would fit a block's
        // LDS (its LDS part holds twice the waves or more), device memory for
        // tiles no block holds
        Shape l;
        if (wave_bytes(c, l) > (uint32_t)c->max_lds_block) {
            s.gt = TM_MEM;
        } else if (tile_bytes(c) > 8192u && split_possible(c)) {
            s.gt = TM_SPLIT;
            s.lds_log2 = split_log2_default(c);
        }
    }
    return s;
}

// Resident waves per CU when the tile is not the limit (4 waves per SIMD).
constexpr uint32_t kMemTileWavesPerCu = 16u;

Shape default_shape(const soft_ctx *c) {
    Shape s = placement(c);
    const uint32_t wb = wave_bytes(c, s);
    const uint32_t cap = s.gt == TM_MEM ? kMemTileWavesPerCu : kMaxWavesPerCu;
    const uint32_t waves_cu = std::max<uint32_t>(1u, std::min<uint32_t>(cap, kLdsPerCu / wb));
    s.wpb = (waves_cu >= 16u && 2u * wb <= (uint32_t)c->max_lds_block) ? 2u : 1u;
    while (s.wpb > 1 && s.wpb * wb > (uint32_t)c->max_lds_block) s.wpb /= 2;
    s.bpc = std::max<uint32_t>(1u, waves_cu / s.wpb);
    // no more blocks than stay resident (registers can be the tighter limit)
    int res = 0;
    if (sampler_occupancy(c->bits == 64, noise_source(c), s.gt, (int)(64u * s.wpb), (size_t)s.wpb * wb,
                          &res) == hipSuccess && res > 0)
        s.bpc = std::min<uint32_t>(s.bpc, (uint32_t)res);
    else
        (void)hipGetLastError();
    s.grab = 16;
    return s;
}

TuneKey tune_key(const soft_ctx *c) {
    return TuneKey(c->arch, c->num_cus, c->hash, c->bits, tau_of(c), c->support_cap,
                   c->tile_mode | (int)(c->split_log2 << 8), c->noise_mode);
}

Shape current_shape(const soft_ctx *c) {
    Shape s = default_shape(c);
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        auto it = g_tuned.find(tune_key(c));
        if (it != g_tuned.end()) s = it->second;
    }
    if (c->tile_mode) {  // an explicit placement overrides a tuned one
        const Shape p = placement(c);
        if (p.gt != s.gt || (p.gt == TM_SPLIT && c->split_log2)) {
            s.gt = p.gt;
            s.lds_log2 = p.lds_log2;
        }
    }
    if (c->user.wpb) s.wpb = c->user.wpb;
    if (c->user.bpc) s.bpc = c->user.bpc;
    if (c->user.grab) s.grab = c->user.grab;
    return s;
}

int check_shape(soft_ctx *c, const Shape &s) {
    if (s.gt == TM_SPLIT && (s.lds_log2 < kSplitMinLog2 || s.lds_log2 >= c->kmax))
        return fail(c, SOFT_EINVAL, "split tile: LDS part out of range");
    const uint64_t lds = (uint64_t)s.wpb * wave_bytes(c, s);
    if (s.wpb < 1 || s.wpb > 4) return fail(c, SOFT_EINVAL, "waves_per_block must be 1..4");
    if (lds > (uint64_t)c->max_lds_block)
        return fail(c, SOFT_ECAPACITY, "coefficient tile needs " + std::to_string(lds) + " bytes of LDS per block; the device allows " +
                                           std::to_string(c->max_lds_block) + " (span dimension " + std::to_string(c->kmax) + ")");
    if (s.bpc < 1 || s.grab < 1 || s.grab > 64) return fail(c, SOFT_EINVAL, "blocks_per_cu must be >= 1 and grab in 1..64");
    return SOFT_OK;
}

// Launch reset + sampler on `stream` through an instantiated graph: a slot
// whose kernel and launch shape match gets the new arguments, else a slot is
// built (reset node -> sampler node) and instantiated.
// Blocks of a launch: the resident blocks of the shape, at most one per
// `wpb` shots.
uint64_t grid_blocks(const soft_ctx *c, const Shape &s, uint64_t n_shots) {
    const uint64_t blocks_needed = (n_shots + s.wpb - 1) / s.wpb;
    return std::min<uint64_t>((uint64_t)c->num_cus * s.bpc, std::max<uint64_t>(blocks_needed, 1));
}

// LDS layout of a wave's slot (tile unless in device memory, record words
// past kRecSgpr).
void set_wave_layout(const soft_ctx *c, const Shape &s, RunParams &rp) {
    rp.wave_bytes = wave_bytes(c, s);
    rp.rec_off = (s.gt != TM_MEM && rec_words(c) > kRecSgpr) ? ((lds_tile_bytes(c, s) + 15u) & ~15u) : 0u;
    rp.gtile = nullptr;
    rp.tile_mode = s.gt;
    rp.lds_entries = s.gt == TM_SPLIT ? (1u << s.lds_log2) : 0u;
}

int launch(soft_ctx *c, RunParams rp, const Shape &s, uint64_t n_shots, hipStream_t stream) {
    const uint32_t wb = wave_bytes(c, s);
    const size_t lds = (size_t)s.wpb * wb;
    const uint64_t grid = grid_blocks(c, s, n_shots);
    const dim3 g((uint32_t)grid), b(64u * s.wpb);
    set_wave_layout(c, s, rp);
    if (s.gt != TM_LDS) {  // one slab per wave of the grid
        int rc = ensure(c, c->d_gtile, (size_t)grid * s.wpb * slab_bytes(c, s));
        if (rc) return rc;
        rp.gtile = c->d_gtile.p;
    }
    // shared-prefix slots, filled by the build launch before the sampler
    const bool pfx = use_prefix(c);
    rp.prefix = nullptr;
    rp.prefix_stride = 0;
    if (pfx) {
        int rc = ensure(c, c->d_prefix, (size_t)c->n_ckpt * prefix_stride(c));
        if (rc) return rc;
        rp.prefix = c->d_prefix.p;
        rp.prefix_stride = prefix_stride(c);
    }
    const uint64_t bgrid = std::min<uint64_t>(grid, (2ull * rp.n_vars + s.wpb - 1) / s.wpb);
    const uint32_t ns = rp.words != nullptr ? NS_EXPLICIT : (rp.noise_mode == 1u ? NS_GAPS : NS_SLOTS);
    const void *kfn = sampler_kernel(c->bits == 64, ns, s.gt, sampler_lean(rp));
    // what the nodes' launch configuration and the reset node depend on
    const uint64_t kv[9] = {(uint64_t)(uintptr_t)kfn, grid, (uint64_t)b.x, (uint64_t)lds,
                            (uint64_t)(uintptr_t)rp.counters, (uint64_t)rp.n_vars, (uint64_t)(uintptr_t)rp.next,
                            (uint64_t)pfx, pfx ? bgrid : 0ull};
    std::vector<unsigned char> key((const unsigned char *)kv, (const unsigned char *)kv + sizeof(kv));
    // The slot to use: one with this key whose last launch is done; else an
    // empty one (instantiated below); else one with this key (after waiting
    // for its launch); else the next in turn (rebuilt).
    auto idle = [&](const soft_ctx::GraphSlot &gs) {
        if (!gs.launched) return true;
        const hipError_t q = hipEventQuery(gs.done);
        if (q != hipSuccess) (void)hipGetLastError();  // "not ready" is no error here
        return q == hipSuccess;
    };
    soft_ctx::GraphSlot *slot = nullptr;
    for (auto &gs : c->slots)
        if (!slot && gs.exec && gs.key == key && idle(gs)) slot = &gs;
    for (auto &gs : c->slots)
        if (!slot && !gs.exec) slot = &gs;
    for (auto &gs : c->slots)
        if (!slot && gs.key == key) slot = &gs;
    if (!slot) {
        slot = &c->slots[c->next_slot];
        c->next_slot ^= 1u;
    }
    soft_ctx::GraphSlot &gs = *slot;
    if (gs.launched) HIPCHK(c, hipEventSynchronize(gs.done));  // its previous launch may still read its arguments
    gs.args = rp;
    gs.bargs = build_params(rp);
    void *args[7] = {(void *)&gs.args.ev, (void *)&gs.args.nz, (void *)&gs.args.tm1, (void *)&gs.args.det,
                     (void *)&gs.args.words, (void *)&gs.args.bm, (void *)&gs.args};
    void *bargs[7] = {(void *)&gs.bargs.ev, (void *)&gs.bargs.nz, (void *)&gs.bargs.tm1, (void *)&gs.bargs.det,
                      (void *)&gs.bargs.words, (void *)&gs.bargs.bm, (void *)&gs.bargs};
    hipKernelNodeParams kp, kb;
    std::memset(&kp, 0, sizeof(kp));
    kp.func = const_cast<void *>(kfn);
    kp.gridDim = g;
    kp.blockDim = b;
    kp.sharedMemBytes = (unsigned int)lds;
    kp.kernelParams = args;
    kb = kp;
    kb.func = const_cast<void *>(prefix_kernel(c->bits == 64, s.gt));
    kb.gridDim = dim3((uint32_t)bgrid);
    kb.kernelParams = bargs;
    if (gs.exec && gs.key == key) {
        if (pfx) HIPCHK(c, hipGraphExecKernelNodeSetParams(gs.exec, gs.build, &kb));
        HIPCHK(c, hipGraphExecKernelNodeSetParams(gs.exec, gs.sampler, &kp));
    } else {
        drop_slot(c, gs);
        gs.r_counters = rp.counters;
        gs.r_n = rp.n_vars * (uint32_t)C_COUNT;
        gs.r_next = rp.next;
        void *rargs[3] = {(void *)&gs.r_counters, (void *)&gs.r_n, (void *)&gs.r_next};
        hipKernelNodeParams rk;
        std::memset(&rk, 0, sizeof(rk));
        rk.func = const_cast<void *>(reset_kernel());
        rk.gridDim = dim3(1);
        rk.blockDim = dim3(256);
        rk.kernelParams = rargs;
        hipGraphNode_t rnode = nullptr;
        hipError_t e = hipGraphCreate(&gs.graph, 0);
        if (e == hipSuccess) e = hipGraphAddKernelNode(&rnode, gs.graph, nullptr, 0, &rk);
        hipGraphNode_t before = rnode;
        if (e == hipSuccess && pfx) {
            e = hipGraphAddKernelNode(&gs.build, gs.graph, &rnode, 1, &kb);
            before = gs.build;
        }
        if (e == hipSuccess) e = hipGraphAddKernelNode(&gs.sampler, gs.graph, &before, 1, &kp);
        if (e == hipSuccess) e = hipGraphInstantiate(&gs.exec, gs.graph, nullptr, nullptr, 0);
        if (e == hipSuccess && !gs.done) e = hipEventCreateWithFlags(&gs.done, hipEventDisableTiming);
        if (e != hipSuccess) {
            drop_slot(c, gs);
            return fail(c, SOFT_EDEVICE, std::string("graph build: ") + hipGetErrorString(e));
        }
        gs.key = key;
        ++c->graph_instantiations;
    }
    HIPCHK(c, hipGraphLaunch(gs.exec, stream));
    HIPCHK(c, hipEventRecord(gs.done, stream));
    gs.launched = true;
    ++c->graph_launches;
    return SOFT_OK;
}

int make_params(soft_ctx *c, uint64_t shot0, uint64_t n_shots, uint32_t *outcomes, uint32_t *status, uint32_t *abort_op,
                uint32_t *obs, RunParams &rp) {
    std::memset(&rp, 0, sizeof(rp));
    rp.ev = c->d_ev.p;
    rp.nz = c->d_nz.p;
    rp.tm1 = c->d_tm1.p;
    rp.det = c->d_det.p;
    rp.bm = c->d_bm.p;
    rp.diag = c->d_diag.p;
    rp.ckpts = c->d_ckpt.p;
    rp.defer = c->defer_t ? 1u : 0u;
    rp.speculate = c->speculate ? 1u : 0u;
    rp.gaps = c->d_gap.p;
    rp.noise_mode = (uint32_t)c->noise_mode;
    rp.vars = c->d_vars.p;
    rp.n_vars = (uint32_t)c->vars.size();
    rp.words = c->words_dev;
    rp.phase_tab = c->d_phase;
    rp.word_stride = (uint64_t)c->vars[0].prog.n_noise + c->vars[0].prog.n_meas;
    rp.outcomes = outcomes;
    rp.status = status;
    rp.abort_op = abort_op;
    rp.obs = obs;
    rp.counters = c->d_counters;
    rp.next = c->d_counters + kCounterWords - 2;
    rp.seed = c->seed;
    rp.shot0 = shot0;
    rp.n_shots = n_shots;
    rp.rec_words = rec_words(c);
    rp.support_cap = c->support_cap ? c->support_cap : 0xFFFFFFFFu;
    rp.tile_entries = tile_entries(c);
    rp.tile_bytes = tile_bytes(c);
    const double t = tau_of(c);
    rp.tau2 = t * t;
    rp.grab = 1;
    if (c->keep_n) {
        const uint32_t te = tile_entries(c);
        if ((uint64_t)c->keep_n * te * 16u > kMaxKeepBytes)
            return fail(c, SOFT_ECAPACITY, "kept states would take more than 4 GiB (" + std::to_string(c->keep_n) +
                                               " shots of 2^" + std::to_string(c->kmax) + " entries); keep fewer shots");
        int rc;
        if ((rc = ensure(c, c->d_keep_meta, (size_t)c->keep_n * KM_COUNT)) ||
            (rc = ensure(c, c->d_keep_v, (size_t)c->keep_n * te * 2)))
            return rc;
        rp.keep_meta = c->d_keep_meta.p;
        rp.keep_v = c->d_keep_v.p;
        rp.keep_lo = c->keep_lo;
        rp.keep_n = c->keep_n;
        c->keep_tile = te;
    }
    if (c->trace_n) {
        const uint32_t te = tile_entries(c);
        int rc;
        if ((rc = ensure(c, c->d_trace_meta, (size_t)c->trace_n * KM_COUNT)) ||
            (rc = ensure(c, c->d_trace_v, (size_t)c->trace_n * te * 2)))
            return rc;
        rp.trace_meta = c->d_trace_meta.p;
        rp.trace_v = c->d_trace_v.p;
        rp.trace_shot = c->trace_shot;
        rp.trace_n = c->trace_n;
        c->trace_tile = te;
    }
    return SOFT_OK;
}

int run_impl(soft_ctx *c, uint64_t shot0, uint64_t n_shots, uint32_t *outcomes, uint32_t *status, uint32_t *abort_op,
             uint32_t *obs, hipStream_t stream, const Shape &s, const uint64_t *shot_list = nullptr) {
    RunParams rp;
    int rc = make_params(c, shot0, n_shots, outcomes, status, abort_op, obs, rp);
    if (rc) return rc;
    rp.grab = s.grab;
    rp.shot_list = shot_list;
    if (c->trace_n)  // outside the graph: mark every trace step unwritten
        HIPCHK(c, hipMemsetAsync(c->d_trace_meta.p, 0, (size_t)c->trace_n * KM_COUNT * sizeof(unsigned long long), stream));
    if ((rc = launch(c, rp, s, n_shots, stream))) return rc;
    c->ran = true;
    c->last_counters = c->d_counters;
    c->last_stream = stream;
    c->last_shot0 = shot0;
    c->last_n = n_shots;
    c->last_list = shot_list != nullptr;
    return SOFT_OK;
}

// The event list that produced a dumped state.
const Program &program_of(const soft_ctx *c, const std::vector<unsigned long long> &meta) {
    const Variant &V = c->vars[meta[KM_VAR]];
    return (meta[KM_PROG] || !V.has_fast) ? V.prog : V.fast;
}

// Frame (x/z bits and span basis) in which a dumped state is expressed.
const Frame *frame_of(soft_ctx *c, const std::vector<unsigned long long> &meta, int &rc) {
    const uint64_t v = meta[KM_VAR], term = meta[KM_TERM_EV];
    if (v >= c->vars.size()) {
        rc = fail(c, SOFT_EDEVICE, "corrupt dumped state");
        return nullptr;
    }
    const Program &P = program_of(c, meta);
    if (term >= P.events.size()) {
        rc = fail(c, SOFT_EDEVICE, "corrupt dumped state");
        return nullptr;
    }
    return meta[KM_AFTER] ? &P.after[term] : &P.before[term];
}

const Frame *kept_frame(soft_ctx *c, uint64_t shot, std::vector<unsigned long long> &meta, std::vector<double> &tile, int &rc) {
    rc = SOFT_OK;
    if (!c->ran) { rc = fail(c, SOFT_ESTATE, "no run yet"); return nullptr; }
    if (!c->keep_n || shot < c->keep_lo || shot - c->keep_lo >= c->keep_n ||
        (!c->last_list && (shot < c->last_shot0 || shot - c->last_shot0 >= c->last_n))) {
        rc = fail(c, SOFT_EINVAL, "shot was not kept by the last run (see soft_set_keep)");
        return nullptr;
    }
    hipError_t e = hipStreamSynchronize(c->last_stream);
    if (e != hipSuccess) { rc = fail(c, SOFT_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(e)); return nullptr; }
    const uint64_t kk = shot - c->keep_lo;
    meta.resize(KM_COUNT);
    tile.resize((size_t)c->keep_tile * 2);
    e = hipMemcpy(meta.data(), c->d_keep_meta.p + kk * KM_COUNT, KM_COUNT * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
        e = hipMemcpy(tile.data(), c->d_keep_v.p + kk * (uint64_t)c->keep_tile * 2, tile.size() * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) { rc = fail(c, SOFT_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e)); return nullptr; }
    return frame_of(c, meta, rc);
}

// Coefficients of a dumped state: alpha(j) = a ^ sum_t j_t b_t over the
// frame's span basis; entries below the pruning threshold are left out.
int decode_coeffs(soft_ctx *c, const Frame &f, const std::vector<unsigned long long> &meta,
                  const std::vector<double> &tile, uint64_t *alpha, double *re, double *im, uint32_t cap,
                  uint32_t *count) {
    const uint32_t k = (uint32_t)meta[KM_K];
    if (k != f.basis.size() || (1ull << k) * 2 > tile.size())
        return fail(c, SOFT_EDEVICE, "dumped state does not match the compiled frame");
    const uint64_t a = meta[KM_A];
    const uint32_t cnt = 1u << k;
    double n2 = 0.0;
    for (uint32_t j = 0; j < cnt; ++j) n2 += tile[2 * j] * tile[2 * j] + tile[2 * j + 1] * tile[2 * j + 1];
    const double t = tau_of(c);
    std::vector<std::pair<uint64_t, uint32_t>> keep;
    for (uint32_t j = 0; j < cnt; ++j) {
        const double q = tile[2 * j] * tile[2 * j] + tile[2 * j + 1] * tile[2 * j + 1];
        if (q == 0.0 || q < t * t * n2) continue;
        uint64_t al = a;
        for (uint32_t b = 0; b < k; ++b)
            if ((j >> b) & 1u) al ^= f.basis[b];
        keep.push_back({al, j});
    }
    std::sort(keep.begin(), keep.end());
    *count = (uint32_t)keep.size();
    for (uint32_t i = 0; i < keep.size() && i < cap; ++i) {
        if (alpha) alpha[i] = keep[i].first;
        if (re) re[i] = tile[2 * keep[i].second];
        if (im) im[i] = tile[2 * keep[i].second + 1];
    }
    return SOFT_OK;
}

// Tableau rows of a dumped state: x/z from the frame, signs from the shot.
void decode_tableau(const Frame &f, const std::vector<unsigned long long> &meta, uint64_t *x,
                    uint64_t *z, uint8_t *r) {
    const int n = (int)f.xd.size();
    for (int i = 0; i < n; ++i) {
        uint64_t xd = 0, zd = 0, xs = 0, zs = 0;
        for (int q = 0; q < n; ++q) {
            xd |= ((f.xd[q] >> i) & 1ull) << q;
            zd |= ((f.zd[q] >> i) & 1ull) << q;
            xs |= ((f.xs[q] >> i) & 1ull) << q;
            zs |= ((f.zs[q] >> i) & 1ull) << q;
        }
        if (x) { x[i] = xd; x[n + i] = xs; }
        if (z) { z[i] = zd; z[n + i] = zs; }
        if (r) {
            r[i] = (uint8_t)((meta[KM_RD] >> i) & 1ull);
            r[n + i] = (uint8_t)((meta[KM_RS] >> i) & 1ull);
        }
    }
}

}  // namespace

extern "C" {

int soft_create(soft_ctx **out, int hip_device) {
    if (!out) return SOFT_EINVAL;
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess || hip_device < 0 || hip_device >= ndev) {
        g_create_error = e != hipSuccess ? std::string("hipGetDeviceCount: ") + hipGetErrorString(e) : "no such HIP device";
        return e != hipSuccess ? SOFT_EDEVICE : SOFT_EINVAL;
    }
    soft_ctx *c = new (std::nothrow) soft_ctx();
    if (!c) { g_create_error = "out of host memory"; return SOFT_ECAPACITY; }
    c->device = hip_device;
    auto bad = [&](hipError_t err, const char *what) {
        g_create_error = std::string(what) + ": " + hipGetErrorString(err);
        soft_destroy(c);
        return SOFT_EDEVICE;
    };
    if ((e = hipSetDevice(hip_device)) != hipSuccess) return bad(e, "hipSetDevice");
    if ((e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, hip_device)) != hipSuccess)
        return bad(e, "hipDeviceGetAttribute");
    int lds = 0;
    if ((e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device)) != hipSuccess)
        return bad(e, "hipDeviceGetAttribute");
    c->max_lds_block = lds;
    {
        hipDeviceProp_t prop;
        if ((e = hipGetDeviceProperties(&prop, hip_device)) != hipSuccess) return bad(e, "hipGetDeviceProperties");
        c->arch = prop.gcnArchName;
    }
    if (sampler_set_lds_limit(lds) != hipSuccess) {
        (void)hipGetLastError();
        c->max_lds_block = std::min(lds, 65536);
    }
    if ((e = hipMalloc((void **)&c->d_counters, kCounterWords * sizeof(unsigned long long))) != hipSuccess)
        return bad(e, "hipMalloc");
    if ((e = hipMemset(c->d_counters, 0, kCounterWords * sizeof(unsigned long long))) != hipSuccess) return bad(e, "hipMemset");
    // the static scratch of soft_run_noalloc: its device address on this GPU
    if ((e = scratch_address(hip_device, &c->scratch)) != hipSuccess) return bad(e, "hipGetSymbolAddress(scratch)");
    {
        double tab[32];
        for (int q = 0; q < 16; ++q) {
            tab[q] = std::cos(M_PI * q / 8.0);
            tab[16 + q] = std::sin(M_PI * q / 8.0);
        }
        if ((e = hipMalloc((void **)&c->d_phase, sizeof(tab))) != hipSuccess) return bad(e, "hipMalloc");
        if ((e = hipMemcpy(c->d_phase, tab, sizeof(tab), hipMemcpyHostToDevice)) != hipSuccess) return bad(e, "hipMemcpy");
    }
    *out = c;
    return SOFT_OK;
}

void soft_destroy(soft_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->ran && c->last_stream) (void)hipStreamSynchronize(c->last_stream);
    drop_graph(c);
    release(c->d_ev);
    release(c->d_nz);
    release(c->d_tm1);
    release(c->d_gap);
    release(c->d_det);
    release(c->d_bm);
    release(c->d_diag);
    release(c->d_vars);
    release(c->d_gtile);
    release(c->d_prefix);
    release(c->d_ckpt);
    release(c->d_keep_meta);
    release(c->d_keep_v);
    release(c->d_trace_meta);
    release(c->d_trace_v);
    if (c->d_counters) (void)hipFree(c->d_counters);
    if (c->d_phase) (void)hipFree(c->d_phase);
    for (auto &g : c->slots)
        if (g.done) (void)hipEventDestroy(g.done);
    delete c;
}

const char *soft_last_error(const soft_ctx *c) { return c ? c->err.c_str() : g_create_error.c_str(); }

int soft_load_circuit(soft_ctx *c, const char *text, size_t len) {
    if (!c || (!text && len)) return fail(c, SOFT_EINVAL, "null argument");
    Variant V;
    V.text.assign(text ? text : "", len);
    V.noise = c->noise;
    int rc = compile_variant(c, V);
    if (rc) return rc;
    c->vars.clear();
    c->vars.push_back(std::move(V));
    c->have_text = true;
    c->mixture = false;
    c->dirty = true;
    (void)hipSetDevice(c->device);
    return prepare(c);
}

int soft_load_noise(soft_ctx *c, const soft_noise *m) {
    if (!c || !m) return fail(c, SOFT_EINVAL, "null argument");
    if (c->mixture) return fail(c, SOFT_ESTATE, "a mixture carries one noise model per variant; load it again instead");
    NoiseModel nm;
    nm.p1 = m->p1;
    nm.p2 = m->p2;
    nm.p_idle = m->p_idle;
    nm.p_meas = m->p_meas;
    nm.p_reset = m->p_reset;
    nm.p_mpp = m->p_mpp;
    const double ps[6] = {nm.p1, nm.p2, nm.p_idle, nm.p_meas, nm.p_reset, nm.p_mpp};
    for (double p : ps)
        if (!(p >= 0.0 && p <= 1.0)) return fail(c, SOFT_EINVAL, "noise probability out of [0,1]");
    if (c->have_text) {
        Variant V;
        V.text = c->vars[0].text;
        V.noise = nm;
        int rc = compile_variant(c, V);
        if (rc) return rc;
        c->vars[0] = std::move(V);
        c->dirty = true;
    }
    c->noise = nm;
    if (!c->have_text) return SOFT_OK;
    (void)hipSetDevice(c->device);
    return prepare(c);
}

int soft_load_mixture(soft_ctx *c, uint32_t n_variants, const char *const *texts, const size_t *lens,
                      const soft_noise *models, const uint64_t *shot_ends) {
    if (!c || !texts || !lens || !models || !shot_ends) return fail(c, SOFT_EINVAL, "null argument");
    if (n_variants < 1 || n_variants > kMaxVariants)
        return fail(c, SOFT_EINVAL, "n_variants must be in 1.." + std::to_string(kMaxVariants));
    std::vector<Variant> vs(n_variants);
    for (uint32_t v = 0; v < n_variants; ++v) {
        if (!texts[v] && lens[v]) return fail(c, SOFT_EINVAL, "null circuit text");
        if (shot_ends[v] == 0 || (v > 0 && shot_ends[v] <= shot_ends[v - 1]))
            return fail(c, SOFT_EINVAL, "shot_ends must be positive and strictly increasing");
        const soft_noise &m = models[v];
        NoiseModel nm;
        nm.p1 = m.p1;
        nm.p2 = m.p2;
        nm.p_idle = m.p_idle;
        nm.p_meas = m.p_meas;
        nm.p_reset = m.p_reset;
        nm.p_mpp = m.p_mpp;
        vs[v].text.assign(texts[v] ? texts[v] : "", lens[v]);
        vs[v].noise = nm;
        vs[v].shot_end = shot_ends[v];
        int rc = compile_variant(c, vs[v]);
        if (rc) return fail(c, rc, "variant " + std::to_string(v) + ": " + c->err);
    }
    c->vars = std::move(vs);
    c->have_text = true;
    c->mixture = true;
    c->dirty = true;
    (void)hipSetDevice(c->device);
    return prepare(c);
}

int soft_set_rng(soft_ctx *c, uint64_t seed) {
    if (!c) return SOFT_EINVAL;
    c->seed = seed;
    return SOFT_OK;
}

int soft_set_uniforms(soft_ctx *c, const uint32_t *words_dev, uint64_t n_shots, uint32_t noise_slots, uint32_t meas_slots) {
    if (!c) return SOFT_EINVAL;
    if (!words_dev) {
        c->words_dev = nullptr;
        c->words_n = 0;
        return SOFT_OK;
    }
    if (((uintptr_t)words_dev & 3u) != 0) return fail(c, SOFT_EINVAL, "words_dev must be 4-byte aligned");
    c->words_dev = words_dev;
    c->words_n = n_shots;
    c->words_noise = noise_slots;
    c->words_meas = meas_slots;
    return SOFT_OK;
}

int soft_set_precision(soft_ctx *c, int bits) {
    if (!c) return SOFT_EINVAL;
    if (bits != 32 && bits != 64) return fail(c, SOFT_EINVAL, "coeff_bits must be 32 or 64");
    c->bits = bits;
    return SOFT_OK;
}

int soft_set_prune(soft_ctx *c, double tau) {
    if (!c) return SOFT_EINVAL;
    if (std::isnan(tau) || tau >= 1.0) return fail(c, SOFT_EINVAL, "tau must be < 1");
    c->tau = tau < 0.0 ? -1.0 : tau;
    return SOFT_OK;
}

int soft_set_caps(soft_ctx *c, uint32_t support_cap, uint32_t wpb, uint32_t bpc, uint32_t grab) {
    if (!c) return SOFT_EINVAL;
    if (wpb > 4) return fail(c, SOFT_EINVAL, "waves_per_block must be <= 4");
    if (bpc > kMaxWavesPerCu) return fail(c, SOFT_EINVAL, "blocks_per_cu must be <= 32");
    if (grab > 64) return fail(c, SOFT_EINVAL, "grab must be <= 64");
    c->support_cap = support_cap;
    c->user.wpb = wpb;
    c->user.bpc = bpc;
    c->user.grab = grab;
    return SOFT_OK;
}

int soft_set_speculation(soft_ctx *c, int on) {
    if (!c) return SOFT_EINVAL;
    c->speculate = on != 0;
    return SOFT_OK;
}

int soft_set_shared_prefix(soft_ctx *c, int on) {
    if (!c) return SOFT_EINVAL;
    c->shared_prefix = on != 0;
    return SOFT_OK;
}

int soft_set_deferred_t(soft_ctx *c, int on) {
    if (!c) return SOFT_EINVAL;
    c->defer_t = on != 0;
    return SOFT_OK;
}

int soft_set_noise_mode(soft_ctx *c, int mode) {
    if (!c) return SOFT_EINVAL;
    if (mode < 0 || mode > 1) return fail(c, SOFT_EINVAL, "noise mode must be 0 (a word per slot) or 1 (gap sampling)");
    c->noise_mode = mode;
    return SOFT_OK;
}

int soft_set_tile_memory(soft_ctx *c, int mode) {
    if (!c) return SOFT_EINVAL;
    const int base = mode & 0xff, L = mode >> 8;
    if (mode < 0 || base > 3 || (base != 3 && L != 0) || (L != 0 && (L < (int)kSplitMinLog2 || L > 19)))
        return fail(c, SOFT_EINVAL, "tile memory mode must be 0 (auto), 1 (LDS), 2 (device memory), 3 (split) or "
                                    "256 L + 3 (split with 2^L entries in LDS, 7 <= L <= 19)");
    c->tile_mode = base;
    c->split_log2 = (uint32_t)L;
    return SOFT_OK;
}

int soft_set_keep(soft_ctx *c, uint64_t shot_lo, uint32_t count) {
    if (!c) return SOFT_EINVAL;
    if (count > kMaxKeep) return fail(c, SOFT_ECAPACITY, "at most " + std::to_string(kMaxKeep) + " kept shots");
    c->keep_lo = shot_lo;
    c->keep_n = count;
    return SOFT_OK;
}

int soft_run(soft_ctx *c, uint64_t shot0, uint64_t n_shots, uint32_t *outcomes, uint32_t *status, uint32_t *abort_op,
             uint32_t *obs, void *hip_stream) {
    if (!c) return SOFT_EINVAL;
    if (!status && n_shots) return fail(c, SOFT_EINVAL, "status_dev is required");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = prepare(c);
    if (rc) return rc;
    if (c->words_dev) {
        if (c->mixture) return fail(c, SOFT_EUNSUPPORTED, "explicit words are for a single circuit, not a mixture");
        const Program &P = c->vars[0].prog;
        if (c->words_noise != P.n_noise || c->words_meas != P.n_meas)
            return fail(c, SOFT_EINVAL, "explicit words: expected " + std::to_string(P.n_noise) + " noise and " +
                                            std::to_string(P.n_meas) + " measurement slots per shot");
        if (n_shots > c->words_n) return fail(c, SOFT_EINVAL, "explicit words: fewer rows than shots");
    }
    if (shot0 + n_shots < shot0 || shot0 + n_shots > c->vars.back().shot_end)
        return fail(c, SOFT_EINVAL, "shots beyond the last variant's range");
    if (n_shots == 0) return SOFT_OK;
    Shape s = current_shape(c);
    if ((rc = check_shape(c, s))) return rc;
    return run_impl(c, shot0, n_shots, outcomes, status, abort_op, obs, (hipStream_t)hip_stream, s);
}

int soft_run_noalloc(soft_ctx *c, uint64_t shot0, uint64_t n_shots, uint32_t *outcomes, uint32_t *status,
                     uint32_t *abort_op, uint32_t *obs, void *hip_stream) {
    if (!c) return SOFT_EINVAL;
    if (!status && n_shots) return fail(c, SOFT_EINVAL, "status_dev is required");
    HIPCHK(c, hipSetDevice(c->device));
    if (!c->have_text) return fail(c, SOFT_ESTATE, "no circuit loaded");
    if (c->dirty)  // the soft_load_* calls upload the tables; this stays only after a failed upload
        return fail(c, SOFT_ESTATE, "the circuit's device tables are not uploaded (the last soft_load_* failed)");
    if (c->keep_n || c->trace_n)
        return fail(c, SOFT_EUNSUPPORTED, "kept states and traces use buffers the library allocates; turn them off "
                                          "(soft_set_keep(ctx, 0, 0), soft_set_trace(ctx, 0, 0)) for soft_run_noalloc");
    if (c->words_dev) {
        if (c->mixture) return fail(c, SOFT_EUNSUPPORTED, "explicit words are for a single circuit, not a mixture");
        const Program &P = c->vars[0].prog;
        if (c->words_noise != P.n_noise || c->words_meas != P.n_meas)
            return fail(c, SOFT_EINVAL, "explicit words: expected " + std::to_string(P.n_noise) + " noise and " +
                                            std::to_string(P.n_meas) + " measurement slots per shot");
        if (n_shots > c->words_n) return fail(c, SOFT_EINVAL, "explicit words: fewer rows than shots");
    }
    if (shot0 + n_shots < shot0 || shot0 + n_shots > c->vars.back().shot_end)
        return fail(c, SOFT_EINVAL, "shots beyond the last variant's range");
    if (n_shots == 0) return SOFT_OK;
    Shape s = current_shape(c);
    int rc = check_shape(c, s);
    if (rc) return rc;
    RunParams rp;
    if ((rc = make_params(c, shot0, n_shots, outcomes, status, abort_op, obs, rp))) return rc;
    rp.grab = s.grab;
    set_wave_layout(c, s, rp);
    // counters and cursor, then (device-memory tiles) one slab per wave, all
    // in this device's static scratch; with slabs the grid shrinks to what
    // the scratch holds (the kernel is persistent, so fewer waves take more
    // shots each)
    rp.counters = reinterpret_cast<unsigned long long *>(c->scratch);
    rp.next = rp.counters + kCounterWords - 2;
    // shared-prefix slots when they fit their part of the scratch (without
    // them every shot runs from the start: the same results)
    const bool pfx = use_prefix(c) && (uint64_t)c->n_ckpt * prefix_stride(c) <= kScratchPrefixBytes;
    rp.prefix = pfx ? c->scratch + kScratchCounterBytes : nullptr;
    rp.prefix_stride = pfx ? prefix_stride(c) : 0u;
    uint64_t grid = grid_blocks(c, s, n_shots);
    if (s.gt != TM_LDS) {
        const uint64_t slab = (uint64_t)s.wpb * slab_bytes(c, s);
        const uint64_t fit = kScratchTileBytes / slab;
        if (fit == 0)
            return fail(c, SOFT_ECAPACITY, "device-memory tiles of one block need " + std::to_string(slab) +
                                               " bytes; soft_run_noalloc's scratch holds " +
                                               std::to_string(kScratchTileBytes) + " (span dimension " +
                                               std::to_string(c->kmax) + ")");
        grid = std::min<uint64_t>(grid, fit);
        rp.gtile = c->scratch + kScratchCounterBytes + kScratchPrefixBytes;
    }
    const hipStream_t stream = (hipStream_t)hip_stream;
    HIPCHK(c, launch_reset(rp.counters, rp.n_vars * (uint32_t)C_COUNT, rp.next, stream));
    if (pfx)
        HIPCHK(c, launch_prefix_build(build_params(rp), c->bits == 64,
                                 dim3((uint32_t)std::min<uint64_t>(grid, (2ull * rp.n_vars + s.wpb - 1) / s.wpb)),
                                 dim3(64u * s.wpb), (size_t)s.wpb * wave_bytes(c, s), stream));
    HIPCHK(c, launch_sampler(rp, c->bits == 64, dim3((uint32_t)grid), dim3(64u * s.wpb),
                             (size_t)s.wpb * wave_bytes(c, s), stream));
    c->ran = true;
    c->last_counters = rp.counters;
    c->last_stream = stream;
    c->last_shot0 = shot0;
    c->last_n = n_shots;
    c->last_list = false;
    return SOFT_OK;
}

namespace {
// Sum of the counter rows [v0, v1) (maximum for the norm deviation).
int read_rows(soft_ctx *c, uint32_t v0, uint32_t v1, soft_counters *out) {
    if (!c->ran) return fail(c, SOFT_ESTATE, "no run yet");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->last_stream));
    std::vector<unsigned long long> h((size_t)(v1 - v0) * C_COUNT);
    HIPCHK(c, hipMemcpy(h.data(), c->last_counters + (size_t)v0 * C_COUNT, h.size() * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost));
    std::memset(out, 0, sizeof(*out));
    double dev = 0.0;
    for (uint32_t v = 0; v < v1 - v0; ++v) {
        const unsigned long long *r = h.data() + (size_t)v * C_COUNT;
        out->shots += r[C_SHOTS];
        out->passed += r[C_PASSED];
        out->discarded += r[C_DISCARDED];
        out->overflow += r[C_OVERFLOW];
        out->numeric += r[C_NUMERIC];
        out->logical_errors += r[C_LOGICAL];
        out->entries_t += r[C_ENTRIES_T];
        out->entries_m += r[C_ENTRIES_M];
        out->noise_slots += r[C_NOISE];
        out->events += r[C_EVENTS];
        out->restarts += r[C_RESTARTS];
        out->prefix_shots += r[C_PREFIX];
        out->redo_shots += r[C_REDO];
        for (int b = 0; b < 16; ++b) out->support_hist[b] += r[C_HIST0 + b];
        double d;
        std::memcpy(&d, &r[C_NORMDEV_BITS], sizeof(double));
        dev = std::max(dev, d);
    }
    out->max_norm_dev = dev;
    return SOFT_OK;
}
}  // namespace

int soft_run_list(soft_ctx *c, const uint64_t *shots_dev, uint64_t n_shots, uint32_t *outcomes, uint32_t *status,
                  uint32_t *abort_op, uint32_t *obs, void *hip_stream) {
    if (!c) return SOFT_EINVAL;
    if (!status && n_shots) return fail(c, SOFT_EINVAL, "status_dev is required");
    if (!shots_dev && n_shots) return fail(c, SOFT_EINVAL, "shots_dev is required");
    if (((uintptr_t)shots_dev & 7u) != 0) return fail(c, SOFT_EINVAL, "shots_dev must be 8-byte aligned");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = prepare(c);
    if (rc) return rc;
    if (c->words_dev) return fail(c, SOFT_EUNSUPPORTED, "explicit words are for soft_run");
    if (n_shots == 0) return SOFT_OK;
    Shape s = current_shape(c);
    if ((rc = check_shape(c, s))) return rc;
    return run_impl(c, 0, n_shots, outcomes, status, abort_op, obs, (hipStream_t)hip_stream, s, shots_dev);
}

int soft_read_counters(soft_ctx *c, soft_counters *out) {
    if (!c || !out) return fail(c, SOFT_EINVAL, "null argument");
    return read_rows(c, 0, (uint32_t)c->vars.size(), out);
}

int soft_read_variant_counters(soft_ctx *c, uint32_t variant, soft_counters *out) {
    if (!c || !out) return fail(c, SOFT_EINVAL, "null argument");
    if (variant >= c->vars.size()) return fail(c, SOFT_EINVAL, "no such variant");
    return read_rows(c, variant, variant + 1, out);
}

int soft_read_coeffs(soft_ctx *c, uint64_t shot, uint64_t *alpha, double *re, double *im, uint32_t cap, uint32_t *count) {
    if (!c || !count) return fail(c, SOFT_EINVAL, "null argument");
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<unsigned long long> meta;
    std::vector<double> tile;
    int rc;
    const Frame *f = kept_frame(c, shot, meta, tile, rc);
    if (!f) return rc;
    return decode_coeffs(c, *f, meta, tile, alpha, re, im, cap, count);
}

int soft_read_tableau(soft_ctx *c, uint64_t shot, uint64_t *x, uint64_t *z, uint8_t *r) {
    if (!c) return SOFT_EINVAL;
    HIPCHK(c, hipSetDevice(c->device));
    std::vector<unsigned long long> meta;
    std::vector<double> tile;
    int rc;
    const Frame *f = kept_frame(c, shot, meta, tile, rc);
    if (!f) return rc;
    decode_tableau(*f, meta, x, z, r);
    return SOFT_OK;
}

int soft_set_trace(soft_ctx *c, uint64_t shot, uint32_t steps) {
    if (!c) return SOFT_EINVAL;
    if (steps > 65536) return fail(c, SOFT_ECAPACITY, "at most 65536 traced steps");
    c->trace_shot = shot;
    c->trace_n = steps;
    return SOFT_OK;
}

int soft_read_trace(soft_ctx *c, uint32_t step, uint64_t info[6], uint64_t *x, uint64_t *z, uint8_t *r,
                    uint64_t *alpha, double *re, double *im, uint32_t cap, uint32_t *count) {
    if (!c || !info) return fail(c, SOFT_EINVAL, "null argument");
    if (!c->ran || !c->trace_n || !c->trace_tile) return fail(c, SOFT_ESTATE, "no traced run");
    if (step >= c->trace_n) return fail(c, SOFT_EINVAL, "step beyond the traced range");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->last_stream));
    std::vector<unsigned long long> meta(KM_COUNT);
    std::vector<double> tile((size_t)c->trace_tile * 2);
    HIPCHK(c, hipMemcpy(meta.data(), c->d_trace_meta.p + (uint64_t)step * KM_COUNT, KM_COUNT * sizeof(unsigned long long),
                        hipMemcpyDeviceToHost));
    for (int i = 0; i < 6; ++i) info[i] = 0;
    if (count) *count = 0;
    if (meta[KM_VALID] != kStateValid) return SOFT_OK;
    HIPCHK(c, hipMemcpy(tile.data(), c->d_trace_v.p + (uint64_t)step * c->trace_tile * 2, tile.size() * sizeof(double),
                        hipMemcpyDeviceToHost));
    int rc = SOFT_OK;
    const Frame *f = frame_of(c, meta, rc);
    if (!f) return rc;
    const Event &E = program_of(c, meta).events[meta[KM_TERM_EV]];
    info[0] = 1;
    info[1] = (meta[KM_STATUS] != ST_PASSED && meta[KM_ABORT] != 0xFFFFFFFFull) ? meta[KM_ABORT] : E.src;
    info[2] = meta[KM_STATUS];
    info[3] = meta[KM_K];
    info[4] = meta[KM_NRM2];
    info[5] = (meta[KM_STATUS] != ST_PASSED || E.kind == EV_END) ? 1 : 0;
    decode_tableau(*f, meta, x, z, r);
    uint32_t cnt = 0;
    rc = decode_coeffs(c, *f, meta, tile, alpha, re, im, cap, &cnt);
    if (count) *count = cnt;
    return rc;
}

namespace {
void program_info(const Program &P, uint64_t info[8]) {
    info[0] = (uint64_t)P.n;
    info[1] = P.n_rec;
    info[2] = P.n_noise;
    info[3] = P.n_meas;
    info[4] = P.n_obs;
    info[5] = P.events.size();
    info[6] = P.kmax;
    info[7] = (P.n_rec + 31u) / 32u;
}
}  // namespace

int soft_circuit_info(soft_ctx *c, uint64_t info[8]) {
    if (!c || !info) return fail(c, SOFT_EINVAL, "null argument");
    (void)hipSetDevice(c->device);
    int rc = prepare(c);
    if (rc) return rc;
    for (int i = 0; i < 8; ++i) info[i] = 0;
    for (const Variant &V : c->vars) {
        uint64_t vi[8];
        program_info(V.prog, vi);
        for (int i = 0; i < 8; ++i) info[i] = std::max(info[i], vi[i]);
    }
    return SOFT_OK;
}

int soft_variant_info(soft_ctx *c, uint32_t variant, uint64_t info[8]) {
    if (!c || !info) return fail(c, SOFT_EINVAL, "null argument");
    if (!c->have_text) return fail(c, SOFT_ESTATE, "no circuit loaded");
    if (variant >= c->vars.size()) return fail(c, SOFT_EINVAL, "no such variant");
    program_info(c->vars[variant].prog, info);
    return SOFT_OK;
}

int soft_graph_info(soft_ctx *c, uint64_t out[2]) {
    if (!c || !out) return fail(c, SOFT_EINVAL, "null argument");
    out[0] = c->graph_instantiations;
    out[1] = c->graph_launches;
    return SOFT_OK;
}

int soft_launch_shape(soft_ctx *c, uint32_t out[5]) {
    if (!c || !out) return fail(c, SOFT_EINVAL, "null argument");
    (void)hipSetDevice(c->device);
    int rc = prepare(c);
    if (rc) return rc;
    Shape s = current_shape(c);
    out[0] = s.wpb;
    out[1] = s.bpc;
    out[2] = s.grab;
    out[3] = wave_bytes(c, s);
    out[4] = s.gt;
    return SOFT_OK;
}

int soft_autotune(soft_ctx *c, uint64_t sample_shots, void *hip_stream) {
    if (!c) return SOFT_EINVAL;
    if (sample_shots == 0) return fail(c, SOFT_EINVAL, "sample_shots must be > 0");
    HIPCHK(c, hipSetDevice(c->device));
    int rc = prepare(c);
    if (rc) return rc;
    if (c->words_dev) return fail(c, SOFT_ESTATE, "autotune runs on Philox draws; clear explicit uniforms first");
    uint32_t *d_status_holder = nullptr;
    hipStream_t st = (hipStream_t)hip_stream;
    // The sample: the first shots of each variant's range, sample_shots in all,
    // as one shot list so that every timing is a single launch.
    std::vector<uint64_t> list;
    {
        const uint64_t per = std::max<uint64_t>(1, sample_shots / c->vars.size());
        uint64_t lo = 0;
        for (const Variant &V : c->vars) {
            const uint64_t n = std::min<uint64_t>(per, V.shot_end - lo);
            for (uint64_t i = 0; i < n; ++i) list.push_back(lo + i);
            lo = V.shot_end;
        }
    }
    uint32_t *d_status = nullptr;
    uint64_t *d_list = nullptr;
    HIPCHK(c, hipMalloc((void **)&d_status, list.size() * sizeof(uint32_t)));
    d_status_holder = d_status;
    if (hipMalloc((void **)&d_list, list.size() * sizeof(uint64_t)) != hipSuccess ||
        hipMemcpy(d_list, list.data(), list.size() * sizeof(uint64_t), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipFree(d_status);
        if (d_list) (void)hipFree(d_list);
        return fail(c, SOFT_EDEVICE, "autotune: could not stage the shot list");
    }
    auto sample_pass = [&](const Shape &s) {
        return run_impl(c, 0, list.size(), nullptr, d_status_holder, nullptr, nullptr, st, s, d_list);
    };
    hipEvent_t t0 = nullptr, t1 = nullptr;
    HIPCHK(c, hipEventCreate(&t0));
    HIPCHK(c, hipEventCreate(&t1));
    const uint32_t keep_n = c->keep_n;
    c->keep_n = 0;
    // Candidates: the default shape first, then a grid of shapes per tile
    // placement.  Each is run once untimed and twice timed; the faster timing
    // counts, so one noisy launch cannot pick a worse shape than the default.
    std::vector<Shape> cands;
    cands.push_back(default_shape(c));
    const uint32_t wpbs[3] = {1, 2, 4};
    const uint32_t grabs[2] = {16, 64};
    // placements: the one asked for; in auto mode LDS (when it fits), device
    // memory, and splits whose LDS part is 1/2, 1/4 or 1/8 of the tile
    std::vector<Shape> places;
    if (c->tile_mode != 0) {
        places.push_back(placement(c));
        if (places[0].gt == TM_SPLIT && !c->split_log2)  // other LDS parts of the split
            for (uint32_t d = 1; d <= 3; ++d) {
                Shape p = places[0];
                p.lds_log2 = c->kmax - d;
                if (p.lds_log2 >= kSplitMinLog2 && p.lds_log2 != places[0].lds_log2) places.push_back(p);
            }
    } else {
        const Shape lds_p;  // the whole tile in LDS, when a block holds it
        if (wave_bytes(c, lds_p) <= (uint32_t)c->max_lds_block) places.push_back(lds_p);
        Shape m;
        m.gt = TM_MEM;
        places.push_back(m);
        for (uint32_t d = 1; d <= 3 && split_possible(c); ++d) {
            Shape p;
            p.gt = TM_SPLIT;
            p.lds_log2 = c->kmax - d;
            if (p.lds_log2 >= kSplitMinLog2) places.push_back(p);
        }
    }
    for (const Shape &place : places) {
        const uint32_t wb = wave_bytes(c, place);
        for (uint32_t wpb : wpbs) {
            if (wpb * wb > (uint32_t)c->max_lds_block) continue;
            const uint32_t cap = place.gt == TM_MEM ? kMemTileWavesPerCu : kMaxWavesPerCu;
            const uint32_t occ = std::max<uint32_t>(1u, std::min<uint32_t>(kLdsPerCu / (wpb * wb), cap / wpb));
            std::vector<uint32_t> bpcs;
            for (uint32_t d : {4u, 2u, 1u}) {
                uint32_t v = std::max<uint32_t>(1u, occ / d);
                if (std::find(bpcs.begin(), bpcs.end(), v) == bpcs.end()) bpcs.push_back(v);
            }
            for (uint32_t bpc : bpcs)
                for (uint32_t grab : grabs) {
                    Shape sh = place;
                    sh.wpb = wpb;
                    sh.bpc = bpc;
                    sh.grab = grab;
                    cands.push_back(sh);
                }
        }
    }
    Shape best = cands[0];
    float best_ms = 1e30f;
    for (const Shape &sh : cands) {
        if (check_shape(c, sh) != SOFT_OK) continue;
        rc = sample_pass(sh);  // untimed: graph capture, caches
        float ms = 1e30f;
        for (int rep = 0; rep < 2 && !rc; ++rep) {
            float t = 0.0f;
            hipError_t e = hipEventRecord(t0, st);
            if (e == hipSuccess) rc = sample_pass(sh);
            if (!rc && e == hipSuccess) e = hipEventRecord(t1, st);
            if (!rc && e == hipSuccess) e = hipEventSynchronize(t1);
            if (!rc && e == hipSuccess) e = hipEventElapsedTime(&t, t0, t1);
            if (!rc && e != hipSuccess) rc = fail(c, SOFT_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
            if (!rc) ms = std::min(ms, t);
        }
        if (rc) break;
        if (ms < best_ms) {
            best_ms = ms;
            best = sh;
        }
    }
    c->keep_n = keep_n;
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    (void)hipStreamSynchronize(st);
    (void)hipFree(d_status);
    (void)hipFree(d_list);
    if (rc) return rc;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned[tune_key(c)] = best;
    }
    c->ran = false;  // counters of the last sample run are not a user run
    return SOFT_OK;
}

}  // extern "C"
