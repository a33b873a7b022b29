// sampler.h -- launch interface of the shot-sampling kernels (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "program.h"

namespace soft {

// Where a wave's coefficient tile lives: all in LDS, all in a slab of device
// memory, or split (the low lds_entries entries in LDS, the rest in a slab).
enum TileMode : uint32_t { TM_LDS = 0, TM_MEM = 1, TM_SPLIT = 2 };

struct RunParams {
    const Event *ev;
    const NoiseLoc *nz;
    const uint32_t *tm1;      // per noise slot: threshold - 1 (padded to 256)
    const uint32_t *gaps;     // gap sampling tables of the variants (VariantDesc::gap_off)
    const uint32_t *det;      // DETECTOR/OBSERVABLE (word, mask) pairs
    const BatchMember *bm;    // members of side-by-side measurement runs
    const DiagInfo *diag;     // diagonal gates (EV_DIAG)
    const VariantDesc *vars;  // shot ranges of the circuits in this run
    const uint32_t *words;    // explicit uniforms [n_shots][word_stride] or null
    const uint64_t *shot_list;  // global shot index of each run position, or null (shot0 + i)
    const double *phase_tab;  // cos(k pi/8) for k = 0..15, then sin(k pi/8)
    uint32_t *outcomes;       // [rec_words][n_shots] or null
    uint32_t *status;         // [n_shots]
    uint32_t *abort_op;       // [n_shots] or null
    uint32_t *obs;            // [n_shots] or null
    unsigned long long *counters;  // [variants][C_COUNT]
    unsigned long long *next;      // work-stealing cursor
    unsigned long long *keep_meta; // [keep_n][KM_COUNT] or null
    double *keep_v;                // [keep_n][tile_entries][2] or null
    unsigned long long *trace_meta;  // [trace_n][KM_COUNT] or null
    double *trace_v;                 // [trace_n][tile_entries][2] or null
    void *gtile;              // device-memory slabs, one per wave (TM_MEM: tile_entries entries; TM_SPLIT:
                              // tile_entries - lds_entries), or null (TM_LDS)
    const Checkpoint *ckpts;  // checkpoint table (VariantDesc::ck_off / ck_cnt index it)
    unsigned char *prefix;    // checkpoint state slots, one per table entry (CkptState, record, tile), or
                              // null (every shot runs from the start)
    uint64_t trace_shot;
    uint64_t seed, shot0, n_shots, keep_lo;
    uint64_t word_stride;
    uint32_t keep_n, n_vars, rec_words, support_cap;
    uint32_t trace_n, pad_;
    uint32_t wave_bytes, tile_bytes, tile_entries, grab;
    uint32_t rec_off;         // byte offset of the record in a wave's LDS slot (LDS tiles; 0 when the
                              // record fits in scalar registers and never touches LDS)
    uint32_t speculate;       // 1: run the speculative event list first
    uint32_t noise_mode;      // 0: a word per noise slot, 1: gap sampling (ignored with explicit words)
    uint32_t tile_mode;       // TileMode
    uint32_t lds_entries;     // TM_SPLIT: tile entries in LDS (a power of two, 128 .. tile_entries / 2)
    uint32_t prefix_build;    // 1: the build launch -- item i runs variant i / 2's list (i odd: the full
                              // list) without noise up to its last checkpoint, writing each checkpoint's
                              // slot
    uint32_t prefix_stride;   // bytes per prefix slot
    uint32_t defer;           // 1: skip deferrable T runs (EVF_DEFER) until an event needs their tile
    double tau2;              // pruning threshold squared
};

// Zero `n` counters and the two work cursors next[0] (sampler) and next[1]
// (prefix build): a kernel, so it can live in a graph.
hipError_t launch_reset(unsigned long long *counters, uint32_t n, unsigned long long *next, hipStream_t stream);

// The persistent sampler: grid x block threads, `lds` bytes of dynamic LDS.
hipError_t launch_sampler(const RunParams &p, bool fp64, dim3 grid, dim3 block, size_t lds, hipStream_t stream);

// Host handles of the kernels, for graphs built from explicit kernel nodes:
// the sampler instantiation for a precision, noise source and tile mode
// (arguments: ev, nz, tm1, det, words, bm, then the RunParams by value), and
// the counter reset (arguments: counters, n, next; one block of 256 threads).
const void *sampler_kernel(bool fp64, uint32_t noise_source, uint32_t tile_mode, bool lean);
// Whether a launch with these parameters runs the lean kernel (no kept
// states, no trace, no support cap, no shot list, no explicit words; see
// sampler.hip).
bool sampler_lean(const RunParams &p);
const void *reset_kernel();
// The shared-prefix build kernel for a precision and tile mode (arguments as
// the sampler's, with RunParams::prefix_build set), and a direct launch of it.
const void *prefix_kernel(bool fp64, uint32_t tile_mode);
hipError_t launch_prefix_build(const RunParams &p, bool fp64, dim3 grid, dim3 block, size_t lds, hipStream_t stream);

// Blocks of `block` threads with `lds` bytes of dynamic LDS that one CU keeps
// resident (registers and LDS).
hipError_t sampler_occupancy(bool fp64, uint32_t noise_source, uint32_t tile_mode, int block, size_t lds,
                             int *blocks_per_cu);

// Raise the dynamic-LDS limit of every sampler instantiation (called once).
hipError_t sampler_set_lds_limit(int bytes);

// Device scratch of the allocation-free run (soft_run_noalloc): a static
// device array per GPU, held until the process ends.  The counter rows and
// the work cursor take the first kScratchCounterBytes; device-memory tiles
// take the rest, one slab per resident wave.
constexpr size_t kScratchCounterBytes = 64u << 10;
constexpr size_t kScratchPrefixBytes = 4u << 20;
constexpr size_t kScratchTileBytes = 32u << 20;
constexpr size_t kScratchBytes = kScratchCounterBytes + kScratchPrefixBytes + kScratchTileBytes;

// Device address of that array on `device` (looked up once per device with
// the device current, then cached).  Layout: counters and cursors,
// checkpoint slots (kScratchPrefixBytes), tile slabs.  Host code must use this address, never
// the array's own name, which on the host is only a stand-in.
hipError_t scratch_address(int device, unsigned char **out);

}  // namespace soft
