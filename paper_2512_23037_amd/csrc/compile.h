// compile.h -- circuit text -> Program (events + noise table + frames).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "program.h"

namespace soft {

struct NoiseModel {
    double p1 = 0, p2 = 0, p_idle = 0, p_meas = 0, p_reset = 0, p_mpp = 0;
};

// Shot-independent part of the state at one point of the circuit: the x/z
// bits of the tableau stored by column (for qubit q, the rows whose x bit q is
// set, as a destabilizer word and a stabilizer word) and the span basis.
struct Frame {
    std::vector<uint64_t> xd, xs, zd, zs;
    std::vector<uint64_t> basis;
};

struct Program {
    int n = 0;
    uint32_t n_src = 0, n_rec = 0, n_noise = 0, n_meas = 0, n_obs = 0;
    uint32_t kmax = 0;
    std::vector<Event> events;
    std::vector<NoiseLoc> noise;
    std::vector<uint32_t> noise_tm1;  // per slot: thr-1 (hit iff word <= it), padded
    std::vector<double> noise_p;      // per slot: probability
    std::vector<uint32_t> gap;        // gap sampling: [g - 1] = floor(q^g 2^32), g = 1..n_noise
    double gap_pmax = 0.0;            //   p_max (q = 1 - p_max); 0 without noise
    std::vector<uint32_t> det_pairs;  // (record word, mask) pairs
    std::vector<BatchMember> batch;   // members of side-by-side measurement runs
    std::vector<DiagInfo> diag;       // diagonal gates (EV_DIAG events point here)
    std::vector<Frame> before;        // frame when event e starts
    std::vector<Frame> after;         // frame when event e has finished
    uint64_t hash = 0;                // of the text and the noise model
    // Checkpoints of the noiseless trajectory, by increasing event and noise
    // slot: a shot with no noise hit among slots [0, nz) reaches event ev in
    // the same state as every other such shot.
    std::vector<Checkpoint> ckpts;
};

struct CompileError {
    int line;
    std::string msg;
};

// Largest span dimension the compiler accepts.
constexpr uint32_t kMaxSpanDim = 20;

// Throws CompileError.  With `speculate`, the event list also carries DROP
// events that return the span to its size before a run of T gates once all of
// them have met their inverses (the full list has none; both assign the same
// noise and measurement slots and records).
void compile_circuit(const std::string &text, const NoiseModel &nm, Program &out, bool speculate = false);

}  // namespace soft
