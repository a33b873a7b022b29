// oracle.cpp -- plain CPU FP64 reference for generalized-stabilizer (GS) shot
// sampling of noisy Clifford+T circuits (arXiv 2512.23037).
//
// TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
// CPU-baseline leg of the benchmark to check the GPU sampler.  It shares no
// code with the product library.  Everything here is written for clarity, not
// speed: a per-shot literal tableau, a std::map coefficient vector, and one
// Philox evaluation per random word.
//
// Conventions fixed where the paper is silent (each one is a reading of the
// paper, listed with its reason in the design notes of the repository):
//   * signs are tracked on all 2n rows (needed for Theorem 1 part 1: v is
//     unchanged by a Clifford only if the destabilizer signs move with it);
//   * T keeps the exact global phase e^{+-i pi/8} of Eqs. 1-2;
//   * a measurement with beta != 0 pivots on the lowest anticommuting
//     stabilizer (Aaronson-Gottesman) and the new stabilizer state is
//     sqrt(2) * Pi_m |psi_S>;
//   * outcome +1 (record bit 0) iff u < p0 with u = (w + 1/2) 2^-32;
//   * entries with |v|^2 < tau^2 * sum|v|^2 are dropped after every T and
//     measurement;
//   * noise: DEP1 picks X/Y/Z with p/3 each, DEP2 one of the 15 non-identity
//     two-qubit Paulis with p/15 each, XERR an X, ZERR a Z, FLIP a classical
//     record flip; X-basis readouts and resets (MX, RX, MRX) take ZERR where
//     Z-basis ones take XERR.
#include "oracle.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <sstream>
#include <string>
#include <thread>
#include <vector>

typedef std::complex<double> cplx;

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10, written from Salmon et al., "Parallel random numbers: as easy
// as 1, 2, 3", SC'11: ten rounds of two 32x32->64 multiplies with the round
// key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
void philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod0 = (uint64_t)0xD2511F53u * c0;
        uint64_t prod1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(prod0 >> 32), lo0 = (uint32_t)prod0;
        uint32_t hi1 = (uint32_t)(prod1 >> 32), lo1 = (uint32_t)prod1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Word number `slot` of per-shot stream `stream` (0 = noise, 1 = measurement):
// counter = (slot / 4, shot low, shot high, stream), key = seed, word slot % 4.
uint32_t philox_word(uint64_t seed, uint64_t shot, uint32_t stream, uint64_t slot) {
    uint32_t ctr[4] = {(uint32_t)(slot >> 2), (uint32_t)shot, (uint32_t)(shot >> 32), stream};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    philox4x32_10(ctr, key, out);
    return out[slot & 3];
}

// ---------------------------------------------------------------------------
// Circuit representation after parsing and noise insertion.
// ---------------------------------------------------------------------------
enum Kind {
    K_H, K_S, K_SDG, K_X, K_Y, K_Z, K_CX, K_CZ, K_T, K_TDG, K_HXY, K_HNXY,
    K_M, K_MPP, K_R, K_MX, K_RX, K_MR, K_MRX,
    K_DEP1, K_DEP2, K_XERR, K_ZERR, K_FLIP,
    K_DETECTOR, K_OBSERVABLE,
    K_FEEDBACK,  // Pauli `b` (1 X, 2 Y, 3 Z) on qubit a when its condition holds
    K_DIAG       // diagonal gate: phase e^{i phi[x]} on basis state x of qubits qs (bit j = qubit qs[j]),
                 // when its condition holds (always, if it has none)
};

struct Op {
    Kind kind;
    int a = -1, b = -1;       // qubits
    uint64_t px = 0, pz = 0;  // MPP Pauli string (sign +)
    std::vector<int> recs;    // DETECTOR / OBSERVABLE record indices
    int expect = 0;           // DETECTOR / OBSERVABLE constant
    uint64_t thr = 0;         // noise threshold floor(p * 2^32)
    double p = 0.0;           // noise probability
    int src = -1;             // index of the source op it came from
    int slot = -1;            // noise slot (noise ops) or measurement slot
    int rec = -1;             // record written (M, MPP) or flipped (FLIP)
    int obs = -1;             // observable index
    std::vector<int> qs;      // DIAG qubits
    std::vector<double> phi;  // DIAG phases, 2^|qs| of them
    // Classical condition of FEEDBACK / DIAG on earlier record bits: their
    // XOR, or (cond_and) their AND.  Empty: unconditional.
    std::vector<int> cond;
    bool cond_and = false;
};

}  // namespace

struct oracle_circuit {
    int n = 0;
    int n_src = 0, n_rec = 0, n_noise = 0, n_meas = 0, n_obs = 0;
    std::vector<Op> ops;
    // Noise sampling: mode 0 draws one word per noise slot; mode 1 draws
    // geometric gaps between candidate slots (see gap_of) and thins them.
    int noise_mode = 0;
    std::vector<uint64_t> gap_thr;   // [g] = floor(q^g 2^32), g = 0..n_noise, q = 1 - p_max
    std::vector<uint64_t> accept;    // per slot: floor(p / p_max * 2^32)
};

namespace {

struct ParseError {
    int line;
    std::string msg;
};

uint64_t threshold_of(double p) {
    return (uint64_t)std::floor(p * 4294967296.0);
}

int to_int(const std::string &s, int line) {
    if (s.empty()) throw ParseError{line, "empty integer"};
    for (char ch : s)
        if (ch < '0' || ch > '9') throw ParseError{line, "bad integer '" + s + "'"};
    if (s.size() > 9) throw ParseError{line, "integer too large '" + s + "'"};
    return std::stoi(s);
}

double to_prob(const std::string &s, int line) {
    char *end = nullptr;
    double p = std::strtod(s.c_str(), &end);
    if (end == s.c_str() || *end != '\0') throw ParseError{line, "bad probability '" + s + "'"};
    if (!(p >= 0.0 && p <= 1.0)) throw ParseError{line, "probability out of [0,1]"};
    return p;
}

// Names of the diagonal gates taken by the Z-string expansion when bare (the
// Clifford and T names join them under IF).
bool is_diag_name(const std::string &g) {
    return g == "CCZ" || g == "CCX" || g == "CS" || g == "CSDG" || g == "CPHASE" || g == "RZ" || g == "DIAG";
}
bool is_cond_diag_name(const std::string &g) {
    return is_diag_name(g) || g == "S" || g == "SDG" || g == "T" || g == "TDG" || g == "CZ";
}

// Parse the circuit text and lower it: every noise location with p > 0 gets a
// noise slot, every M / MPP / R a measurement slot, every M / MPP a record.
void compile(const char *text, const oracle_noise &nm, oracle_circuit &c) {
    std::istringstream in(text);
    std::string raw;
    int line = 0;
    bool have_qubits = false;
    std::vector<char> active;  // qubits touched since the last TICK

    auto qubit = [&](const std::string &s) {
        int q = to_int(s, line);
        if (q >= c.n) throw ParseError{line, "qubit out of range"};
        return q;
    };
    auto add_noise = [&](Kind k, double p, int a, int b, int src) {
        if (p <= 0.0) return;
        Op o;
        o.kind = k; o.a = a; o.b = b; o.thr = threshold_of(p); o.p = p; o.src = src;
        o.slot = c.n_noise++;
        c.ops.push_back(o);
    };
    auto add_flip = [&](double p, int rec, int src) {
        if (p <= 0.0) return;
        Op o;
        o.kind = K_FLIP; o.rec = rec; o.thr = threshold_of(p); o.p = p; o.src = src;
        o.slot = c.n_noise++;
        c.ops.push_back(o);
    };

    auto hgate = [&](int q, int src) {
        Op h;
        h.kind = K_H; h.a = q; h.src = src;
        c.ops.push_back(h);
    };
    // Diagonal gates, each one multiplying computational basis state x of its
    // qubits (bit j of x = qubit qs[j]) by e^{i phi[x]}:
    //   S / SDG q: phi = +-pi/2 where q = 1;  T / TDG q: +-pi/4 (T = diag(1, e^{i pi/4}));
    //   CZ a b: phi = pi where a = b = 1;
    //   CCZ a b c: phi = pi where a = b = c = 1;  CCX = H_c CCZ H_c;
    //   CS a b / CSDG a b: phi = +-pi/2 where a = b = 1;
    //   CPHASE theta a b: phi = theta where a = b = 1;
    //   RZ theta q: exp(-i theta Z / 2), phi = (-theta/2, +theta/2);
    //   DIAG k q_0 .. q_{k-1} phi_0 .. phi_{2^k - 1} (k = 1..3, radians).
    // S, SDG, T, TDG and CZ take this form only under IF; bare, they are the
    // Clifford / T ops.  tok[at] names the gate.
    auto diag_op = [&](const std::vector<std::string> &tok, size_t at, int src) {
        const std::string &name = tok[at];
        Op o;
        o.kind = K_DIAG;
        o.src = src;
        const double pi = 3.14159265358979323846;
        size_t nq = 0, first = at + 1;
        if (name == "CCZ" || name == "CCX") nq = 3;
        else if (name == "CS" || name == "CSDG" || name == "CZ") nq = 2;
        else if (name == "S" || name == "SDG" || name == "T" || name == "TDG") nq = 1;
        else if (name == "CPHASE") { nq = 2; first = at + 2; }
        else if (name == "RZ") { nq = 1; first = at + 2; }
        else {
            if (tok.size() < at + 2) throw ParseError{line, "DIAG takes k, k qubits and 2^k phases"};
            const int k = to_int(tok[at + 1], line);
            if (k < 1 || k > 3) throw ParseError{line, "DIAG takes 1 to 3 qubits"};
            nq = (size_t)k;
            first = at + 2;
        }
        const size_t want = name == "DIAG" ? first + nq + (1u << nq) : first + nq;
        if (tok.size() != want) throw ParseError{line, name + ": wrong number of arguments"};
        for (size_t i = 0; i < nq; ++i) o.qs.push_back(qubit(tok[first + i]));
        for (size_t i = 0; i < nq; ++i)
            for (size_t j = 0; j < i; ++j)
                if (o.qs[i] == o.qs[j]) throw ParseError{line, name + " on repeated qubits"};
        auto angle = [&](const std::string &t) {
            char *end = nullptr;
            double v = std::strtod(t.c_str(), &end);
            if (end == t.c_str() || *end != '\0' || !std::isfinite(v)) throw ParseError{line, "bad angle '" + t + "'"};
            return v;
        };
        o.phi.assign((size_t)1 << nq, 0.0);
        if (name == "CCZ" || name == "CCX") o.phi[7] = pi;
        else if (name == "CZ") o.phi[3] = pi;
        else if (name == "S") o.phi[1] = pi / 2;
        else if (name == "SDG") o.phi[1] = -pi / 2;
        else if (name == "T") o.phi[1] = pi / 4;
        else if (name == "TDG") o.phi[1] = -pi / 4;
        else if (name == "CS") o.phi[3] = pi / 2;
        else if (name == "CSDG") o.phi[3] = -pi / 2;
        else if (name == "CPHASE") o.phi[3] = angle(tok[at + 1]);
        else if (name == "RZ") { o.phi[0] = -angle(tok[at + 1]) / 2; o.phi[1] = angle(tok[at + 1]) / 2; }
        else
            for (size_t x = 0; x < o.phi.size(); ++x) o.phi[x] = angle(tok[first + nq + x]);
        return o;
    };

    while (std::getline(in, raw)) {
        ++line;
        std::string s = raw.substr(0, raw.find('#'));
        std::istringstream ts(s);
        std::vector<std::string> tok;
        std::string t;
        while (ts >> t) tok.push_back(t);
        if (tok.empty()) continue;
        const std::string &name = tok[0];
        if (!have_qubits) {
            if (name != "QUBITS" || tok.size() != 2) throw ParseError{line, "first line must be QUBITS n"};
            c.n = to_int(tok[1], line);
            if (c.n < 1 || c.n > 64) throw ParseError{line, "QUBITS must be in 1..64"};
            active.assign(c.n, 0);
            have_qubits = true;
            continue;
        }
        int src = c.n_src++;
        static const char *one_q[] = {"H", "S", "SDG", "X", "Y", "Z", "T", "TDG", "H_XY", "H_NXY"};
        static const Kind one_k[] = {K_H, K_S, K_SDG, K_X, K_Y, K_Z, K_T, K_TDG, K_HXY, K_HNXY};
        bool done = false;
        for (int i = 0; i < 10 && !done; ++i) {
            if (name == one_q[i]) {
                if (tok.size() != 2) throw ParseError{line, name + " takes one qubit"};
                Op o;
                o.kind = one_k[i]; o.a = qubit(tok[1]); o.src = src;
                c.ops.push_back(o);
                active[o.a] = 1;
                add_noise(K_DEP1, nm.p1, o.a, -1, src);
                done = true;
            }
        }
        if (done) continue;
        if (name == "CX" || name == "CZ") {
            if (tok.size() != 3) throw ParseError{line, name + " takes two qubits"};
            Op o;
            o.kind = name == "CX" ? K_CX : K_CZ;
            o.a = qubit(tok[1]); o.b = qubit(tok[2]); o.src = src;
            if (o.a == o.b) throw ParseError{line, "two-qubit gate on one qubit"};
            c.ops.push_back(o);
            active[o.a] = active[o.b] = 1;
            add_noise(K_DEP2, nm.p2, o.a, o.b, src);
        } else if (name == "M") {
            if (tok.size() != 2) throw ParseError{line, "M takes one qubit"};
            int q = qubit(tok[1]);
            add_noise(K_XERR, nm.p_meas, q, -1, src);
            Op o;
            o.kind = K_M; o.a = q; o.src = src; o.slot = c.n_meas++; o.rec = c.n_rec++;
            c.ops.push_back(o);
            active[q] = 1;
        } else if (name == "R") {
            if (tok.size() != 2) throw ParseError{line, "R takes one qubit"};
            int q = qubit(tok[1]);
            Op o;
            o.kind = K_R; o.a = q; o.src = src; o.slot = c.n_meas++;
            c.ops.push_back(o);
            active[q] = 1;
            add_noise(K_XERR, nm.p_reset, q, -1, src);
        } else if (is_diag_name(name)) {
            Op o = diag_op(tok, 0, src);
            const bool ccx = name == "CCX";
            if (ccx) hgate(o.qs[2], src);
            c.ops.push_back(o);
            if (ccx) hgate(o.qs[2], src);
            for (int q : o.qs) active[q] = 1;
            // model noise: DEP2(p2) after a two-qubit diagonal gate, DEP1(p1)
            // on each qubit after a one- or three-qubit one
            if (o.qs.size() == 2) add_noise(K_DEP2, nm.p2, o.qs[0], o.qs[1], src);
            else
                for (int q : o.qs) add_noise(K_DEP1, nm.p1, q, -1, src);
        } else if (name == "IF") {
            // Classically controlled gate (the corrections of gate
            // teleportation): IF r0,r1,.. GATE args applies GATE when the XOR
            // of the listed record bits is 1, IF r0&r1&.. GATE args when all of
            // them are 1.  GATE is a Pauli (X, Y, Z) or a diagonal gate (S,
            // SDG, T, TDG, CZ and the diagonal gates above).  No model noise.
            if (tok.size() < 3) throw ParseError{line, "IF takes record bits and a gate"};
            std::vector<int> cond;
            const std::string &cs = tok[1];
            const bool has_and = cs.find('&') != std::string::npos, has_xor = cs.find(',') != std::string::npos;
            if (has_and && has_xor) throw ParseError{line, "IF: use ',' (XOR) or '&' (AND), not both"};
            size_t pos = 0;
            while (true) {
                const size_t e = cs.find(has_and ? '&' : ',', pos);
                const int r = to_int(cs.substr(pos, e == std::string::npos ? std::string::npos : e - pos), line);
                if (r >= c.n_rec) throw ParseError{line, "record index not yet measured"};
                cond.push_back(r);
                if (e == std::string::npos) break;
                pos = e + 1;
            }
            const std::string &g = tok[2];
            if (g == "X" || g == "Y" || g == "Z") {
                if (tok.size() != 4) throw ParseError{line, "IF: " + g + " takes one qubit"};
                Op o;
                o.kind = K_FEEDBACK; o.src = src;
                o.a = qubit(tok[3]);
                o.b = g == "X" ? 1 : g == "Y" ? 2 : 3;
                o.cond = cond;
                o.cond_and = has_and;
                c.ops.push_back(o);
            } else if (is_cond_diag_name(g)) {
                Op o = diag_op(tok, 2, src);
                o.cond = cond;
                o.cond_and = has_and;
                const bool ccx = g == "CCX";  // H is unconditional: H IF(CCZ) H
                if (ccx) hgate(o.qs[2], src);
                c.ops.push_back(o);
                if (ccx) hgate(o.qs[2], src);
                for (int q : o.qs) active[q] = 1;
            } else {
                throw ParseError{line, "IF: '" + g + "' is neither a Pauli nor a diagonal gate"};
            }
        } else if (name == "MX" || name == "RX" || name == "MR" || name == "MRX") {
            // X-basis measurement / reset to |+>, and measure-then-reset.  The
            // measurement-error flip before a readout and the reset-error flip
            // after a reset anticommute with the measured Pauli: X for Z-basis
            // ops, Z for X-basis ops.
            if (tok.size() != 2) throw ParseError{line, name + " takes one qubit"};
            int q = qubit(tok[1]);
            const bool xb = name == "MX" || name == "RX" || name == "MRX";
            const bool readout = name != "RX", reset = name != "MX";
            const Kind flip = xb ? K_ZERR : K_XERR;
            if (readout) add_noise(flip, nm.p_meas, q, -1, src);
            Op o;
            o.kind = name == "MX" ? K_MX : name == "RX" ? K_RX : name == "MR" ? K_MR : K_MRX;
            o.a = q; o.src = src; o.slot = c.n_meas++;
            if (readout) o.rec = c.n_rec++;
            c.ops.push_back(o);
            active[q] = 1;
            if (reset) add_noise(flip, nm.p_reset, q, -1, src);
        } else if (name == "XIF" || name == "YIF" || name == "ZIF") {
            // classically controlled Pauli: apply it when the record bit is 1
            if (tok.size() != 3) throw ParseError{line, name + " takes a record index and a qubit"};
            Op o;
            o.kind = K_FEEDBACK; o.src = src;
            const int r = to_int(tok[1], line);
            if (r >= c.n_rec) throw ParseError{line, "record index not yet measured"};
            o.cond.push_back(r);
            o.a = qubit(tok[2]);
            o.b = name == "XIF" ? 1 : name == "YIF" ? 2 : 3;
            c.ops.push_back(o);
        } else if (name == "MPP") {
            if (tok.size() != 2) throw ParseError{line, "MPP takes one Pauli product"};
            Op o;
            o.kind = K_MPP; o.src = src;
            std::string prod = tok[1];
            size_t pos = 0;
            while (pos <= prod.size()) {
                size_t star = prod.find('*', pos);
                std::string f = prod.substr(pos, star == std::string::npos ? std::string::npos : star - pos);
                if (f.size() < 2) throw ParseError{line, "bad Pauli factor '" + f + "'"};
                int q = qubit(f.substr(1));
                uint64_t bit = 1ULL << q;
                if ((o.px | o.pz) & bit) throw ParseError{line, "repeated qubit in MPP"};
                if (f[0] == 'X') o.px |= bit;
                else if (f[0] == 'Z') o.pz |= bit;
                else if (f[0] == 'Y') { o.px |= bit; o.pz |= bit; }
                else throw ParseError{line, "bad Pauli letter"};
                active[q] = 1;
                if (star == std::string::npos) break;
                pos = star + 1;
            }
            o.slot = c.n_meas++;
            o.rec = c.n_rec++;
            c.ops.push_back(o);
            add_flip(nm.p_mpp, o.rec, src);
        } else if (name == "DEP1" || name == "XERR" || name == "ZERR") {
            if (tok.size() < 3) throw ParseError{line, name + " takes p and qubits"};
            double p = to_prob(tok[1], line);
            const Kind k = name == "DEP1" ? K_DEP1 : name == "XERR" ? K_XERR : K_ZERR;
            for (size_t i = 2; i < tok.size(); ++i) add_noise(k, p, qubit(tok[i]), -1, src);
        } else if (name == "DEP2") {
            if (tok.size() < 4 || (tok.size() - 2) % 2 != 0) throw ParseError{line, "DEP2 takes p and qubit pairs"};
            double p = to_prob(tok[1], line);
            for (size_t i = 2; i < tok.size(); i += 2) {
                int a = qubit(tok[i]), b = qubit(tok[i + 1]);
                if (a == b) throw ParseError{line, "DEP2 on one qubit"};
                add_noise(K_DEP2, p, a, b, src);
            }
        } else if (name == "TICK") {
            if (tok.size() != 1) throw ParseError{line, "TICK takes no arguments"};
            for (int q = 0; q < c.n; ++q)
                if (!active[q]) add_noise(K_DEP1, nm.p_idle, q, -1, src);
            active.assign(c.n, 0);
        } else if (name == "DETECTOR" || name == "OBSERVABLE") {
            if (tok.size() < 2) throw ParseError{line, name + " takes an expected bit"};
            Op o;
            o.kind = name == "DETECTOR" ? K_DETECTOR : K_OBSERVABLE;
            o.src = src;
            o.expect = to_int(tok[1], line);
            if (o.expect > 1) throw ParseError{line, "expected bit must be 0 or 1"};
            for (size_t i = 2; i < tok.size(); ++i) {
                int r = to_int(tok[i], line);
                if (r >= c.n_rec) throw ParseError{line, "record index not yet measured"};
                o.recs.push_back(r);
            }
            if (o.kind == K_OBSERVABLE) {
                if (c.n_obs >= 32) throw ParseError{line, "at most 32 observables"};
                o.obs = c.n_obs++;
            }
            c.ops.push_back(o);
        } else {
            throw ParseError{line, "unknown op '" + name + "'"};
        }
    }
    if (!have_qubits) throw ParseError{line, "missing QUBITS line"};
}

// ---------------------------------------------------------------------------
// Pauli rows.  A row (x, z, e) means i^e * (x) sigma(x_j, z_j) with
// sigma(0,0)=I, sigma(1,0)=X, sigma(0,1)=Z, sigma(1,1)=Y.  Tableau rows carry
// e = 2 r (a sign).
// ---------------------------------------------------------------------------
struct Pauli {
    uint64_t x = 0, z = 0;
    int e = 0;  // exponent of i, mod 4
};

int popc(uint64_t w) { return __builtin_popcountll(w); }

int mod4(int k) { return ((k % 4) + 4) % 4; }

// 1 iff A and B anticommute (symplectic product).
int anticommute(uint64_t ax, uint64_t az, uint64_t bx, uint64_t bz) {
    return popc((ax & bz) ^ (az & bx)) & 1;
}

// C = A * B.  With sigma(x,z) = i^{xz} X^x Z^z per qubit, moving each Z^{zA}
// past X^{xB} costs (-1)^{zA.xB}, hence
//   e_C = e_A + e_B + |xA&zA| + |xB&zB| + 2|zA&xB| - |xC&zC|  (mod 4).
Pauli mul(const Pauli &A, const Pauli &B) {
    Pauli C;
    C.x = A.x ^ B.x;
    C.z = A.z ^ B.z;
    C.e = mod4(A.e + B.e + popc(A.x & A.z) + popc(B.x & B.z) + 2 * popc(A.z & B.x) - popc(C.x & C.z));
    return C;
}

const double kPi = 3.14159265358979323846;

struct ShotState {
    int n;
    std::vector<uint64_t> x, z;  // rows 0..n-1: destabilizers, n..2n-1: stabilizers
    std::vector<int> r;          // sign bits
    std::map<uint64_t, cplx> v;  // alpha -> v_alpha
};

Pauli row(const ShotState &st, int i) {
    Pauli p;
    p.x = st.x[i]; p.z = st.z[i]; p.e = 2 * st.r[i];
    return p;
}

void set_row(ShotState &st, int i, const Pauli &p) {
    if (p.e % 2 != 0) { std::fprintf(stderr, "oracle: non-Hermitian tableau row\n"); std::abort(); }
    st.x[i] = p.x; st.z[i] = p.z; st.r[i] = p.e / 2;
}

int bit(uint64_t w, int q) { return (int)((w >> q) & 1ULL); }

void set_bit(uint64_t &w, int q, int b) {
    w = (w & ~(1ULL << q)) | ((uint64_t)b << q);
}

// Clifford conjugation rules of the Aaronson-Gottesman tableau, signs included.
void apply_clifford(ShotState &st, Kind k, int a, int b) {
    for (int i = 0; i < 2 * st.n; ++i) {
        int xa = bit(st.x[i], a), za = bit(st.z[i], a);
        switch (k) {
            case K_H:
                st.r[i] ^= xa & za;
                set_bit(st.x[i], a, za);
                set_bit(st.z[i], a, xa);
                break;
            case K_S:
                st.r[i] ^= xa & za;
                set_bit(st.z[i], a, za ^ xa);
                break;
            case K_SDG:
                st.r[i] ^= xa & (za ^ 1);
                set_bit(st.z[i], a, za ^ xa);
                break;
            case K_HXY:
                // (X + Y)/sqrt2: X -> Y, Y -> X, Z -> -Z
                st.r[i] ^= za & (xa ^ 1);
                set_bit(st.z[i], a, za ^ xa);
                break;
            case K_HNXY:
                // (X - Y)/sqrt2: X -> -Y, Y -> -X, Z -> -Z
                st.r[i] ^= xa | za;
                set_bit(st.z[i], a, za ^ xa);
                break;
            case K_X: st.r[i] ^= za; break;
            case K_Z: st.r[i] ^= xa; break;
            case K_Y: st.r[i] ^= xa ^ za; break;
            case K_CX: {
                int xb = bit(st.x[i], b), zb = bit(st.z[i], b);
                st.r[i] ^= xa & zb & (xb ^ za ^ 1);
                set_bit(st.x[i], b, xb ^ xa);
                set_bit(st.z[i], a, za ^ zb);
                break;
            }
            case K_CZ: {
                int xb = bit(st.x[i], b), zb = bit(st.z[i], b);
                st.r[i] ^= xa & xb & (za ^ zb);
                set_bit(st.z[i], a, za ^ xb);
                set_bit(st.z[i], b, zb ^ xa);
                break;
            }
            default: std::abort();
        }
    }
}

// Single-qubit Pauli code 0=I 1=X 2=Y 3=Z applied as a conjugation.
void apply_pauli_code(ShotState &st, int code, int q) {
    if (code == 1) apply_clifford(st, K_X, q, -1);
    if (code == 2) apply_clifford(st, K_Y, q, -1);
    if (code == 3) apply_clifford(st, K_Z, q, -1);
}

// Q = c * d_beta * s_gamma with beta_i = [Q anticommutes with s_i] and
// gamma_i = [Q anticommutes with d_i] (the index shift of Eq. 4).  The product
// is taken left to right in index order; c = i^{e_Q - e_R}.
struct Decomp {
    uint64_t beta = 0, gamma = 0;
    int c_exp = 0;
};

Decomp decompose(const ShotState &st, const Pauli &Q) {
    Decomp d;
    int n = st.n;
    for (int i = 0; i < n; ++i) {
        if (anticommute(Q.x, Q.z, st.x[n + i], st.z[n + i])) d.beta |= 1ULL << i;
        if (anticommute(Q.x, Q.z, st.x[i], st.z[i])) d.gamma |= 1ULL << i;
    }
    Pauli R;
    for (int i = 0; i < n; ++i)
        if (bit(d.beta, i)) R = mul(R, row(st, i));
    for (int i = 0; i < n; ++i)
        if (bit(d.gamma, i)) R = mul(R, row(st, n + i));
    if (R.x != Q.x || R.z != Q.z) { std::fprintf(stderr, "oracle: decomposition failed\n"); std::abort(); }
    d.c_exp = mod4(Q.e - R.e);
    return d;
}

cplx ipow(int k) {
    static const cplx tab[4] = {cplx(1, 0), cplx(0, 1), cplx(-1, 0), cplx(0, -1)};
    return tab[mod4(k)];
}

double sgn_parity(uint64_t w) { return (popc(w) & 1) ? -1.0 : 1.0; }

double norm2(const std::map<uint64_t, cplx> &v) {
    double s = 0.0;
    for (const auto &kv : v) s += std::norm(kv.second);
    return s;
}

// Drop entries with |v_alpha|^2 < tau^2 * sum |v|^2.
void prune(std::map<uint64_t, cplx> &v, double tau) {
    double limit = tau * tau * norm2(v);
    for (auto it = v.begin(); it != v.end();) {
        if (std::norm(it->second) < limit) it = v.erase(it);
        else ++it;
    }
}

// T^s on qubit q (s = +1 for T, -1 for T-dagger):
// T^s = e^{i s theta} (cos theta I - i s sin theta Z_q), theta = pi/8 (Eqs. 1-2),
// with Z_q |b_alpha> = c (-1)^{gamma.alpha} |b_{alpha^beta}> (Eq. 4).
// *flips counts the entries that pick up the phase when beta = 0 (work count).
void apply_t(ShotState &st, int q, int s, double tau, uint64_t *flips) {
    Pauli Z;
    Z.z = 1ULL << q;
    Decomp d = decompose(st, Z);
    const double th = kPi / 8.0;
    const cplx glob = std::exp(cplx(0.0, s * th));
    const double cs = std::cos(th), sn = std::sin(th);
    const cplx c = ipow(d.c_exp);
    const cplx mi_s(0.0, -(double)s);  // -i s
    std::map<uint64_t, cplx> out;
    if (d.beta == 0) {
        for (const auto &kv : st.v) {
            cplx lam = c * sgn_parity(d.gamma & kv.first);
            if (lam.real() < 0) ++*flips;
            out[kv.first] = glob * (cs + mi_s * sn * lam) * kv.second;
        }
    } else {
        std::set<uint64_t> keys;
        for (const auto &kv : st.v) {
            keys.insert(kv.first);
            keys.insert(kv.first ^ d.beta);
        }
        for (uint64_t a : keys) {
            auto it0 = st.v.find(a);
            auto it1 = st.v.find(a ^ d.beta);
            cplx v0 = it0 == st.v.end() ? cplx(0) : it0->second;
            cplx v1 = it1 == st.v.end() ? cplx(0) : it1->second;
            out[a] = glob * (cs * v0 + mi_s * sn * c * sgn_parity(d.gamma & (a ^ d.beta)) * v1);
        }
    }
    st.v.swap(out);
    prune(st.v, tau);
}

// Diagonal gate U = sum_x e^{i phi_x} |x><x| on the qubits qs.  Expanded over
// the Z-strings of those qubits (the expansion behind Proposition 1),
// U = sum_g c_g Z^g with c_g = 2^-m sum_x e^{i phi_x} (-1)^{g.x}, and each
// Z^g acts on the basis by Eq. 4: Z^g |b_alpha> = c (-1)^{gamma.alpha}
// |b_{alpha ^ beta}>.  One pass over the 2^m terms.
void apply_diag(ShotState &st, const std::vector<int> &qs, const std::vector<double> &phi, double tau) {
    const size_t m = qs.size(), ng = (size_t)1 << m;
    std::map<uint64_t, cplx> out;
    for (size_t g = 0; g < ng; ++g) {
        cplx cg(0.0, 0.0);
        for (size_t x = 0; x < ng; ++x) cg += std::exp(cplx(0.0, phi[x])) * sgn_parity((uint64_t)(g & x));
        cg /= (double)ng;
        Pauli Z;
        for (size_t j = 0; j < m; ++j)
            if ((g >> j) & 1) Z.z |= 1ULL << qs[j];
        const Decomp d = decompose(st, Z);
        const cplx w = cg * ipow(d.c_exp);
        for (const auto &kv : st.v) out[kv.first ^ d.beta] += w * sgn_parity(d.gamma & kv.first) * kv.second;
    }
    st.v.swap(out);
    prune(st.v, tau);
}

// Measurement of the Hermitian Pauli P with uniform u.  Returns the record
// bit, or -1 for a numerically empty branch.  p0 receives P(outcome +1).
// *pairs receives the number of representative pairs (beta != 0; work count).
int measure(ShotState &st, const Pauli &P, double u, double tau, double *p0_out, uint64_t *pairs) {
    Decomp d = decompose(st, P);
    const cplx c = ipow(d.c_exp);
    const int n = st.n;
    if (d.beta == 0) {
        // P = c * s_gamma acts diagonally: P |b_alpha> = lambda_alpha |b_alpha>.
        double Np = 0.0, Nm = 0.0;
        for (const auto &kv : st.v) {
            double lam = (c * sgn_parity(d.gamma & kv.first)).real();
            if (lam > 0) Np += std::norm(kv.second);
            else Nm += std::norm(kv.second);
        }
        double p0 = Np / (Np + Nm);
        if (p0_out) *p0_out = p0;
        int m = u < p0 ? +1 : -1;
        double Nsel = m > 0 ? Np : Nm;
        if (!(Nsel > 1e-300)) return -1;
        std::map<uint64_t, cplx> out;
        for (const auto &kv : st.v) {
            double lam = (c * sgn_parity(d.gamma & kv.first)).real();
            if ((lam > 0) == (m > 0)) out[kv.first] = kv.second / std::sqrt(Nsel);
        }
        st.v.swap(out);
        prune(st.v, tau);
        return m > 0 ? 0 : 1;
    }
    // beta != 0: pivot on the lowest stabilizer that anticommutes with P.
    int p = __builtin_ctzll(d.beta);
    std::set<uint64_t> reps;
    for (const auto &kv : st.v) {
        uint64_t a = kv.first;
        reps.insert(bit(a, p) ? (a ^ d.beta) : a);
    }
    *pairs += reps.size();
    std::map<uint64_t, cplx> wplus, wminus;
    double Np = 0.0, Nm = 0.0;
    for (uint64_t a : reps) {
        auto it0 = st.v.find(a);
        auto it1 = st.v.find(a ^ d.beta);
        cplx v0 = it0 == st.v.end() ? cplx(0) : it0->second;
        cplx v1 = it1 == st.v.end() ? cplx(0) : it1->second;
        cplx f = std::conj(c) * sgn_parity(d.gamma & a);
        wplus[a] = v0 + f * v1;
        wminus[a] = v0 - f * v1;
        Np += 0.5 * std::norm(wplus[a]);
        Nm += 0.5 * std::norm(wminus[a]);
    }
    double p0 = Np / (Np + Nm);
    if (p0_out) *p0_out = p0;
    int m = u < p0 ? +1 : -1;
    double Nsel = m > 0 ? Np : Nm;
    if (!(Nsel > 1e-300)) return -1;
    std::map<uint64_t, cplx> out;
    for (uint64_t a : reps) out[a] = (m > 0 ? wplus[a] : wminus[a]) / std::sqrt(2.0 * Nsel);
    // Tableau: rows anticommuting with P (other than s_p, d_p) absorb s_p;
    // d_p takes the old s_p; s_p becomes m P.
    Pauli sp = row(st, n + p);
    for (int i = 0; i < 2 * n; ++i) {
        if (i == p || i == n + p) continue;
        if (anticommute(P.x, P.z, st.x[i], st.z[i])) set_row(st, i, mul(row(st, i), sp));
    }
    set_row(st, p, sp);
    Pauli mp = P;
    mp.e = mod4(P.e + (m > 0 ? 0 : 2));
    set_row(st, n + p, mp);
    st.v.swap(out);
    prune(st.v, tau);
    return m > 0 ? 0 : 1;
}

struct ShotResult {
    std::vector<uint32_t> record;
    oracle_shot_info info;
    bool on_path = true;  // still on the noiseless trajectory every shot shares
};

// The work counters of `at` in the order of oracle_batch's sums, with the
// shot's own noise draws left out (they are never shared).
void shared_of(const oracle_shot_info &at, uint64_t out[ORACLE_WORK_COUNT]) {
    const uint64_t w[ORACLE_WORK_COUNT] = {at.t_entries, at.t_phase_entries, at.m_entries, 0, at.events, 0,
                                           at.m_out_entries, at.m_pairs, at.t_phase_flips, at.meas_words};
    for (int k = 0; k < ORACLE_WORK_COUNT; ++k) out[k] = w[k];
}

// The shot leaves the shared trajectory; `at` holds its counters just before
// the event that made it leave.
void leave_path(ShotResult &res, const oracle_shot_info &at) {
    if (!res.on_path) return;
    res.on_path = false;
    shared_of(at, res.info.shared);
}

double uniform_of(uint32_t w) { return ((double)w + 0.5) * (1.0 / 4294967296.0); }

void run_ops(const oracle_circuit &c, uint64_t seed, uint64_t shot, const uint32_t *words, double tau,
             uint32_t cap, ShotState &st, ShotResult &res, double *p0_trace) {
    const int n = c.n;
    st.n = n;
    st.x.assign(2 * n, 0);
    st.z.assign(2 * n, 0);
    st.r.assign(2 * n, 0);
    for (int i = 0; i < n; ++i) {
        st.x[i] = 1ULL << i;      // d_i = +X_i
        st.z[n + i] = 1ULL << i;  // s_i = +Z_i
    }
    st.v.clear();
    st.v[0] = cplx(1.0, 0.0);
    res.record.assign((c.n_rec + 31) / 32, 0u);
    std::memset(&res.info, 0, sizeof(res.info));
    res.on_path = true;
    res.info.abort_op = 0xffffffffu;
    res.info.max_support = 1;

    auto noise_word = [&](int slot) {
        return words ? words[slot] : philox_word(seed, shot, 0, (uint64_t)slot);
    };
    // Mode 1: a Bernoulli(p_slot) hit on every slot, drawn as a Bernoulli(p_max)
    // candidate process thinned by p_slot / p_max.  Candidates: the gap G
    // before the next one has P(G >= g) = q^g, drawn from one word w as the
    // number of g >= 1 with w < floor(q^g 2^32); a second word a accepts the
    // candidate iff a < floor(p_slot / p_max 2^32) and then picks its Pauli
    // the way mode 0 uses its word.  Words come from stream 2 in order.
    uint64_t draw = 0;
    int64_t cand = -1;          // last candidate slot
    int next_hit = -1;          // pending accepted slot (mode 1), -1 = none left
    uint32_t hit_word = 0;
    auto advance = [&]() {
        next_hit = -1;
        while (true) {
            const uint32_t w = philox_word(seed, shot, 2, draw++);
            ++res.info.noise_words;
            int64_t g = 0;
            while (g + 1 <= c.n_noise && (uint64_t)w < c.gap_thr[g + 1]) ++g;
            cand += 1 + g;
            if (cand >= c.n_noise) return;
            const uint32_t a = philox_word(seed, shot, 2, draw++);
            ++res.info.noise_words;
            if ((uint64_t)a < c.accept[cand]) {
                next_hit = (int)cand;
                hit_word = a;
                return;
            }
        }
    };
    const bool gaps = c.noise_mode == 1 && !words;
    if (gaps) advance();
    auto meas_word = [&](int slot) {
        return words ? words[c.n_noise + slot] : philox_word(seed, shot, 1, (uint64_t)slot);
    };
    auto rec_bit = [&](int k) { return (int)((res.record[k >> 5] >> (k & 31)) & 1u); };
    // condition of a classically controlled op: XOR (or AND) of its record bits
    auto cond_holds = [&](const Op &o) {
        if (o.cond.empty()) return true;
        int v = o.cond_and ? 1 : 0;
        for (int r : o.cond) v = o.cond_and ? (v & rec_bit(r)) : (v ^ rec_bit(r));
        return v != 0;
    };
    auto note_support = [&]() {
        res.info.max_support = std::max<uint32_t>(res.info.max_support, (uint32_t)st.v.size());
    };

    for (const Op &o : c.ops) {
        switch (o.kind) {
            case K_H: case K_S: case K_SDG: case K_X: case K_Y: case K_Z: case K_CX: case K_CZ: case K_HXY:
            case K_HNXY:
                apply_clifford(st, o.kind, o.a, o.b);
                break;
            case K_FEEDBACK:
                if (cond_holds(o)) apply_pauli_code(st, o.b, o.a);
                break;
            case K_T: case K_TDG: {
                Pauli Z;
                Z.z = 1ULL << o.a;
                bool branching = decompose(st, Z).beta != 0;
                if (!branching) res.info.t_phase_entries += st.v.size();
                apply_t(st, o.a, o.kind == K_T ? +1 : -1, tau, &res.info.t_phase_flips);
                if (branching) res.info.t_entries += st.v.size();
                res.info.events++;
                note_support();
                if (st.v.size() > cap) {
                    res.info.status = ORACLE_OVERFLOW;
                    res.info.abort_op = o.src;
                    res.info.norm2 = norm2(st.v);
                    return;
                }
                break;
            }
            case K_DIAG: {
                if (!cond_holds(o)) break;  // a classically controlled gate that does not fire
                apply_diag(st, o.qs, o.phi, tau);
                res.info.t_entries += st.v.size();
                res.info.events++;
                note_support();
                if (st.v.size() > cap) {
                    res.info.status = ORACLE_OVERFLOW;
                    res.info.abort_op = o.src;
                    res.info.norm2 = norm2(st.v);
                    return;
                }
                break;
            }
            case K_M: case K_MPP: case K_R: case K_MX: case K_RX: case K_MR: case K_MRX: {
                const bool xb = o.kind == K_MX || o.kind == K_RX || o.kind == K_MRX;
                Pauli P;
                if (o.kind == K_MPP) { P.x = o.px; P.z = o.pz; }
                else if (xb) P.x = 1ULL << o.a;
                else P.z = 1ULL << o.a;
                const oracle_shot_info before = res.info;
                res.info.m_entries += st.v.size();
                res.info.events++;
                double p0 = 0.0;
                ++res.info.meas_words;
                int b = measure(st, P, uniform_of(meas_word(o.slot)), tau, &p0, &res.info.m_pairs);
                if (p0_trace) p0_trace[o.slot] = p0;
                if (p0 > 0.0 && p0 < 1.0) leave_path(res, before);  // the outcome was drawn
                if (b < 0) {
                    res.info.status = ORACLE_NUMERIC;
                    res.info.abort_op = o.src;
                    res.info.norm2 = norm2(st.v);
                    return;
                }
                res.info.m_out_entries += st.v.size();
                if (b && o.rec >= 0) res.record[o.rec >> 5] |= 1u << (o.rec & 31);
                // resets bring outcome 1 back to the +1 eigenstate of the measured Pauli
                if (b && (o.kind == K_R || o.kind == K_MR)) apply_clifford(st, K_X, o.a, -1);
                if (b && (o.kind == K_RX || o.kind == K_MRX)) apply_clifford(st, K_Z, o.a, -1);
                note_support();
                break;
            }
            case K_DEP1: case K_DEP2: case K_XERR: case K_ZERR: case K_FLIP: {
                res.info.noise_slots++;
                uint32_t w;
                uint64_t thr;
                if (gaps) {
                    if (o.slot != next_hit) break;
                    w = hit_word;
                    thr = c.accept[o.slot];
                    advance();
                } else {
                    w = noise_word(o.slot);
                    ++res.info.noise_words;
                    thr = o.thr;
                    if ((uint64_t)w >= thr) break;
                }
                leave_path(res, res.info);  // a hit
                if (o.kind == K_DEP1) {
                    int idx = (int)((3ULL * w) / thr);  // 0,1,2 -> X,Y,Z
                    apply_pauli_code(st, idx + 1, o.a);
                } else if (o.kind == K_DEP2) {
                    int code = (int)((15ULL * w) / thr) + 1;  // 1..15
                    apply_pauli_code(st, code >> 2, o.a);
                    apply_pauli_code(st, code & 3, o.b);
                } else if (o.kind == K_XERR) {
                    apply_pauli_code(st, 1, o.a);
                } else if (o.kind == K_ZERR) {
                    apply_pauli_code(st, 3, o.a);
                } else {
                    res.record[o.rec >> 5] ^= 1u << (o.rec & 31);
                }
                break;
            }
            case K_DETECTOR: case K_OBSERVABLE: {
                int par = o.expect;
                for (int k : o.recs) par ^= rec_bit(k);
                if (o.kind == K_DETECTOR) {
                    if (par) {
                        res.info.status = ORACLE_DISCARDED;
                        res.info.abort_op = o.src;
                        res.info.norm2 = norm2(st.v);
                        return;
                    }
                } else if (par) {
                    res.info.obs |= 1u << o.obs;
                }
                break;
            }
        }
    }
    res.info.status = ORACLE_PASSED;
    res.info.norm2 = norm2(st.v);
}

void run_shot(const oracle_circuit &c, uint64_t seed, uint64_t shot, const uint32_t *words, double tau,
              uint32_t cap, ShotState &st, ShotResult &res, double *p0_trace) {
    run_ops(c, seed, shot, words, tau, cap, st, res, p0_trace);
    if (res.on_path) shared_of(res.info, res.info.shared);  // it never left: all of its work was shared
}

}  // namespace

extern "C" {

oracle_circuit *oracle_compile(const char *text, const oracle_noise *noise, char *err, int errlen) {
    oracle_noise nm = {0, 0, 0, 0, 0, 0};
    if (noise) nm = *noise;
    const double ps[6] = {nm.p1, nm.p2, nm.p_idle, nm.p_meas, nm.p_reset, nm.p_mpp};
    for (double p : ps) {
        if (!(p >= 0.0 && p <= 1.0)) {
            if (err && errlen > 0) std::snprintf(err, errlen, "noise probability out of [0,1]");
            return nullptr;
        }
    }
    oracle_circuit *c = new oracle_circuit();
    try {
        compile(text ? text : "", nm, *c);
    } catch (const ParseError &e) {
        if (err && errlen > 0) std::snprintf(err, errlen, "line %d: %s", e.line, e.msg.c_str());
        delete c;
        return nullptr;
    }
    return c;
}

void oracle_free(oracle_circuit *c) { delete c; }

int oracle_set_noise_mode(oracle_circuit *c, int mode) {
    if (!c || mode < 0 || mode > 1) return -1;
    c->noise_mode = mode;
    c->gap_thr.clear();
    c->accept.clear();
    if (mode == 1) {
        // a slot whose threshold floor(p 2^32) is 0 is never hit in mode 0;
        // it takes no part here either (acceptance 0, no say in p_max)
        auto live = [](const Op &o) {
            return o.slot >= 0 && o.thr > 0 &&
                   (o.kind == K_DEP1 || o.kind == K_DEP2 || o.kind == K_XERR || o.kind == K_ZERR || o.kind == K_FLIP);
        };
        double pmax = 0.0;
        for (const Op &o : c->ops)
            if (live(o)) pmax = std::max(pmax, o.p);
        c->accept.assign(c->n_noise, 0);
        for (const Op &o : c->ops)
            if (live(o)) c->accept[o.slot] = (uint64_t)std::floor(o.p / pmax * 4294967296.0);
        // q^g by repeated multiplication (the same IEEE products on every machine)
        const double q = 1.0 - pmax;
        c->gap_thr.assign(c->n_noise + 1, 0);
        double t = 1.0;
        c->gap_thr[0] = 1ull << 32;
        for (int g = 1; g <= c->n_noise; ++g) {
            t *= q;
            c->gap_thr[g] = (uint64_t)std::floor(t * 4294967296.0);
        }
    }
    return 0;
}

void oracle_counts(const oracle_circuit *c, uint64_t counts[7]) {
    counts[0] = c->n;
    counts[1] = c->n_src;
    counts[2] = c->n_rec;
    counts[3] = c->n_noise;
    counts[4] = c->n_meas;
    counts[5] = c->n_obs;
    counts[6] = c->ops.size();
}

int oracle_shot(const oracle_circuit *c, uint64_t seed, uint64_t shot, const uint32_t *words, double tau,
                uint32_t cap, uint32_t *record, oracle_shot_info *info, uint64_t *tab_x, uint64_t *tab_z,
                uint8_t *tab_r, uint64_t *alpha, double *re, double *im, uint32_t coeff_cap, uint32_t *n_coeff,
                double *p0_trace) {
    if (!c || !(tau >= 0.0)) return -1;
    ShotState st;
    ShotResult res;
    run_shot(*c, seed, shot, words, tau, cap, st, res, p0_trace);
    if (record)
        for (size_t i = 0; i < res.record.size(); ++i) record[i] = res.record[i];
    if (info) *info = res.info;
    for (int i = 0; i < 2 * c->n; ++i) {
        if (tab_x) tab_x[i] = st.x[i];
        if (tab_z) tab_z[i] = st.z[i];
        if (tab_r) tab_r[i] = (uint8_t)st.r[i];
    }
    if (n_coeff) *n_coeff = (uint32_t)st.v.size();
    uint32_t k = 0;
    for (const auto &kv : st.v) {
        if (k >= coeff_cap) break;
        if (alpha) alpha[k] = kv.first;
        if (re) re[k] = kv.second.real();
        if (im) im[k] = kv.second.imag();
        ++k;
    }
    return 0;
}

int oracle_batch(const oracle_circuit *c, uint64_t seed, uint64_t shot0, uint64_t n, const uint32_t *words,
                 double tau, uint32_t cap, int threads, uint32_t *outcomes, uint32_t *status, uint32_t *abort_op,
                 uint32_t *obs, uint32_t *max_support, uint64_t *work, uint64_t *shared_work) {
    if (!c || !(tau >= 0.0)) return -1;
    if (threads < 1) threads = 1;
    const uint64_t stride = (uint64_t)c->n_noise + c->n_meas;
    const int nw = (c->n_rec + 31) / 32;
    std::vector<std::vector<uint64_t>> part(threads, std::vector<uint64_t>(2 * ORACLE_WORK_COUNT, 0));
    auto worker = [&](int t) {
        uint64_t lo = n * t / threads, hi = n * (t + 1) / threads;
        ShotState st;
        ShotResult res;
        for (uint64_t i = lo; i < hi; ++i) {
            run_shot(*c, seed, shot0 + i, words ? words + i * stride : nullptr, tau, cap, st, res, nullptr);
            for (int w = 0; w < nw; ++w)
                if (outcomes) outcomes[(uint64_t)w * n + i] = res.record[w];
            if (status) status[i] = res.info.status;
            if (abort_op) abort_op[i] = res.info.abort_op;
            if (obs) obs[i] = res.info.obs;
            if (max_support) max_support[i] = res.info.max_support;
            part[t][0] += res.info.t_entries;
            part[t][1] += res.info.t_phase_entries;
            part[t][2] += res.info.m_entries;
            part[t][3] += res.info.noise_slots;
            part[t][4] += res.info.events;
            part[t][5] += res.info.noise_words;
            part[t][6] += res.info.m_out_entries;
            part[t][7] += res.info.m_pairs;
            part[t][8] += res.info.t_phase_flips;
            part[t][9] += res.info.meas_words;
            for (int k = 0; k < ORACLE_WORK_COUNT; ++k) part[t][ORACLE_WORK_COUNT + k] += res.info.shared[k];
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; ++t) pool.emplace_back(worker, t);
    worker(0);
    for (auto &th : pool) th.join();
    if (work)
        for (int k = 0; k < ORACLE_WORK_COUNT; ++k) {
            work[k] = 0;
            for (int t = 0; t < threads; ++t) work[k] += part[t][k];
        }
    if (shared_work)
        for (int k = 0; k < ORACLE_WORK_COUNT; ++k) {
            shared_work[k] = 0;
            for (int t = 0; t < threads; ++t) shared_work[k] += part[t][ORACLE_WORK_COUNT + k];
        }
    return 0;
}

void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) { philox4x32_10(ctr, key, out); }

void oracle_pauli_mul(const uint64_t a[3], const uint64_t b[3], uint64_t out[3]) {
    Pauli A, B;
    A.x = a[0]; A.z = a[1]; A.e = mod4((int)(a[2] & 3));
    B.x = b[0]; B.z = b[1]; B.e = mod4((int)(b[2] & 3));
    Pauli C = mul(A, B);
    out[0] = C.x; out[1] = C.z; out[2] = (uint64_t)C.e;
}

}  // extern "C"
