// compile.cpp -- parse circuit text, insert model noise, and compile the
// shot-independent frame into events for the sampler kernel.
//
// Method (arXiv 2512.23037): the generalized stabilizer state of
// Definition 1, updated by the rules of Theorem 1 -- Cliffords conjugate the
// tableau, T/T-dagger expand into I and Z_q (Eqs. 1-2) acting on the basis
// through the index shift of Eq. 4, and Pauli measurements project with
// (I +- P)/2 after the Aaronson-Gottesman pivot.  This file does the part of
// that work that is the same for every shot (see program.h).
#include "compile.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <map>

namespace soft {
namespace {

// ---------------------------------------------------------------------------
// Pauli strings with a phase: i^ph * prod_q sigma(x_q, z_q), sigma(1,1) = Y.
// Products go qubit by qubit through the single-qubit table
// sigma_a sigma_b = i^{kTab[a][b]} sigma_{a^b}, codes I=0, X=1, Z=2, Y=3.
// ---------------------------------------------------------------------------
struct PauliStr {
    uint64_t x = 0, z = 0;
    int ph = 0;
};

const int kTab[4][4] = {
    // I  X  Z  Y   (right factor)
    {0, 0, 0, 0},   // I
    {0, 0, 3, 1},   // X: XZ = -iY, XY = iZ
    {0, 1, 0, 3},   // Z: ZX = iY,  ZY = -iX
    {0, 3, 1, 0},   // Y: YX = -iZ, YZ = iX
};

PauliStr times(const PauliStr &a, const PauliStr &b) {
    PauliStr c;
    c.x = a.x ^ b.x;
    c.z = a.z ^ b.z;
    int ph = a.ph + b.ph;
    uint64_t both = (a.x | a.z) & (b.x | b.z);
    while (both) {
        int q = __builtin_ctzll(both);
        both &= both - 1;
        int ca = (int)((a.x >> q) & 1) | (int)(((a.z >> q) & 1) << 1);
        int cb = (int)((b.x >> q) & 1) | (int)(((b.z >> q) & 1) << 1);
        ph += kTab[ca][cb];
    }
    c.ph = ph & 3;
    return c;
}

inline int par64(uint64_t w) { return __builtin_parityll(w); }
inline uint64_t bitq(int q) { return 1ULL << q; }

// Two-word row mask: bit i of d = destabilizer row i, of s = stabilizer row i.
struct RowMask {
    uint64_t d = 0, s = 0;
    RowMask operator^(const RowMask &o) const { return {d ^ o.d, s ^ o.s}; }
    RowMask operator&(const RowMask &o) const { return {d & o.d, s & o.s}; }
    RowMask operator|(const RowMask &o) const { return {d | o.d, s | o.s}; }
    RowMask &operator^=(const RowMask &o) { d ^= o.d; s ^= o.s; return *this; }
};

// A GF(2) span kept in reduced echelon form (each row has its own top bit,
// which no other row has).
struct Echelon {
    std::vector<uint64_t> rows;
    static uint64_t top(uint64_t v) { return 1ULL << (63 - __builtin_clzll(v)); }
    uint64_t reduce(uint64_t v) const {
        for (uint64_t r : rows)
            if (v & top(r)) v ^= r;
        return v;
    }
    bool contains(uint64_t v) const { return reduce(v) == 0; }
    void add(uint64_t v) {
        v = reduce(v);
        if (!v) return;
        for (uint64_t &r : rows)
            if (r & top(v)) r ^= v;
        rows.push_back(v);
    }
};

// Tile entries a T writes at span dimension k: 2^k if its index shift lies
// in the span (butterfly or phase), 2^(k+1) if it adds a coordinate.
// cheap_order: an order of gates with index shifts `shift`, applied from the
// span `basis`, with a small sum of those costs: the better of a greedy order
// (a gate inside the span first, else the one that brings the most remaining
// shifts into the span) and a beam search over partial orders (states with
// the same span and the same gates left are merged).
static uint64_t order_cost(const std::vector<uint64_t> &shift, const std::vector<uint64_t> &basis,
                           const std::vector<size_t> &order) {
    Echelon span;
    for (uint64_t v : basis) span.add(v);
    uint64_t c = 0;
    for (size_t i : order) {
        const size_t k = span.rows.size();
        if (span.contains(shift[i])) {
            c += 1ull << k;
        } else {
            c += 2ull << k;
            span.add(shift[i]);
        }
    }
    return c;
}

static std::vector<size_t> cheap_order(const std::vector<uint64_t> &shift, const std::vector<uint64_t> &basis) {
    const size_t n = shift.size();
    Echelon start;
    for (uint64_t v : basis) start.add(v);
    // greedy
    std::vector<size_t> greedy;
    {
        Echelon span = start;
        std::vector<bool> done(n, false);
        for (size_t step = 0; step < n; ++step) {
            size_t pick = n;
            for (size_t i = 0; i < n && pick == n; ++i)
                if (!done[i] && span.contains(shift[i])) pick = i;
            if (pick == n) {
                int best = -1;
                for (size_t i = 0; i < n; ++i) {
                    if (done[i]) continue;
                    Echelon grown = span;
                    grown.add(shift[i]);
                    int inside = 0;
                    for (size_t j = 0; j < n; ++j)
                        if (!done[j] && j != i && grown.contains(shift[j])) ++inside;
                    if (inside > best) {
                        best = inside;
                        pick = i;
                    }
                }
            }
            done[pick] = true;
            span.add(shift[pick]);
            greedy.push_back(pick);
        }
    }
    if (n > 64) return greedy;
    // beam search
    struct State {
        uint64_t cost;
        Echelon span;
        uint64_t left;  // bit i: gate i not placed yet
        std::vector<size_t> order;
    };
    constexpr size_t kWidth = 256;
    std::vector<State> beam{{0, start, n == 64 ? ~0ull : ((1ull << n) - 1ull), {}}};
    for (size_t step = 0; step < n; ++step) {
        std::map<std::pair<std::vector<uint64_t>, uint64_t>, State> next;
        for (const State &st : beam) {
            const size_t k = st.span.rows.size();
            for (size_t i = 0; i < n; ++i) {
                if (!((st.left >> i) & 1ull)) continue;
                State nx{st.cost, st.span, st.left & ~(1ull << i), st.order};
                if (nx.span.contains(shift[i])) {
                    nx.cost += 1ull << k;
                } else {
                    nx.cost += 2ull << k;
                    nx.span.add(shift[i]);
                }
                nx.order.push_back(i);
                std::vector<uint64_t> key = nx.span.rows;
                std::sort(key.begin(), key.end());
                auto it = next.find({key, nx.left});
                if (it == next.end() || nx.cost < it->second.cost) next[{key, nx.left}] = std::move(nx);
            }
        }
        beam.clear();
        for (auto &kv : next) beam.push_back(std::move(kv.second));
        std::stable_sort(beam.begin(), beam.end(), [](const State &a, const State &b) { return a.cost < b.cost; });
        if (beam.size() > kWidth) beam.resize(kWidth);
    }
    return beam[0].cost < order_cost(shift, basis, greedy) ? beam[0].order : greedy;
}

// The shot-independent tableau, by column, plus the span and the event list.
class FrameCompiler {
  public:
    FrameCompiler(int n, Program &prog, bool speculate) : spec_(speculate), n_(n), P_(prog), cx_(n), cz_(n) {
        for (int q = 0; q < n; ++q) {
            cx_[q].d = bitq(q);  // d_q = X_q
            cz_[q].s = bitq(q);  // s_q = Z_q
        }
    }

    // ---- Cliffords: x/z columns move, sign flips accumulate in acc_ ----
    void h(int a) {
        sync();
        spec_touch(a);
        acc_ ^= cx_[a] & cz_[a];
        std::swap(cx_[a], cz_[a]);
    }
    void s(int a) {
        sync();
        acc_ ^= cx_[a] & cz_[a];
        cz_[a] ^= cx_[a];
    }
    void sdg(int a) {
        sync();
        RowMask notz = {~cz_[a].d, ~cz_[a].s};
        acc_ ^= cx_[a] & notz;
        cz_[a] ^= cx_[a];
    }
    // (X + Y)/sqrt2: X -> Y, Y -> X, Z -> -Z
    void hxy(int a) {
        sync();
        spec_touch(a);
        RowMask notx = {~cx_[a].d, ~cx_[a].s};
        acc_ ^= cz_[a] & notx;
        cz_[a] ^= cx_[a];
    }
    // (X - Y)/sqrt2: X -> -Y, Y -> -X, Z -> -Z
    void hnxy(int a) {
        sync();
        spec_touch(a);
        acc_ ^= cx_[a] | cz_[a];
        cz_[a] ^= cx_[a];
    }
    void px(int a) {
        sync();
        spec_touch(a);
        acc_ ^= cz_[a];
    }
    void pz(int a) {
        sync();
        acc_ ^= cx_[a];
    }
    void py(int a) {
        sync();
        spec_touch(a);
        acc_ ^= cx_[a] ^ cz_[a];
    }
    void cnot(int a, int b) {
        sync();
        spec_touch(b);  // Z_a commutes with CNOT(a -> b), Z_b does not
        RowMask t = cx_[b] ^ cz_[a];
        RowMask nt = {~t.d, ~t.s};
        acc_ ^= cx_[a] & cz_[b] & nt;
        cx_[b] ^= cx_[a];
        cz_[a] ^= cz_[b];
    }
    void cz(int a, int b) {
        sync();
        acc_ ^= cx_[a] & cx_[b] & (cz_[a] ^ cz_[b]);
        cz_[a] ^= cx_[b];
        cz_[b] ^= cx_[a];
    }

    // ---- noise locations ----
    void noise(uint32_t kind, double p, int a, int b, uint32_t rec) {
        if (!(p > 0.0)) return;
        // noise on qubits whose closing T is held back commutes with the
        // other held-back T gates and stays after its own: it may wait
        if (!buf_.empty() && !(kind != NZ_FLIP && a >= 0 && ((buf_mask_ >> a) & 1ull) &&
                               (b < 0 || ((buf_mask_ >> b) & 1ull))))
            sync();
        NoiseLoc L;
        std::memset(&L, 0, sizeof(L));
        L.thr = (uint64_t)std::floor(p * 4294967296.0);
        L.kind = L.thr == 0 ? NZ_NONE : kind;
        L.rec = rec;
        if (a >= 0) {
            L.masks[0] = cz_[a].d; L.masks[1] = cz_[a].s;   // anticommute with X_a
            L.masks[2] = cx_[a].d; L.masks[3] = cx_[a].s;   // anticommute with Z_a
        }
        if (b >= 0) {
            L.masks[4] = cz_[b].d; L.masks[5] = cz_[b].s;
            L.masks[6] = cx_[b].d; L.masks[7] = cx_[b].s;
        }
        P_.noise.push_back(L);
        P_.noise_p.push_back(p);
        P_.noise_tm1.push_back(L.thr == 0 ? 0u : (uint32_t)(L.thr - 1));
    }

    // ---- events ----
    void t_gate(int q, bool dagger, uint32_t src) {
        if (spec_) {
            // A T joins the held-back layer when its qubit is not in it yet
            // and it is of the layer's kind (it undoes an open T, or it opens
            // one); otherwise the layer is emitted first and a new one starts.
            const bool closing = open_match(q, dagger) >= 0;
            if (((buf_mask_ >> q) & 1ull) || (!buf_.empty() && closing != buf_closing_)) sync();
            const int idx = open_match(q, dagger);
            if (buf_.empty()) {
                buf_noise_ = (uint32_t)P_.noise.size();
                buf_closing_ = idx >= 0;
            }
            buf_.push_back({q, dagger, src, idx >= 0 ? (size_t)idx : 0u});
            buf_mask_ |= bitq(q);
            return;
        }
        emit_t(q, dagger, src);
    }

    void emit_t(int q, bool dagger, uint32_t src) {
        PauliStr Z;
        Z.z = bitq(q);
        const uint32_t k_before = (uint32_t)basis_.size();
        Event E = begin(src);
        uint64_t beta, gamma;
        int cexp;
        decompose(Z, beta, gamma, cexp);
        E.beta = beta;
        E.gamma = gamma;
        E.cexp = (uint32_t)cexp;
        E.g = gmask(gamma);
        if (dagger) E.flags |= EVF_TDG;
        const double s = dagger ? -1.0 : 1.0;
        const double th = M_PI / 8.0;
        const double cs = std::cos(th), sn = std::sin(th);
        if (beta == 0) {
            if (cexp & 1) throw CompileError{0, "internal: imaginary phase on a diagonal T"};
            E.kind = EV_T_PHASE;
            // lambda = -1 entries: e^{i s theta}(cos theta + i s sin theta) = e^{i s pi/4}
            E.Are = std::sqrt(0.5);
            E.Aim = s * std::sqrt(0.5);
        } else {
            // T^s = e^{i s theta}(cos theta - i s sin theta Z_q).  The global
            // factor e^{i s theta} is counted per shot; the rest is
            // cos theta v + sin theta i^qb c' v_partner with i^qb = (-i s) i^cexp.
            E.Tn = sn / cs;
            E.Cs2 = cs * cs;
            E.iCs2 = 1.0 / E.Cs2;
            E.Tnf = (float)E.Tn;
            E.qb = (uint32_t)((cexp + (dagger ? 1 : 3)) & 3);
            uint32_t mu;
            if (coords(beta, mu)) {
                E.kind = EV_T_BFLY;
                E.mu = mu;
                E.tstar = 31 - __builtin_clz(mu);
            } else {
                E.kind = EV_T_DOUBLE;
                basis_.push_back(beta);
                if (basis_.size() > kMaxSpanDim)
                    throw CompileError{0, "coefficient span dimension exceeds " + std::to_string(kMaxSpanDim)};
                if (basis_.size() > P_.kmax) P_.kmax = (uint32_t)basis_.size();
            }
            pass_shape(E);
        }
        finish(E);
        // coordinates this T's term needs: its new coordinate, or mu's top bit
        const uint32_t need = E.kind == EV_T_DOUBLE ? k_before + 1u : E.kind == EV_T_BFLY ? E.tstar + 1u : 0u;
        spec_after_t(q, dagger, k_before, src, need);
    }

    // Diagonal gate e^{i phi_x} on basis state x of the qubits qs (bit j of x
    // = qubit qs[j]), m <= 3, in one pass: U = sum_g c_g Z^g over the Z-strings
    // of its qubits, each term shifting the coefficients by its beta (Eq. 4).
    // The span grows by the new betas (terms with c_g = 0 are left out), and
    // the kernel runs one coset of the shifts' span per lane (DiagInfo).
    // With a condition (`cond` not empty: record bits, XOR or with and_form
    // AND) the gate is applied only in shots where it holds; the span grows in
    // every shot and holds zeros at the new coordinates where it does not.
    void diag(const std::vector<int> &qs, const std::vector<double> &phi, uint32_t src,
              const std::vector<int> &cond = std::vector<int>(), bool and_form = false) {
        sync();
        spec_reset();  // the span grows: no T pair of an open run can be dropped past this gate
        const uint32_t m = (uint32_t)qs.size(), ng = 1u << m;
        Event E = begin(src);
        E.kind = EV_DIAG;
        if (!cond.empty()) {
            E.flags |= EVF_COND;
            set_condition(E, cond, and_form);
        }
        DiagInfo D;
        std::memset(&D, 0, sizeof(D));
        D.ng = ng;
        uint64_t beta[8], gamma[8];
        int cexp[8];
        std::complex<double> dg[8];
        for (uint32_t g = 0; g < ng; ++g) {
            std::complex<double> c(0.0, 0.0);
            for (uint32_t x = 0; x < ng; ++x) {
                const std::complex<double> e = std::polar(1.0, phi[x]);
                if (__builtin_parity(g & x)) c -= e;
                else c += e;
            }
            c /= (double)ng;
            PauliStr Z;
            for (uint32_t j = 0; j < m; ++j)
                if ((g >> j) & 1u) Z.z |= bitq(qs[j]);
            decompose(Z, beta[g], gamma[g], cexp[g]);
            static const std::complex<double> ipw[4] = {{1, 0}, {0, 1}, {-1, 0}, {0, -1}};
            dg[g] = c * ipw[cexp[g] & 3];
            // a new index shift adds a coordinate (as a T doubling does)
            uint32_t mu;
            if ((c.real() != 0.0 || c.imag() != 0.0) && !coords(beta[g], mu)) {
                basis_.push_back(beta[g]);
                if (basis_.size() > kMaxSpanDim)
                    throw CompileError{0, "coefficient span dimension exceeds " + std::to_string(kMaxSpanDim)};
                if (basis_.size() > P_.kmax) P_.kmax = (uint32_t)basis_.size();
            }
        }
        D.knew = (uint32_t)basis_.size();
        // the shifts in the grown span, and a reduced echelon basis of their span
        uint32_t mus[8];
        std::vector<uint32_t> ech;  // rows with distinct top bits
        for (uint32_t g = 0; g < ng; ++g) {
            mus[g] = 0;
            if (dg[g].real() == 0.0 && dg[g].imag() == 0.0) continue;
            if (!coords(beta[g], mus[g])) throw CompileError{0, "internal: diagonal term outside the span"};
            uint32_t v = mus[g];
            for (uint32_t e : ech)
                if (v & (1u << (31 - __builtin_clz(e)))) v ^= e;
            if (!v) continue;
            const uint32_t tb = 1u << (31 - __builtin_clz(v));
            for (uint32_t &e : ech)
                if (e & tb) e ^= v;
            ech.push_back(v);
        }
        std::sort(ech.begin(), ech.end());  // ascending top bits
        D.r = (uint32_t)ech.size();
        for (uint32_t i = 0; i < D.r; ++i) D.lead |= (uint32_t)(31 - __builtin_clz(ech[i])) << (5 * i);
        for (uint32_t u = 0; u < (1u << D.r); ++u) {
            D.E[u] = 0;
            for (uint32_t i = 0; i < D.r; ++i)
                if ((u >> i) & 1u) D.E[u] ^= ech[i];
        }
        for (uint32_t g = 0; g < ng; ++g) {
            D.beta[g] = beta[g];
            D.gamma[g] = gamma[g];
            D.dre[g] = dg[g].real();
            D.dim[g] = dg[g].imag();
            D.fre[g] = (float)D.dre[g];
            D.fim[g] = (float)D.dim[g];
            D.gm[g] = gmask(gamma[g]);
            uint32_t ug = 0;
            for (uint32_t i = 0; i < D.r; ++i)
                if ((mus[g] >> (31 - __builtin_clz(ech[i]))) & 1u) ug |= 1u << i;
            D.ug[g] = ug;
        }
        E.boff = (uint32_t)P_.diag.size();
        E.bcnt = D.knew;
        P_.diag.push_back(D);
        finish(E);
    }

    // The branching T pass runs its entries 64 lanes at a time; iteration
    // bit u sets coordinate bit pos(u) (a new coordinate: u + 6; a butterfly:
    // the bits outside the lane bits and tstar).  The iterations' signs
    // (-1)^(g . J) pair up on the lowest such bit in g.
    static void pass_shape(Event &E) {
        const bool bfly = E.kind == EV_T_BFLY;
        const uint32_t h = bfly ? E.tstar : 32u;
        const uint32_t entries = bfly ? (1u << (E.k - 1u)) : (1u << E.k);
        const uint32_t iters = (entries + 63u) >> 6;
        E.tpair = 0;
        for (uint32_t u = 0; (1u << u) < iters; ++u) {
            const uint32_t b = u + 6u < h ? u + 6u : u + 7u;
            if ((E.g >> b) & 1u) {
                E.tpair = 1u << b;
                break;
            }
        }
        E.lmask = bfly ? (((63u >> h) << (h + 1u)) | (63u & ((1u << h) - 1u))) : 63u;
    }

    // Measurement of P (Hermitian, sign +); reset adds a conditional X_q.
    // reset_z: the reset flips with Z_q (X-basis reset) instead of X_q.
    void measure(const PauliStr &P, uint32_t mslot, int rec, int reset_q, uint32_t src, bool reset_z = false) {
        sync();
        if ((P.x & open_mask_) || (reset_q >= 0 && !reset_z && ((open_mask_ >> reset_q) & 1ull))) spec_reset();
        Event E = begin(src);
        uint64_t beta, gamma;
        int cexp;
        decompose(P, beta, gamma, cexp);
        E.beta = beta;
        E.gamma = gamma;
        E.cexp = (uint32_t)cexp;
        E.g = gmask(gamma);
        E.gbeta = (uint32_t)par64(gamma & beta);
        E.mslot = mslot;
        if (rec >= 0) {
            E.flags |= EVF_RECORD;
            E.rec = (uint32_t)rec;
        }
        const uint32_t k = (uint32_t)basis_.size();
        if (beta == 0) {
            if (cexp & 1) throw CompileError{0, "internal: imaginary phase on a diagonal measurement"};
            if (E.g == 0) {
                E.kind = EV_M_DET;
            } else {
                E.kind = EV_M_CUT;
                uint32_t ts = 31 - __builtin_clz(E.g);
                E.tstar = ts;
                E.avec = basis_[ts];
                std::vector<uint64_t> nb;
                for (uint32_t t = 0; t < k; ++t)
                    if (t != ts) nb.push_back(basis_[t] ^ (((E.g >> t) & 1) ? basis_[ts] : 0));
                basis_.swap(nb);
            }
        } else {
            const int p = __builtin_ctzll(beta);
            E.pbit = (uint32_t)p;
            E.avec = beta;
            uint32_t pm = 0;
            for (uint32_t t = 0; t < k; ++t) pm |= (uint32_t)((basis_[t] >> p) & 1) << t;
            E.pm = pm;
            uint32_t mu;
            std::vector<uint64_t> nb;
            auto L = [&](uint64_t v) { return ((v >> p) & 1) ? (v ^ beta) : v; };
            if (coords(beta, mu)) {
                E.kind = EV_M_MERGE;
                E.mu = mu;
                uint32_t ts = 31 - __builtin_clz(mu);
                E.tstar = ts;
                for (uint32_t t = 0; t < k; ++t)
                    if (t != ts) nb.push_back(L(basis_[t]));
            } else {
                E.kind = EV_M_SPLIT;
                for (uint32_t t = 0; t < k; ++t) nb.push_back(L(basis_[t]));
            }
            basis_.swap(nb);
            // Tableau: rows anticommuting with P (other than d_p, s_p) absorb
            // s_p, d_p takes s_p, s_p becomes +-P.
            PauliStr sp = row_s(p);
            RowMask A = {gamma & ~bitq(p), beta & ~bitq(p)};
            E.AD = A.d;
            E.AS = A.s;
            for (uint64_t w = A.d; w; w &= w - 1) {
                int i = __builtin_ctzll(w);
                PauliStr prod = times(row_d(i), sp);
                if (prod.ph & 1) throw CompileError{0, "internal: non-Hermitian row"};
                if (prod.ph == 2) E.PhD |= bitq(i);
            }
            for (uint64_t w = A.s; w; w &= w - 1) {
                int i = __builtin_ctzll(w);
                PauliStr prod = times(row_s(i), sp);
                if (prod.ph & 1) throw CompileError{0, "internal: non-Hermitian row"};
                if (prod.ph == 2) E.PhS |= bitq(i);
            }
            for (uint64_t w = sp.x; w; w &= w - 1) {
                int q = __builtin_ctzll(w);
                cx_[q] ^= A;
            }
            for (uint64_t w = sp.z; w; w &= w - 1) {
                int q = __builtin_ctzll(w);
                cz_[q] ^= A;
            }
            set_row(false, p, sp.x, sp.z);
            set_row(true, p, P.x, P.z);
        }
        if (E.kind != EV_M_DET) spec_reset();  // the span changed
        if (reset_q >= 0) {  // rows anticommuting with the flip, in the frame after the measurement
            E.flags |= EVF_RESET;
            const RowMask &m = reset_z ? cx_[reset_q] : cz_[reset_q];
            E.xD = m.d;
            E.xS = m.s;
        }
        finish(E);
    }

    // Record indices as (word, mask) pairs appended to the pair table: under
    // XOR repeated bits cancel, under AND (merge) they stand once.  Returns the
    // number of pairs; `off` receives the first.
    uint32_t record_pairs(const std::vector<int> &recs, bool merge, uint32_t &off) {
        std::vector<uint32_t> words, masks;
        for (int r : recs) {
            uint32_t w = (uint32_t)r >> 5, m = 1u << (r & 31);
            size_t i = 0;
            while (i < words.size() && words[i] != w) ++i;
            if (i == words.size()) { words.push_back(w); masks.push_back(0); }
            masks[i] = merge ? (masks[i] | m) : (masks[i] ^ m);
        }
        off = (uint32_t)(P_.det_pairs.size() / 2);
        for (size_t i = 0; i < words.size(); ++i)
            if (masks[i]) { P_.det_pairs.push_back(words[i]); P_.det_pairs.push_back(masks[i]); }
        return (uint32_t)(P_.det_pairs.size() / 2) - off;
    }

    // The condition of a classically controlled event: its record pairs, the
    // first one inline, and EVF_AND for the all-bits form.
    void set_condition(Event &E, const std::vector<int> &recs, bool and_form) {
        uint32_t off = 0;
        const uint32_t cnt = record_pairs(recs, and_form, off);
        E.det_off = off;
        E.det_cnt = cnt;
        if (cnt) {
            E.dw0 = P_.det_pairs[2 * off];
            E.dm0 = P_.det_pairs[2 * off + 1];
        }
        if (and_form) E.flags |= EVF_AND;
    }

    void parity_check(bool detector, int expect, const std::vector<int> &recs, uint32_t obs, uint32_t src) {
        sync();
        uint32_t off = 0;
        const uint32_t cnt = record_pairs(recs, false, off);
        auto fill = [&](Event &E) {
            E.expect = (uint32_t)expect;
            E.det_off = off;
            E.det_cnt = cnt;
            if (cnt) {
                E.dw0 = P_.det_pairs[2 * off];
                E.dm0 = P_.det_pairs[2 * off + 1];
            }
        };
        // A detector right after a measurement, with no noise and no Clifford
        // in between, becomes a check inside that measurement's event.
        if (detector && !P_.events.empty()) {
            Event &last = P_.events.back();
            const bool meas = last.kind >= EV_M_DET && last.kind <= EV_M_MERGE;
            if (meas && !(last.flags & EVF_CHECK) && P_.noise.size() == noise_at_finish_ && acc_.d == 0 &&
                acc_.s == 0) {
                last.flags |= EVF_CHECK;
                last.chk_src = src;
                fill(last);
                return;
            }
        }
        Event E = begin(src);
        E.kind = detector ? EV_DETECTOR : EV_OBSERVABLE;
        E.rec = obs;
        fill(E);
        finish(E);
    }

    // Pauli (1 X, 2 Y, 3 Z) on qubit q when the XOR (and_form: the AND) of
    // the record bits `recs` is 1.
    void feedback(int pauli, int q, const std::vector<int> &recs, bool and_form, uint32_t src) {
        sync();
        if (pauli != 3) spec_touch(q);
        Event E = begin(src);
        E.kind = EV_FEEDBACK;
        E.rec = recs.empty() ? 0u : (uint32_t)recs[0];
        set_condition(E, recs, and_form);
        RowMask m;
        if (pauli == 1 || pauli == 2) m ^= cz_[q];
        if (pauli == 3 || pauli == 2) m ^= cx_[q];
        E.xD = m.d;
        E.xS = m.s;
        finish(E);
    }

    void end(uint32_t src) {
        sync();
        Event E = begin(src);
        E.kind = EV_END;
        finish(E);
        // two more END events so that the kernel may always load events e + 1
        // and e + 2
        for (int i = 0; i < 2; ++i) {
            Event pad = E;
            P_.events.push_back(pad);
            P_.before.push_back(P_.before.back());
            P_.after.push_back(P_.after.back());
        }
    }

  private:
    // ---- speculative span truncation ----
    // T gates opened since a checkpoint (a point with span dimension ckpt_k_).
    // When every one of them has met its inverse on the same qubit, with
    // nothing in between that fails to commute with its Z, the product of the
    // pairs is the identity, so a shot whose noise did not break a pair has its
    // coefficients back on coordinates < ckpt_k_: a DROP event returns the span
    // to that dimension (the kernel checks the entries above are zero and
    // restarts the shot on the full event list otherwise).
    //
    // A layer of T gates on distinct qubits (with only noise on those qubits
    // in between) is held back and emitted in another order: the gates
    // commute, and each one's noise stays after it (all of the layer's noise
    // follows the layer).  A layer that undoes open T gates goes latest-opened
    // first, so the span can shrink step by step: after each closing T, the
    // still-open T gates need only the coordinates below the largest of their
    // `need` values (and the checkpoint's), so a DROP returns the span there.
    // A layer that opens T gates goes in an order with few tile entries
    // written (cheap_order).
    struct OpenT {
        int q;
        bool dagger;
        uint32_t need;  // coordinates its term reaches: new coordinate + 1, or mu's top bit + 1
    };
    struct HeldT {
        int q;
        bool dagger;
        uint32_t src;
        size_t open_idx;  // the open T it undoes
    };
    bool spec_;
    std::vector<OpenT> open_;
    uint64_t open_mask_ = 0;
    uint32_t ckpt_k_ = 0;
    std::vector<HeldT> buf_;
    uint64_t buf_mask_ = 0;
    uint32_t buf_noise_ = 0;          // noise slots when the layer started
    bool buf_closing_ = false;        // the held layer undoes open T gates
    int64_t noise_end_override_ = -1;  // noise_end of events emitted from the held layer

    int open_match(int q, bool dagger) const {
        for (size_t i = open_.size(); i-- > 0;)
            if (open_[i].q == q && open_[i].dagger != dagger) return (int)i;
        return -1;
    }
    // Emit the held-back layer, latest-opened first.
    void sync() {
        if (buf_.empty()) return;
        std::vector<HeldT> b;
        b.swap(buf_);
        buf_mask_ = 0;
        noise_end_override_ = buf_noise_;
        if (buf_closing_) {
            std::sort(b.begin(), b.end(), [](const HeldT &x, const HeldT &y) { return x.open_idx > y.open_idx; });
            for (const HeldT &t : b) emit_t(t.q, t.dagger, t.src);
        } else {
            std::vector<uint64_t> shift(b.size());
            for (size_t i = 0; i < b.size(); ++i) {
                PauliStr Z;
                Z.z = bitq(b[i].q);
                uint64_t gamma;
                int cexp;
                decompose(Z, shift[i], gamma, cexp);
            }
            for (size_t i : cheap_order(shift, basis_)) emit_t(b[i].q, b[i].dagger, b[i].src);
        }
        noise_end_override_ = -1;
    }

    void spec_reset() {
        open_.clear();
        open_mask_ = 0;
    }
    void spec_touch(int q) {
        if ((open_mask_ >> q) & 1ull) spec_reset();
    }
    void spec_after_t(int q, bool dagger, uint32_t k_before, uint32_t src, uint32_t need) {
        if (!spec_) return;
        const int i = open_match(q, dagger);
        if (i >= 0) {
            open_.erase(open_.begin() + i);
            open_mask_ = 0;
            uint32_t keep = ckpt_k_;
            for (const OpenT &o : open_) {
                open_mask_ |= bitq(o.q);
                keep = std::max(keep, o.need);
            }
            if (basis_.size() > keep) {
                Event &last = P_.events.back();  // the closing T just emitted
                if (keep + 1u == basis_.size() && last.kind == EV_T_BFLY && last.tstar + 1u == basis_.size()) {
                    // the butterfly's partner outputs are exactly the top
                    // coordinate's half: its pass checks them, no DROP event
                    last.flags |= EVF_DROP1;
                    basis_.resize(keep);
                    P_.after.back() = snapshot();
                } else {
                    Event D = begin(src);
                    D.kind = EV_DROP;
                    D.mu = keep;
                    basis_.resize(keep);
                    finish(D);
                }
            }
            return;
        }
        if (open_.empty()) ckpt_k_ = k_before;
        open_.push_back({q, dagger, need});
        open_mask_ |= bitq(q);
    }

    int n_;
    Program &P_;
    std::vector<RowMask> cx_, cz_;
    RowMask acc_;
    std::vector<uint64_t> basis_;
    size_t noise_at_finish_ = 0;  // noise slots when the last event was finished

    PauliStr row_d(int i) const {
        PauliStr r;
        for (int q = 0; q < n_; ++q) {
            r.x |= ((cx_[q].d >> i) & 1) << q;
            r.z |= ((cz_[q].d >> i) & 1) << q;
        }
        return r;
    }
    PauliStr row_s(int i) const {
        PauliStr r;
        for (int q = 0; q < n_; ++q) {
            r.x |= ((cx_[q].s >> i) & 1) << q;
            r.z |= ((cz_[q].s >> i) & 1) << q;
        }
        return r;
    }
    void set_row(bool stab, int i, uint64_t x, uint64_t z) {
        for (int q = 0; q < n_; ++q) {
            uint64_t &cxw = stab ? cx_[q].s : cx_[q].d;
            uint64_t &czw = stab ? cz_[q].s : cz_[q].d;
            cxw = (cxw & ~bitq(i)) | (((x >> q) & 1) << i);
            czw = (czw & ~bitq(i)) | (((z >> q) & 1) << i);
        }
    }

    // P = c * d_beta * s_gamma (Eq. 4): beta over the stabilizers, gamma over
    // the destabilizers, c = i^cexp when every row sign is +.
    void decompose(const PauliStr &P, uint64_t &beta, uint64_t &gamma, int &cexp) const {
        RowMask anti;
        for (uint64_t w = P.x; w; w &= w - 1) anti ^= cz_[__builtin_ctzll(w)];
        for (uint64_t w = P.z; w; w &= w - 1) anti ^= cx_[__builtin_ctzll(w)];
        beta = anti.s;
        gamma = anti.d;
        PauliStr R;
        for (uint64_t w = beta; w; w &= w - 1) R = times(R, row_d(__builtin_ctzll(w)));
        for (uint64_t w = gamma; w; w &= w - 1) R = times(R, row_s(__builtin_ctzll(w)));
        if (R.x != P.x || R.z != P.z) throw CompileError{0, "internal: decomposition mismatch"};
        cexp = (P.ph - R.ph + 8) & 3;
    }

    uint32_t gmask(uint64_t gamma) const {
        uint32_t g = 0;
        for (size_t t = 0; t < basis_.size(); ++t) g |= (uint32_t)par64(gamma & basis_[t]) << t;
        return g;
    }

    // Coordinates of v in the span basis, if it lies in the span.
    bool coords(uint64_t v, uint32_t &mu) const {
        // echelon form with coordinate bookkeeping
        std::vector<uint64_t> vec;
        std::vector<uint32_t> crd;
        for (size_t t = 0; t < basis_.size(); ++t) {
            uint64_t b = basis_[t];
            uint32_t c = 1u << t;
            for (size_t i = 0; i < vec.size(); ++i) {
                uint64_t top = 1ULL << (63 - __builtin_clzll(vec[i]));
                if (b & top) { b ^= vec[i]; c ^= crd[i]; }
            }
            if (!b) throw CompileError{0, "internal: dependent span basis"};
            // keep vec[] reduced: clear b's top bit from the others
            uint64_t top = 1ULL << (63 - __builtin_clzll(b));
            for (size_t i = 0; i < vec.size(); ++i)
                if (vec[i] & top) { vec[i] ^= b; crd[i] ^= c; }
            vec.push_back(b);
            crd.push_back(c);
        }
        uint32_t m = 0;
        for (size_t i = 0; i < vec.size(); ++i) {
            uint64_t top = 1ULL << (63 - __builtin_clzll(vec[i]));
            if (v & top) { v ^= vec[i]; m ^= crd[i]; }
        }
        mu = m;
        return v == 0;
    }

    Frame snapshot() const {
        Frame f;
        f.xd.resize(n_); f.xs.resize(n_); f.zd.resize(n_); f.zs.resize(n_);
        for (int q = 0; q < n_; ++q) {
            f.xd[q] = cx_[q].d; f.xs[q] = cx_[q].s; f.zd[q] = cz_[q].d; f.zs[q] = cz_[q].s;
        }
        f.basis = basis_;
        return f;
    }

    Event begin(uint32_t src) {
        Event E;
        std::memset(&E, 0, sizeof(E));
        E.src = src;
        E.noise_end = noise_end_override_ >= 0 ? (uint32_t)noise_end_override_ : (uint32_t)P_.noise.size();
        E.k = (uint32_t)basis_.size();
        E.cliffD = acc_.d;
        E.cliffS = acc_.s;
        acc_ = RowMask();
        P_.before.push_back(snapshot());
        return E;
    }
    void finish(const Event &E0) {
        Event E = E0;
        if (E.cliffD || E.cliffS) E.flags |= EVF_CLIFF;
        P_.events.push_back(E);
        P_.after.push_back(snapshot());
        noise_at_finish_ = P_.noise.size();
    }
};

// ---------------------------------------------------------------------------
// Runs of outcome-fixed measurements evaluated side by side (see BatchMember).
// ---------------------------------------------------------------------------
bool batchable(const Event &E) { return E.kind == EV_M_DET && (!(E.flags & EVF_CHECK) || E.det_cnt <= 1); }

void form_batches(Program &P) {
    const size_t ne = P.events.size();
    size_t e = 0;
    while (e < ne) {
        if (!batchable(P.events[e])) { ++e; continue; }
        std::vector<BatchMember> run;
        uint64_t cumD = 0, cumS = 0;
        int rl0 = -1, rc = 0;
        uint32_t r0 = 0;
        for (size_t i = e; i < ne && run.size() < kBatchMax; ++i) {
            const Event &E = P.events[i];
            const uint32_t m = (uint32_t)run.size();
            if (!batchable(E)) break;
            if (m > 0) {
                bool ok = true;
                // no record flips between the previous member and this one
                for (uint32_t s = P.events[i - 1].noise_end; s < E.noise_end && ok; ++s)
                    if (P.noise[s].kind == NZ_FLIP) ok = false;
                // earlier resets must commute with this measurement
                for (const BatchMember &B : run)
                    if ((B.info & BM_RESET) && (par64(B.xD & E.beta) ^ par64(B.xS & E.gamma))) ok = false;
                // recorded members on consecutive lanes with consecutive records
                if ((E.flags & EVF_RECORD) && rl0 >= 0 && !(rl0 + rc == (int)m && r0 + (uint32_t)rc == E.rec)) ok = false;
                // a folded check may read its own bit and bits from before the run
                if ((E.flags & EVF_CHECK) && E.det_cnt == 1 && rl0 >= 0) {
                    for (uint32_t mk = E.dm0; mk; mk &= mk - 1) {
                        const uint32_t r = E.dw0 * 32u + (uint32_t)__builtin_ctz(mk);
                        const bool own = (E.flags & EVF_RECORD) && r == E.rec;
                        if (!own && r >= r0) ok = false;
                    }
                }
                if (!ok) break;
                cumD ^= E.cliffD;
                cumS ^= E.cliffS;
            }
            BatchMember B;
            std::memset(&B, 0, sizeof(B));
            B.beta = E.beta;
            B.gamma = E.gamma;
            B.cumD = cumD;
            B.cumS = cumS;
            B.noise_end = E.noise_end;
            B.info = (E.cexp == 2 ? BM_CSIGN : 0u);
            if (E.flags & EVF_RECORD) {
                B.info |= BM_RECORD;
                if (rl0 < 0) { rl0 = (int)m; r0 = E.rec; }
                ++rc;
            }
            if (E.flags & EVF_RESET) {
                B.info |= BM_RESET;
                B.xD = E.xD;
                B.xS = E.xS;
            }
            if (E.flags & EVF_CHECK) {
                B.info |= BM_CHECK | (E.expect ? BM_EXPECT : 0u);
                B.chk_src = E.chk_src;
                if (E.det_cnt == 1) {
                    B.dw0 = E.dw0;
                    B.dm0 = E.dm0;
                    if ((E.flags & EVF_RECORD) && E.dw0 == (E.rec >> 5) && ((E.dm0 >> (E.rec & 31u)) & 1u)) {
                        B.info |= BM_OWN;
                        B.dm0 &= ~(1u << (E.rec & 31u));
                    }
                }
            }
            run.push_back(B);
        }
        if (run.size() < 2) { ++e; continue; }
        for (BatchMember &B : run) {
            B.r0 = r0;
            B.rlane = rl0 < 0 ? 0u : ((uint32_t)rl0 | ((uint32_t)rc << 8));
        }
        Event &F = P.events[e];
        F.flags |= EVF_BATCH;
        F.bcnt = (uint32_t)run.size();
        F.boff = (uint32_t)P.batch.size();
        P.batch.insert(P.batch.end(), run.begin(), run.end());
        e += run.size();
    }
}

// ---------------------------------------------------------------------------
// Text front end: one op per line, '#' comments, "QUBITS n" first.
// ---------------------------------------------------------------------------
struct Cursor {
    const std::string &t;
    size_t pos = 0;
    int line = 0;
};

bool next_line(Cursor &c, std::vector<std::string> &tok) {
    tok.clear();
    while (c.pos < c.t.size()) {
        size_t eol = c.t.find('\n', c.pos);
        if (eol == std::string::npos) eol = c.t.size();
        ++c.line;
        size_t end = c.t.find('#', c.pos);
        if (end == std::string::npos || end > eol) end = eol;
        size_t i = c.pos;
        while (i < end) {
            while (i < end && (c.t[i] == ' ' || c.t[i] == '\t' || c.t[i] == '\r')) ++i;
            size_t j = i;
            while (j < end && !(c.t[j] == ' ' || c.t[j] == '\t' || c.t[j] == '\r')) ++j;
            if (j > i) tok.emplace_back(c.t, i, j - i);
            i = j;
        }
        c.pos = eol + 1;
        if (!tok.empty()) return true;
    }
    return false;
}

int parse_uint(const std::string &s, int line) {
    if (s.empty() || s.size() > 9) throw CompileError{line, "bad integer '" + s + "'"};
    int v = 0;
    for (char ch : s) {
        if (ch < '0' || ch > '9') throw CompileError{line, "bad integer '" + s + "'"};
        v = v * 10 + (ch - '0');
    }
    return v;
}

double parse_prob(const std::string &s, int line) {
    char *endp = nullptr;
    double p = std::strtod(s.c_str(), &endp);
    if (endp == s.c_str() || *endp != '\0') throw CompileError{line, "bad probability '" + s + "'"};
    if (!(p >= 0.0 && p <= 1.0)) throw CompileError{line, "probability out of [0,1]"};
    return p;
}

uint64_t fnv1a(const void *data, size_t len, uint64_t h) {
    const unsigned char *p = (const unsigned char *)data;
    for (size_t i = 0; i < len; ++i) { h ^= p[i]; h *= 1099511628211ULL; }
    return h;
}

}  // namespace

// Speculative lists: a run of T doublings with no noise slot and no Clifford
// sign flip between them, whose final tile has at most 64 entries, runs as one
// pass (EVF_TRUN on the first; the members stay in the list, so the work
// counts do not change, and the kernel skips them).  Final entry J comes from
// entry J mod 2^k turned by i^{r_J + 2 (dynamic signs of the members whose
// coordinate J sets)} and multiplied by tan(pi/8) once per such member, in
// member order (the products of the separate passes, rounding included).
static void fuse_doublings(Program &P) {
    std::vector<Event> &ev = P.events;
    for (size_t s = 0; s < ev.size();) {
        Event &A = ev[s];
        if (A.kind != EV_T_DOUBLE || (A.flags & ~(EVF_TDG | EVF_CLIFF)) != 0u) {
            ++s;
            continue;
        }
        size_t m = 1;
        while (s + m < ev.size() && A.k + m + 1u <= 6u) {
            const Event &B = ev[s + m];
            if (B.kind != EV_T_DOUBLE || (B.flags & ~EVF_TDG) != 0u || B.noise_end != A.noise_end ||
                B.k != A.k + m || std::memcmp(&B.Tn, &A.Tn, sizeof(double)) != 0 ||
                std::memcmp(&B.iCs2, &A.iCs2, sizeof(double)) != 0)
                break;
            ++m;
        }
        if (m < 2) {
            ++s;
            continue;
        }
        const uint32_t k0 = A.k, K = A.k + (uint32_t)m;
        uint64_t r0 = 0, r1 = 0;
        uint32_t ph = 0;
        for (uint32_t J = 0; J < (1u << K); ++J) {
            uint32_t r = 0;
            for (uint32_t i = 0; i < m; ++i) {
                if (!((J >> (k0 + i)) & 1u)) continue;
                const Event &B = ev[s + i];
                const uint32_t j = J & ((1u << (k0 + i)) - 1u);
                r += B.qb + 2u * (uint32_t)(__builtin_popcount(B.g & j) & 1);
            }
            r0 |= (uint64_t)(r & 1u) << J;
            r1 |= (uint64_t)((r >> 1) & 1u) << J;
        }
        for (size_t i = 0; i < m; ++i) ph += (ev[s + i].flags & EVF_TDG) ? 15u : 1u;
        A.flags |= EVF_TRUN;
        A.bcnt = (uint32_t)m;
        A.boff = ph & 15u;
        A.trot0 = r0;
        A.trot1 = r1;
        s += m;
    }
}

// Speculative lists: a run of butterflies that each drop the top coordinate
// (EVF_DROP1), with no noise slot and no Clifford sign flip between them, on
// a tile of at most 64 entries, runs in registers (EVF_BRUN on the first; the
// members stay in the list and the kernel skips them).  Each member is the
// same butterfly, pruning and drop check as its own pass.
static void fuse_drop_runs(Program &P) {
    std::vector<Event> &ev = P.events;
    auto is_member = [](const Event &B) {
        return B.kind == EV_T_BFLY && (B.flags & EVF_DROP1) && B.tstar + 1u == B.k;
    };
    for (size_t s = 0; s < ev.size();) {
        Event &A = ev[s];
        if (!is_member(A) || A.k > 6u || (A.flags & ~(EVF_TDG | EVF_CLIFF | EVF_DROP1)) != 0u) {
            ++s;
            continue;
        }
        size_t m = 1;
        while (s + m < ev.size() && m < A.k) {
            const Event &B = ev[s + m];
            if (!is_member(B) || (B.flags & ~(EVF_TDG | EVF_DROP1)) != 0u || B.noise_end != A.noise_end ||
                B.k != A.k - m || std::memcmp(&B.Tn, &A.Tn, sizeof(double)) != 0 ||
                std::memcmp(&B.iCs2, &A.iCs2, sizeof(double)) != 0)
                break;
            ++m;
        }
        if (m < 2) {
            ++s;
            continue;
        }
        uint32_t ph = 0;
        for (size_t i = 0; i < m; ++i) ph += (ev[s + i].flags & EVF_TDG) ? 15u : 1u;
        A.flags |= EVF_BRUN;
        A.bcnt = (uint32_t)m;
        A.boff = ph & 15u;
        s += m;
    }
}

// Running work counts of the event list (see Event::cum_t): the span
// dimension before each event is the same in every shot, so the work of a
// shot that stops after event e is the sum over the events up to e.
// Events that read or write the coefficient tile.
static bool touches_tile(const Event &E) {
    return E.kind == EV_T_PHASE || E.kind == EV_T_DOUBLE || E.kind == EV_T_BFLY || E.kind == EV_M_CUT ||
           E.kind == EV_M_SPLIT || E.kind == EV_M_MERGE || E.kind == EV_DROP || E.kind == EV_DIAG;
}

// Checkpoints of the noiseless trajectory.  The kernel steps over a list one
// iteration at a time (a fused run of doublings or of dropping butterflies,
// or a run of outcome-fixed measurements, is one iteration), and a shot can
// start at any iteration boundary.  Up to the first measurement with a random
// outcome every event is deterministic in a shot that no noise has hit.  A
// checkpoint goes at each boundary where the iterations switch between those
// that touch the tile and those that do not (outcome-fixed measurements,
// checks, feedback), and before the first random measurement or the list's
// end, when noise slots lie between it and the last one; the first
// tile-touching iteration at or after a checkpoint is flagged EVF_MAT (a shot
// started there loads the checkpoint's tile then, if ever).
static void checkpoints(Program &out) {
    out.ckpts.clear();
    const uint32_t n = (uint32_t)out.events.size();
    uint32_t e = 0, nz = 0, last_nz = 0;
    int prev_tile = -1;
    bool need_mat = false;
    while (e < n) {
        Event &E = out.events[e];
        const bool tile = touches_tile(E);
        // the end of the list, or a measurement whose outcome is random: the
        // trajectory stops being shared here (a last checkpoint before it)
        const bool stop = E.kind == EV_END || E.kind == EV_M_CUT || E.kind == EV_M_SPLIT || E.kind == EV_M_MERGE;
        if (e > 0 && prev_tile >= 0 && ((int)tile != prev_tile || stop) && (nz > last_nz || out.ckpts.empty()) &&
            out.ckpts.size() < kMaxCheckpoints) {
            out.ckpts.push_back(Checkpoint{e, nz});
            last_nz = nz;
            need_mat = true;
        }
        if (tile && need_mat) {
            E.flags |= EVF_MAT;
            need_mat = false;
        }
        if (stop) break;
        const uint32_t step = (E.flags & (EVF_TRUN | EVF_BRUN)) ? E.bcnt
                            : (E.kind == EV_M_DET && (E.flags & EVF_BATCH)) ? E.bcnt : 1u;
        for (uint32_t i = 0; i < step && e + i < n; ++i) nz = std::max(nz, out.events[e + i].noise_end);
        prev_tile = tile ? 1 : 0;
        e += step;
    }
}

// Deferrable T runs: consecutive iterations of T gates (non-branching,
// doublings, butterflies that do not drop, fused runs of doublings) with no
// noise slot and no Clifford sign flip between their events, after which the
// list goes on with events that do not touch the tile.  The signs do not
// depend on T gates, so the events up to the next tile-touching one run the
// same whether the run was applied or not; a shot that a check ends before
// then never needs the run's coefficients.  The first event gets EVF_DEFER
// (mslot = the run's events) and the next tile-touching iteration EVF_MAT.
static void deferrable_runs(Program &out) {
    const uint32_t n = (uint32_t)out.events.size();
    auto step_of = [&](const Event &E) -> uint32_t {
        return (E.flags & (EVF_TRUN | EVF_BRUN)) ? E.bcnt : (E.kind == EV_M_DET && (E.flags & EVF_BATCH)) ? E.bcnt : 1u;
    };
    auto is_t = [&](const Event &E) {
        return E.kind == EV_T_PHASE || E.kind == EV_T_DOUBLE || (E.kind == EV_T_BFLY && !(E.flags & (EVF_DROP1 | EVF_BRUN)));
    };
    uint32_t e = 0;
    while (e < n && out.events[e].kind != EV_END) {
        if (!is_t(out.events[e])) {
            e += step_of(out.events[e]);
            continue;
        }
        // the longest run from e
        const uint32_t d0 = e, nz = out.events[e].noise_end;
        uint32_t d1 = e;
        while (d1 < n && is_t(out.events[d1])) {
            const Event &E = out.events[d1];
            const uint32_t st = step_of(E);
            bool ok = true;
            for (uint32_t i = 0; i < st; ++i) {
                const Event &M = out.events[d1 + i];
                if (M.noise_end != nz || (d1 + i > d0 && (M.flags & EVF_CLIFF))) ok = false;
            }
            if (!ok) break;
            d1 += st;
        }
        // followed by events that do not touch the tile, then (maybe) one that does
        uint32_t f = d1;
        while (f < n && out.events[f].kind != EV_END && !touches_tile(out.events[f])) f += step_of(out.events[f]);
        if (f > d1) {
            out.events[d0].flags |= EVF_DEFER;
            out.events[d0].mslot = d1 - d0;
            if (f < n && out.events[f].kind != EV_END) out.events[f].flags |= EVF_MAT;
        }
        e = d1;
    }
}

// Butterfly pairs: a plain butterfly (mu) followed by a butterfly (mu'),
// plain or the last before a drop, on the same span with no noise slot and no
// Clifford flip between them.  The pair runs as one pass over the quads
// {j, j^mu, j^mu', j^mu^mu'}: the first butterfly on the quad's two mu-pairs,
// then the second on its two mu'-pairs, so each entry is read and written once
// instead of twice.  The quads are indexed by the coordinates less two bits
// that mu and mu' pivot on: mu's top bit, and the top bit of mu' once mu is
// taken out of it (so the two are independent and the quads tile the span).
// Spans below 2^8 (fewer than 64 quads) are left alone.
static void butterfly_pairs(Program &out) {
    const uint32_t n = (uint32_t)out.events.size();
    auto plain = [](const Event &E) {
        return E.kind == EV_T_BFLY && !(E.flags & (EVF_DROP1 | EVF_TRUN | EVF_BRUN | EVF_PAIR));
    };
    for (uint32_t e = 0; e + 1 < n; ++e) {
        Event &A = out.events[e];
        const Event &B = out.events[e + 1];
        if (!plain(A) || B.kind != EV_T_BFLY || (B.flags & (EVF_TRUN | EVF_BRUN | EVF_CLIFF | EVF_MAT | EVF_DEFER)))
            continue;
        if (B.noise_end != A.noise_end || B.k != A.k || A.k < 8u) continue;
        const uint32_t p1 = A.tstar;
        const uint32_t m2 = ((B.mu >> p1) & 1u) ? (B.mu ^ A.mu) : B.mu;
        if (m2 == 0u) continue;  // the same coordinate shift twice
        const uint32_t p2 = 31u - (uint32_t)__builtin_clz(m2);
        A.flags |= EVF_PAIR;
        A.pbit = std::min(p1, p2) | (std::max(p1, p2) << 8);
        ++e;  // B is taken
    }
}

static void work_sums(Program &out) {
    uint64_t t = 0, m = 0;
    uint32_t n = 0;
    for (Event &E : out.events) {
        E.cum_t = t;
        E.cum_m = m;
        E.cum_e = n;
        switch (E.kind) {
            case EV_T_PHASE: ++n; break;
            case EV_T_DOUBLE: t += 2ull << E.k; ++n; break;
            case EV_T_BFLY: t += 1ull << E.k; ++n; break;
            case EV_M_DET: ++n; break;
            case EV_M_CUT: case EV_M_SPLIT: case EV_M_MERGE: m += 1ull << E.k; ++n; break;
            case EV_DIAG: t += 1ull << E.bcnt; ++n; break;  // bcnt: span dimension after the gate
            default: break;
        }
    }
}

// Gap sampling tables (see NoiseLoc): acceptance per slot and the gap table
// floor(q^g 2^32), q^g formed by repeated multiplication.  Slots with thr = 0
// take no part (acc = 0) and do not set p_max.  Without live slots every
// acceptance is 0, and the table content does not matter.
static void gap_tables(Program &out) {
    const size_t n = out.noise.size();
    double pmax = 0.0;
    for (size_t s = 0; s < n; ++s)
        if (out.noise[s].thr) pmax = std::max(pmax, out.noise_p[s]);
    for (size_t s = 0; s < n; ++s)
        out.noise[s].acc = out.noise[s].thr ? (uint64_t)std::floor(out.noise_p[s] / pmax * 4294967296.0) : 0u;
    out.gap.assign(n, 0xFFFFFFFFu);
    out.gap_pmax = pmax;
    if (pmax > 0.0) {
        const double q = 1.0 - pmax;
        double t = 1.0;
        for (size_t g = 1; g <= n; ++g) {
            t *= q;
            out.gap[g - 1] = (uint32_t)std::floor(t * 4294967296.0);
        }
    }
}

void compile_circuit(const std::string &text, const NoiseModel &nm, Program &out, bool speculate) {
    out = Program();
    const double probs[6] = {nm.p1, nm.p2, nm.p_idle, nm.p_meas, nm.p_reset, nm.p_mpp};
    for (double p : probs)
        if (!(p >= 0.0 && p <= 1.0)) throw CompileError{0, "noise probability out of [0,1]"};

    Cursor cur{text};
    std::vector<std::string> tok;
    if (!next_line(cur, tok) || tok[0] != "QUBITS" || tok.size() != 2)
        throw CompileError{cur.line, "first line must be QUBITS n"};
    const int n = parse_uint(tok[1], cur.line);
    if (n < 1 || n > 64) throw CompileError{cur.line, "QUBITS must be in 1..64"};
    out.n = n;
    FrameCompiler fc(n, out, speculate);
    std::vector<char> busy(n, 0);
    uint32_t src = 0;

    while (next_line(cur, tok)) {
        const int ln = cur.line;
        const std::string &op = tok[0];
        auto qubit = [&](const std::string &s) {
            int q = parse_uint(s, ln);
            if (q >= n) throw CompileError{ln, "qubit out of range"};
            return q;
        };
        auto want = [&](size_t k) {
            if (tok.size() != k) throw CompileError{ln, op + ": wrong number of arguments"};
        };
        // A diagonal gate named by tok[at]: basis state x of its qubits (bit j
        // = j-th qubit) picks up e^{i phi_x}.  CCZ: phi = pi at x = 7 (CCX =
        // H_c CCZ H_c); CS / CSDG: +-pi/2 at x = 3; CPHASE t a b: t at x = 3;
        // RZ t q = exp(-i t Z / 2): (-t/2, t/2); DIAG k q.. phi_0..phi_{2^k-1}.
        // Under IF also S / SDG (+-pi/2 at x = 1), T / TDG (+-pi/4, T =
        // diag(1, e^{i pi/4})) and CZ (pi at x = 3).
        auto diag_spec = [&](size_t at, std::vector<int> &qs, std::vector<double> &phi) {
            const std::string &g = tok[at];
            size_t nq = 0, first = at + 1;
            if (g == "CCZ" || g == "CCX") nq = 3;
            else if (g == "CS" || g == "CSDG" || g == "CZ") nq = 2;
            else if (g == "S" || g == "SDG" || g == "T" || g == "TDG") nq = 1;
            else if (g == "CPHASE") { nq = 2; first = at + 2; }
            else if (g == "RZ") { nq = 1; first = at + 2; }
            else {
                if (tok.size() < at + 2) throw CompileError{ln, "DIAG takes k, k qubits and 2^k phases"};
                const int k = parse_uint(tok[at + 1], ln);
                if (k < 1 || k > 3) throw CompileError{ln, "DIAG takes 1 to 3 qubits"};
                nq = (size_t)k;
                first = at + 2;
            }
            const size_t need = g == "DIAG" ? first + nq + ((size_t)1 << nq) : first + nq;
            if (tok.size() != need) throw CompileError{ln, g + ": wrong number of arguments"};
            qs.clear();
            for (size_t i = 0; i < nq; ++i) qs.push_back(qubit(tok[first + i]));
            for (size_t i = 0; i < nq; ++i)
                for (size_t j = 0; j < i; ++j)
                    if (qs[i] == qs[j]) throw CompileError{ln, g + " on repeated qubits"};
            auto angle = [&](const std::string &t) {
                char *endp = nullptr;
                const double v = std::strtod(t.c_str(), &endp);
                if (endp == t.c_str() || *endp != '\0' || !std::isfinite(v)) throw CompileError{ln, "bad angle '" + t + "'"};
                return v;
            };
            phi.assign((size_t)1 << nq, 0.0);
            if (g == "CCZ" || g == "CCX") phi[7] = M_PI;
            else if (g == "CZ") phi[3] = M_PI;
            else if (g == "S") phi[1] = M_PI / 2;
            else if (g == "SDG") phi[1] = -M_PI / 2;
            else if (g == "T") phi[1] = M_PI / 4;
            else if (g == "TDG") phi[1] = -M_PI / 4;
            else if (g == "CS") phi[3] = M_PI / 2;
            else if (g == "CSDG") phi[3] = -M_PI / 2;
            else if (g == "CPHASE") phi[3] = angle(tok[at + 1]);
            else if (g == "RZ") { phi[0] = -angle(tok[at + 1]) / 2; phi[1] = angle(tok[at + 1]) / 2; }
            else
                for (size_t x = 0; x < phi.size(); ++x) phi[x] = angle(tok[first + nq + x]);
        };
        if (op == "H" || op == "S" || op == "SDG" || op == "X" || op == "Y" || op == "Z" || op == "T" ||
            op == "TDG" || op == "H_XY" || op == "H_NXY") {
            want(2);
            int q = qubit(tok[1]);
            busy[q] = 1;
            if (op == "H") fc.h(q);
            else if (op == "H_XY") fc.hxy(q);
            else if (op == "H_NXY") fc.hnxy(q);
            else if (op == "S") fc.s(q);
            else if (op == "SDG") fc.sdg(q);
            else if (op == "X") fc.px(q);
            else if (op == "Y") fc.py(q);
            else if (op == "Z") fc.pz(q);
            else fc.t_gate(q, op == "TDG", src);
            fc.noise(NZ_DEP1, nm.p1, q, -1, 0);
        } else if (op == "CX" || op == "CZ") {
            want(3);
            int a = qubit(tok[1]), b = qubit(tok[2]);
            if (a == b) throw CompileError{ln, "two-qubit gate on one qubit"};
            busy[a] = busy[b] = 1;
            if (op == "CX") fc.cnot(a, b);
            else fc.cz(a, b);
            fc.noise(NZ_DEP2, nm.p2, a, b, 0);
        } else if (op == "M" || op == "R") {
            want(2);
            int q = qubit(tok[1]);
            busy[q] = 1;
            PauliStr Z;
            Z.z = bitq(q);
            if (op == "M") {
                fc.noise(NZ_XERR, nm.p_meas, q, -1, 0);
                fc.measure(Z, out.n_meas++, (int)out.n_rec++, -1, src);
            } else {
                fc.measure(Z, out.n_meas++, -1, q, src);
                fc.noise(NZ_XERR, nm.p_reset, q, -1, 0);
            }
        } else if (op == "CCZ" || op == "CCX" || op == "CS" || op == "CSDG" || op == "CPHASE" || op == "RZ" ||
                   op == "DIAG") {
            std::vector<int> qs;
            std::vector<double> phi;
            diag_spec(0, qs, phi);
            for (int q : qs) busy[q] = 1;
            if (op == "CCX") fc.h(qs[2]);
            fc.diag(qs, phi, src);
            if (op == "CCX") fc.h(qs[2]);
            // model noise: DEP2(p2) after a two-qubit diagonal gate, DEP1(p1) on
            // each qubit after a one- or three-qubit one
            if (qs.size() == 2) fc.noise(NZ_DEP2, nm.p2, qs[0], qs[1], 0);
            else
                for (int q : qs) fc.noise(NZ_DEP1, nm.p1, q, -1, 0);
        } else if (op == "IF") {
            // Classically controlled gate (the corrections of gate
            // teleportation): IF r0,r1,.. GATE args applies GATE when the XOR of
            // the record bits is 1, IF r0&r1&.. GATE args when all of them are
            // 1.  GATE is a Pauli (X, Y, Z: sign flips) or a diagonal gate (S,
            // SDG, T, TDG, CZ and the diagonal gates above), which acts on the
            // coefficients by its Z-string expansion so that the x/z frame stays
            // the same in every shot.  No model noise.
            if (tok.size() < 3) throw CompileError{ln, "IF takes record bits and a gate"};
            const std::string &cs = tok[1];
            const bool has_and = cs.find('&') != std::string::npos, has_xor = cs.find(',') != std::string::npos;
            if (has_and && has_xor) throw CompileError{ln, "IF: use ',' (XOR) or '&' (AND), not both"};
            std::vector<int> cond;
            size_t pos = 0;
            while (true) {
                const size_t e = cs.find(has_and ? '&' : ',', pos);
                const int r = parse_uint(cs.substr(pos, e == std::string::npos ? std::string::npos : e - pos), ln);
                if ((uint32_t)r >= out.n_rec) throw CompileError{ln, "record index not yet measured"};
                cond.push_back(r);
                if (e == std::string::npos) break;
                pos = e + 1;
            }
            const std::string &g = tok[2];
            if (g == "X" || g == "Y" || g == "Z") {
                if (tok.size() != 4) throw CompileError{ln, "IF: " + g + " takes one qubit"};
                fc.feedback(g == "X" ? 1 : g == "Y" ? 2 : 3, qubit(tok[3]), cond, has_and, src);
            } else if (g == "S" || g == "SDG" || g == "T" || g == "TDG" || g == "CZ" || g == "CCZ" || g == "CCX" ||
                       g == "CS" || g == "CSDG" || g == "CPHASE" || g == "RZ" || g == "DIAG") {
                std::vector<int> qs;
                std::vector<double> phi;
                diag_spec(2, qs, phi);
                for (int q : qs) busy[q] = 1;
                if (g == "CCX") fc.h(qs[2]);  // the H pair is unconditional: H IF(CCZ) H
                fc.diag(qs, phi, src, cond, has_and);
                if (g == "CCX") fc.h(qs[2]);
            } else {
                throw CompileError{ln, "IF: '" + g + "' is neither a Pauli nor a diagonal gate"};
            }
        } else if (op == "MX" || op == "RX" || op == "MR" || op == "MRX") {
            // X-basis readout / reset to |+>, measure-then-reset; the error
            // flips anticommute with the measured Pauli (Z for the X basis)
            want(2);
            int q = qubit(tok[1]);
            busy[q] = 1;
            const bool xb = op != "MR", readout = op != "RX", reset = op != "MX";
            const uint32_t flip = xb ? NZ_ZERR : NZ_XERR;
            PauliStr P;
            if (xb) P.x = bitq(q);
            else P.z = bitq(q);
            if (readout) fc.noise(flip, nm.p_meas, q, -1, 0);
            const int rec = readout ? (int)out.n_rec++ : -1;
            fc.measure(P, out.n_meas++, rec, reset ? q : -1, src, xb);
            if (reset) fc.noise(flip, nm.p_reset, q, -1, 0);
        } else if (op == "XIF" || op == "YIF" || op == "ZIF") {
            want(3);
            int r = parse_uint(tok[1], ln);
            if ((uint32_t)r >= out.n_rec) throw CompileError{ln, "record index not yet measured"};
            int q = qubit(tok[2]);
            fc.feedback(op == "XIF" ? 1 : op == "YIF" ? 2 : 3, q, std::vector<int>(1, r), false, src);
        } else if (op == "MPP") {
            want(2);
            PauliStr P;
            const std::string &spec = tok[1];
            size_t i = 0;
            while (true) {
                size_t j = spec.find('*', i);
                std::string f = spec.substr(i, j == std::string::npos ? std::string::npos : j - i);
                if (f.size() < 2) throw CompileError{ln, "bad Pauli factor '" + f + "'"};
                int q = qubit(f.substr(1));
                if (((P.x | P.z) >> q) & 1) throw CompileError{ln, "repeated qubit in MPP"};
                switch (f[0]) {
                    case 'X': P.x |= bitq(q); break;
                    case 'Z': P.z |= bitq(q); break;
                    case 'Y': P.x |= bitq(q); P.z |= bitq(q); break;
                    default: throw CompileError{ln, "bad Pauli letter"};
                }
                busy[q] = 1;
                if (j == std::string::npos) break;
                i = j + 1;
            }
            uint32_t rec = out.n_rec++;
            fc.measure(P, out.n_meas++, (int)rec, -1, src);
            fc.noise(NZ_FLIP, nm.p_mpp, -1, -1, rec);
        } else if (op == "DEP1" || op == "XERR" || op == "ZERR") {
            if (tok.size() < 3) throw CompileError{ln, op + ": wrong number of arguments"};
            double p = parse_prob(tok[1], ln);
            const uint32_t k = op == "DEP1" ? NZ_DEP1 : op == "XERR" ? NZ_XERR : NZ_ZERR;
            for (size_t i = 2; i < tok.size(); ++i) fc.noise(k, p, qubit(tok[i]), -1, 0);
        } else if (op == "DEP2") {
            if (tok.size() < 4 || tok.size() % 2 != 0) throw CompileError{ln, "DEP2: wrong number of arguments"};
            double p = parse_prob(tok[1], ln);
            for (size_t i = 2; i < tok.size(); i += 2) {
                int a = qubit(tok[i]), b = qubit(tok[i + 1]);
                if (a == b) throw CompileError{ln, "DEP2 on one qubit"};
                fc.noise(NZ_DEP2, p, a, b, 0);
            }
        } else if (op == "TICK") {
            want(1);
            for (int q = 0; q < n; ++q)
                if (!busy[q]) fc.noise(NZ_DEP1, nm.p_idle, q, -1, 0);
            std::fill(busy.begin(), busy.end(), 0);
        } else if (op == "DETECTOR" || op == "OBSERVABLE") {
            if (tok.size() < 2) throw CompileError{ln, op + ": wrong number of arguments"};
            int e = parse_uint(tok[1], ln);
            if (e > 1) throw CompileError{ln, "expected bit must be 0 or 1"};
            std::vector<int> recs;
            for (size_t i = 2; i < tok.size(); ++i) {
                int r = parse_uint(tok[i], ln);
                if ((uint32_t)r >= out.n_rec) throw CompileError{ln, "record index not yet measured"};
                recs.push_back(r);
            }
            uint32_t obs = 0;
            if (op == "OBSERVABLE") {
                if (out.n_obs >= 32) throw CompileError{ln, "at most 32 observables"};
                obs = out.n_obs++;
            }
            fc.parity_check(op == "DETECTOR", e, recs, obs, src);
        } else {
            throw CompileError{ln, "unknown op '" + op + "'"};
        }
        ++src;
    }
    fc.end(src);
    form_batches(out);
    if (speculate) {
        fuse_doublings(out);
        fuse_drop_runs(out);
    }
    out.n_src = src;
    out.n_noise = (uint32_t)out.noise.size();
    checkpoints(out);
    deferrable_runs(out);
    butterfly_pairs(out);
    work_sums(out);
    gap_tables(out);
    // pad the threshold table to whole 256-slot chunks
    while (out.noise_tm1.size() % 256) out.noise_tm1.push_back(0);
    if (out.noise_tm1.empty()) out.noise_tm1.assign(256, 0);
    uint64_t h = fnv1a(text.data(), text.size(), 1469598103934665603ULL);
    out.hash = fnv1a(probs, sizeof(probs), h);
}

}  // namespace soft
