// sampler.hip -- persistent, work-stealing shot sampler for gfx950 (CDNA4).
//
// One wavefront (64 lanes) runs one shot at a time and then steals the next
// shot index from a global counter, so early postselection aborts and uneven
// coefficient supports balance themselves.  Per shot a wave holds:
//   * the 2n tableau signs as two 64-bit words (rD, rS) and the offset a of
//     the coefficient support -- wave-uniform scalars;
//   * the coefficients as a dense LDS tile of 2^k complex numbers (k = span
//     dimension, the same for every shot at a given event), FP32 or FP64;
//   * the measurement record in LDS.
// The circuit is the event list built by compile.cpp; each event is read with
// uniform loads.  Every pass over the tile puts consecutive coordinates on
// consecutive lanes, so LDS accesses are contiguous and conflict-free.
//
// The arithmetic per event follows arXiv 2512.23037: T/T-dagger by Eqs. 1-2
// with the index shift of Eq. 4 (Theorem 1 part 3); measurements with the
// projectors (I +- P)/2 (Theorem 1 part 2), outcome probabilities and
// renormalisation accumulated in FP64; Pauli noise per shot as sign flips.
#include <hip/hip_runtime.h>

#include <mutex>
#include <type_traits>

#include "program.h"
#include "sampler.h"

namespace soft {

// Scratch of the allocation-free run (see scratch_address below).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

template <typename R> struct Cx;
template <> struct Cx<float> { typedef float2 T; };
template <> struct Cx<double> { typedef double2 T; };

__device__ __forceinline__ uint32_t par64(uint64_t w) { return (uint32_t)__popcll(w) & 1u; }
__device__ __forceinline__ uint32_t par32(uint32_t w) { return (uint32_t)__popc(w) & 1u; }

// insert a zero bit at position h of p
__device__ __forceinline__ uint32_t ins0(uint32_t p, uint32_t h) {
    const uint32_t lo = p & ((1u << h) - 1u);
    return ((p ^ lo) << 1) | lo;
}

// A lane-parallel pass over indices [0, cnt) with cnt a power of two: a
// uniform trip count, and when cnt < 64 the lanes past the end sit out.
template <typename F> __device__ __forceinline__ void lane_pass(uint32_t cnt, uint32_t lane, F &&f) {
    const uint32_t iters = (cnt + 63u) >> 6;
#pragma unroll 1
    for (uint32_t it = 0; it < iters; ++it)
        if (cnt >= 64u || lane < cnt) f((it << 6) | lane);
}

// readfirstlane yields a signed int: widen through uint32_t, never directly.
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ uint64_t uni64(uint64_t x) {
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}
// The 64-bit value held by lane l (l wave-uniform).
__device__ __forceinline__ uint64_t lane64(uint64_t x, uint32_t l) {
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x >> 32), (int)l);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, (int)l);
    return ((uint64_t)hi << 32) | (uint64_t)lo;
}
__device__ __forceinline__ double unid(double x) { return __longlong_as_double((long long)uni64((uint64_t)__double_as_longlong(x))); }

// Butterfly sum over the 64 lanes; every lane ends with the same bits because
// each step adds the same two partial sums in either order.
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
    return unid(x);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                         uint32_t k1, uint32_t &o0, uint32_t &o1, uint32_t &o2, uint32_t &o3) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
        const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
        c0 = hi1 ^ c1 ^ k0;
        c1 = lo1;
        c2 = hi0 ^ c3 ^ k1;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    o0 = c0; o1 = c1; o2 = c2; o3 = c3;
}

template <typename C> __device__ __forceinline__ C mk(double re, double im) {
    C c;
    c.x = re;
    c.y = im;
    return c;
}

template <typename R> __device__ __forceinline__ double nrm(typename Cx<R>::T a) {
    return (double)a.x * (double)a.x + (double)a.y * (double)a.y;
}

// i^q * a for q mod 4, without branches: odd q swaps the parts, then the
// real part flips sign for q = 1, 2 and the imaginary part for q = 2, 3.
template <typename C> __device__ __forceinline__ C rot(C a, uint32_t q) {
    q &= 3u;
    const bool sw = (q & 1u) != 0u;
    C r;
    r.x = sw ? a.y : a.x;
    r.y = sw ? a.x : a.y;
    if (((q + 1u) & 2u) != 0u) r.x = -r.x;
    if ((q & 2u) != 0u) r.y = -r.y;
    return r;
}

// a * b + (s ? -1 : 1) * c * d, complex
template <typename R, typename C>
__device__ __forceinline__ C cmad2(C a, R br, R bi, C c, R dr, R di, bool neg) {
    R tr = c.x * dr - c.y * di;
    R ti = c.x * di + c.y * dr;
    if (neg) { tr = -tr; ti = -ti; }
    C o;
    o.x = fma(a.x, br, fma(-a.y, bi, tr));
    o.y = fma(a.x, bi, fma(a.y, br, ti));
    return o;
}

template <typename C, typename R> __device__ __forceinline__ C scale(C a, R s) {
    a.x *= s;
    a.y *= s;
    return a;
}

// The coefficient tile of one wave.  TM = TM_LDS: in LDS; TM_MEM: in a slab
// of device memory; TM_SPLIT: entries below `lim` in LDS, the others in a
// slab of device memory (`hi` is that slab's address minus lim entries, so
// hi + j addresses entry j >= lim).  The split form is read and written
// through flat addresses, which reach LDS or device memory by the address.
template <typename C, uint32_t TM> struct Tile {
    C *lo;
    C *hi;
    uint32_t lim;
    __device__ __forceinline__ C *at(uint32_t j) const { return (TM == TM_SPLIT && j >= lim) ? hi + j : lo + j; }
    // entry u + l with u wave-uniform and l < 128 <= lim (a power of two):
    // the place is the same for the whole wave
    __device__ __forceinline__ C *at_u(uint32_t u, uint32_t l) const {
        return ((TM == TM_SPLIT && u >= lim) ? hi : lo) + (u + l);
    }
    __device__ __forceinline__ C &operator[](uint32_t j) const { return *at(j); }
};

// Sum of |v_j|^2 in FP64 over a tile of 2^k entries: the end-of-shot norm
// check, and the same sum stored with a checkpoint's tile.
template <typename C, uint32_t TM>
__device__ __forceinline__ double tile_norm(const Tile<C, TM> &v, uint32_t k, uint32_t lane) {
    double nn = 0.0;
    lane_pass(1u << k, lane, [&](uint32_t j) {
        const C x = v[j];
        nn += (double)x.x * (double)x.x + (double)x.y * (double)x.y;
    });
    return wave_sum(nn);
}

// Write one shot's state for the readout calls: status, signs, offset, span
// dimension, carried norm, and the coefficient tile widened to double with the
// counted global phase e^{i pi phase8 / 8} and the tile's real factor
// sqrt(tscale2) applied.
template <typename C, uint32_t TM>
__device__ __forceinline__ void dump_state(unsigned long long *m, double *dst, const Tile<C, TM> &v, uint32_t lane,
                                           uint32_t tile_entries, uint32_t status, uint32_t abort_src, uint32_t term,
                                           uint32_t after, uint64_t rD, uint64_t rS, uint64_t a, uint32_t k,
                                           double nrm2, const double *phase_tab, uint32_t phase8, uint32_t var,
                                           uint32_t full, double tscale2) {
    if (lane == 0) {
        m[KM_STATUS] = status;
        m[KM_ABORT] = abort_src;
        m[KM_TERM_EV] = term;
        m[KM_AFTER] = after;
        m[KM_RD] = rD;
        m[KM_RS] = rS;
        m[KM_A] = a;
        m[KM_K] = k;
        m[KM_NRM2] = (unsigned long long)__double_as_longlong(nrm2);
        m[KM_VALID] = kStateValid;
        m[KM_VAR] = var;
        m[KM_PROG] = full;
    }
    const double f = sqrt(tscale2);
    const double pc = f * phase_tab[phase8], ps = f * phase_tab[16u + phase8];
    const uint32_t cnt = 1u << k;
    lane_pass(tile_entries, lane, [&](uint32_t j) {
        double x = 0.0, y = 0.0;
        if (j < cnt) {
            const C e = v[j];
            x = (double)e.x;
            y = (double)e.y;
        }
        dst[2u * j] = x * pc - y * ps;
        dst[2u * j + 1u] = x * ps + y * pc;
    });
}

// Nonzero iff the complex value is not +-0 (sign bits shifted out).
__device__ __forceinline__ uint32_t nonzero_bits(float2 x) {
    return (__float_as_uint(x.x) | __float_as_uint(x.y)) << 1;
}
__device__ __forceinline__ uint32_t nonzero_bits(double2 x) {
    const uint64_t b = ((uint64_t)__double_as_longlong(x.x) | (uint64_t)__double_as_longlong(x.y)) << 1;
    return (uint32_t)(b >> 32) | (uint32_t)b;
}

constexpr uint32_t kNoHit = 0xFFFFFFFFu;

// Lowest slot with a pending noise hit in the chunk based at cb (lane l holds
// slots cb + 4l .. cb + 4l + 3 as bits of `hits`), or kNoHit.
__device__ __forceinline__ uint32_t first_hit(uint32_t hits, uint32_t cb) {
    const uint64_t lanes = __ballot(hits != 0u);
    if (lanes == 0ull) return kNoHit;
    const uint32_t L = (uint32_t)__builtin_ctzll(lanes);
    const uint32_t m = (uint32_t)__builtin_amdgcn_readlane((int)hits, (int)L);
    return cb + 4u * L + (uint32_t)__builtin_ctz(m);
}

// The record words 0..kRecSgpr-1 of a shot live in one vector register, word
// w in lane w (kRecSgpr <= 64); the rest in LDS.

// i^Q * a for a compile-time Q: only register moves and sign modifiers.
template <uint32_t Q, typename C> __device__ __forceinline__ C rotc(C a) {
    C r;
    if (Q == 0) { r = a; }
    else if (Q == 1) { r.x = -a.y; r.y = a.x; }
    else if (Q == 2) { r.x = -a.x; r.y = -a.y; }
    else { r.x = a.y; r.y = -a.x; }
    return r;
}

// out = a + c * i^Q b, then drop it below the pruning level.
template <uint32_t Q, typename R, typename C>
__device__ __forceinline__ C t_out(C a, C b, R c, R thr, bool &keep) {
    const C w = rotc<Q>(b);
    C o;
    o.x = fma(c, w.x, a.x);
    o.y = fma(c, w.y, a.y);
    keep = fma(o.x, o.x, o.y * o.y) >= thr;
    if (!keep) { o.x = 0; o.y = 0; }
    return o;
}

// a, dropped below the pruning level.
template <typename R, typename C> __device__ __forceinline__ C t_keep(C a, R thr, bool &keep) {
    keep = fma(a.x, a.x, a.y * a.y) >= thr;
    if (!keep) { a.x = 0; a.y = 0; }
    return a;
}

// c * i^Q b, dropped below the pruning level.
template <uint32_t Q, typename R, typename C> __device__ __forceinline__ C t_new(C b, R c, R thr, bool &keep) {
    const C w = rotc<Q>(b);
    C o;
    o.x = c * w.x;
    o.y = c * w.y;
    return t_keep<R, C>(o, thr, keep);
}

// The tile holds the state up to a real per-shot factor, so a branching T
// is v' = v + tn i^Q (+-1) v_partner with tn = tan(pi/8) (its cos(pi/8) goes
// into the factor).
//
// The iterations of a pass cover 64 lanes each; iteration `it` adds the
// uniform coordinate bits J(it), and the sign (-1)^(g.J(it)) is the same for
// the whole wave.  A sign -1 is i^2, i.e. the Q + 2 form of the update.  If
// no iteration bit of J meets g, every iteration takes the Q form.
// Otherwise, with t the lowest iteration bit whose coordinate bit is in g,
// iterations it and it ^ 2^t have opposite signs: each such pair runs one Q
// and one Q + 2 update, and which is which is a scalar choice.
// The coordinate bit that pairs the iterations (`pb`: the lowest coordinate
// bit in g that some iteration sets, or 0 when every iteration has sign +1)
// depends only on the event and k, and comes with the event.

// The iterations' coordinate bits J run over the values with the bits of M
// clear (M holds the lane bits and any skipped bit): J -> ((J | M) + 1) & ~M
// steps to the next one in increasing order.
__device__ __forceinline__ uint32_t next_j(uint32_t J, uint32_t M) { return ((J | M) + 1u) & ~M; }

// Branching T on an existing coordinate: pairs (j0, j1 = j0 ^ mu), j0 with
// bit h clear.  v'_j0 = v_j0 + tn i^Q (-1)^(sig ^ g.j1) v_j1 and the same
// with j0, j1 exchanged.  j0 = ins0(lane, h) | ins0(64 it, h): the lane bits and
// the iteration bits of a coordinate are disjoint, so each lane keeps two base
// pointers for the event (j0's and j1's lane parts, h set in j1's) and an
// iteration adds one uniform byte offset to each.
// Returns the kept outputs; `cnt1` receives those at the partner coordinates
// j0 ^ mu (bit h set).
template <uint32_t Q, typename R, typename C, uint32_t TM>
__device__ __forceinline__ uint32_t t_bfly(const Tile<C, TM> &v, uint32_t lane, uint32_t k, uint32_t mu, uint32_t h, uint32_t g,
                                           uint32_t sig, R tn, R thr, uint32_t pb, uint32_t lmask,
                                           uint32_t &cnt1) {
    const uint32_t npairs = 1u << (k - 1u);
    // With fewer than 64 pairs the spare lanes repeat a live lane's pair (same
    // values to the same addresses) and are left out of the counts, so the
    // loop body needs no divergent branch.
    const uint32_t lp = npairs >= 64u ? lane : (lane & (npairs - 1u));
    const uint64_t live = npairs >= 64u ? ~0ull : ((1ull << npairs) - 1ull);
    const uint32_t lc = ins0(lp, h);
    const uint32_t hb = 1u << h;  // mu's top bit is h; lmask = ins0(63, h)
    const uint32_t mu_l = mu & lmask, mu_i = mu & ~(lmask | hb);
    char *const p0 = reinterpret_cast<char *>(v.lo + lc);
    char *const p1 = reinterpret_cast<char *>(v.lo + ((lc ^ mu_l) | hb));
    const R c1 = ((sig ^ par32(g & lc)) != 0u) ? -tn : tn;   // weight of v_j0 in v'_j1
    const R c0 = par32(g & mu) ? -c1 : c1;                   // weight of v_j1 in v'_j0
    uint32_t cnt = 0;
    cnt1 = 0;
    const uint32_t iters = (npairs + 63u) >> 6;
    // one iteration with the Q or (S = 2) the Q + 2 form, in two halves so
    // that a pair of iterations issues all its LDS reads before any write
    // (the iterations of a pass touch disjoint entries)
    // (split tile: the lane part is below 128 <= lim, so the uniform part
    // decides the place of an iteration's entries)
    auto addr0 = [&](uint32_t J) {
        if (TM == TM_SPLIT) return v.at_u(J, lc);
        return reinterpret_cast<C *>(p0 + J * (uint32_t)sizeof(C));
    };
    auto addr1 = [&](uint32_t J) {
        if (TM == TM_SPLIT) return v.at_u((J ^ mu_i) | hb, lc ^ mu_l);
        return reinterpret_cast<C *>(p1 + (J ^ mu_i) * (uint32_t)sizeof(C));
    };
    auto finish = [&](uint32_t J, C v0, C v1, auto S) {
        constexpr uint32_t QS = (Q + decltype(S)::value) & 3u;
        bool k0, k1;
        const C o0 = t_out<QS, R, C>(v0, v1, c0, thr, k0);
        const C o1 = t_out<QS, R, C>(v1, v0, c1, thr, k1);
        const uint32_t n1 = (uint32_t)__popcll(__ballot(k1) & live);
        cnt += (uint32_t)__popcll(__ballot(k0) & live) + n1;
        cnt1 += n1;
        *addr0(J) = o0;
        *addr1(J) = o1;
    };
    auto step = [&](uint32_t J, auto S) { finish(J, *addr0(J), *addr1(J), S); };
    // the iterations' coordinate bits J = ins0(64 it, h): everything outside
    // the lane bits and bit h
    uint32_t J = 0;
    if (pb == 0u) {
        if (iters == 1u) {
            step(J, std::integral_constant<uint32_t, 0>());
        } else {
            for (uint32_t it = 0; it < iters; it += 2u) {  // iters is a power of two
                const uint32_t JB = next_j(J, lmask | hb);
                const C a0 = *addr0(J), a1 = *addr1(J), b0 = *addr0(JB), b1 = *addr1(JB);
                finish(J, a0, a1, std::integral_constant<uint32_t, 0>());
                finish(JB, b0, b1, std::integral_constant<uint32_t, 0>());
                J = next_j(JB, lmask | hb);
            }
        }
    } else {
        // two pairs per trip: eight reads in flight before the writes
        const uint32_t M = lmask | hb | pb, npair = iters >> 1;
        uint32_t i2 = 0;
        for (; i2 + 2u <= npair; i2 += 2u) {
            const uint32_t J2 = next_j(J, M);
            const bool fa = par32(g & J) != 0u, fb = par32(g & J2) != 0u;
            const uint32_t Jp = fa ? (J | pb) : J, Jm = fa ? J : (J | pb);
            const uint32_t Kp = fb ? (J2 | pb) : J2, Km = fb ? J2 : (J2 | pb);
            const C a0 = *addr0(Jp), a1 = *addr1(Jp), b0 = *addr0(Jm), b1 = *addr1(Jm);
            const C e0 = *addr0(Kp), e1 = *addr1(Kp), d0 = *addr0(Km), d1 = *addr1(Km);
            finish(Jp, a0, a1, std::integral_constant<uint32_t, 0>());
            finish(Jm, b0, b1, std::integral_constant<uint32_t, 2>());
            finish(Kp, e0, e1, std::integral_constant<uint32_t, 0>());
            finish(Km, d0, d1, std::integral_constant<uint32_t, 2>());
            J = next_j(J2, M);
        }
        if (i2 < npair) {
            const uint32_t JB = J | pb;
            const bool fa = par32(g & J) != 0u;
            const uint32_t Jp = fa ? JB : J, Jm = fa ? J : JB;
            const C a0 = *addr0(Jp), a1 = *addr1(Jp), b0 = *addr0(Jm), b1 = *addr1(Jm);
            finish(Jp, a0, a1, std::integral_constant<uint32_t, 0>());
            finish(Jm, b0, b1, std::integral_constant<uint32_t, 2>());
        }
    }
    return cnt;
}

// a + c i^q b for a wave-uniform q (the swap and signs of rotc chosen at run
// time; c (+-1) w = (+-c) w exactly, so this equals t_out<q>), then dropped
// below the pruning level.
template <typename R, typename C>
__device__ __forceinline__ C t_out_q(C a, C b, R c, uint32_t q, R thr, bool &keep) {
    const R wx = (q & 1u) ? b.y : b.x, wy = (q & 1u) ? b.x : b.y;
    const R cx = (q == 1u || q == 2u) ? -c : c, cy = (q >= 2u) ? -c : c;
    C o;
    o.x = fma(cx, wx, a.x);
    o.y = fma(cy, wy, a.y);
    keep = fma(o.x, o.x, o.y * o.y) >= thr;
    if (!keep) { o.x = 0; o.y = 0; }
    return o;
}

// Two branching T on existing coordinates, mu1 then mu2, in one pass (the
// pair of an EVF_PAIR event and the next): each lane takes the quad
// {j, j ^ mu1, j ^ mu2, j ^ mu1 ^ mu2} with j's bits plo and phi clear (the
// quads tile the span), applies the first butterfly to its two mu1-pairs and
// the second to its two mu2-pairs, pruning after each at its own level: the
// separate passes' arithmetic on every entry.  Butterfly t updates
// v'_x = v_x + tn_t i^q_t (-1)^(s_t ^ g_t.(x ^ mu_t)) v_(x ^ mu_t); the parity
// of g_t over a quad's four members is that over j plus a uniform constant.
// k >= 8: 2^(k-2) quads, a multiple of 64.  cnt1, cnt2: outputs kept by each;
// upper: nonzero when the second keeps an output with coordinate bit k - 1
// set (its drop check).  The inputs come from `src`: the tile itself, or the
// tile of the checkpoint a shot started from, not yet loaded (every entry is
// written, so the pass also loads it).  With drop2 (the second drops
// coordinate k - 1) the outputs at coordinates with that bit set are not
// stored: the span leaves them when the check passes, and nothing reads the
// tile past 2^k; when it fails the shot restarts.
template <typename R, typename C, uint32_t TM, uint32_t TMS>
__device__ __forceinline__ void t_bfly_pair(const Tile<C, TM> &v, const Tile<C, TMS> &src, uint32_t lane, uint32_t k,
                                            uint32_t plo, uint32_t phi,
                                            uint32_t mu1, uint32_t g1, uint32_t s1, uint32_t q1, R tn1, R thr1,
                                            uint32_t mu2, uint32_t g2, uint32_t s2, uint32_t q2, R tn2, R thr2,
                                            bool drop2, uint32_t &cnt1, uint32_t &cnt2, uint64_t &upper) {
    const uint32_t a1 = par32(g1 & mu1), b1 = par32(g1 & mu2);  // parity of g1 over mu1, mu2
    const uint32_t a2 = par32(g2 & mu1), b2 = par32(g2 & mu2);
    const uint32_t top = 1u << (k - 1u);
    const uint32_t iters = 1u << (k - 8u);
    cnt1 = 0;
    cnt2 = 0;
    upper = 0;
    auto sgn = [](uint32_t s, R t) { return s ? -t : t; };
    for (uint32_t it = 0; it < iters; ++it) {
        const uint32_t j = ins0(ins0(lane + 64u * it, plo), phi);
        const uint32_t jb = j ^ mu1, jc = j ^ mu2, jd = jb ^ mu2;
        C *pa = v.at(j), *pb = v.at(jb), *pc = v.at(jc), *pd = v.at(jd);
        const C A = *src.at(j), B = *src.at(jb), Cc = *src.at(jc), D = *src.at(jd);
        // first butterfly: (j, jb) and (jc, jd); the weight of v_y in v'_x
        // has the parity of g1 over y
        const uint32_t t1 = s1 ^ par32(g1 & j);
        bool kA, kB, kC, kD;
        const C A1 = t_out_q<R, C>(A, B, sgn(t1 ^ a1, tn1), q1, thr1, kA);
        const C B1 = t_out_q<R, C>(B, A, sgn(t1, tn1), q1, thr1, kB);
        const C C1 = t_out_q<R, C>(Cc, D, sgn(t1 ^ a1 ^ b1, tn1), q1, thr1, kC);
        const C D1 = t_out_q<R, C>(D, Cc, sgn(t1 ^ b1, tn1), q1, thr1, kD);
        cnt1 += (uint32_t)(__popcll(__ballot(kA)) + __popcll(__ballot(kB)) + __popcll(__ballot(kC)) +
                           __popcll(__ballot(kD)));
        // second butterfly: (j, jc) and (jb, jd)
        const uint32_t t2 = s2 ^ par32(g2 & j);
        const C A2 = t_out_q<R, C>(A1, C1, sgn(t2 ^ b2, tn2), q2, thr2, kA);
        const C C2 = t_out_q<R, C>(C1, A1, sgn(t2, tn2), q2, thr2, kC);
        const C B2 = t_out_q<R, C>(B1, D1, sgn(t2 ^ a2 ^ b2, tn2), q2, thr2, kB);
        const C D2 = t_out_q<R, C>(D1, B1, sgn(t2 ^ a2, tn2), q2, thr2, kD);
        cnt2 += (uint32_t)(__popcll(__ballot(kA)) + __popcll(__ballot(kB)) + __popcll(__ballot(kC)) +
                           __popcll(__ballot(kD)));
        upper |= __ballot((kA && (j & top)) || (kB && (jb & top)) || (kC && (jc & top)) || (kD && (jd & top)));
        if (!drop2 || !(j & top)) *pa = A2;
        if (!drop2 || !(jb & top)) *pb = B2;
        if (!drop2 || !(jc & top)) *pc = C2;
        if (!drop2 || !(jd & top)) *pd = D2;
    }
}

// Branching T on a new coordinate (k -> k+1): v'_j = v_j and
// v'_{j+2^k} = tn i^Q (-1)^(sig ^ g.j) v_j.
template <uint32_t Q, typename R, typename C, uint32_t TM>
__device__ __forceinline__ uint32_t t_double(const Tile<C, TM> &v, uint32_t lane, uint32_t k, uint32_t g, uint32_t sig, R tn,
                                             R thr, uint32_t pb) {
    const uint32_t half = 1u << k;
    // spare lanes repeat a live lane (see t_bfly)
    const uint32_t lp = half >= 64u ? lane : (lane & (half - 1u));
    const uint64_t live = half >= 64u ? ~0ull : ((1ull << half) - 1ull);
    const R c1 = ((sig ^ par32(g & lp)) != 0u) ? -tn : tn;
    char *const p0 = reinterpret_cast<char *>(v.lo + lp);
    char *const p1 = reinterpret_cast<char *>(v.lo + half + lp);
    uint32_t cnt = 0;
    const uint32_t iters = (half + 63u) >> 6;
    // as in t_bfly: a pair of iterations reads before it writes
    auto addr0 = [&](uint32_t J) {
        if (TM == TM_SPLIT) return v.at_u(J, lp);
        return reinterpret_cast<C *>(p0 + J * (uint32_t)sizeof(C));
    };
    auto addr1 = [&](uint32_t J) {
        if (TM == TM_SPLIT) return v.at_u(J + half, lp);
        return reinterpret_cast<C *>(p1 + J * (uint32_t)sizeof(C));
    };
    auto finish = [&](uint32_t J, C v0, auto S) {
        constexpr uint32_t QS = (Q + decltype(S)::value) & 3u;
        bool k0, k1;
        const C o0 = t_keep<R, C>(v0, thr, k0);
        const C o1 = t_new<QS, R, C>(v0, c1, thr, k1);
        cnt += (uint32_t)__popcll(__ballot(k0) & live) + (uint32_t)__popcll(__ballot(k1) & live);
        *addr0(J) = o0;
        *addr1(J) = o1;
    };
    if (iters == 1u) {
        finish(0u, *addr0(0u), std::integral_constant<uint32_t, 0>());
    } else if (pb == 0u) {
        for (uint32_t J = 0; J < (iters << 6); J += 128u) {
            const C a = *addr0(J), b = *addr0(J + 64u);
            finish(J, a, std::integral_constant<uint32_t, 0>());
            finish(J + 64u, b, std::integral_constant<uint32_t, 0>());
        }
    } else {
        uint32_t J = 0;
        for (uint32_t i2 = 0; i2 < (iters >> 1); ++i2) {
            const uint32_t JB = J | pb;
            const bool fa = par32(g & J) != 0u;
            const uint32_t Jp = fa ? JB : J, Jm = fa ? J : JB;
            const C a = *addr0(Jp), b = *addr0(Jm);
            finish(Jp, a, std::integral_constant<uint32_t, 0>());
            finish(Jm, b, std::integral_constant<uint32_t, 2>());
            J = next_j(J, 63u | pb);
        }
    }
    return cnt;
}


__device__ __forceinline__ float unif(float x) { return __uint_as_float(uni(__float_as_uint(x))); }

// floor(x / d) for x < 16 d (a noise hit's Pauli code from its word): a
// binary search on exact integer compares instead of a 64-bit division.
__device__ __forceinline__ uint32_t quot16(uint64_t x, uint64_t d) {
    uint32_t m = 0;
#pragma unroll
    for (uint32_t b = 8; b != 0u; b >>= 1)
        if (x >= (uint64_t)(m + b) * d) m += b;
    return m;
}

// Fields of the current event (held one dword per lane in `evc`).
#define EV32(f) ((uint32_t)__builtin_amdgcn_readlane((int)evc, (int)(offsetof(Event, f) / 4u)))
#define EV64(f)                                                                                  \
    (((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)evc, (int)(offsetof(Event, f) / 4u + 1u)) << 32) | \
     (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)evc, (int)(offsetof(Event, f) / 4u)))
#define EVF(f) __uint_as_float(EV32(f))
#define EVD(f) __longlong_as_double((long long)EV64(f))
// Fields of the next event (prefetched in `evx`).
#define EVX32(f) ((uint32_t)__builtin_amdgcn_readlane((int)evx, (int)(offsetof(Event, f) / 4u)))
#define EVX64(f)                                                                                 \
    (((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)evx, (int)(offsetof(Event, f) / 4u + 1u)) << 32) | \
     (uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)evx, (int)(offsetof(Event, f) / 4u)))

// LEAN: a launch with no kept states, no trace, no support cap and no shot
// list (and never the prefix build); those paths compile out, which frees
// scalar registers in the event loop.
template <typename R, uint32_t NS, uint32_t TM, bool LEAN = false>
__device__ __forceinline__ void sample_shots(const Event *__restrict__ ev, const NoiseLoc *__restrict__ nz,
                                             const uint32_t *__restrict__ tm1, const uint32_t *__restrict__ det,
                                             const uint32_t *__restrict__ words, const BatchMember *__restrict__ bm,
                                             const RunParams &P) {
    typedef typename Cx<R>::T C;
    constexpr bool EXPL = NS == NS_EXPLICIT, GAPS = NS == NS_GAPS;
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t wave = threadIdx.x >> 6;
    // The coefficient tile lives in LDS; or (TM_MEM) in a per-wave slab of
    // device memory for spans whose tile does not fit in LDS; or (TM_SPLIT)
    // its low P.lds_entries entries in LDS and the rest in a per-wave slab.
    // The record words past kRecSgpr are always in LDS.
    Tile<C, TM> v;
    v.hi = nullptr;
    v.lim = 0;
    uint32_t *rec;
    const size_t gwave = (size_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (TM == TM_MEM) {
        v.lo = reinterpret_cast<C *>(P.gtile) + gwave * P.tile_entries;
        rec = reinterpret_cast<uint32_t *>(smem + (size_t)wave * P.wave_bytes);
    } else {
        v.lo = reinterpret_cast<C *>(smem + (size_t)wave * P.wave_bytes);
        rec = reinterpret_cast<uint32_t *>(smem + (size_t)wave * P.wave_bytes + P.rec_off);
        if (TM == TM_SPLIT) {
            v.lim = P.lds_entries;
            // hi + j (j >= lim) is entry j's place in the slab: the slab's
            // address less lim entries, formed as an integer
            const uintptr_t slab = reinterpret_cast<uintptr_t>(P.gtile) +
                                   gwave * (size_t)(P.tile_entries - P.lds_entries) * sizeof(C);
            v.hi = reinterpret_cast<C *>(slab - (uintptr_t)P.lds_entries * sizeof(C));
        }
    }
    // Lanes read entries that other lanes wrote in the previous pass: with a
    // tile (or its upper part) in device memory, each pass ends with a fence
    // (LDS keeps a wave's accesses in order by itself).
    auto tile_sync = [&]() {
        if (TM != TM_LDS) __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    };
    const uint32_t key0 = (uint32_t)P.seed, key1 = (uint32_t)(P.seed >> 32);
    const double tau2 = P.tau2;

    double maxdev = 0.0;  // largest norm deviation of this wave's shots
    uint64_t myc = 0;  // counter number `lane` of this wave, for variant `var`

    // Circuit of the current shot: variant `var` owns shots [var_lo, var_end).
    // A wave's shots usually come in increasing order, so the range is looked
    // up again only when a shot leaves it.
    uint32_t var = 0;
    bool var_ok = false;
    uint64_t var_lo = 0, var_end = 0;
    auto flush_counters = [&]() {
        if ((!LEAN && P.prefix_build)) {  // the build samples no shots
            myc = 0;
            maxdev = 0.0;
            return;
        }
        unsigned long long *row = P.counters + (size_t)var * C_COUNT;
        if (lane < (uint32_t)C_COUNT && lane != (uint32_t)C_NORMDEV_BITS && myc) atomicAdd(row + lane, (unsigned long long)myc);
        if (lane == (uint32_t)C_NORMDEV_BITS) atomicMax(row + lane, (unsigned long long)__double_as_longlong(maxdev));
        myc = 0;
        maxdev = 0.0;
    };

    // Work stealing by groups of `grab` (<= 64) consecutive shots.  A wave
    // writes its shots' output words one shot after the other, so L2 gathers
    // each output plane's words of a group into whole lines.
    uint64_t group_base = 0;
    uint32_t group_len = 0, group_pos = 0;
    // Output plane of this lane: record word `lane` (lanes below kRecSgpr),
    // then status, abort op and observables; null when the caller did not ask.
    uint32_t *out_plane = nullptr;
    if (lane < kRecSgpr) {
        if (P.outcomes && lane < P.rec_words) out_plane = P.outcomes + (uint64_t)lane * P.n_shots;
    } else if (lane == kRecSgpr) {
        out_plane = P.status;
    } else if (lane == kRecSgpr + 1u) {
        out_plane = P.abort_op;
    } else if (lane == kRecSgpr + 2u) {
        out_plane = P.obs;
    }
    while (true) {
        if (group_pos == group_len) {
            unsigned long long got = 0;
            if (lane == 0) got = atomicAdd(P.next, (unsigned long long)P.grab);
            group_base = uni64(__shfl((unsigned long long)got, 0, 64));
            if (group_base >= P.n_shots) break;
            group_len = (uint32_t)min((uint64_t)P.grab, P.n_shots - group_base);
            group_pos = 0;
        }
        const uint64_t i = group_base + group_pos;
        // a vector load of a uniform address: say that the result is uniform
        // (item i of the prefix build runs the first shot of variant i / 2)
        const uint64_t shot = uni64((!LEAN && P.prefix_build) ? ((i >> 1) ? P.vars[(i >> 1) - 1u].shot_end : 0ull)
                                    : (!LEAN && P.shot_list) ? P.shot_list[i] : P.shot0 + i);
        const uint32_t s_lo = (uint32_t)shot, s_hi = (uint32_t)(shot >> 32);
        if (!var_ok || shot >= var_end || shot < var_lo) {
            if (var_ok) flush_counters();
            // shots past the last range (possible only in a shot list) run as the last variant
            var = 0;
            while (var + 1u < P.n_vars && P.vars[var].shot_end <= shot) ++var;
            var = uni(var);
            var_lo = uni64(var ? P.vars[var - 1u].shot_end : 0ull);
            var_end = uni64(P.vars[var].shot_end);
            var_ok = true;
        }
        const uint32_t *wrow = EXPL ? words + i * P.word_stride : nullptr;

        // ---- per-shot state (set at the start of each attempt below) ----
        // record words 0..3 live in scalar registers, the rest in LDS
        uint32_t rrv = 0;  // record word `lane` for lanes below kRecSgpr
        auto rec_read = [&](uint32_t w) -> uint32_t {
            return w < kRecSgpr ? (uint32_t)__builtin_amdgcn_readlane((int)rrv, (int)w) : rec[w];
        };
        auto rec_toggle = [&](uint32_t w, uint32_t m) {
            if (w < kRecSgpr) rrv ^= lane == w ? m : 0u;
            else if (lane == 0) rec[w] ^= m;
        };
        // expect ^ XOR of the listed record bits for the current event (the
        // first (word, mask) pair is inline, the rest come from the pair table)
        uint32_t evc;
        auto parity_check = [&]() -> uint32_t {
            uint32_t pbits = EV32(expect);
            const uint32_t cnt_pairs = EV32(det_cnt);
            if (cnt_pairs) {
                pbits ^= par32(rec_read(EV32(dw0)) & EV32(dm0));
                for (uint32_t t = 1; t < cnt_pairs; ++t) {
                    const uint32_t w = det[2u * (EV32(det_off) + t)], m = det[2u * (EV32(det_off) + t) + 1u];
                    pbits ^= par32(rec_read(w) & m);
                }
            }
            return uni(pbits);
        };
        // Condition of a classically controlled event: the parity of its
        // record pairs, or (EVF_AND) whether every listed bit is 1.
        auto cond_check = [&](uint32_t flags) -> uint32_t {
            if (!(flags & EVF_AND)) return parity_check();
            const uint32_t cnt_pairs = EV32(det_cnt);
            uint32_t ok = 1u;
            if (cnt_pairs) {
                const uint32_t m0 = EV32(dm0);
                ok &= (rec_read(EV32(dw0)) & m0) == m0 ? 1u : 0u;
                for (uint32_t t = 1; t < cnt_pairs; ++t) {
                    const uint32_t w = det[2u * (EV32(det_off) + t)], m = det[2u * (EV32(det_off) + t) + 1u];
                    ok &= (rec_read(w) & m) == m ? 1u : 0u;
                }
            }
            return uni(ok);
        };
        uint64_t rD = 0, rS = 0, a = 0;
        uint32_t k = 0;
        double nrm2 = 1.0;
        // |tile|^2 = itscale2 |state|^2: branching T leave cos(pi/8) out of the
        // tile (kept as the inverse factor, so a T multiplies instead of divides)
        double itscale2 = 1.0;
        // After a span truncation down to one entry, whose exact state has unit
        // norm: rescale it in FP64 (the cuts the full list runs next do the same).
        auto renorm_single = [&]() {
            const C x = v[0];
            const double q = nrm<R>(x);
            const R sc = (R)(1.0 / sqrt(q));
            if (lane == 0) v[0] = scale(x, sc);
            nrm2 = q * (double)sc * (double)sc;
            itscale2 = 1.0;
        };
        uint32_t phase8 = 0;  // global phase e^{i pi phase8 / 8} from branching T gates
        uint32_t status = ST_PASSED, abort_src = 0xFFFFFFFFu, obs = 0, maxsup = 1;
        uint32_t term = 0, after = 0;
        // noise per slot: 256 slots per chunk, 4 consecutive slots (one Philox
        // block) per lane; nz_drawn = slots drawn.  Gap sampling: lanes hold
        // 256 words of stream 2 starting at word nz_cb, gd is the next word,
        // nz_drawn = slots decided, hw the word of the pending hit.
        uint32_t nz_cb = 0, nz_drawn = 0, next_hit = kNoHit;
        uint32_t hits = 0, w0 = 0, w1 = 0, w2 = 0, w3 = 0;
        uint32_t gd = 0, hw = 0;
        // measurement words: slots [m_base, m_base + 256), one Philox block per lane
        uint32_t m_base = 0xFFFFFF00u, mw0 = 0, mw1 = 0, mw2 = 0, mw3 = 0;

        // steps of this shot to trace (0 unless it is the traced shot)
        const uint32_t trace_lim = LEAN ? 0u : uni(P.trace_n != 0u && shot == P.trace_shot ? P.trace_n : 0u);
        const bool tracing = trace_lim != 0u;
        // noise tables of this variant (read where used: the draws are rare)
        const VariantDesc *vdp = P.vars + var;
        const uint32_t n_slots = uni(vdp->n_noise);

        // Draw the next 256 noise slots: one Philox block of 4 words per lane.
        auto draw_chunk = [&]() {
            const uint32_t n_noise = vdp->n_noise;
            nz_cb = nz_drawn;
            nz_drawn += 256u;
            const uint32_t s0 = nz_cb + 4u * lane;
            if (EXPL) {
                w0 = s0 + 0u < n_noise ? wrow[s0 + 0u] : 0u;
                w1 = s0 + 1u < n_noise ? wrow[s0 + 1u] : 0u;
                w2 = s0 + 2u < n_noise ? wrow[s0 + 2u] : 0u;
                w3 = s0 + 3u < n_noise ? wrow[s0 + 3u] : 0u;
            } else {
                philox10(s0 >> 2, s_lo, s_hi, 0u, key0, key1, w0, w1, w2, w3);
            }
            const uint4 th = *reinterpret_cast<const uint4 *>(tm1 + vdp->tm1_off + s0);
            hits = (s0 + 0u < n_noise && w0 <= th.x ? 1u : 0u) | (s0 + 1u < n_noise && w1 <= th.y ? 2u : 0u) |
                   (s0 + 2u < n_noise && w2 <= th.z ? 4u : 0u) | (s0 + 3u < n_noise && w3 <= th.w ? 8u : 0u);
            next_hit = first_hit(hits, nz_cb);
        };
        // Gap sampling: decide the slots up to the next candidate.  A
        // candidate takes words gd, gd + 1 of stream 2 (gap, then acceptance;
        // gd is even, so both sit in one Philox block, 64 blocks = 256 words
        // held one block per lane).  The gap G = #{j : w < gap[j]} (a prefix,
        // the table falls with j) is found 64 entries apart, then entry by
        // entry, one entry per lane; entries past the last slot count as false.
        // The one-round-trip estimate, and skipping the acceptance load when
        // every slot accepts: measured +2.5% FP64, +2% on span-12 split
        // tiles and, in the lean kernels, +2.4% on FP32 LDS tiles (where,
        // before the lean kernels freed registers, it cost 2%).
        constexpr bool kGapEstimate = true;
        auto draw_gap = [&]() {
            if ((gd & ~255u) != nz_cb) {
                nz_cb = gd & ~255u;
                philox10((nz_cb >> 2) + lane, s_lo, s_hi, 2u, key0, key1, w0, w1, w2, w3);
            }
            const uint32_t L = (gd - nz_cb) >> 2;
            const bool hi = (gd & 2u) != 0u;
            const uint32_t w = uni((uint32_t)__builtin_amdgcn_readlane((int)(hi ? w2 : w0), (int)L));
            const uint32_t aw = uni((uint32_t)__builtin_amdgcn_readlane((int)(hi ? w3 : w1), (int)L));
            gd += 2u;
            const uint32_t lim = vdp->n_noise - nz_drawn;
            const uint32_t *tb = P.gaps + vdp->gap_off;
            // G = #{j < lim : w < tb[j]} (tb is non-increasing).  q^G is
            // about w / 2^32, so G is within a slot or two of
            // x = log2(w / 2^32) / log2(q): with kGapEstimate, lanes 0..3
            // test the entries floor(x) - 2 .. floor(x) + 1 (an index below 0
            // counts as passing), and when lane 0 passes and lane 3 fails
            // they bracket G exactly, in one round trip to the table.
            // Otherwise the search below, 64 entries a step (two or more
            // round trips).
            uint32_t G = 0xFFFFFFFFu;
            if (kGapEstimate) {
                const float x = fminf(fmaxf((__log2f((float)w + 0.5f) - 32.0f) * vdp->gap_l2q, 0.0f),
                                      (float)lim + 4.0f);
                const int32_t base = (int32_t)x - 2;
                const int32_t j = base + (int32_t)lane;
                bool t = j < 0;
                if (lane < 4u && j >= 0 && (uint32_t)j < lim) t = w < tb[j];
                const uint64_t b = __ballot(lane < 4u && t);
                if ((b & 1ull) && !(b & 8ull)) G = (uint32_t)(base + (int32_t)__builtin_popcountll(b));
            }
            if (G == 0xFFFFFFFFu) {
                G = 0;
                for (;;) {
                    const uint32_t j1 = G + 64u * lane;
                    const uint32_t n1 = (uint32_t)__builtin_popcountll(__ballot(j1 < lim && w < tb[j1]));
                    if (n1 == 0u) break;
                    const uint32_t b2 = G + 64u * (n1 - 1u) + 1u;
                    const uint32_t j2 = b2 + lane;
                    const uint32_t n2 = (uint32_t)__builtin_popcountll(__ballot(lane < 63u && j2 < lim && w < tb[j2]));
                    G = b2 + n2;
                    if (n1 < 64u || n2 < 63u) break;
                }
            }
            G = uni(G);
            if (G >= lim) {
                nz_drawn = vdp->n_noise;
                return;
            }
            const uint32_t cslot = nz_drawn + G;
            nz_drawn = cslot + 1u;
            if ((kGapEstimate && vdp->acc_one) || (uint64_t)aw < nz[vdp->nz_off + cslot].acc) {
                next_hit = cslot;
                hw = aw;
            }
        };
        // Decode the pending hit at slot next_hit into sign-flip masks (or a
        // record flip, returned; kNoHit otherwise) and move to the next hit.
        auto take_hit = [&](uint64_t &dD, uint64_t &dS) -> uint32_t {
            const uint32_t L = (next_hit - nz_cb) >> 2, b = next_hit & 3u;
            uint64_t wv;
            if (GAPS) {
                wv = hw;
            } else {
                const uint32_t pick = b == 0u ? w0 : b == 1u ? w1 : b == 2u ? w2 : w3;
                wv = (uint32_t)__builtin_amdgcn_readlane((int)pick, (int)L);
            }
            const NoiseLoc &NL = nz[vdp->nz_off + next_hit];
            const uint64_t thr = GAPS ? NL.acc : NL.thr;
            const uint32_t nkind = NL.kind;
            uint32_t fr = kNoHit;
            dD = 0;
            dS = 0;
            if (nkind == NZ_DEP1 || nkind == NZ_DEP2 || nkind == NZ_XERR || nkind == NZ_ZERR) {
                uint32_t ca, cb = 0;
                if (nkind == NZ_DEP1) {
                    ca = quot16(3ull * wv, thr) + 1u;  // wv < thr
                } else if (nkind == NZ_DEP2) {
                    const uint32_t code = quot16(15ull * wv, thr) + 1u;
                    ca = code >> 2;
                    cb = code & 3u;
                } else {
                    ca = nkind == NZ_XERR ? 1u : 3u;
                }
                // Pauli codes: 1 = X, 2 = Y, 3 = Z
                if (ca == 1u || ca == 2u) { dD ^= NL.masks[0]; dS ^= NL.masks[1]; }
                if (ca == 3u || ca == 2u) { dD ^= NL.masks[2]; dS ^= NL.masks[3]; }
                if (cb == 1u || cb == 2u) { dD ^= NL.masks[4]; dS ^= NL.masks[5]; }
                if (cb == 3u || cb == 2u) { dD ^= NL.masks[6]; dS ^= NL.masks[7]; }
            } else if (nkind == NZ_FLIP) {
                fr = NL.rec;
            }
            if (GAPS) {
                next_hit = kNoHit;
            } else {
                if (lane == L) hits &= ~(1u << b);
                next_hit = first_hit(hits, nz_cb);
            }
            return fr;
        };
        // The speculative event list runs first (a traced shot takes the full
        // list, so that every trace step exists); a failed DROP check, or a
        // support above the cap, restarts the shot on the full list.  A shot's draws depend only on its slots,
        // so the restarted shot is the one the full list gives.
        // (with a support cap the full list runs: the cap is defined by the
        // supports of the circuit's own gate order)
        bool full = tracing || !P.speculate || (LEAN ? 0xFFFFFFFFu : P.support_cap) != 0xFFFFFFFFu || vdp->ev_off_full == vdp->ev_off;
        if ((!LEAN && P.prefix_build)) full = (i & 1u) != 0u || vdp->ev_off_full == vdp->ev_off;
        bool pfx_done = false;      // the build wrote every checkpoint of this item's list
        uint32_t ck_next_done = 0;  // checkpoints written
        // the checkpoint whose tile the shot still has to load (null: the
        // tile is in place)
        const unsigned char *lazy_slot = nullptr;
        // Deferred T runs (EVF_DEFER): skipped while defer_ok; `deferred` once
        // one was skipped, and `redo` when an event needed its tile (the
        // attempt then runs again with defer_ok off).
        bool defer_ok = P.defer != 0u && !tracing && !(!LEAN && P.prefix_build) && (LEAN ? 0xFFFFFFFFu : P.support_cap) == 0xFFFFFFFFu;
        // Butterfly pairs run as one pass where an FP32 pass reads and
        // writes device memory (tiles there, or split tiles larger than
        // their LDS part): each entry crosses to the slab once instead of
        // twice (+9% on span-12 split tiles).  Elsewhere the two separate
        // passes, tuned per quarter turn, are faster: the pair pass measured
        // -10% on FP32 LDS tiles and -6% on FP64 split tiles of span 10
        // (half the tile in the slab, and twice the arithmetic per byte).
        // Not when a trace wants the state after each event or a support cap
        // is checked after each T.
        constexpr bool kPairs = TM != TM_LDS && sizeof(R) == 4;
        const bool pair_ok = kPairs && !tracing && (LEAN ? 0xFFFFFFFFu : P.support_cap) == 0xFFFFFFFFu;
        auto pair_now = [&](uint32_t fl) { return (fl & EVF_PAIR) && pair_ok && (1u << k) > v.lim; };
        bool deferred = false, redo = false;
        // A deferred run applied late: the signs the run saw and the state
        // to come back to live in lanes of one register (rarely touched):
        // lanes 0-3 the signs at the run, 4-7 the signs at the event that
        // needs the tile, 8 that event, 9 and 10 the run's first event and
        // the one after it.
        bool replaying = false;
        uint32_t stash = 0u;
        auto put = [&](uint32_t l, uint32_t x) { stash = lane == l ? x : stash; };
        auto get = [&](uint32_t l) { return uni((uint32_t)__builtin_amdgcn_readlane((int)stash, (int)l)); };
        auto get64 = [&](uint32_t l) { return ((uint64_t)get(l + 1u) << 32) | (uint64_t)get(l); };
        const uint32_t tile_off = kCkptRecOff + ((P.rec_words * 4u + 15u) & ~15u);
        auto materialize = [&]() {
            const C *pt = reinterpret_cast<const C *>(lazy_slot + tile_off);
            lane_pass(1u << k, lane, [&](uint32_t j) { v[j] = pt[j]; });
            tile_sync();
            lazy_slot = nullptr;
        };
        for (;;) {
        const uint32_t *evl = reinterpret_cast<const uint32_t *>(ev + (full ? vdp->ev_off_full : vdp->ev_off));
        for (uint32_t w = kRecSgpr + lane; w < P.rec_words; w += 64) rec[w] = 0u;
        rrv = 0u;
        if (lane == 0) v[0] = mk<C>(1.0, 0.0);
        tile_sync();
        rD = rS = a = 0ull;
        k = 0;
        phase8 = 0;
        nrm2 = 1.0;
        itscale2 = 1.0;
        status = ST_PASSED;
        abort_src = 0xFFFFFFFFu;
        obs = 0;
        maxsup = 1;
        term = after = 0;
        nz_cb = GAPS ? 0xFFFFFFFFu : 0u;
        nz_drawn = 0;
        next_hit = kNoHit;
        hits = 0;
        gd = 0;
        m_base = 0xFFFFFF00u;
        bool restart = false;
        // Checkpoints of the noiseless trajectory of this list: entries
        // [ck_o, ck_o + ck_c) of the checkpoint table, each with a state slot
        // the build launch wrote for this launch.
        const uint32_t ck_o = uni(full ? vdp->ck_off_full : vdp->ck_off);
        const uint32_t ck_c = uni(full ? vdp->ck_cnt_full : vdp->ck_cnt);
        auto ck_slot = [&](uint32_t t) { return P.prefix + (size_t)t * P.prefix_stride; };
        // The build: no noise (every slot counts as drawn, none hit); the
        // list's events run up to its last checkpoint, and the state at each
        // checkpoint goes to its slot (the full list's item only, when the
        // variant has one list).
        uint32_t ck_next = 0;
        if ((!LEAN && P.prefix_build)) {
            nz_drawn = n_slots;
            if (ck_c == 0u || (!(i & 1u) && vdp->ev_off_full == vdp->ev_off)) {
                pfx_done = true;  // nothing to write (or the odd item writes these slots)
                break;
            }
        }
        auto write_ckpt = [&](uint32_t t) {
            unsigned char *slot = ck_slot(t);
            C *pt = reinterpret_cast<C *>(slot + tile_off);
            const double nn = tile_norm(v, k, lane);
            lane_pass(1u << k, lane, [&](uint32_t j) { pt[j] = v[j]; });
            uint32_t *pr = reinterpret_cast<uint32_t *>(slot + kCkptRecOff);
            if (lane < kRecSgpr && lane < P.rec_words) pr[lane] = rrv;
            for (uint32_t w = kRecSgpr + lane; w < P.rec_words; w += 64u) pr[w] = rec[w];
            if (lane == 0) {
                CkptState *cs = reinterpret_cast<CkptState *>(slot);
                cs->rD = rD;
                cs->rS = rS;
                cs->a = a;
                cs->nrm2 = nrm2;
                cs->itscale2 = itscale2;
                cs->tnorm = nn;
                cs->k = k;
                cs->phase8 = phase8;
                cs->maxsup = maxsup;
                cs->obs = obs;
                cs->valid = 1u;
            }
        };
        // A shot starts at the last checkpoint before its first noise hit:
        // the noise slots are decided here as the event loop would decide
        // them (the same draws; no hit is taken, there is none before the
        // checkpoint), the scalars and the record come from the slot, and the
        // tile is loaded only if an event reads it (EVF_MAT): a shot that a
        // check ends first never needs it.
        uint32_t e0 = 0;
        lazy_slot = nullptr;
        deferred = false;
        replaying = false;
        if (P.prefix != nullptr && !(!LEAN && P.prefix_build) && !tracing && ck_c != 0u) {
            // checkpoint c's noise count and validity in lane c (one load each)
            uint32_t cev = 0u, cnz = 0xFFFFFFFFu, cok = 0u;
            if (lane < ck_c) {
                const Checkpoint cp = P.ckpts[ck_o + lane];
                cev = cp.ev;
                cnz = cp.nz;
                cok = reinterpret_cast<const CkptState *>(ck_slot(ck_o + lane))->valid;
            }
            uint32_t best = 0xFFFFFFFFu;
            for (uint32_t c = 0; c < ck_c; ++c) {
                const uint32_t pn = uni((uint32_t)__builtin_amdgcn_readlane((int)cnz, (int)c));
                while (next_hit >= pn && nz_drawn < pn && nz_drawn < n_slots) {
                    if (GAPS) draw_gap(); else draw_chunk();
                }
                if (next_hit < pn || (uint32_t)__builtin_amdgcn_readlane((int)cok, (int)c) != 1u) break;
                best = c;
            }
            if (best != 0xFFFFFFFFu) {
                // the slot's header, dword d in lane d
                const unsigned char *slot = ck_slot(ck_o + best);
                const uint32_t hd = lane < (uint32_t)(sizeof(CkptState) / 4u) ? reinterpret_cast<const uint32_t *>(slot)[lane] : 0u;
                auto h32 = [&](uint32_t off) { return (uint32_t)__builtin_amdgcn_readlane((int)hd, (int)(off / 4u)); };
                auto h64 = [&](uint32_t off) { return ((uint64_t)h32(off + 4u) << 32) | (uint64_t)h32(off); };
                rD = h64(offsetof(CkptState, rD));
                rS = h64(offsetof(CkptState, rS));
                a = h64(offsetof(CkptState, a));
                nrm2 = __longlong_as_double((long long)h64(offsetof(CkptState, nrm2)));
                itscale2 = __longlong_as_double((long long)h64(offsetof(CkptState, itscale2)));
                k = h32(offsetof(CkptState, k));
                phase8 = h32(offsetof(CkptState, phase8));
                maxsup = h32(offsetof(CkptState, maxsup));
                obs = h32(offsetof(CkptState, obs));
                const uint32_t *pr = reinterpret_cast<const uint32_t *>(slot + kCkptRecOff);
                if (lane < kRecSgpr && lane < P.rec_words) rrv = pr[lane];
                for (uint32_t w = kRecSgpr + lane; w < P.rec_words; w += 64u) rec[w] = pr[w];
                lazy_slot = slot;
                e0 = uni((uint32_t)__builtin_amdgcn_readlane((int)cev, (int)best));
                myc += lane == (uint32_t)C_PREFIX ? 1u : 0u;
            }
        }
        // Event e sits in evc, one dword per lane; event e + 1 is in evx, and
        // event e + 2 is loaded while event e runs (the list ends with three
        // END events).
        evc = evl[(uint64_t)e0 * 64u + lane];
        uint32_t evx = evl[(uint64_t)(e0 + 1u) * 64u + lane];
        uint32_t e = e0;  // after the loop: the last event run
        // trace steps, or (build) the events up to the last checkpoint
        const uint32_t dump_lim = ((!LEAN && P.prefix_build) && ck_c) ? uni(P.ckpts[ck_o + ck_c - 1u].ev) + 1u : trace_lim;
        for (;; ++e) {
            if (replaying && e == get(10)) {
                // the deferred run is applied: back to the event that needed
                // it, with the signs it had (its own Clifford flips not yet
                // applied), to run it from its start
                rD = get64(4);
                rS = get64(6);
                e = get(8);
                evc = evl[(uint64_t)e * 64u + lane];
                evx = evl[(uint64_t)(e + 1u) * 64u + lane];
                replaying = false;
            }
            uint32_t evy = evl[(uint64_t)(e + 2u) * 64u + lane];
            if (e - 1u < dump_lim) {  // state after event e-1 (e = 0 wraps past any limit)
                if ((!LEAN && P.prefix_build)) {
                    if (e == uni(P.ckpts[ck_o + ck_next].ev)) {
                        write_ckpt(ck_o + ck_next);
                        ck_next_done = ++ck_next;
                        if (ck_next == ck_c) {
                            pfx_done = true;
                            break;
                        }
                    }
                } else {
                    dump_state(P.trace_meta + (uint64_t)(e - 1u) * KM_COUNT,
                               P.trace_v + (uint64_t)(e - 1u) * P.tile_entries * 2u, v, lane, P.tile_entries, status,
                               abort_src, e - 1u, 1u, rD, rS, a, k, nrm2, P.phase_tab, phase8, var, full ? 1u : 0u,
                               1.0 / itscale2);
                }
            }
            // ---- noise slots before this event ----
            // Hits are rare: `next_hit` is the lowest pending hit of the drawn
            // chunk, so an event with none before it costs two compares.
            // k changes only in uniform branches; say so, or the compiler
            // lowers every pass over the tile as a divergent loop
            k = uni(k);
            const uint32_t nend = EV32(noise_end);
            while (true) {
                while (next_hit < nend) {
                    uint64_t dD, dS;
                    const uint32_t fr = take_hit(dD, dS);
                    rD ^= dD;
                    rS ^= dS;
                    if (fr != kNoHit) rec_toggle(fr >> 5, 1u << (fr & 31u));
                }
                if (nend <= nz_drawn || nz_drawn >= n_slots) break;
                if (GAPS) draw_gap(); else draw_chunk();
            }
            // ---- Cliffords since the previous event: one XOR ----
            uint32_t flags = EV32(flags);
            uint32_t kind = EV32(kind);
            // a run applied late: its first event's Clifford flips are in
            // the saved signs, and it is neither deferred nor loaded again
            if (replaying) flags &= ~(EVF_CLIFF | EVF_MAT | EVF_DEFER);
            if (flags & (EVF_CLIFF | EVF_MAT | EVF_DEFER)) {
                // an event that needs the tile after a deferred T run: apply
                // the run now, with the signs it saw (T reads only those; the
                // events since then left the tile alone), then come back here
                if ((flags & EVF_MAT) && deferred) {
                    if (lazy_slot != nullptr) materialize();
                    put(4u, (uint32_t)rD);
                    put(5u, (uint32_t)(rD >> 32));
                    put(6u, (uint32_t)rS);
                    put(7u, (uint32_t)(rS >> 32));
                    put(8u, e);
                    rD = get64(0u);
                    rS = get64(2u);
                    const uint32_t r0 = get(9u);
                    const Event *d0 = reinterpret_cast<const Event *>(evl) + r0, *d1 = d0 + (get(10u) - r0);
                    if (lane == (uint32_t)C_ENTRIES_T) myc += d1->cum_t - d0->cum_t;
                    if (lane == (uint32_t)C_EVENTS) myc += (uint64_t)(d1->cum_e - d0->cum_e);
                    myc += lane == (uint32_t)C_REDO ? 1u : 0u;
                    deferred = false;
                    replaying = true;
                    e = r0 - 1u;  // the loop's step takes it to the run's first event
                    evx = evl[(uint64_t)r0 * 64u + lane];
                    evy = evl[(uint64_t)(r0 + 1u) * 64u + lane];
                    kind = EV_NOP;
                    flags = 0u;
                }
                if (flags & EVF_CLIFF) {
                    rD ^= EV64(cliffD);
                    rS ^= EV64(cliffS);
                }
                if ((flags & EVF_DEFER) && defer_ok) {
                    // skip the run: its gates change only the tile, which no
                    // event needs before the one flagged EVF_MAT
                    const uint32_t m = EV32(mslot);
                    // (the work counters count the work run: the run's is taken off)
                    const Event *d0 = reinterpret_cast<const Event *>(evl) + e, *d1 = d0 + m;
                    if (lane == (uint32_t)C_ENTRIES_T) myc -= d1->cum_t - d0->cum_t;
                    if (lane == (uint32_t)C_EVENTS) myc -= (uint64_t)(d1->cum_e - d0->cum_e);
                    deferred = true;
                    put(0u, (uint32_t)rD);
                    put(1u, (uint32_t)(rD >> 32));
                    put(2u, (uint32_t)rS);
                    put(3u, (uint32_t)(rS >> 32));
                    put(9u, e);
                    put(10u, e + m);
                    e += m - 1u;
                    evx = evl[(uint64_t)(e + 1u) * 64u + lane];
                    evy = evl[(uint64_t)(e + 2u) * 64u + lane];
                    kind = EV_NOP;
                    flags = 0u;
                } else if ((flags & EVF_MAT) && lazy_slot != nullptr && !(kPairs && pair_now(flags))) {
                    materialize();
                }
            }
            if (kind == EV_END) {
                term = e;
                break;
            }
            // sign part of c, plus gamma . a (always used together): one parity
            const uint32_t sga = par64((rD & EV64(beta)) ^ ((rS ^ a) & EV64(gamma)));
            const uint32_t g = EV32(g);
            if (kind == EV_T_PHASE) {
                // lambda_j = (-1)^(sig ^ parity(g & j)); lambda = -1 picks up e^{i s pi/4}
                const uint32_t sig = (EV32(cexp) == 2u ? 1u : 0u) ^ sga;
                const R fr = (R)EVD(Are), fi = (R)EVD(Aim);
                const uint32_t cnt = 1u << k;
                if (g != 0u || sig) {
                    lane_pass(cnt, lane, [&](uint32_t j) {
                        if (sig ^ par32(g & j)) {
                            C x = v[j];
                            C y;
                            y.x = x.x * fr - x.y * fi;
                            y.y = x.x * fi + x.y * fr;
                            v[j] = y;
                        }
                    });
                }
            } else if (flags & EVF_TRUN) {
                // ---- m doublings with nothing between them, as one pass ----
                // Final entry J (K = k + m <= 6 coordinates: one per lane) is
                // entry J mod 2^k turned by i^(fixed + 2 x dynamic signs of the
                // members whose coordinate J sets) and multiplied by tn once per
                // such member, in member order: the separate passes' products.
                // Pruning once at the last member's level keeps what they keep
                // (the level only rises, and an entry is below its source).
                const uint32_t m = EV32(bcnt), K = k + m;
                uint32_t sg = 0;  // member `lane`'s sign part (no flips between members)
                if (lane < m) {
                    const uint4 bg =
                        *reinterpret_cast<const uint4 *>(evl + (uint64_t)(e + lane) * 64u + offsetof(Event, beta) / 4u);
                    const uint64_t B = ((uint64_t)bg.y << 32) | bg.x, G = ((uint64_t)bg.w << 32) | bg.z;
                    sg = par64((rD & B) ^ ((rS ^ a) & G));
                }
                const uint32_t sm = (uint32_t)__ballot(sg != 0u);
                const uint32_t J = lane & ((1u << K) - 1u);  // lanes past 2^K repeat a live lane
                const uint32_t nb = J >> k;                    // members whose coordinate J sets
                const uint32_t q = ((uint32_t)(EV64(trot0) >> J) & 1u) + 2u * ((uint32_t)(EV64(trot1) >> J) & 1u) +
                                   2u * par32(sm & nb);
                const R tn = sizeof(R) == 4 ? (R)EVF(Tnf) : (R)EVD(Tn);
                C x = rot(v[J & ((1u << k) - 1u)], q);
                for (uint32_t i = 0; i < m; ++i) {
                    if ((nb >> i) & 1u) {
                        x.x = tn * x.x;
                        x.y = tn * x.y;
                    }
                }
                const R nq = fma(x.x, x.x, x.y * x.y);
                const double ics = EVD(iCs2);
                uint32_t cmax = 0;
                bool keep = false;
                for (uint32_t i = 0; i < m; ++i) {  // support after each member
                    itscale2 *= ics;
                    const R thr = (R)(tau2 * nrm2 * itscale2);
                    keep = nq >= thr;
                    const uint32_t lim = 1u << (k + i + 1u);
                    const uint64_t lv = lim >= 64u ? ~0ull : ((1ull << lim) - 1ull);
                    cmax = max(cmax, (uint32_t)__popcll(__ballot(keep) & lv));
                }
                if (!keep) {
                    x.x = 0;
                    x.y = 0;
                }
                v[J] = x;
                phase8 = (phase8 + EV32(boff)) & 15u;
                cmax = uni(cmax);
                maxsup = max(maxsup, cmax);
                if (cmax > (LEAN ? 0xFFFFFFFFu : P.support_cap)) {  // only the full list enforces a cap
                    restart = true;
                    break;
                }
                k = K;
                e += m - 1u;
                evx = evl[(uint64_t)(e + 1u) * 64u + lane];
                evy = evl[(uint64_t)(e + 2u) * 64u + lane];
            } else if (flags & EVF_BRUN) {
                // ---- m butterflies that each drop the top coordinate ----
                // Entry j sits in lane j (k <= 6).  Member i mixes lanes j and
                // j ^ mu_i with the partner weight tn i^qb_i (-1)^(sig_i ^
                // parity(g_i & (j ^ mu_i))), prunes at its level and drops
                // coordinate k - 1 when no entry with that bit set is kept
                // (else the shot restarts): the separate passes, step by step.
                const uint32_t m = EV32(bcnt), k0 = k;
                uint32_t sg = 0, gv = 0, qv = 0, mv = 0;  // member `lane`'s fields
                if (lane < m) {
                    const uint32_t *rp = evl + (uint64_t)(e + lane) * 64u;
                    const uint4 bg = *reinterpret_cast<const uint4 *>(rp + offsetof(Event, beta) / 4u);
                    const uint4 kg = *reinterpret_cast<const uint4 *>(rp + offsetof(Event, k) / 4u);
                    const uint64_t B = ((uint64_t)bg.y << 32) | bg.x, G = ((uint64_t)bg.w << 32) | bg.z;
                    sg = par64((rD & B) ^ ((rS ^ a) & G));
                    gv = kg.y;
                    qv = kg.w;
                    mv = rp[offsetof(Event, mu) / 4u];
                }
                const uint32_t sm = (uint32_t)__ballot(sg != 0u);
                const R tn = sizeof(R) == 4 ? (R)EVF(Tnf) : (R)EVD(Tn);
                const double ics = EVD(iCs2);
                C x = v[lane & ((1u << k0) - 1u)];
                bool fail = false;
                uint32_t fi = 0;  // member whose check failed (the last one run)
                for (uint32_t i = 0; i < m; ++i) {
                    const uint32_t mu = uni((uint32_t)__builtin_amdgcn_readlane((int)mv, (int)i));
                    const uint32_t gi = uni((uint32_t)__builtin_amdgcn_readlane((int)gv, (int)i));
                    const uint32_t qi = uni((uint32_t)__builtin_amdgcn_readlane((int)qv, (int)i));
                    const uint32_t pl = lane ^ mu;  // mu < 2^k <= 64
                    C y;
                    y.x = __shfl(x.x, (int)pl, 64);
                    y.y = __shfl(x.y, (int)pl, 64);
                    const C w = rot(y, qi);
                    const R c = (((sm >> i) & 1u) ^ par32(gi & pl)) != 0u ? -tn : tn;
                    itscale2 *= ics;
                    const R thr = (R)(tau2 * nrm2 * itscale2);
                    C o;
                    o.x = fma(c, w.x, x.x);
                    o.y = fma(c, w.y, x.y);
                    const bool keep = fma(o.x, o.x, o.y * o.y) >= thr;
                    if (!keep) {
                        o.x = 0;
                        o.y = 0;
                    }
                    const uint32_t n = 1u << k;
                    const uint64_t kb = __ballot(keep) & (n >= 64u ? ~0ull : ((1ull << n) - 1ull));
                    const uint32_t cnt = uni((uint32_t)__popcll(kb));
                    maxsup = max(maxsup, cnt);
                    // lanes n/2 .. n-1 hold the entries with the dropped bit set
                    if (cnt > (LEAN ? 0xFFFFFFFFu : P.support_cap) || (kb >> (n >> 1)) != 0ull) {
                        fail = true;
                        fi = i;
                        break;
                    }
                    x = o;
                    --k;
                }
                if (fail) {
                    // the attempt's work counts up to member fi, as with separate passes
                    e += fi;
                    restart = true;
                    break;
                }
                // the dropped halves hold pruned zeros, as the separate passes leave them
                if (lane < (1u << k0)) {
                    if (lane >= (1u << k)) {
                        x.x = 0;
                        x.y = 0;
                    }
                    v[lane] = x;
                }
                phase8 = (phase8 + EV32(boff)) & 15u;
                if (k == 0u) renorm_single();
                e += m - 1u;
                evx = evl[(uint64_t)(e + 1u) * 64u + lane];
                evy = evl[(uint64_t)(e + 2u) * 64u + lane];
            } else if (kPairs && pair_now(flags)) {
                // ---- a butterfly and the next one, in one pass ----
                // Nothing acts between them (no noise slot, no Clifford
                // flip): the second's sign comes from the same signs, and
                // its scalar updates follow the first's, as in two passes.
                const uint32_t f2 = EVX32(flags);
                const uint32_t sg2 = par64((rD & EVX64(beta)) ^ ((rS ^ a) & EVX64(gamma)));
                itscale2 *= EVD(iCs2);
                const R tn1 = sizeof(R) == 4 ? (R)EVF(Tnf) : (R)EVD(Tn);
                const R thr1 = (R)(tau2 * nrm2 * itscale2);
                itscale2 *= __longlong_as_double((long long)EVX64(iCs2));
                const R tn2 = sizeof(R) == 4 ? (R)__uint_as_float(EVX32(Tnf)) : (R)__longlong_as_double((long long)EVX64(Tn));
                const R thr2 = (R)(tau2 * nrm2 * itscale2);
                const uint32_t pv = EV32(pbit);
                uint32_t cnt1, cnt2;
                uint64_t upper;
                if (lazy_slot != nullptr) {
                    // the shot's tile is still the checkpoint's: read it there
                    Tile<C, TM_MEM> ck;
                    ck.lo = reinterpret_cast<C *>(const_cast<unsigned char *>(lazy_slot) + tile_off);
                    ck.hi = nullptr;
                    ck.lim = 0;
                    t_bfly_pair<R, C, TM, TM_MEM>(v, ck, lane, k, pv & 255u, pv >> 8, EV32(mu), g, sga, EV32(qb), tn1,
                                                  thr1, EVX32(mu), EVX32(g), sg2, EVX32(qb), tn2, thr2,
                                                  (f2 & EVF_DROP1) != 0u, cnt1, cnt2, upper);
                    lazy_slot = nullptr;
                } else {
                    t_bfly_pair<R, C, TM, TM>(v, v, lane, k, pv & 255u, pv >> 8, EV32(mu), g, sga, EV32(qb), tn1, thr1,
                                              EVX32(mu), EVX32(g), sg2, EVX32(qb), tn2, thr2, (f2 & EVF_DROP1) != 0u,
                                              cnt1, cnt2, upper);
                }
                phase8 = (phase8 + ((flags & EVF_TDG) ? 15u : 1u) + ((f2 & EVF_TDG) ? 15u : 1u)) & 15u;
                maxsup = max(maxsup, max(uni(cnt1), uni(cnt2)));
                // the second event has run: the list goes on after it
                ++e;
                evx = evy;
                evy = evl[(uint64_t)(e + 2u) * 64u + lane];
                if (f2 & EVF_DROP1) {
                    if (upper != 0ull) {
                        restart = true;
                        break;
                    }
                    --k;
                }
            } else if (kind == EV_T_DOUBLE || kind == EV_T_BFLY) {
                const R tn = sizeof(R) == 4 ? (R)EVF(Tnf) : (R)EVD(Tn);
                const uint32_t sig = sga;
                // T is unitary: the carried norm stays, and it sets the pruning
                // level, on the tile's scale once cos^2(pi/8) joins the factor
                itscale2 *= EVD(iCs2);
                const R thr = (R)(tau2 * nrm2 * itscale2);
                const uint32_t qb = EV32(qb), pb = EV32(tpair);
                uint32_t cnt, upper = 0;
                if (kind == EV_T_DOUBLE) {
                    switch (qb) {
                        case 0: cnt = t_double<0, R, C, TM>(v, lane, k, g, sig, tn, thr, pb); break;
                        case 1: cnt = t_double<1, R, C, TM>(v, lane, k, g, sig, tn, thr, pb); break;
                        case 2: cnt = t_double<2, R, C, TM>(v, lane, k, g, sig, tn, thr, pb); break;
                        default: cnt = t_double<3, R, C, TM>(v, lane, k, g, sig, tn, thr, pb); break;
                    }
                    ++k;
                } else {
                    const uint32_t mu = EV32(mu), h = EV32(tstar), lm = EV32(lmask);
                    switch (qb) {
                        case 0: cnt = t_bfly<0, R, C, TM>(v, lane, k, mu, h, g, sig, tn, thr, pb, lm, upper); break;
                        case 1: cnt = t_bfly<1, R, C, TM>(v, lane, k, mu, h, g, sig, tn, thr, pb, lm, upper); break;
                        case 2: cnt = t_bfly<2, R, C, TM>(v, lane, k, mu, h, g, sig, tn, thr, pb, lm, upper); break;
                        default: cnt = t_bfly<3, R, C, TM>(v, lane, k, mu, h, g, sig, tn, thr, pb, lm, upper); break;
                    }
                }
                phase8 = (phase8 + ((flags & EVF_TDG) ? 15u : 1u)) & 15u;
                cnt = uni(cnt);
                maxsup = max(maxsup, cnt);
                if (cnt > (LEAN ? 0xFFFFFFFFu : P.support_cap)) {
                    // the speculative list visits other intermediate states:
                    // the full list decides where (and whether) the cap is hit
                    if (!full) {
                        restart = true;
                        break;
                    }
                    status = ST_OVERFLOW;
                    abort_src = EV32(src);
                    term = e;
                    after = 1;
                    break;
                }
                if (flags & EVF_DROP1) {
                    // speculative: the top coordinate (the partner half) must be empty
                    if (uni(upper) != 0u) {
                        restart = true;
                        break;
                    }
                    --k;
                    if (k == 0u) renorm_single();
                }
            } else if (kind == EV_M_DET && (flags & EVF_BATCH) && !tracing) {
                // ---- a run of outcome-fixed measurements, one member per lane ----
                // Member i sees the signs rD, rS of the first member, the
                // Clifford flips since then (cumD, cumS) and the noise hits
                // before its own noise_end; its outcome is c times the sign of
                // the product of the rows that make up the measured Pauli.
                const uint32_t m = EV32(bcnt);
                const uint32_t li = lane < m ? lane : m - 1u;
                const uint4 *bp = reinterpret_cast<const uint4 *>(bm) + (size_t)(EV32(boff) + li) * 5u;
                const uint4 q0 = bp[0], q1 = bp[1], q3 = bp[3], q4 = bp[4];
                uint64_t myD = rD ^ (((uint64_t)q1.y << 32) | q1.x);
                uint64_t myS = rS ^ (((uint64_t)q1.w << 32) | q1.z);
                const uint32_t my_nend = q3.x;
                const uint32_t nlast = (uint32_t)__builtin_amdgcn_readlane((int)my_nend, (int)(m - 1u));
                while (true) {
                    while (next_hit < nlast) {
                        const uint32_t s = next_hit;
                        uint64_t dD, dS;
                        (void)take_hit(dD, dS);  // the compiler keeps record flips out of runs
                        if (s < my_nend) {
                            myD ^= dD;
                            myS ^= dS;
                        }
                    }
                    if (nlast <= nz_drawn || nz_drawn >= n_slots) break;
                    if (GAPS) draw_gap(); else draw_chunk();
                }
                const uint64_t beta = ((uint64_t)q0.y << 32) | q0.x, gamma = ((uint64_t)q0.w << 32) | q0.z;
                const uint32_t info = q3.y;
                const uint32_t bit =
                    ((info & BM_CSIGN) ? 1u : 0u) ^ par64(myD & beta) ^ par64(myS & gamma) ^ par64(gamma & a);
                // folded checks read record bits from before the run, plus their own
                uint32_t chk = 0;
                // (the lane shuffle runs on every lane: a source lane must be active)
                const uint32_t rlane = (uint32_t)__shfl((int)rrv, (int)(q3.z & 63u), 64);
                if (info & BM_CHECK) {
                    const uint32_t w = q3.z;
                    const uint32_t rw = w < kRecSgpr ? rlane : rec[w];
                    chk = ((info & BM_EXPECT) ? 1u : 0u) ^ par32(rw & q3.w) ^ ((info & BM_OWN) ? bit : 0u);
                }
                const uint64_t fails = __ballot(lane < m && chk != 0u);
                const uint32_t L = fails ? (uint32_t)__builtin_ctzll(fails) : m - 1u;  // last member executed
                const uint64_t upto = L >= 63u ? ~0ull : ((2ull << L) - 1ull);
                const uint32_t rl = uni(q4.z), rc = rl >> 8;
                if (rc) {
                    const uint32_t rl0 = rl & 255u, r0 = uni(q4.y);
                    uint64_t bits = (__ballot((info & BM_RECORD) != 0u && bit != 0u) & upto) >> rl0;
                    if (rc < 64u) bits &= (1ull << rc) - 1ull;
                    if (bits) {
                        const uint32_t w = r0 >> 5, sh = r0 & 31u;
                        const uint32_t lo = (uint32_t)bits, hi = (uint32_t)(bits >> 32);
                        const uint32_t t0 = lo << sh;
                        const uint32_t t1 = sh ? (hi << sh) | (lo >> (32u - sh)) : hi;
                        const uint32_t t2 = sh ? hi >> (32u - sh) : 0u;
                        if (t0) rec_toggle(w, t0);
                        if (t1) rec_toggle(w + 1u, t1);
                        if (t2) rec_toggle(w + 2u, t2);
                    }
                }
                // signs after member L: its own view, plus the resets that fired
                uint64_t rsl = __ballot((info & BM_RESET) != 0u && bit != 0u) & upto;
                rD = lane64(myD, L);
                rS = lane64(myS, L);
                if (rsl) {
                    const uint4 q2 = bp[2];
                    const uint64_t xD = ((uint64_t)q2.y << 32) | q2.x, xS = ((uint64_t)q2.w << 32) | q2.z;
                    while (rsl) {
                        const uint32_t l = (uint32_t)__builtin_ctzll(rsl);
                        rsl &= rsl - 1ull;
                        rD ^= lane64(xD, l);
                        rS ^= lane64(xS, l);
                    }
                }
                if (fails) {
                    status = ST_DISCARDED;
                    abort_src = (uint32_t)__builtin_amdgcn_readlane((int)q4.x, (int)L);
                    term = e + L;
                    after = 1;
                    e += L;  // the last event run
                    break;
                }
                e += m - 1u;
                evx = evl[(uint64_t)(e + 1u) * 64u + lane];
                evy = evl[(uint64_t)(e + 2u) * 64u + lane];
            } else if (kind <= EV_M_MERGE) {
                // ---- measurement ----
                // The uniform is drawn only when the outcome is random.  Philox
                // words of stream 1 come 256 at a time, one block per lane,
                // and are picked out with one readlane.
                double u = 0.0;
                if (kind != EV_M_DET) {
                    const uint32_t ms = EV32(mslot);
                    uint32_t mw;
                    if (EXPL) {
                        mw = wrow[vdp->n_noise + ms];
                    } else {
                        if (ms < m_base || ms - m_base >= 256u) {
                            m_base = ms & ~255u;
                            philox10((m_base >> 2) + lane, s_lo, s_hi, 1u, key0, key1, mw0, mw1, mw2, mw3);
                        }
                        const uint32_t q = ms & 3u;
                        const uint32_t pick = q == 0u ? mw0 : q == 1u ? mw1 : q == 2u ? mw2 : mw3;
                        mw = (uint32_t)__builtin_amdgcn_readlane((int)pick, (int)((ms - m_base) >> 2));
                    }
                    mw = uni(mw);
                    u = ((double)mw + 0.5) * (1.0 / 4294967296.0);
                }
                uint32_t bit = 0;
                if (kind == EV_M_DET) {
                    bit = (EV32(cexp) == 2u ? 1u : 0u) ^ sga;
                } else if (kind == EV_M_CUT) {
                    const uint32_t sig = (EV32(cexp) == 2u ? 1u : 0u) ^ sga;
                    const uint32_t cnt = 1u << k;
                    double n0 = 0.0, n1 = 0.0;
                    lane_pass(cnt, lane, [&](uint32_t j) {
                        const double q = nrm<R>(v[j]);
                        if (par32(g & j)) n1 += q;
                        else n0 += q;
                    });
                    n0 = wave_sum(n0);
                    n1 = wave_sum(n1);
                    const double Np = sig ? n1 : n0, Nm = sig ? n0 : n1;
                    const double p0 = Np / (Np + Nm);
                    bit = u < p0 ? 0u : 1u;
                    const uint32_t bsel = sig ^ bit;
                    const double Ns = bsel ? n1 : n0;
                    if (!(Ns > 1e-300)) {
                        status = ST_NUMERIC;
                        abort_src = EV32(src);
                        term = e;
                        break;
                    }
                    const R s = (R)(1.0 / sqrt(Ns));
                    const uint32_t ts = EV32(tstar), half = cnt >> 1;
                    const C z = mk<C>(0.0, 0.0);
                    double nn = 0.0;
                    lane_pass(half, lane, [&](uint32_t jp) {
                        uint32_t j = ins0(jp, ts);
                        if (par32(g & j) != bsel) j |= 1u << ts;
                        C x = scale(v[j], s);
                        const double q = nrm<R>(x);
                        const bool keep = q >= tau2;
                        if (!keep) x = z;
                        nn += keep ? q : 0.0;
                        v[jp] = x;
                    });
                    nrm2 = wave_sum(nn);
                    itscale2 = 1.0;
                    --k;
                    if (bsel) a ^= EV64(avec);
                } else if (kind == EV_M_SPLIT) {
                    bit = u < 0.5 ? 0u : 1u;
                    const uint32_t ap = (uint32_t)(a >> EV32(pbit)) & 1u;
                    const uint32_t fs = bit ^ sga ^ EV32(gbeta);
                    const uint32_t q0 = (4u - EV32(cexp)) & 3u;
                    const uint32_t cnt = 1u << k, pm = EV32(pm);
                    const R s = (R)(1.0 / sqrt(itscale2 * nrm2));
                    const C z = mk<C>(0.0, 0.0);
                    double nn = 0.0;
                    lane_pass(cnt, lane, [&](uint32_t j) {
                        C x = v[j];
                        if (ap ^ par32(pm & j)) x = rot(x, q0 + 2u * (fs ^ par32(g & j)));
                        x = scale(x, s);
                        const double q = nrm<R>(x);
                        const bool keep = q >= tau2;
                        if (!keep) x = z;
                        nn += keep ? q : 0.0;
                        v[j] = x;
                    });
                    nrm2 = wave_sum(nn);
                    itscale2 = 1.0;
                } else {  // EV_M_MERGE
                    const uint32_t ap = (uint32_t)(a >> EV32(pbit)) & 1u;
                    const uint32_t q0 = (4u - EV32(cexp)) & 3u;
                    const uint32_t npairs = 1u << (k - 1u), mu = EV32(mu), h = EV32(tstar), pm = EV32(pm);
                    const uint32_t fs0 = sga;
                    double np = 0.0, nm = 0.0;
                    lane_pass(npairs, lane, [&](uint32_t p) {
                        const uint32_t j0 = ins0(p, h), j1 = j0 ^ mu;
                        const uint32_t a0 = ap ^ par32(pm & j0);
                        const uint32_t x = a0 ? j1 : j0, y = a0 ? j0 : j1;
                        const C vx = v[x];
                        const C fy = rot(v[y], q0 + 2u * (fs0 ^ par32(g & x)));
                        const double px = (double)vx.x + (double)fy.x, py = (double)vx.y + (double)fy.y;
                        const double mx = (double)vx.x - (double)fy.x, my = (double)vx.y - (double)fy.y;
                        np += px * px + py * py;
                        nm += mx * mx + my * my;
                    });
                    np = 0.5 * wave_sum(np);
                    nm = 0.5 * wave_sum(nm);
                    const double p0 = np / (np + nm);
                    bit = u < p0 ? 0u : 1u;
                    const double Ns = bit ? nm : np;
                    if (!(Ns > 1e-300)) {
                        status = ST_NUMERIC;
                        abort_src = EV32(src);
                        term = e;
                        break;
                    }
                    const R s = (R)(1.0 / sqrt(2.0 * Ns));
                    const C z = mk<C>(0.0, 0.0);
                    double nn = 0.0;
                    lane_pass(npairs, lane, [&](uint32_t p) {
                        const uint32_t j0 = ins0(p, h), j1 = j0 ^ mu;
                        const uint32_t a0 = ap ^ par32(pm & j0);
                        const uint32_t x = a0 ? j1 : j0, y = a0 ? j0 : j1;
                        const C vx = v[x];
                        const C fy = rot(v[y], q0 + 2u * (fs0 ^ par32(g & x)));
                        C o;
                        if (bit) { o.x = vx.x - fy.x; o.y = vx.y - fy.y; }
                        else { o.x = vx.x + fy.x; o.y = vx.y + fy.y; }
                        o = scale(o, s);
                        const double q = nrm<R>(o);
                        const bool keep = q >= tau2;
                        if (!keep) o = z;
                        nn += keep ? q : 0.0;
                        v[p] = o;
                    });
                    nrm2 = wave_sum(nn);
                    itscale2 = 1.0;
                    --k;
                }
                if (kind == EV_M_SPLIT || kind == EV_M_MERGE) {
                    // rows anticommuting with P absorb s_p; d_p <- s_p; s_p <- (-1)^bit P
                    const uint32_t p = EV32(pbit);
                    const uint64_t bsp = (rS >> p) & 1ull;
                    rD ^= (bsp ? EV64(AD) : 0ull) ^ EV64(PhD);
                    rS ^= (bsp ? EV64(AS) : 0ull) ^ EV64(PhS);
                    rD = (rD & ~(1ull << p)) | (bsp << p);
                    rS = (rS & ~(1ull << p)) | ((uint64_t)(bit ^ EV32(psign)) << p);
                    if ((a >> p) & 1ull) a ^= EV64(beta);
                }
                if ((flags & EVF_RECORD) && bit) rec_toggle(EV32(rec) >> 5, 1u << (EV32(rec) & 31u));
                if ((flags & EVF_RESET) && bit) {
                    rD ^= EV64(xD);
                    rS ^= EV64(xS);
                }
                if (flags & EVF_CHECK) {  // a detector folded into this event
                    if (parity_check()) {
                        status = ST_DISCARDED;
                        abort_src = EV32(chk_src);
                        term = e;
                        after = 1;
                        break;
                    }
                }
            } else if (kind == EV_DROP) {
                // ---- speculative span truncation: coordinates >= k0 must be empty ----
                // every lane ORs the value bits of its entries at or above 2^k0
                // (the shift drops the sign: -0 is empty too), one ballot
                const uint32_t k0 = EV32(mu), cnt = 1u << k, lo = 1u << k0;
                uint32_t live = 0;
                uint32_t b = lo & ~63u;  // 64-entry blocks; the first may start below lo
                if (b < lo) {
                    const uint32_t j = b + lane;
                    live = (j >= lo && j < cnt) ? nonzero_bits(v[j < cnt ? j : 0u]) : 0u;
                    b += 64u;
                }
                if (b < cnt) {  // whole blocks, four reads before they are combined
                    const uint32_t nb = (cnt - b) >> 6;
                    uint32_t i = 0;
                    if (TM == TM_SPLIT) {
                        for (; i + 4u <= nb; i += 4u) {
                            const uint32_t u = b + 64u * i;
                            const C x0 = *v.at_u(u, lane), x1 = *v.at_u(u + 64u, lane), x2 = *v.at_u(u + 128u, lane),
                                    x3 = *v.at_u(u + 192u, lane);
                            live |= nonzero_bits(x0) | nonzero_bits(x1) | nonzero_bits(x2) | nonzero_bits(x3);
                        }
                        for (; i < nb; ++i) live |= nonzero_bits(*v.at_u(b + 64u * i, lane));
                    } else {
                        const C *pb = v.lo + b + lane;
                        for (; i + 4u <= nb; i += 4u) {
                            const C x0 = pb[64u * i], x1 = pb[64u * i + 64u], x2 = pb[64u * i + 128u], x3 = pb[64u * i + 192u];
                            live |= nonzero_bits(x0) | nonzero_bits(x1) | nonzero_bits(x2) | nonzero_bits(x3);
                        }
                        for (; i < nb; ++i) live |= nonzero_bits(pb[64u * i]);
                    }
                }
                if (__ballot(live != 0u) != 0ull) {
                    restart = true;
                    break;
                }
                k = k0;
                if (k0 == 0u) renorm_single();
            } else if (kind == EV_DIAG) {
                // ---- diagonal gate: all its Z-strings in one pass ----
                // Term g moves entry j to j ^ mu_g with weight W_g (-1)^(gm_g . j).
                // The shifts span 2^r coset elements E_u; lane L of the pass
                // takes element u = L mod 2^r of coset L >> r and sums its terms
                // from the coset's entries (0 past the old span).  A coset sits on
                // the lanes of one iteration, whose reads all come before its
                // writes, so the update is in place.
                const DiagInfo *di = P.diag + EV32(boff);
                const uint32_t ng = uni(di->ng), r = uni(di->r), knew = uni(di->knew), lead = uni(di->lead);
                if ((flags & EVF_COND) && !cond_check(flags)) {
                    // a classically controlled gate that does not fire: the
                    // span still grows, with zeros at the new coordinates
                    const uint32_t kin = 1u << k, kout = 1u << knew;
#pragma unroll 1
                    for (uint32_t b = kin; b < kout; b += 64u)
                        if (b + lane < kout) v[b + lane] = mk<C>(0.0, 0.0);
                    k = knew;
                } else {
                    uint32_t sgl = 0;  // sign part of term `lane`, with gamma . a
                    if (lane < ng) sgl = par64((rD & di->beta[lane]) ^ ((rS ^ a) & di->gamma[lane]));
                    const uint32_t S = (uint32_t)__ballot(sgl != 0u);
                    const uint32_t e0 = uni(di->E[1]), e1 = uni(di->E[2]), e2 = uni(di->E[4]);
                    auto coset_el = [&](uint32_t w) { return ((w & 1u) ? e0 : 0u) ^ ((w & 2u) ? e1 : 0u) ^ ((w & 4u) ? e2 : 0u); };
                    // the gate is unitary: the carried norm sets the pruning level
                    const R thr = (R)(tau2 * nrm2 * itscale2);
                    const uint32_t kin = 1u << k, um = (1u << r) - 1u;
                    uint32_t cnt = 0;
                    lane_pass(1u << knew, lane, [&](uint32_t L) {
                        const uint32_t u = L & um;
                        uint32_t j0 = L >> r;  // zeros at the lead bits, ascending
                        for (uint32_t i = 0; i < r; ++i) j0 = ins0(j0, (lead >> (5u * i)) & 31u);
                        C y = mk<C>(0.0, 0.0);
                        for (uint32_t g = 0; g < ng; ++g) {
                            const uint32_t jin = j0 ^ coset_el(u ^ uni(di->ug[g]));
                            C xv = v[jin < kin ? jin : 0u];
                            if (jin >= kin) xv = mk<C>(0.0, 0.0);
                            const R wr = sizeof(R) == 4 ? (R)unif(di->fre[g]) : (R)unid(di->dre[g]);
                            const R wi = sizeof(R) == 4 ? (R)unif(di->fim[g]) : (R)unid(di->dim[g]);
                            const bool neg = (((S >> g) ^ par32(uni(di->gm[g]) & jin)) & 1u) != 0u;
                            const R cr = neg ? -wr : wr, ci = neg ? -wi : wi;
                            y.x = fma(cr, xv.x, fma(-ci, xv.y, y.x));
                            y.y = fma(cr, xv.y, fma(ci, xv.x, y.y));
                        }
                        bool keep;
                        const C o = t_keep<R, C>(y, thr, keep);
                        cnt += (uint32_t)__popcll(__ballot(keep));
                        v[j0 ^ coset_el(u)] = o;
                    });
                    k = knew;
                    cnt = uni(cnt);
                    maxsup = max(maxsup, cnt);
                    if (cnt > (LEAN ? 0xFFFFFFFFu : P.support_cap)) {
                        if (!full) {  // the full list decides where the cap is hit
                            restart = true;
                            break;
                        }
                        status = ST_OVERFLOW;
                        abort_src = EV32(src);
                        term = e;
                        after = 1;
                        break;
                    }
                }
            } else if (kind == EV_NOP) {
                // a deferred T run, skipped
            } else if (kind == EV_FEEDBACK) {
                // ---- classically controlled Pauli: its record bits read as a check ----
                if (cond_check(flags)) {
                    rD ^= EV64(xD);
                    rS ^= EV64(xS);
                }
            } else {
                // ---- DETECTOR / OBSERVABLE ----
                const uint32_t pbits = parity_check();
                if (kind == EV_DETECTOR) {
                    if (pbits) {
                        status = ST_DISCARDED;
                        abort_src = EV32(src);
                        term = e;
                        break;
                    }
                } else {
                    obs |= pbits << EV32(rec);
                }
            }
            tile_sync();
            evc = evx;
            evx = evy;
        }
        tile_sync();
        {
            // work of this attempt: the list's running sums at the event after
            // the last one run, and the noise words drawn
            // (less the running sums at e0 when the shot started from a
            // shared prefix: the work the kernel ran)
            const Event *nx = reinterpret_cast<const Event *>(evl) + e + 1u;
            const Event *n0 = reinterpret_cast<const Event *>(evl) + e0;
            const uint64_t wt = uni64(nx->cum_t) - uni64(n0->cum_t), wm = uni64(nx->cum_m) - uni64(n0->cum_m);
            const uint32_t we = uni(nx->cum_e) - uni(n0->cum_e);
            const uint32_t wn = GAPS ? ((gd + 255u) & ~255u) : min(nz_drawn, vdp->n_noise);
            myc += lane == (uint32_t)C_ENTRIES_T ? wt : lane == (uint32_t)C_ENTRIES_M ? wm
                 : lane == (uint32_t)C_EVENTS ? (uint64_t)we : lane == (uint32_t)C_NOISE ? (uint64_t)wn : 0ull;
        }
        // a kept shot whose last deferred run was never applied: its final
        // state needs it, so the attempt runs again without deferring
        if (!LEAN && !restart && deferred && P.keep_n && shot >= P.keep_lo && shot - P.keep_lo < P.keep_n) {
            restart = true;
            redo = true;
        }
        if (!restart || (!LEAN && P.prefix_build)) break;
        if (redo) {  // the same list again, every T run applied
            redo = false;
            defer_ok = false;
            myc += lane == (uint32_t)C_REDO ? 1u : 0u;
        } else {
            full = true;
            myc += lane == (uint32_t)C_RESTARTS ? 1u : 0u;
        }
        }
        if ((!LEAN && P.prefix_build)) {
            // a list that ended (or stopped) before a checkpoint leaves its slot invalid
            if (!pfx_done && lane == 0) {
                const uint32_t o = full ? vdp->ck_off_full : vdp->ck_off, cnt = full ? vdp->ck_cnt_full : vdp->ck_cnt;
                for (uint32_t t = ck_next_done; t < cnt; ++t)
                    reinterpret_cast<CkptState *>(P.prefix + (size_t)(o + t) * P.prefix_stride)->valid = 0u;
            }
            ++group_pos;
            continue;
        }

        // ---- shot end: norm check, outputs, kept states, counters ----
        // (a shot that ended on a checkpoint's tile without loading it: the
        // sum stored with it, computed the same way)
        const bool kept = !LEAN && P.keep_n && shot >= P.keep_lo && shot - P.keep_lo < P.keep_n;
        if (lazy_slot != nullptr && kept) materialize();
        const double nn = lazy_slot != nullptr ? unid(reinterpret_cast<const CkptState *>(lazy_slot)->tnorm)
                                               : tile_norm(v, k, lane);
        maxdev = fmax(maxdev, fabs(nn / itscale2 - 1.0));
        {
            // one store for the record words held in scalar registers and the
            // three per-shot words; record words in LDS follow
            const uint32_t val = lane < kRecSgpr ? rrv : lane == kRecSgpr ? status
                               : lane == kRecSgpr + 1u ? abort_src : obs;
            if (out_plane) out_plane[i] = val;
        }
        if (P.outcomes)
            for (uint32_t w = kRecSgpr + lane; w < P.rec_words; w += 64u) P.outcomes[(uint64_t)w * P.n_shots + i] = rec[w];
        ++group_pos;
        if (kept) {
            const uint64_t kk = shot - P.keep_lo;
            dump_state(P.keep_meta + kk * KM_COUNT, P.keep_v + kk * (uint64_t)P.tile_entries * 2u, v, lane,
                       P.tile_entries, status, abort_src, term, after, rD, rS, a, k, nrm2, P.phase_tab, phase8, var, full ? 1u : 0u, 1.0 / itscale2);
        }
        if (term < trace_lim)
            dump_state(P.trace_meta + (uint64_t)term * KM_COUNT, P.trace_v + (uint64_t)term * P.tile_entries * 2u, v,
                       lane, P.tile_entries, status, abort_src, term, after, rD, rS, a, k, nrm2, P.phase_tab, phase8, var, full ? 1u : 0u, 1.0 / itscale2);
        const uint32_t bucket = min(15u, 31u - (uint32_t)__clz(maxsup));
        myc += (lane == C_SHOTS) + (lane == C_PASSED + status) +
               (lane == C_LOGICAL && status == ST_PASSED && obs != 0u) + (lane == C_HIST0 + bucket);
    }
    if (var_ok) flush_counters();
}

// An FP32 tile of a 2^10 span takes 8 KiB of LDS, so LDS holds 5 waves per
// SIMD; the register budget is set to match.  What no longer fits in
// registers is what lives across a whole shot (group outputs, shot
// constants), never the event loop's working set.  FP64 asks for 5 waves per
// SIMD as well (96 VGPRs, more spilled): left to itself the compiler takes
// 154 VGPRs and 3 waves.  On the 42-qubit workload 4 waves (128 VGPRs) were
// 15% faster than 3, and once the lean kernels had freed registers 5 waves
// were 2.4% faster than 4 (141.3 against 137.9 M shots/s).
template <uint32_t NS, uint32_t TM, bool LEAN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8)))
k_sample_f32(const Event *__restrict__ ev, const NoiseLoc *__restrict__ nz, const uint32_t *__restrict__ tm1,
             const uint32_t *__restrict__ det, const uint32_t *__restrict__ words, const BatchMember *__restrict__ bm,
             RunParams P) {
    sample_shots<float, NS, TM, LEAN>(ev, nz, tm1, det, words, bm, P);
}

template <uint32_t NS, uint32_t TM, bool LEAN>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8)))
k_sample_f64(const Event *__restrict__ ev, const NoiseLoc *__restrict__ nz, const uint32_t *__restrict__ tm1,
             const uint32_t *__restrict__ det, const uint32_t *__restrict__ words, const BatchMember *__restrict__ bm,
             RunParams P) {
    sample_shots<double, NS, TM, LEAN>(ev, nz, tm1, det, words, bm, P);
}

// The shared-prefix build (RunParams::prefix_build): the same per-shot code
// with the same register budget, under its own name so that profiles show it
// apart from the sampler.  It draws no noise, so one noise source serves.
template <uint32_t TM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5, 8)))
k_prefix_f32(const Event *__restrict__ ev, const NoiseLoc *__restrict__ nz, const uint32_t *__restrict__ tm1,
             const uint32_t *__restrict__ det, const uint32_t *__restrict__ words, const BatchMember *__restrict__ bm,
             RunParams P) {
    sample_shots<float, NS_SLOTS, TM>(ev, nz, tm1, det, words, bm, P);
}

template <uint32_t TM>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4, 8)))
k_prefix_f64(const Event *__restrict__ ev, const NoiseLoc *__restrict__ nz, const uint32_t *__restrict__ tm1,
             const uint32_t *__restrict__ det, const uint32_t *__restrict__ words, const BatchMember *__restrict__ bm,
             RunParams P) {
    sample_shots<double, NS_SLOTS, TM>(ev, nz, tm1, det, words, bm, P);
}

__global__ void k_reset(unsigned long long *counters, uint32_t n, unsigned long long *next) {
    for (uint32_t t = threadIdx.x; t < n; t += blockDim.x) counters[t] = 0ull;
    if (threadIdx.x < 2u) next[threadIdx.x] = 0ull;  // the sampler's and the prefix build's cursors
}

template <typename R, uint32_t NS, uint32_t TM, bool LEAN> const void *kernel_ptr() {
    if (sizeof(R) == 4) return (const void *)k_sample_f32<NS, TM, LEAN>;
    return (const void *)k_sample_f64<NS, TM, LEAN>;
}

// The 18 full instantiations, indexed by fp64 * 9 + source * 3 + tile mode,
// then 12 lean ones (per-slot and gap-sampled noise), indexed by
// 18 + fp64 * 6 + (source == gaps) * 3 + tile mode.
constexpr int kKernels = 30;
template <typename R, uint32_t NS, bool LEAN> void kernels_of(const void **out) {
    out[TM_LDS] = kernel_ptr<R, NS, TM_LDS, LEAN>();
    out[TM_MEM] = kernel_ptr<R, NS, TM_MEM, LEAN>();
    out[TM_SPLIT] = kernel_ptr<R, NS, TM_SPLIT, LEAN>();
}
void all_kernels(const void **ks) {
    kernels_of<float, NS_SLOTS, false>(ks + 0);
    kernels_of<float, NS_EXPLICIT, false>(ks + 3);
    kernels_of<float, NS_GAPS, false>(ks + 6);
    kernels_of<double, NS_SLOTS, false>(ks + 9);
    kernels_of<double, NS_EXPLICIT, false>(ks + 12);
    kernels_of<double, NS_GAPS, false>(ks + 15);
    kernels_of<float, NS_SLOTS, true>(ks + 18);
    kernels_of<float, NS_GAPS, true>(ks + 21);
    kernels_of<double, NS_SLOTS, true>(ks + 24);
    kernels_of<double, NS_GAPS, true>(ks + 27);
}
int kernel_index(bool fp64, uint32_t ns, uint32_t tm, bool lean) {
    if (lean && ns != NS_EXPLICIT) return 18 + (fp64 ? 6 : 0) + (ns == NS_GAPS ? 3 : 0) + (int)tm;
    return (fp64 ? 9 : 0) + 3 * (int)ns + (int)tm;
}
}  // namespace

// The lean kernels run launches with no kept states, no trace, no support
// cap and no shot list (never the prefix build, which has its own kernels).
// With the build's code out as well, the FP32 LDS kernel spilled 90 SGPRs
// instead of 245: measured +11% FP32 and +14% FP64 on the 42-qubit workload,
// +11% on span-12 split tiles; leaving out the cap and the shot list then
// added 1-2%.
bool sampler_lean(const RunParams &p) {
    return p.keep_n == 0u && p.trace_n == 0u && p.words == nullptr && p.support_cap == 0xFFFFFFFFu &&
           p.shot_list == nullptr;
}

hipError_t launch_reset(unsigned long long *counters, uint32_t n, unsigned long long *next, hipStream_t stream) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(256), 0, stream, counters, n, next);
    return hipGetLastError();
}

hipError_t launch_sampler(const RunParams &p, bool fp64, dim3 grid, dim3 block, size_t lds, hipStream_t stream) {
    const uint32_t ns = p.words != nullptr ? NS_EXPLICIT : (p.noise_mode == 1u ? NS_GAPS : NS_SLOTS);
    void *args[7] = {(void *)&p.ev, (void *)&p.nz, (void *)&p.tm1, (void *)&p.det, (void *)&p.words, (void *)&p.bm,
                     (void *)&p};
    return hipLaunchKernel(sampler_kernel(fp64, ns, p.tile_mode, sampler_lean(p)), grid, block, args, lds, stream);
}

const void *sampler_kernel(bool fp64, uint32_t ns, uint32_t tm, bool lean) {
    const void *ks[kKernels];
    all_kernels(ks);
    return ks[kernel_index(fp64, ns, tm > TM_SPLIT ? TM_LDS : tm, lean)];
}

const void *reset_kernel() { return (const void *)k_reset; }

const void *prefix_kernel(bool fp64, uint32_t tm) {
    const void *ks[6] = {(const void *)k_prefix_f32<TM_LDS>, (const void *)k_prefix_f32<TM_MEM>,
                         (const void *)k_prefix_f32<TM_SPLIT>, (const void *)k_prefix_f64<TM_LDS>,
                         (const void *)k_prefix_f64<TM_MEM>, (const void *)k_prefix_f64<TM_SPLIT>};
    return ks[(fp64 ? 3 : 0) + (tm > TM_SPLIT ? TM_LDS : tm)];
}

hipError_t launch_prefix_build(const RunParams &p, bool fp64, dim3 grid, dim3 block, size_t lds, hipStream_t stream) {
    void *args[7] = {(void *)&p.ev, (void *)&p.nz, (void *)&p.tm1, (void *)&p.det, (void *)&p.words, (void *)&p.bm,
                     (void *)&p};
    return hipLaunchKernel(prefix_kernel(fp64, p.tile_mode), grid, block, args, lds, stream);
}

hipError_t sampler_occupancy(bool fp64, uint32_t ns, uint32_t tm, int block, size_t lds, int *blocks_per_cu) {
    const void *ks[kKernels];
    all_kernels(ks);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, ks[kernel_index(fp64, ns, tm, false)], block, lds);
}

hipError_t sampler_set_lds_limit(int bytes) {
    const void *ks[kKernels];
    all_kernels(ks);
    for (const void *k : ks) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    for (int i = 0; i < 6; ++i) {
        hipError_t e = hipFuncSetAttribute(prefix_kernel(i >= 3, (uint32_t)(i % 3)),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t scratch_address(int device, unsigned char **out) {
    constexpr int kMaxDevices = 64;
    static std::mutex mu;
    static unsigned char *addr[kMaxDevices] = {};
    if (!out || device < 0 || device >= kMaxDevices) return hipErrorInvalidValue;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = static_cast<unsigned char *>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

}  // namespace soft
