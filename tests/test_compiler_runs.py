"""Host-side checks of the speculative list's fused runs (no GPU): the circuit
compiler is built with g++ into a small driver that prints the events.

- A run of doublings (EVF_TRUN) stores, per final entry J, the fixed quarter
  turns of its weight.  Applying the members one after the other (each new
  entry j + 2^k gets tan(pi/8) i^qb (-1)^(sig ^ parity(g & j)) times entry j,
  Eq. 4 on a new coordinate) must give the same vector as the one-pass form
  the kernel uses: entry J mod 2^k0 times tan(pi/8)^(new bits of J) times
  i^(r_J + 2 parity(sigs & new bits)).
- Runs of dropping butterflies (EVF_BRUN) and of doublings hold only members
  that nothing separates (same noise slots, no Clifford sign flips), span
  dimensions that step by one, tiles of at most 64 entries, and the summed
  global-phase step.
- A butterfly pair (EVF_PAIR) joins a plain butterfly and the next butterfly
  that nothing separates, on a span of 2^8 or more; its two left-out bits
  make the quads {j, j^mu, j^mu', j^mu^mu'} tile the span, and the quad pass
  (both butterflies on each quad, the second's partner weights from parities
  over j plus constants) equals the two butterflies applied one after the
  other to the whole vector.
"""
from __future__ import annotations

import os
import subprocess

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_23037_amd", "csrc")

EV_T_DOUBLE, EV_T_BFLY = 1, 2
EVF_TDG, EVF_CLIFF, EVF_DROP1, EVF_TRUN, EVF_BRUN = 1, 32, 64, 128, 256

DRIVER = r"""
#include "compile.h"
#include <cstdio>
#include <fstream>
#include <sstream>
using namespace soft;
int main(int argc, char **argv) {
    std::ifstream f(argv[1]);
    std::stringstream ss;
    ss << f.rdbuf();
    NoiseModel nm;
    nm.p1 = nm.p2 = nm.p_idle = nm.p_meas = nm.p_reset = nm.p_mpp = 1e-3;
    Program P;
    compile_circuit(ss.str(), nm, P, true);
    for (const Event &E : P.events)
        std::printf("%u %u %u %u %u %u %u %u %u %u %llu %llu %u\n", E.kind, E.k, E.flags, E.bcnt, E.boff, E.qb, E.g,
                    E.mu, E.tstar, E.noise_end, (unsigned long long)E.trot0, (unsigned long long)E.trot1, E.pbit);
    return 0;
}
"""

FIELDS = ("kind", "k", "flags", "bcnt", "boff", "qb", "g", "mu", "tstar", "noise_end", "trot0", "trot1", "pbit")
EVF_MAT, EVF_DEFER, EVF_PAIR = 2048, 4096, 8192


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("compiler_runs")
    src = d / "dump.cpp"
    src.write_text(DRIVER)
    exe = d / "dump"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, "-I", os.path.join(ROOT, "include"), str(src),
                    os.path.join(CSRC, "compile.cpp"), "-o", str(exe)], check=True)
    return d, exe


def events(driver, text):
    d, exe = driver
    path = d / "circuit.txt"
    path.write_text(text)
    out = subprocess.run([str(exe), str(path)], capture_output=True, text=True, check=True).stdout
    return [dict(zip(FIELDS, (int(x) for x in line.split()))) for line in out.splitlines()]


def circuits():
    yield "cultivation_42q", workloads.config("cultivation_42q", seed=1).text
    yield "cultivation_42q_k12", workloads.config("cultivation_42q_k12", seed=1).text
    shapes = [(7, 8, 3, [7, 4], 4), (9, 6, 3, [9, 5], 6), (8, 6, 2, [8], 6), (10, 6, 3, [10, 6, 3], 6)]
    for seed, (nd, na, rz, br, w) in enumerate(shapes):
        yield "bracket%d" % seed, workloads.cultivation_shaped(100 + seed, nd, na, rz, br, check_weight=w,
                                                               inverse_order="shuffled").text


def parity(x):
    return bin(x).count("1") & 1


def phase_step(members):
    return sum(15 if m["flags"] & EVF_TDG else 1 for m in members) & 15


def check_common(ev, i, m):
    head, members = ev[i], ev[i:i + m]
    assert m >= 2
    assert all(x["noise_end"] == head["noise_end"] for x in members)
    for x in members[1:]:
        assert not (x["flags"] & (EVF_CLIFF | EVF_TRUN | EVF_BRUN))
    assert head["boff"] == phase_step(members)
    return members


@pytest.mark.parametrize("name,text", list(circuits()), ids=[n for n, _ in circuits()])
def test_doubling_runs_match_separate_doublings(driver, name, text):
    ev = events(driver, text)
    rng = np.random.default_rng(7)
    tn = np.tan(np.pi / 8)
    runs = 0
    for i, head in enumerate(ev):
        if not head["flags"] & EVF_TRUN:
            continue
        runs += 1
        m, k0 = head["bcnt"], head["k"]
        members = check_common(ev, i, m)
        assert all(x["kind"] == EV_T_DOUBLE and x["k"] == k0 + t for t, x in enumerate(members))
        K = k0 + m
        assert K <= 6
        v0 = rng.normal(size=1 << k0) + 1j * rng.normal(size=1 << k0)
        for _ in range(4):
            sig = [int(b) for b in rng.integers(0, 2, size=m)]
            seq = np.zeros(1 << K, dtype=complex)
            seq[:1 << k0] = v0
            for t, x in enumerate(members):
                kk = k0 + t
                for j in range(1 << kk):
                    s = sig[t] ^ parity(x["g"] & j)
                    seq[j + (1 << kk)] = tn * (1j ** x["qb"]) * (-1) ** s * seq[j]
            sm = sum(b << t for t, b in enumerate(sig))
            fused = np.empty(1 << K, dtype=complex)
            for J in range(1 << K):
                nb = J >> k0
                r = ((head["trot0"] >> J) & 1) + 2 * ((head["trot1"] >> J) & 1) + 2 * parity(sm & nb)
                fused[J] = tn ** bin(nb).count("1") * (1j ** (r % 4)) * v0[J & ((1 << k0) - 1)]
            np.testing.assert_allclose(fused, seq, rtol=0, atol=1e-12)
    if name == "cultivation_42q":
        assert runs >= 4


@pytest.mark.parametrize("name,text", list(circuits()), ids=[n for n, _ in circuits()])
def test_dropping_butterfly_runs_are_well_formed(driver, name, text):
    ev = events(driver, text)
    runs = 0
    for i, head in enumerate(ev):
        if not head["flags"] & EVF_BRUN:
            continue
        runs += 1
        m, k0 = head["bcnt"], head["k"]
        members = check_common(ev, i, m)
        assert k0 <= 6 and m < k0 + 1
        for t, x in enumerate(members):
            assert x["kind"] == EV_T_BFLY and x["flags"] & EVF_DROP1
            assert x["k"] == k0 - t and x["tstar"] == x["k"] - 1
            assert (x["mu"] >> x["tstar"]) == 1  # mu's top bit is the dropped coordinate
    if name == "cultivation_42q":
        assert runs >= 4


def ins0(p, h):
    lo = p & ((1 << h) - 1)
    return ((p ^ lo) << 1) | lo


def bfly(v, mu, g, s, q, tn):
    """One branching T on an existing coordinate, over the whole vector:
    v'_x = v_x + tn i^q (-1)^(s ^ g.(x ^ mu)) v_(x ^ mu)."""
    out = v.copy()
    for x in range(len(v)):
        y = x ^ mu
        out[x] = v[x] + tn * (1j ** q) * (-1) ** (s ^ parity(g & y)) * v[y]
    return out


@pytest.mark.parametrize("name,text", list(circuits()), ids=[n for n, _ in circuits()])
def test_butterfly_pairs_tile_the_span_and_match_two_passes(driver, name, text):
    ev = events(driver, text)
    rng = np.random.default_rng(11)
    tn = np.tan(np.pi / 8)
    pairs = 0
    for i, A in enumerate(ev):
        if not A["flags"] & EVF_PAIR:
            continue
        pairs += 1
        B = ev[i + 1]
        assert A["kind"] == EV_T_BFLY and not A["flags"] & (EVF_DROP1 | EVF_TRUN | EVF_BRUN)
        assert B["kind"] == EV_T_BFLY and not B["flags"] & (EVF_TRUN | EVF_BRUN | EVF_CLIFF | EVF_MAT | EVF_DEFER | EVF_PAIR)
        assert A["noise_end"] == B["noise_end"] and A["k"] == B["k"] >= 8
        k = A["k"]
        plo, phi = A["pbit"] & 255, A["pbit"] >> 8
        assert plo < phi < k
        mu1, mu2 = A["mu"], B["mu"]
        # the quads tile the span
        seen = set()
        for qi in range(1 << (k - 2)):
            j = ins0(ins0(qi, plo), phi)
            seen.update((j, j ^ mu1, j ^ mu2, j ^ mu1 ^ mu2))
        assert seen == set(range(1 << k))
        # the quad pass equals the two butterflies in turn (for both signs)
        v = rng.normal(size=1 << k) + 1j * rng.normal(size=1 << k)
        for s1, s2 in ((0, 0), (1, 0), (0, 1), (1, 1)):
            ref = bfly(bfly(v, mu1, A["g"], s1, A["qb"], tn), mu2, B["g"], s2, B["qb"], tn)
            out = v.copy()
            g1, g2 = A["g"], B["g"]
            a1, b1, a2, b2 = parity(g1 & mu1), parity(g1 & mu2), parity(g2 & mu1), parity(g2 & mu2)
            w1, w2 = tn * 1j ** A["qb"], tn * 1j ** B["qb"]
            sg = lambda t: -1.0 if t else 1.0
            for qi in range(1 << (k - 2)):
                j = ins0(ins0(qi, plo), phi)
                jb, jc = j ^ mu1, j ^ mu2
                jd = jb ^ mu2
                a, b, c, d = out[j], out[jb], out[jc], out[jd]
                t1 = s1 ^ parity(g1 & j)
                a, b, c, d = (a + sg(t1 ^ a1) * w1 * b, b + sg(t1) * w1 * a,
                              c + sg(t1 ^ a1 ^ b1) * w1 * d, d + sg(t1 ^ b1) * w1 * c)
                t2 = s2 ^ parity(g2 & j)
                a, c, b, d = (a + sg(t2 ^ b2) * w2 * c, c + sg(t2) * w2 * a,
                              b + sg(t2 ^ a2 ^ b2) * w2 * d, d + sg(t2 ^ a2) * w2 * b)
                out[j], out[jb], out[jc], out[jd] = a, b, c, d
            np.testing.assert_allclose(out, ref, rtol=0, atol=1e-12)
    # every plain butterfly that could pair with the next one does
    for i in range(len(ev) - 1):
        A, B = ev[i], ev[i + 1]
        if (A["kind"] == EV_T_BFLY == B["kind"] and A["k"] >= 8 and A["noise_end"] == B["noise_end"]
                and not A["flags"] & (EVF_DROP1 | EVF_TRUN | EVF_BRUN)
                and not B["flags"] & (EVF_TRUN | EVF_BRUN | EVF_CLIFF | EVF_MAT | EVF_DEFER)
                and not (i > 0 and ev[i - 1]["flags"] & EVF_PAIR)):
            assert A["flags"] & EVF_PAIR, i
    expect = {"cultivation_42q": 5, "cultivation_42q_k12": 4}
    if name in expect:
        assert pairs == expect[name]
