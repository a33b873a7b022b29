"""Pins of the oracle's classical flip of MPP results (test code, CPU).

The noise model of Sec. III is uniform depolarizing noise; on a Pauli-product
readout it shows as a flip of the recorded bit with probability p_mpp (the
state is the one the unflipped readout leaves).  Two independent checks:

* exact enumeration: every flip pattern and every measurement branch of a
  small circuit is run on a dense statevector, with the flips applied to the
  listed record bits and the detectors evaluated on the flipped bits; the
  oracle's sampled (status, failing detector, record) distribution must match
  it (chi^2), with per-slot draws and with gap sampling;
* a record XOR: with explicit words, the oracle's records equal the records of
  the same circuit without the flip noise, XORed with exactly the flips whose
  words hit, and its detectors fail where the flipped bits say.

A flip on the wrong record, a flip dropped in either draw mode, a flip applied
after a detector that should read it, or a flip that also moves the state
fails one of them.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
from tests import ref_dense


def _enumerate(text, p):
    """Exact distribution of (status, failing detector ordinal or -1, record
    tuple) for `text` where every MPP result is flipped with probability p.
    Records after an abort stay 0, as the oracle leaves them."""
    n, ops = ref_dense.parse(text)
    n_rec = sum(1 for t in ops if t[0] in ("M", "MPP"))
    n_mpp = sum(1 for t in ops if t[0] == "MPP")
    dist = {}
    for flips in itertools.product((0, 1), repeat=n_mpp):
        pf = float(np.prod([p if f else 1.0 - p for f in flips]))
        if pf == 0.0:
            continue
        psi0 = np.zeros(1 << n, dtype=complex)
        psi0[0] = 1.0
        # (state, probability, record, status key)
        states = [(psi0, pf, [0] * n_rec, None)]
        r = 0      # next record index
        k = 0      # next MPP ordinal
        det = 0    # next detector ordinal
        for tok in ops:
            g = tok[0]
            new = []
            for psi, pr, rec, st in states:
                if st is not None:
                    new.append((psi, pr, rec, st))
                    continue
                if g in ref_dense.MATS:
                    psi = ref_dense.apply_1q(psi, ref_dense.MATS[g], int(tok[1]), n)
                    new.append((psi, pr, rec, st))
                elif g == "CX":
                    new.append((ref_dense.apply_cx(psi, int(tok[1]), int(tok[2]), n), pr, rec, st))
                elif g in ("M", "MPP"):
                    x, z = (0, 1 << int(tok[1])) if g == "M" else ref_dense.mpp_pauli(tok[1])
                    P = ref_dense.pauli_apply(psi, x, z, 0, n)
                    for m in (1, -1):
                        proj = 0.5 * (psi + m * P)
                        w = float(np.real(np.vdot(proj, proj)))
                        if w > 1e-15:
                            rr = list(rec)
                            bit = (1 - m) // 2
                            if g == "MPP" and flips[k]:
                                bit ^= 1
                            rr[r] = bit
                            new.append((proj / np.sqrt(w), pr * w, rr, st))
                elif g == "DETECTOR":
                    par = int(tok[1])
                    for q in tok[2:]:
                        par ^= rec[int(q)]
                    new.append((psi, pr, rec, (oracle.DISCARDED, det) if par else None))
                else:
                    raise AssertionError("op not handled here: %s" % g)
            states = new
            if g in ("M", "MPP"):
                r += 1
            if g == "MPP":
                k += 1
            if g == "DETECTOR":
                det += 1
        for _, pr, rec, st in states:
            key = (oracle.PASSED, -1, tuple(rec)) if st is None else (st[0], st[1], tuple(rec))
            dist[key] = dist.get(key, 0.0) + pr
    return dist


# Record 0 is random (X0 X1 on a T-rotated Bell pair), record 1 is fixed at
# +1 and read by a detector (it fails exactly when record 1 was flipped),
# record 2 (Y0 Y1) is random again, record 3 is a plain Z readout (never
# flipped by p_mpp), and the second detector reads records 0 and 3.
FLIP_CIRCUIT = """QUBITS 2
H 0
T 0
CX 0 1
MPP X0*X1
MPP Z0*Z1
DETECTOR 0 1
MPP Y0*Y1
M 0
DETECTOR 0 0 3
"""


def _detector_srcs(text):
    srcs, src = [], 0
    for line in text.splitlines()[1:]:
        if not line.split():
            continue
        if line.startswith("DETECTOR"):
            srcs.append(src)
        src += 1
    return srcs


@pytest.mark.parametrize("mode", [0, 1])
def test_mpp_flip_matches_exact_enumeration(mode):
    p = 0.15
    exact = _enumerate(FLIP_CIRCUIT, p)
    circ = oracle.Circuit(FLIP_CIRCUIT, {"p_mpp": p}, noise_mode=mode)
    assert circ.n_noise_slots == 3  # one flip slot per MPP, none for M
    N = 200000
    res = circ.batch(17 + mode, 0, N)
    dsrc = _detector_srcs(FLIP_CIRCUIT)
    counts = {}
    rec = res["outcomes"][0]
    for st, ab, w in zip(res["status"], res["abort_op"], rec):
        d = -1 if st == oracle.PASSED else dsrc.index(int(ab))
        key = (int(st), d, tuple(int((int(w) >> i) & 1) for i in range(4)))
        counts[key] = counts.get(key, 0) + 1
    assert set(counts) <= set(exact), sorted(set(counts) - set(exact))[:5]
    chi2, dof = 0.0, -1
    for key, pr in exact.items():
        e = pr * N
        chi2 += (counts.get(key, 0) - e) ** 2 / e
        dof += 1
    # P(chi2 > 2 dof + 30) is far below 1e-4 for the dof here (about 20)
    assert chi2 < 2 * dof + 30, (chi2, dof)
    # and the two flip-driven rates directly: detector 0 fails iff record 1
    # was flipped (rate p); the second detector reads a flipped record 0
    d0 = np.mean((res["status"] == oracle.DISCARDED) & (res["abort_op"] == dsrc[0]))
    assert abs(d0 - p) < 5 * np.sqrt(p * (1 - p) / N)


def test_mpp_flip_is_a_record_xor_with_explicit_words():
    # Without detectors in the way, the records with p_mpp > 0 equal the
    # records without it XOR the flips whose words hit; the measurement words
    # are shared, so the states (and later outcomes) must not move.
    rng = np.random.default_rng(5)
    n = 4
    body = []
    n_rec, mpp_recs = 0, []
    for _ in range(40):
        r = rng.random()
        if r < 0.3:
            q = rng.choice(n, size=int(rng.integers(1, n + 1)), replace=False)
            body.append("MPP " + "*".join("%s%d" % ("XYZ"[int(rng.integers(3))], int(x)) for x in sorted(q)))
            mpp_recs.append(n_rec)
            n_rec += 1
        elif r < 0.4:
            body.append("M %d" % int(rng.integers(n)))
            n_rec += 1
        elif r < 0.5:
            body.append("T %d" % int(rng.integers(n)))
        elif r < 0.75:
            body.append("H %d" % int(rng.integers(n)))
        else:
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            body.append("CX %d %d" % (a, b))
    text = "QUBITS %d\n" % n + "\n".join(body) + "\n"
    p = 0.3
    noisy = oracle.Circuit(text, {"p_mpp": p})
    clean = oracle.Circuit(text)
    n_mpp = len(mpp_recs)
    assert noisy.n_noise_slots == n_mpp and clean.n_noise_slots == 0
    thr = int(np.floor(p * 2 ** 32))
    for shot in range(300):
        flip_words = rng.integers(0, 2 ** 32, size=n_mpp, dtype=np.uint64).astype(np.uint32)
        meas_words = rng.integers(0, 2 ** 32, size=noisy.n_meas_slots, dtype=np.uint64).astype(np.uint32)
        a = noisy.shot(0, shot, words=np.concatenate([flip_words, meas_words]))
        b = clean.shot(0, shot, words=meas_words)
        expect = list(b.record)
        for i, r in enumerate(mpp_recs):
            if int(flip_words[i]) < thr:
                expect[r] ^= 1
        assert a.record == expect, shot
        assert (a.tab_x == b.tab_x).all() and (a.tab_z == b.tab_z).all() and (a.tab_r == b.tab_r).all()
        assert set(a.coeffs) == set(b.coeffs)
        assert max(abs(a.coeffs[k] - b.coeffs[k]) for k in a.coeffs) < 1e-13


def test_mpp_flip_reaches_the_detector_that_reads_it():
    # A detector right after a flipped, otherwise deterministic MPP fails
    # exactly when the flip word hits; a detector on an earlier record does not.
    text = "QUBITS 2\nH 0\nCX 0 1\nMPP X0*X1\nMPP Z0*Z1\nDETECTOR 0 0\nDETECTOR 0 1\nM 0\n"
    c = oracle.Circuit(text, {"p_mpp": 0.5})
    thr = int(np.floor(0.5 * 2 ** 32))
    for f0, f1 in itertools.product((0, 1), repeat=2):
        words = np.array([0 if f0 else thr, 0 if f1 else thr, 7, 7, 7], dtype=np.uint32)
        r = c.shot(0, 0, words=words)
        if f0:
            assert r.status == oracle.DISCARDED and r.abort_op == 4
        elif f1:
            assert r.status == oracle.DISCARDED and r.abort_op == 5
        else:
            assert r.status == oracle.PASSED and r.record == [0, 0, r.record[2]]
