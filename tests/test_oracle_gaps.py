"""Pins of the oracle's gap sampling of noise hits (noise mode 1).

Mode 1 draws the same hit distribution as mode 0 with different random words:
every noise location is hit independently with its own probability, and a
hit's Pauli is uniform over the channel's list.  These tests check that
against exact enumeration, binomial rates, the geometric law of the first hit,
and the degenerate cases (p = 1, p below 2^-32, no noise, explicit words).
"""
import numpy as np
import pytest

import oracle
from tests.test_oracle_pins import _exact_distribution

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _bits(outcomes, n_rec):
    """uint32 record words [words][shots] -> bit matrix [shots][n_rec]."""
    o = np.asarray(outcomes, dtype=np.uint64)
    cols = [((o[r >> 5] >> np.uint64(r & 31)) & np.uint64(1)).astype(np.int64) for r in range(n_rec)]
    return np.stack(cols, axis=1)


def test_gap_sampling_matches_exact_distribution():
    # Distinct probabilities, so every candidate but the p_max site is thinned.
    p1, p2, p3 = 0.2, 0.05, 0.12
    body = [("H 0", None), ("NOISE", ("DEP1", p1, [0])), ("T 0", None), ("CX 0 1", None),
            ("NOISE", ("DEP2", p2, [0, 1])), ("H 1", None), ("NOISE", ("XERR", p3, [1])), ("M 0", None),
            ("M 1", None)]
    sites = [s for _, s in body if s]
    exact = _exact_distribution("QUBITS 2\n" + "\n".join(l for l, _ in body) + "\n", sites, 2)
    text = "QUBITS 2\nH 0\nDEP1 %g 0\nT 0\nCX 0 1\nDEP2 %g 0 1\nH 1\nXERR %g 1\nM 0\nM 1\n" % (p1, p2, p3)
    c = oracle.Circuit(text, noise_mode=1)
    N = 200000
    recs = c.batch(13, 0, N)["outcomes"][0].astype(np.int64)
    keys = (recs & 1) + 2 * ((recs >> 1) & 1)
    counts = np.bincount(keys, minlength=4)
    chi2 = sum((counts[a + 2 * b] - pr * N) ** 2 / (pr * N) for (a, b), pr in exact.items())
    # 3 degrees of freedom: P(chi2 > 16.27) = 0.001
    assert chi2 < 16.27, (chi2, exact, counts)


def test_gap_sampling_per_slot_rates_and_independence():
    # XERR_i then M_i on separate qubits: record bit i is exactly slot i's hit.
    rng = np.random.default_rng(5)
    ps = rng.choice([0.002, 0.01, 0.03, 0.05], size=40)
    text = "QUBITS 40\n" + "".join("XERR %r %d\nM %d\n" % (float(p), q, q) for q, p in enumerate(ps))
    c = oracle.Circuit(text, noise_mode=1)
    N = 200000
    hits = _bits(c.batch(21, 0, N)["outcomes"], 40)
    rate = hits.mean(axis=0)
    sd = np.sqrt(ps * (1 - ps) / N)
    assert np.all(np.abs(rate - ps) < 5 * sd), np.max(np.abs(rate - ps) / sd)
    # pairwise independence, neighbours and far pairs
    for i, j in [(0, 1), (5, 6), (10, 30), (38, 39), (0, 39)]:
        pij = ps[i] * ps[j]
        both = (hits[:, i] & hits[:, j]).mean()
        assert abs(both - pij) < 5 * np.sqrt(pij * (1 - pij) / N) + 1e-6, (i, j, both, pij)
    # total hit count: binomial-sum mean and variance
    tot = hits.sum(axis=1)
    mean, var = ps.sum(), (ps * (1 - ps)).sum()
    assert abs(tot.mean() - mean) < 5 * np.sqrt(var / N)
    assert abs(tot.var() / var - 1) < 0.05


def test_gap_sampling_geometric_first_hit():
    # 300 slots of one probability on one qubit (measure and reset after each):
    # P(no hit among the first m) = (1 - p)^m.
    p, n = 0.01, 300
    text = "QUBITS 1\n" + "XERR %r 0\nM 0\nR 0\n" % p * n
    c = oracle.Circuit(text, noise_mode=1)
    N = 100000
    hits = _bits(c.batch(3, 0, N)["outcomes"], n)
    first = np.where(hits.any(axis=1), hits.argmax(axis=1), n)
    for m in (1, 10, 50, 100, 250):
        q = (1 - p) ** m
        got = (first >= m).mean()
        assert abs(got - q) < 5 * np.sqrt(q * (1 - q) / N), (m, got, q)


def test_gap_sampling_dep1_paulis_uniform_under_thinning():
    # Slot 0 (DEP1 0.3) is thinned by 0.3 / 0.6 against slot 1 (DEP1 0.6 on a
    # spare qubit).  Its Pauli, read out in the Z, X and Y bases, flips the
    # outcome with P(X)+P(Y), P(Z)+P(Y), P(X)+P(Z): 2p/3 each when uniform.
    p = 0.3
    pre = {"Z": "", "X": "H 0\n", "Y": "H 0\nS 0\n"}
    post = {"Z": "", "X": "H 0\n", "Y": "SDG 0\nH 0\n"}
    N = 100000
    for basis in "ZXY":
        text = "QUBITS 2\n%sDEP1 %r 0\nDEP1 0.6 1\n%sM 0\n" % (pre[basis], p, post[basis])
        c = oracle.Circuit(text, noise_mode=1)
        got = _bits(c.batch(17, 0, N)["outcomes"], 1)[:, 0].mean()
        e = 2 * p / 3
        assert abs(got - e) < 5 * np.sqrt(e * (1 - e) / N), (basis, got, e)


def test_gap_sampling_certain_and_negligible_noise():
    # p = 1: q = 0, every slot is a candidate and every candidate is accepted.
    c = oracle.Circuit("QUBITS 3\nXERR 1 0\nXERR 1 1\nXERR 1 2\nM 0\nM 1\nM 2\n", noise_mode=1)
    assert (c.batch(1, 0, 500)["outcomes"][0] == 7).all()
    # p below 2^-32: threshold 0, never hit in either mode.
    for mode in (0, 1):
        c = oracle.Circuit("QUBITS 2\nXERR 1e-12 0\nXERR 1e-12 1\nM 0\nM 1\n", noise_mode=mode)
        assert (c.batch(1, 0, 2000)["outcomes"] == 0).all()
    # ... and does not set p_max for the slots that can be hit
    c = oracle.Circuit("QUBITS 2\nXERR 1e-12 0\nXERR 1 1\nM 0\nM 1\n", noise_mode=1)
    assert (c.batch(2, 0, 500)["outcomes"][0] == 2).all()


def test_gap_sampling_leaves_measurement_draws_alone():
    # No noise: the outcome draws (stream 1) are the same in both modes.
    text = "QUBITS 3\nH 0\nT 0\nH 0\nCX 0 1\nH 2\nM 0\nM 1\nM 2\n"
    a = oracle.Circuit(text).batch(8, 0, 3000)
    b = oracle.Circuit(text, noise_mode=1).batch(8, 0, 3000)
    assert (a["outcomes"] == b["outcomes"]).all()
    # explicit words always use the per-slot form
    text = "QUBITS 1\nDEP1 0.5 0\nM 0\n"
    w = np.array([0, 7], dtype=np.uint32)
    assert oracle.Circuit(text, noise_mode=1).shot(0, 0, words=w).record == [1]


def test_gap_sampling_bad_mode():
    with pytest.raises(ValueError, match="noise mode"):
        oracle.Circuit("QUBITS 1\nM 0\n", noise_mode=2)
