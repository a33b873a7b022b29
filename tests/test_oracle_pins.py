"""Pins of the CPU oracle against things other than itself (no GPU).

* Pauli products against 2x2 / Kronecker matrix products;
* every tableau rule against dense conjugation U P U^dagger;
* random Clifford+T+measurement circuits against a dense statevector with a
  phase-tracked stabilizer shadow, exact to 1e-12 with no global-phase freedom
  (Definition 1, Eqs. 1-4, Theorem 1);
* Clifford-only circuits against an independent Aaronson-Gottesman tableau;
* identities T^2 = S, T^8 = I, T T^dagger = I, S^4 = H^2 = I, unit norm;
* closed forms for T|+>, T|1>, P(X=+1) after T;
* the support bounds of Theorem 1, the 2^min(t,n) bound, Proposition 1's coset
  bound and Theorem 2's |v| <= 16 / 1024;
* Philox4x32-10 known-answer vectors;
* the noise model and outcome sampling against exact enumeration (chi^2).
"""
from __future__ import annotations

import itertools
import os

import numpy as np
import pytest

import oracle
import workloads
from tests import ref_chp, ref_dense
from tests.gen_small import random_circuit, random_words

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


# ---------------------------------------------------------------------------
# Philox
# ---------------------------------------------------------------------------
def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 3
    for r in rows:
        v = [int(t, 16) for t in r]
        out = oracle.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


# ---------------------------------------------------------------------------
# Pauli products (the word-level phase formula)
# ---------------------------------------------------------------------------
def _pauli_matrix(x, z, e, n):
    m = np.array([[1.0 + 0j]])
    for q in reversed(range(n)):
        xb, zb = (x >> q) & 1, (z >> q) & 1
        if xb and zb:
            f = ref_dense.MATS["Y"]
        elif xb:
            f = ref_dense.MATS["X"]
        elif zb:
            f = ref_dense.MATS["Z"]
        else:
            f = np.eye(2)
        m = np.kron(m, f)
    return (1j ** e) * m


def test_pauli_product_single_qubit_exhaustive():
    for ax, az, ae, bx, bz, be in itertools.product((0, 1), (0, 1), range(4), (0, 1), (0, 1), range(4)):
        cx, cz, ce = oracle.pauli_mul((ax, az, ae), (bx, bz, be))
        want = _pauli_matrix(ax, az, ae, 1) @ _pauli_matrix(bx, bz, be, 1)
        assert np.allclose(_pauli_matrix(cx, cz, ce, 1), want, atol=1e-15)


def test_pauli_product_multi_qubit_matrices():
    rng = np.random.default_rng(5)
    for _ in range(200):
        n = 4
        a = [int(rng.integers(16)), int(rng.integers(16)), int(rng.integers(4))]
        b = [int(rng.integers(16)), int(rng.integers(16)), int(rng.integers(4))]
        c = oracle.pauli_mul(a, b)
        assert np.allclose(_pauli_matrix(*c, n), _pauli_matrix(*a, n) @ _pauli_matrix(*b, n), atol=1e-14)


def test_pauli_product_64_qubit_words_compose_per_qubit():
    # A 64-qubit product is the tensor product of per-qubit products, whose
    # phases multiply: check against the exhaustive single-qubit table.
    rng = np.random.default_rng(6)
    table = {}
    for ax, az, bx, bz in itertools.product((0, 1), repeat=4):
        table[(ax, az, bx, bz)] = oracle.pauli_mul((ax, az, 0), (bx, bz, 0))
    for _ in range(200):
        ax, az, bx, bz = (int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(2)) for _ in range(4))
        ae, be = int(rng.integers(4)), int(rng.integers(4))
        cx, cz, ce = oracle.pauli_mul((ax, az, ae), (bx, bz, be))
        e = ae + be
        for q in range(64):
            t = table[((ax >> q) & 1, (az >> q) & 1, (bx >> q) & 1, (bz >> q) & 1)]
            assert t[0] == ((cx >> q) & 1) and t[1] == ((cz >> q) & 1)
            e += t[2]
        assert e % 4 == ce


# ---------------------------------------------------------------------------
# Tableau rules against dense conjugation
# ---------------------------------------------------------------------------
def _unitary(text, n):
    cols = []
    for k in range(1 << n):
        psi = np.zeros(1 << n, dtype=complex)
        psi[k] = 1
        _, ops = ref_dense.parse(text)
        for tok in ops:
            g = tok[0]
            if g in ref_dense.MATS:
                psi = ref_dense.apply_1q(psi, ref_dense.MATS[g], int(tok[1]), n)
            elif g == "CX":
                psi = ref_dense.apply_cx(psi, int(tok[1]), int(tok[2]), n)
            elif g == "CZ":
                psi = ref_dense.apply_cz(psi, int(tok[1]), int(tok[2]), n)
        cols.append(psi)
    return np.array(cols).T


@pytest.mark.parametrize("seed", range(40))
def test_every_gate_rule_matches_dense_conjugation(seed):
    # Random Clifford words on 2-3 qubits reach rows containing every Pauli and
    # sign; every final row must equal U P U^dagger exactly, sign included.
    n = 2 + seed % 2
    text, _ = random_circuit(seed, n, 12, clifford_only=True, p_meas=0, p_mpp=0, p_reset=0, p_pauli=0.3,
                             gates=("H", "S", "SDG", "CX", "CZ"))
    r = oracle.Circuit(text).shot(0, 0)
    U = _unitary(text, n)
    for i in range(n):
        for P0, row in ((_pauli_matrix(1 << i, 0, 0, n), i), (_pauli_matrix(0, 1 << i, 0, n), n + i)):
            want = U @ P0 @ U.conj().T
            got = _pauli_matrix(int(r.tab_x[row]), int(r.tab_z[row]), 2 * int(r.tab_r[row]), n)
            assert np.allclose(got, want, atol=1e-12)


@pytest.mark.parametrize("seed", range(16))
def test_hxy_gate_rules_match_dense_conjugation(seed):
    n = 2
    rng = np.random.default_rng(seed)
    ops = []
    for _ in range(10):
        g = ["H_XY", "H_NXY", "H", "S", "CX"][int(rng.integers(5))]
        ops.append("CX 0 1" if g == "CX" else "%s %d" % (g, int(rng.integers(2))))
    text = "QUBITS 2\n" + "\n".join(ops) + "\n"
    r = oracle.Circuit(text).shot(0, 0)
    U = _unitary(text, n)
    for i in range(n):
        for P0, row in ((_pauli_matrix(1 << i, 0, 0, n), i), (_pauli_matrix(0, 1 << i, 0, n), n + i)):
            want = U @ P0 @ U.conj().T
            got = _pauli_matrix(int(r.tab_x[row]), int(r.tab_z[row]), 2 * int(r.tab_r[row]), n)
            assert np.allclose(got, want, atol=1e-12), text


def test_hxy_single_qubit_images():
    # (X+Y)/sqrt2: X -> Y, Z -> -Z;  (X-Y)/sqrt2: X -> -Y, Z -> -Z
    for g, sx in (("H_XY", 0), ("H_NXY", 1)):
        r = oracle.Circuit("QUBITS 1\n%s 0\n" % g).shot(0, 0)
        assert (int(r.tab_x[0]), int(r.tab_z[0]), int(r.tab_r[0])) == (1, 1, sx)   # d_0 = X image
        assert (int(r.tab_x[1]), int(r.tab_z[1]), int(r.tab_r[1])) == (0, 1, 1)    # s_0 = Z image


# ---------------------------------------------------------------------------
# Dense statevector with phase-tracked shadow
# ---------------------------------------------------------------------------
def _check_dense(text, seed, tol=1e-12):
    c = oracle.Circuit(text)
    words = random_words(seed, c.words_per_shot)
    r = c.shot(0, 0, words=words, coeff_cap=1 << 14)
    assert r.status == oracle.PASSED
    phi, shadow, record, p0s = ref_dense.run(text, words[c.n_noise_slots:])
    n = c.n_qubits
    assert r.record == record
    assert np.allclose(r.p0, p0s, atol=tol, rtol=0)
    ref_dense.check_tableau(r.tab_x, r.tab_z, r.tab_r, shadow, n)
    got = ref_dense.reconstruct(r.tab_x, r.tab_z, r.tab_r, r.coeffs, shadow, n)
    assert np.max(np.abs(got - phi)) < tol, np.max(np.abs(got - phi))
    assert abs(sum(abs(v) ** 2 for v in r.coeffs.values()) - 1) < tol
    return r


@pytest.mark.parametrize("seed", range(60))
def test_random_clifford_t_measure_matches_dense(seed):
    n = 1 + seed % 5
    text, _ = random_circuit(1000 + seed, n, 40 + 3 * (seed % 7))
    _check_dense(text, seed)


@pytest.mark.parametrize("seed", range(12))
def test_every_prefix_matches_dense(seed):
    # Step-by-step identity (the paper's Sec. V-B cross-check): every prefix of
    # a circuit gives the same state as the dense run of that prefix.
    text, _ = random_circuit(5000 + seed, 3 + seed % 2, 30)
    lines = text.strip().splitlines()
    for k in range(2, len(lines) + 1):
        _check_dense("\n".join(lines[:k]) + "\n", seed)


@pytest.mark.parametrize("seed", range(40))
def test_msc_ops_match_dense(seed):
    # X-basis readouts and resets, measure-and-reset, H_XY / H_NXY and
    # record-controlled Paulis mixed into random Clifford+T circuits
    n = 1 + seed % 5
    text, _ = random_circuit(7000 + seed, n, 45, p_msc=0.3)
    _check_dense(text, seed)


@pytest.mark.parametrize("seed", range(6))
def test_msc_ops_every_prefix_matches_dense(seed):
    text, _ = random_circuit(7700 + seed, 3, 30, p_msc=0.35)
    lines = text.strip().splitlines()
    for k in range(2, len(lines) + 1):
        _check_dense("\n".join(lines[:k]) + "\n", seed)


def test_x_basis_reset_and_readout():
    # RX prepares |+>: an MX right after reads 0 with certainty, M reads 50/50
    c = oracle.Circuit("QUBITS 1\nH 0\nS 0\nRX 0\nMX 0\n")
    for w in (0, 1 << 31, 0xFFFFFFFF):
        r = c.shot(0, 0, words=np.array([w, w], dtype=np.uint32))
        assert r.record == [0]
    c = oracle.Circuit("QUBITS 1\nRX 0\nM 0\n")
    r = c.shot(0, 0, words=np.array([5, 5], dtype=np.uint32))
    assert abs(r.p0[1] - 0.5) < 1e-15
    # MR leaves |0>: a second M reads 0 whatever the first read
    c = oracle.Circuit("QUBITS 1\nH 0\nMR 0\nM 0\n")
    for w in (0, 0xFFFFFFFF):
        r = c.shot(0, 0, words=np.array([w, 3], dtype=np.uint32))
        assert r.record[1] == 0 and r.record[0] == (0 if w == 0 else 1)


def test_feedback_applies_pauli_on_record():
    # M of |+> gives a random bit b; XIF b then M again reads 0 for b = 0 and
    # 1 (X on |1> after the collapse gives |0>) -- in both cases the second
    # readout is 0 after X-correction of a Z-basis collapse.
    c = oracle.Circuit("QUBITS 1\nH 0\nM 0\nXIF 0 0\nM 0\n")
    for w in (0, 0xFFFFFFFF):
        r = c.shot(0, 0, words=np.array([w, 3], dtype=np.uint32))
        assert r.record[1] == 0
    # ZIF acts on the X basis the same way
    c = oracle.Circuit("QUBITS 1\nMX 0\nZIF 0 0\nMX 0\n")
    for w in (0, 0xFFFFFFFF):
        r = c.shot(0, 0, words=np.array([w, 3], dtype=np.uint32))
        assert r.record[1] == 0


def test_msc_model_noise_matches_explicit_noise_ops():
    # X-basis readouts take a Z flip before, X-basis resets a Z flip after
    text = "QUBITS 2\nMX 0\nRX 1\nMR 0\nMRX 1\n"
    explicit = ("QUBITS 2\nZERR 0.4 0\nMX 0\nRX 1\nZERR 0.5 1\nXERR 0.4 0\nMR 0\nXERR 0.5 0\n"
                "ZERR 0.4 1\nMRX 1\nZERR 0.5 1\n")
    model = {"p1": 0.0, "p2": 0.0, "p_idle": 0.0, "p_meas": 0.4, "p_reset": 0.5, "p_mpp": 0.0}
    a = oracle.Circuit(text, model).batch(5, 0, 2000)
    b = oracle.Circuit(explicit).batch(5, 0, 2000)
    assert (a["outcomes"] == b["outcomes"]).all()
    assert a["outcomes"].any()


@pytest.mark.parametrize("seed", range(30))
def test_ccz_ccx_match_dense(seed):
    # CCZ / CCX (Toffoli) mixed into random Clifford+T circuits with
    # measurements, against the dense statevector
    n = 3 + seed % 4
    text, _ = random_circuit(8100 + seed, n, 40, p_ccz=0.15)
    assert "CC" in text
    _check_dense(text, seed)


def test_ccz_closed_forms():
    # CCZ|+++> = (1/sqrt8) sum_x (-1)^{x0 x1 x2}|x>: the X-basis readouts of the
    # three qubits are correlated exactly as that state predicts, and the
    # support after one CCZ is at most 8 (Proposition 1, |Q| - r_Q = 3)
    c = oracle.Circuit("QUBITS 3\nH 0\nH 1\nH 2\nCCZ 0 1 2\n")
    r = c.shot(0, 0)
    assert 1 < len(r.coeffs) <= 8
    c = oracle.Circuit("QUBITS 3\nH 0\nH 1\nH 2\nCCZ 0 1 2\nMPP X0*X1*X2\n")
    r = c.shot(0, 0, words=np.array([0], dtype=np.uint32))
    # <X X X> on CCZ|+++> = 1/2 (the -1 sign on one of 8 amplitudes): P(+1) = 3/4
    assert abs(r.p0[0] - 0.75) < 1e-12
    # CCZ twice is the identity on the coefficients
    a = oracle.Circuit("QUBITS 3\nH 0\nH 1\nT 2\nH 2\nCCZ 0 1 2\nCCZ 0 1 2\n").shot(0, 0)
    b = oracle.Circuit("QUBITS 3\nH 0\nH 1\nT 2\nH 2\n").shot(0, 0)
    keys = set(a.coeffs) | set(b.coeffs)
    assert max(abs(a.coeffs.get(k, 0) - b.coeffs.get(k, 0)) for k in keys) < 1e-12
    # Toffoli truth table on basis inputs
    for x in range(8):
        prep = "".join("X %d\n" % q for q in range(3) if (x >> q) & 1)
        r = oracle.Circuit("QUBITS 3\n" + prep + "CCX 0 1 2\nM 0\nM 1\nM 2\n").shot(0, 0)
        want = x ^ (4 if (x & 3) == 3 else 0)
        assert r.record == [(want >> q) & 1 for q in range(3)]


def test_dense_on_larger_register():
    text, _ = random_circuit(77, 10, 120, p_t=0.1)
    _check_dense(text, 77, tol=1e-11)


# ---------------------------------------------------------------------------
# Clifford-only circuits against an independent CHP tableau
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(40))
def test_clifford_only_matches_chp_bit_exact(seed):
    n = 2 + seed % 7
    text, _ = random_circuit(2000 + seed, n, 80, clifford_only=True, allow_mpp=False,
                             gates=("H", "S", "SDG", "CX", "CZ"))
    c = oracle.Circuit(text)
    words = random_words(seed, c.words_per_shot)
    r = c.shot(0, 0, words=words)
    sim, record = ref_chp.run(text, words[c.n_noise_slots:])
    assert r.record == record
    assert [int(v) for v in r.tab_x] == sim.x[: 2 * n]
    assert [int(v) for v in r.tab_z] == sim.z[: 2 * n]
    assert [int(v) for v in r.tab_r] == sim.r[: 2 * n]
    # a Clifford-only state keeps a single coefficient of modulus 1
    assert len(r.coeffs) == 1 and abs(abs(list(r.coeffs.values())[0]) - 1) < 1e-12


# ---------------------------------------------------------------------------
# Identities and closed forms
# ---------------------------------------------------------------------------
def _state(text, words=None):
    c = oracle.Circuit(text)
    r = c.shot(0, 0, words=words)
    phi, shadow, _, _ = ref_dense.run(text, [] if words is None else words[c.n_noise_slots:])
    return r, ref_dense.reconstruct(r.tab_x, r.tab_z, r.tab_r, r.coeffs, shadow, c.n_qubits)


def test_t_squared_is_s_exactly():
    for prep in ("H 0", "H 0\nS 0", "H 0\nH 1\nCX 0 1", "X 0\nH 1"):
        _, a = _state("QUBITS 2\n%s\nT 0\nT 0\n" % prep)
        _, b = _state("QUBITS 2\n%s\nS 0\n" % prep)
        assert np.max(np.abs(a - b)) < 1e-14  # includes the global phase


def test_t8_and_t_tdg_are_identity_on_coefficients():
    for prep in ("H 0", "H 0\nS 0\nH 1\nCX 0 1"):
        base = oracle.Circuit("QUBITS 2\n%s\n" % prep).shot(0, 0)
        for body in ("T 0\n" * 8, "T 0\nTDG 0\n", "TDG 0\nT 0\n", "T 0\nT 0\nTDG 0\nTDG 0\n"):
            r = oracle.Circuit("QUBITS 2\n%s\n%s" % (prep, body)).shot(0, 0)
            assert set(r.coeffs) == set(base.coeffs)
            for a in base.coeffs:
                assert abs(r.coeffs[a] - base.coeffs[a]) < 1e-12
            assert (r.tab_x == base.tab_x).all() and (r.tab_z == base.tab_z).all() and (r.tab_r == base.tab_r).all()


def test_s4_h2_identity_on_tableau():
    base = oracle.Circuit("QUBITS 2\nH 0\nCX 0 1\n").shot(0, 0)
    for body in ("S 1\n" * 4, "H 1\nH 1\n", "SDG 0\nS 0\n", "CZ 0 1\nCZ 0 1\n"):
        r = oracle.Circuit("QUBITS 2\nH 0\nCX 0 1\n" + body).shot(0, 0)
        assert (r.tab_x == base.tab_x).all() and (r.tab_z == base.tab_z).all() and (r.tab_r == base.tab_r).all()


def test_t_plus_closed_form():
    r = oracle.Circuit("QUBITS 1\nH 0\nT 0\n").shot(0, 0)
    w = np.exp(1j * np.pi / 4)
    assert abs(r.coeffs[0] - (1 + w) / 2) < 1e-15
    assert abs(r.coeffs[1] - (1 - w) / 2) < 1e-15


def test_x_measurement_after_t_plus_probability():
    r = oracle.Circuit("QUBITS 1\nH 0\nT 0\nH 0\nM 0\n").shot(0, 0)
    assert abs(r.p0[0] - 0.8535533905932737) < 1e-15          # cos^2(pi/8)
    assert abs(np.cos(np.pi / 8) ** 2 - 0.8535533905932737) < 1e-16


def test_t_on_one_does_not_branch():
    # Observation 3: Z_q in the stabilizer group -> no branching, phase only.
    r = oracle.Circuit("QUBITS 1\nX 0\nT 0\n").shot(0, 0)
    assert list(r.coeffs) == [0]
    assert abs(r.coeffs[0] - np.exp(1j * np.pi / 4)) < 1e-15
    assert r.work["t_phase_entries"] == 1 and r.work["t_entries"] == 0


def test_unit_norm_after_every_measurement():
    for seed in range(10):
        text, _ = random_circuit(300 + seed, 4, 60)
        lines = text.strip().splitlines()
        c = oracle.Circuit(text)
        words = random_words(seed, c.words_per_shot)
        for k in range(2, len(lines) + 1):
            if lines[k - 1].split()[0] in ("M", "MPP", "R"):
                ck = oracle.Circuit("\n".join(lines[:k]) + "\n")
                r = ck.shot(0, 0, words=words[: ck.words_per_shot])
                assert abs(r.norm2 - 1) < 1e-13


# ---------------------------------------------------------------------------
# Support bounds
# ---------------------------------------------------------------------------
def test_theorem1_support_changes():
    # Clifford: |v'| = |v|; T: |v'| <= 2|v|; measurement: |v'| <= |v|.
    for seed in range(15):
        text, _ = random_circuit(400 + seed, 5, 70, p_t=0.3)
        lines = text.strip().splitlines()
        c = oracle.Circuit(text)
        words = random_words(seed, c.words_per_shot)
        prev = 1
        for k in range(2, len(lines) + 1):
            ck = oracle.Circuit("\n".join(lines[:k]) + "\n")
            size = len(ck.shot(0, 0, words=words[: ck.words_per_shot]).coeffs)
            g = lines[k - 1].split()[0]
            if g in ("T", "TDG"):
                assert size <= 2 * prev
            elif g in ("M", "MPP", "R"):
                assert size <= prev
            else:
                assert size == prev
            prev = size


def test_support_at_most_two_to_min_t_n():
    for seed in range(20):
        text, _ = random_circuit(600 + seed, 4, 80, p_t=0.3, p_meas=0, p_mpp=0, p_reset=0)
        t = text.count("\nT ") + text.count("\nTDG ")
        r = oracle.Circuit(text).shot(0, 0)
        assert r.max_support <= 2 ** min(t, 4)


def _gf2_rank(rows):
    basis = {}
    for r in rows:
        while r:
            h = r.bit_length() - 1
            if h in basis:
                r ^= basis[h]
            else:
                basis[h] = r
                break
    return len(basis)


@pytest.mark.parametrize("seed", range(12))
def test_proposition1_coset_bound(seed):
    # Random stabilizer state on 5 qubits, then a layer of T/T^dagger on Q:
    # |v| <= 2^{|Q| - r_Q}, with r_Q the rank of the Z-strings on Q that
    # stabilize the state up to sign (found by brute force on the statevector).
    n = 5
    text, _ = random_circuit(700 + seed, n, 40, clifford_only=True, p_meas=0, p_mpp=0, p_reset=0)
    rng = np.random.default_rng(seed)
    Q = sorted(rng.choice(n, size=int(rng.integers(2, n + 1)), replace=False).tolist())
    phi, _, _, _ = ref_dense.run(text, [])
    stab = [g for g in range(1, 1 << n) if all(((g >> q) & 1) == 0 or q in Q for q in range(n))
            and abs(abs(ref_dense.expval(phi, 0, g, 0, n)) - 1) < 1e-9]
    r_q = _gf2_rank(stab)
    layer = "".join("%s %d\n" % ("T" if rng.integers(2) == 0 else "TDG", q) for q in Q)
    r = oracle.Circuit(text + layer).shot(0, 0)
    assert len(r.coeffs) <= 2 ** (len(Q) - r_q)


def test_theorem2_bounds_on_cultivation_shaped_circuits():
    # Thm 2: |v| <= 2^{|Q| - r_Z} = 16 (7 data, r_Z = 3) and 1024 (19 data,
    # r_Z = 9), reached by the noiseless run.
    for name, bound in (("cultivation_15q", 16), ("cultivation_42q", 1024)):
        w = workloads.config(name, seed=1)
        r = oracle.Circuit(w.text).batch(3, 0, 4)
        assert (r["status"] == oracle.PASSED).all() and (r["obs"] == 0).all()
        assert r["max_support"].max() == bound
        noisy = oracle.Circuit(w.text, w.noise).batch(3, 0, 64)
        assert noisy["max_support"].max() <= bound


# ---------------------------------------------------------------------------
# Noise model and sampling against exact enumeration
# ---------------------------------------------------------------------------
def _exact_distribution(text, noise_sites, n):
    """Enumerate every Pauli pattern of the listed noise sites with its
    probability and return the exact distribution of the record."""
    dist = {}
    options = []
    for kind, p, qs in noise_sites:
        if kind == "DEP1":
            options.append([(1 - p, [])] + [(p / 3, [(P, qs[0])]) for P in "XYZ"])
        elif kind == "DEP2":
            opts = [(1 - p, [])]
            for code in range(1, 16):
                pa, pb = "IXYZ"[code >> 2], "IXYZ"[code & 3]
                opts.append((p / 15, [(P, q) for P, q in ((pa, qs[0]), (pb, qs[1])) if P != "I"]))
            options.append(opts)
        elif kind == "XERR":
            options.append([(1 - p, []), (p, [("X", qs[0])])])
    for combo in itertools.product(*options):
        prob = float(np.prod([c[0] for c in combo]))
        # substitute the chosen Paulis into the marked lines
        out = []
        k = 0
        for line in text.splitlines():
            if line.startswith("NOISE"):
                out += ["%s %d" % (P, q) for P, q in combo[k][1]]
                k += 1
            else:
                out.append(line)
        sub = "\n".join(out) + "\n"
        # exact outcome probabilities by branching over measurements
        _branch(sub, n, prob, dist)
    return dist


def _branch(text, n, prob, dist):
    _, ops = ref_dense.parse(text)
    states = [(np.eye(1 << n, dtype=complex)[0], prob, ())]
    for tok in ops:
        g = tok[0]
        new = []
        for psi, pr, rec in states:
            if g in ref_dense.MATS:
                new.append((ref_dense.apply_1q(psi, ref_dense.MATS[g], int(tok[1]), n), pr, rec))
            elif g == "CX":
                new.append((ref_dense.apply_cx(psi, int(tok[1]), int(tok[2]), n), pr, rec))
            elif g == "M":
                P = ref_dense.pauli_apply(psi, 0, 1 << int(tok[1]), 0, n)
                for m in (1, -1):
                    proj = 0.5 * (psi + m * P)
                    w = float(np.real(np.vdot(proj, proj)))
                    if w > 1e-15:
                        new.append((proj / np.sqrt(w), pr * w, rec + ((1 - m) // 2,)))
        states = new
    for _, pr, rec in states:
        dist[rec] = dist.get(rec, 0.0) + pr


def test_noise_and_sampling_chi_square():
    p = 0.2
    body = [("H 0", None), ("NOISE", ("DEP1", p, [0])), ("T 0", None), ("CX 0 1", None),
            ("NOISE", ("DEP2", p, [0, 1])), ("H 1", None), ("NOISE", ("XERR", p, [1])), ("M 0", None), ("M 1", None)]
    sites = [s for l, s in body if s]
    enum_text = "QUBITS 2\n" + "\n".join(l for l, _ in body) + "\n"
    exact = _exact_distribution(enum_text, sites, 2)
    sim_text = "QUBITS 2\nH 0\nDEP1 %g 0\nT 0\nCX 0 1\nDEP2 %g 0 1\nH 1\nXERR %g 1\nM 0\nM 1\n" % (p, p, p)
    c = oracle.Circuit(sim_text)
    N = 200000
    r = c.batch(11, 0, N)
    recs = r["outcomes"][0]
    counts = {}
    for v in recs:
        key = (int(v) & 1, (int(v) >> 1) & 1)
        counts[key] = counts.get(key, 0) + 1
    chi2 = 0.0
    for key, pr in exact.items():
        e = pr * N
        chi2 += (counts.get(key, 0) - e) ** 2 / e
    assert set(counts) <= set(exact)
    # 3 degrees of freedom: P(chi2 > 16.27) = 0.001
    assert chi2 < 16.27, (chi2, exact, counts)


def test_model_noise_matches_explicit_noise_ops():
    # Model insertion (p1 after 1q gates, p2 after 2q gates, XERR before M,
    # after R, idle DEP1 per TICK, MPP flip) equals the same noise written out.
    text = "QUBITS 3\nH 0\nCX 0 1\nTICK\nT 1\nM 2\nR 1\nTICK\nMPP X0*Z1\n"
    explicit = ("QUBITS 3\nH 0\nDEP1 0.1 0\nCX 0 1\nDEP2 0.2 0 1\nTICK\nDEP1 0.3 2\nT 1\nDEP1 0.1 1\n"
                "XERR 0.4 2\nM 2\nR 1\nXERR 0.5 1\nTICK\nDEP1 0.3 0\nMPP X0*Z1\n")
    model = {"p1": 0.1, "p2": 0.2, "p_idle": 0.3, "p_meas": 0.4, "p_reset": 0.5, "p_mpp": 0.0}
    a = oracle.Circuit(text, model).batch(5, 0, 2000)
    b = oracle.Circuit(explicit).batch(5, 0, 2000)
    assert (a["outcomes"] == b["outcomes"]).all()


def test_forced_noise_words():
    # w = 0 < thr always hits; DEP1 index floor(3 w / thr) = 0 -> X.
    c = oracle.Circuit("QUBITS 1\nDEP1 0.5 0\nM 0\n")
    r = c.shot(0, 0, words=np.array([0, 7], dtype=np.uint32))
    assert r.record == [1]
    thr = int(np.floor(0.5 * 2 ** 32))
    r = c.shot(0, 0, words=np.array([thr, 7], dtype=np.uint32))   # no hit
    assert r.record == [0]
    r = c.shot(0, 0, words=np.array([thr - 1, 7], dtype=np.uint32))  # index 2 -> Z
    assert r.record == [0]


# ---------------------------------------------------------------------------
# Host logic: parse errors, postselection, overflow, shard determinism
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("text,frag", [
    ("H 0\n", "line 1"), ("QUBITS 2\nH 2\n", "line 2"), ("QUBITS 2\nCX 1 1\n", "line 2"),
    ("QUBITS 2\nFOO 1\n", "unknown"), ("QUBITS 2\nDETECTOR 0 0\n", "record"),
    ("QUBITS 2\nDEP1 1.5 0\n", "probability"), ("QUBITS 2\nMPP X0*X0\n", "repeated"),
    ("QUBITS 65\n", "QUBITS"), ("QUBITS 2\nXIF 0 1\n", "record"), ("QUBITS 2\nM 0\nZIF 0\n", "record index"),
    ("QUBITS 3\nCCZ 0 1 1\n", "repeated"),
])
def test_parse_errors(text, frag):
    with pytest.raises(ValueError, match=frag):
        oracle.Circuit(text)


def test_postselection_abort_and_overflow_flags():
    c = oracle.Circuit("QUBITS 1\nX 0\nM 0\nDETECTOR 0 0\nH 0\nT 0\n")
    r = c.shot(0, 0)
    assert r.status == oracle.DISCARDED and r.abort_op == 2
    c = oracle.Circuit("QUBITS 2\nH 0\nH 1\nT 0\nT 1\n")
    r = c.shot(0, 0, cap=3)
    assert r.status == oracle.OVERFLOW and r.abort_op == 3 and r.max_support == 4


def test_shard_determinism():
    w = workloads.config("cultivation_15q", seed=2)
    c = oracle.Circuit(w.text, w.noise)
    a = c.batch(9, 100, 400)
    b1 = c.batch(9, 100, 200)
    b2 = c.batch(9, 300, 200)
    assert (a["outcomes"] == np.concatenate([b1["outcomes"], b2["outcomes"]], axis=1)).all()
    assert (a["status"] == np.concatenate([b1["status"], b2["status"]])).all()


def test_forced_dep2_code_mapping():
    # code = floor(15 w / thr) + 1 -> Pauli (code >> 2) on the first qubit and
    # (code & 3) on the second, with 0=I 1=X 2=Y 3=Z.  A Z-basis readout of |00>
    # shows the X part, an X-basis readout of |++> shows the Z part.
    thr = int(np.floor(0.5 * 2 ** 32))
    zc = oracle.Circuit("QUBITS 2\nDEP2 0.5 0 1\nM 0\nM 1\n")
    xc = oracle.Circuit("QUBITS 2\nH 0\nH 1\nDEP2 0.5 0 1\nH 0\nH 1\nM 0\nM 1\n")
    for code in range(1, 16):
        w = -((-(code - 1) * thr) // 15)           # ceil((code-1) thr / 15)
        assert (15 * w) // thr + 1 == code
        pa, pb = code >> 2, code & 3
        words = np.array([w, 3, 3], dtype=np.uint32)
        assert zc.shot(0, 0, words=words).record == [int(pa in (1, 2)), int(pb in (1, 2))]
        assert xc.shot(0, 0, words=words).record == [int(pa in (2, 3)), int(pb in (2, 3))]


# ---------------------------------------------------------------------------
# The top bits of the 64-bit words (n = 64)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(4))
def test_clifford_only_matches_chp_64_qubits(seed):
    # 64 qubits: every bit of the x/z words and of the two sign words, and
    # qubit 63 in particular, against the independent CHP tableau.
    n = 64
    text, _ = random_circuit(2500 + seed, n, 500, clifford_only=True, allow_mpp=False,
                             gates=("H", "S", "SDG", "CX", "CZ"))
    lines = text.strip().split("\n")
    lines += ["H 63", "CX 63 0", "S 63", "M 63", "CZ 62 63", "M 0"]
    text = "\n".join(lines) + "\n"
    c = oracle.Circuit(text)
    words = random_words(seed, c.words_per_shot)
    r = c.shot(0, 0, words=words)
    sim, record = ref_chp.run(text, words[c.n_noise_slots:])
    assert r.record == record
    assert [int(v) for v in r.tab_x] == sim.x[: 2 * n]
    assert [int(v) for v in r.tab_z] == sim.z[: 2 * n]
    assert [int(v) for v in r.tab_r] == sim.r[: 2 * n]
    assert any(int(v) >> 63 for v in r.tab_x) and any(int(v) >> 63 for v in r.tab_z)


def _relabel(text, f):
    """The same circuit with qubit q renamed f(q) (QUBITS line left out)."""
    out = []
    for line in text.strip().split("\n")[1:]:
        tok = line.split()
        g = tok[0]
        if g == "MPP":
            facs = ["%s%d" % (x[0], f(int(x[1:]))) for x in tok[1].split("*")]
            out.append("MPP " + "*".join(facs))
        elif g in ("DETECTOR", "OBSERVABLE"):
            out.append(line)
        elif g in ("XIF", "YIF", "ZIF"):
            out.append("%s %s %d" % (g, tok[1], f(int(tok[2]))))
        elif g in ("DEP1", "DEP2", "XERR", "ZERR"):
            out.append("%s %s %s" % (g, tok[1], " ".join(str(f(int(q))) for q in tok[2:])))
        else:
            out.append(" ".join([g] + [str(f(int(q))) for q in tok[1:]]))
    return "\n".join(out) + "\n"


def _spread(x, f, n):
    y = 0
    for q in range(n):
        if (x >> q) & 1:
            y |= 1 << f(q)
    return y


@pytest.mark.parametrize("seed", range(8))
def test_relabel_onto_64_qubits(seed):
    # An 8-qubit Clifford+T+measurement circuit (pinned to the dense
    # statevector by the tests above) renamed onto 8 of 64 qubits by an
    # increasing map that uses qubit 63: the other 56 qubits stay idle, the
    # pivots keep their order, so records, tableau rows and coefficients are
    # the 8-qubit ones with every index renamed.
    n = 8
    text, _ = random_circuit(2700 + seed, n, 120, p_msc=0.1 if seed % 2 else 0.0, p_ccz=0.03)
    f = (lambda q: 9 * q) if seed % 2 == 0 else (lambda q: 56 + q)
    wide = "QUBITS 64\n" + _relabel(text, f)
    assert f(7) == 63
    c8, c64 = oracle.Circuit(text), oracle.Circuit(wide)
    assert c8.words_per_shot == c64.words_per_shot
    words = random_words(seed, c8.words_per_shot)
    a, b = c8.shot(0, 0, words=words), c64.shot(0, 0, words=words)
    assert a.record == b.record and a.status == b.status
    inv = {f(q): q for q in range(n)}
    for i in range(64):
        src = inv.get(i)
        for half in (0, 64):
            if src is None:
                ex = (1 << i, 0) if half == 0 else (0, 1 << i)
                assert (int(b.tab_x[half + i]), int(b.tab_z[half + i]), int(b.tab_r[half + i])) == ex + (0,)
            else:
                j = (0 if half == 0 else n) + src
                assert int(b.tab_x[half + i]) == _spread(int(a.tab_x[j]), f, n)
                assert int(b.tab_z[half + i]) == _spread(int(a.tab_z[j]), f, n)
                assert int(b.tab_r[half + i]) == int(a.tab_r[j])
    assert {_spread(k, f, n): v for k, v in a.coeffs.items()} == pytest.approx(b.coeffs, abs=1e-14)


def test_work_counts_closed_forms():
    # The oracle's work counts that price the roofline, on states whose
    # supports are known in closed form.
    def work(text):
        c = oracle.Circuit(text)
        return c.shot(0, 0, words=np.full(c.words_per_shot, 1 << 31, dtype=np.uint32)).work
    w = work("QUBITS 1\nX 0\nT 0\n")        # |1>: Z_0 = -s_0, lambda = -1 on the one entry
    assert (w["t_phase_entries"], w["t_phase_flips"], w["t_entries"]) == (1, 1, 0)
    w = work("QUBITS 1\nT 0\n")             # |0>: lambda = +1
    assert (w["t_phase_entries"], w["t_phase_flips"]) == (1, 0)
    w = work("QUBITS 1\nH 0\nT 0\nMPP X0\n")  # T|+>: two entries; X_0 = s_0 splits them by parity
    assert (w["t_entries"], w["m_entries"], w["m_out_entries"], w["m_pairs"], w["meas_words"]) == (2, 2, 1, 0, 1)
    w = work("QUBITS 1\nH 0\nT 0\nM 0\n")     # Z_0 anticommutes with s_0: one representative pair
    assert (w["m_entries"], w["m_out_entries"], w["m_pairs"], w["meas_words"]) == (2, 1, 1, 1)
    w = work("QUBITS 2\nH 0\nH 1\nT 0\nT 1\nM 0\nM 1\n")
    assert (w["t_entries"], w["m_entries"], w["m_pairs"], w["m_out_entries"], w["events"]) == (2 + 4, 4 + 2, 2 + 1, 2 + 1, 4)


# ---------------------------------------------------------------------------
# Diagonal gates in one pass: U = sum_g c_g Z^g over the Z-strings of their
# qubits (CS, CSDG, CPHASE, RZ, CCZ, CCX, DIAG of 1-3 qubits)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(40))
def test_diagonal_gates_match_dense(seed):
    n = 2 + seed % 5
    text, _ = random_circuit(8300 + seed, n, 50, p_diag=0.2, p_t=0.08)
    assert any(g in text for g in ("CS ", "CSDG", "CPHASE", "RZ", "CCZ", "DIAG"))
    _check_dense(text, seed)


@pytest.mark.parametrize("seed", range(6))
def test_diagonal_gates_every_prefix_matches_dense(seed):
    n = 3 + seed % 3
    text, _ = random_circuit(8400 + seed, n, 30, p_diag=0.3)
    lines = text.strip().split("\n")
    for cut in range(2, len(lines) + 1):
        _check_dense("\n".join(lines[:cut]) + "\n", seed)


def _coeff_diff(a, b):
    keys = set(a) | set(b)
    return max([abs(a.get(k, 0) - b.get(k, 0)) for k in keys] + [0.0])


def test_ccz_equals_its_seven_t_phase_polynomial():
    # 4xyz = x + y + z - (x^y) - (x^z) - (y^z) + (x^y^z): T on a, b, c and on
    # a^b^c, T-dagger on a^b, a^c, b^c (parities formed by CNOTs and undone)
    # is CCZ with T = diag(1, e^{i pi/4}) exactly.  The one-pass CCZ gives the
    # same tableau and coefficients on random states.
    seven = ("T 0\nT 1\nT 2\nCX 0 1\nTDG 1\nCX 0 1\nCX 0 2\nTDG 2\nCX 0 2\nCX 1 2\nTDG 2\nCX 1 2\n"
             "CX 0 2\nCX 1 2\nT 2\nCX 1 2\nCX 0 2\n")
    for seed in range(12):
        prep, _ = random_circuit(8500 + seed, 4, 25, p_meas=0, p_mpp=0, p_reset=0)
        body = prep.split("\n", 1)[1]
        a = oracle.Circuit("QUBITS 4\n" + body + "CCZ 0 1 2\n").shot(0, 0)
        b = oracle.Circuit("QUBITS 4\n" + body + seven).shot(0, 0)
        assert (a.tab_x == b.tab_x).all() and (a.tab_z == b.tab_z).all() and (a.tab_r == b.tab_r).all()
        assert _coeff_diff(a.coeffs, b.coeffs) < 1e-12


def _gs_state(text):
    """The oracle's final state of a measurement-free circuit as a
    statevector: sum_alpha v_alpha d_alpha |psi_S> (Definition 1), with the
    phase-tracked stabilizer state of the dense checker."""
    r = oracle.Circuit(text).shot(0, 0)
    _, shadow, _, _ = ref_dense.run(text, [])
    return ref_dense.reconstruct(r.tab_x, r.tab_z, r.tab_r, r.coeffs, shadow, r.tab_x.size // 2)


def test_diagonal_gate_closed_forms():
    def coeffs(text):
        return oracle.Circuit(text).shot(0, 0).coeffs
    # RZ(pi/4) = e^{-i pi/8} T exactly (T keeps the e^{i pi/8} of Eqs. 1-2;
    # both take the non-Clifford route, so the coefficients agree), and
    # RZ(pi/2) = e^{-i pi/4} S as states (S is Clifford: another tableau)
    for pre in ("H 0\n", "H 0\nT 0\nH 0\n", "X 0\nH 0\nS 0\n"):
        a, b = coeffs("QUBITS 1\n" + pre + "RZ 0.7853981633974483 0\n"), coeffs("QUBITS 1\n" + pre + "T 0\n")
        assert _coeff_diff(a, {k: v * np.exp(-1j * np.pi / 8) for k, v in b.items()}) < 1e-12
        a = _gs_state("QUBITS 1\n" + pre + "RZ 1.5707963267948966 0\n")
        b = _gs_state("QUBITS 1\n" + pre + "S 0\n")
        assert np.max(np.abs(a - np.exp(-1j * np.pi / 4) * b)) < 1e-12
    # CS twice = CZ and CPHASE(pi) = CZ as states; CS then CSDG = I; a DIAG
    # with equal phases is a global phase; CCZ twice = I (coefficients)
    prep = "QUBITS 3\nH 0\nH 1\nT 1\nH 2\nCX 0 2\n"
    base = coeffs(prep)
    assert np.max(np.abs(_gs_state(prep + "CS 0 1\nCS 0 1\n") - _gs_state(prep + "CZ 0 1\n"))) < 1e-12
    assert np.max(np.abs(_gs_state(prep + "CPHASE 3.141592653589793 0 1\n") - _gs_state(prep + "CZ 0 1\n"))) < 1e-12
    assert _coeff_diff(coeffs(prep + "CS 0 1\nCSDG 0 1\n"), base) < 1e-12
    assert _coeff_diff(coeffs(prep + "DIAG 2 0 2 0.3 0.3 0.3 0.3\n"), {k: v * np.exp(0.3j) for k, v in base.items()}) < 1e-12
    assert _coeff_diff(coeffs(prep + "CCZ 0 1 2\nCCZ 0 1 2\n"), base) < 1e-12
    # CS|++> : <X0 X1> = 1/2 and support 4 (two new span directions)
    r = oracle.Circuit("QUBITS 2\nH 0\nH 1\nCS 0 1\nMPP X0*X1\n").shot(0, 0, words=np.array([0], dtype=np.uint32))
    assert abs(r.p0[0] - 0.75) < 1e-12
    assert len(oracle.Circuit("QUBITS 2\nH 0\nH 1\nCS 0 1\n").shot(0, 0).coeffs) == 4
    # on a computational basis state a diagonal gate only turns the phase: one entry
    r = oracle.Circuit("QUBITS 3\nX 0\nX 2\nDIAG 3 0 1 2 0.1 0.2 0.3 0.4 0.5 1.25 0.7 0.8\n").shot(0, 0)
    assert len(r.coeffs) == 1 and abs(list(r.coeffs.values())[0] - np.exp(1.25j)) < 1e-12


def test_diagonal_gate_parse_errors_and_noise():
    for bad, frag in (("QUBITS 2\nCS 0 0\n", "repeated"), ("QUBITS 2\nRZ x 0\n", "angle"),
                      ("QUBITS 3\nDIAG 4 0 1 2 3\n", "1 to 3"), ("QUBITS 2\nDIAG 2 0 1 0.1 0.2 0.3\n", "arguments"),
                      ("QUBITS 2\nCPHASE 0.5 0\n", "arguments"), ("QUBITS 2\nRZ inf 0\n", "angle")):
        with pytest.raises(ValueError, match=frag):
            oracle.Circuit(bad)
    # model noise: DEP1 after 1- and 3-qubit diagonal gates, DEP2 after 2-qubit ones
    model = {"p1": 0.1, "p2": 0.2}
    for text, slots in (("QUBITS 3\nRZ 0.3 0\n", 1), ("QUBITS 3\nCS 0 1\n", 1), ("QUBITS 3\nCCZ 0 1 2\n", 3),
                        ("QUBITS 3\nCCX 0 1 2\n", 3), ("QUBITS 3\nDIAG 2 1 2 0 0 0 1\n", 1)):
        assert oracle.Circuit(text, model).n_noise_slots == slots
    a = oracle.Circuit("QUBITS 3\nH 0\nH 1\nCS 0 1\nM 0\nM 1\n", model).batch(3, 0, 3000)
    b = oracle.Circuit("QUBITS 3\nH 0\nDEP1 0.1 0\nH 1\nDEP1 0.1 1\nCS 0 1\nDEP2 0.2 0 1\nM 0\nM 1\n").batch(3, 0, 3000)
    assert (a["outcomes"] == b["outcomes"]).all()


# ---------------------------------------------------------------------------
# Work on the shared noiseless trajectory: the part of a shot's work done
# before its first noise hit and before its first measurement whose outcome
# was drawn.  Prices the roofline of a sampler that computes that part once.
# ---------------------------------------------------------------------------
_NOISE_FREE = ("noise_slots", "noise_words")


def _no_noise(work):
    return {k: (0 if k in _NOISE_FREE else v) for k, v in work.items()}


def test_shared_work_closed_forms():
    def shot(text, noise_words=None):
        c = oracle.Circuit(text)
        w = np.full(c.words_per_shot, 1 << 31, dtype=np.uint32)
        w[: c.n_noise_slots] = 0xFFFFFFFF if noise_words is None else noise_words
        return c.shot(0, 0, words=w)
    r = shot("QUBITS 1\nH 0\nT 0\nM 0\n")  # M on T|+> has p0 = 1/2: the shot leaves at the M
    assert r.shared_work["t_entries"] == 2 and r.shared_work["events"] == 1
    assert r.shared_work["m_entries"] == 0 and r.shared_work["meas_words"] == 0
    r = shot("QUBITS 1\nT 0\nM 0\n")       # |0> stays |0>: every outcome is certain
    assert r.shared_work == _no_noise(r.work)
    text = "QUBITS 2\nH 0\nT 0\nXERR 0.5 1\nM 1\nH 0\nT 0\n"
    r = shot(text, noise_words=[0xFFFFFFFF])   # no hit: M 1 is certain, so all is shared
    assert r.shared_work == _no_noise(r.work) and r.work["events"] == 3
    r = shot(text, noise_words=[0])            # a hit before M 1: only the first T is shared
    assert r.shared_work["t_entries"] == 2 and r.shared_work["events"] == 1 and r.shared_work["m_entries"] == 0
    assert r.record == [1]


def _noisy_random_circuit(seed, n, length):
    """Clifford+T with explicit DEP1 noise after some gates and Z readouts;
    returns the lines and, per line, ('noise', slot, thr), ('meas', slot) or
    None."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lines, tags = [], []
    ns = ms = 0
    for _ in range(length):
        u = rng.random()
        q = int(rng.integers(n))
        if u < 0.25:
            lines.append("H %d" % q)
        elif u < 0.35:
            lines.append("S %d" % q)
        elif u < 0.55:
            a, b = (int(x) for x in rng.choice(n, size=2, replace=False))
            lines.append("CX %d %d" % (a, b))
        elif u < 0.7:
            lines.append("%s %d" % ("T" if rng.integers(2) == 0 else "TDG", q))
        elif u < 0.8:
            lines.append("M %d" % q)
            tags.append(("meas", ms))
            ms += 1
            continue
        else:
            p = 0.3
            lines.append("DEP1 %.1f %d" % (p, q))
            tags.append(("noise", ns, int(np.floor(p * 2 ** 32))))
            ns += 1
            continue
        tags.append(None)
    return lines, tags, ns, ms


@pytest.mark.parametrize("seed", range(12))
def test_shared_work_is_the_noiseless_run_cut_where_the_shot_leaves_it(seed):
    # Brute force: find where each shot leaves the noiseless trajectory from
    # the noiseless run's own p0 trace and the shot's noise words, cut the
    # circuit there and run the cut circuit without noise; its work is the
    # shot's shared work.
    n = 2 + seed % 4
    lines, tags, ns, ms = _noisy_random_circuit(9100 + seed, n, 60)
    text = "QUBITS %d\n" % n + "\n".join(lines) + "\n"
    c = oracle.Circuit(text)
    assert (c.n_noise_slots, c.n_meas_slots) == (ns, ms)
    rng = np.random.Generator(np.random.PCG64(seed))
    for s in range(20):
        w = rng.integers(0, 2 ** 32, size=ns + ms, dtype=np.uint64).astype(np.uint32)
        w0 = w.copy()
        w0[:ns] = 0xFFFFFFFF
        clean = c.shot(0, 0, words=w0)
        cut = len(lines)
        for j, t in enumerate(tags):
            if t is None:
                continue
            if t[0] == "noise" and int(w[t[1]]) < t[2]:
                cut = j
                break
            if t[0] == "meas" and 0.0 < clean.p0[t[1]] < 1.0:
                cut = j
                break
        r = c.shot(0, 0, words=w)
        sub = oracle.Circuit("QUBITS %d\n" % n + "".join(x + "\n" for x in lines[:cut]))
        wn = [w0[t[1]] for t in tags[:cut] if t and t[0] == "noise"]
        wm = [w[ns + t[1]] for t in tags[:cut] if t and t[0] == "meas"]
        ref = sub.shot(0, 0, words=np.array(wn + wm, dtype=np.uint32))
        assert r.shared_work == _no_noise(ref.work), (seed, s, cut)


def test_shared_work_batch_sums_and_noiseless_workload():
    # Batch sums equal the per-shot values; with no noise the 15-qubit
    # cultivation circuit never draws an outcome, so all of its work is shared.
    w = workloads.config("cultivation_15q", seed=2)
    c = oracle.Circuit(w.text, w.noise, noise_mode=1)
    b = c.batch(3, 0, 40, threads=2)
    tot = {k: 0 for k in oracle.WORK_KEYS}
    for s in range(40):
        r = c.shot(3, s)
        for k in tot:
            tot[k] += r.shared_work[k]
        assert all(r.shared_work[k] <= r.work[k] for k in tot)
    assert b["shared_work"] == tot
    assert tot["noise_words"] == 0 and tot["noise_slots"] == 0
    c0 = oracle.Circuit(w.text, {})
    b0 = c0.batch(3, 0, 10, threads=2)
    assert b0["shared_work"] == _no_noise(b0["work"])
