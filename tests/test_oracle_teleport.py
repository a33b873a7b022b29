"""Oracle pins for classically controlled gates (IF) and gate teleportation.

The conclusion of the paper names gate teleportation as the next step: a
non-Clifford gate consumed from a prepared magic state through a Clifford
circuit, a measurement and a correction chosen by its outcome.  The
corrections of T and CCZ teleportation are diagonal Cliffords (S, CZ) and
Paulis conditioned on record bits.  In the oracle a conditional diagonal gate
acts on the coefficients through the Z-string expansion U = sum_g c_g Z^g
(Eq. 4 per term, as the proof of Prop. 1 expands gate products) and leaves
the tableau alone; a conditional Pauli flips tableau signs.  These tests pin
that reading to the dense statevector (random circuits, every prefix) and to
the closed forms of teleportation: for every outcome branch the data holds
exactly the gate applied to its input, up to one global phase.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

import oracle
from tests import ref_dense
from tests.gen_small import random_circuit, random_words


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


@pytest.mark.parametrize("seed", range(40))
def test_conditional_gates_match_dense(seed):
    n = 2 + seed % 5
    text, _ = random_circuit(9100 + seed, n, 60, p_if=0.25, p_diag=0.08, p_meas=0.12)
    assert "IF " in text
    _check_dense(text, seed)


@pytest.mark.parametrize("seed", range(6))
def test_conditional_gates_every_prefix_matches_dense(seed):
    text, _ = random_circuit(9200 + seed, 3 + seed % 2, 36, p_if=0.3, p_meas=0.15)
    lines = text.strip().split("\n")
    for cut in range(2, len(lines) + 1):
        _check_dense("\n".join(lines[:cut]) + "\n", seed)


def _state(text, words):
    """The oracle's final state (Definition 1 written out as a statevector,
    with the dense checker's phase-tracked stabilizer state) and its record."""
    c = oracle.Circuit(text)
    r = c.shot(0, 0, words=np.asarray(words, dtype=np.uint32))
    _, shadow, record, _ = ref_dense.run(text, words)
    assert r.record == record
    return ref_dense.reconstruct(r.tab_x, r.tab_z, r.tab_r, r.coeffs, shadow, c.n_qubits), r


def _same_up_to_phase(a, b, tol=1e-12):
    ov = np.vdot(a, b)
    assert abs(abs(ov) - 1.0) < tol, abs(ov)
    assert np.max(np.abs(a * ov - b)) < 1e-11


def _basis(m):
    e = np.zeros(2, dtype=complex)
    e[m] = 1.0
    return e


T_MAT = np.diag([1.0, np.exp(1j * np.pi / 4)])


@pytest.mark.parametrize("seed", range(10))
@pytest.mark.parametrize("dagger", [False, True])
def test_t_teleportation_every_branch(seed, dagger):
    # |A> = T|+> on the ancilla; CX data -> ancilla; M ancilla = m; S^m (S-dagger
    # for T-dagger).  Branch m = 0 leaves T|psi>, branch m = 1 leaves
    # T-dagger|psi>, which S turns into T|psi> (up to a global phase).
    prep, _ = random_circuit(9300 + seed, 1, 12, p_meas=0, p_mpp=0, p_reset=0)
    body = prep.split("\n", 1)[1]
    g, corr = ("TDG", "SDG") if dagger else ("T", "S")
    text = "QUBITS 2\n" + body + "H 1\n%s 1\nCX 0 1\nM 1\nIF 0 %s 0\n" % (g, corr)
    psi1 = ref_dense.run("QUBITS 1\n" + body, [])[0]
    want_data = (T_MAT.conj().T if dagger else T_MAT) @ psi1
    seen = set()
    for w in (0, 2 ** 32 - 1):  # u below / above p0 = 1/2: both outcomes
        phi, r = _state(text, [w])
        m = r.record[0]
        seen.add(m)
        assert abs(r.p0[0] - 0.5) < 1e-12  # the outcome carries no information about psi
        _same_up_to_phase(phi, np.kron(_basis(m), want_data))
    assert seen == {0, 1}


CCZ_TELEPORT = (
    # |CCZ> = CCZ|+++> on ancillas 3, 4, 5; CX data i -> ancilla i; M ancillas
    # (records r0, r1, r2).  With m = ancilla outcomes the data holds
    # (-1)^{f(y ^ m)} psi_y, f = y0 y1 y2, whose expansion over GF(2) gives
    # the corrections below: CZ on the other pair for each single bit, Z on the
    # third qubit for each pair of bits (an AND).
    "H 3\nH 4\nH 5\nCCZ 3 4 5\nCX 0 3\nCX 1 4\nCX 2 5\nM 3\nM 4\nM 5\n"
    "IF 0 CZ 1 2\nIF 1 CZ 0 2\nIF 2 CZ 0 1\nIF 0&1 Z 2\nIF 0&2 Z 1\nIF 1&2 Z 0\n")


@pytest.mark.parametrize("seed", range(6))
def test_ccz_teleportation_every_branch(seed):
    prep, _ = random_circuit(9400 + seed, 3, 30, p_meas=0, p_mpp=0, p_reset=0)
    body = prep.split("\n", 1)[1]
    text = "QUBITS 6\n" + body + CCZ_TELEPORT
    psi3 = ref_dense.run("QUBITS 3\n" + body, [])[0]
    y = np.arange(8)
    ccz_psi = np.where(y == 7, -psi3, psi3)
    for branch in itertools.product((0, 1), repeat=3):
        words = [0 if b == 0 else 2 ** 32 - 1 for b in branch]
        phi, r = _state(text, words)
        assert tuple(r.record) == branch
        assert np.allclose(r.p0, 0.5, atol=1e-12, rtol=0)
        anc = np.zeros(8, dtype=complex)
        anc[branch[0] | branch[1] << 1 | branch[2] << 2] = 1.0
        _same_up_to_phase(phi, np.kron(anc, ccz_psi))


def test_condition_semantics():
    # records 1, 1, 0 (deterministic); the XOR of 0,1 is 0, the AND is 1
    pre = "QUBITS 4\nX 0\nX 1\nM 0\nM 1\nM 2\n"
    cases = (("IF 0,1 X 3\n", 0), ("IF 0&1 X 3\n", 1), ("IF 0,2 X 3\n", 1), ("IF 0&2 X 3\n", 0),
             ("IF 0,1,0,1 X 3\n", 0), ("IF 1 X 3\n", 1), ("IF 0&1&1 X 3\n", 1), ("IF 1,1 X 3\n", 0))
    for line, want in cases:
        r = oracle.Circuit(pre + line + "M 3\n").shot(0, 0, words=np.zeros(4, dtype=np.uint32))
        assert r.record == [1, 1, 0, want], line
    # a conditional S that fires is S on the state (P(X=+1) of S|+> is 1/2,
    # of S S|+> = Z|+> is 0), and one that does not fire leaves it
    for cond, p0 in (("0", 0.0), ("2", 0.5), ("0&1", 0.0), ("0,1", 0.5)):
        text = pre + "H 3\nS 3\nIF %s S 3\nMX 3\n" % cond
        r = oracle.Circuit(text).shot(0, 0, words=np.zeros(4, dtype=np.uint32))
        assert abs(r.p0[3] - p0) < 1e-12, cond


def test_unfired_conditions_leave_the_state_alone():
    # the oracle skips a gate whose condition is 0: same tableau and
    # coefficients as the circuit without it
    prep = "QUBITS 4\nH 0\nT 0\nH 1\nCX 1 2\nT 2\nH 3\nM 3\n"
    r0 = oracle.Circuit(prep).shot(0, 0, words=np.zeros(1, dtype=np.uint32))
    assert r0.record == [0]
    for line in ("IF 0 S 1\n", "IF 0 CCZ 0 1 2\n", "IF 0 DIAG 2 0 2 0.1 0.2 0.3 0.4\n", "IF 0 X 1\n",
                 "IF 0 CCX 0 1 2\n", "IF 0 RZ 0.3 2\n"):
        r = oracle.Circuit(prep + line).shot(0, 0, words=np.zeros(1, dtype=np.uint32))
        assert (r.tab_x == r0.tab_x).all() and (r.tab_z == r0.tab_z).all() and (r.tab_r == r0.tab_r).all()
        assert set(r.coeffs) == set(r0.coeffs)
        assert max(abs(r.coeffs[k] - r0.coeffs[k]) for k in r0.coeffs) == 0.0


def test_if_pauli_equals_record_controlled_pauli():
    prep = "QUBITS 3\nH 0\nM 0\nH 1\nT 1\nCX 1 2\n"
    for w in (0, 2 ** 32 - 1):
        words = np.array([w], dtype=np.uint32)
        for p in "XYZ":
            a = oracle.Circuit(prep + "%sIF 0 1\n" % p).shot(0, 0, words=words)
            b = oracle.Circuit(prep + "IF 0 %s 1\n" % p).shot(0, 0, words=words)
            assert (a.tab_r == b.tab_r).all() and (a.tab_x == b.tab_x).all() and (a.tab_z == b.tab_z).all()
            assert a.coeffs == b.coeffs


def test_if_parse_errors_and_no_model_noise():
    for bad, frag in (("QUBITS 2\nIF 0 S 1\n", "not yet measured"), ("QUBITS 2\nM 0\nIF 0,0&0 S 1\n", "not both"),
                      ("QUBITS 2\nM 0\nIF 0 H 1\n", "neither"), ("QUBITS 2\nM 0\nIF 0\n", "record bits and a gate"),
                      ("QUBITS 2\nM 0\nIF 0 CZ 1 1\n", "repeated"), ("QUBITS 2\nM 0\nIF x S 1\n", "integer"),
                      ("QUBITS 2\nM 0\nIF 0 S 1 0\n", "arguments")):
        with pytest.raises(ValueError, match=frag):
            oracle.Circuit(bad)
    model = {"p1": 0.1, "p2": 0.2, "p_meas": 0.05}
    base = oracle.Circuit("QUBITS 3\nH 0\nM 0\n", model).n_noise_slots
    for line in ("IF 0 S 1\n", "IF 0 CZ 1 2\n", "IF 0 X 2\n", "IF 0 CCZ 0 1 2\n"):
        assert oracle.Circuit("QUBITS 3\nH 0\nM 0\n" + line, model).n_noise_slots == base


def test_teleported_t_layer_matches_the_direct_layer_in_distribution():
    # With noise off, the teleported layer is T on every data qubit: the
    # records of the data readout have the direct circuit's distribution.
    # Exact: compare the outcome probabilities p0 of a final MPP of X on all
    # data qubits, which is the same in every teleportation branch.
    direct = "QUBITS 6\nH 0\nH 1\nH 2\nT 0\nT 1\nTDG 2\nMPP X0*X1*X2\n"
    tele = ("QUBITS 6\nH 0\nH 1\nH 2\nH 3\nT 3\nH 4\nT 4\nH 5\nTDG 5\n"
            "CX 0 3\nCX 1 4\nCX 2 5\nM 3\nM 4\nM 5\nIF 0 S 0\nIF 1 S 1\nIF 2 SDG 2\nMPP X0*X1*X2\n")
    p_direct = oracle.Circuit(direct).shot(0, 0, words=np.zeros(1, dtype=np.uint32)).p0[0]
    for branch in itertools.product((0, 1), repeat=3):
        words = np.array([0 if b == 0 else 2 ** 32 - 1 for b in branch] + [0], dtype=np.uint32)
        r = oracle.Circuit(tele).shot(0, 0, words=words)
        assert tuple(r.record[:3]) == branch
        assert abs(r.p0[3] - p_direct) < 1e-12
